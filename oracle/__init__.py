"""Test-infrastructure oracle: plain scalar FP64 CPU radiance Monte Carlo.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  The GPU library never imports, links or calls it.
"""
from .oracle import (  # noqa: F401
    Medium, Source, Run, Ledger, run_mc, trace, residual, gradient, detect,
    philox, philox_fill, u01, hg_dtheta, free_path, build, EV_LAUNCH, EV_CROSS,
    EV_SCATTER, EV_ESCAPE, EV_KILL, PENCIL, LINE, POINT, MAP, medium_from, sources_from,
    FLAG_LITERAL_TRUNCATION, FLAG_EQUAL_COUNT,
)

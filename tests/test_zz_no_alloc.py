"""mc_run_noalloc: the entry point for callers that cannot allocate (its
workspace is the library's static scratch) gives what mc_forward / mc_adjoint
give for the same run, on two calls in a row -- the second on a smaller
input, so the scratch holds the first call's leftovers when it starts -- and
refuses runs that do not fit the scratch before touching the device."""
import ctypes as C

import numpy as np
import pytest

import phantoms as P

pytestmark = pytest.mark.gpu


def _bind():
    import torch  # noqa: F401
    from paper_1608_05238_amd import _lib as L, rmc
    lib = L.load()
    return L, lib, rmc


def _noalloc(L, lib, rmc, ph, specs, run, adjoint):
    import torch
    med = rmc.Medium.from_phantom(ph)
    src = rmc._Sources(specs, med.mua.device)
    K = 2 * run.n_harm + 1
    out = torch.full((K, ph.nz, ph.nx), float("nan"), dtype=torch.float64, device=med.mua.device)
    led = torch.zeros(C.sizeof(L.mc_ledger), dtype=torch.uint8, device=med.mua.device)
    rc = lib.mc_run_noalloc(C.byref(med.c()), src.arr, src.n, C.byref(run), int(adjoint), None, out.data_ptr(),
                            led.data_ptr(), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == L.MC_OK, lib.mc_status_string(rc)
    torch.cuda.synchronize()
    return out.cpu().numpy(), rmc.ledger_dict(led)


def _reference(rmc, ph, specs, run, adjoint):
    med = rmc.Medium.from_phantom(ph)
    fn = rmc.mc_adjoint if adjoint else rmc.mc_forward
    co, led = fn(med, specs, run)
    return co.cpu().numpy(), rmc.ledger_dict(led)


def test_noalloc_equals_the_allocating_entry_points():
    L, lib, rmc = _bind()
    c = P.config2()
    ph2 = P.disc_phantom(64, 0.2, 0.02, 8.0, 0.9, seed=12, radius=(1.0, 2.5))
    cases = [
        # the 256x256 workload's forward run (tiled transport, pool fitted to the scratch)
        (c.phantom, c.sources, rmc.make_run(300_000, 16, seed=5), False),
        # then a smaller adjoint run with a signed map source
        (ph2, [P.map_source(P.residual_like_map(ph2, seed=3))], rmc.make_run(60_000, 16, seed=6, stream_tag=1), True),
        # and a whole-grid run (the 32x32 pencil beam at N = 8)
        (P.config1().phantom, P.config1().sources, rmc.make_run(50_000, 8, seed=7), False),
    ]
    for ph, specs, run, adj in cases:
        got, lg = _noalloc(L, lib, rmc, ph, specs, run, adj)
        ref, lr = _reference(rmc, ph, specs, run, adj)
        assert np.array_equal(got, ref), (ph.nx, adj, np.nanmax(np.abs(got - ref)))
        for k in ("packets", "segments", "visits", "scatters"):
            assert lg[k] == lr[k], (k, lg[k], lr[k])
        assert lg["absorbed"] == pytest.approx(lr["absorbed"], rel=1e-9)


def test_noalloc_refuses_runs_beyond_the_scratch():
    L, lib, rmc = _bind()
    import torch
    big = P.homogeneous(4096, 4096, 0.01, 0.01, 1.0, 0.5)   # FP64 tally alone: 4096^2 x 65 x 8 bytes
    med = rmc.Medium(*(torch.as_tensor(a, device="cuda") for a in (big.mua, big.mus, big.g)), big.dx)
    src = rmc._Sources(P.pencil_top_centre(big), med.mua.device)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    run = rmc.make_run(1000, 32)
    rc = lib.mc_run_noalloc(C.byref(med.c()), src.arr, src.n, C.byref(run), 0, None, out.data_ptr(), None, None)
    assert rc == L.MC_ERR_SCRATCH
    # the caller's own pool size is honoured, and refused when it does not fit
    c = P.config2()
    med = rmc.Medium.from_phantom(c.phantom)
    src = rmc._Sources(c.sources, med.mua.device)
    opts = rmc._Options({"live_packets": 1 << 26}, None)
    rc = lib.mc_run_noalloc(C.byref(med.c()), src.arr, src.n, C.byref(rmc.make_run(1 << 27, 16)), 0, opts.ref(),
                            out.data_ptr(), None, None)
    assert rc == L.MC_ERR_SCRATCH
    # a timer would allocate events: refused
    timer = rmc.Timer()
    opts = rmc._Options(None, timer)
    rc = lib.mc_run_noalloc(C.byref(med.c()), src.arr, src.n, C.byref(rmc.make_run(1000, 16)), 0, opts.ref(),
                            out.data_ptr(), None, None)
    assert rc == L.MC_ERR_INVALID_ARG

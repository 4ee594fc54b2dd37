"""Quantitative PAT reconstruction with the radiance Monte Carlo gradients.

Minimises eps = (A/2) sum (Hmeas - H(mua, mus))^2 (eq. error_function3) over
log mua and/or log mus with L-BFGS (torch.optim.LBFGS, strong-Wolfe line
search).  The gradient of every evaluation comes from the adjoint Monte Carlo
(`autograd.absorbed_energy`); the seed is fixed, so every evaluation uses the
same random numbers and the objective is a deterministic function of the
coefficients.  The paper itself used gradient descent with line searches
(Sec. 6); L-BFGS is the quasi-Newton alternative on the same gradients.

    python -m paper_1608_05238_amd.recon            # 256x256 two-inclusion phantom

Before the iterations it checks the gradient at the initial guess against a
reference from 1e9 + 1e9 packets (--ref-packets).
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import Sequence

import numpy as np
import torch

from . import rmc
from .autograd import MCConfig, absorbed_energy, error_functional


def reconstruct(mua0: torch.Tensor, mus0: torch.Tensor, g: torch.Tensor, dx: float, sources: Sequence,
                hmeas: torch.Tensor, cfg: MCConfig, iters: int, fit_mua: bool = True, fit_mus: bool = True,
                log=None):
    """Run `iters` L-BFGS iterations from (mua0, mus0).  Returns the final
    coefficient maps and a history of (evaluation, eps) pairs."""
    th_a = torch.log(mua0.double()).clone().requires_grad_(fit_mua)
    th_s = torch.log(mus0.double()).clone().requires_grad_(fit_mus)
    params = [t for t, f in ((th_a, fit_mua), (th_s, fit_mus)) if f]
    opt = torch.optim.LBFGS(params, lr=1.0, max_iter=iters, history_size=10, line_search_fn="strong_wolfe",
                            tolerance_grad=0.0, tolerance_change=0.0)
    hist = []
    scale = {}

    def closure():
        opt.zero_grad()
        h = absorbed_energy(torch.exp(th_a), torch.exp(th_s), g, dx, sources, cfg)
        eps = error_functional(h, hmeas, dx)
        if "eps0" not in scale:
            scale["eps0"] = float(eps.detach())
        loss = eps / scale["eps0"]
        loss.backward()
        hist.append(float(eps.detach()))
        if log:
            log(f"evaluation {len(hist)}: eps = {hist[-1]:.6e}")
        return loss

    opt.step(closure)
    return torch.exp(th_a).detach(), torch.exp(th_s).detach(), hist


def reference_check(mua0, mus0, g, dx, sources, hmeas, packets: int, ref_packets: int, n_harm: int = 16,
                    margin: int = 10, log=None) -> dict:
    """The autograd gradient of eps at (mua0, mus0) from `packets`-packet runs
    (two seeds) against the explicit residual / adjoint / gradient chain from
    ref_packets + ref_packets packets: relative L2 errors over pixels at least
    `margin` from the boundary, and the error the two seeds' difference
    predicts from Monte Carlo noise alone."""
    from .autograd import MCConfig
    med = rmc.Medium(mua0.float().contiguous(), mus0.float().contiguous(), g.float().contiguous(), float(dx))
    t0 = time.time()
    f, _ = rmc.mc_forward(med, sources, rmc.make_run(ref_packets, n_harm, seed=555), ledger=False)
    q, _ = rmc.mc_residual(med, f, hmeas)
    a, _ = rmc.mc_adjoint(med, [rmc.Source("map", map=q)], rmc.make_run(ref_packets, n_harm, seed=555, stream_tag=1),
                          ledger=False)
    ref = rmc.mc_gradient(med, n_harm, f, a, hmeas)
    if log:
        log(f"reference gradient from {ref_packets:.0e} + {ref_packets:.0e} packets: {time.time() - t0:.1f} s")
    grads = []
    for seed in (7, 8):
        ta = mua0.double().clone().requires_grad_(True)
        ts = mus0.double().clone().requires_grad_(True)
        h = absorbed_energy(ta, ts, g, dx, sources, MCConfig(packets, n_harm, seed=seed))
        error_functional(h, hmeas, dx).backward()
        grads.append((ta.grad.detach(), ts.grad.detach()))
    m = margin
    out = {"packets": packets, "reference_packets": ref_packets}
    for k, name in ((0, "dmua"), (1, "dmus")):
        r = ref[k][m:-m, m:-m]
        g1, g2 = grads[0][k][m:-m, m:-m], grads[1][k][m:-m, m:-m]
        out[f"err_{name}"] = [float((gg - r).norm() / r.norm()) for gg in (g1, g2)]
        out[f"noise_{name}"] = float((g1 - g2).norm() / 2 ** 0.5 / r.norm())
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--dx", type=float, default=0.1)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--packets", type=float, default=1e7)
    ap.add_argument("--hmeas-packets", type=float, default=1e8)
    ap.add_argument("--fit", choices=("mua", "mus", "both"), default="both")
    ap.add_argument("--ref-packets", type=float, default=1e9,
                    help="packets per run of the reference gradient at the initial guess (0: skip)")
    args = ap.parse_args(argv)
    dev = torch.device("cuda", 0)
    n, dx = args.n, args.dx
    L = n * dx
    c = (np.arange(n) + 0.5) * dx
    X, Z = np.meshgrid(c, c)
    mua_t = np.full((n, n), 0.01, np.float32)
    mus_t = np.full((n, n), 10.0, np.float32)
    mua_t[(X - 0.35 * L) ** 2 + (Z - 0.4 * L) ** 2 <= (0.1 * L) ** 2] = 0.05
    mus_t[(X - 0.65 * L) ** 2 + (Z - 0.6 * L) ** 2 <= (0.1 * L) ** 2] = 20.0
    g = torch.full((n, n), 0.9, dtype=torch.float32, device=dev)
    sources = [rmc.Source("line", 0.0, 0.0, L, 0.0, 0.0, 1.0, 0, 0.25), rmc.Source("line", 0.0, L, L, L, 0.0, -1.0, 0, 0.25),
               rmc.Source("line", 0.0, 0.0, 0.0, L, 1.0, 0.0, 0, 0.25), rmc.Source("line", L, 0.0, L, L, -1.0, 0.0, 0, 0.25)]
    true = rmc.Medium(torch.as_tensor(mua_t, device=dev), torch.as_tensor(mus_t, device=dev), g, dx)
    f, _ = rmc.mc_forward(true, sources, rmc.make_run(int(args.hmeas_packets), 16, seed=12345), ledger=False)
    hmeas = rmc.mc_absorbed(true, f)
    mua0 = torch.full((n, n), 0.01, dtype=torch.float32, device=dev) if args.fit != "mus" else true.mua.clone()
    mus0 = torch.full((n, n), 10.0, dtype=torch.float32, device=dev) if args.fit != "mua" else true.mus.clone()
    check = None
    if args.ref_packets > 0:
        check = reference_check(mua0, mus0, g, dx, sources, hmeas, int(args.packets), int(args.ref_packets),
                                log=lambda m: print(m, file=sys.stderr, flush=True))
    t0 = time.time()
    mua, mus, hist = reconstruct(mua0, mus0, g, dx, sources, hmeas, MCConfig(int(args.packets), 16, seed=7),
                                 args.iters, fit_mua=args.fit != "mus", fit_mus=args.fit != "mua",
                                 log=lambda m: print(m, file=sys.stderr, flush=True))
    wall = time.time() - t0
    ta, ts = true.mua.double(), true.mus.double()
    out = {"grid": n, "dx_mm": dx, "fit": args.fit, "packets_per_run": int(args.packets),
           "lbfgs_iterations": args.iters, "evaluations": len(hist), "wall_s": wall,
           "eps_initial": hist[0], "eps_final": hist[-1],
           "mua_rel_l2_error_initial": float((mua0.double() - ta).norm() / ta.norm()),
           "mua_rel_l2_error_final": float((mua.double() - ta).norm() / ta.norm()),
           "mus_rel_l2_error_initial": float((mus0.double() - ts).norm() / ts.norm()),
           "mus_rel_l2_error_final": float((mus.double() - ts).norm() / ts.norm()),
           "gradient_vs_reference_at_start": check}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

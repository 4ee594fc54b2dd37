"""Functional gradients of Sec. 5 (the mua and mus formulas built from
forward and adjoint harmonic coefficients) against central finite
differences of eps at single pixels of the 256x256 disc phantom (four line
sources, N = 16, measured data from the second disc phantom).

For each of 20 seeded interior pixels (at least 10 pixels from the boundary)
and each parameter, eps is evaluated with that pixel's value scaled by
1 +- h.  The two sides use common random numbers (same seed, same packet
ids): a packet that never enters the pixel contributes identically to both,
so the difference is carried by the packets that do.  All 80 perturbed
problems of one seed run in one batched launch.  The adjoint gradient
(forward, residual, adjoint, harmonic products) and the finite difference
are each averaged over independent seeds, which also give their standard
errors.

A change of mus in one pixel moves every later scatter site of the packets
that cross it, so the difference of the two sides picks up grazing crossings
of later pixel faces, roulette and escape decisions that flip: terms of large
variance that grows as the step shrinks.  The mus step is therefore 10% (the
O(h^2) error of the central difference stays near 0.2%); mua, which changes
weights and not paths, takes 1%.  Even so, a single pixel's mus derivative in
the interior is below the finite differences' noise at this packet count (the
low signal-to-noise ratio of the mus gradient that the paper reports), so for
mus the per-pixel bound is supplemented by the inverse-variance weighted mean
of the differences over the 20 pixels; the resolved mus check is the
directional derivative along a smooth perturbation (test_gpu_autograd).  For
mua the pixels are resolved and their agreement is asserted as well.

Both estimators use eps of a single run, whose expectation carries the
variance of that run's H (O(1/Np)); the adjoint gradient, whose residual
comes from the same forward run, carries the same term.  Runs of equal
packet count on both sides keep that bias common.  The allowance covers the
pixel-averaged coefficients in the gradient formula (the exact derivative of
the discrete eps needs the pixel average of the product of forward and
adjoint radiance, the formula takes the product of the averages) and the
truncation of the harmonic sum at N.
"""
import json
import os

import numpy as np
import pytest

import phantoms as P

pytestmark = pytest.mark.gpu

OUT = os.environ.get("RMC_PARITY_STATS_DIR")

N_HARM = 16
H_REL = {"mua": 0.01, "mus": 0.10}   # relative finite-difference steps
N_RUN = 500_000       # packets per run, gradient and finite-difference runs alike
B_FD = 16             # seeds of the finite differences
B_G = 64              # seeds of the adjoint gradient
ALLOW = 0.05          # relative allowance (pixel averaging, harmonic truncation)


def test_gradient_matches_pixel_finite_differences_disc256():
    import torch
    from paper_1608_05238_amd import rmc
    c = P.config2()
    ph, true = c.phantom, c.extra["true"]
    dev = torch.device("cuda", 0)
    med = rmc.Medium.from_phantom(ph, dev)
    src = c.sources
    tmed = rmc.Medium.from_phantom(true, dev)
    ft, _ = rmc.mc_forward(tmed, src, rmc.make_run(20_000_000, N_HARM, seed=1), ledger=False)
    hm = rmc.mc_absorbed(tmed, ft)
    pix = P.interior_pixels(ph, count=20, margin=10, seed=2)
    iz, ix = pix[:, 0], pix[:, 1]
    npx = len(pix)

    # adjoint gradient at the pixels, per seed
    g = np.zeros((B_G, 2, npx))
    for b in range(B_G):
        f, _ = rmc.mc_forward(med, src, rmc.make_run(N_RUN, N_HARM, seed=1000 + b), ledger=False)
        q, _ = rmc.mc_residual(med, f, hm)
        a, _ = rmc.mc_adjoint(med, [rmc.Source("map", map=q)],
                              rmc.make_run(N_RUN, N_HARM, seed=1000 + b, stream_tag=1), ledger=False)
        dmua, dmus = rmc.mc_gradient(med, N_HARM, f, a, hm)
        g[b, 0] = dmua.cpu().numpy()[iz, ix]
        g[b, 1] = dmus.cpu().numpy()[iz, ix]

    # perturbed media: [pixel][parameter][+h, -h]; the step is taken from the FP32 values used
    media, step = [], np.zeros((2, npx))
    for k in range(npx):
        for p, name in enumerate(("mua", "mus")):
            vals = []
            for s in (1.0, -1.0):
                mua, mus = med.mua.clone(), med.mus.clone()
                t = mua if name == "mua" else mus
                t[iz[k], ix[k]] *= 1.0 + s * H_REL[name]
                vals.append(float(t[iz[k], ix[k]]))
                media.append(rmc.Medium(mua, mus, med.g, med.dx))
            step[p, k] = vals[0] - vals[1]
    fd = np.zeros((B_FD, 2, npx))
    for b in range(B_FD):
        outs = rmc.mc_run_batch([rmc.Problem(m, src, rmc.make_run(N_RUN, N_HARM, seed=2000 + b)) for m in media],
                                ledger=False)
        eps = torch.stack([rmc.mc_residual(m, o, hm)[1] for m, (o, _) in zip(media, outs)]).cpu().numpy()
        eps = eps.reshape(npx, 2, 2)
        fd[b] = (eps[:, :, 0] - eps[:, :, 1]).T / step
        del outs

    stats = {}
    for p, name in enumerate(("mua", "mus")):
        m_fd, m_g = fd[:, p].mean(0), g[:, p].mean(0)
        se = np.sqrt(fd[:, p].var(0, ddof=1) / B_FD + g[:, p].var(0, ddof=1) / B_G)
        tol = 4.0 * se + ALLOW * np.abs(m_fd)
        z = (m_fd - m_g) / se
        stats[name] = {"fd": m_fd.tolist(), "grad": m_g.tolist(), "se": se.tolist(), "z": z.tolist(),
                       "resolved": int((np.abs(m_fd) > 4.0 * se).sum())}
        bad = np.abs(m_fd - m_g) > tol
        assert not bad.any(), (name, pix[bad].tolist(), m_fd[bad], m_g[bad], se[bad])
        w = 1.0 / se ** 2
        dm, dse = float(((m_fd - m_g) * w).sum() / w.sum()), float(1.0 / np.sqrt(w.sum()))
        stats[name]["weighted_mean_diff"] = [dm, dse]
        assert abs(dm) <= 4.0 * dse + ALLOW * abs(float((m_fd * w).sum() / w.sum())), (name, dm, dse)
        if name == "mua":
            assert stats[name]["resolved"] >= 15, stats[name]["resolved"]
            rel = float(np.linalg.norm(m_fd - m_g) / np.linalg.norm(m_fd))
            assert rel < 0.1, rel
    if OUT:
        os.makedirs(OUT, exist_ok=True)
        with open(os.path.join(OUT, "parity_stats.jsonl"), "a") as f:
            f.write(json.dumps({"test": "gradient_pixel_fd_disc256", "pixels": pix.tolist(), **stats}) + "\n")

"""Test helpers: exact ray/pixel intersection, batch statistics.

These are independent of both the oracle and the GPU library: they give the
closed forms and brute-force quadratures the Monte Carlo is pinned against.
"""
from __future__ import annotations

import numpy as np


def ray_pixel_segments(x0, z0, sx, sz, nx, nz, dx, smax=None):
    """Exact chords of the ray (x0,z0) + s (sx,sz), s >= 0, through the pixel grid.

    Parametric intersection with every grid line (Siddon's method): returns a
    list of (ix, iz, s_in, s_out) in the order the ray meets them.
    """
    W, D = nx * dx, nz * dx
    cand = [0.0]
    if sx != 0:
        for k in range(nx + 1):
            s = (k * dx - x0) / sx
            if s > 0:
                cand.append(s)
    if sz != 0:
        for k in range(nz + 1):
            s = (k * dx - z0) / sz
            if s > 0:
                cand.append(s)
    cand = np.unique(np.array(cand))
    if smax is not None:
        cand = np.concatenate([cand[cand < smax], [smax]])
    out = []
    for a, b in zip(cand[:-1], cand[1:]):
        if b - a <= 0:
            continue
        m = 0.5 * (a + b)
        xm, zm = x0 + m * sx, z0 + m * sz
        if not (0 <= xm < W and 0 <= zm < D):
            continue
        out.append((int(np.floor(xm / dx)), int(np.floor(zm / dx)), a, b))
    return out


def ballistic_tally(mua, dx, x0, z0, theta, N):
    """Harmonic maps of a non-scattering unit-power beam along angle theta.

    For each pixel chord [s_in, s_out] the track length weighted by the
    surviving fraction is (e^{-tau_in} - e^{-tau_out}) / mua_i (or the chord
    length when mua_i = 0); the harmonic moments are that times cos/sin(n
    theta); the pixel value is divided by the pixel area.
    """
    nz, nx = mua.shape
    sx, sz = np.sin(theta), np.cos(theta)
    K = 2 * N + 1
    out = np.zeros((K, nz, nx))
    tau = 0.0
    for ix, iz, a, b in ray_pixel_segments(x0, z0, sx, sz, nx, nz, dx):
        m = float(mua[iz, ix])
        l = b - a
        T = (np.exp(-tau) - np.exp(-tau - m * l)) / m if m > 0 else np.exp(-tau) * l
        tau += m * l
        out[0, iz, ix] += T
        for n in range(1, N + 1):
            out[n, iz, ix] += T * np.cos(n * theta)
            out[N + n, iz, ix] += T * np.sin(n * theta)
    return out / (dx * dx)


def batch_mean_se(samples: np.ndarray):
    """Mean and standard error over the leading (batch) axis."""
    s = np.asarray(samples)
    B = s.shape[0]
    return s.mean(axis=0), s.std(axis=0, ddof=1) / np.sqrt(B)

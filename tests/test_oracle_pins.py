"""Pins of the FP64 CPU oracle to what the paper and the mathematics fix.

Each test compares the oracle with something other than itself: published
known-answer vectors, closed forms, brute-force quadrature, invariants.
Paper: Hochuli, Powell, Arridge & Cox, arXiv:1608.05238.
"""
import os

import numpy as np
import pytest
from scipy import integrate

import phantoms as P
from tests.helpers import ballistic_tally, batch_mean_se, ray_pixel_segments

HERE = os.path.dirname(os.path.abspath(__file__))


def _batches(O, med, src, run_kw, B, n_per, threads=8, **kw):
    outs, leds = [], []
    for b in range(B):
        r = O.Run(n_packets=n_per, first_packet_id=b * n_per, **run_kw)
        res = O.run_mc(med, src, r, n_threads=threads, **kw)
        outs.append(res[0])
        leds.append(res[1])
    return np.array(outs), leds


# ---------------------------------------------------------------- random numbers
def test_philox_known_answers(oracle_lib):
    """Philox4x32-10 against the published known-answer vectors (Salmon et al., SC'11)."""
    O = oracle_lib
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) if l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        assert O.philox(w[0:4], w[4:6]) == w[6:10]


def test_uniform_mapping_exact(oracle_lib):
    """u = ((x >> 9) + 1/2) 2^-23: strictly inside (0,1), exact in FP32."""
    O = oracle_lib
    assert O.u01(0) == 2.0 ** -24
    assert O.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    for x in [1, 511, 512, 12345678, 0x80000000, 0xDEADBEEF]:
        u = O.u01(x)
        assert 0 < u < 1
        assert float(np.float32(u)) == u
        assert u == ((x >> 9) + 0.5) / 2 ** 23


def test_philox_fill_matches_block_function(oracle_lib):
    O = oracle_lib
    out = O.philox_fill(seed=0x1234_5678_9ABC, tag=3, pid0=(1 << 32) - 2, n=4, j=7)
    for i in range(4):
        pid = (1 << 32) - 2 + i
        ref = O.philox([7, 3, pid & 0xFFFFFFFF, pid >> 32], [0x5678_9ABC, 0x1234])
        assert list(out[i]) == ref


# ---------------------------------------------------------------- sampling laws
@pytest.mark.parametrize("g", [0.0, 0.5, 0.8, 0.9, 0.99, -0.6])
def test_hg_sampler_inverts_the_phase_function_cdf(oracle_lib, g):
    """Sec. 3 eq. scattering_angle inverts the CDF of the 2D HG law eq. scattering2D.

    For u on a grid, the probability mass of eq. scattering2D below the
    sampled deflection must equal u (quadrature of the printed density)."""
    O = oracle_lib
    pdf = lambda t: (1 - g * g) / (2 * np.pi * (1 + g * g - 2 * g * np.cos(t)))
    for u in np.linspace(0.01, 0.99, 33):
        t = O.hg_dtheta(g, u)
        mass, _ = integrate.quad(pdf, -np.pi, t, epsabs=1e-12, epsrel=1e-12, limit=200)
        assert mass == pytest.approx(u, abs=2e-9)


@pytest.mark.parametrize("g", [0.0, 0.5, 0.9, -0.4])
def test_hg_fourier_moments(oracle_lib, g):
    """E[cos l dt] = g^l and E[sin l dt] = 0 (Sec. 5 eq. HGFourier), by midpoint quadrature in u."""
    O = oracle_lib
    M = 100_000
    u = (np.arange(M) + 0.5) / M
    t = np.array([O.hg_dtheta(g, x) for x in u])
    for l in range(1, 17):
        assert np.mean(np.cos(l * t)) == pytest.approx(g ** l, abs=2e-6)
        assert abs(np.mean(np.sin(l * t))) < 1e-9


def test_free_path_is_exponential(oracle_lib):
    """s = -ln U / mu_s (the exponential law; Sec. 3 prints U / mu_s): mean 1, P(s > a) = e^-a."""
    O = oracle_lib
    M = 200_000
    u = (np.arange(M) + 0.5) / M
    s = np.array([O.free_path(x) for x in u])
    assert s.mean() == pytest.approx(1.0, abs=2e-5)
    for a in (0.5, 1.0, 2.0, 4.0):
        assert np.mean(s > a) == pytest.approx(np.exp(-a), abs=2e-5)


# ---------------------------------------------------------------- exact transport cases
def test_beer_lambert_pencil_column(oracle_lib):
    """mu_s = 0: every packet is identical, the maps are Beer-Lambert exactly.

    Pencil at (x = 8.0, z = 0) down +z on a pixel face: the half-open pixel
    rule puts the beam in column 16.  a_n = a0 (t = 0), b_n = 0."""
    O = oracle_lib
    rng = np.random.default_rng(5)
    nz, nx, dx = 32, 32, 0.5
    mua = rng.uniform(0.01, 0.3, size=(nz, nx))
    med = O.Medium(mua, np.zeros((nz, nx)), np.full((nz, nx), 0.8), dx)
    src = [O.Source(O.PENCIL, x0=8.0, z0=0.0, dir_x=0.0, dir_z=1.0, power=1.0)]
    co, L = O.run_mc(med, src, O.Run(1000, 0, 8))
    exp = ballistic_tally(mua, dx, 8.0 + 1e-12, 0.0, 0.0, 8)   # just inside column 16
    np.testing.assert_allclose(co, exp, rtol=1e-11, atol=1e-14)
    assert np.count_nonzero(co[0]) == nz and np.all(co[0][:, 16] > 0)
    # energy: absorbed + escaped = launched; absorbed = sum mua a0 A
    assert L.launched == pytest.approx(L.absorbed + L.escaped, rel=1e-13)
    assert (mua * co[0]).sum() * dx * dx == pytest.approx(L.absorbed * L.scale, rel=1e-12)


@pytest.mark.parametrize("theta", [0.3, -1.1, 2.5, np.pi / 4])
def test_beer_lambert_tilted_pencil(oracle_lib, theta):
    """Non-scattering tilted beam against exact ray/pixel chords (Siddon)."""
    O = oracle_lib
    rng = np.random.default_rng(7)
    nz, nx, dx = 12, 12, 0.25
    mua = rng.uniform(0.0, 2.0, size=(nz, nx))
    mua[3, :] = 0.0
    x0, z0 = 1.37, 1.61
    med = O.Medium(mua, np.zeros((nz, nx)), np.zeros((nz, nx)), dx)
    src = [O.Source(O.PENCIL, x0=x0, z0=z0, dir_x=np.sin(theta), dir_z=np.cos(theta))]
    co, _ = O.run_mc(med, src, O.Run(10, 0, 6))
    exp = ballistic_tally(mua, dx, x0, z0, theta, 6)
    np.testing.assert_allclose(co, exp, rtol=1e-10, atol=1e-12)


def test_isotropic_point_source_quadrature(oracle_lib):
    """mu_s = 0, heterogeneous mu_a, isotropic point source: brute-force angular quadrature.

    Expected a_n of a pixel = (1/A) int dt/(2pi) T(t) cos(n t), T the
    attenuated chord of the ray at angle t (exact chords), on 4000 angles."""
    O = oracle_lib
    rng = np.random.default_rng(11)
    nz, nx, dx, N = 4, 4, 1.0, 3
    mua = rng.uniform(0.05, 1.0, size=(nz, nx))
    x0, z0 = 1.3, 1.7
    M = 4000
    exp = np.zeros((2 * N + 1, nz, nx))
    for t in (np.arange(M) + 0.5) / M * 2 * np.pi - np.pi:
        exp += ballistic_tally(mua, dx, x0, z0, t, N)
    exp /= M
    med = O.Medium(mua, np.zeros((nz, nx)), np.zeros((nz, nx)), dx)
    src = [O.Source(O.POINT, x0=x0, z0=z0)]
    outs, _ = _batches(O, med, src, dict(seed=1, n_harm=N), B=10, n_per=20_000)
    mean, se = batch_mean_se(outs)
    z = np.abs(mean - exp) / np.maximum(se, 1e-12)
    assert np.max(z) < 5.0, np.max(z)
    assert np.abs(mean[0] - exp[0]).max() < 0.02 * exp[0].max()


def test_energy_ledger_with_roulette(oracle_lib):
    """Per-run FP64 balance launched + gain - loss = absorbed + escaped, with roulette active;
    absorbed power also equals sum_i mua_i a0_i A from the tally (H = mua Phi, Sec. 2)."""
    O = oracle_lib
    ph = P.homogeneous(8, 8, 0.5, 2.0, 20.0, 0.0)
    med = O.medium_from(ph)
    src = O.sources_from(P.pencil_top_centre(ph))
    co, L = O.run_mc(med, src, O.Run(20000, 3, 4, w_threshold=0.05, roulette_m=4.0), n_threads=4)
    assert L.roulette_gain > 0 and L.roulette_loss > 0
    lhs = L.launched + L.roulette_gain - L.roulette_loss
    assert lhs == pytest.approx(L.absorbed + L.escaped, rel=1e-12)
    assert (ph.mua * co[0]).sum() * ph.dx ** 2 == pytest.approx(L.absorbed * L.scale, rel=1e-12)


@pytest.mark.parametrize("mus,g", [(0.0, 0.0), (5.0, 0.8), (12.0, -0.3)])
def test_mean_path_invariance(oracle_lib, mus, g):
    """mu_a = 0 with uniform Lambertian illumination of the boundary: the mean path
    length inside the domain is pi A / perimeter for any scattering (invariance
    property of Blanco & Fournier 2003; Cauchy's chord formula when mu_s = 0).
    With unit power, sum_i a0_i A is that mean path."""
    O = oracle_lib
    ph = P.homogeneous(8, 8, 0.5, 0.0, mus, g)
    ph.mus[2:5, 3:6] *= 2.0   # heterogeneous scattering leaves it unchanged
    med = O.medium_from(ph)
    src = O.sources_from(P.lambertian_boundary(ph, 1.0))
    outs, _ = _batches(O, med, src, dict(seed=2, n_harm=0), B=8, n_per=25_000)
    paths = outs[:, 0].sum(axis=(1, 2)) * ph.dx ** 2
    m, se = batch_mean_se(paths)
    L = ph.width
    assert abs(m - np.pi * L / 4) < 4 * se + 1e-12, (m, np.pi * L / 4, se)


def test_forward_peaked_limit(oracle_lib):
    """g = 1: scattering never turns the packet, so the maps do not depend on mu_s,
    and d eps / d mu_s = 0 exactly (factor 1 - g^n of eq. scattering_gradient3)."""
    O = oracle_lib
    nz, nx, dx = 10, 10, 0.3
    rng = np.random.default_rng(3)
    mua = rng.uniform(0.01, 0.2, size=(nz, nx))
    g = np.ones((nz, nx))
    src = [O.Source(O.LINE, 0.0, 0.0, 3.0, 0.0, 0.3, np.sqrt(1 - 0.09))]
    a, _ = O.run_mc(O.Medium(mua, np.full((nz, nx), 1.0), g, dx), src, O.Run(3000, 0, 4))
    b, _ = O.run_mc(O.Medium(mua, np.full((nz, nx), 9.0), g, dx), src, O.Run(3000, 0, 4))
    np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-13)
    med = O.Medium(mua, np.full((nz, nx), 9.0), g, dx)
    dmua, dmus = O.gradient(med, 4, a, b, np.zeros((nz, nx)))
    assert np.all(dmus == 0.0)


def test_symmetry_and_angle_convention(oracle_lib):
    """Centred isotropic source in a homogeneous square: mirror symmetries of the maps
    with the sign rules of cos/sin(n t) for t measured from +z (Sec. 3.1), and net
    flux pointing away from the source (b1 > 0 on the +x side, a1 > 0 on the +z side)."""
    O = oracle_lib
    N = 3
    ph = P.homogeneous(8, 8, 0.5, 0.2, 4.0, 0.7)
    med = O.medium_from(ph)
    src = O.sources_from([P.point_source(2.0, 2.0)])
    outs, _ = _batches(O, med, src, dict(seed=4, n_harm=N), B=8, n_per=25_000)
    m, se = batch_mean_se(outs)
    sx_ = np.ones(2 * N + 1)
    sx_[N + 1:] = -1                                # x -> -x: b_n flips
    sz_ = np.array([1] + [(-1) ** n for n in range(1, N + 1)] + [(-1) ** (n + 1) for n in range(1, N + 1)])
    mx = m[:, :, ::-1] * sx_[:, None, None]
    mz = m[:, ::-1, :] * sz_[:, None, None]
    for other, name in ((mx, "x"), (mz, "z")):
        z = np.abs(m - other) / np.sqrt(2 * se ** 2 + 1e-300)
        assert np.percentile(z, 99) < 4.5, name
    assert m[2 * N - N + 1, 3, 6] > 10 * se[N + 1, 3, 6]   # b1 right of the source
    assert m[1, 6, 3] > 10 * se[1, 6, 3]                   # a1 below the source


# ---------------------------------------------------------------- adjoint reciprocity (Sec. 4.1)
def _recip_setup():
    ph = P.homogeneous(16, 16, 0.25, 0.1, 5.0, 0.8)
    ph.mua[5:9, 9:13] = 0.4
    ph.mus[2:6, 2:7] = 9.0
    s, d = (5, 7), (11, 8)            # (iz, ix): source and detector pixels, apart along z
    return ph, s, d


def _pixel_map(ph, iz, ix, val):
    m = np.zeros((ph.nz, ph.nx))
    m[iz, ix] = val
    return m


@pytest.mark.parametrize("case", ["iso", "odd_detector", "odd_source"])
def test_adjoint_reciprocity(oracle_lib, case):
    """<L a, b> = <a, L* b> (eq. adj_definition) for pixel sources/detectors.

    iso: the paper's case 1.  odd_detector / odd_source: detector or source
    profile (1 + cos t)/2pi, which has an order-1 term, so the direction
    mirroring of the adjoint field is exercised (the paper's cases use only
    even orders)."""
    O = oracle_lib
    ph, s, d = _recip_setup()
    A = ph.dx ** 2
    med = O.medium_from(ph)
    prof = np.array([1.0, 0.5, 0.0])          # p = (1 + cos t) / 2pi
    src_prof = prof if case == "odd_source" else None
    det_prof = prof if case == "odd_detector" else None
    fwd_src = [O.Source(O.MAP, map=_pixel_map(ph, *s, 1.0 / (2 * np.pi * A)), prof=src_prof)]
    adj_src = [O.Source(O.MAP, map=_pixel_map(ph, *d, 1.0 / A), prof=det_prof)]
    fo, _ = _batches(O, med, fwd_src, dict(seed=8, n_harm=2), B=8, n_per=25_000)
    ad, _ = _batches(O, med, adj_src, dict(seed=9, n_harm=2, stream_tag=1, adjoint=1), B=8, n_per=25_000)
    if case == "odd_detector":
        lhs = fo[:, 0][:, d[0], d[1]] + fo[:, 1][:, d[0], d[1]]
    else:
        lhs = fo[:, 0][:, d[0], d[1]]
    if case == "odd_source":
        rhs = (ad[:, 0][:, s[0], s[1]] + ad[:, 1][:, s[0], s[1]]) / (2 * np.pi)
    else:
        rhs = ad[:, 0][:, s[0], s[1]] / (2 * np.pi)
    ml, sl = batch_mean_se(lhs)
    mr, sr = batch_mean_se(rhs)
    assert abs(ml - mr) < 4 * np.hypot(sl, sr), (ml, mr, sl, sr)
    assert abs(ml - mr) < 0.05 * abs(ml)


def test_adjoint_mirror_is_detected(oracle_lib):
    """Without the output mirroring the odd_source identity fails: the a1 term
    changes sign, which the test above would see (guards the test's power)."""
    O = oracle_lib
    ph, s, d = _recip_setup()
    A = ph.dx ** 2
    med = O.medium_from(ph)
    ad, _ = _batches(O, med, [O.Source(O.MAP, map=_pixel_map(ph, *d, 1.0 / A))],
                     dict(seed=9, n_harm=2, stream_tag=1, adjoint=1), B=8, n_per=25_000)
    a1, se = batch_mean_se(ad[:, 1][:, s[0], s[1]])
    assert abs(a1) > 8 * se


# ---------------------------------------------------------------- gradient algebra (Sec. 5)
def _fourier(phi_vals, t, N):
    dt = t[1] - t[0]
    c = [np.sum(phi_vals) * dt]
    c += [np.sum(phi_vals * np.cos(n * t)) * dt for n in range(1, N + 1)]
    c += [np.sum(phi_vals * np.sin(n * t)) * dt for n in range(1, N + 1)]
    return np.array(c)


def test_gradient_formulas_against_angular_quadrature(oracle_lib):
    """eqs. grad_2D_abs_integral3 and scattering_gradient3 versus direct quadrature
    of int phi phi* dt and int int phi* P phi' dt dt' (eq. scattering2D), for smooth
    angular fields with known harmonic coefficients a_n = int phi cos(nt) dt."""
    O = oracle_lib
    M, N = 2048, 32
    t = (np.arange(M) + 0.5) / M * 2 * np.pi - np.pi
    dt = t[1] - t[0]
    rng = np.random.default_rng(1)
    nz, nx = 2, 3
    fwd = np.zeros((2 * N + 1, nz, nx))
    adj = np.zeros_like(fwd)
    exp_a, exp_s = np.zeros((nz, nx)), np.zeros((nz, nx))
    mua = rng.uniform(0.05, 0.5, (nz, nx))
    g = rng.uniform(0.1, 0.95, (nz, nx))
    hm = rng.uniform(0.0, 1.0, (nz, nx))
    dx = 0.7
    for iz in range(nz):
        for ix in range(nx):
            k1, k2, al, be = rng.uniform(0.5, 3), rng.uniform(0.5, 3), rng.uniform(-3, 3), rng.uniform(-3, 3)
            phi = np.exp(k1 * np.cos(t - al)) + 0.3
            phs = np.exp(k2 * np.cos(t - be)) - 0.8          # adjoint fields may be signed
            fwd[:, iz, ix] = _fourier(phi, t, N)
            adj[:, iz, ix] = _fourier(phs, t, N)
            gg = g[iz, ix]
            D = t[:, None] - t[None, :]
            Pm = (1 - gg ** 2) / (2 * np.pi * (1 + gg ** 2 - 2 * gg * np.cos(D)))
            a0 = fwd[0, iz, ix]
            both = np.sum(phi * phs) * dt
            exp_a[iz, ix] = -a0 * (hm[iz, ix] - mua[iz, ix] * a0) + both
            exp_s[iz, ix] = both - phs @ Pm @ phi * dt * dt
    med = O.Medium(mua, np.ones((nz, nx)), g, dx)
    dmua, dmus = O.gradient(med, N, fwd, adj, hm)
    np.testing.assert_allclose(dmua, dx * dx * exp_a, rtol=1e-9)
    np.testing.assert_allclose(dmus, dx * dx * exp_s, rtol=1e-6, atol=1e-9 * np.abs(exp_s).max())


def test_detector_readout_against_quadrature(oracle_lib):
    """<phi, b> from harmonic maps equals the angular integral of phi b (orthogonality)."""
    O = oracle_lib
    M, N = 1024, 16
    t = (np.arange(M) + 0.5) / M * 2 * np.pi - np.pi
    phi = np.exp(1.5 * np.cos(t - 0.4)) + 0.2
    b = np.sin(2 * t) ** 2 / np.pi
    f = _fourier(phi, t, N)[:, None, None]
    d = _fourier(b, t, N)[:, None, None]
    med = O.Medium(np.ones((1, 1)), np.ones((1, 1)), np.zeros((1, 1)), 0.5)
    assert O.detect(med, N, f, d) == pytest.approx(0.25 * np.sum(phi * b) * (t[1] - t[0]), rel=1e-10)


def test_residual_definition(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(2)
    mua = rng.uniform(0.01, 0.1, (3, 4))
    co = rng.uniform(0, 2, (5, 3, 4))
    hm = rng.uniform(0, 0.2, (3, 4))
    med = O.Medium(mua, np.ones((3, 4)), np.zeros((3, 4)), 0.2)
    eps, q = O.residual(med, co, hm)
    r = hm - mua * co[0]
    assert eps == pytest.approx(0.5 * 0.04 * np.sum(r * r), rel=1e-14)
    np.testing.assert_allclose(q, mua * r, rtol=1e-15)


def test_harmonic_tally_parseval_against_binned_radiance(oracle_lib):
    """The harmonic tally and an angle-binned tally of the same packets agree:
    int phi phi* dt from 360 bins equals a0 a0*/2pi + (1/pi) sum (a a* + b b*)
    (Sec. 5, orthogonality), in a diffusive pixel, within binning + truncation error."""
    O = oracle_lib
    ph = P.homogeneous(8, 8, 0.5, 0.05, 4.0, 0.6)
    med = O.medium_from(ph)
    N = 24
    src_f = O.sources_from([P.point_source(1.1, 1.3)])
    src_a = [O.Source(O.MAP, map=_pixel_map(ph, 5, 5, 1.0))]
    f, _, fb = O.run_mc(med, src_f, O.Run(200_000, 1, N), n_threads=8, n_bins=360)
    a, _, ab = O.run_mc(med, src_a, O.Run(200_000, 2, N, stream_tag=1, adjoint=1), n_threads=8, n_bins=360)
    dtb = 2 * np.pi / 360
    for (iz, ix) in [(4, 4), (5, 3), (3, 6)]:
        binned = np.sum(fb[:, iz, ix] * ab[:, iz, ix]) * dtb
        harm = f[0, iz, ix] * a[0, iz, ix] / (2 * np.pi) + np.sum(
            f[1:, iz, ix] * a[1:, iz, ix]) / np.pi
        assert harm == pytest.approx(binned, rel=0.03), (iz, ix, harm, binned)


def test_signed_map_source_quadrature(oracle_lib):
    """Volumetric isotropic source (Sec. 6: launch spread uniformly over the source
    pixel, isotropic, weight sign of q*) in a non-scattering medium: brute-force
    quadrature over source positions and angles with exact chords, midpoint rules
    at two resolutions Richardson-extrapolated (the error is second order)."""
    O = oracle_lib
    rng = np.random.default_rng(13)
    nz, nx, dx, N = 4, 4, 0.5, 2
    mua = rng.uniform(0.1, 1.5, size=(nz, nx))
    q = np.zeros((nz, nx))
    q[1, 1], q[2, 3] = 0.7, -0.4

    def quad(npos, nang):
        e = np.zeros((2 * N + 1, nz, nx))
        for (iz, ix) in [(1, 1), (2, 3)]:
            for a in (np.arange(npos) + 0.5) / npos:
                for b in (np.arange(npos) + 0.5) / npos:
                    for t in (np.arange(nang) + 0.5) / nang * 2 * np.pi - np.pi:
                        e += q[iz, ix] * ballistic_tally(mua, dx, (ix + a) * dx, (iz + b) * dx, t, N) \
                            * (dx * dx / npos ** 2) * (2 * np.pi / nang)
        return e

    coarse, fine = quad(6, 180), quad(12, 360)
    exp = fine + (fine - coarse) / 3.0
    med = O.Medium(mua, np.zeros((nz, nx)), np.zeros((nz, nx)), dx)
    outs, _ = _batches(O, med, [O.Source(O.MAP, map=q)], dict(seed=5, n_harm=N), B=10, n_per=20_000)
    mean, se = batch_mean_se(outs)
    z = np.abs(mean - exp) / np.maximum(se, 1e-12)
    assert np.max(z) < 5.0, np.max(z)
    assert np.abs(mean[0] - exp[0]).max() < 0.02 * np.abs(exp[0]).max()


def test_gradient_chain_matches_finite_differences(oracle_lib):
    """The whole adjoint chain -- forward tally, residual and adjoint source
    q* = mua (Hmeas - H) (Sec. 6), adjoint MC with mirrored output (Sec. 4),
    harmonic-product gradients (Sec. 5) -- against central finite differences of
    the discrete error functional eps = A/2 sum (Hmeas - mua a0)^2 (Sec. 2).

    d/d mua: common random numbers make the finite difference nearly noiseless
    (packet paths do not depend on mua), so per-pixel and directional
    derivatives are compared within 4 standard errors of the adjoint estimate
    plus 0.5% for the pixel-average discretisation of the products.
    d/d mus along a smooth direction: paths change with mus, so the finite
    difference is averaged over seeds and both errors enter the bound."""
    O = oracle_lib
    nz = nx = 12
    dx = 0.25
    ph = P.homogeneous(nx, nz, dx, 0.15, 3.0, 0.7)
    ph.mua[4:8, 3:6] = 0.4
    ph.mus[6:10, 7:10] = 6.0
    src = O.sources_from([P.SourceSpec("line", 0.0, 0.0, nx * dx, 0.0, 0.0, 1.0, 0, 1.0)])
    N = 8
    c = (np.arange(nx) + 0.5) * dx
    X, Z = np.meshgrid(c, c)
    hm = 0.12 + 0.05 * np.cos(2 * X) * np.exp(-Z)
    mua0, mus0 = ph.mua.astype(float), ph.mus.astype(float)
    Np = 400_000

    def eps_of(mua, mus, seed=0):
        med = O.Medium(mua, mus, ph.g, dx)
        co, _ = O.run_mc(med, src, O.Run(Np, seed, N), n_threads=8)
        e, q = O.residual(med, co, hm)
        return e, co, q

    _, co, q = eps_of(mua0, mus0)
    med = O.Medium(mua0, mus0, ph.g, dx)
    grads = []
    for b in range(6):
        ad, _ = O.run_mc(med, [O.Source(O.MAP, map=q)], O.Run(Np, 100 + b, N, stream_tag=1, adjoint=1), n_threads=8)
        grads.append(O.gradient(med, N, co, ad, hm))
    Ga = np.array([g[0] for g in grads])
    Gs = np.array([g[1] for g in grads])
    for (iz, ix) in [(6, 6), (8, 2), (5, 9), (9, 9), (3, 4)]:
        h = 0.01 * mua0[iz, ix]
        mp, mm = mua0.copy(), mua0.copy()
        mp[iz, ix] += h
        mm[iz, ix] -= h
        fd = (eps_of(mp, mus0)[0] - eps_of(mm, mus0)[0]) / (2 * h)
        g, se = batch_mean_se(Ga[:, iz, ix])
        assert abs(g - fd) < 4 * se + 5e-3 * abs(fd), ((iz, ix), g, fd, se)
    v = np.exp(-((X - 1.5) ** 2 + (Z - 1.7) ** 2) / 0.5)
    h = 0.02 * mua0.mean()
    fd = (eps_of(mua0 + h * v, mus0)[0] - eps_of(mua0 - h * v, mus0)[0]) / (2 * h)
    g, se = batch_mean_se((Ga * v).sum(axis=(1, 2)))
    assert abs(g - fd) < 4 * se + 5e-3 * abs(fd), (g, fd, se)
    h = 0.02 * mus0.mean()
    fds = np.array([(eps_of(mua0, mus0 + h * v, seed=10 + s)[0] - eps_of(mua0, mus0 - h * v, seed=10 + s)[0]) / (2 * h)
                    for s in range(4)])
    fm, fse = batch_mean_se(fds)
    g, se = batch_mean_se((Gs * v).sum(axis=(1, 2)))
    assert g > 0 and fm > 0
    assert abs(g - fm) < 4 * np.hypot(se, fse) + 5e-3 * abs(fm), (g, fm, se, fse)


def test_side_sources_deliver_equal_power(oracle_lib):
    """Four collimated line sources, one per side of a homogeneous square whose side
    (96 x 0.1 mm) is not exactly representable: by the square's symmetry each side
    delivers the same absorbed power.  Guards the rule that a source on the outer
    boundary, pointing inward, starts inside the domain."""
    O = oracle_lib
    ph = P.homogeneous(96, 96, 0.1, 0.05, 4.0, 0.8)
    med = O.medium_from(ph)
    specs = P.four_side_lines(ph)
    vals = []
    for s in specs:
        _, L = O.run_mc(med, O.sources_from([s]), O.Run(4000, 0, 0), n_threads=8)
        vals.append(L.absorbed / L.launched)
    vals = np.array(vals)
    assert np.all(vals > 0.05)
    assert vals.max() - vals.min() < 0.1 * vals.mean(), vals


def test_equal_count_map_launch_is_unbiased(oracle_lib):
    """Sec. 6 read literally (every pixel equally likely, launch weight ~ q_i)
    and the importance-sampled launch (pixels ~ |q_i|, weight sign q_i) are two
    unbiased estimators of the same field: their maps agree within the
    combined standard error, and both ledgers balance.  A wrong weight scale
    in the equal-count branch (e.g. a missing 1/mean|q|) fails this."""
    O = oracle_lib
    ph = P.disc_phantom(16, 0.5, 0.05, 4.0, 0.7, seed=8, radius=(1.0, 2.0))
    q = P.residual_like_map(ph, seed=5)
    q[:4, :] = 0.0                                   # pixels with no source at all
    med, src = O.medium_from(ph), O.sources_from([P.map_source(q)])
    outs = {0: [], O.FLAG_EQUAL_COUNT: []}
    for flag in outs:
        for b in range(8):
            r = O.Run(20_000, 40 + b, 3, stream_tag=1, adjoint=1, flags=flag)
            m, led = O.run_mc(med, src, r, n_threads=8)
            bal = led.launched + led.roulette_gain - led.roulette_loss - led.absorbed - led.escaped
            assert abs(bal) < 1e-9 * max(abs(led.launched), 1.0)
            outs[flag].append(m)
    a, b = np.array(outs[0]), np.array(outs[O.FLAG_EQUAL_COUNT])
    ma, mb = a.mean(0), b.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / len(a) + b.var(0, ddof=1) / len(b))
    big = np.abs(ma[0]) > 0.05 * np.abs(ma[0]).max()
    z = np.abs(ma - mb)[:, big] / np.maximum(se[:, big], 1e-300)
    assert np.mean(z < 3) > 0.98 and np.max(z) < 6, (np.mean(z < 3), np.max(z))
    # the summed absorbed power agrees too (a global check of the normalisation)
    pa, pb = (ph.mua * a[:, 0]).sum((1, 2)), (ph.mua * b[:, 0]).sum((1, 2))
    assert abs(pa.mean() - pb.mean()) < 3 * np.sqrt(pa.var(ddof=1) / 8 + pb.var(ddof=1) / 8)


# ---------------------------------------------------------------- roulette law (Sec. 3, Sec. 6)
def _roulette_case():
    """A medium where most packets fall below w_th = 0.05 before they leave:
    strong absorption (albedo 0.91) and scattering in a small square."""
    ph = P.homogeneous(8, 8, 0.5, 2.0, 20.0, 0.0)
    return ph, P.pencil_top_centre(ph)


def test_roulette_maps_match_a_negligible_threshold(oracle_lib):
    """Russian roulette at w_th = 0.05 (survive with 1/m, weight x m, m = 4)
    is an unbiased termination: its maps agree within the standard error with
    those of w_th = 1e-8, where roulette (almost) never fires and packets end
    only by escape.  Roulette here kills a large share of the packets, so a
    wrong survival branch (probability or weight factor) shifts every map."""
    O = oracle_lib
    ph, specs = _roulette_case()
    med, src = O.medium_from(ph), O.sources_from(specs)
    res = {}
    for wth in (0.05, 1e-8):
        outs, leds = _batches(O, med, src, dict(seed=6, n_harm=3, w_threshold=wth, roulette_m=4.0), B=8,
                              n_per=40_000)
        res[wth] = (outs, leds)
    high = res[0.05][1]
    launched = sum(l.launched for l in high)
    # roulette decides the fate of a large share of the packets: its kills
    # remove at least 20% of them (each kill carries less than w_th of weight,
    # so loss / w_th bounds the number of kills from below)
    assert sum(l.roulette_loss for l in high) / 0.05 > 0.2 * launched
    assert sum(l.roulette_gain for l in high) > 0.01 * launched
    assert sum(l.roulette_gain for l in res[1e-8][1]) < 1e-6 * launched
    a, b = res[0.05][0], res[1e-8][0]
    ma, mb = a.mean(0), b.mean(0)
    se = np.sqrt(a.var(0, ddof=1) / len(a) + b.var(0, ddof=1) / len(b))
    big = np.abs(ma[0]) > 0.02 * np.abs(ma[0]).max()
    z = np.abs(ma - mb)[:, big] / np.maximum(se[:, big], 1e-300)
    assert np.mean(z < 3) > 0.97 and np.max(z) < 5.5, (np.mean(z < 3), np.max(z))
    # the absorbed power of the whole map agrees too
    pa, pb = (ph.mua * a[:, 0]).sum((1, 2)), (ph.mua * b[:, 0]).sum((1, 2))
    assert abs(pa.mean() - pb.mean()) < 3.5 * np.sqrt(pa.var(ddof=1) / 8 + pb.var(ddof=1) / 8)


def test_roulette_expected_gain_equals_expected_loss(oracle_lib):
    """At a roulette event of weight W, survival with probability 1/m and
    weight m W gains (m-1) W with probability 1/m and loses W with
    probability 1 - 1/m: the expected gain and loss are both (1 - 1/m) W.
    So the per-packet mean of (gain - loss) is zero within its standard
    error, while the gain itself is far from zero.  A survival probability p
    other than 1/m with the weight factor m makes gain / loss = (m-1) p / (1-p)."""
    O = oracle_lib
    ph, specs = _roulette_case()
    med, src = O.medium_from(ph), O.sources_from(specs)
    for m in (4.0, 10.0):
        _, leds = _batches(O, med, src, dict(seed=9, n_harm=0, w_threshold=0.05, roulette_m=m), B=16,
                           n_per=20_000)
        net = np.array([(l.roulette_gain - l.roulette_loss) / l.launched for l in leds])
        gain = np.array([l.roulette_gain / l.launched for l in leds])
        mn, se = batch_mean_se(net)
        mg, _ = batch_mean_se(gain)
        assert mg > 30 * se, (m, mg, se)
        assert abs(mn) < 4 * se, (m, mn, se)


# ---------------------------------------------------------------- angular source profiles
def test_point_source_profile_quadrature(oracle_lib):
    """A point source with an angular profile of cosine and sine terms up to
    order 5 (p = c0/2pi + (1/pi) sum (c_n cos nt + s_n sin nt), the expansion
    of Sec. 3.1) in a non-scattering medium: the maps equal the angular
    quadrature of p(t) times the exact attenuated chords.  Every coefficient
    of the profile, its sign and its cosine/sine role shows in the maps."""
    O = oracle_lib
    rng = np.random.default_rng(17)
    nz, nx, dx, N = 5, 5, 1.0, 6
    mua = rng.uniform(0.05, 0.8, size=(nz, nx))
    x0, z0 = 2.3, 2.6
    n = 5
    prof = np.zeros(2 * n + 1)
    prof[0] = 1.0
    prof[1:n + 1] = [0.3, -0.2, 0.15, 0.1, -0.08]        # c_1..c_5
    prof[n + 1:] = [0.25, 0.12, -0.18, 0.07, 0.05]       # s_1..s_5
    M = 4000
    exp = np.zeros((2 * N + 1, nz, nx))
    for t in (np.arange(M) + 0.5) / M * 2 * np.pi - np.pi:
        p = prof[0] / (2 * np.pi) + sum(prof[k] * np.cos(k * t) + prof[n + k] * np.sin(k * t)
                                        for k in range(1, n + 1)) / np.pi
        exp += 2 * np.pi * p * ballistic_tally(mua, dx, x0, z0, t, N)
    exp /= M
    med = O.Medium(mua, np.zeros((nz, nx)), np.zeros((nz, nx)), dx)
    src = [O.Source(O.POINT, x0=x0, z0=z0, prof=prof)]
    outs, _ = _batches(O, med, src, dict(seed=3, n_harm=N), B=10, n_per=30_000)
    mean, se = batch_mean_se(outs)
    z = np.abs(mean - exp) / np.maximum(se, 1e-12)
    assert np.max(z) < 5.0, np.max(z)
    # the profile's own harmonics reach the tally: the source pixel's a_n, b_n
    # track c_n, s_n (an isotropic or cosine-only profile would not)
    assert np.abs(mean[N + 1:N + n + 1]).max() > 20 * se[N + 1:N + n + 1].max()


# ---------------------------------------------------------------- reciprocity at the paper's validation geometry
def _e2_setup():
    """The adjoint validation geometry of Sec. 4.1: 40 mm x 40 mm on 101 x 101
    pixels, 10 harmonics, source at the centre, detectors on the line 23.6 mm
    deep.  The paper gives no optical properties for it; those of its forward
    validation (mua 0.01, mus 10 1/mm, g 0.9) are used."""
    n = 101
    ph = P.homogeneous(n, n, 40.0 / n, 0.01, 10.0, 0.9)
    dx = ph.dx
    s = (int(20.0 / dx), int(20.0 / dx))                 # (iz, ix) of the centre
    d = (int(23.6 / dx), int(21.4 / dx))                 # a detector pixel on the line z = 23.6 mm
    return ph, s, d


def test_reciprocity_anisotropic_detector_e2(oracle_lib):
    """Case 2 of Sec. 4.1 (eq. adj_definition): an isotropic source and a
    detector with angular weight sin^2(2(t - alpha))/pi, rotated by alpha so
    that the profile has a sine term of order 4 as well as a cosine term.  The
    forward readout int phi P_d dt = c0 a0 + 2 (c4 a4 + s4 b4) at the
    detector equals the adjoint field (detector as source, profile mirrored
    for the adjoint) read isotropically at the source."""
    O = oracle_lib
    ph, s, d = _e2_setup()
    A = ph.dx ** 2
    med = O.medium_from(ph)
    al = 0.3
    prof = np.zeros(9)                                   # P_d = 2 pi p: c0, c1..c4, s1..s4
    prof[0] = 1 / (2 * np.pi)
    prof[4] = -np.cos(4 * al) / (4 * np.pi)
    prof[8] = -np.sin(4 * al) / (4 * np.pi)
    N = 10
    fwd_src = [O.Source(O.MAP, map=_pixel_map(ph, *s, 1.0 / (2 * np.pi * A)))]
    adj_src = [O.Source(O.MAP, map=_pixel_map(ph, *d, 1.0 / A), prof=prof)]
    fo, _ = _batches(O, med, fwd_src, dict(seed=31, n_harm=N), B=8, n_per=12_500)
    ad, _ = _batches(O, med, adj_src, dict(seed=32, n_harm=N, stream_tag=1, adjoint=1), B=8, n_per=12_500)
    lhs = (prof[0] * fo[:, 0] + 2 * (prof[4] * fo[:, 4] + prof[8] * fo[:, N + 4]))[:, d[0], d[1]]
    rhs = ad[:, 0][:, s[0], s[1]] / (2 * np.pi)
    ml, sl = batch_mean_se(lhs)
    mr, sr = batch_mean_se(rhs)
    assert abs(ml - mr) < 4 * np.hypot(sl, sr), (ml, mr, sl, sr)
    assert abs(ml - mr) < 0.1 * abs(ml)


def test_reciprocity_distributed_e2(oracle_lib):
    """Case 3 of Sec. 4.1: a distributed isotropic source density S(x) and a
    distributed isotropic detector D(x) (smooth blobs, signed detector):
    <L S, D> = sum_i A D_i a0_i of the forward field equals
    <S, L* D> = sum_i A S_i a0*_i of the adjoint field whose source is D."""
    O = oracle_lib
    ph, _, _ = _e2_setup()
    A = ph.dx ** 2
    c = (np.arange(ph.nx) + 0.5) * ph.dx
    X, Z = np.meshgrid(c, c)
    S = np.exp(-((X - 18.0) ** 2 + (Z - 19.0) ** 2) / (2 * 1.5 ** 2))
    D = np.exp(-((X - 21.5) ** 2 + (Z - 23.6) ** 2) / (2 * 1.0 ** 2)) \
        - 0.3 * np.exp(-((X - 25.0) ** 2 + (Z - 20.0) ** 2) / (2 * 1.2 ** 2))
    med = O.medium_from(ph)
    N = 10
    fo, _ = _batches(O, med, [O.Source(O.MAP, map=S)], dict(seed=41, n_harm=N), B=8, n_per=12_500)
    ad, _ = _batches(O, med, [O.Source(O.MAP, map=D)], dict(seed=42, n_harm=N, stream_tag=1, adjoint=1), B=8,
                     n_per=12_500)
    lhs = (fo[:, 0] * D).sum((1, 2)) * A
    rhs = (ad[:, 0] * S).sum((1, 2)) * A
    ml, sl = batch_mean_se(lhs)
    mr, sr = batch_mean_se(rhs)
    # the comparison resolves the readout to a few percent, and both sides agree within it
    assert np.hypot(sl, sr) < 0.05 * abs(ml), (ml, sl, sr)
    assert abs(ml - mr) < 4 * np.hypot(sl, sr), (ml, mr, sl, sr)

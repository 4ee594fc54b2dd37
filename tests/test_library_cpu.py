"""Host-side checks of librmc.so that need no GPU: it loads, exports every entry
point declared in include/*.h, its structs match the binding, and invalid
arguments are rejected on the host before anything touches a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1608_05238_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1608_05238_amd import build
        build.build()
    return L, L.load()


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b((?:mc|dn|mb)_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_entry_point():
    L, lib = _lib()
    declared = _declared_functions()
    assert "mc_forward" in declared and "mc_adjoint" in declared and "mc_gradient" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(L.SYMBOLS)


def test_struct_layouts():
    L, _ = _lib()
    assert C.sizeof(L.mc_event) == 48
    assert C.sizeof(L.mc_ledger) == 88
    assert C.sizeof(L.mc_tuning) == 56 and C.sizeof(L.mc_options) == 16
    assert C.sizeof(L.mc_run) == 48
    assert C.sizeof(L.mc_medium) == 40


def test_status_strings_and_build_info():
    L, lib = _lib()
    assert lib.mc_status_string(0) == b"ok"
    assert b"invalid" in lib.mc_status_string(1)
    assert b"gfx950" in lib.mc_build_info()


def _medium(L, nx=4, nz=4, dx=0.5, ptr=0x1000):
    return L.mc_medium(nx, nz, dx, ptr, ptr, ptr)


def _pencil(L):
    s = L.mc_source()
    s.kind, s.x0, s.z0, s.dir_x, s.dir_z, s.power = L.MC_SRC_PENCIL, 1.0, 0.0, 0.0, 1.0, 1.0
    return s


@pytest.mark.parametrize("bad", ["nx", "harm", "packets", "power", "outside", "dir", "roulette", "nsrc", "flags"])
def test_invalid_arguments_rejected_on_host(bad):
    """Every check runs before any HIP call, so these need no GPU."""
    L, lib = _lib()
    m = _medium(L)
    src = (L.mc_source * 1)(_pencil(L))
    run = L.mc_run(1000, 0, 0, 0, 4, 1e-4, 10.0, 0)
    n_src = 1
    if bad == "nx":
        m.nx = 0
    elif bad == "harm":
        run.n_harm = L.MC_NHARM_MAX + 1
    elif bad == "packets":
        run.n_packets = 0
    elif bad == "power":
        src[0].power = 0.0
    elif bad == "outside":
        src[0].x0 = 5.0
    elif bad == "dir":
        src[0].dir_x = 1.0
    elif bad == "roulette":
        run.roulette_m = 1.0
    elif bad == "nsrc":
        n_src = 9
    elif bad == "flags":
        run.flags = 4
    assert lib.mc_workspace_bytes(C.byref(m), src, n_src, C.byref(run), None) == 0
    rc = lib.mc_forward(C.byref(m), src, n_src, C.byref(run), None, 0x2000, None, 0x3000, 1 << 30, None)
    assert rc == L.MC_ERR_INVALID_ARG


def test_map_source_must_be_alone_and_workspace_checked():
    L, lib = _lib()
    m = _medium(L)
    a = L.mc_source()
    a.kind, a.map_d = L.MC_SRC_MAP, 0x4000
    srcs = (L.mc_source * 2)(a, _pencil(L))
    run = L.mc_run(1000, 0, 0, 0, 4, 1e-4, 10.0, 0)
    assert lib.mc_workspace_bytes(C.byref(m), srcs, 2, C.byref(run), None) == 0
    one = (L.mc_source * 1)(_pencil(L))
    need = lib.mc_workspace_bytes(C.byref(m), one, 1, C.byref(run), None)
    assert need > 0
    rc = lib.mc_forward(C.byref(m), one, 1, C.byref(run), None, 0x2000, None, 0x3000, need - 1, None)
    assert rc == L.MC_ERR_WORKSPACE
    rc = lib.mc_forward(C.byref(m), one, 1, C.byref(run), None, 0x2000, None, 0x3001, need + 256, None)
    assert rc == L.MC_ERR_WORKSPACE


def test_workspace_grows_with_grid_and_harmonics():
    L, lib = _lib()
    one = (L.mc_source * 1)(_pencil(L))
    small = lib.mc_workspace_bytes(C.byref(_medium(L, 4, 4)), one, 1, C.byref(L.mc_run(10, 0, 0, 0, 2, 1e-4, 10.0, 0)), None)
    big = lib.mc_workspace_bytes(C.byref(_medium(L, 256, 256, 0.1)), one, 1,
                                 C.byref(L.mc_run(10, 0, 0, 0, 16, 1e-4, 10.0, 0)), None)
    assert big > 65536 * 33 * 8 > small > 0


def test_tuning_is_per_call_and_checked():
    """The defaults round-trip through mc_default_tuning; a call's tuning
    (mc_options) sizes its queues -- the library keeps none -- and a tuning
    out of range makes the call invalid (host only)."""
    L, lib = _lib()
    from paper_1608_05238_amd import rmc
    d = rmc.default_tuning()
    assert d == {"live_packets": 1 << 26, "job_packets": 16384, "max_visits": 64, "tile": 0,
                 "finish_packets": 1 << 16, "grid_max_packets": 1 << 21, "flush_track": 65536.0,
                 "tail_visits": 1, "max_generations": 0, "min_job_packets": 1024, "quiet_percent": 50}
    m = _medium(L)
    m.nx = m.nz = 256
    src = (L.mc_source * 1)(_pencil(L))
    run = L.mc_run(1 << 26, 0, 0, 0, 16, 1e-4, 10.0, 0)

    def ws(t):
        return lib.mc_workspace_bytes(C.byref(m), src, 1, C.byref(run), rmc._Options(t, None).ref())

    small = ws({"live_packets": 1 << 20})
    big = ws({"live_packets": 1 << 22, "job_packets": 1024, "max_visits": 7, "tile": 9})
    assert big > small + 3 * (1 << 20) * 64 * 2
    assert ws(None) == lib.mc_workspace_bytes(C.byref(m), src, 1, C.byref(run), None) > big
    # the same call again is unchanged: nothing was kept
    assert ws({"live_packets": 1 << 20}) == small
    for bad in ({"live_packets": 10}, {"job_packets": 1}, {"tile": 1000}, {"flush_track": 1e6},
                {"flush_track": -1.0}, {"flush_track": float("nan")}, {"tail_visits": (1 << 30) + 1},
                {"max_generations": 70000}, {"min_job_packets": 10}, {"quiet_percent": 101}):
        assert ws(bad) == 0, bad
        rc = lib.mc_forward(C.byref(m), src, 1, C.byref(run), rmc._Options(bad, None).ref(), 0x2000, None, 0x3000,
                            1 << 40, None)
        assert rc == L.MC_ERR_INVALID_ARG, bad


def test_timer_handles():
    """mc_timer: created and destroyed on the host; an empty timer reads zero."""
    L, lib = _lib()
    h = C.c_void_p()
    assert lib.mc_timer_create(C.byref(h)) == 0 and h.value
    ms, n = C.c_double(1.0), C.c_uint64(7)
    assert lib.mc_timer_read(h, C.byref(ms), C.byref(n), 1) == 0
    assert ms.value == 0.0 and n.value == 0
    assert lib.mc_timer_destroy(h) == 0
    assert lib.mc_timer_create(None) == L.MC_ERR_INVALID_ARG
    assert lib.mc_timer_read(None, None, None, 0) == L.MC_ERR_INVALID_ARG


def test_batch_arguments_checked_on_host():
    """mc_batch_workspace_bytes / mc_run_batch reject empty or oversized
    batches, mixed harmonic orders and invalid problems before any GPU work."""
    L, lib = _lib()
    m = _medium(L)
    src = (L.mc_source * 1)(_pencil(L))
    run4 = L.mc_run(1000, 0, 0, 0, 4, 1e-4, 10.0, 0)
    run5 = L.mc_run(1000, 0, 0, 0, 5, 1e-4, 10.0, 0)
    ok = L.mc_problem(m, src, 1, run4, 0, 0x2000, None)
    assert lib.mc_batch_workspace_bytes((L.mc_problem * 1)(ok), 1, None) > 0
    assert lib.mc_batch_workspace_bytes((L.mc_problem * 1)(ok), 0, None) == 0
    assert lib.mc_batch_workspace_bytes(None, 1, None) == 0
    mixed = (L.mc_problem * 2)(ok, L.mc_problem(m, src, 1, run5, 0, 0x2000, None))
    assert lib.mc_batch_workspace_bytes(mixed, 2, None) == 0
    assert lib.mc_run_batch(mixed, 2, None, 0x3000, 1 << 30, None) == L.MC_ERR_INVALID_ARG
    bad = L.mc_problem(m, src, 1, L.mc_run(0, 0, 0, 0, 4, 1e-4, 10.0, 0), 0, 0x2000, None)
    assert lib.mc_run_batch((L.mc_problem * 1)(bad), 1, None, 0x3000, 1 << 30, None) == L.MC_ERR_INVALID_ARG
    nocoeffs = L.mc_problem(m, src, 1, run4, 0, None, None)
    assert lib.mc_run_batch((L.mc_problem * 1)(nocoeffs), 1, None, 0x3000, 1 << 30, None) == L.MC_ERR_INVALID_ARG
    assert lib.mc_run_batch((L.mc_problem * 1)(ok), 5000, None, 0x3000, 1 << 30, None) == \
        L.MC_ERR_INVALID_ARG
    # too small a workspace is reported before anything is enqueued
    assert lib.mc_run_batch((L.mc_problem * 1)(ok), 1, None, 0x3000, 16, None) == L.MC_ERR_WORKSPACE


def test_denoiser_arguments_checked_on_host():
    L, lib = _lib()
    assert lib.dn_conv3x3_fwd(None, 0x1000, None, 0x2000, 1, 1, 1, 4, 4, None) == L.MC_ERR_INVALID_ARG
    assert lib.dn_conv3x3_fwd(0x1000, 0x1000, None, 0x2000, 0, 1, 1, 4, 4, None) == L.MC_ERR_INVALID_ARG
    assert lib.dn_conv3x3_wgrad(0x1000, 0x1000, 0x2000, 1, 1, 1, 4, -1, None) == L.MC_ERR_INVALID_ARG
    # channels-last operands: a multiple of 8 channels, 16-byte aligned rows
    assert lib.dn_conv3x3_fwd(0x1000, 0x1000, None, 0x2000, 1, 12, 8, 4, 4, None) == L.MC_ERR_INVALID_ARG
    assert lib.dn_conv3x3_fwd(0x1008, 0x1000, None, 0x2000, 1, 8, 8, 4, 4, None) == L.MC_ERR_INVALID_ARG
    assert lib.dn_conv3x3_fwd(0x1000, 0x1000, None, 0x2004, 1, 8, 8, 4, 4, None) == L.MC_ERR_INVALID_ARG
    assert lib.dn_conv3x3_wgrad(0x1000, 0x1000, 0x2000, 1, 8, 12, 4, 4, None) == L.MC_ERR_INVALID_ARG
    assert lib.dn_conv3x3_wgrad(0x1000, 0x1008, 0x2000, 1, 8, 8, 4, 4, None) == L.MC_ERR_INVALID_ARG


def test_microbenchmark_arguments_checked_on_host():
    L, lib = _lib()
    bad = L.MC_ERR_INVALID_ARG
    sink = 0x1000
    # LDS kinds, block shape and LDS size are checked before any launch
    assert lib.mb_lds_atomics(9, 65536, 512, 8, 4, 0, sink, None, None) == bad
    assert lib.mb_lds_atomics(L.MB_LDS_ADD_F64, 65536, 500, 8, 4, 0, sink, None, None) == bad
    assert lib.mb_lds_atomics(L.MB_LDS_ADD_F64, 65536, 2048, 8, 4, 0, sink, None, None) == bad
    assert lib.mb_lds_atomics(L.MB_LDS_ADD_F64, 160 * 1024 + 8, 512, 8, 4, 0, sink, None, None) == bad
    assert lib.mb_lds_atomics(L.MB_LDS_ADD_F64, 512, 512, 8, 4, 0, sink, None, None) == bad
    assert lib.mb_lds_atomics(L.MB_LDS_ADD_F64, 65540, 512, 8, 4, 0, sink, None, None) == bad
    assert lib.mb_lds_atomics(L.MB_LDS_ADD_F64, 65536, 512, 0, 4, 0, sink, None, None) == bad
    assert lib.mb_lds_atomics(L.MB_LDS_ADD_F64, 65536, 512, 8, 4, 0, None, None, None) == bad
    assert lib.mb_global_atomics_f64(sink, 0, 8, 4, 0, None) == bad
    assert lib.mb_global_atomics_f64(sink, 1 << 32, 8, 4, 0, None) == bad
    for args in ((0, 33, 8, 4), (10, 0, 8, 4), (10, 5000, 8, 4), (1 << 28, 33, 8, 4), (10, 33, 0, 4), (10, 33, 8, 0)):
        assert lib.mb_global_atomics_rows_f64(sink, *args, 0, None) == bad, args
    assert lib.mb_copy(0x1000, 0x1008, 4, None) == bad          # misaligned destination
    assert lib.mb_copy(0x1000, 0x1010, 4, None) == bad          # overlapping
    assert lib.mb_copy(None, 0x100000, 4, None) == bad
    assert lib.mb_fma_f32(None, 8, 4, None, None) == bad
    assert lib.mb_wall_clock_khz(0, None) == bad


def test_weight_bound_beyond_the_fixed_point_range_is_unsupported():
    """The tile tally is 64-bit fixed point scaled by 2^(32 - e), 2^e >= the
    largest packet weight; a profile or roulette gain that could exceed 2^32
    is refused on the host.  The bound is |c0| + 2 sum |c_n|, times the
    roulette factor max(1, m W_th)."""
    L, lib = _lib()
    m = _medium(L)
    prof = (C.c_double * 3)(1.0, 0.5, 0.0)            # N = 1: c0, c1, s1 -> bound 2
    pt = L.mc_source()
    pt.kind, pt.x0, pt.z0, pt.power, pt.prof_h, pt.n_prof = L.MC_SRC_POINT, 1.0, 1.0, 1.0, prof, 1
    src = (L.mc_source * 1)(pt)
    run = L.mc_run(1000, 0, 0, 0, 4, 1e-4, 10.0, 0)
    assert lib.mc_workspace_bytes(C.byref(m), src, 1, C.byref(run), None) > 0
    run.w_threshold, run.roulette_m = 1.0, 2.0 ** 31      # 2 x 2^31 = 2^32: still inside
    assert lib.mc_workspace_bytes(C.byref(m), src, 1, C.byref(run), None) > 0
    run.roulette_m = 2.0 ** 32                           # 2^33
    assert lib.mc_workspace_bytes(C.byref(m), src, 1, C.byref(run), None) == 0
    rc = lib.mc_forward(C.byref(m), src, 1, C.byref(run), None, 0x2000, None, 0x3000, 1 << 30, None)
    assert rc == L.MC_ERR_UNSUPPORTED
    run.roulette_m, run.w_threshold = 10.0, 1e-4
    prof[0] = 1e10
    assert lib.mc_forward(C.byref(m), src, 1, C.byref(run), None, 0x2000, None, 0x3000, 1 << 30, None) == \
        L.MC_ERR_UNSUPPORTED


def test_binned_arguments_checked_on_host():
    """The discrete-ordinates tally takes an even bin count in 2 .. 4096 and a
    0/1 direction; anything else is refused before any device work."""
    L, lib = _lib()
    m = _medium(L)
    src = (L.mc_source * 1)(_pencil(L))
    run = L.mc_run(1000, 0, 0, 0, 4, 1e-4, 10.0, 0)
    assert lib.mc_binned_workspace_bytes(C.byref(m), src, 1, C.byref(run), 16) > 0
    for nb in (0, 1, 15, 4098):
        assert lib.mc_binned_workspace_bytes(C.byref(m), src, 1, C.byref(run), nb) == 0
        assert lib.mc_run_binned(C.byref(m), src, 1, C.byref(run), 0, nb, 0x2000, None, 0x3000, 1 << 30,
                                 None) == L.MC_ERR_INVALID_ARG
    assert lib.mc_run_binned(C.byref(m), src, 1, C.byref(run), 2, 16, 0x2000, None, 0x3000, 1 << 30,
                             None) == L.MC_ERR_INVALID_ARG
    assert lib.mc_run_binned(C.byref(m), src, 1, C.byref(run), 0, 16, None, None, 0x3000, 1 << 30,
                             None) == L.MC_ERR_INVALID_ARG
    assert lib.mc_run_binned(C.byref(m), src, 1, C.byref(run), 0, 16, 0x2000, None, 0x3000, 16,
                             None) == L.MC_ERR_WORKSPACE

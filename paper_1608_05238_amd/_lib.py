"""ctypes declarations of the C ABI in include/mcrad.h (librmc.so).

Loading fails loudly if the in-tree library has not been built: there is no
CPU fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librmc.so")

MC_OK, MC_ERR_INVALID_ARG, MC_ERR_UNSUPPORTED, MC_ERR_DEVICE, MC_ERR_WORKSPACE, MC_ERR_SCRATCH = range(6)
MC_SRC_PENCIL, MC_SRC_LINE, MC_SRC_POINT, MC_SRC_MAP = range(4)
MC_FLAG_LITERAL_TRUNCATION = 1
MC_FLAG_EQUAL_COUNT = 2
MC_NHARM_MAX = 32

# exported symbols declared in include/*.h
SYMBOLS = ("mc_workspace_bytes", "mc_forward", "mc_adjoint", "mc_residual", "mc_gradient", "mc_absorbed",
           "mc_adjoint_source", "mc_gradient_h", "mc_detect", "mc_trace", "mc_philox_fill", "mc_default_tuning",
           "mc_timer_create", "mc_timer_destroy", "mc_timer_read", "mc_batch_workspace_bytes", "mc_run_batch",
           "mc_run_noalloc",
           "mc_binned_workspace_bytes", "mc_run_binned",
           "mc_status_string", "mc_build_info", "dn_conv3x3_fwd", "dn_conv3x3_wgrad",
           "mb_lds_atomics", "mb_global_atomics_f64", "mb_global_atomics_rows_f64", "mb_copy", "mb_fma_f32", "mb_wall_clock_khz")
(MB_LDS_ADD_F64, MB_LDS_ADD_F32, MB_LDS_ADD_U64, MB_LDS_ADD_U32, MB_LDS_ADD_F64_ROW33, MB_LDS_ADD_U64_ROW33,
 MB_LDS_ADD_U64_PRE) = range(7)


class mc_medium(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nz", C.c_int32), ("dx", C.c_float),
                ("mua_d", C.c_void_p), ("mus_d", C.c_void_p), ("g_d", C.c_void_p)]


class mc_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("x0", C.c_float), ("z0", C.c_float), ("x1", C.c_float),
                ("z1", C.c_float), ("dir_x", C.c_float), ("dir_z", C.c_float),
                ("lambertian", C.c_int32), ("power", C.c_double), ("map_d", C.c_void_p),
                ("n_prof", C.c_int32), ("prof_h", C.POINTER(C.c_double))]


class mc_run(C.Structure):
    _fields_ = [("n_packets", C.c_uint64), ("seed", C.c_uint64), ("first_packet_id", C.c_uint64),
                ("stream_tag", C.c_uint32), ("n_harm", C.c_int32), ("w_threshold", C.c_float),
                ("roulette_m", C.c_float), ("flags", C.c_uint32)]


class mc_ledger(C.Structure):
    _fields_ = [("launched", C.c_double), ("absorbed", C.c_double), ("escaped", C.c_double),
                ("roulette_gain", C.c_double), ("roulette_loss", C.c_double), ("scale", C.c_double),
                ("packets", C.c_uint64), ("segments", C.c_uint64), ("visits", C.c_uint64),
                ("scatters", C.c_uint64), ("generations", C.c_uint64)]


class mc_event(C.Structure):
    _fields_ = [("pid", C.c_uint64), ("k", C.c_int32), ("type", C.c_int32), ("ix", C.c_int32),
                ("iz", C.c_int32), ("x", C.c_float), ("z", C.c_float), ("sx", C.c_float),
                ("sz", C.c_float), ("w", C.c_float), ("t", C.c_float)]


class mc_problem(C.Structure):
    _fields_ = [("medium", mc_medium), ("src", C.POINTER(mc_source)), ("n_src", C.c_int32), ("run", mc_run),
                ("adjoint", C.c_int32), ("coeffs_d", C.c_void_p), ("ledger_d", C.c_void_p)]


class mc_tuning(C.Structure):
    _fields_ = [("live_packets", C.c_uint64), ("job_packets", C.c_uint32), ("max_visits", C.c_uint32),
                ("tile", C.c_uint32), ("grid_max_packets", C.c_uint32), ("finish_packets", C.c_uint64),
                ("flush_track", C.c_float), ("tail_visits", C.c_uint32), ("max_generations", C.c_uint32),
                ("min_job_packets", C.c_uint32), ("quiet_percent", C.c_uint32), ("reserved", C.c_uint32)]


class mc_options(C.Structure):
    _fields_ = [("tuning", C.POINTER(mc_tuning)), ("timer", C.c_void_p)]


_lib = None


def load() -> C.CDLL:
    """Load librmc.so (raises if it is missing: build it with paper_1608_05238_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_1608_05238_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, V, St = C.POINTER, C.c_void_p, C.c_int
    lib.mc_workspace_bytes.argtypes = [P(mc_medium), P(mc_source), C.c_int, P(mc_run), P(mc_options)]
    lib.mc_workspace_bytes.restype = C.c_size_t
    for name in ("mc_forward", "mc_adjoint"):
        f = getattr(lib, name)
        f.argtypes = [P(mc_medium), P(mc_source), C.c_int, P(mc_run), P(mc_options), V, V, V, C.c_size_t, V]
        f.restype = St
    lib.mc_residual.argtypes = [P(mc_medium), V, V, V, V, V]
    lib.mc_residual.restype = St
    lib.mc_gradient.argtypes = [P(mc_medium), C.c_int, V, V, V, V, V, V]
    lib.mc_gradient.restype = St
    lib.mc_absorbed.argtypes = [P(mc_medium), V, V, V]
    lib.mc_absorbed.restype = St
    lib.mc_adjoint_source.argtypes = [P(mc_medium), V, V, V]
    lib.mc_adjoint_source.restype = St
    lib.mc_gradient_h.argtypes = [P(mc_medium), C.c_int, V, V, V, V, V, V]
    lib.mc_gradient_h.restype = St
    lib.mc_detect.argtypes = [P(mc_medium), C.c_int, V, V, V, V]
    lib.mc_detect.restype = St
    lib.mc_trace.argtypes = [P(mc_medium), P(mc_source), C.c_int, P(mc_run), C.c_int, P(C.c_uint64), C.c_int,
                             P(mc_event), C.c_size_t, P(C.c_size_t)]
    lib.mc_trace.restype = St
    lib.mc_philox_fill.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32, V, V]
    lib.mc_philox_fill.restype = St
    lib.mc_timer_create.argtypes = [P(V)]
    lib.mc_timer_create.restype = St
    lib.mc_timer_destroy.argtypes = [V]
    lib.mc_timer_destroy.restype = St
    lib.mc_timer_read.argtypes = [V, P(C.c_double), P(C.c_uint64), C.c_int]
    lib.mc_timer_read.restype = St
    lib.mc_default_tuning.argtypes = [P(mc_tuning)]
    lib.mc_default_tuning.restype = St
    lib.mc_run_noalloc.argtypes = [P(mc_medium), P(mc_source), C.c_int, P(mc_run), C.c_int, P(mc_options), V, V, V]
    lib.mc_run_noalloc.restype = St
    lib.mc_batch_workspace_bytes.argtypes = [P(mc_problem), C.c_int, P(mc_options)]
    lib.mc_batch_workspace_bytes.restype = C.c_size_t
    lib.mc_run_batch.argtypes = [P(mc_problem), C.c_int, P(mc_options), V, C.c_size_t, V]
    lib.mc_run_batch.restype = St
    lib.mc_binned_workspace_bytes.argtypes = [P(mc_medium), P(mc_source), C.c_int, P(mc_run), C.c_int]
    lib.mc_binned_workspace_bytes.restype = C.c_size_t
    lib.mc_run_binned.argtypes = [P(mc_medium), P(mc_source), C.c_int, P(mc_run), C.c_int, C.c_int, V, V, V,
                                  C.c_size_t, V]
    lib.mc_run_binned.restype = St
    lib.dn_conv3x3_fwd.argtypes = [V, V, V, V, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, V]
    lib.dn_conv3x3_fwd.restype = St
    lib.dn_conv3x3_wgrad.argtypes = [V, V, V, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, V]
    lib.dn_conv3x3_wgrad.restype = St
    lib.mb_lds_atomics.argtypes = [C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, V, V, V]
    lib.mb_lds_atomics.restype = St
    lib.mb_global_atomics_f64.argtypes = [V, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, V]
    lib.mb_global_atomics_f64.restype = St
    lib.mb_global_atomics_rows_f64.argtypes = [V, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, V]
    lib.mb_global_atomics_rows_f64.restype = St
    lib.mb_copy.argtypes = [V, V, C.c_uint64, V]
    lib.mb_copy.restype = St
    lib.mb_fma_f32.argtypes = [V, C.c_uint32, C.c_uint32, V, V]
    lib.mb_fma_f32.restype = St
    lib.mb_wall_clock_khz.argtypes = [C.c_int, P(C.c_int)]
    lib.mb_wall_clock_khz.restype = St
    lib.mc_status_string.argtypes = [C.c_int]
    lib.mc_status_string.restype = C.c_char_p
    lib.mc_build_info.argtypes = []
    lib.mc_build_info.restype = C.c_char_p
    _lib = lib
    return lib


class MCError(RuntimeError):
    def __init__(self, fn: str, code: int):
        msg = load().mc_status_string(code).decode()
        super().__init__(f"{fn} failed: {msg} (status {code})")
        self.code = code


def check(fn: str, code: int) -> None:
    if code != MC_OK:
        raise MCError(fn, code)

"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Wraps ``liboracle.so`` built from ``rmc_oracle.c`` with gcc.  Inputs are numpy
arrays; every map is converted to float64 and row-major ``[nz][nx]``.
The paper is Hochuli, Powell, Arridge & Cox, arXiv:1608.05238; the section
each routine follows is named in ``rmc_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

PENCIL, LINE, POINT, MAP = 0, 1, 2, 3
FLAG_LITERAL_TRUNCATION, FLAG_EQUAL_COUNT = 1, 2
EV_LAUNCH, EV_CROSS, EV_SCATTER, EV_ESCAPE, EV_KILL = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no fast-math), OpenMP over packets."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC", "-shared",
               os.path.join(_HERE, "rmc_oracle.c"), "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Medium(C.Structure):
    _fields_ = [("nx", C.c_int), ("nz", C.c_int), ("dx", C.c_double),
                ("mua", C.POINTER(C.c_double)), ("mus", C.POINTER(C.c_double)),
                ("g", C.POINTER(C.c_double))]


class _Source(C.Structure):
    _fields_ = [("kind", C.c_int), ("x0", C.c_double), ("z0", C.c_double),
                ("x1", C.c_double), ("z1", C.c_double), ("dir_x", C.c_double),
                ("dir_z", C.c_double), ("lambertian", C.c_int), ("power", C.c_double),
                ("map", C.POINTER(C.c_double)), ("n_prof", C.c_int),
                ("prof", C.POINTER(C.c_double))]


class _Run(C.Structure):
    _fields_ = [("n_packets", C.c_uint64), ("seed", C.c_uint64), ("first_packet_id", C.c_uint64),
                ("stream_tag", C.c_uint32), ("n_harm", C.c_int), ("w_threshold", C.c_double),
                ("roulette_m", C.c_double), ("flags", C.c_uint32), ("adjoint", C.c_int)]


class _Ledger(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("launched", "absorbed", "escaped", "roulette_gain",
                                         "roulette_loss", "segments", "visits", "scatters",
                                         "packets", "scale")]


class _Event(C.Structure):
    _fields_ = [("pid", C.c_uint64), ("k", C.c_int32), ("type", C.c_int32), ("ix", C.c_int32),
                ("iz", C.c_int32), ("x", C.c_double), ("z", C.c_double), ("sx", C.c_double),
                ("sz", C.c_double), ("w", C.c_double), ("t", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = C.CDLL(_LIB_PATH)
        d = C.POINTER(C.c_double)
        lib.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        lib.or_philox_fill.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint32,
                                       C.POINTER(C.c_uint32)]
        lib.or_u01.argtypes = [C.c_uint32]
        lib.or_u01.restype = C.c_double
        lib.or_hg_dtheta.argtypes = [C.c_double, C.c_double]
        lib.or_hg_dtheta.restype = C.c_double
        lib.or_free_path.argtypes = [C.c_double]
        lib.or_free_path.restype = C.c_double
        lib.or_mc.argtypes = [C.POINTER(_Medium), C.POINTER(_Source), C.c_int, C.POINTER(_Run),
                              d, C.POINTER(_Ledger), d, C.c_int, C.c_int]
        lib.or_mc.restype = C.c_int
        lib.or_trace.argtypes = [C.POINTER(_Medium), C.POINTER(_Source), C.c_int, C.POINTER(_Run),
                                 C.POINTER(C.c_uint64), C.c_int, C.POINTER(_Event), C.c_int,
                                 C.POINTER(C.c_int)]
        lib.or_trace.restype = C.c_int
        lib.or_residual.argtypes = [C.POINTER(_Medium), d, d, d]
        lib.or_residual.restype = C.c_double
        lib.or_gradient.argtypes = [C.POINTER(_Medium), C.c_int, d, d, d, d, d]
        lib.or_detect.argtypes = [C.POINTER(_Medium), C.c_int, d, d]
        lib.or_detect.restype = C.c_double
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class Medium:
    """Pixel maps [nz][nx] of mua (1/mm), mus (1/mm) and g; square pixels of side dx (mm)."""
    mua: np.ndarray
    mus: np.ndarray
    g: np.ndarray
    dx: float

    def __post_init__(self):
        self.mua, self.mus, self.g = _f64(self.mua), _f64(self.mus), _f64(self.g)
        assert self.mua.shape == self.mus.shape == self.g.shape and self.mua.ndim == 2

    @property
    def nz(self):
        return self.mua.shape[0]

    @property
    def nx(self):
        return self.mua.shape[1]

    def _c(self):
        return _Medium(self.nx, self.nz, float(self.dx), _dp(self.mua), _dp(self.mus), _dp(self.g))


@dataclass
class Source:
    kind: int
    x0: float = 0.0
    z0: float = 0.0
    x1: float = 0.0
    z1: float = 0.0
    dir_x: float = 0.0
    dir_z: float = 1.0
    lambertian: int = 0
    power: float = 1.0
    map: Optional[np.ndarray] = None
    prof: Optional[np.ndarray] = None     # [2n+1] c0, c1..cn, s1..sn

    def _c(self, keep: list):
        s = _Source(self.kind, self.x0, self.z0, self.x1, self.z1, self.dir_x, self.dir_z,
                    self.lambertian, self.power, None, 0, None)
        if self.map is not None:
            m = _f64(self.map)
            keep.append(m)
            s.map = _dp(m)
        if self.prof is not None:
            p = _f64(self.prof)
            assert p.ndim == 1 and p.size % 2 == 1
            keep.append(p)
            s.n_prof = (p.size - 1) // 2
            s.prof = _dp(p)
        return s


@dataclass
class Run:
    n_packets: int
    seed: int = 0
    n_harm: int = 8
    first_packet_id: int = 0
    stream_tag: int = 0
    w_threshold: float = 1e-4
    roulette_m: float = 10.0
    flags: int = 0
    adjoint: int = 0

    def _c(self):
        return _Run(self.n_packets, self.seed, self.first_packet_id, self.stream_tag, self.n_harm,
                    self.w_threshold, self.roulette_m, self.flags, self.adjoint)


@dataclass
class Ledger:
    launched: float = 0.0
    absorbed: float = 0.0
    escaped: float = 0.0
    roulette_gain: float = 0.0
    roulette_loss: float = 0.0
    segments: float = 0.0
    visits: float = 0.0
    scatters: float = 0.0
    packets: float = 0.0
    scale: float = 0.0
    extra: dict = field(default_factory=dict)


def _sources(sources: Sequence[Source], keep: list):
    arr = (_Source * len(sources))()
    for i, s in enumerate(sources):
        arr[i] = s._c(keep)
    return arr


def run_mc(medium: Medium, sources: Sequence[Source], run: Run, n_threads: int = 1,
           n_bins: int = 0):
    """Run the oracle MC.  Returns (coeffs [2N+1][nz][nx], Ledger[, binned])."""
    lib = _load()
    keep: list = []
    K = 2 * run.n_harm + 1
    out = np.zeros((K, medium.nz, medium.nx))
    binned = np.zeros((n_bins, medium.nz, medium.nx)) if n_bins else None
    led = _Ledger()
    m = medium._c()
    srcs = _sources(sources, keep)
    r = run._c()
    rc = lib.or_mc(C.byref(m), srcs, len(sources), C.byref(r), _dp(out), C.byref(led),
                   _dp(binned) if binned is not None else None, n_bins, n_threads)
    if rc != 0:
        raise ValueError(f"oracle or_mc failed with code {rc}")
    L = Ledger(**{f: getattr(led, f) for f, _ in _Ledger._fields_})
    return (out, L, binned) if n_bins else (out, L)


def trace(medium: Medium, sources: Sequence[Source], run: Run, pids, cap: int = 1 << 20):
    """Per-event trace of the given packet ids; returns a numpy structured array."""
    lib = _load()
    keep: list = []
    pids = np.ascontiguousarray(np.asarray(pids, dtype=np.uint64))
    ev = (_Event * cap)()
    n = C.c_int(0)
    m = medium._c()
    rc = lib.or_trace(C.byref(m), _sources(sources, keep), len(sources), C.byref(run._c()),
                      pids.ctypes.data_as(C.POINTER(C.c_uint64)), len(pids), ev, cap, C.byref(n))
    if rc != 0:
        raise ValueError(f"oracle or_trace failed with code {rc}")
    if n.value > cap:
        raise ValueError("trace capacity exceeded")
    dt = np.dtype([("pid", "<u8"), ("k", "<i4"), ("type", "<i4"), ("ix", "<i4"), ("iz", "<i4"),
                   ("x", "<f8"), ("z", "<f8"), ("sx", "<f8"), ("sz", "<f8"), ("w", "<f8"),
                   ("t", "<f8")])
    buf = np.frombuffer(ev, dtype=dt, count=n.value).copy()
    return buf


def residual(medium: Medium, coeffs: np.ndarray, h_meas: np.ndarray):
    """Returns (eps, q_star) with q* = mua (Hmeas - mua a0)."""
    lib = _load()
    c = _f64(coeffs)
    hm = _f64(h_meas)
    q = np.zeros((medium.nz, medium.nx))
    eps = lib.or_residual(C.byref(medium._c()), _dp(c), _dp(hm), _dp(q))
    return eps, q


def gradient(medium: Medium, n_harm: int, fwd: np.ndarray, adj: np.ndarray, h_meas: np.ndarray):
    lib = _load()
    f, a, hm = _f64(fwd), _f64(adj), _f64(h_meas)
    dmua = np.zeros((medium.nz, medium.nx))
    dmus = np.zeros((medium.nz, medium.nx))
    lib.or_gradient(C.byref(medium._c()), n_harm, _dp(f), _dp(a), _dp(hm), _dp(dmua), _dp(dmus))
    return dmua, dmus


def detect(medium: Medium, n_harm: int, coeffs: np.ndarray, det: np.ndarray) -> float:
    lib = _load()
    c, d = _f64(coeffs), _f64(det)
    return lib.or_detect(C.byref(medium._c()), n_harm, _dp(c), _dp(d))


def philox(ctr, key):
    lib = _load()
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib.or_philox4x32_10(c, k, o)
    return list(o)


def philox_fill(seed: int, tag: int, pid0: int, n: int, j: int) -> np.ndarray:
    lib = _load()
    out = np.zeros((n, 4), dtype=np.uint32)
    lib.or_philox_fill(seed, tag, pid0, n, j, out.ctypes.data_as(C.POINTER(C.c_uint32)))
    return out


def u01(x: int) -> float:
    return _load().or_u01(x)


def hg_dtheta(g: float, u: float) -> float:
    return _load().or_hg_dtheta(g, u)


def free_path(u: float) -> float:
    return _load().or_free_path(u)


_KINDS = {"pencil": PENCIL, "line": LINE, "point": POINT, "map": MAP}


def medium_from(ph) -> Medium:
    """Oracle medium from a phantoms.Phantom (float32 maps widened exactly to float64)."""
    return Medium(ph.mua, ph.mus, ph.g, float(ph.dx))


def sources_from(specs) -> list:
    """Oracle sources from phantoms.SourceSpec descriptions."""
    out = []
    for s in specs:
        out.append(Source(_KINDS[s.kind], s.x0, s.z0, s.x1, s.z1, s.dir_x, s.dir_z, s.lambertian,
                          s.power, s.map, s.prof))
    return out

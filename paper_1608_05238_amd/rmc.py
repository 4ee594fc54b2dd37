"""Python binding of librmc.so: argument marshalling only.

Every computation runs in the HIP kernels behind include/mcrad.h; PyTorch
only supplies device memory and the stream.  Function names follow the C ABI.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Iterable, Optional, Sequence

import numpy as np
import torch

from . import _lib as L

_KIND = {"pencil": L.MC_SRC_PENCIL, "line": L.MC_SRC_LINE, "point": L.MC_SRC_POINT, "map": L.MC_SRC_MAP}


def _device() -> torch.device:
    if not torch.cuda.is_available():
        raise RuntimeError("librmc needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch.device("cuda", torch.cuda.current_device())


def _stream(stream: Optional[torch.cuda.Stream]) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


@dataclass
class Medium:
    """mua, mus, g: device float32 [nz][nx]; dx in mm."""
    mua: torch.Tensor
    mus: torch.Tensor
    g: torch.Tensor
    dx: float

    @classmethod
    def from_phantom(cls, ph, device=None) -> "Medium":
        dev = device or _device()
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev)
        return cls(f(ph.mua), f(ph.mus), f(ph.g), float(ph.dx))

    @property
    def nz(self) -> int:
        return self.mua.shape[0]

    @property
    def nx(self) -> int:
        return self.mua.shape[1]

    def c(self) -> L.mc_medium:
        for t in (self.mua, self.mus, self.g):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.shape != self.mua.shape:
                raise ValueError("medium maps must be contiguous float32 device tensors of one shape")
        return L.mc_medium(self.nx, self.nz, float(self.dx), self.mua.data_ptr(), self.mus.data_ptr(),
                           self.g.data_ptr())


@dataclass
class Source:
    """A source as the C ABI's mc_source: kind is "pencil", "line", "point" or
    "map"; positions in mm; map: FP64 [nz][nx] array or device tensor (MAP);
    prof: angular profile coefficients c0, c1..cn, s1..sn (POINT/MAP)."""
    kind: str
    x0: float = 0.0
    z0: float = 0.0
    x1: float = 0.0
    z1: float = 0.0
    dir_x: float = 0.0
    dir_z: float = 1.0
    lambertian: int = 0
    power: float = 1.0
    map: Optional[object] = None
    prof: Optional[object] = None


class _Sources:
    """Holds the ctypes source array and every buffer it points to."""

    def __init__(self, specs: Sequence, device: torch.device):
        self.keep = []
        self.arr = (L.mc_source * len(specs))()
        for i, s in enumerate(specs):
            c = L.mc_source()
            c.kind = _KIND[s.kind]
            c.x0, c.z0, c.x1, c.z1 = s.x0, s.z0, s.x1, s.z1
            c.dir_x, c.dir_z = s.dir_x, s.dir_z
            c.lambertian = int(s.lambertian)
            c.power = float(s.power)
            if s.map is not None:
                m = torch.as_tensor(np.ascontiguousarray(s.map, dtype=np.float64), device=device) \
                    if not isinstance(s.map, torch.Tensor) else s.map.to(device=device, dtype=torch.float64).contiguous()
                self.keep.append(m)
                c.map_d = m.data_ptr()
            if s.prof is not None:
                p = np.ascontiguousarray(np.asarray(s.prof, dtype=np.float64))
                if p.ndim != 1 or p.size % 2 != 1:
                    raise ValueError("angular profile must have 2n+1 coefficients")
                self.keep.append(p)
                c.n_prof = (p.size - 1) // 2
                c.prof_h = p.ctypes.data_as(C.POINTER(C.c_double))
            self.arr[i] = c
        self.n = len(specs)


def make_run(n_packets: int, n_harm: int, seed: int = 0, first_packet_id: int = 0, stream_tag: int = 0,
             w_threshold: float = 1e-4, roulette_m: float = 10.0, flags: int = 0) -> L.mc_run:
    return L.mc_run(int(n_packets), int(seed), int(first_packet_id), int(stream_tag), int(n_harm),
                    float(w_threshold), float(roulette_m), int(flags))


def ledger_dict(buf: torch.Tensor) -> dict:
    """Decode a device mc_ledger buffer (synchronises on its stream)."""
    raw = bytes(buf.cpu().numpy().tobytes())
    led = L.mc_ledger.from_buffer_copy(raw)
    return {f: getattr(led, f) for f, _ in L.mc_ledger._fields_}


_TUNING_FIELDS = ("live_packets", "job_packets", "max_visits", "tile", "finish_packets", "grid_max_packets",
                  "flush_track", "tail_visits", "max_generations", "min_job_packets",
                  "quiet_percent")


def default_tuning() -> dict:
    """The library's built-in tuning of the tiled transport (see mc_tuning in include/mcrad.h)."""
    t = L.mc_tuning()
    L.check("mc_default_tuning", L.load().mc_default_tuning(C.byref(t)))
    return {f: getattr(t, f) for f in _TUNING_FIELDS}


class Timer:
    """A caller-owned mc_timer: HIP events around every transport launch of
    the calls it is passed to."""

    def __init__(self):
        self._h = C.c_void_p()
        L.check("mc_timer_create", L.load().mc_timer_create(C.byref(self._h)))

    def read(self, reset: bool = True):
        """(total transport milliseconds, launches) since the last reset; waits for the events."""
        ms, n = C.c_double(0), C.c_uint64(0)
        L.check("mc_timer_read", L.load().mc_timer_read(self._h, C.byref(ms), C.byref(n), int(bool(reset))))
        return ms.value, n.value

    def close(self):
        if self._h:
            L.load().mc_timer_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Options:
    """The mc_options of one call and the buffers it points to."""

    def __init__(self, tuning: Optional[dict], timer: Optional[Timer]):
        self.t = None
        if tuning:
            self.t = L.mc_tuning()
            for f in _TUNING_FIELDS:
                v = tuning.get(f, 0)
                setattr(self.t, f, float(v) if f == "flush_track" else int(v))
        self.o = L.mc_options(C.pointer(self.t) if self.t is not None else None, timer._h if timer else None)

    def ref(self):
        return C.byref(self.o)


def mc_workspace_bytes(medium: Medium, sources: Sequence, run: L.mc_run, tuning: Optional[dict] = None) -> int:
    dev = medium.mua.device
    src = _Sources(sources, dev)
    return L.load().mc_workspace_bytes(C.byref(medium.c()), src.arr, src.n, C.byref(run), _Options(tuning, None).ref())


def _mc(name: str, medium: Medium, sources: Sequence, run: L.mc_run, out: Optional[torch.Tensor],
        workspace: Optional[torch.Tensor], want_ledger: bool, stream, tuning=None, timer=None):
    lib = L.load()
    dev = medium.mua.device
    src = _Sources(sources, dev)
    m = medium.c()
    opts = _Options(tuning, timer)
    need = lib.mc_workspace_bytes(C.byref(m), src.arr, src.n, C.byref(run), opts.ref())
    if need == 0:
        raise L.MCError("mc_workspace_bytes", L.MC_ERR_INVALID_ARG)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    base = workspace.data_ptr()
    off = (-base) % 256
    K = 2 * run.n_harm + 1
    if out is None:
        out = torch.empty((K, medium.nz, medium.nx), dtype=torch.float64, device=dev)
    if out.dtype != torch.float64 or not out.is_contiguous() or tuple(out.shape) != (K, medium.nz, medium.nx):
        raise ValueError("output must be contiguous float64 [2N+1][nz][nx]")
    led = torch.zeros(C.sizeof(L.mc_ledger), dtype=torch.uint8, device=dev) if want_ledger else None
    fn = getattr(lib, name)
    L.check(name, fn(C.byref(m), src.arr, src.n, C.byref(run), opts.ref(), out.data_ptr(), _ptr(led), base + off,
                     workspace.numel() - off, _stream(stream)))
    if stream is not None:
        workspace.record_stream(stream)   # freed by the caching allocator only after the stream's work
    return out, led, workspace


def mc_forward(medium: Medium, sources: Sequence, run: L.mc_run, out=None, workspace=None, ledger=True,
               stream=None, tuning: Optional[dict] = None, timer: Optional[Timer] = None):
    """Forward radiance MC.  Returns (coeffs [2N+1][nz][nx] float64, ledger buffer or None).
    tuning: mc_tuning fields (dict; missing or zero fields take the defaults);
    timer: a Timer that records this call's transport launches."""
    out, led, _ = _mc("mc_forward", medium, sources, run, out, workspace, ledger, stream, tuning, timer)
    return out, led


def mc_adjoint(medium: Medium, sources: Sequence, run: L.mc_run, out=None, workspace=None, ledger=True,
               stream=None, tuning: Optional[dict] = None, timer: Optional[Timer] = None):
    """Adjoint radiance MC (adjoint field phi*, orders already mirrored)."""
    out, led, _ = _mc("mc_adjoint", medium, sources, run, out, workspace, ledger, stream, tuning, timer)
    return out, led


def mc_run_noalloc(medium: Medium, sources: Sequence, run: L.mc_run, adjoint: bool = False, out=None, ledger=True,
                   stream=None, tuning: Optional[dict] = None):
    """A forward or adjoint run on the library's static scratch (no workspace,
    no allocation inside the call; see mc_run_noalloc in include/mcrad.h).
    The binding itself allocates the output and ledger if not given."""
    lib = L.load()
    dev = medium.mua.device
    src = _Sources(sources, dev)
    K = 2 * run.n_harm + 1
    if out is None:
        out = torch.empty((K, medium.nz, medium.nx), dtype=torch.float64, device=dev)
    led = torch.zeros(C.sizeof(L.mc_ledger), dtype=torch.uint8, device=dev) if ledger else None
    L.check("mc_run_noalloc", lib.mc_run_noalloc(C.byref(medium.c()), src.arr, src.n, C.byref(run), int(bool(adjoint)),
                                                 _Options(tuning, None).ref(), out.data_ptr(), _ptr(led),
                                                 _stream(stream)))
    return out, led


def mc_binned(medium: Medium, sources: Sequence, run: L.mc_run, n_bins: int, adjoint: bool = False, ledger=True,
              stream=None):
    """Discrete-ordinates comparison tally: radiance averaged over n_bins equal
    angular bins of [-pi, pi), from the same transport as mc_forward /
    mc_adjoint.  Returns (binned [n_bins][nz][nx] float64, ledger buffer or None)."""
    lib = L.load()
    dev = medium.mua.device
    src = _Sources(sources, dev)
    m = medium.c()
    need = lib.mc_binned_workspace_bytes(C.byref(m), src.arr, src.n, C.byref(run), int(n_bins))
    if need == 0:
        raise L.MCError("mc_binned_workspace_bytes", L.MC_ERR_INVALID_ARG)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    out = torch.empty((int(n_bins), medium.nz, medium.nx), dtype=torch.float64, device=dev)
    led = torch.zeros(C.sizeof(L.mc_ledger), dtype=torch.uint8, device=dev) if ledger else None
    L.check("mc_run_binned", lib.mc_run_binned(C.byref(m), src.arr, src.n, C.byref(run), int(bool(adjoint)),
                                               int(n_bins), out.data_ptr(), _ptr(led), ws.data_ptr() + off,
                                               ws.numel() - off, _stream(stream)))
    if stream is not None:
        ws.record_stream(stream)
    return out, led


def mc_residual(medium: Medium, coeffs: torch.Tensor, hmeas: torch.Tensor, stream=None):
    """Returns (q_star [nz][nx] float64, eps device scalar float64)."""
    lib = L.load()
    q = torch.empty((medium.nz, medium.nx), dtype=torch.float64, device=coeffs.device)
    eps = torch.empty((), dtype=torch.float64, device=coeffs.device)
    hm = hmeas.to(torch.float64).contiguous()
    L.check("mc_residual", lib.mc_residual(C.byref(medium.c()), coeffs.data_ptr(), hm.data_ptr(), q.data_ptr(),
                                           eps.data_ptr(), _stream(stream)))
    return q, eps


def mc_gradient(medium: Medium, n_harm: int, fwd: torch.Tensor, adj: torch.Tensor, hmeas: torch.Tensor,
                stream=None):
    """Returns (d eps/d mua, d eps/d mus) per pixel, float64 [nz][nx]."""
    lib = L.load()
    dmua = torch.empty((medium.nz, medium.nx), dtype=torch.float64, device=fwd.device)
    dmus = torch.empty_like(dmua)
    hm = hmeas.to(torch.float64).contiguous()
    L.check("mc_gradient", lib.mc_gradient(C.byref(medium.c()), int(n_harm), fwd.data_ptr(), adj.data_ptr(),
                                           hm.data_ptr(), dmua.data_ptr(), dmus.data_ptr(), _stream(stream)))
    return dmua, dmus


def mc_absorbed(medium: Medium, coeffs: torch.Tensor, stream=None) -> torch.Tensor:
    """H = mua a0, float64 [nz][nx]."""
    lib = L.load()
    h = torch.empty((medium.nz, medium.nx), dtype=torch.float64, device=coeffs.device)
    L.check("mc_absorbed", lib.mc_absorbed(C.byref(medium.c()), coeffs.data_ptr(), h.data_ptr(), _stream(stream)))
    return h


def mc_adjoint_source(medium: Medium, grad_h: torch.Tensor, stream=None) -> torch.Tensor:
    """q* = -mua grad_h / dx^2 for an upstream gradient grad_h = dL/dH."""
    lib = L.load()
    g = grad_h.to(torch.float64).contiguous()
    q = torch.empty((medium.nz, medium.nx), dtype=torch.float64, device=g.device)
    L.check("mc_adjoint_source", lib.mc_adjoint_source(C.byref(medium.c()), g.data_ptr(), q.data_ptr(),
                                                       _stream(stream)))
    return q


def mc_gradient_h(medium: Medium, n_harm: int, fwd: torch.Tensor, adj: torch.Tensor, grad_h: torch.Tensor,
                  stream=None):
    """(dL/dmua, dL/dmus) per pixel for an upstream gradient grad_h = dL/dH."""
    lib = L.load()
    g = grad_h.to(torch.float64).contiguous()
    dmua = torch.empty((medium.nz, medium.nx), dtype=torch.float64, device=fwd.device)
    dmus = torch.empty_like(dmua)
    L.check("mc_gradient_h", lib.mc_gradient_h(C.byref(medium.c()), int(n_harm), fwd.data_ptr(), adj.data_ptr(),
                                               g.data_ptr(), dmua.data_ptr(), dmus.data_ptr(), _stream(stream)))
    return dmua, dmus


def mc_detect(medium: Medium, n_harm: int, coeffs: torch.Tensor, det: torch.Tensor, stream=None) -> torch.Tensor:
    lib = L.load()
    out = torch.empty((), dtype=torch.float64, device=coeffs.device)
    d = det.to(torch.float64).contiguous()
    L.check("mc_detect", lib.mc_detect(C.byref(medium.c()), int(n_harm), coeffs.data_ptr(), d.data_ptr(),
                                       out.data_ptr(), _stream(stream)))
    return out


@dataclass
class Problem:
    """One problem of mc_run_batch: medium, sources, run and direction."""
    medium: Medium
    sources: Sequence
    run: L.mc_run
    adjoint: bool = False


def mc_run_batch(problems: Sequence[Problem], ledger: bool = True, stream=None, tuning: Optional[dict] = None,
                 timer: Optional[Timer] = None):
    """Run many problems in one packet pool.  Returns a list of (coeffs, ledger
    buffer or None), in the order given."""
    lib = L.load()
    n = len(problems)
    arr = (L.mc_problem * n)()
    keep, outs = [], []
    for i, pr in enumerate(problems):
        dev = pr.medium.mua.device
        src = _Sources(pr.sources, dev)
        keep.append(src)
        K = 2 * pr.run.n_harm + 1
        out = torch.empty((K, pr.medium.nz, pr.medium.nx), dtype=torch.float64, device=dev)
        led = torch.zeros(C.sizeof(L.mc_ledger), dtype=torch.uint8, device=dev) if ledger else None
        outs.append((out, led))
        arr[i] = L.mc_problem(pr.medium.c(), src.arr, src.n, pr.run, int(bool(pr.adjoint)), out.data_ptr(), _ptr(led))
    opts = _Options(tuning, timer)
    need = lib.mc_batch_workspace_bytes(arr, n, opts.ref())
    if need == 0:
        raise L.MCError("mc_batch_workspace_bytes", L.MC_ERR_INVALID_ARG)
    dev = problems[0].medium.mua.device
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    L.check("mc_run_batch", lib.mc_run_batch(arr, n, opts.ref(), ws.data_ptr() + off, ws.numel() - off,
                                             _stream(stream)))
    if stream is not None:
        ws.record_stream(stream)   # freed by the caching allocator only after the stream's work
    return outs


_EVENT_DTYPE = np.dtype([("pid", "<u8"), ("k", "<i4"), ("type", "<i4"), ("ix", "<i4"), ("iz", "<i4"),
                         ("x", "<f4"), ("z", "<f4"), ("sx", "<f4"), ("sz", "<f4"), ("w", "<f4"), ("t", "<f4")])


def mc_trace(medium: Medium, sources: Sequence, run: L.mc_run, pids: Iterable[int], adjoint: bool = False,
             cap: int = 1 << 20) -> np.ndarray:
    """Per-event trace of the given packet ids (synchronous)."""
    lib = L.load()
    src = _Sources(sources, medium.mua.device)
    ids = np.ascontiguousarray(np.asarray(list(pids), dtype=np.uint64))
    ev = (L.mc_event * cap)()
    n = C.c_size_t(0)
    torch.cuda.synchronize()
    L.check("mc_trace", lib.mc_trace(C.byref(medium.c()), src.arr, src.n, C.byref(run), int(bool(adjoint)),
                                     ids.ctypes.data_as(C.POINTER(C.c_uint64)), len(ids), ev, cap, C.byref(n)))
    if n.value > cap:
        raise ValueError("trace capacity exceeded")
    return np.frombuffer(ev, dtype=_EVENT_DTYPE, count=n.value).copy()


def mc_philox_fill(seed: int, tag: int, pid0: int, n: int, j: int, stream=None) -> torch.Tensor:
    """Philox4x32-10 blocks as int32 tensor [n][4] (bit patterns of uint32)."""
    lib = L.load()
    out = torch.empty((n, 4), dtype=torch.int32, device=_device())
    L.check("mc_philox_fill", lib.mc_philox_fill(seed, tag, pid0, n, j, out.data_ptr(), _stream(stream)))
    return out


def build_info() -> str:
    return L.load().mc_build_info().decode()

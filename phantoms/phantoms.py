"""Seeded phantom, source and map generators (inputs only; no transport arithmetic).

The workloads follow the paper's set-ups (Hochuli et al., arXiv:1608.05238):
pixelated 2D media with absorbing / scattering inclusions (Sec. 6.1), collimated
line sources on the boundary (Sec. 6.1), isotropic point sources (Sec. 3.2,
Sec. 4.1) and a signed volumetric adjoint source shaped like a residual
(Sec. 6).  All maps are float32 ``[nz][nx]`` (x = column, z = row = depth).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Phantom:
    mua: np.ndarray
    mus: np.ndarray
    g: np.ndarray
    dx: float

    @property
    def nz(self) -> int:
        return self.mua.shape[0]

    @property
    def nx(self) -> int:
        return self.mua.shape[1]

    @property
    def width(self) -> float:
        return self.nx * self.dx

    @property
    def depth(self) -> float:
        return self.nz * self.dx

    def copy(self) -> "Phantom":
        return Phantom(self.mua.copy(), self.mus.copy(), self.g.copy(), self.dx)


@dataclass
class SourceSpec:
    """Plain description of a source; each side converts it to its own struct."""
    kind: str                      # "pencil" | "line" | "point" | "map"
    x0: float = 0.0
    z0: float = 0.0
    x1: float = 0.0
    z1: float = 0.0
    dir_x: float = 0.0
    dir_z: float = 1.0
    lambertian: int = 0
    power: float = 1.0
    map: Optional[np.ndarray] = None     # float64 [nz][nx], per unit angle per unit area
    prof: Optional[np.ndarray] = None    # float64 [2n+1]: c0, c1..cn, s1..sn


def homogeneous(nx: int, nz: int, dx: float, mua: float, mus: float, g: float) -> Phantom:
    f = np.float32
    return Phantom(np.full((nz, nx), mua, f), np.full((nz, nx), mus, f), np.full((nz, nx), g, f), dx)


def disc_phantom(n: int = 256, dx: float = 0.1, mua_bg: float = 0.01, mus_bg: float = 10.0,
                 g: float = 0.9, seed: int = 0, count=(3, 6), radius=(1.0, 4.0),
                 mua_fac=(2.0, 10.0), mus_fac=(0.5, 2.0)) -> Phantom:
    """Background plus 3-6 random discs (radius 1-4 mm, mua x2-10, mus x0.5-2).

    Later discs overwrite earlier ones; a pixel belongs to a disc when its
    centre does.
    """
    rng = np.random.default_rng(seed)
    L = n * dx
    ph = homogeneous(n, n, dx, mua_bg, mus_bg, g)
    k = int(rng.integers(count[0], count[1] + 1))
    c = (np.arange(n) + 0.5) * dx
    X, Z = np.meshgrid(c, c)
    for _ in range(k):
        r = rng.uniform(*radius)
        cx, cz = rng.uniform(r, L - r, size=2)
        fa, fs = rng.uniform(*mua_fac), rng.uniform(*mus_fac)
        inside = (X - cx) ** 2 + (Z - cz) ** 2 <= r * r
        ph.mua[inside] = np.float32(mua_bg * fa)
        ph.mus[inside] = np.float32(mus_bg * fs)
    return ph


def two_inclusion_phantom(n: int = 256, dx: float = 0.1, mua_bg: float = 0.01, mus_bg: float = 10.0,
                          g: float = 0.9) -> Phantom:
    """Background with one absorbing and one scattering circular inclusion."""
    ph = homogeneous(n, n, dx, mua_bg, mus_bg, g)
    L = n * dx
    c = (np.arange(n) + 0.5) * dx
    X, Z = np.meshgrid(c, c)
    a = (X - 0.35 * L) ** 2 + (Z - 0.4 * L) ** 2 <= (0.1 * L) ** 2
    s = (X - 0.65 * L) ** 2 + (Z - 0.6 * L) ** 2 <= (0.1 * L) ** 2
    ph.mua[a] = np.float32(mua_bg * 5)
    ph.mus[s] = np.float32(mus_bg * 2)
    return ph


def pencil_top_centre(ph: Phantom, power: float = 1.0) -> List[SourceSpec]:
    return [SourceSpec("pencil", x0=ph.width / 2, z0=0.0, dir_x=0.0, dir_z=1.0, power=power)]


def four_side_lines(ph: Phantom, power_each: float = 0.25, lambertian: int = 0) -> List[SourceSpec]:
    """Collimated (or Lambertian) line sources along each full side, pointing inward."""
    W, D = ph.width, ph.depth
    return [
        SourceSpec("line", 0.0, 0.0, W, 0.0, 0.0, 1.0, lambertian, power_each),     # top, +z
        SourceSpec("line", 0.0, D, W, D, 0.0, -1.0, lambertian, power_each),        # bottom, -z
        SourceSpec("line", 0.0, 0.0, 0.0, D, 1.0, 0.0, lambertian, power_each),     # left, +x
        SourceSpec("line", W, 0.0, W, D, -1.0, 0.0, lambertian, power_each),        # right, -x
    ]


def lambertian_boundary(ph: Phantom, total_power: float = 1.0) -> List[SourceSpec]:
    """Uniform Lambertian illumination of the whole boundary (power per side by length)."""
    W, D = ph.width, ph.depth
    per = total_power / (2 * (W + D))
    return [
        SourceSpec("line", 0.0, 0.0, W, 0.0, 0.0, 1.0, 1, per * W),
        SourceSpec("line", 0.0, D, W, D, 0.0, -1.0, 1, per * W),
        SourceSpec("line", 0.0, 0.0, 0.0, D, 1.0, 0.0, 1, per * D),
        SourceSpec("line", W, 0.0, W, D, -1.0, 0.0, 1, per * D),
    ]


def point_source(x: float, z: float, power: float = 1.0, prof: Optional[np.ndarray] = None) -> SourceSpec:
    return SourceSpec("point", x0=x, z0=z, power=power,
                      prof=None if prof is None else np.asarray(prof, np.float64))


def map_source(q: np.ndarray, prof: Optional[np.ndarray] = None) -> SourceSpec:
    return SourceSpec("map", map=np.ascontiguousarray(q, dtype=np.float64),
                      prof=None if prof is None else np.asarray(prof, np.float64))


def residual_like_map(ph: Phantom, seed: int = 3, n_blobs: int = 6, scale: float = 1e-3) -> np.ndarray:
    """Signed smooth map shaped like an absorbed-energy residual times mua."""
    rng = np.random.default_rng(seed)
    c = (np.arange(ph.nx) + 0.5) * ph.dx
    cz = (np.arange(ph.nz) + 0.5) * ph.dx
    X, Z = np.meshgrid(c, cz)
    q = np.zeros((ph.nz, ph.nx))
    for _ in range(n_blobs):
        x0, z0 = rng.uniform(0, ph.width), rng.uniform(0, ph.depth)
        s = rng.uniform(0.05, 0.2) * max(ph.width, ph.depth)
        q += rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 1.5) * np.exp(-((X - x0) ** 2 + (Z - z0) ** 2) / (2 * s * s))
    return (scale * q * ph.mua.astype(np.float64) / ph.mua.astype(np.float64).mean()).astype(np.float64)


def smooth_hmeas(ph: Phantom, seed: int = 4, level: float = 0.01) -> np.ndarray:
    """A positive smooth absorbed-energy-like map (for residual / gradient inputs)."""
    rng = np.random.default_rng(seed)
    c = (np.arange(ph.nx) + 0.5) * ph.dx
    cz = (np.arange(ph.nz) + 0.5) * ph.dx
    X, Z = np.meshgrid(c, cz)
    d = np.minimum.reduce([X, Z, ph.width - X, ph.depth - Z])
    base = np.exp(-d / max(ph.width, ph.depth) * rng.uniform(2, 4))
    return (level * ph.mua.astype(np.float64) / ph.mua.astype(np.float64).mean() * base).astype(np.float64)


def interior_pixels(ph: Phantom, count: int = 20, margin: int = 10, seed: int = 2) -> np.ndarray:
    """Random distinct (iz, ix) pixels at least `margin` pixels from the boundary."""
    rng = np.random.default_rng(seed)
    iz = np.arange(margin, ph.nz - margin)
    ix = np.arange(margin, ph.nx - margin)
    flat = rng.choice(iz.size * ix.size, size=count, replace=False)
    return np.stack([iz[flat // ix.size], ix[flat % ix.size]], axis=1)


@dataclass
class Config:
    name: str
    phantom: Phantom
    sources: List[SourceSpec]
    n_packets: int
    n_harm: int
    seed: int = 0
    extra: dict = field(default_factory=dict)


def config1() -> Config:
    """32x32 pixels of 0.5 mm, mua 0.05, mus 5, g 0.8, pencil at top centre, 1e5 packets, N = 8."""
    ph = homogeneous(32, 32, 0.5, 0.05, 5.0, 0.8)
    return Config("pencil32", ph, pencil_top_centre(ph), 100_000, 8, 0)


def config2() -> Config:
    """256x256 pixels of 0.1 mm disc phantom (seed 0), four line sources, 1e8 packets, N = 16.

    The measured data come from a second disc phantom (seed 1); the adjoint
    source is then mua (Hmeas - H).
    """
    ph = disc_phantom(256, 0.1, 0.01, 10.0, 0.9, seed=0)
    true = disc_phantom(256, 0.1, 0.01, 10.0, 0.9, seed=1)
    return Config("disc256", ph, four_side_lines(ph), 100_000_000, 16, 0, {"true": true})

"""Seeded synthetic inputs of the three-dimensional path (no part of the
method's arithmetic): the grid and parameter records, velocity models and
initial data on [n3][n2][n1] arrays."""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np

from . import rng


@dataclasses.dataclass(frozen=True)
class Grid3:
    n1: int
    n2: int
    n3: int
    o1: float
    o2: float
    o3: float
    d1: float
    d2: float
    d3: float

    @property
    def shape(self):
        return (self.n3, self.n2, self.n1)

    @property
    def n(self):
        return (self.n1, self.n2, self.n3)

    @property
    def o(self):
        return (self.o1, self.o2, self.o3)

    @property
    def d(self):
        return (self.d1, self.d2, self.d3)

    def coords(self):
        """Node coordinates (x1[n1], x2[n2], x3[n3])."""
        return tuple(o + d * np.arange(n) for o, d, n in zip(self.o, self.d, self.n))


@dataclasses.dataclass(frozen=True)
class Params3:
    """Numerical parameters of a three-dimensional run; per-axis tuples are
    ordered (x1, x2, x3)."""
    eps: float
    qb: Tuple[int, int, int]
    qs: Tuple[int, int, int]
    nq: Tuple[int, int, int]
    np: Tuple[int, int, int]
    dp: Tuple[float, float, float]
    tau: float
    tau_fbi: float
    tau_win: float
    dt: float
    nsteps: int

    def replace(self, **kw) -> "Params3":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Workload3:
    name: str
    grid: Grid3
    params: Params3
    c: np.ndarray                 # [n3][n2][n1]
    f0: np.ndarray                # [nshots][n3][n2][n1]
    f1: Optional[np.ndarray]

    @property
    def nshots(self) -> int:
        return self.f0.shape[0]


def smooth_layered_velocity3(grid: Grid3, seed: int, smooth_cells: float = 4.0,
                             vmin: float = 1.5, vmax: float = 3.5) -> np.ndarray:
    """Seeded smooth model layered in depth x3 with folded interfaces and one
    Gaussian lens, smoothed by a Gaussian of ``smooth_cells`` cells."""
    from scipy.ndimage import gaussian_filter

    g = rng(seed)
    x1, x2, x3 = grid.coords()
    Z = grid.n3 * grid.d3
    zb = np.sort(g.uniform(0.25, 0.8, 2)) * Z
    amp = g.uniform(0.03, 0.08, 2) * Z
    k1, k2 = g.uniform(1.0, 3.0, 2), g.uniform(1.0, 3.0, 2)
    vel = np.linspace(vmin, vmax, 3)
    X3 = x3[:, None, None]
    c = np.full(grid.shape, vel[0])
    for i in range(2):
        surf = zb[i] + amp[i] * np.sin(k1[i] * x1[None, None, :]) * np.cos(k2[i] * x2[None, :, None])
        c = np.where(X3 > surf, vel[i + 1], c)
    cen = g.uniform(0.3, 0.7, 3) * np.array([grid.n1 * grid.d1, grid.n2 * grid.d2, Z])
    r2 = ((x1[None, None, :] - cen[0]) ** 2 + (x2[None, :, None] - cen[1]) ** 2
          + (x3[:, None, None] - cen[2]) ** 2)
    c = c - 0.3 * np.exp(-r2 / (2 * (0.1 * Z) ** 2))
    c = gaussian_filter(c, smooth_cells, mode="nearest")
    return np.ascontiguousarray(np.clip(c, vmin * 0.8, vmax))


def gaussian_source3(grid: Grid3, center, sigma: float) -> np.ndarray:
    x1, x2, x3 = grid.coords()
    r2 = ((x1[None, None, :] - center[0]) ** 2 + (x2[None, :, None] - center[1]) ** 2
          + (x3[:, None, None] - center[2]) ** 2)
    return np.ascontiguousarray(np.exp(-r2 / (2 * sigma * sigma)))


def wavepacket_source3(grid: Grid3, center, sigma: float, k, eps: float) -> np.ndarray:
    """exp(-|x - x0|^2 / (2 sigma^2)) cos(k.(x - x0) / eps)."""
    x1, x2, x3 = grid.coords()
    dx = [x1[None, None, :] - center[0], x2[None, :, None] - center[1],
          x3[:, None, None] - center[2]]
    r2 = dx[0] ** 2 + dx[1] ** 2 + dx[2] ** 2
    ph = (k[0] * dx[0] + k[1] * dx[1] + k[2] * dx[2]) / eps
    return np.ascontiguousarray(np.exp(-r2 / (2 * sigma * sigma)) * np.cos(ph))


def workload3(name: str) -> Workload3:
    """point3d: 96 x 96 x 64 smooth layered model, eps = 1/64, point source,
    q every 6 nodes, p 20^3 over [-2, 2]^3, tau = 1e-3, 100 RK4 steps of 1 ms."""
    if name == "point3d":
        grid = Grid3(96, 96, 64, 0.0, 0.0, 0.0, 1 / 64, 1 / 64, 1 / 64)
        eps = 1 / 64
        c = smooth_layered_velocity3(grid, seed=7)
        f0 = gaussian_source3(grid, (0.75, 0.75, 0.5), 2 * grid.d1)
        p = Params3(eps, (3, 3, 2), (6, 6, 6), (15, 15, 10), (20, 20, 20), (0.2, 0.2, 0.2),
                    1e-3, 1e-16, 1e-16, 1e-3, 100)
        return Workload3(name, grid, p, c, f0[None], None)
    raise KeyError(name)

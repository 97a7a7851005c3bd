"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This module holds no arithmetic of the frozen Gaussian approximation: it only
builds grids, velocity models, initial wavefields, receiver sets and the
numerical parameters of each workload.  Every array is float64, C-ordered
``[n2][n1]`` (axis 1 = x, horizontal, fastest; axis 2 = z, depth), on the
node-centred grid ``x_i = o + i*d``.

Workloads (units: km, s, km/s; T = 0.25 s and dt = 1 ms as in the paper's
numerical test section):

* ``wavepacket``   128 x 128 on [0,1]^2, c = 1, eps = 1/128, a Gaussian
  wavepacket of width 0.05 modulated by cos(x1/eps) with its one-way time
  derivative, q-mesh 64 x 64 (stride 2), p-mesh 32 x 32, tau = 1e-6.
* ``point512``     512 x 512 on [0,2]x[0,1], seeded smooth layered model with
  two lenses, eps = 1/256, a point-like Gaussian source (sigma = 2 cells),
  q-mesh 40 x 20 (strides 13, 26), p-mesh 112 x 112, tau = 1e-6.
* ``shots512``     the point512 model with 64 surface sources of random width
  and dominant wavenumber (uneven beam counts), q-mesh 20 x 10, p-mesh 56^2,
  tau = 1e-4.
* ``adjoint256``   256 x 256 on [0,2]x[0,1], eps = 1/128, 8 surface shots,
  receivers on the top row every 10 steps, perturbed "true" model.
* ``large2048``    2048 x 1024 on [0,2]x[0,1], eps = 1/1024, point source,
  q-mesh 147 x 74, p-mesh 400^2, tau = 1e-6.

The paper's own test uses the smoothed Marmousi model, which is not available
here; the seeded layered models below (smooth, layered, with lenses, 1.5-4.5
km/s) stand in for it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Grid", "Params", "Workload", "rng", "constant_velocity", "linear_velocity",
    "smooth_layered_velocity", "gaussian_anomaly", "gaussian_source",
    "wavepacket_source", "one_way_f1", "surface_shots", "workload",
    "WORKLOADS",
]


@dataclasses.dataclass(frozen=True)
class Grid:
    n1: int
    n2: int
    o1: float
    o2: float
    d1: float
    d2: float

    @property
    def shape(self):
        return (self.n2, self.n1)

    def coords(self):
        """Node coordinates (x1[n1], x2[n2])."""
        return (self.o1 + self.d1 * np.arange(self.n1),
                self.o2 + self.d2 * np.arange(self.n2))


@dataclasses.dataclass(frozen=True)
class Params:
    """Numerical parameters of one run (all lengths in km)."""
    eps: float
    qb1: int
    qb2: int
    qs1: int
    qs2: int
    nq1: int
    nq2: int
    np1: int
    np2: int
    dp1: float
    dp2: float
    tau: float          # relative threshold on |psi|
    tau_fbi: float      # truncation level of the FBI Gaussian window
    tau_win: float      # truncation level of the reconstruction window
    dt: float
    nsteps: int
    top_n: int = 0      # > 0: keep the top_n largest |psi| per branch and shot instead
    amp_closed: int = 0  # 1: a = c(Q)/c(q) (det Z)^(1/2) instead of integrating a
    dz_divided: int = 0  # 1: dzQ, dzP from divided differences of neighbouring rays
    dz_scale: float = 1.0  # their spacing in mesh steps (1: the neighbouring mesh nodes)
    deterministic: int = 0  # 1: gradients reduce dJ/dc in a fixed order (bit-identical runs)
    grad_log: int = 0  # dJ/dc logs per beam when not deterministic (0 auto, -1 none, n slots)
    ckpt_every_step: int = 0  # 1: checkpoints of every step (adjoints read, not recompute)

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    params: Params
    c: np.ndarray                 # [n2][n1]
    f0: np.ndarray                # [nshots][n2][n1]
    f1: Optional[np.ndarray]      # [nshots][n2][n1] or None (zero)
    receivers: Optional[np.ndarray] = None   # flat node indices (int32)
    rec_every: int = 0
    c_true: Optional[np.ndarray] = None

    @property
    def nshots(self) -> int:
        return self.f0.shape[0]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------- velocity

def constant_velocity(grid: Grid, c0: float = 1.0) -> np.ndarray:
    return np.full(grid.shape, float(c0))


def linear_velocity(grid: Grid, c0: float, g1: float, g2: float) -> np.ndarray:
    """c(x) = c0 + g1*x1 + g2*x2 sampled on the nodes."""
    x1, x2 = grid.coords()
    return c0 + g1 * x1[None, :] + g2 * x2[:, None]


def smooth_layered_velocity(grid: Grid, seed: int, smooth_cells: float = 8.0,
                            vmin: float = 1.5, vmax: float = 4.5) -> np.ndarray:
    """Seeded smooth layered model: 4 layers split by 3 folded interfaces,
    two Gaussian lenses, clipped to [vmin, vmax] and smoothed by a Gaussian
    of ``smooth_cells`` cells per axis."""
    from scipy.ndimage import gaussian_filter

    g = rng(seed)
    x1, x2 = grid.coords()
    X = grid.n1 * grid.d1
    Z = grid.n2 * grid.d2
    zbar = np.sort(g.uniform(0.2, 0.85, 3)) * Z
    amp = g.uniform(0.02, 0.08, 3) * Z
    lam = g.uniform(0.3, 1.0, 3) * X
    ph1 = g.uniform(0, 2 * np.pi, 3)
    ph2 = g.uniform(0, 2 * np.pi, 3)
    vel = np.sort(g.uniform(vmin, vmax, 4))
    c = np.full(grid.shape, vel[0])
    for j in range(3):
        zj = (zbar[j] + amp[j] * np.sin(2 * np.pi * x1 / lam[j] + ph1[j])
              + 0.5 * amp[j] * np.sin(4 * np.pi * x1 / lam[j] + ph2[j]))
        below = x2[:, None] > zj[None, :]
        c = np.where(below, vel[j + 1], c)
    for _ in range(2):
        cx = g.uniform(0.15, 0.85) * X + grid.o1
        cz = g.uniform(0.15, 0.85) * Z + grid.o2
        r = g.uniform(0.05, 0.15)
        a = g.uniform(0.3, 0.8) * (1.0 if g.uniform() < 0.5 else -1.0)
        c = c + a * np.exp(-((x1[None, :] - cx) ** 2 + (x2[:, None] - cz) ** 2) / (2 * r * r))
    c = np.clip(c, vmin, vmax)
    c = gaussian_filter(c, sigma=smooth_cells, mode="reflect", truncate=4.0)
    return np.ascontiguousarray(np.clip(c, vmin, vmax))


def gaussian_anomaly(grid: Grid, c: np.ndarray, center, width: float,
                     rel_amp: float) -> np.ndarray:
    x1, x2 = grid.coords()
    bump = np.exp(-((x1[None, :] - center[0]) ** 2 + (x2[:, None] - center[1]) ** 2)
                  / (2 * width * width))
    return np.ascontiguousarray(c * (1.0 + rel_amp * bump))


# ------------------------------------------------------------------ sources

def gaussian_source(grid: Grid, center, sigma: float) -> np.ndarray:
    x1, x2 = grid.coords()
    r2 = (x1[None, :] - center[0]) ** 2 + (x2[:, None] - center[1]) ** 2
    return np.ascontiguousarray(np.exp(-r2 / (2 * sigma * sigma)))


def wavepacket_source(grid: Grid, center, sigma: float, k, eps: float) -> np.ndarray:
    """exp(-|x-x0|^2/(2 sigma^2)) cos(k.(x-x0)/eps)."""
    x1, x2 = grid.coords()
    dx1 = x1[None, :] - center[0]
    dx2 = x2[:, None] - center[1]
    env = np.exp(-(dx1 ** 2 + dx2 ** 2) / (2 * sigma * sigma))
    return np.ascontiguousarray(env * np.cos((k[0] * dx1 + k[1] * dx2) / eps))


def one_way_f1(grid: Grid, f0: np.ndarray, c0: float) -> np.ndarray:
    """Time derivative that makes f0 travel in +x1 in a constant medium c0:
    f1 = F^-1[-i c0 |xi| sgn(xi1) F f0] on the periodic box."""
    xi1 = 2 * np.pi * np.fft.fftfreq(grid.n1, d=grid.d1)
    xi2 = 2 * np.pi * np.fft.fftfreq(grid.n2, d=grid.d2)
    mag = np.sqrt(xi1[None, :] ** 2 + xi2[:, None] ** 2)
    mult = -1j * c0 * mag * np.sign(xi1)[None, :]
    return np.ascontiguousarray(np.real(np.fft.ifft2(mult * np.fft.fft2(f0))))


def surface_shots(grid: Grid, nshots: int, seed: int, eps: float,
                  depth: float = 0.1):
    """Sources near the surface with seeded position, width (1-4 cells) and
    dominant wavenumber (0.5-2), aimed 60-120 degrees from horizontal
    (down-going)."""
    g = rng(seed)
    X = grid.n1 * grid.d1
    out = np.empty((nshots,) + grid.shape)
    for s in range(nshots):
        xs = g.uniform(0.05, 0.95) * X + grid.o1
        sig = g.uniform(1.0, 4.0) * grid.d1
        kap = g.uniform(0.5, 2.0)
        ang = math.radians(g.uniform(60.0, 120.0))
        k = (kap * math.cos(ang), kap * math.sin(ang))
        out[s] = wavepacket_source(grid, (xs, grid.o2 + depth), sig, k, eps)
    return out


# ---------------------------------------------------------------- workloads


def workload(name: str, precision: str = "fp64", nshots: Optional[int] = None) -> Workload:
    """Build one of the named workloads.  ``precision`` picks the window
    truncation levels: 1e-16 for the FP64 path, 1e-8 for the mixed path."""
    tw = 1e-16 if precision == "fp64" else 1e-8
    if name == "wavepacket":
        grid = Grid(128, 128, 0.0, 0.0, 1 / 128, 1 / 128)
        eps = 1 / 128
        c = constant_velocity(grid, 1.0)
        f0 = wavepacket_source(grid, (0.5, 0.5), 0.05, (1.0, 0.0), eps)
        f1 = one_way_f1(grid, f0, 1.0)
        p = Params(eps, 0, 0, 2, 2, 64, 64, 32, 32, 0.1125, 0.1125,
                   1e-6, tw, tw, 1e-3, 250)
        return Workload(name, grid, p, c, f0[None], f1[None])
    if name == "point512":
        grid = Grid(512, 512, 0.0, 0.0, 1 / 256, 1 / 512)
        eps = 1 / 256
        c = smooth_layered_velocity(grid, seed=2)
        f0 = gaussian_source(grid, (1.0, 0.5), 2 * grid.d1)
        p = Params(eps, 2, 8, 13, 26, 40, 20, 112, 112, 0.05, 0.05,
                   1e-6, tw, tw, 1e-3, 250)
        return Workload(name, grid, p, c, f0[None], None)
    if name == "topn512":
        # point512 with the N-largest selection of the paper's experiment
        # (N = 5650 beams per wave branch)
        W = workload("point512", precision)
        return Workload(name, W.grid, W.params.replace(top_n=5650), W.c, W.f0, None)
    if name == "shots512":
        grid = Grid(512, 512, 0.0, 0.0, 1 / 256, 1 / 512)
        eps = 1 / 256
        c = smooth_layered_velocity(grid, seed=2)
        ns = 64 if nshots is None else nshots
        f0 = surface_shots(grid, ns, seed=3, eps=eps)
        p = Params(eps, 8, 8, 26, 52, 20, 10, 56, 56, 0.1, 0.1,
                   1e-4, tw, tw, 1e-3, 250)
        return Workload(name, grid, p, c, f0, None)
    if name == "adjoint256":
        grid = Grid(256, 256, 0.0, 0.0, 1 / 128, 1 / 256)
        eps = 1 / 128
        c = smooth_layered_velocity(grid, seed=4)
        ns = 8 if nshots is None else nshots
        f0 = surface_shots(grid, ns, seed=4, eps=eps)
        p = Params(eps, 2, 2, 18, 36, 15, 8, 40, 40, 0.141, 0.141,
                   1e-4, tw, tw, 1e-3, 250)
        rec = np.arange(grid.n1, dtype=np.int32)          # top row, i2 = 0
        c_true = gaussian_anomaly(grid, c, (1.0, 0.5), 0.1, 0.05)
        return Workload(name, grid, p, c, f0, None, receivers=rec,
                        rec_every=10, c_true=c_true)
    if name == "large2048":
        grid = Grid(2048, 1024, 0.0, 0.0, 1 / 1024, 1 / 1024)
        eps = 1 / 1024
        c = smooth_layered_velocity(grid, seed=5)
        f0 = gaussian_source(grid, (1.0, 0.5), 2 * grid.d1)
        p = Params(eps, 3, 0, 14, 14, 147, 74, 400, 400, 0.0141, 0.0141,
                   1e-6, tw, tw, 1e-3, 250)
        return Workload(name, grid, p, c, f0[None], None)
    raise KeyError(name)


WORKLOADS = ("wavepacket", "point512", "topn512", "shots512", "adjoint256", "large2048")

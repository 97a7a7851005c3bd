"""Three-dimensional FP64 oracle of the frozen Gaussian approximation (test
infrastructure; see fga_oracle3.c for the arithmetic).  The numpy steps here
follow the paper's three-step algorithm (Algorithm section) exactly as the
two-dimensional oracle does: branch data u_{+-,0} = (f0 +- i eps/(c(q)|p|)
f1)/2 taken through the FBI, the relative threshold |psi| >= tau max |psi|
per shot over both branches, C = w psi / (2 pi eps)^{3d/2} with d = 3,
initial state Q = q, P = p, S = 0, A = I, B = -iI, a = 2^{d/2}."""
from __future__ import annotations

import ctypes
import dataclasses
import math
from typing import Optional

import numpy as np

from . import lib as _lib2d

NST3 = 45
_L = None


def lib():
    global _L
    if _L is None:
        L = _lib2d()
        P, I64, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        I32 = ctypes.c_int
        L.or3_velocity_points.argtypes = [P, I32, I32, I32, D, D, D, D, D, D, I64, P, P]
        L.or3_fbi.argtypes = [P, P, P, D, D, P, P, P, P, P, P]
        L.or3_rhs.argtypes = [P, P, P, P, D, P, P]
        L.or3_propagate.argtypes = [P, P, P, P, I64, P, P, D, I32]
        L.or3_reconstruct.argtypes = [P, P, P, D, D, I64, P, P, P]
        _L = L
    return _L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _iv(t):
    return np.ascontiguousarray(np.asarray(t, dtype=np.int32))


def _dv(t):
    return np.ascontiguousarray(np.asarray(t, dtype=np.float64))


def pmesh(n: int, dp: float) -> np.ndarray:
    return (np.arange(n) - 0.5 * (n - 1)) * dp


def velocity(c, grid, x):
    """[npts][10]: c, grad c (3), Hessian (11, 12, 13, 22, 23, 33) at x [npts][3]."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    out = np.empty((x.shape[0], 10))
    lib().or3_velocity_points(_p(c), grid.n1, grid.n2, grid.n3, grid.o1, grid.o2, grid.o3,
                              grid.d1, grid.d2, grid.d3, x.shape[0], _p(x), _p(out))
    return out


def fbi(f, grid, params):
    """psi [Nq][Np] complex (q and p flat with axis 1 fastest)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    NQ, NP = int(np.prod(params.nq)), int(np.prod(params.np))
    out = np.empty((NQ, NP, 2))
    lib().or3_fbi(_p(f), _p(_iv(grid.n)), _p(_dv(grid.d)), params.eps, params.tau_fbi,
                  _p(_iv(params.qb)), _p(_iv(params.qs)), _p(_iv(params.nq)),
                  _p(_iv(params.np)), _p(_dv(params.dp)), _p(out))
    return out[..., 0] + 1j * out[..., 1]


def qnodes(params):
    return [params.qb[a] + params.qs[a] * np.arange(params.nq[a]) for a in range(3)]


@dataclasses.dataclass
class Beams3:
    shot: np.ndarray
    sigma: np.ndarray
    cand: np.ndarray
    psi: np.ndarray
    coef: np.ndarray      # [nb][2]
    state: np.ndarray     # [nb][45]
    offsets: np.ndarray

    @property
    def n(self) -> int:
        return self.shot.size


def decompose(f0, f1, c, grid, params) -> Beams3:
    ns = f0.shape[0]
    NQ, NP = int(np.prod(params.nq)), int(np.prod(params.np))
    k = qnodes(params)
    qx = [grid.o[a] + grid.d[a] * k[a] for a in range(3)]
    pm = [pmesh(params.np[a], params.dp[a]) for a in range(3)]
    # q and p flat (axis 1 fastest)
    Q3, Q2, Q1 = np.meshgrid(qx[2], qx[1], qx[0], indexing="ij")
    qflat = np.stack([Q1.ravel(), Q2.ravel(), Q3.ravel()], 1)
    P3, P2, P1 = np.meshgrid(pm[2], pm[1], pm[0], indexing="ij")
    pflat = np.stack([P1.ravel(), P2.ravel(), P3.ravel()], 1)
    pn = np.linalg.norm(pflat, axis=1)
    w = float(np.prod([params.qs[a] * grid.d[a] for a in range(3)]) * np.prod(params.dp))
    norm = w / (2 * math.pi * params.eps) ** 4.5
    cq = velocity(c, grid, qflat)[:, 0]
    shots, sig, cand, psis, coefs, states = [], [], [], [], [], []
    offsets = [0]
    for s in range(ns):
        psi0 = fbi(f0[s], grid, params)
        if f1 is not None:
            psi1 = fbi(f1[s], grid, params)
            r = params.eps / (cq[:, None] * pn[None, :])
            br = [0.5 * (psi0 + 1j * r * psi1), 0.5 * (psi0 - 1j * r * psi1)]
        else:
            br = [0.5 * psi0, 0.5 * psi0]
        M = max(np.abs(br[0]).max(), np.abs(br[1]).max())
        for b, sg in ((0, 1), (1, -1)):
            mag = np.abs(br[b]).ravel()
            keep = np.nonzero((mag >= params.tau * M) & (mag > 0))[0]
            qf, pf = keep // NP, keep % NP
            st = np.zeros((keep.size, NST3))
            st[:, 0:3] = qflat[qf]
            st[:, 3:6] = pflat[pf]
            for j in range(3):
                st[:, 7 + 2 * (3 * j + j)] = 1.0          # A = I
                st[:, 26 + 2 * (3 * j + j)] = -1.0        # B = -iI
            st[:, 43] = 2.0 ** 1.5
            ps = br[b].ravel()[keep]
            shots.append(np.full(keep.size, s, np.int32))
            sig.append(np.full(keep.size, sg, np.int8))
            cand.append(((s * 2 + b) * NQ + qf) * NP + pf)
            psis.append(ps)
            coefs.append(np.stack([(norm * ps).real, (norm * ps).imag], 1))
            states.append(st)
        offsets.append(offsets[-1] + sum(x.size for x in shots[-2:]))
    return Beams3(np.concatenate(shots), np.concatenate(sig), np.concatenate(cand).astype(np.int64),
                  np.concatenate(psis), np.concatenate(coefs), np.concatenate(states),
                  np.array(offsets, np.int64))


def rhs(y, sigma, c, grid):
    c = np.ascontiguousarray(c, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    dy = np.empty(NST3)
    lib().or3_rhs(_p(c), _p(_iv(grid.n)), _p(_dv(grid.o)), _p(_dv(grid.d)), float(sigma),
                  _p(y), _p(dy))
    return dy


def propagate(beams: Beams3, c, grid, dt: float, nsteps: int) -> None:
    c = np.ascontiguousarray(c, dtype=np.float64)
    sig = np.ascontiguousarray(beams.sigma, dtype=np.int8)
    assert beams.state.flags.c_contiguous
    lib().or3_propagate(_p(c), _p(_iv(grid.n)), _p(_dv(grid.o)), _p(_dv(grid.d)), beams.n,
                        _p(sig), _p(beams.state), dt, nsteps)


def reconstruct(beams: Beams3, grid, params, shot: Optional[int] = None):
    sl = slice(None) if shot is None else slice(int(beams.offsets[shot]),
                                                int(beams.offsets[shot + 1]))
    coef = np.ascontiguousarray(beams.coef[sl])
    st = np.ascontiguousarray(beams.state[sl])
    u = np.empty(grid.shape)
    lib().or3_reconstruct(_p(_iv(grid.n)), _p(_dv(grid.o)), _p(_dv(grid.d)), params.eps,
                          params.tau_win, coef.shape[0], _p(coef), _p(st), _p(u))
    return u


def forward(f0, f1, c, grid, params):
    b = decompose(f0, f1, c, grid, params)
    propagate(b, c, grid, params.dt, params.nsteps)
    return b, [reconstruct(b, grid, params, shot=s) for s in range(f0.shape[0])]

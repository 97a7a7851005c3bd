"""Plain FP64 CPU oracle of the frozen Gaussian approximation (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this package.  It shares no code with the HIP path: the
arithmetic lives in ``fga_oracle.c`` (direct double-precision loops) and in
the few numpy steps below (branch combination, thresholding, beam set-up),
each following the paper's three-step algorithm (Algorithm section):

1. decomposition: FBI transform of f0 and f1 (psi eq. and its rewriting as a
   windowed Fourier transform, Initial wavefield decomposition section),
   branch data u_{+-,0} = (f0 +- i eps/(c(q)|p|) f1)/2, and thresholding;
2. propagation: the characteristic equations for H = +-c(Q)|P|, the dynamic
   ray tracing equations for dzQ, dzP and the amplitude equation, integrated
   by classical RK4 (Numerical test section);
3. reconstruction: the frozen-Gaussian sum (recons eq.).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fga_oracle.c")
LIB = os.path.join(HERE, "_fga_oracle.so")
NSTATE = 23

_lib = None


def build() -> str:
    """Compile the C oracle with gcc (OpenMP, -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-o", LIB + ".tmp", SRC, os.path.join(HERE, "fga_oracle3.c"), "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        I32, I64, D = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        G = [P, I32, I32, D, D, D, D]
        L.or_velocity.argtypes = G + [D, D, P]
        L.or_fbi_bound.argtypes = [P, I32, I32, D, D, D, D, I32, I32, I32, I32, I32,
                                   I32, P]
        L.or_velocity_points.argtypes = G + [I64, P, P, P]
        L.or_fbi.argtypes = [P, I32, I32, D, D, D, D, I32, I32, I32, I32, I32,
                             I32, I32, I32, D, D, P]
        L.or_propagate.argtypes = G + [I64, P, P, D, I32]
        L.or_propagate_closed.argtypes = G + [I64, P, P, P, D, I32]
        L.or_propagate_dd.argtypes = G + [I64, P, P, P, D, I32, P]
        L.or_rhs.argtypes = G + [D, P, P]
        L.or_reconstruct.argtypes = [I32, I32, D, D, D, D, D, D, I64, P, P, P, P]
        L.or_reconstruct_points.argtypes = [I32, I32, D, D, D, D, D, D, I64, P,
                                            P, I64, P, P, P]
        L.or_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _grid_args(c, grid):
    return [_p(c), grid.n1, grid.n2, grid.o1, grid.o2, grid.d1, grid.d2]


def threads() -> int:
    return int(lib().or_max_threads())


# ------------------------------------------------------------ velocity

def velocity(c: np.ndarray, grid, x1, x2) -> np.ndarray:
    """Cubic B-spline interpolant of c and its derivatives up to third order
    at the points (x1, x2): columns c, c1, c2, c11, c12, c22, c111, c112,
    c122, c222."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    x1 = np.ascontiguousarray(np.atleast_1d(x1), dtype=np.float64)
    x2 = np.ascontiguousarray(np.atleast_1d(x2), dtype=np.float64)
    out = np.empty((x1.size, 10))
    lib().or_velocity_points(*_grid_args(c, grid), x1.size, _p(x1), _p(x2), _p(out))
    return out


# ------------------------------------------------------ step 1: decompose

def pmesh(n: int, dp: float) -> np.ndarray:
    """Staggered symmetric p-mesh: p_l = (l - (n-1)/2) dp."""
    return (np.arange(n) - 0.5 * (n - 1)) * dp


def qnodes(params):
    k1 = params.qb1 + params.qs1 * np.arange(params.nq1)
    k2 = params.qb2 + params.qs2 * np.arange(params.nq2)
    return k1, k2


def fbi(f: np.ndarray, grid, params) -> np.ndarray:
    """psi(q, p) of the FBI transform as complex [nq2][nq1][np2][np1]."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    pr = params
    out = np.empty((pr.nq2, pr.nq1, pr.np2, pr.np1, 2))
    lib().or_fbi(_p(f), grid.n1, grid.n2, grid.d1, grid.d2, pr.eps, pr.tau_fbi,
                 pr.qb1, pr.qb2, pr.qs1, pr.qs2, pr.nq1, pr.nq2, pr.np1, pr.np2,
                 pr.dp1, pr.dp2, _p(out))
    return out[..., 0] + 1j * out[..., 1]


def fbi_bound(f: np.ndarray, grid, params) -> np.ndarray:
    """d1 d2 sum_m |f(k+m)| exp(-|m d|^2/(2 eps)) over the FBI box of every q
    node, [nq2][nq1]: no |psi(q, p)| exceeds it, whatever p (the Fourier
    factor of the psi eq. has modulus 1)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    pr = params
    out = np.empty((pr.nq2, pr.nq1))
    lib().or_fbi_bound(_p(f), grid.n1, grid.n2, grid.d1, grid.d2, pr.eps, pr.tau_fbi,
                       pr.qb1, pr.qb2, pr.qs1, pr.qs2, pr.nq1, pr.nq2, _p(out))
    return out


@dataclasses.dataclass
class Beams:
    """Thresholded beams in the order (shot, branch + then -, q flat, p flat)."""
    shot: np.ndarray      # int32 [nb]
    sigma: np.ndarray     # int8  [nb]  (+1 / -1)
    cand: np.ndarray      # int64 [nb]  ((shot*2 + (sigma<0))*Nq + qflat)*Np + pflat
    psi: np.ndarray       # complex [nb]  psi_{+-}(q, p)
    coef: np.ndarray      # [nb][2]  w psi / (2 pi eps)^3
    state: np.ndarray     # [nb][23]
    offsets: np.ndarray   # int64 [nshots+1]

    @property
    def n(self) -> int:
        return self.shot.size

    def subset(self, idx) -> "Beams":
        idx = np.asarray(idx)
        return Beams(self.shot[idx], self.sigma[idx], self.cand[idx],
                     self.psi[idx], np.ascontiguousarray(self.coef[idx]),
                     np.ascontiguousarray(self.state[idx]),
                     np.array([0, idx.size], dtype=np.int64))


def branches(psi0, psi1, c, grid, params):
    """psi_{+-} = (psi0 +- i eps / (c(q)|p|) psi1) / 2  (u_{+-,0} in the psi eq.)."""
    k1, k2 = qnodes(params)
    q1 = grid.o1 + grid.d1 * k1
    q2 = grid.o2 + grid.d2 * k2
    Q1, Q2 = np.meshgrid(q1, q2)                       # [nq2][nq1]
    cq = velocity(c, grid, Q1.ravel(), Q2.ravel())[:, 0].reshape(Q1.shape)
    p1 = pmesh(params.np1, params.dp1)
    p2 = pmesh(params.np2, params.dp2)
    pabs = np.sqrt(p1[None, :] ** 2 + p2[:, None] ** 2)  # [np2][np1]
    if psi1 is None:
        return 0.5 * psi0, 0.5 * psi0
    ratio = 1j * params.eps / (cq[:, :, None, None] * pabs[None, None, :, :])
    return 0.5 * (psi0 + ratio * psi1), 0.5 * (psi0 - ratio * psi1)


def select_top_n(mags: np.ndarray, n: int) -> np.ndarray:
    """Indices of the n largest entries of mags (one branch of one shot), as
    in the Numerical test section (the N largest amplitudes of psi_+- for
    each wave branch), in increasing index order.  Equal magnitudes are
    taken in increasing index order; zero magnitudes are never taken, so
    fewer than n come back when fewer are nonzero."""
    order = np.lexsort((np.arange(mags.size), -mags))   # by -|psi|, then index
    sel = order[:n]
    return np.sort(sel[mags[sel] > 0])


def _branch_bound(f0s, f1s, c, grid, pr) -> np.ndarray:
    """A bound of |psi_+-(q, p)| over every p, per q node (flat): from
    |psi_+-| <= (|psi0| + eps/(c(q)|p|) |psi1|)/2 with the fbi_bound of each
    and |p| at least the smallest |p| of the staggered mesh."""
    b = 0.5 * fbi_bound(f0s, grid, pr).ravel()
    if f1s is not None:
        k1, k2 = qnodes(pr)
        Q1, Q2 = np.meshgrid(grid.o1 + grid.d1 * k1, grid.o2 + grid.d2 * k2)
        cq = velocity(c, grid, Q1.ravel(), Q2.ravel())[:, 0]
        pmin = math.hypot(0.5 * pr.dp1, 0.5 * pr.dp2)
        b = b + 0.5 * pr.eps / (cq * pmin) * fbi_bound(f1s, grid, pr).ravel()
    return b


def _skipped_q_candidates(f0s, f1s, c, grid, pr):
    """psi_+- at the q nodes that can hold a kept beam, for the relative
    threshold: q nodes are visited in decreasing order of their bound
    (_branch_bound) while the bound reaches tau times the largest |psi_+-|
    found so far.  Every q node left out has |psi_+-| below tau M at every p
    (its bound is, and M is at least the running maximum), so it keeps no
    beam, and M itself is attained at a visited node.  Returns the visited q
    nodes in increasing flat order and their psi_+ and psi_- [nvisited][np]."""
    bnd = _branch_bound(f0s, f1s, c, grid, pr)
    order = np.argsort(-bnd, kind="stable")
    found = {}
    run = 0.0
    slack = 1.0 + 1e-9          # rounding of the bound and of |psi|
    for q in order:
        if bnd[q] * slack < pr.tau * run:
            break
        j2, j1 = divmod(int(q), pr.nq1)
        one = dataclasses.replace(pr, qb1=pr.qb1 + pr.qs1 * j1, qb2=pr.qb2 + pr.qs2 * j2,
                                  nq1=1, nq2=1)
        psi0 = fbi(f0s, grid, one)
        psi1 = None if f1s is None else fbi(f1s, grid, one)
        pp, pm = branches(psi0, psi1, c, grid, one)
        found[int(q)] = (pp.ravel(), pm.ravel())
        run = max(run, float(np.abs(pp).max()), float(np.abs(pm).max()))
    qs = np.array(sorted(found), dtype=np.int64)
    pp = np.stack([found[q][0] for q in qs])
    pm = np.stack([found[q][1] for q in qs])
    return qs, pp, pm


def decompose(f0: np.ndarray, f1: Optional[np.ndarray], c, grid, params,
              psi_cache=None, q_skip: bool = False) -> Beams:
    """Step 1 for every shot: FBI, branch split, selection, initial state.

    With params.top_n == 0, thresholding keeps (sigma, q, p) with
    |psi_sigma| >= tau * M, M the largest |psi| over both branches of the
    shot, and |psi| > 0; with top_n > 0 each branch keeps its top_n largest
    |psi_sigma| (select_top_n).  q_skip (threshold only) evaluates the FBI
    only at q nodes whose bound can reach tau M (_skipped_q_candidates):
    the same beams, for sources much smaller than the q-mesh.
    """
    pr = params
    k1, k2 = qnodes(pr)
    p1m = pmesh(pr.np1, pr.dp1)
    p2m = pmesh(pr.np2, pr.dp2)
    nq = pr.nq1 * pr.nq2
    npp = pr.np1 * pr.np2
    w = (pr.qs1 * grid.d1) * (pr.qs2 * grid.d2) * pr.dp1 * pr.dp2
    norm = w / (2 * math.pi * pr.eps) ** 3          # (2 pi eps)^{-3d/2}, d = 2
    if q_skip and pr.top_n > 0:
        raise ValueError("q_skip applies to the relative threshold only")
    parts = []
    offsets = [0]
    for s in range(f0.shape[0]):
        qlist = None
        if q_skip:
            qlist, pp, pm = _skipped_q_candidates(f0[s], None if f1 is None else f1[s],
                                                  c, grid, pr)
        elif psi_cache is not None and s in psi_cache:
            psi0, psi1 = psi_cache[s]
            pp, pm = branches(psi0, psi1, c, grid, pr)
        else:
            psi0 = fbi(f0[s], grid, pr)
            psi1 = None if f1 is None else fbi(f1[s], grid, pr)
            pp, pm = branches(psi0, psi1, c, grid, pr)
        mags = np.stack([np.abs(pp).ravel(), np.abs(pm).ravel()])   # [2][nq*np]
        if pr.top_n > 0:
            keep = np.zeros(mags.shape, bool)
            for br in range(2):
                keep[br, select_top_n(mags[br], pr.top_n)] = True
        else:
            M = mags.max()
            keep = (mags >= pr.tau * M) & (mags > 0)
        vals = np.stack([pp.ravel(), pm.ravel()])
        sidx, flat = np.nonzero(keep)           # row-major: branch +, then -
        qf, pf = flat // npp, flat % npp
        if qlist is not None:
            # visited q nodes (increasing) -> mesh flat index: the order stays
            # (branch, q flat, p flat)
            qf = qlist[qf]
        j2, j1 = qf // pr.nq1, qf % pr.nq1
        l2, l1 = pf // pr.np1, pf % pr.np1
        nb = flat.size
        st = np.zeros((nb, NSTATE))
        st[:, 0] = grid.o1 + grid.d1 * k1[j1]
        st[:, 1] = grid.o2 + grid.d2 * k2[j2]
        st[:, 2] = p1m[l1]
        st[:, 3] = p2m[l2]
        # A = dzQ(0) = I, B = dzP(0) = -i I (dz = dq - i dp applied to Q = q, P = p)
        st[:, 5] = 1.0
        st[:, 11] = 1.0
        st[:, 14] = -1.0
        st[:, 20] = -1.0
        st[:, 21] = 2.0      # a(0) = 2^{d/2}
        psi = vals[sidx, flat]
        coef = np.stack([psi.real * norm, psi.imag * norm], axis=1)
        cand = ((s * 2 + sidx) * nq + qf) * npp + pf
        parts.append((np.full(nb, s, np.int32), np.where(sidx == 0, 1, -1).astype(np.int8),
                      cand.astype(np.int64), psi, coef, st))
        offsets.append(offsets[-1] + nb)
    cat = [np.concatenate([p[i] for p in parts]) for i in range(6)]
    return Beams(cat[0], cat[1], cat[2], cat[3], np.ascontiguousarray(cat[4]),
                 np.ascontiguousarray(cat[5]), np.array(offsets, dtype=np.int64))


# ----------------------------------------------------- step 2: propagate

def beam_nodes(beams: Beams, grid, params) -> np.ndarray:
    """The mesh node q [nb][2] of every beam, from its candidate index."""
    nq, npp = params.nq1 * params.nq2, params.np1 * params.np2
    qf = (beams.cand // npp) % nq
    k1, k2 = qnodes(params)
    return np.stack([grid.o1 + grid.d1 * k1[qf % params.nq1],
                     grid.o2 + grid.d2 * k2[qf // params.nq1]], 1)


def propagate(beams: Beams, c, grid, dt: float, nsteps: int, q=None, dd=None) -> None:
    """Classical RK4 of the ray, dynamic ray tracing and amplitude equations,
    in place on beams.state.  With q ([nb][2], the beams' mesh nodes) the
    amplitude is instead a = c(Q)/c(q) (det Z)^{1/2} after every step, the
    root continuous in time (the closed form following the amplitude
    equation, Formulation section).  With dd = (h_q1, h_q2, h_p1, h_p2) as
    well, dzQ and dzP come from central divided differences of the rays of
    the neighbouring mesh nodes at these spacings instead of the dynamic ray
    tracing equations (or_propagate_dd)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    sig = np.ascontiguousarray(beams.sigma, dtype=np.int8)
    assert beams.state.flags.c_contiguous and beams.state.dtype == np.float64
    if q is None:
        assert dd is None, "the divided-difference mode takes the closed-form amplitude"
        lib().or_propagate(*_grid_args(c, grid), beams.n, _p(sig), _p(beams.state),
                           dt, nsteps)
        return
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.shape == (beams.n, 2)
    if dd is None:
        lib().or_propagate_closed(*_grid_args(c, grid), beams.n, _p(sig), _p(q),
                                  _p(beams.state), dt, nsteps)
    else:
        h = np.ascontiguousarray(dd, dtype=np.float64)
        assert h.shape == (4,) and np.all(h > 0)
        lib().or_propagate_dd(*_grid_args(c, grid), beams.n, _p(sig), _p(q),
                              _p(beams.state), dt, nsteps, _p(h))


def dd_spacings(grid, params):
    """Spacings of the divided differences: dz_scale times the mesh steps
    (qs1 d1, qs2 d2, dp1, dp2); dz_scale = 1 gives the neighbouring nodes of
    the mesh."""
    s = float(getattr(params, "dz_scale", 1.0))
    return (s * (params.qs1 * grid.d1), s * (params.qs2 * grid.d2), s * params.dp1,
            s * params.dp2)


def _prop_mode(beams, grid, params):
    q = beam_nodes(beams, grid, params) if params.amp_closed else None
    dd = dd_spacings(grid, params) if getattr(params, "dz_divided", 0) else None
    return q, dd


def rhs(y, sigma: float, c, grid) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    dy = np.empty(NSTATE)
    lib().or_rhs(*_grid_args(c, grid), float(sigma), _p(y), _p(dy))
    return dy


# -------------------------------------------------- step 3: reconstruct

def reconstruct(beams: Beams, grid, params, shot: Optional[int] = None,
                imag: bool = False):
    """u(x) on the whole grid from the beams of one shot (recons eq.)."""
    sl = slice(None)
    if shot is not None:
        sl = slice(int(beams.offsets[shot]), int(beams.offsets[shot + 1]))
    coef = np.ascontiguousarray(beams.coef[sl])
    st = np.ascontiguousarray(beams.state[sl])
    ure = np.empty(grid.shape)
    uim = np.empty(grid.shape) if imag else None
    lib().or_reconstruct(grid.n1, grid.n2, grid.o1, grid.o2, grid.d1, grid.d2,
                         params.eps, params.tau_win, coef.shape[0], _p(coef),
                         _p(st), _p(ure), _p(uim))
    return (ure, uim) if imag else ure


def reconstruct_points(beams: Beams, grid, params, nodes, shot: Optional[int] = None,
                       imag: bool = False):
    """The reconstruction sum at a list of flat node indices (i2*n1 + i1)."""
    sl = slice(None)
    if shot is not None:
        sl = slice(int(beams.offsets[shot]), int(beams.offsets[shot + 1]))
    coef = np.ascontiguousarray(beams.coef[sl])
    st = np.ascontiguousarray(beams.state[sl])
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    ore = np.empty(nodes.size)
    oim = np.empty(nodes.size) if imag else None
    lib().or_reconstruct_points(grid.n1, grid.n2, grid.o1, grid.o2, grid.d1,
                                grid.d2, params.eps, params.tau_win,
                                coef.shape[0], _p(coef), _p(st), nodes.size,
                                _p(nodes), _p(ore), _p(oim))
    return (ore, oim) if imag else ore


def trace(beams: Beams, c, grid, params, receivers, rec_every: int,
          nrec: int) -> np.ndarray:
    """Receiver traces [nshots][nrec][len(receivers)]: u at the receiver nodes
    at t_k = k * rec_every * dt, k = 1..nrec (beams are advanced in place)."""
    ns = beams.offsets.size - 1
    out = np.empty((ns, nrec, len(receivers)))
    q, dd = _prop_mode(beams, grid, params)
    for k in range(nrec):
        propagate(beams, c, grid, params.dt, rec_every, q=q, dd=dd)
        for s in range(ns):
            out[s, k] = reconstruct_points(beams, grid, params, receivers, shot=s)
    return out


def frozen_beams(f0, f1, c, grid, params, cand, psi_cache=None) -> Beams:
    """The initial beams of a given candidate set (the threshold set held
    fixed): coefficients from the FBI of f0 (and f1) at their (q, p) nodes,
    the t = 0 state of step 1.  psi_cache {shot: (psi0, psi1)} may hold FBI
    values already computed for these f0, f1."""
    pr = params
    ns = f0.shape[0]
    nq, npp = pr.nq1 * pr.nq2, pr.np1 * pr.np2
    k1, k2 = qnodes(pr)
    pm1, pm2 = pmesh(pr.np1, pr.dp1), pmesh(pr.np2, pr.dp2)
    w = (pr.qs1 * grid.d1) * (pr.qs2 * grid.d2) * pr.dp1 * pr.dp2
    norm = w / (2 * math.pi * pr.eps) ** 3
    coef, states, sig, shot, psis, offs = [], [], [], [], [], [0]
    for s in range(ns):
        if psi_cache is not None and s in psi_cache:
            psi0, psi1 = psi_cache[s]
        else:
            psi0 = fbi(f0[s], grid, pr)
            psi1 = None if f1 is None else fbi(f1[s], grid, pr)
        pp, pm = branches(psi0, psi1, c, grid, pr)
        vals = np.stack([pp.ravel(), pm.ravel()])
        mine = cand[(cand // (2 * nq * npp)) == s] - s * 2 * nq * npp
        sb, flat = mine // (nq * npp), mine % (nq * npp)
        psi = vals[sb, flat]
        qf, pf = flat // npp, flat % npp
        st = np.zeros((mine.size, NSTATE))
        st[:, 0] = grid.o1 + grid.d1 * k1[qf % pr.nq1]
        st[:, 1] = grid.o2 + grid.d2 * k2[qf // pr.nq1]
        st[:, 2] = pm1[pf % pr.np1]
        st[:, 3] = pm2[pf // pr.np1]
        st[:, 5] = st[:, 11] = 1.0
        st[:, 14] = st[:, 20] = -1.0
        st[:, 21] = 2.0
        coef.append(np.stack([psi.real, psi.imag], 1) * norm)
        states.append(st)
        sig.append(np.where(sb == 0, 1, -1).astype(np.int8))
        shot.append(np.full(mine.size, s, np.int32))
        psis.append(psi)
        offs.append(offs[-1] + mine.size)
    return Beams(np.concatenate(shot), np.concatenate(sig), np.asarray(cand, np.int64).copy(),
                 np.concatenate(psis), np.ascontiguousarray(np.concatenate(coef)),
                 np.ascontiguousarray(np.concatenate(states)), np.array(offs, np.int64))


def trace_frozen(c, f0, f1, grid, params, cand, receivers, rec_every, nrec,
                 c_for_branches=None, psi_cache=None) -> np.ndarray:
    """Receiver traces (trace) of the beams `cand` with the threshold set held
    fixed, for velocity c and initial data f0, f1 (c_for_branches, if given,
    is the velocity whose c(q) enters u_{+-,0})."""
    cb = c if c_for_branches is None else c_for_branches
    b = frozen_beams(f0, f1, cb, grid, params, cand, psi_cache)
    return trace(b, c, grid, params, receivers, rec_every, nrec)


def forward(f0, f1, c, grid, params, imag=False):
    """The whole three-step algorithm: u(T) for every shot."""
    b = decompose(f0, f1, c, grid, params)
    q, dd = _prop_mode(b, grid, params)
    propagate(b, c, grid, params.dt, params.nsteps, q=q, dd=dd)
    us = [reconstruct(b, grid, params, shot=s, imag=imag) for s in range(f0.shape[0])]
    return b, us

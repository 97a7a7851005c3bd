"""Write the oracle's values for the full-size workloads at sampled points.

Calls only ``oracle`` and ``fga_inputs``.  The full-size oracle runs take
minutes, so their results at a seeded sample of output nodes are stored here
for the GPU tests (which compare the HIP path at the same nodes):

  point512_fp64.npz   512 x 512 smooth layered model, eps = 1/256, point
                      source, tau = 1e-6, FP64 windows (1e-16): beam count,
                      a sample of beams (id, coefficient, state at T) and
                      u(T) at 2048 seeded nodes.
  wavepacket_fp64.npz 128 x 128, c = 1, eps = 1/128, one-way wavepacket:
                      the same items, nodes plus the packet's row.

  large2048_fp64.npz  2048 x 1024 smooth layered model, eps = 1/1024, point
                      source, tau = 1e-6, FP64 windows: beam count and
                      offsets, a seeded sample of beams (id, coefficient,
                      state at T) and u(T) at 1024 seeded nodes plus the
                      nodes nearest 1024 seeded beams' centres at T.  The
                      FBI is evaluated only at the q nodes whose bound can
                      reach the threshold (oracle.decompose(q_skip=True):
                      the same beams); about 1.5 h on 8 cores.
  adjoint256_fp64.npz 256 x 256, 8 surface shots, receivers on the top row
                      every 10 steps: the oracle's traces on the model with
                      the +5 % anomaly (the misfit data), the misfit J on the
                      background model, and central differences of J with
                      the beam set held fixed at seeded velocity cells (and
                      cells under the sources) and at seeded f0 nodes.

Usage: python tests/golden/make_golden.py [point512] [wavepacket] [large2048] [adjoint256]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import fga_inputs as fi  # noqa: E402
import oracle  # noqa: E402


def sample_nodes(grid, n, seed):
    r = fi.rng(seed)
    return np.sort(r.choice(grid.n1 * grid.n2, size=n, replace=False)).astype(np.int64)


def point512():
    W = fi.workload("point512", "fp64")
    g, p = W.grid, W.params
    t0 = time.time()
    b = oracle.decompose(W.f0, W.f1, W.c, g, p)
    t1 = time.time()
    print(f"decompose: {b.n} beams in {t1 - t0:.1f} s", flush=True)
    rs = fi.rng(1234)
    pick = np.sort(rs.choice(b.n, size=min(4096, b.n), replace=False))
    oracle.propagate(b, W.c, g, p.dt, p.nsteps)
    t2 = time.time()
    print(f"propagate: {t2 - t1:.1f} s", flush=True)
    nodes = sample_nodes(g, 2048, 99)
    u_re, u_im = oracle.reconstruct_points(b, g, p, nodes, shot=0, imag=True)
    t3 = time.time()
    print(f"reconstruct at {nodes.size} nodes: {t3 - t2:.1f} s", flush=True)
    np.savez_compressed(
        os.path.join(HERE, "point512_fp64.npz"),
        nbeams=np.int64(b.n), offsets=b.offsets, pick=pick, ids=b.cand[pick],
        coef=b.coef[pick], stateT=b.state[pick], nodes=nodes, u=u_re, u_im=u_im,
        seconds=np.array([t1 - t0, t2 - t1, t3 - t2]))


def wavepacket():
    """128 x 128, c = 1, eps = 1/128, one-way wavepacket, tau = 1e-6, FP64
    windows: beam count and u(T) at 2048 seeded nodes and at every node of
    row 64 (the packet's row)."""
    W = fi.workload("wavepacket", "fp64")
    g, p = W.grid, W.params
    t0 = time.time()
    b = oracle.decompose(W.f0, W.f1, W.c, g, p)
    t1 = time.time()
    print(f"decompose: {b.n} beams in {t1 - t0:.1f} s", flush=True)
    rs = fi.rng(4321)
    pick = np.sort(rs.choice(b.n, size=min(4096, b.n), replace=False))
    oracle.propagate(b, W.c, g, p.dt, p.nsteps)
    t2 = time.time()
    print(f"propagate: {t2 - t1:.1f} s", flush=True)
    nodes = np.unique(np.concatenate([sample_nodes(g, 2048, 98),
                                      64 * g.n1 + np.arange(g.n1)])).astype(np.int64)
    u_re, u_im = oracle.reconstruct_points(b, g, p, nodes, shot=0, imag=True)
    t3 = time.time()
    print(f"reconstruct at {nodes.size} nodes: {t3 - t2:.1f} s", flush=True)
    np.savez_compressed(
        os.path.join(HERE, "wavepacket_fp64.npz"),
        nbeams=np.int64(b.n), offsets=b.offsets, pick=pick, ids=b.cand[pick],
        coef=b.coef[pick], stateT=b.state[pick], nodes=nodes, u=u_re, u_im=u_im,
        seconds=np.array([t1 - t0, t2 - t1, t3 - t2]))


def large2048():
    W = fi.workload("large2048", "fp64")
    g, p = W.grid, W.params
    t0 = time.time()
    b = oracle.decompose(W.f0, W.f1, W.c, g, p, q_skip=True)
    t1 = time.time()
    print(f"decompose: {b.n} beams in {t1 - t0:.1f} s", flush=True)
    rs = fi.rng(2048)
    pick = np.sort(rs.choice(b.n, size=min(4096, b.n), replace=False))
    coef_pick = b.coef[pick].copy()
    chunk = 1 << 21
    for i in range(0, b.n, chunk):
        j = min(b.n, i + chunk)
        part = oracle.Beams(b.shot[i:j], b.sigma[i:j], b.cand[i:j], b.psi[i:j],
                            b.coef[i:j], b.state[i:j], np.array([0, j - i], np.int64))
        oracle.propagate(part, W.c, g, p.dt, p.nsteps)
        print(f"propagate: {j} of {b.n} beams, {time.time() - t1:.0f} s", flush=True)
    t2 = time.time()
    # 1024 uniform nodes and the nodes nearest 1024 seeded beams' centres at T
    # (where the field is large)
    near = np.sort(rs.choice(b.n, size=1024, replace=False))
    i1 = np.clip(np.floor((b.state[near, 0] - g.o1) / g.d1 + 0.5), 0, g.n1 - 1).astype(np.int64)
    i2 = np.clip(np.floor((b.state[near, 1] - g.o2) / g.d2 + 0.5), 0, g.n2 - 1).astype(np.int64)
    nodes = np.unique(np.concatenate([sample_nodes(g, 1024, 97), i2 * g.n1 + i1]))
    u_re, u_im = oracle.reconstruct_points(b, g, p, nodes, shot=0, imag=True)
    t3 = time.time()
    print(f"reconstruct at {nodes.size} nodes: {t3 - t2:.1f} s", flush=True)
    np.savez_compressed(
        os.path.join(HERE, "large2048_fp64.npz"),
        nbeams=np.int64(b.n), offsets=b.offsets, pick=pick, ids=b.cand[pick],
        coef=coef_pick, stateT=b.state[pick], nodes=nodes, u=u_re, u_im=u_im,
        seconds=np.array([t1 - t0, t2 - t1, t3 - t2]))


def adjoint256():
    W = fi.workload("adjoint256", "fp64")
    g, p = W.grid, W.params
    ns = W.nshots
    nrec = p.nsteps // W.rec_every
    rec = W.receivers
    t0 = time.time()
    b = oracle.decompose(W.f0, None, W.c, g, p)
    cand = b.cand
    # f1 = 0: psi_+- = psi0 / 2 does not depend on c, so one FBI serves
    # every velocity below
    cache = {s: (oracle.fbi(W.f0[s], g, p), None) for s in range(ns)}
    print(f"decompose: {b.n} beams in {time.time() - t0:.1f} s", flush=True)
    data = oracle.trace_frozen(W.c_true, W.f0, None, g, p, cand, rec, W.rec_every, nrec,
                               psi_cache=cache)
    tr0 = oracle.trace_frozen(W.c, W.f0, None, g, p, cand, rec, W.rec_every, nrec,
                              psi_cache=cache)
    J0 = 0.5 * float(((tr0 - data) ** 2).sum())
    print(f"data and J0 = {J0:.6e}: {time.time() - t0:.1f} s", flush=True)

    def J_c(cg):
        tr = oracle.trace_frozen(cg, W.f0, None, g, p, cand, rec, W.rec_every, nrec,
                                 psi_cache=cache)
        return 0.5 * float(((tr - data) ** 2).sum())

    # velocity cells: 8 seeded anywhere, and the node of each shot's source
    # with its neighbour 4 cells down (where every ray of the shot starts)
    r = fi.rng(256)
    cells = list(r.choice(g.n1 * g.n2, 8, replace=False))
    x1, x2 = g.coords()
    for s in range(ns):
        k = int(np.argmax(np.abs(W.f0[s])))
        cells += [k, k + 4 * g.n1]
    cells = np.array(cells, np.int64)
    fd_c = np.empty(cells.size)
    for n, k in enumerate(cells):
        i2, i1 = divmod(int(k), g.n1)
        h = 1e-6 * W.c[i2, i1]
        cp, cm = W.c.copy(), W.c.copy()
        cp[i2, i1] += h
        cm[i2, i1] -= h
        fd_c[n] = (J_c(cp) - J_c(cm)) / (2 * h)
        print(f"dJ/dc cell {k}: {fd_c[n]:.6e} ({time.time() - t0:.0f} s)", flush=True)

    # f0 nodes: 8 seeded (shot, node) pairs inside the sources' support.
    # J is quadratic in f0 with the beam set fixed, so central differences
    # are exact up to rounding; only the perturbed shot's traces change.
    f0_nodes = []
    for s in r.choice(ns, 8):
        supp = np.flatnonzero(np.abs(W.f0[s]).ravel() > 1e-2 * np.abs(W.f0[s]).max())
        f0_nodes.append((int(s), int(r.choice(supp))))
    f0_nodes = np.array(f0_nodes, np.int64)
    fd_f0 = np.empty(len(f0_nodes))
    for n, (s, k) in enumerate(f0_nodes):
        h = 1e-4 * np.abs(W.f0[s]).max()
        mine = cand[(cand // (2 * p.nq1 * p.nq2 * p.np1 * p.np2)) == s] - s * 2 * p.nq1 * p.nq2 * p.np1 * p.np2
        vals = []
        for sg in (1.0, -1.0):
            f = W.f0[s:s + 1].copy()
            f.flat[k] += sg * h
            tr = oracle.trace_frozen(W.c, f, None, g, p, mine, rec, W.rec_every, nrec)
            vals.append(0.5 * float(((tr[0] - data[s]) ** 2).sum()))
        fd_f0[n] = (vals[0] - vals[1]) / (2 * h)
        print(f"dJ/df0 shot {s} node {k}: {fd_f0[n]:.6e} ({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(
        os.path.join(HERE, "adjoint256_fp64.npz"),
        nbeams=np.int64(b.n), offsets=b.offsets, ids=cand, data=data, traces=tr0, J=J0,
        cells=cells, fd_c=fd_c, f0_nodes=f0_nodes, fd_f0=fd_f0,
        seconds=np.float64(time.time() - t0))


if __name__ == "__main__":
    which = sys.argv[1:] or ["point512"]
    for w in which:
        globals()[w]()

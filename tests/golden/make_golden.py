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

Usage: python tests/golden/make_golden.py [point512] [wavepacket]
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


if __name__ == "__main__":
    which = sys.argv[1:] or ["point512"]
    for w in which:
        globals()[w]()

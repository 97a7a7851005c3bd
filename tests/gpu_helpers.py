"""Shared helpers of the GPU tests: run the HIP path through the C ABI and
compare its results with the oracle on the same seeded inputs."""
import math

import numpy as np

import fga_inputs as fi


def small_case(seed=21, nshots=1, with_f1=True):
    """Ragged heterogeneous case: 96 x 80 grid, partial output tiles, q- and
    p-meshes that do not divide the grid, both f0 and f1."""
    g = fi.Grid(96, 80, 0.0, 0.0, 1 / 64, 1 / 64)
    eps = 1 / 200
    c = fi.smooth_layered_velocity(g, seed=seed, smooth_cells=4.0)
    r = fi.rng(seed)
    f0 = np.empty((nshots,) + g.shape)
    f1 = np.empty((nshots,) + g.shape)
    for s in range(nshots):
        cen = (r.uniform(0.5, 1.0), r.uniform(0.4, 0.85))
        k = r.uniform(-1, 1, 2)
        f0[s] = fi.wavepacket_source(g, cen, 0.06, k, eps)
        f1[s] = 2.0 * fi.wavepacket_source(g, (cen[0] + 0.03, cen[1]), 0.05, (k[1], -k[0]), eps)
    p = fi.Params(eps, 3, 5, 5, 6, 17, 12, 16, 18, 0.2, 0.18, 1e-6, 1e-16, 1e-16, 1e-3, 50)
    return g, p, c, f0, (f1 if with_f1 else None)


def mixed_params(p):
    return p.replace(tau_fbi=1e-8, tau_win=1e-8)


def gpu_run(g, p, c, f0, f1, precision="fp64", capacity=None, nsteps=None, want_u=True):
    import torch
    import paper_1304_3542_amd as fga
    ns = f0.shape[0]
    ctx = fga.FGA(g, p, precision, max_shots=ns)
    ctx.set_velocity(torch.from_numpy(np.ascontiguousarray(c)).cuda())
    cand = 2 * p.nq1 * p.nq2 * p.np1 * p.np2 * ns
    beams = fga.Beams(capacity or cand, ns)
    f0t = torch.from_numpy(np.ascontiguousarray(f0)).cuda()
    f1t = None if f1 is None else torch.from_numpy(np.ascontiguousarray(f1)).cuda()
    ctx.decompose(f0t, f1t, beams)
    st, need = ctx.status()
    off = ctx.offsets(beams, ns)
    out = {"status": st, "needed": need, "offsets": off, "ctx": ctx, "beams": beams}
    nb = int(off[-1])
    out["id0"] = beams.id[:nb].cpu().numpy()
    out["f0"] = beams.f[:, :nb].cpu().numpy()
    steps = p.nsteps if nsteps is None else nsteps
    if steps > 0:
        ctx.propagate(beams, ns, steps)
    if want_u:
        out["u"] = ctx.reconstruct(beams, ns).cpu().numpy()
    out["fT"] = beams.f[:, :nb].cpu().numpy()
    out["status_end"] = ctx.status()
    return out


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def pairwise_state_err(gpu_state, or_state):
    """max |difference| over beams, per state component scaled by
    max(1, max |oracle value|) (every component is O(1) except S = 0)."""
    scale = np.maximum(np.abs(or_state).max(axis=0), 1.0)
    return float((np.abs(gpu_state - or_state) / scale).max())

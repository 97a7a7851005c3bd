"""Batched shots (uneven beam counts in one set of launches), HIP-graph
capture and replay, and the splat autotuner, through the C ABI."""
import os

import numpy as np
import pytest

import fga_inputs as fi
import oracle
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu


def shots_case(ns=6, seed=51):
    g = fi.Grid(128, 96, 0.0, 0.0, 1 / 64, 1 / 96)
    eps = 1 / 160
    c = fi.smooth_layered_velocity(g, seed=seed, smooth_cells=4.0)
    f0 = fi.surface_shots(g, ns, seed=seed, eps=eps, depth=0.2)
    p = fi.Params(eps, 2, 3, 9, 9, 14, 10, 20, 20, 0.16, 0.16, 1e-4, 1e-16, 1e-16, 1e-3, 40)
    return g, p, c, f0


def run(g, p, c, f0, precision="fp64", graph=False):
    import torch
    import paper_1304_3542_amd as fga
    ns = f0.shape[0]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = fga.FGA(g, p, precision, max_shots=ns)
        ctx.set_velocity(torch.from_numpy(c).cuda())
        beams = fga.Beams(2 * p.nq1 * p.nq2 * p.np1 * p.np2 * ns, ns)
        f0t = torch.from_numpy(np.ascontiguousarray(f0)).cuda()
        u = torch.empty((ns, g.n2, g.n1), dtype=torch.float64, device="cuda")
        ctx.decompose(f0t, None, beams)
        ctx.propagate(beams, ns, p.nsteps)
        ctx.reconstruct(beams, ns, u)
        stream.synchronize()
    return ctx, beams, f0t, u, stream


def test_batched_equals_per_shot():
    g, p, c, f0 = shots_case()
    ctx, beams, _, u, _ = run(g, p, c, f0)
    off = ctx.offsets(beams, f0.shape[0])
    counts = np.diff(off)
    assert counts.min() > 0 and counts.max() > 1.5 * counts.min()     # uneven
    ids = beams.id[: off[-1]].cpu().numpy()
    ub = u.cpu().numpy()
    for s in range(f0.shape[0]):
        ctx1, beams1, _, u1, _ = run(g, p, c, f0[s:s + 1])
        off1 = ctx1.offsets(beams1, 1)
        assert off1[-1] == counts[s]
        nqp = 2 * p.nq1 * p.nq2 * p.np1 * p.np2
        np.testing.assert_array_equal(beams1.id[: off1[-1]].cpu().numpy() + s * nqp,
                                      ids[off[s]:off[s + 1]])
        assert rel_l2(ub[s], u1.cpu().numpy()[0]) <= 1e-12


def test_batched_matches_oracle():
    g, p, c, f0 = shots_case(ns=3, seed=52)
    p = p.replace(nsteps=20)
    _, _, _, u, _ = run(g, p, c, f0)
    b = oracle.decompose(f0, None, c, g, p)
    oracle.propagate(b, c, g, p.dt, p.nsteps)
    for s in range(3):
        assert rel_l2(u.cpu().numpy()[s], oracle.reconstruct(b, g, p, shot=s)) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_is_bitwise_and_picks_up_inputs(precision):
    import torch
    g, p, c, f0 = shots_case(ns=4, seed=53)
    if precision == "mixed":
        p = p.replace(tau_fbi=1e-8, tau_win=1e-8)
    ctx, beams, f0t, u, stream = run(g, p, c, f0, precision)
    eager = u.clone()
    with torch.cuda.stream(stream):
        ctx.graph_capture(f0t, None, beams, p.nsteps, u)
        stream.synchronize()
        np.testing.assert_array_equal(u.cpu().numpy(), eager.cpu().numpy())
        for k in range(3):
            u.fill_(0.0)
            ctx.graph_launch()
            stream.synchronize()
            np.testing.assert_array_equal(u.cpu().numpy(), eager.cpu().numpy())
            # eager work on the same stream between replays
            ctx.reconstruct(beams, f0.shape[0])
            stream.synchronize()
        # inputs changed in place are picked up: doubling f0 doubles u exactly
        f0t.mul_(2.0)
        ctx.graph_launch()
        stream.synchronize()
    np.testing.assert_array_equal(u.cpu().numpy(), 2.0 * eager.cpu().numpy())
    assert ctx.status()[0] == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_choice_and_cache(precision, tmp_path):
    import torch
    g, p, c, f0 = shots_case(ns=3, seed=54)
    if precision == "mixed":
        p = p.replace(tau_fbi=1e-8, tau_win=1e-8)
    ctx, beams, _, u, stream = run(g, p, c, f0, precision)
    ref = u.clone()
    cache = str(tmp_path / "splat_tune.jsonl")
    with torch.cuda.stream(stream):
        v = ctx.autotune(beams, f0.shape[0], u, cache)
        stream.synchronize()
    allowed = {"mixed": {4, 8, 16, 32, 64, 128}, "fp64": {1, 2, 4, 8, 16}}[precision]
    assert v in allowed
    assert os.path.exists(cache) and '"splat_units_per_cu": %d' % v in open(cache).read()
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert rel_l2(u.cpu().numpy(), ref.cpu().numpy()) <= tol
    # a second context reads the cached choice
    ctx2, beams2, _, u2, stream2 = run(g, p, c, f0, precision)
    with torch.cuda.stream(stream2):
        assert ctx2.autotune(beams2, f0.shape[0], u2, cache) == v

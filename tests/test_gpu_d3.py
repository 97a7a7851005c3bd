"""The three-dimensional path (fga3_*, FP64) through the C ABI against the
three-dimensional oracle on the same seeded inputs: beam ids bit-exact,
coefficients, states after the RK4 and the field within 1e-10, on a ragged
case with f0 and f1 (q- and p-meshes that do not divide the grid, partial
16 x 32 x 32 tiles) and two shots, and on a grid three tiles deep in x3; the
full-size point3d workload against the oracle's propagation of sampled
beams."""
import numpy as np
import pytest

import fga_inputs as fi
import fga_inputs.d3 as i3
import oracle.d3 as o3
from gpu_helpers import pairwise_state_err, rel_l2

pytestmark = pytest.mark.gpu


def _case(seed=31, nshots=1):
    g = i3.Grid3(26, 22, 19, 0.0, 0.1, -0.05, 1 / 24, 1 / 22, 1 / 20)
    eps = 1 / 48
    c = i3.smooth_layered_velocity3(g, seed, 2.0)
    r = fi.rng(seed)
    f0 = np.stack([i3.wavepacket_source3(g, (r.uniform(0.4, 0.7), r.uniform(0.4, 0.7),
                                             r.uniform(0.3, 0.5)), 0.08,
                                         tuple(r.uniform(-1, 1, 3)), eps) for _ in range(nshots)])
    f1 = np.stack([0.5 * i3.gaussian_source3(g, (0.5, 0.55, 0.4), 0.1) for _ in range(nshots)])
    p = i3.Params3(eps, (2, 1, 3), (3, 4, 3), (8, 5, 5), (8, 6, 8), (0.3, 0.35, 0.28), 1e-5,
                   1e-16, 1e-16, 1e-3, 20)
    return g, p, c, f0, f1


def _gpu(g, p, c, f0, f1, capacity, nsteps):
    import torch
    import paper_1304_3542_amd as fga
    ns = f0.shape[0]
    ctx = fga.FGA3(g, p, max_shots=ns)
    ctx.set_velocity(torch.from_numpy(np.ascontiguousarray(c)).cuda())
    beams = fga.Beams3(capacity, ns)
    ctx.decompose(torch.from_numpy(np.ascontiguousarray(f0)).cuda(),
                  None if f1 is None else torch.from_numpy(np.ascontiguousarray(f1)).cuda(), beams)
    st0 = ctx.status()
    nb = int(beams.offsets[ns].item())
    out = {"status0": st0, "nb": nb, "offsets": beams.offsets.cpu().numpy(),
           "id": beams.id[:nb].cpu().numpy(), "f0": beams.f[:, :nb].cpu().numpy()}
    ctx.propagate(beams, ns, nsteps)
    out["fT"] = beams.f[:, :nb].cpu().numpy()
    out["u"] = ctx.reconstruct(beams, ns).cpu().numpy()
    out["status"] = ctx.status()
    return out


@pytest.mark.parametrize("nshots", [1, 2])
def test_d3_fp64_matches_oracle(nshots):
    g, p, c, f0, f1 = _case(nshots=nshots)
    b, us = o3.forward(f0, f1, c, g, p)
    assert 100 < b.n
    r = _gpu(g, p, c, f0, f1, b.n + 100, p.nsteps)
    assert r["status0"][0] == 0 and r["status"][0] == 0
    np.testing.assert_array_equal(r["offsets"], b.offsets)
    np.testing.assert_array_equal(r["id"], b.cand)
    coef = r["f0"][6:8].T
    assert np.abs(coef - b.coef).max() <= 1e-10 * np.abs(b.coef).max()
    assert pairwise_state_err(r["fT"][8:].T, b.state) <= 1e-10
    for s in range(nshots):
        assert rel_l2(r["u"][s], us[s]) <= 1e-10


def test_d3_field_over_three_x3_tiles():
    """n3 = 70: the reconstruction's tiles (32 deep) split x3 twice, the
    last one ragged, with packets on both sides of the splits and truncation
    boxes that straddle them."""
    g = i3.Grid3(12, 10, 70, 0.0, 0.1, -0.05, 1 / 24, 1 / 24, 1 / 24)
    eps = 1 / 48
    c = i3.smooth_layered_velocity3(g, 41, 2.0)
    f0 = (i3.wavepacket_source3(g, (0.22, 0.3, 0.8), 0.08, (0.6, -0.3, 0.7), eps) +
          i3.wavepacket_source3(g, (0.25, 0.28, 2.55), 0.08, (-0.4, 0.5, -0.6), eps))[None]
    p = i3.Params3(eps, (1, 1, 2), (3, 3, 7), (4, 3, 10), (6, 6, 6), (0.3, 0.3, 0.3), 1e-5,
                   1e-16, 1e-16, 1e-3, 5)
    b, us = o3.forward(f0, None, c, g, p)
    assert 50 < b.n
    r = _gpu(g, p, c, f0, None, b.n + 10, p.nsteps)
    assert r["status0"][0] == 0 and r["status"][0] == 0
    np.testing.assert_array_equal(r["id"], b.cand)
    assert rel_l2(r["u"][0], us[0]) <= 1e-10
    lo, hi = np.abs(us[0][:64]).max(), np.abs(us[0][64:]).max()
    assert lo > 0 and hi > 0


def test_d3_capacity_overflow_reports_count():
    import paper_1304_3542_amd as fga
    g, p, c, f0, f1 = _case(seed=32)
    b = o3.decompose(f0, f1, c, g, p)
    r = _gpu(g, p, c, f0, f1, b.n - 7, 3)
    assert r["status0"][0] == fga.FGA_ECAPACITY and r["status0"][1] == b.n
    assert r["offsets"].max() <= b.n - 7 and r["status"][0] == 0   # later steps stay in bounds


def test_d3_point3d_sampled_beams_match_oracle():
    """point3d (96 x 96 x 64, every kept beam, 100 steps): 32 seeded beams of
    the GPU run against the oracle's propagation of the same initial states,
    and a finite field."""
    import torch
    import paper_1304_3542_amd as fga
    W = i3.workload3("point3d")
    g, p = W.grid, W.params
    ctx = fga.FGA3(g, p)
    ctx.set_velocity(torch.from_numpy(W.c).cuda())
    beams = fga.Beams3(3_000_000, 1)
    ctx.decompose(torch.from_numpy(np.ascontiguousarray(W.f0)).cuda(), None, beams)
    st = ctx.status()
    nb = int(beams.offsets[1].item())
    assert st[0] == 0 and nb > 10000, (st, nb)
    idx = np.sort(fi.rng(93).choice(nb, 32, replace=False))
    f_init = beams.f[:, idx].cpu().numpy()
    ids = beams.id[idx].cpu().numpy()
    ctx.propagate(beams, 1, p.nsteps)
    u = ctx.reconstruct(beams, 1)
    assert ctx.status()[0] == 0
    assert bool(torch.isfinite(u).all()) and float(u.abs().max()) > 0
    got = beams.f[8:, idx].cpu().numpy().T
    NQNP = int(np.prod(p.nq)) * int(np.prod(p.np))
    sig = np.where((ids // NQNP) % 2 == 0, 1, -1).astype(np.int8)
    b = o3.Beams3(np.zeros(32, np.int32), sig, ids, np.ones(32, complex), np.zeros((32, 2)),
                  np.ascontiguousarray(f_init[8:].T), np.array([0, 32], np.int64))
    o3.propagate(b, W.c, g, p.dt, p.nsteps)
    err = pairwise_state_err(got, b.state)
    print(f"point3d sampled beams vs oracle: {err:.2e}", flush=True)
    assert err <= 1e-10

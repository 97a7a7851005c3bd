"""The splats at the binning's limits.  17 shots on a 2048 x 1024 grid
(512 tiles of 64 x 64 each, 8704 (shot, tile) pairs, past the 8192 the
binning handles) go through the unbinned MFMA splat and its ordered
reduction; 15 shots (7680 pairs) stay binned, but their difference-array
counters (15 x 33 x 17) do not fit, so the tile hits are counted one by one.
The FP64 splat bins 128 x 128 tiles (128 per shot): binned at 15 and 17
shots, unbinned at 65 (8320 pairs).  Hand-built beams (random centres,
momenta, phases, amplitudes and coefficients, a few per shot, some with
boxes clipped by the grid edge) against the oracle's windowed sum and
against the FP64 path on the same beams, with FP32 and with split FP16
products."""
import numpy as np
import pytest

import fga_inputs as fi
import oracle
from gpu_helpers import rel_l2

pytestmark = pytest.mark.gpu


def _beams(g, ns, per_shot, seed):
    r = fi.rng(seed)
    nb = ns * per_shot
    st = np.zeros((nb, oracle.NSTATE))
    st[:, 0] = r.uniform(-0.05, 2.05, nb)              # some centres past the edge
    st[:, 1] = r.uniform(-0.05, 1.05, nb)
    ang = r.uniform(0, 2 * np.pi, nb)
    mag = r.uniform(0.3, 2.8, nb)
    st[:, 2] = mag * np.cos(ang)
    st[:, 3] = mag * np.sin(ang)
    st[:, 4] = r.uniform(-1e-13, 1e-13, nb)
    st[:, 21:23] = r.standard_normal((nb, 2))
    coef = r.standard_normal((nb, 2))
    shot = np.repeat(np.arange(ns, dtype=np.int32), per_shot)
    offsets = np.arange(0, nb + 1, per_shot, dtype=np.int64)
    return oracle.Beams(shot, np.ones(nb, np.int8), np.arange(nb, dtype=np.int64),
                        np.ones(nb, complex), coef, st, offsets)


@pytest.mark.parametrize("ns", [17, 15])
def test_mixed_splat_at_the_binning_limits(ns):
    import torch
    import paper_1304_3542_amd as fga
    g = fi.Grid(2048, 1024, 0.0, 0.0, 1 / 1024, 1 / 1024)
    per_shot = 24
    tiles = ns * (2048 // 64) * (1024 // 64)
    assert (tiles > 8192) == (ns == 17) and ns * 33 * 17 > 8192
    b = _beams(g, ns, per_shot, seed=17)
    nb = b.n
    fields = np.zeros((fga.FGA_NFIELD, nb))
    fields[4:6] = b.coef.T
    fields[fga.FGA_F_STATE:] = b.state.T
    # candidate ids carry the shot: 2 x 1 q node x 4 x 4 p nodes = 32 per shot
    ids = np.concatenate([s * 32 + np.arange(per_shot) for s in range(ns)]).astype(np.int64)
    out = {}
    for prec, tw in (("mixed", 1e-8), ("mixed_split", 1e-8), ("fp64", 1e-16)):
        p = fi.Params(1 / 1024, 0, 0, 1, 1, 1, 1, 4, 4, 0.1, 0.1, 1e-6, tw, tw, 1e-3, 0)
        ctx = fga.FGA(g, p, prec, max_shots=ns)
        beams = fga.Beams(nb, ns)
        beams.f.copy_(torch.from_numpy(fields))
        beams.id.copy_(torch.from_numpy(ids))
        beams.offsets.copy_(torch.from_numpy(b.offsets))
        out[prec] = ctx.reconstruct(beams, ns).cpu().numpy()
        assert ctx.status()[0] == 0
        ctx.close()
        out[prec + "_p"] = p
    # oracle at nodes near every beam's centre and at seeded nodes
    r = fi.rng(18)
    for s in range(ns):
        sl = slice(s * per_shot, (s + 1) * per_shot)
        i1 = np.clip(np.floor(b.state[sl, 0] * 1024 + 0.5).astype(np.int64)
                     + r.integers(-40, 41, per_shot), 0, g.n1 - 1)
        i2 = np.clip(np.floor(b.state[sl, 1] * 1024 + 0.5).astype(np.int64)
                     + r.integers(-40, 41, per_shot), 0, g.n2 - 1)
        nodes = np.unique(np.concatenate([i2 * g.n1 + i1, r.choice(g.n1 * g.n2, 64)]))
        ref = oracle.reconstruct_points(b, g, out["fp64_p"], nodes, shot=s)
        assert np.abs(ref).max() > 0
        got64 = out["fp64"][s].ravel()[nodes]
        assert np.abs(got64 - ref).max() <= 1e-10 * np.abs(ref).max(), s
        for prec in ("mixed", "mixed_split"):
            gotm = out[prec][s].ravel()[nodes]
            assert rel_l2(gotm, ref) <= 1e-5, (prec, s, rel_l2(gotm, ref))
    for prec in ("mixed", "mixed_split"):
        rel = rel_l2(out[prec], out["fp64"])
        print(f"{prec} splat, {ns} shots: rel-L2 vs FP64 {rel:.3e}", flush=True)
        assert rel <= 1e-5


def test_fp64_splat_past_the_binning_limit():
    import torch
    import paper_1304_3542_amd as fga
    g = fi.Grid(2048, 1024, 0.0, 0.0, 1 / 1024, 1 / 1024)
    ns, per_shot = 65, 6
    assert ns * (2048 // 128) * (1024 // 128) > 8192
    b = _beams(g, ns, per_shot, seed=19)
    nb = b.n
    fields = np.zeros((fga.FGA_NFIELD, nb))
    fields[4:6] = b.coef.T
    fields[fga.FGA_F_STATE:] = b.state.T
    ids = np.concatenate([s * 32 + np.arange(per_shot) for s in range(ns)]).astype(np.int64)
    p = fi.Params(1 / 1024, 0, 0, 1, 1, 1, 1, 4, 4, 0.1, 0.1, 1e-6, 1e-16, 1e-16, 1e-3, 0)
    ctx = fga.FGA(g, p, "fp64", max_shots=ns)
    beams = fga.Beams(nb, ns)
    beams.f.copy_(torch.from_numpy(fields))
    beams.id.copy_(torch.from_numpy(ids))
    beams.offsets.copy_(torch.from_numpy(b.offsets))
    u = ctx.reconstruct(beams, ns).cpu().numpy()
    assert ctx.status()[0] == 0
    ctx.close()
    r = fi.rng(20)
    for s in r.choice(ns, 8, replace=False):
        sl = slice(s * per_shot, (s + 1) * per_shot)
        i1 = np.clip(np.floor(b.state[sl, 0] * 1024 + 0.5).astype(np.int64)
                     + r.integers(-40, 41, per_shot), 0, g.n1 - 1)
        i2 = np.clip(np.floor(b.state[sl, 1] * 1024 + 0.5).astype(np.int64)
                     + r.integers(-40, 41, per_shot), 0, g.n2 - 1)
        nodes = np.unique(np.concatenate([i2 * g.n1 + i1, r.choice(g.n1 * g.n2, 32)]))
        ref = oracle.reconstruct_points(b, g, p, nodes, shot=int(s))
        assert np.abs(ref).max() > 0
        got = u[s].ravel()[nodes]
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max(), s

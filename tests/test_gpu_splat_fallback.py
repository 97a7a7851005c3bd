"""The mixed splat beyond the binning's limit of 8192 (shot, tile) pairs:
17 shots on a 2048 x 1024 grid (512 tiles of 64 x 64 each, 8704 pairs) go
through the unbinned MFMA splat and its ordered reduction.  Hand-built beams
(random centres, momenta, phases, amplitudes and coefficients, a few per
shot, some with boxes clipped by the grid edge) against the oracle's
windowed sum and against the FP64 path on the same beams."""
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


def test_unbinned_mixed_splat_past_8192_shot_tiles():
    import torch
    import paper_1304_3542_amd as fga
    g = fi.Grid(2048, 1024, 0.0, 0.0, 1 / 1024, 1 / 1024)
    ns, per_shot = 17, 24
    assert ns * (2048 // 64) * (1024 // 64) > 8192
    b = _beams(g, ns, per_shot, seed=17)
    nb = b.n
    fields = np.zeros((fga.FGA_NFIELD, nb))
    fields[4:6] = b.coef.T
    fields[fga.FGA_F_STATE:] = b.state.T
    out = {}
    for prec, tw in (("mixed", 1e-8), ("fp64", 1e-16)):
        p = fi.Params(1 / 1024, 0, 0, 1, 1, 1, 1, 2, 2, 0.1, 0.1, 1e-6, tw, tw, 1e-3, 0)
        ctx = fga.FGA(g, p, prec, max_shots=ns)
        beams = fga.Beams(nb, ns)
        beams.f.copy_(torch.from_numpy(fields))
        beams.id.copy_(torch.arange(nb, dtype=torch.int64))
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
        gotm = out["mixed"][s].ravel()[nodes]
        assert np.abs(got64 - ref).max() <= 1e-10 * np.abs(ref).max(), s
        assert rel_l2(gotm, ref) <= 1e-5, (s, rel_l2(gotm, ref))
    rel = rel_l2(out["mixed"], out["fp64"])
    print(f"unbinned mixed splat, {ns} shots: rel-L2 vs FP64 {rel:.3e}", flush=True)
    assert rel <= 1e-5

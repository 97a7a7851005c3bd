"""The closed-form amplitude mode (amp_closed = 1: a = c(Q)/c(q) (det Z)^{1/2}
with the root followed step by step) through the C ABI against the oracle's
closed form: fields, states, traces over several segments, hand-built rays
whose det Z winds past 2 pi, and the refusal of the gradient."""
import numpy as np
import pytest

import fga_inputs as fi
import oracle
from gpu_helpers import gpu_run, mixed_params, rel_l2, small_case

pytestmark = pytest.mark.gpu


def test_closed_fp64_matches_oracle():
    g, p, c, f0, f1 = small_case(seed=71)
    p = p.replace(amp_closed=1, nsteps=40)
    r = gpu_run(g, p, c, f0, f1, "fp64")
    assert r["status"] == 0 and r["status_end"][0] == 0
    b = oracle.decompose(f0, f1, c, g, p)
    np.testing.assert_array_equal(r["id0"], b.cand)
    oracle.propagate(b, c, g, p.dt, p.nsteps, q=oracle.beam_nodes(b, g, p))
    a_gpu = r["fT"][27] + 1j * r["fT"][28]
    a_or = b.state[:, 21] + 1j * b.state[:, 22]
    assert np.abs(a_gpu - a_or).max() <= 1e-10 * np.abs(a_or).max()
    assert rel_l2(r["u"][0], oracle.reconstruct(b, g, p)) <= 1e-10
    # and it differs from the integrated amplitude only at the RK4 level
    ri = gpu_run(g, p.replace(amp_closed=0), c, f0, f1, "fp64")
    a_int = ri["fT"][27] + 1j * ri["fT"][28]
    assert 0 < np.abs(a_gpu - a_int).max() <= 1e-6 * np.abs(a_int).max()


def test_closed_mixed_within_1e5():
    g, p, c, f0, f1 = small_case(seed=72)
    p = mixed_params(p.replace(amp_closed=1, nsteps=40))
    rm = gpu_run(g, p, c, f0, f1, "mixed")
    rd = gpu_run(g, p, c, f0, f1, "fp64")
    assert rm["status"] == 0 and rd["status"] == 0
    assert rel_l2(rm["u"], rd["u"]) <= 1e-5


def test_closed_trace_segments_match_oracle():
    import torch
    import paper_1304_3542_amd as fga
    g, p, c, f0, _ = small_case(seed=73, nshots=2, with_f1=False)
    p = p.replace(amp_closed=1)
    rec = np.arange(0, g.n1 * 3, 2, dtype=np.int32)
    b = oracle.decompose(f0, None, c, g, p)
    tr_or = oracle.trace(b, c, g, p, rec, rec_every=5, nrec=4)
    ctx = fga.FGA(g, p, "fp64", max_shots=2)
    ctx.set_velocity(torch.from_numpy(c).cuda())
    beams = fga.Beams(int(b.offsets[-1]) + 10, 2)
    ctx.decompose(torch.from_numpy(f0).cuda(), None, beams)
    ckpt = torch.empty((4, fga.FGA_NSTATE, beams.capacity), dtype=torch.float64, device="cuda")
    rec_t = torch.from_numpy(rec).cuda()
    tr = ctx.trace(beams, 2, rec_t, 5, 4, ckpt)
    assert ctx.status()[0] == 0
    assert rel_l2(tr.cpu().numpy(), tr_or) <= 1e-10
    # the gradient needs the integrated amplitude
    dc = torch.zeros((g.n2, g.n1), dtype=torch.float64, device="cuda")
    with pytest.raises(fga.FGAError):
        ctx.trace_adjoint(beams, 2, rec_t, 5, 4, ckpt, tr.contiguous(), dc)


def test_closed_root_tracking_through_caustics():
    """Rays in a parabolic low-velocity channel (det Z winds by ~2.4 pi):
    beams written directly into the caller's buffer, propagated with the
    closed form on the GPU, agree with the oracle's closed form, and their
    amplitude is the negative of the principal-root formula."""
    import torch
    import paper_1304_3542_amd as fga
    g = fi.Grid(96, 96, 0.0, 0.0, 1 / 96, 1 / 96)
    x2 = g.coords()[1]
    c = np.ascontiguousarray(np.repeat((1.0 + 40.0 * (x2 - 0.5) ** 2)[:, None], g.n1, 1))
    r = fi.rng(12)
    nb = 32
    q = np.stack([np.full(nb, 0.08), r.uniform(0.45, 0.55, nb)], 1)
    ang = r.uniform(-0.25, 0.25, nb)
    pv = np.stack([np.cos(ang), np.sin(ang)], 1) * r.uniform(0.7, 1.5, nb)[:, None]
    st = np.zeros((nb, oracle.NSTATE))
    st[:, 0:2] = q
    st[:, 2:4] = pv
    st[:, 5] = st[:, 11] = 1.0
    st[:, 14] = st[:, 20] = -1.0
    st[:, 21] = 2.0
    b = oracle.Beams(np.zeros(nb, np.int32), np.ones(nb, np.int8), np.arange(nb, dtype=np.int64),
                     np.ones(nb, complex), np.zeros((nb, 2)), st.copy(),
                     np.array([0, nb], np.int64))
    nst, dt = 800, 1e-3
    oracle.propagate(b, c, g, dt, nst, q=q)
    p = fi.Params(1 / 96, 0, 0, 1, 1, 8, 8, 4, 4, 0.5, 0.5, 1e-6, 1e-16, 1e-16, dt, nst,
                  amp_closed=1)
    ctx = fga.FGA(g, p, "fp64")
    ctx.set_velocity(torch.from_numpy(c).cuda())
    beams = fga.Beams(nb, 1)
    fh = np.zeros((fga.FGA_NFIELD, nb))
    fh[0:2] = q.T
    fh[2:4] = pv.T
    fh[fga.FGA_F_STATE:] = st.T
    beams.f.copy_(torch.from_numpy(fh))
    beams.id.copy_(torch.arange(nb, dtype=torch.int64))   # branch +: id < Nq Np
    beams.offsets.copy_(torch.tensor([0, nb], dtype=torch.int64))
    ctx.propagate(beams, 1, nst)
    assert ctx.status()[0] == 0
    out = beams.f.cpu().numpy()[fga.FGA_F_STATE:].T
    np.testing.assert_allclose(out[:, :21], b.state[:, :21], rtol=0, atol=1e-10)
    a_gpu = out[:, 21] + 1j * out[:, 22]
    a_or = b.state[:, 21] + 1j * b.state[:, 22]
    assert np.abs(a_gpu - a_or).max() <= 1e-10 * np.abs(a_or).max()
    Z = (out[:, 5:13:2] + 1j * out[:, 6:13:2]) + 1j * (out[:, 13:21:2] + 1j * out[:, 14:21:2])
    cq = oracle.velocity(c, g, q[:, 0], q[:, 1])[:, 0]
    cQ = oracle.velocity(c, g, out[:, 0], out[:, 1])[:, 0]
    principal = cQ / cq * np.sqrt(Z[:, 0] * Z[:, 3] - Z[:, 1] * Z[:, 2])
    assert np.all(np.abs(principal + a_gpu) < 1e-6 * np.abs(a_gpu))


def test_closed_point512_sampled_beams_match_oracle():
    """point512 in FP64 at full size (250 steps, every kept beam, the launch
    the bench times) with the closed-form amplitude: 96 seeded beams against
    the oracle's closed-form propagation of the same initial states."""
    import torch
    import paper_1304_3542_amd as fga
    W = fi.workload("point512", "fp64")
    g, p = W.grid, W.params.replace(amp_closed=1)
    ctx = fga.FGA(g, p, "fp64")
    ctx.set_velocity(torch.from_numpy(W.c).cuda())
    beams = fga.Beams(1_500_000, 1)
    ctx.decompose(torch.from_numpy(np.ascontiguousarray(W.f0)).cuda(), None, beams)
    nb = int(ctx.offsets(beams, 1)[-1])
    assert ctx.status()[0] == 0 and nb > 1_000_000
    idx = np.sort(fi.rng(91).choice(nb, 96, replace=False))
    f_init = beams.f[:, idx].cpu().numpy()
    ids = beams.id[idx].cpu().numpy()
    ctx.propagate(beams, 1, p.nsteps)
    assert ctx.status()[0] == 0
    got = beams.f[fga.FGA_F_STATE:, idx].cpu().numpy().T
    NqNp = p.nq1 * p.nq2 * p.np1 * p.np2
    sig = np.where((ids // NqNp) % 2 == 0, 1, -1).astype(np.int8)
    b = oracle.Beams(np.zeros(96, np.int32), sig, ids, np.ones(96, complex), np.zeros((96, 2)),
                     np.ascontiguousarray(f_init[fga.FGA_F_STATE:].T),
                     np.array([0, 96], np.int64))
    oracle.propagate(b, W.c, g, p.dt, p.nsteps, q=np.ascontiguousarray(f_init[0:2].T))
    from gpu_helpers import pairwise_state_err
    err = pairwise_state_err(got, b.state)
    print(f"closed-form sampled beams vs oracle: {err:.2e}", flush=True)
    assert err <= 1e-10

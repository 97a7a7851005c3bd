"""The divided-difference mode (dz_divided = 1: dzQ, dzP from central
differences of the rays of the neighbouring mesh nodes, amplitude from the
closed form) through the C ABI against the oracle's divided-difference mode:
states and fields, traces over several segments, hand-built beam counts that
leave partial wavefronts, rays through caustics, and a sample of the full
point source at its real size."""
import numpy as np
import pytest

import fga_inputs as fi
import oracle
from gpu_helpers import gpu_run, mixed_params, pairwise_state_err, rel_l2, small_case

pytestmark = pytest.mark.gpu

DD = dict(amp_closed=1, dz_divided=1)


def test_dd_fp64_matches_oracle():
    g, p, c, f0, f1 = small_case(seed=81)
    p = p.replace(nsteps=40, **DD)
    r = gpu_run(g, p, c, f0, f1, "fp64")
    assert r["status"] == 0 and r["status_end"][0] == 0
    b, us = oracle.forward(f0, f1, c, g, p)
    np.testing.assert_array_equal(r["id0"], b.cand)
    assert pairwise_state_err(r["fT"][6:].T, b.state) <= 1e-10
    assert rel_l2(r["u"][0], us[0]) <= 1e-10
    # the rays are those of the dynamic ray tracing run; A, B and a are not
    # (here the q-mesh step is longer than the scale on which c varies, so
    # the differences over it are far from the derivatives)
    rc = gpu_run(g, p.replace(dz_divided=0), c, f0, f1, "fp64")
    np.testing.assert_allclose(r["fT"][6:11], rc["fT"][6:11], rtol=0, atol=1e-12)
    assert np.abs(r["fT"][11:27] - rc["fT"][11:27]).max() > 1e-3


def test_dd_fine_spacing_matches_oracle_and_dynamic_ray_tracing():
    """dz_scale = 1e-3 (rays 1e-3 mesh steps apart): the GPU equals the
    oracle (differences of rays 8e-5 apart magnify rounding by ~1e4, hence
    1e-9 on the state), and the field is within 1e-6 of the dynamic ray
    tracing run (the oracle gives 2.4e-7 for this case)."""
    g, p, c, f0, f1 = small_case(seed=84)
    p = p.replace(nsteps=40, dz_scale=1e-3, **DD)
    r = gpu_run(g, p, c, f0, f1, "fp64")
    assert r["status"] == 0 and r["status_end"][0] == 0
    b, us = oracle.forward(f0, f1, c, g, p)
    assert pairwise_state_err(r["fT"][6:].T, b.state) <= 1e-9
    assert rel_l2(r["u"][0], us[0]) <= 1e-10
    rc = gpu_run(g, p.replace(dz_divided=0), c, f0, f1, "fp64")
    assert rel_l2(r["u"][0], rc["u"][0]) <= 1e-6


def test_dd_mixed_within_1e5():
    g, p, c, f0, f1 = small_case(seed=82)
    p = mixed_params(p.replace(nsteps=40, **DD))
    rm = gpu_run(g, p, c, f0, f1, "mixed")
    rd = gpu_run(g, p, c, f0, f1, "fp64")
    assert rm["status"] == 0 and rd["status"] == 0
    assert rel_l2(rm["u"], rd["u"]) <= 1e-5


def test_dd_trace_segments_match_oracle():
    """Four segments of five steps: every segment restarts the neighbouring
    rays from the stored A, B, on both sides alike."""
    import torch
    import paper_1304_3542_amd as fga
    g, p, c, f0, _ = small_case(seed=83, nshots=2, with_f1=False)
    p = p.replace(**DD)
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
    nb = int(b.offsets[-1])
    np.testing.assert_allclose(beams.f[6:, :nb].cpu().numpy().T, b.state, rtol=0, atol=1e-10)
    dc = torch.zeros((g.n2, g.n1), dtype=torch.float64, device="cuda")
    with pytest.raises(fga.FGAError):
        ctx.trace_adjoint(beams, 2, rec_t, 5, 4, ckpt, tr.contiguous(), dc)


def _channel_beams(nb, seed):
    g = fi.Grid(96, 96, 0.0, 0.0, 1 / 96, 1 / 96)
    x2 = g.coords()[1]
    c = np.ascontiguousarray(np.repeat((1.0 + 40.0 * (x2 - 0.5) ** 2)[:, None], g.n1, 1))
    r = fi.rng(seed)
    q = np.stack([np.full(nb, 0.08), r.uniform(0.45, 0.55, nb)], 1)
    ang = r.uniform(-0.25, 0.25, nb)
    pv = np.stack([np.cos(ang), np.sin(ang)], 1) * r.uniform(0.7, 1.5, nb)[:, None]
    st = np.zeros((nb, oracle.NSTATE))
    st[:, 0:2] = q
    st[:, 2:4] = pv
    st[:, 5] = st[:, 11] = 1.0
    st[:, 14] = st[:, 20] = -1.0
    st[:, 21] = 2.0
    return g, c, q, pv, st


@pytest.mark.parametrize("nb", [1, 7, 8, 29, 250])
def test_dd_partial_wavefronts_and_caustics(nb):
    """Beams written into the caller's buffer (counts that fill 1, 7 and 8
    lanes-groups of a wavefront, and several wavefronts with a ragged last
    one) in a parabolic channel where det Z winds past 2 pi: the GPU's
    divided-difference run equals the oracle's, root tracking included."""
    import torch
    import paper_1304_3542_amd as fga
    g, c, q, pv, st = _channel_beams(nb, seed=40 + nb)
    nst, dt = 800, 1e-3
    p = fi.Params(1 / 96, 0, 0, 1, 1, 8, 8, 4, 4, 0.05, 0.04, 1e-6, 1e-16, 1e-16, dt, nst, **DD)
    b = oracle.Beams(np.zeros(nb, np.int32), np.ones(nb, np.int8), np.arange(nb, dtype=np.int64),
                     np.ones(nb, complex), np.zeros((nb, 2)), st.copy(),
                     np.array([0, nb], np.int64))
    oracle.propagate(b, c, g, dt, nst, q=q, dd=oracle.dd_spacings(g, p))
    ctx = fga.FGA(g, p, "fp64")
    ctx.set_velocity(torch.from_numpy(c).cuda())
    beams = fga.Beams(nb + 5, 1)
    fh = np.zeros((fga.FGA_NFIELD, nb + 5))
    fh[0:2, :nb] = q.T
    fh[2:4, :nb] = pv.T
    fh[fga.FGA_F_STATE:, :nb] = st.T
    fh[fga.FGA_F_STATE:, nb:] = 7.0                       # beyond the count: left alone
    beams.f.copy_(torch.from_numpy(fh))
    beams.id.copy_(torch.arange(nb + 5, dtype=torch.int64))
    beams.offsets.copy_(torch.tensor([0, nb], dtype=torch.int64))
    ctx.propagate(beams, 1, nst)
    assert ctx.status()[0] == 0
    out = beams.f.cpu().numpy()
    assert np.all(out[fga.FGA_F_STATE:, nb:] == 7.0)
    assert pairwise_state_err(out[fga.FGA_F_STATE:, :nb].T, b.state) <= 1e-10
    a = b.state[:, 21] + 1j * b.state[:, 22]
    Z = (b.state[:, 5:13:2] + 1j * b.state[:, 6:13:2]) + 1j * (b.state[:, 13:21:2] + 1j * b.state[:, 14:21:2])
    det = Z[:, 0] * Z[:, 3] - Z[:, 1] * Z[:, 2]
    cq = oracle.velocity(c, g, q[:, 0], q[:, 1])[:, 0]
    cQ = oracle.velocity(c, g, b.state[:, 0], b.state[:, 1])[:, 0]
    principal = cQ / cq * np.sqrt(det)
    assert np.any(np.abs(principal + a) < 1e-9 * np.abs(a))   # some roots wound past the cut


def test_dd_point512_sampled_beams_match_oracle():
    """point512 in FP64 at full size (250 steps, every kept beam, the
    launch the bench times): 96 seeded beams against the oracle's
    divided-difference propagation of the same initial states."""
    import torch
    import paper_1304_3542_amd as fga
    W = fi.workload("point512", "fp64")
    g, p = W.grid, W.params.replace(**DD)
    ctx = fga.FGA(g, p, "fp64")
    ctx.set_velocity(torch.from_numpy(W.c).cuda())
    beams = fga.Beams(1_500_000, 1)
    ctx.decompose(torch.from_numpy(np.ascontiguousarray(W.f0)).cuda(), None, beams)
    nb = int(ctx.offsets(beams, 1)[-1])
    assert ctx.status()[0] == 0 and nb > 1_000_000
    idx = np.sort(fi.rng(90).choice(nb, 96, replace=False))
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
    oracle.propagate(b, W.c, g, p.dt, p.nsteps, q=np.ascontiguousarray(f_init[0:2].T),
                     dd=oracle.dd_spacings(g, p))
    err = pairwise_state_err(got, b.state)
    print(f"dd point512 sampled beams vs oracle: {err:.2e}", flush=True)
    assert err <= 1e-10

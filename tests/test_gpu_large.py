"""The large configuration at full size: 2048 x 1024 smooth layered model,
eps = 1/1024, point source, q-mesh 147 x 74, p-mesh 400 x 400, tau = 1e-6
(~5e7 beams from ~3.5e9 candidates).  The oracle cannot run at this size;
the mixed path is compared with the FP64 GPU path (itself parity-checked
against the oracle at smaller sizes and at sampled nodes of point512)."""
import numpy as np
import pytest

import fga_inputs as fi

pytestmark = pytest.mark.gpu


def run(W, precision):
    import torch
    import paper_1304_3542_amd as fga
    ctx = fga.FGA(W.grid, W.params, precision)
    ctx.set_velocity(torch.from_numpy(W.c).cuda())
    f0 = torch.from_numpy(np.ascontiguousarray(W.f0)).cuda()
    beams = fga.Beams(8_000_000, 1)
    ctx.decompose(f0, None, beams)
    st, need = ctx.status()
    if st == fga.FGA_ECAPACITY:
        del beams
        torch.cuda.empty_cache()
        beams = fga.Beams(need + 1024, 1)
        ctx.decompose(f0, None, beams)
        st, need = ctx.status()
    assert st == fga.FGA_OK
    nb = int(ctx.offsets(beams, 1)[-1])
    ctx.propagate(beams, 1, W.params.nsteps)
    u = ctx.reconstruct(beams, 1)[0].cpu().numpy()
    assert ctx.status()[0] == fga.FGA_OK
    ids = beams.id[:nb].cpu().numpy()
    ctx.close()
    del beams
    torch.cuda.empty_cache()
    return nb, ids, u


def test_large_mixed_matches_fp64():
    Wd = fi.workload("large2048", "fp64")
    Wm = fi.workload("large2048", "mixed")
    nb64, ids64, u64 = run(Wd, "fp64")
    print(f"large2048: FP64 beams {nb64}", flush=True)
    assert 1e7 < nb64 < 2e8
    for prec in ("mixed", "mixed_split"):
        nbm, idsm, um = run(Wm, prec)
        # beams whose |psi| sits within rounding of the threshold may differ
        flips = len(np.setxor1d(ids64, idsm))
        assert flips <= 1e-3 * nb64, flips
        rel = np.linalg.norm(um - u64) / np.linalg.norm(u64)
        print(f"large2048: {prec} beams {nbm}, vs FP64 rel-L2 {rel:.3e}, threshold flips "
              f"{flips}", flush=True)
        assert rel <= 1e-5


def test_large_fp64_sampled_against_oracle():
    """large2048 in FP64 at full size (the launches the bench times): the
    coefficients of every kept beam at two seeded q nodes against the
    oracle's windowed DFT at those nodes, and 32 seeded beams after the 250
    RK4 steps against the oracle's propagation of the initial states it forms
    from the beams' (q, p) mesh nodes."""
    import torch
    import oracle
    import paper_1304_3542_amd as fga
    from gpu_helpers import pairwise_state_err
    W = fi.workload("large2048", "fp64")
    g, p = W.grid, W.params
    ctx = fga.FGA(g, p, "fp64")
    ctx.set_velocity(torch.from_numpy(W.c).cuda())
    f0 = torch.from_numpy(np.ascontiguousarray(W.f0)).cuda()
    beams = fga.Beams(8_000_000, 1)
    ctx.decompose(f0, None, beams)
    st, need = ctx.status()
    if st == fga.FGA_ECAPACITY:
        del beams
        torch.cuda.empty_cache()
        beams = fga.Beams(need + 1024, 1)
        ctx.decompose(f0, None, beams)
        st, need = ctx.status()
    assert st == fga.FGA_OK
    nb = int(ctx.offsets(beams, 1)[-1])
    print(f"large2048 FP64: {nb} beams", flush=True)
    ids = beams.id[:nb].cpu().numpy()
    coef = beams.f[4:6, :nb].cpu().numpy()
    Np, Nq = p.np1 * p.np2, p.nq1 * p.nq2
    sb, rem = ids // (Nq * Np), ids % (Nq * Np)
    qf, pf = rem // Np, rem % Np
    # coefficients at two seeded q nodes among those that kept beams
    r = fi.rng(77)
    for q in r.choice(np.unique(qf), 2, replace=False):
        j2, j1 = divmod(int(q), p.nq1)
        one = p.replace(qb1=p.qb1 + p.qs1 * j1, qb2=p.qb2 + p.qs2 * j2, nq1=1, nq2=1)
        psi = oracle.fbi(W.f0[0], g, one)[0, 0]              # [np2][np1]
        w = (p.qs1 * g.d1) * (p.qs2 * g.d2) * p.dp1 * p.dp2 / (2 * np.pi * p.eps) ** 3
        ref = 0.5 * w * psi.ravel()                          # f1 = 0: both branches psi/2
        sel = qf == q
        got = coef[0, sel] + 1j * coef[1, sel]
        want = ref[pf[sel]]
        assert np.abs(got - want).max() <= 1e-10 * np.abs(ref).max(), (q, sel.sum())
    # propagation of 32 seeded beams
    idx = np.sort(r.choice(nb, 32, replace=False))
    ctx.propagate(beams, 1, p.nsteps)
    assert ctx.status()[0] == fga.FGA_OK
    got = beams.f[fga.FGA_F_STATE:, idx].cpu().numpy().T
    k1, k2 = oracle.qnodes(p)
    pm1, pm2 = oracle.pmesh(p.np1, p.dp1), oracle.pmesh(p.np2, p.dp2)
    j2s, j1s = qf[idx] // p.nq1, qf[idx] % p.nq1
    l2s, l1s = pf[idx] // p.np1, pf[idx] % p.np1
    st0 = np.zeros((32, oracle.NSTATE))
    st0[:, 0] = g.o1 + g.d1 * k1[j1s]
    st0[:, 1] = g.o2 + g.d2 * k2[j2s]
    st0[:, 2] = pm1[l1s]
    st0[:, 3] = pm2[l2s]
    st0[:, 5] = st0[:, 11] = 1.0      # A = I
    st0[:, 14] = st0[:, 20] = -1.0    # B = -i I
    st0[:, 21] = 2.0                  # a = 2^{d/2}
    sig = np.where(sb[idx] == 0, 1, -1).astype(np.int8)
    b = oracle.Beams(np.zeros(32, np.int32), sig, ids[idx], np.ones(32, complex),
                     np.zeros((32, 2)), st0, np.array([0, 32], np.int64))
    oracle.propagate(b, W.c, g, p.dt, p.nsteps)
    assert pairwise_state_err(got, b.state) <= 1e-9
    ctx.close()
    del beams
    torch.cuda.empty_cache()

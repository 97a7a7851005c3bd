"""The large configuration at full size: 2048 x 1024 smooth layered model,
eps = 1/1024, point source, q-mesh 147 x 74, p-mesh 400 x 400, tau = 1e-6
(5.0e7 beams from 3.5e9 candidates): both paths against the oracle's values
stored by tests/golden/make_golden.py (beam count, sampled beams, u(T) at
sampled nodes), the mixed paths against the FP64 path on the whole field,
and the FP64 decomposition and propagation against the oracle recomputed at
sampled q nodes and beams."""
import os

import numpy as np
import pytest

import fga_inputs as fi

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large2048_fp64.npz")


def test_large_against_stored_oracle_values():
    """Against the oracle at full size (values written by make_golden.py,
    which calls only the oracle): FP64 beam count and ids of a seeded sample
    of 4096 beams exact, their coefficients (t = 0) and states at T within
    1e-10, u(T) at 2007 nodes (1024 seeded and the nodes nearest 1024
    seeded beams' centres at T, duplicates merged) within 1e-10; the two
    mixed paths' u(T) at the same nodes within 1e-5."""
    import torch
    import paper_1304_3542_amd as fga
    from gpu_helpers import pairwise_state_err, rel_l2
    z = np.load(GOLDEN)
    pick, nodes = z["pick"], z["nodes"]
    for prec in ("fp64", "mixed", "mixed_split"):
        W = fi.workload("large2048", "fp64" if prec == "fp64" else "mixed")
        ctx = fga.FGA(W.grid, W.params, prec)
        ctx.set_velocity(torch.from_numpy(W.c).cuda())
        f0 = torch.from_numpy(np.ascontiguousarray(W.f0)).cuda()
        beams = fga.Beams(int(z["nbeams"]) + 65536, 1)
        ctx.decompose(f0, None, beams)
        assert ctx.status()[0] == fga.FGA_OK
        nb = int(ctx.offsets(beams, 1)[-1])
        pk = torch.from_numpy(pick).cuda()
        ids = beams.id[pk].cpu().numpy() if prec == "fp64" else None
        coef = beams.f[4:6][:, pk].cpu().numpy().T if prec == "fp64" else None
        ctx.propagate(beams, 1, W.params.nsteps)
        u = ctx.reconstruct(beams, 1)[0].cpu().numpy().ravel()[nodes]
        stT = beams.f[fga.FGA_F_STATE:][:, pk].cpu().numpy().T if prec == "fp64" else None
        assert ctx.status()[0] == fga.FGA_OK
        ctx.close()
        del beams
        torch.cuda.empty_cache()
        err_u = rel_l2(u, z["u"])
        if prec == "fp64":
            assert nb == int(z["nbeams"])
            np.testing.assert_array_equal(ids, z["ids"])
            err_c = np.abs(coef - z["coef"]).max() / np.abs(z["coef"]).max()
            err_s = pairwise_state_err(stT, z["stateT"])
            print(f"large2048 fp64 vs oracle: coef {err_c:.2e}, states {err_s:.2e}, u {err_u:.2e}",
                  flush=True)
            assert err_c <= 1e-10 and err_s <= 1e-10 and err_u <= 1e-10
        else:
            print(f"large2048 {prec} vs oracle: {nb} beams, u {err_u:.2e}", flush=True)
            assert abs(nb - int(z["nbeams"])) <= 1e-3 * int(z["nbeams"])
            assert err_u <= 1e-5


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
    err = pairwise_state_err(got, b.state)
    print(f"large2048 sampled beams vs oracle: {err:.2e}", flush=True)
    assert err <= 1e-10
    ctx.close()
    del beams
    torch.cuda.empty_cache()

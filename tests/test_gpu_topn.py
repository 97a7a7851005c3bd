"""The N-largest selection per branch (top_n > 0) through the C ABI against
the oracle: selected beams, coefficients and the reconstruction (FP64), the
mixed path against FP64, several shots, and the degenerate sizes."""
import numpy as np
import pytest

import fga_inputs as fi
import oracle
from gpu_helpers import gpu_run, mixed_params, rel_l2, small_case

pytestmark = pytest.mark.gpu


def _branch_sets(ids, shot, nqp):
    """Shot-local candidate indices of each branch."""
    out = []
    for br in range(2):
        lo = (2 * shot + br) * nqp
        out.append(set((ids[(ids >= lo) & (ids < lo + nqp)] - lo).tolist()))
    return out


def _check_selection(gpu_ids, mags_by_shot, n, nqp, rel_gap):
    """Per shot and branch: the GPU keeps min(n, #nonzero) candidates; every
    candidate it keeps and the oracle's N-largest rule drops (or the reverse)
    lies within rel_gap of the N-th largest magnitude (near-ties decided by
    rounding), and nothing else differs."""
    for s, mags in enumerate(mags_by_shot):
        got = _branch_sets(gpu_ids, s, nqp)
        for br in range(2):
            m = mags[br]
            want = set(oracle.select_top_n(m, n).tolist())
            assert len(got[br]) == min(n, int((m > 0).sum())), (s, br)
            diff = got[br] ^ want
            if diff:
                nth = np.sort(m)[::-1][min(n, m.size) - 1]
                assert all(abs(m[i] - nth) <= rel_gap * nth for i in diff), (s, br, len(diff))


def _oracle_mags(g, p, c, f0, f1):
    out = []
    for s in range(f0.shape[0]):
        psi0 = oracle.fbi(f0[s], g, p)
        psi1 = None if f1 is None else oracle.fbi(f1[s], g, p)
        pp, pm = oracle.branches(psi0, psi1, c, g, p)
        out.append(np.stack([np.abs(pp).ravel(), np.abs(pm).ravel()]))
    return out


@pytest.mark.parametrize("n", [1, 13, 500])
def test_topn_fp64_matches_oracle(n):
    g, p, c, f0, f1 = small_case(seed=61)
    p = p.replace(top_n=n, nsteps=20)
    nqp = p.nq1 * p.nq2 * p.np1 * p.np2
    r = gpu_run(g, p, c, f0, f1, "fp64")
    assert r["status"] == 0
    _check_selection(r["id0"], _oracle_mags(g, p, c, f0, f1), n, nqp, 1e-12)
    b = oracle.decompose(f0, f1, c, g, p)
    np.testing.assert_array_equal(r["id0"], b.cand)
    np.testing.assert_allclose(r["f0"][4], b.coef[:, 0], rtol=0, atol=1e-12 * np.abs(b.coef).max())
    np.testing.assert_allclose(r["f0"][5], b.coef[:, 1], rtol=0, atol=1e-12 * np.abs(b.coef).max())
    oracle.propagate(b, c, g, p.dt, p.nsteps)
    assert rel_l2(r["u"][0], oracle.reconstruct(b, g, p)) <= 1e-10


def test_topn_mixed_selection_and_field():
    """Mixed precision compares FP32 magnitudes: the set may differ from the
    FP64 rule only at near-ties, and u stays within 1e-5 of the FP64 path."""
    g, p, c, f0, f1 = small_case(seed=62)
    p = p.replace(top_n=400, nsteps=20)
    nqp = p.nq1 * p.nq2 * p.np1 * p.np2
    rm = gpu_run(g, mixed_params(p), c, f0, f1, "mixed")
    rd = gpu_run(g, mixed_params(p), c, f0, f1, "fp64")
    assert rm["status"] == 0 and rd["status"] == 0
    _check_selection(rm["id0"], _oracle_mags(g, p, c, f0, f1), 400, nqp, 1e-5)
    assert rel_l2(rm["u"], rd["u"]) <= 1e-5


def test_topn_several_shots_and_degenerate_sizes():
    """Three shots with uneven content; N above the candidate count keeps
    every nonzero candidate (= threshold mode with tau = 0); a zero shot
    keeps nothing."""
    g, p, c, f0, f1 = small_case(seed=63, nshots=3)
    f0 = f0.copy()
    f1 = f1.copy()
    f1[1] *= 0.0
    nqp = p.nq1 * p.nq2 * p.np1 * p.np2
    p = p.replace(nsteps=0)
    for n in (7, 250):
        r = gpu_run(g, p.replace(top_n=n), c, f0, f1, "fp64", want_u=False)
        _check_selection(r["id0"], _oracle_mags(g, p, c, f0, f1), n, nqp, 1e-12)
        np.testing.assert_array_equal(np.diff(r["offsets"]), [2 * n] * 3)
    big = gpu_run(g, p.replace(top_n=10 ** 9), c, f0, f1, "fp64", want_u=False)
    allnz = gpu_run(g, p.replace(tau=0.0), c, f0, f1, "fp64", want_u=False)
    np.testing.assert_array_equal(big["id0"], allnz["id0"])
    z = gpu_run(g, p.replace(top_n=5), c, np.zeros_like(f0[:1]), None, "fp64", want_u=False)
    assert int(z["offsets"][-1]) == 0 and z["status"] == 0


def test_topn_full_size_counts_and_order():
    """topn512 (point512 with N = 5650 per branch): the kept beams are 5650 per
    branch, in candidate order, with |C| of every kept beam of a branch at
    least that of the largest dropped one (the dropped maximum taken from
    the threshold run that keeps a superset; in mixed precision up to the
    FP32 rounding of the magnitudes)."""
    import torch
    import paper_1304_3542_amd as fga
    for prec in ("fp64", "mixed"):
        W = fi.workload("topn512", prec)
        g, p = W.grid, W.params
        ctx = fga.FGA(g, p, prec)
        ctx.set_velocity(torch.from_numpy(W.c).cuda())
        beams = fga.Beams(4 * p.top_n, 1)
        ctx.decompose(torch.from_numpy(W.f0).cuda(), None, beams)
        assert ctx.status()[0] == 0
        off = ctx.offsets(beams, 1)
        assert off[-1] == 2 * p.top_n
        ids = beams.id[: off[-1]].cpu().numpy()
        assert np.all(np.diff(ids) > 0)
        C = beams.f[4:6, : off[-1]].cpu().numpy()
        mag = np.hypot(C[0], C[1])
        # superset: the relative threshold at the smallest kept magnitude
        ref = fga.FGA(g, p.replace(top_n=0, tau=0.5 * mag.min() / mag.max()), prec)
        ref.set_velocity(torch.from_numpy(W.c).cuda())
        rb = fga.Beams(2_000_000, 1)
        ref.decompose(torch.from_numpy(W.f0).cuda(), None, rb)
        roff = ref.offsets(rb, 1)
        rids = rb.id[: roff[-1]].cpu().numpy()
        rC = rb.f[4:6, : roff[-1]].cpu().numpy()
        rmag = np.hypot(rC[0], rC[1])
        kept = np.isin(rids, ids)
        assert kept.sum() == ids.size
        nqp = p.nq1 * p.nq2 * p.np1 * p.np2
        # the mixed path orders FP32 magnitudes: near-ties may swap at the
        # FP32 rounding of |psi| (relative ~1e-7)
        slack = 0.0 if prec == "fp64" else 1e-6
        for br in range(2):
            inb = (rids // nqp) == br
            assert rmag[inb & kept].min() >= (1.0 - slack) * rmag[inb & ~kept].max()

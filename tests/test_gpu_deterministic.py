"""Deterministic mode of the gradient entry points (deterministic = 1): dJ/dc
reduced in a fixed order from per-beam logs.  Repeated calls, in the same
context (log length already known) and in fresh ones (logs rerun after an
overflow), give bit-identical gradients, equal to the atomic mode's to
rounding and to the gradient oracle."""
import numpy as np
import pytest

import fga_inputs as fi
import oracle
import oracle.adjoint as oadj
from test_gpu_adjoint import gpu_gradient, rel_max
from test_gpu_field_adjoint import _field_chain
from test_oracle_adjoint import adjoint_case, c_oracle_traces

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("with_f1", [False, True])
def test_deterministic_trace_adjoint_bit_identical_and_exact(with_f1):
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(with_f1)
    b = oracle.decompose(f0, f1, c, g, p)
    data = 0.5 * c_oracle_traces(c * 1.02, f0, f1, g, p, b.cand, rec, every, nrec)
    J, dc, df0, df1, tr = oadj.gradient(c, f0, f1, g, p, b.cand, rec, every, nrec, data)
    pd = p.replace(deterministic=1)
    r1 = gpu_gradient(g, pd, c, f0, f1, rec, every, nrec, data)
    r2 = gpu_gradient(g, pd, c, f0, f1, rec, every, nrec, data)
    ra = gpu_gradient(g, p, c, f0, f1, rec, every, nrec, data)
    for r in (r1, r2):
        assert r["status"][0] == 0
    for k in ("dc", "df0") + (("df1",) if with_f1 else ()):
        np.testing.assert_array_equal(r1[k], r2[k])
        assert rel_max(r1[k], ra[k]) <= 1e-12
    assert rel_max(r1["dc"], dc) <= 1e-10
    assert rel_max(r1["df0"], df0) <= 1e-10


def test_deterministic_field_chain_bit_identical_and_exact():
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(True)
    ns = f0.shape[0]
    b = oracle.decompose(f0, f1, c, g, p)
    nodes = np.arange(g.n1 * g.n2, dtype=np.int32)
    d = 0.5 * c_oracle_traces(c * 1.02, f0, f1, g, p, b.cand, nodes, p.nsteps, 1)
    J, dc, df0, df1, tr = oadj.gradient(c, f0, f1, g, p, b.cand, nodes, p.nsteps, 1, d)
    pd = p.replace(deterministic=1)
    d3 = d.reshape(ns, g.n2, g.n1)
    r1 = _field_chain(g, pd, c, f0, f1, d3, 5, 3)
    r2 = _field_chain(g, pd, c, f0, f1, d3, 5, 3)
    for k in ("dc", "df0", "df1", "lam0"):
        np.testing.assert_array_equal(r1[k], r2[k])
    assert rel_max(r1["dc"], dc) <= 1e-10
    assert rel_max(r1["df0"], df0) <= 1e-10
    assert rel_max(r1["df1"], df1) <= 1e-10


def test_deterministic_full_size_adjoint_repeatable():
    """adjoint256 at full size (8 shots, 250 steps): the first call's logs
    overflow their initial length and are rerun; a second call in the same
    context and a call in a fresh context give bit-identical dJ/dc and
    dJ/dC, which equal the atomic mode's to rounding."""
    import torch
    import paper_1304_3542_amd as fga
    W = fi.workload("adjoint256", "fp64")
    g = W.grid
    ns = W.nshots
    nrec_t = W.params.nsteps // W.rec_every

    def run(ctx):
        beams = fga.Beams(2 * W.params.nq1 * W.params.nq2 * W.params.np1 * W.params.np2 * ns, ns)
        ctx.set_velocity(torch.from_numpy(W.c_true).cuda())
        f0 = torch.from_numpy(np.ascontiguousarray(W.f0)).cuda()
        ctx.decompose(f0, None, beams)
        rec = torch.from_numpy(W.receivers).cuda()
        data = ctx.trace(beams, ns, rec, W.rec_every, nrec_t)
        ctx.set_velocity(torch.from_numpy(W.c).cuda())
        ctx.decompose(f0, None, beams)
        ckpt = torch.empty((nrec_t, fga.FGA_NSTATE, beams.capacity), dtype=torch.float64,
                           device="cuda")
        tr = ctx.trace(beams, ns, rec, W.rec_every, nrec_t, ckpt)
        dc = torch.zeros((g.n2, g.n1), dtype=torch.float64, device="cuda")
        gcoef = ctx.trace_adjoint(beams, ns, rec, W.rec_every, nrec_t, ckpt,
                                  (tr - data).contiguous(), dc)
        assert ctx.status()[0] == 0
        nb = int(ctx.offsets(beams, ns)[-1])
        return dc.cpu().numpy(), gcoef[:, :nb].cpu().numpy()

    ctx = fga.FGA(g, W.params.replace(deterministic=1), "fp64", max_shots=ns)
    dc1, gc1 = run(ctx)
    dc2, gc2 = run(ctx)
    dc3, gc3 = run(fga.FGA(g, W.params.replace(deterministic=1), "fp64", max_shots=ns))
    dca, gca = run(fga.FGA(g, W.params, "fp64", max_shots=ns))
    np.testing.assert_array_equal(dc1, dc2)
    np.testing.assert_array_equal(dc1, dc3)
    np.testing.assert_array_equal(gc1, gc2)
    np.testing.assert_array_equal(gc1, gc3)
    assert np.abs(dc1).max() > 0
    assert rel_max(dc1, dca) <= 1e-12
    assert rel_max(gc1, gca) <= 1e-12

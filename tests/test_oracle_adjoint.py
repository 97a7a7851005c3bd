"""Pins of the gradient oracle (oracle/adjoint.py, torch autograd of a plain
forward): its forward equals the C oracle's receiver traces, and its
gradient equals central finite differences of the C oracle's misfit with
the beam set held fixed."""
import math

import numpy as np
import pytest

import fga_inputs as fi
import oracle
import oracle.adjoint as oadj


def adjoint_case(with_f1=False, seed=41):
    g = fi.Grid(40, 32, 0.0, 0.0, 1 / 32, 1 / 32)
    eps = 1 / 200
    c = fi.smooth_layered_velocity(g, seed=seed, smooth_cells=3.0)
    r = fi.rng(seed)
    ns = 2
    f0 = np.stack([fi.wavepacket_source(g, (r.uniform(0.45, 0.8), 0.35), 0.06,
                                        (r.uniform(-0.4, 0.4), 0.9), eps) for _ in range(ns)])
    f1 = None
    if with_f1:
        f1 = np.stack([0.7 * fi.wavepacket_source(g, (0.6, 0.4), 0.05, (0.8, 0.3), eps)
                       for _ in range(ns)])
    p = fi.Params(eps, 3, 4, 4, 4, 9, 6, 8, 8, 0.35, 0.35, 1e-3, 1e-16, 1e-16, 1e-3, 15)
    rec = np.arange(2 * g.n1, 3 * g.n1, dtype=np.int32)          # row i2 = 2
    return g, p, c, f0, f1, rec, 5, 3


def c_oracle_traces(c, f0, f1, g, p, cand, rec, rec_every, nrec, c_for_branches=None):
    """C-oracle traces of the beams `cand` (frozen set) for the given c and f0."""
    return oracle.trace_frozen(c, f0, f1, g, p, cand, rec, rec_every, nrec,
                               c_for_branches=c_for_branches)


@pytest.mark.parametrize("with_f1", [False, True])
def test_torch_forward_matches_c_oracle(with_f1):
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(with_f1)
    b = oracle.decompose(f0, f1, c, g, p)
    assert 50 < b.n < 8000
    tr_c = oracle.trace(b, c, g, p, rec, every, nrec)
    import torch
    tr_t = oadj.traces(torch.tensor(c), torch.tensor(f0),
                       None if f1 is None else torch.tensor(f1), g, p, b.cand, rec, every,
                       nrec, f0.shape[0]).numpy()
    assert np.abs(tr_c).max() > 1e-3
    np.testing.assert_allclose(tr_t, tr_c, rtol=0, atol=1e-12 * np.abs(tr_c).max())


@pytest.mark.parametrize("with_f1", [False, True])
def test_gradient_matches_finite_differences(with_f1):
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(with_f1)
    b = oracle.decompose(f0, f1, c, g, p)
    cand = b.cand
    data = 0.5 * c_oracle_traces(c * 1.02, f0, f1, g, p, cand, rec, every, nrec)
    J, dc, df0, df1, tr = oadj.gradient(c, f0, f1, g, p, cand, rec, every, nrec, data)

    def Jc(cc, ff0, ff1):
        t = c_oracle_traces(cc, ff0, ff1, g, p, cand, rec, every, nrec)
        return 0.5 * ((t - data) ** 2).sum()

    assert abs(Jc(c, f0, f1) - J) <= 1e-12 * abs(J)
    # the cells and nodes with the largest gradients, plus a few seeded ones
    r = fi.rng(5)
    cells = list(np.argsort(-np.abs(dc).ravel())[:4]) + list(r.choice(c.size, 2, replace=False))
    for idx in cells:
        i2, i1 = np.unravel_index(idx, c.shape)
        h = 1e-6 * c[i2, i1]
        cp, cm = c.copy(), c.copy()
        cp[i2, i1] += h
        cm[i2, i1] -= h
        fd = (Jc(cp, f0, f1) - Jc(cm, f0, f1)) / (2 * h)
        assert abs(fd - dc[i2, i1]) <= 1e-6 * np.abs(dc).max(), (idx, fd, dc[i2, i1])
    nodes = list(np.argsort(-np.abs(df0).ravel())[:3])
    for idx in nodes:
        s, i2, i1 = np.unravel_index(idx, df0.shape)
        h = 1e-6
        fp, fm = f0.copy(), f0.copy()
        fp[s, i2, i1] += h
        fm[s, i2, i1] -= h
        fd = (Jc(c, fp, f1) - Jc(c, fm, f1)) / (2 * h)
        assert abs(fd - df0[s, i2, i1]) <= 1e-6 * np.abs(df0).max(), (idx, fd, df0[s, i2, i1])
    if with_f1:
        idx = int(np.argmax(np.abs(df1).ravel()))
        s, i2, i1 = np.unravel_index(idx, df1.shape)
        fp, fm = f1.copy(), f1.copy()
        fp[s, i2, i1] += 1e-6
        fm[s, i2, i1] -= 1e-6
        fd = (Jc(c, f0, fp) - Jc(c, f0, fm)) / 2e-6
        assert abs(fd - df1[s, i2, i1]) <= 1e-6 * np.abs(df1).max()


def _propagated_case():
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(True)
    b = oracle.decompose(f0, f1, c, g, p)
    oracle.propagate(b, c, g, p.dt, p.nsteps)
    return g, p, c, b, f0.shape[0]


def _field_J(b, g, p, ns, du):
    return sum(float((oracle.reconstruct(b, g, p, shot=s) * du[s]).sum()) for s in range(ns))


def test_recons_oracle_matches_c_oracle_field():
    """The torch windowed sum at every node (recons_at) equals the C oracle's
    field reconstruction (recons eq.)."""
    import torch
    g, p, c, b, ns = _propagated_case()
    st = torch.tensor(b.state)
    Ca = torch.tensor(b.coef[:, 0] + 1j * b.coef[:, 1]) * torch.complex(st[:, 21], st[:, 22])
    u = oadj.recons_at(st[:, 0:2], st[:, 2:4], st[:, 4], Ca, torch.as_tensor(b.shot.astype(np.int64)),
                       np.arange(g.n1 * g.n2), g, p, ns).numpy().reshape(ns, g.n2, g.n1)
    for s in range(ns):
        ref = oracle.reconstruct(b, g, p, shot=s)
        assert np.abs(ref).max() > 1e-3
        np.testing.assert_allclose(u[s], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_recons_vjp_matches_finite_differences_and_is_bilinear_in_C():
    """dJ/d(Q, P, S, a, C) of J = sum du u from recons_vjp against central
    differences of the C oracle's reconstruction for seeded beams and every
    component (boxes unchanged by the small steps), and <u(C = v), du> =
    <v, dJ/dC> exactly (u is linear in C)."""
    g, p, c, b, ns = _propagated_case()
    r = fi.rng(61)
    du = r.standard_normal((ns, g.n2, g.n1))
    ds, dcf = oadj.recons_vjp(b.state, b.coef, b.shot, g, p, ns, du)
    assert np.all(ds[:, 5:21] == 0)
    for bi in r.choice(b.n, 6, replace=False):
        for comp in (0, 1, 2, 3, 4, 21, 22, "C0", "C1"):
            arr, j = (b.coef, int(comp[1])) if isinstance(comp, str) else (b.state, comp)
            x0 = arr[bi, j]
            h = 1e-6 * max(abs(x0), 1e-3 if isinstance(comp, str) else 1.0)
            if isinstance(comp, str):
                h = 1e-6 * np.abs(b.coef).max()
            arr[bi, j] = x0 + h
            jp = _field_J(b, g, p, ns, du)
            arr[bi, j] = x0 - h
            jm = _field_J(b, g, p, ns, du)
            arr[bi, j] = x0
            fd = (jp - jm) / (2 * h)
            got = dcf[bi, j] if isinstance(comp, str) else ds[bi, j]
            scale = np.abs(dcf).max() if isinstance(comp, str) else np.abs(ds[:, j]).max()
            assert abs(fd - got) <= 1e-6 * scale, (bi, comp, fd, got, scale)
    v = r.standard_normal(b.coef.shape)
    bv = oracle.Beams(b.shot, b.sigma, b.cand, b.psi, v, b.state, b.offsets)
    lhs = _field_J(bv, g, p, ns, du)
    rhs = float((v * dcf).sum())
    assert abs(lhs - rhs) <= 1e-12 * np.abs(v).sum() * np.abs(dcf).max() + 1e-12 * abs(lhs)

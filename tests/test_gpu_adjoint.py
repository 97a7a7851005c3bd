"""Parity of the hand-written adjoint (fga_trace_adjoint +
fga_decompose_adjoint, through the C ABI) with the gradient oracle
(reverse-mode autodiff of a plain forward), on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import oracle.adjoint as oadj
from test_oracle_adjoint import adjoint_case, c_oracle_traces

pytestmark = pytest.mark.gpu


def gpu_gradient(g, p, c, f0, f1, rec, every, nrec, data, precision="fp64"):
    import torch
    import paper_1304_3542_amd as fga
    ns = f0.shape[0]
    ctx = fga.FGA(g, p, precision, max_shots=ns)
    ctx.set_velocity(torch.from_numpy(c).cuda())
    cand = 2 * p.nq1 * p.nq2 * p.np1 * p.np2 * ns
    beams = fga.Beams(cand, ns)
    f1t = None if f1 is None else torch.from_numpy(f1).cuda()
    ctx.decompose(torch.from_numpy(f0).cuda(), f1t, beams)
    rec_t = torch.from_numpy(rec).cuda()
    ckpt = torch.empty((ctx.ckpt_rows(every, nrec), fga.FGA_NSTATE, beams.capacity),
                       dtype=torch.float64, device="cuda")
    tr = ctx.trace(beams, ns, rec_t, every, nrec, ckpt)
    gtr = tr - torch.from_numpy(data).cuda()
    dc = torch.zeros_like(ctx_c := torch.from_numpy(c).cuda())
    gcoef = ctx.trace_adjoint(beams, ns, rec_t, every, nrec, ckpt, gtr.contiguous(), dc)
    df1 = None if f1 is None else torch.empty_like(f1t)
    df0 = ctx.decompose_adjoint(beams, ns, gcoef, df1, dc if f1 is not None else None)
    st = ctx.status()
    nb = int(ctx.offsets(beams, ns)[-1])
    return dict(status=st, ids=beams.id[:nb].cpu().numpy(), tr=tr.cpu().numpy(),
                dc=dc.cpu().numpy(), df0=df0.cpu().numpy(),
                df1=None if df1 is None else df1.cpu().numpy())


def rel_max(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("with_f1,layout", [(False, "row"), (True, "row"), (True, "scattered")])
def test_adjoint_fp64_matches_gradient_oracle(with_f1, layout):
    """Receivers along one row (the factors stepped along it) and in general
    position (evaluated one by one)."""
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(with_f1)
    if layout == "scattered":
        rec = np.concatenate([rec[::3], rec[1::7] + 5 * g.n1]).astype(np.int32)
    b = oracle.decompose(f0, f1, c, g, p)
    data = 0.5 * c_oracle_traces(c * 1.02, f0, f1, g, p, b.cand, rec, every, nrec)
    J, dc, df0, df1, tr = oadj.gradient(c, f0, f1, g, p, b.cand, rec, every, nrec, data)
    r = gpu_gradient(g, p, c, f0, f1, rec, every, nrec, data)
    assert r["status"][0] == 0
    np.testing.assert_array_equal(r["ids"], b.cand)
    assert rel_max(r["tr"], tr) <= 1e-10
    assert rel_max(r["dc"], dc) <= 1e-10, rel_max(r["dc"], dc)
    assert rel_max(r["df0"], df0) <= 1e-10, rel_max(r["df0"], df0)
    if with_f1:
        assert rel_max(r["df1"], df1) <= 1e-10


@pytest.mark.parametrize("grad_log", [-1, 2])
def test_adjoint_same_gradient_for_every_log_setting(grad_log):
    """dJ/dc added with atomics where each record is made (grad_log = -1), or
    logged in 2 slots per beam with the rest added where made (the fallback
    of a full log), equals the automatic mode's (every record logged, then
    summed by cell) up to the rounding order, and the oracle's."""
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(True)
    b = oracle.decompose(f0, f1, c, g, p)
    data = 0.5 * c_oracle_traces(c * 1.02, f0, f1, g, p, b.cand, rec, every, nrec)
    J, dc, df0, df1, tr = oadj.gradient(c, f0, f1, g, p, b.cand, rec, every, nrec, data)
    ra = gpu_gradient(g, p, c, f0, f1, rec, every, nrec, data)
    r = gpu_gradient(g, p.replace(grad_log=grad_log), c, f0, f1, rec, every, nrec, data)
    assert r["status"][0] == 0 and ra["status"][0] == 0
    for k in ("dc", "df0", "df1"):
        assert rel_max(r[k], ra[k]) <= 1e-12, (k, rel_max(r[k], ra[k]))
    assert rel_max(r["dc"], dc) <= 1e-10
    assert rel_max(r["df1"], df1) <= 1e-10


@pytest.mark.parametrize("with_f1,mode", [(False, "auto"), (True, "auto"), (True, "det")])
def test_adjoint_with_every_step_checkpoints(with_f1, mode):
    """ckpt_every_step = 1: the forward keeps the state before every step
    and the adjoint reads it instead of recomputing each segment.  The same
    gradient as the default (to rounding: the forward's velocity goes
    through the per-cell coefficients, the recompute through the B-spline
    taps) and as the gradient oracle; in deterministic mode repeatable bit for
    bit."""
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(with_f1)
    if mode == "det":
        p = p.replace(deterministic=1)
    b = oracle.decompose(f0, f1, c, g, p)
    data = 0.5 * c_oracle_traces(c * 1.02, f0, f1, g, p, b.cand, rec, every, nrec)
    J, dc, df0, df1, tr = oadj.gradient(c, f0, f1, g, p, b.cand, rec, every, nrec, data)
    ra = gpu_gradient(g, p, c, f0, f1, rec, every, nrec, data)
    pe = p.replace(ckpt_every_step=1)
    r = gpu_gradient(g, pe, c, f0, f1, rec, every, nrec, data)
    assert r["status"][0] == 0
    np.testing.assert_array_equal(r["tr"], ra["tr"])
    keys = ("dc", "df0") + (("df1",) if with_f1 else ())
    for k in keys:
        assert rel_max(r[k], ra[k]) <= 1e-12, (k, rel_max(r[k], ra[k]))
    assert rel_max(r["dc"], dc) <= 1e-10
    assert rel_max(r["df0"], df0) <= 1e-10
    if mode == "det":
        r2 = gpu_gradient(g, pe, c, f0, f1, rec, every, nrec, data)
        for k in keys:
            np.testing.assert_array_equal(r[k], r2[k])


def test_adjoint_mixed_within_1e5():
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(False)
    b = oracle.decompose(f0, f1, c, g, p)
    data = 0.5 * c_oracle_traces(c * 1.02, f0, f1, g, p, b.cand, rec, every, nrec)
    J, dc, df0, df1, tr = oadj.gradient(c, f0, f1, g, p, b.cand, rec, every, nrec, data)
    r = gpu_gradient(g, p.replace(tau_fbi=1e-8, tau_win=1e-8), c, f0, f1, rec, every, nrec,
                     data, "mixed")
    assert r["status"][0] == 0
    assert np.linalg.norm(r["dc"] - dc) / np.linalg.norm(dc) <= 1e-5
    assert np.linalg.norm(r["df0"] - df0) / np.linalg.norm(df0) <= 1e-5


def test_adjoint_full_size_matches_oracle_finite_differences():
    """adjoint256 at full size (8 shots, 256 receivers, 25 records, 250
    steps) against the oracle (tests/golden/adjoint256_fp64.npz, written by
    make_golden.py calling only the oracle): the misfit data are the oracle's
    traces on the model with the +5 % anomaly; the GPU's traces on the
    background model equal the oracle's (1e-10), so does J; dJ/dc equals the
    oracle's central differences of J (h = 1e-6 c, beam set held fixed) at
    8 seeded cells and 16 cells at and below the sources, and dJ/df0 the
    oracle's central differences (exact up to rounding: J is quadratic in
    f0) at 8 seeded source nodes, with checkpoints per record and of every
    step."""
    import os
    import torch
    import fga_inputs as fi
    import paper_1304_3542_amd as fga
    z = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                             "adjoint256_fp64.npz"))
    W = fi.workload("adjoint256", "fp64")
    g, p = W.grid, W.params
    ns = W.nshots
    nrec_t = p.nsteps // W.rec_every
    data = torch.from_numpy(z["data"]).cuda()
    c = torch.from_numpy(W.c).cuda()
    f0 = torch.from_numpy(np.ascontiguousarray(W.f0)).cuda()
    rec = torch.from_numpy(W.receivers).cuda()
    for every_step in (0, 1):
        ctx = fga.FGA(g, p.replace(ckpt_every_step=every_step), "fp64", max_shots=ns)
        ctx.set_velocity(c)
        beams = fga.Beams(int(z["nbeams"]) + 1024, ns)
        ctx.decompose(f0, None, beams)
        nb = int(ctx.offsets(beams, ns)[-1])
        assert ctx.status()[0] == 0 and nb == int(z["nbeams"])
        np.testing.assert_array_equal(beams.id[:nb].cpu().numpy(), z["ids"])
        ckpt = torch.empty((ctx.ckpt_rows(W.rec_every, nrec_t), fga.FGA_NSTATE, beams.capacity),
                           dtype=torch.float64, device="cuda")
        tr = ctx.trace(beams, ns, rec, W.rec_every, nrec_t, ckpt)
        trn = tr.cpu().numpy()
        err_t = np.abs(trn - z["traces"]).max() / np.abs(z["traces"]).max()
        J = 0.5 * float(((tr - data) ** 2).sum())
        dc = torch.zeros_like(c)
        gcoef = ctx.trace_adjoint(beams, ns, rec, W.rec_every, nrec_t, ckpt,
                                  (tr - data).contiguous(), dc)
        df0 = ctx.decompose_adjoint(beams, ns, gcoef).cpu().numpy()
        assert ctx.status()[0] == 0
        dcn = dc.cpu().numpy().ravel()
        fdc, fdf = z["fd_c"], z["fd_f0"]
        err_c = np.abs(dcn[z["cells"]] - fdc).max() / np.abs(fdc).max()
        got_f = np.array([df0[s].ravel()[k] for s, k in z["f0_nodes"]])
        err_f = np.abs(got_f - fdf).max() / np.abs(fdf).max()
        print(f"adjoint256 (every step {every_step}): traces {err_t:.2e}, J {J:.6e} vs "
              f"{float(z['J']):.6e}, dJ/dc vs oracle FD {err_c:.2e}, dJ/df0 {err_f:.2e}",
              flush=True)
        assert err_t <= 1e-10
        assert abs(J - float(z["J"])) <= 1e-10 * abs(float(z["J"]))
        assert err_c <= 1e-6          # central differences in c: O(h^2) with h = 1e-6 c
        assert err_f <= 1e-9          # J is quadratic in f0: differences exact up to rounding
        ctx.close()
        del ckpt, beams
        torch.cuda.empty_cache()


@pytest.mark.parametrize("with_f1,every_step", [(False, 0), (True, 0), (True, 1)])
def test_autograd_function_matches_oracle_gradient(with_f1, every_step):
    """The adjoint behind torch.autograd: loss.backward() through
    paper_1304_3542_amd.traces gives the gradient oracle's dJ/dc, dJ/df0
    (and dJ/df1), with checkpoints per record or of every step."""
    import torch
    import paper_1304_3542_amd as fga
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(with_f1)
    p = p.replace(ckpt_every_step=every_step)
    b = oracle.decompose(f0, f1, c, g, p)
    data = 0.5 * c_oracle_traces(c * 1.02, f0, f1, g, p, b.cand, rec, every, nrec)
    J, dc, df0, df1, _ = oadj.gradient(c, f0, f1, g, p, b.cand, rec, every, nrec, data)
    ns = f0.shape[0]
    ctx = fga.FGA(g, p, "fp64", max_shots=ns)
    beams = fga.Beams(2 * p.nq1 * p.nq2 * p.np1 * p.np2 * ns, ns)
    ct = torch.from_numpy(c).cuda().requires_grad_(True)
    f0t = torch.from_numpy(f0).cuda().requires_grad_(True)
    f1t = None if f1 is None else torch.from_numpy(f1).cuda().requires_grad_(True)
    tr = fga.traces(ct, f0t, f1t, ctx, beams, torch.from_numpy(rec).cuda(), every, nrec)
    loss = 0.5 * ((tr - torch.from_numpy(data).cuda()) ** 2).sum()
    loss.backward()
    assert ctx.status()[0] == 0
    assert abs(loss.item() - J) <= 1e-10 * abs(J)
    assert rel_max(ct.grad.cpu().numpy(), dc) <= 1e-10
    assert rel_max(f0t.grad.cpu().numpy(), df0) <= 1e-10
    if with_f1:
        assert rel_max(f1t.grad.cpu().numpy(), df1) <= 1e-10


def _dot_case(with_f1):
    """The small adjoint case with every nonzero candidate kept (tau = 0), so
    that the beam set does not depend on the input of the linear map."""
    import torch
    import paper_1304_3542_amd as fga
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(with_f1)
    p = p.replace(tau=0.0)
    ns = f0.shape[0]
    ctx = fga.FGA(g, p, "fp64", max_shots=ns)
    ctx.set_velocity(torch.from_numpy(c).cuda())
    beams = fga.Beams(2 * p.nq1 * p.nq2 * p.np1 * p.np2 * ns, ns)
    return g, p, c, f0, f1, rec, every, nrec, ns, ctx, beams


@pytest.mark.parametrize("with_f1", [False, True])
def test_decompose_adjoint_dot_product(with_f1):
    """<L v, w> = <v, L^T w> for L: (f0, f1) -> C (the psi eq., u_{+-,0} and
    the weight w/(2 pi eps)^3) with the beam set fixed, at random v and w:
    the transposed windowed DFTs of fga_decompose_adjoint are the exact
    transpose of the forward ones."""
    import torch
    g, p, c, f0, f1, rec, every, nrec, ns, ctx, beams = _dot_case(with_f1)
    r = np.random.default_rng(7)
    v0 = r.standard_normal(f0.shape)
    v1 = r.standard_normal(f0.shape) if with_f1 else None
    ctx.decompose(torch.from_numpy(v0).cuda(), None if v1 is None else torch.from_numpy(v1).cuda(),
                  beams)
    nb = int(ctx.offsets(beams, ns)[-1])
    assert ctx.status()[0] == 0 and nb == beams.capacity      # every candidate kept
    Lv = beams.f[4:6, :nb].cpu().numpy()
    w = r.standard_normal((2, beams.capacity))
    df1 = torch.empty(f0.shape, dtype=torch.float64, device="cuda") if with_f1 else None
    dc = torch.zeros(c.shape, dtype=torch.float64, device="cuda") if with_f1 else None
    df0 = ctx.decompose_adjoint(beams, ns, torch.from_numpy(w).cuda(), df1, dc)
    assert ctx.status()[0] == 0
    lhs = float((Lv * w[:, :nb]).sum())
    rhs = float((v0 * df0.cpu().numpy()).sum())
    norm = np.linalg.norm(Lv) * np.linalg.norm(w[:, :nb])
    if with_f1:
        rhs += float((v1 * df1.cpu().numpy()).sum())
    assert abs(lhs) > 1e-4 * norm
    assert abs(lhs - rhs) <= 1e-13 * norm, (lhs, rhs, norm)


def test_trace_adjoint_dot_product_in_coefficients():
    """<T v, g> = <v, T^T g> for T: C -> traces (the receiver sums after the
    RK4 segments, linear in the beam coefficients C for a fixed c), at random
    C and random trace weights g: gcoef of fga_trace_adjoint is the exact
    transpose of the forward receiver sums."""
    import torch
    import paper_1304_3542_amd as fga
    g, p, c, f0, f1, rec, every, nrec, ns, ctx, beams = _dot_case(False)
    ctx.decompose(torch.from_numpy(f0).cuda(), None, beams)
    nb = int(ctx.offsets(beams, ns)[-1])
    assert ctx.status()[0] == 0 and nb > 1000
    r = np.random.default_rng(8)
    v = r.standard_normal((2, nb))
    beams.f[4:6, :nb] = torch.from_numpy(v).cuda()
    rec_t = torch.from_numpy(rec).cuda()
    ckpt = torch.empty((nrec, fga.FGA_NSTATE, beams.capacity), dtype=torch.float64, device="cuda")
    Tv = ctx.trace(beams, ns, rec_t, every, nrec, ckpt)
    gw = r.standard_normal(tuple(Tv.shape))
    dc = torch.zeros(c.shape, dtype=torch.float64, device="cuda")
    gcoef = ctx.trace_adjoint(beams, ns, rec_t, every, nrec, ckpt, torch.from_numpy(gw).cuda(), dc)
    assert ctx.status()[0] == 0
    Tv = Tv.cpu().numpy()
    lhs = float((Tv * gw).sum())
    rhs = float((v * gcoef[:, :nb].cpu().numpy()).sum())
    norm = np.linalg.norm(Tv) * np.linalg.norm(gw)
    assert abs(lhs) > 1e-4 * norm
    assert abs(lhs - rhs) <= 1e-13 * norm, (lhs, rhs, norm)


def test_trace_adjoint_directional_derivative_in_velocity():
    """<dJ/dc, dc> from the adjoint (through the tangent of the RK4 segments
    of the ray, dynamic ray tracing and amplitude equations) equals the
    derivative of J along a smooth direction dc, from central differences of
    the FP64 forward at steps h and h/2 combined by Richardson extrapolation
    (error O(h^4)), with the beam set and the truncation boxes fixed.  At
    h = 0.02 the extrapolated difference itself is off by about 1.5e-7
    relative (the same experiment on the gradient oracle gives -1.5e-7, and
    about 3e-8 at smaller h, where rounding in J takes over), so the bar is
    1e-6."""
    import torch
    import paper_1304_3542_amd as fga
    g, p, c, f0, f1, rec, every, nrec, ns, ctx, beams = _dot_case(True)
    f0t, f1t = torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda()
    ctx.decompose(f0t, f1t, beams)
    nb = int(ctx.offsets(beams, ns)[-1])
    assert ctx.status()[0] == 0 and nb > 1000
    f_init = beams.f.clone()
    rec_t = torch.from_numpy(rec).cuda()
    ctx.set_velocity(torch.from_numpy(c * 1.02).cuda())
    data = ctx.trace(beams, ns, rec_t, every, nrec).cpu().numpy()
    x1 = g.o1 + g.d1 * np.arange(g.n1)
    x2 = g.o2 + g.d2 * np.arange(g.n2)
    dcdir = 0.05 * c * np.sin(2 * np.pi * (1.3 * x1[None, :] + 0.7 * x2[:, None]) + 0.4)

    def J(cgrid):
        # the coefficients C stay those of c (the f1 term through c(q) is
        # the decomposition's part of the gradient, not the traces')
        beams.f.copy_(f_init)
        ctx.set_velocity(torch.from_numpy(cgrid).cuda())
        tr = ctx.trace(beams, ns, rec_t, every, nrec).cpu().numpy()
        return 0.5 * float(((tr - data) ** 2).sum())

    beams.f.copy_(f_init)
    ctx.set_velocity(torch.from_numpy(c).cuda())
    ckpt = torch.empty((nrec, fga.FGA_NSTATE, beams.capacity), dtype=torch.float64, device="cuda")
    tr = ctx.trace(beams, ns, rec_t, every, nrec, ckpt)
    dc = torch.zeros(c.shape, dtype=torch.float64, device="cuda")
    ctx.trace_adjoint(beams, ns, rec_t, every, nrec, ckpt,
                      (tr - torch.from_numpy(data).cuda()).contiguous(), dc)
    assert ctx.status()[0] == 0
    adj = float((dc.cpu().numpy() * dcdir).sum())

    def D(h):
        return (J(c + h * dcdir) - J(c - h * dcdir)) / (2 * h)

    h = 0.02
    rich = (4 * D(h / 2) - D(h)) / 3
    assert abs(adj) > 0
    assert abs(rich - adj) <= 1e-6 * abs(adj), (rich, adj)


def test_short_checkpoint_buffer_rejected_before_any_launch():
    """With ckpt_every_step = 1 a checkpoint buffer of one row per record is
    too short: the binding refuses it (nothing is launched), and accepts the
    nrec_t * rec_every + 1 rows."""
    import torch
    import paper_1304_3542_amd as fga
    g, p, c, f0, f1, rec, every, nrec = adjoint_case(False)
    ns = f0.shape[0]
    ctx = fga.FGA(g, p.replace(ckpt_every_step=1), "fp64", max_shots=ns)
    ctx.set_velocity(torch.from_numpy(c).cuda())
    beams = fga.Beams(2 * p.nq1 * p.nq2 * p.np1 * p.np2 * ns, ns)
    ctx.decompose(torch.from_numpy(f0).cuda(), None, beams)
    rec_t = torch.from_numpy(rec).cuda()
    short = torch.empty((nrec, fga.FGA_NSTATE, beams.capacity), dtype=torch.float64,
                        device="cuda")
    with pytest.raises(ValueError):
        ctx.trace(beams, ns, rec_t, every, nrec, short)
    with pytest.raises(ValueError):
        ctx.propagate_ckpt(beams, ns, every, nrec, short)
    ckpt = torch.empty((nrec * every + 1, fga.FGA_NSTATE, beams.capacity), dtype=torch.float64,
                       device="cuda")
    ctx.trace(beams, ns, rec_t, every, nrec, ckpt)
    assert ctx.status()[0] == 0

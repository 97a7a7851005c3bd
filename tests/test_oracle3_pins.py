"""Pins of the three-dimensional FP64 oracle (oracle/d3.py, fga_oracle3.c)
against facts fixed by the paper (the method for general d, here d = 3) and
by the mathematics: polynomial reproduction of the tricubic B-spline, the
closed-form FBI of a Gaussian wavepacket, straight rays and the closed-form
amplitude in constant velocity, conservation of H, S = 0, symplecticity and
the closed-form amplitude invariant in a heterogeneous model, fourth-order
RK4, the frame identity at t = 0 (which fixes (2 pi eps)^{3d/2} and
a(0) = 2^{d/2}) and the windowed sum against brute force."""
import math

import numpy as np

import fga_inputs.d3 as i3
import oracle.d3 as o3


def _grid():
    return i3.Grid3(20, 18, 16, -0.1, 0.2, 0.05, 1 / 20, 1 / 18, 1 / 16)


def test_tricubic_reproduces_polynomials():
    """Linear fields exactly; x_a^2 -> x_a^2 + d_a^2/3 (the second moment of
    beta3), so the Hessian of a quadratic is exact; away from the clamped
    boundary."""
    g = _grid()
    x1, x2, x3 = g.coords()
    X3, X2, X1 = np.meshgrid(x3, x2, x1, indexing="ij")
    r = np.random.default_rng(1)
    pts = np.stack([g.o[a] + g.d[a] * r.uniform(3, g.n[a] - 4, 60) for a in range(3)], 1)
    lin = 1.2 + 0.3 * X1 - 0.7 * X2 + 0.5 * X3
    v = o3.velocity(lin, g, pts)
    np.testing.assert_allclose(v[:, 0], 1.2 + pts @ np.array([0.3, -0.7, 0.5]), atol=1e-13)
    np.testing.assert_allclose(v[:, 1:4], np.tile([0.3, -0.7, 0.5], (60, 1)), atol=1e-12)
    np.testing.assert_allclose(v[:, 4:], 0.0, atol=1e-10)
    quad = X1 ** 2 + 2 * X2 * X3 - X3 ** 2
    v = o3.velocity(quad, g, pts)
    x, y, z = pts.T
    np.testing.assert_allclose(v[:, 0], x ** 2 + g.d1 ** 2 / 3 + 2 * y * z - z ** 2 - g.d3 ** 2 / 3,
                               atol=1e-12)
    np.testing.assert_allclose(v[:, 1], 2 * x, atol=1e-11)
    np.testing.assert_allclose(v[:, 2], 2 * z, atol=1e-11)
    np.testing.assert_allclose(v[:, 3], 2 * y - 2 * z, atol=1e-11)
    np.testing.assert_allclose(v[:, 4:], np.tile([2, 0, 0, 0, 2, -2], (60, 1)), atol=1e-9)


def _packet_1d(y0, s, kappa, q, p, eps):
    """int exp(-(y-y0)^2/(2 s^2) + i kappa y) exp(-ip(y-q)/eps - (y-q)^2/(2 eps)) dy."""
    a1, a2 = 1 / (2 * s * s), 1 / (2 * eps)
    al = a1 + a2
    yb = (a1 * y0 + a2 * q) / al
    kp = kappa - p / eps
    return (math.sqrt(math.pi / al) * np.exp(-(a1 * a2 / al) * (y0 - q) ** 2 + 1j * kp * yb
                                              - kp ** 2 / (4 * al)) * np.exp(1j * p * q / eps))


def test_fbi_gaussian_packet_closed_form():
    """psi of f = exp(-|y-y0|^2/(2 s^2) + i kappa.y) (real and imaginary parts
    taken as two real inputs) is the product of three one-dimensional closed
    forms, when the grid holds the packet and the window."""
    g = i3.Grid3(40, 40, 40, 0, 0, 0, 1 / 40, 1 / 40, 1 / 40)
    eps = 1 / 160
    y0, s, kap = (0.5, 0.48, 0.52), 0.08, (30.0, -20.0, 10.0)
    x = g.coords()
    E = [np.exp(-(x[a] - y0[a]) ** 2 / (2 * s * s) + 1j * kap[a] * x[a]) for a in range(3)]
    f = E[2][:, None, None] * E[1][None, :, None] * E[0][None, None, :]
    p = i3.Params3(eps, (17, 18, 19), (2, 2, 2), (3, 3, 3), (4, 4, 4), (0.1, 0.15, 0.2), 0.0,
                   1e-16, 1e-16, 1e-3, 0)
    psi = o3.fbi(f.real, g, p) + 1j * o3.fbi(f.imag, g, p)
    qs = o3.qnodes(p)
    pm = [o3.pmesh(p.np[a], p.dp[a]) for a in range(3)]
    for jq in range(27):
        j = (jq % 3, (jq // 3) % 3, jq // 9)
        q = [g.o[a] + g.d[a] * qs[a][j[a]] for a in range(3)]
        for lp in range(64):
            l = (lp % 4, (lp // 4) % 4, lp // 16)
            ref = np.prod([_packet_1d(y0[a], s, kap[a], q[a], pm[a][l[a]], eps) for a in range(3)])
            assert abs(psi[jq, lp] - ref) <= 1e-10 * abs(np.prod([math.sqrt(math.pi * 2 * eps)] * 3))


def _beams(q, p, sig):
    nb = len(q)
    st = np.zeros((nb, o3.NST3))
    st[:, 0:3] = q
    st[:, 3:6] = p
    for j in range(3):
        st[:, 7 + 2 * (3 * j + j)] = 1.0
        st[:, 26 + 2 * (3 * j + j)] = -1.0
    st[:, 43] = 2.0 ** 1.5
    return o3.Beams3(np.zeros(nb, np.int32), np.asarray(sig, np.int8), np.arange(nb),
                     np.ones(nb, complex), np.zeros((nb, 2)), st, np.array([0, nb]))


def _AB(st):
    A = (st[:, 7:25:2] + 1j * st[:, 8:25:2]).reshape(-1, 3, 3)
    B = (st[:, 25:43:2] + 1j * st[:, 26:43:2]).reshape(-1, 3, 3)
    return A, B


def test_constant_velocity_rays_closed_form():
    """c = c0: Q = q + sigma c0 t p/|p|, P = p, S = 0, B = -iI,
    A = I - i sigma (c0 t/|p|)(I - p p^T/|p|^2), and
    a = (det Z)^{1/2} = sqrt(2) (2 - i sigma c0 t/|p|)."""
    g = _grid()
    c0 = 1.6
    c = np.full(g.shape, c0)
    r = np.random.default_rng(2)
    nb = 30
    q = np.stack([g.o[a] + g.d[a] * r.uniform(5, g.n[a] - 6, nb) for a in range(3)], 1)
    p = r.uniform(-2, 2, (nb, 3))
    sig = np.where(np.arange(nb) % 2 == 0, 1, -1)
    b = _beams(q, p, sig)
    T, nst = 0.1, 100
    o3.propagate(b, c, g, T / nst, nst)
    st = b.state
    pn = np.linalg.norm(p, axis=1)
    ph = p / pn[:, None]
    np.testing.assert_allclose(st[:, 0:3], q + (sig * c0 * T)[:, None] * ph, atol=1e-13)
    np.testing.assert_allclose(st[:, 3:6], p, atol=1e-13)
    np.testing.assert_allclose(st[:, 6], 0.0, atol=1e-13)
    A, B = _AB(st)
    Pi = np.eye(3)[None] - ph[:, :, None] * ph[:, None, :]
    np.testing.assert_allclose(A, np.eye(3)[None] - 1j * (sig * c0 * T / pn)[:, None, None] * Pi,
                               atol=1e-12)
    np.testing.assert_allclose(B, -1j * np.eye(3)[None].repeat(nb, 0), atol=1e-13)
    a = st[:, 43] + 1j * st[:, 44]
    np.testing.assert_allclose(a, math.sqrt(2) * (2 - 1j * sig * c0 * T / pn), atol=1e-10)


def _smooth(nb=16, seed=5):
    g = i3.Grid3(28, 28, 28, 0, 0, 0, 1 / 28, 1 / 28, 1 / 28)
    c = i3.smooth_layered_velocity3(g, seed, 3.0)
    r = np.random.default_rng(seed)
    q = r.uniform(0.4, 0.6, (nb, 3))
    d = r.standard_normal((nb, 3))
    p = d / np.linalg.norm(d, axis=1)[:, None] * r.uniform(0.5, 2.0, nb)[:, None]
    sig = np.where(r.uniform(size=nb) < 0.5, 1, -1)
    return g, c, q, p, sig


def test_invariants_in_heterogeneous_medium():
    """H = sigma c(Q)|P| conserved, S = 0, the flow Jacobian
    M = [[Re A, Re B], [-Im A, -Im B]] symplectic, and a^2/(c(Q)^2 det Z)
    conserved (= 1/c(q)^2 from a(0) = 2^{3/2}, Z(0) = 2I)."""
    g, c, q, p, sig = _smooth()
    b = _beams(q, p, sig)
    o3.propagate(b, c, g, 1e-3, 150)
    st = b.state
    cq = o3.velocity(c, g, q)[:, 0]
    cQ = o3.velocity(c, g, st[:, 0:3])[:, 0]
    H0 = cq * np.linalg.norm(p, axis=1)
    H1 = cQ * np.linalg.norm(st[:, 3:6], axis=1)
    np.testing.assert_allclose(H1, H0, rtol=1e-8)   # RK4 level (dt = 1e-3, 150 steps)
    assert np.abs(st[:, 6]).max() < 1e-14
    A, B = _AB(st)
    J = np.block([[np.zeros((3, 3)), np.eye(3)], [-np.eye(3), np.zeros((3, 3))]])
    for i in range(len(q)):
        M = np.block([[A[i].real, B[i].real], [-A[i].imag, -B[i].imag]])
        np.testing.assert_allclose(M @ J @ M.T, J, atol=1e-8)
    Z = A + 1j * B
    a = st[:, 43] + 1j * st[:, 44]
    np.testing.assert_allclose(a ** 2 / (cQ ** 2 * np.linalg.det(Z)), 1 / cq ** 2, rtol=1e-7)


def test_rk4_fourth_order():
    """On a quadratic field (reproduced by the B-spline, so the right-hand
    side is smooth; rays kept inside) halving dt divides the error by ~16."""
    g, _, q, p, sig = _smooth(nb=6, seed=6)
    x1, x2, x3 = g.coords()
    c = (1.5 + 0.8 * (x1[None, None, :] - 0.3) ** 2 + 0.5 * (x2[None, :, None] - 0.6) ** 2
         + 0.3 * (x3[:, None, None] - 0.5) ** 2 + 0.4 * x1[None, None, :] * x2[None, :, None])
    c = np.ascontiguousarray(c)
    res = []
    for nst in (12, 24, 48):
        b = _beams(q, p, sig)
        o3.propagate(b, c, g, 0.12 / nst, nst)
        res.append(b.state.copy())
    assert np.abs(res[2][:, 0:3] - 0.5).max() < 0.4
    e1 = np.abs(res[0] - res[2]).max()
    e2 = np.abs(res[1] - res[2]).max()
    assert 10 < e1 / e2 < 22, (e1, e2)


def test_frame_identity_at_t0():
    """With no propagation the two branches of f0 (f1 = 0) rebuild f0: the
    sum over q on every node and a p-mesh covering the Nyquist band is the
    FBI frame identity, so a wrong normalisation (2 pi eps)^{3d/2} or
    amplitude 2^{d/2} shows as an O(1) error (measured 0.8 %: the smooth
    packet on a 10^3 grid)."""
    n, d = 10, 1 / 16
    g = i3.Grid3(n, n, n, 0, 0, 0, d, d, d)
    eps = 2.0 * d * d
    x1, x2, x3 = g.coords()
    cen = np.array(g.n) * d / 2 - d / 2
    r2 = ((x1[None, None, :] - cen[0]) ** 2 + (x2[None, :, None] - cen[1]) ** 2
          + (x3[:, None, None] - cen[2]) ** 2)
    f0 = np.exp(-r2 / (2 * (1.5 * d) ** 2))
    dp = 2 * math.pi * eps / d / n
    p = i3.Params3(eps, (0, 0, 0), (1, 1, 1), (n, n, n), (n, n, n), (dp, dp, dp), 1e-5, 1e-16,
                   1e-16, 1e-3, 0)
    b = o3.decompose(f0[None], None, np.ones(g.shape), g, p)
    u = o3.reconstruct(b, g, p)
    assert np.linalg.norm(u - f0) / np.linalg.norm(f0) < 0.02


def test_windowed_sum_against_brute_force():
    """The box sum equals the full sum over every node to the window level,
    for propagated beams."""
    g, c, q, p, sig = _smooth(nb=5, seed=8)
    b = _beams(q, p, sig)
    b.coef[:] = np.random.default_rng(3).standard_normal((5, 2))
    o3.propagate(b, c, g, 1e-3, 40)
    pr = i3.Params3(1 / 80, (0,) * 3, (1,) * 3, (1,) * 3, (2,) * 3, (1.0,) * 3, 0.0, 1e-16, 1e-12,
                    1e-3, 0)
    u = o3.reconstruct(b, g, pr)
    x1, x2, x3 = g.coords()
    ref = np.zeros(g.shape)
    for i in range(5):
        st = b.state[i]
        r = [x1[None, None, :] - st[0], x2[None, :, None] - st[1], x3[:, None, None] - st[2]]
        ph = (st[6] + st[3] * r[0] + st[4] * r[1] + st[5] * r[2]) / pr.eps
        ga = -(r[0] ** 2 + r[1] ** 2 + r[2] ** 2) / (2 * pr.eps)
        Ca = (b.coef[i, 0] + 1j * b.coef[i, 1]) * (st[43] + 1j * st[44])
        ref += (Ca * np.exp(1j * ph + ga)).real
    bound = 1e-12 * np.abs((b.coef[:, 0] + 1j * b.coef[:, 1]) * (b.state[:, 43] + 1j * b.state[:, 44])).sum()
    assert np.abs(u - ref).max() <= bound + 1e-13 * np.abs(ref).max()


# --------------------------------------------- decomposition with f1, frame

def _small_case(seed=12):
    g = i3.Grid3(9, 8, 7, 0.0, 0.1, -0.05, 1 / 9, 1 / 8, 1 / 7)
    r = np.random.default_rng(seed)
    x1, x2, x3 = g.coords()
    env = np.exp(-((x1[None, None, :] - 0.45) ** 2 + (x2[None, :, None] - 0.55) ** 2
                   + (x3[:, None, None] - 0.4) ** 2) / (2 * 0.15 ** 2))
    f0 = env * r.standard_normal(g.shape)
    f1 = 0.8 * env * r.standard_normal(g.shape)
    c = 1.0 + 0.6 * r.uniform(size=g.shape)
    p = i3.Params3(1 / 60, (1, 0, 1), (3, 2, 2), (3, 4, 3), (4, 6, 4), (0.3, 0.25, 0.35),
                   0.05, 1e-16, 1e-16, 1e-3, 0)
    return g, p, c, f0, f1


def _brute_psi3(f, g, p):
    """psi [Nq][Np] (axis 1 fastest) by the unwindowed sum over every node."""
    x = g.coords()
    qn = [g.o[a] + g.d[a] * (p.qb[a] + p.qs[a] * np.arange(p.nq[a])) for a in range(3)]
    pm = [o3.pmesh(p.np[a], p.dp[a]) for a in range(3)]
    out = np.zeros((p.nq[2], p.nq[1], p.nq[0], p.np[2], p.np[1], p.np[0]), complex)
    for j3, q3 in enumerate(qn[2]):
        for j2, q2 in enumerate(qn[1]):
            for j1, q1 in enumerate(qn[0]):
                r = [x[0] - q1, x[1] - q2, x[2] - q3]
                gw = f * np.exp(-(r[0][None, None, :] ** 2 + r[1][None, :, None] ** 2
                                  + r[2][:, None, None] ** 2) / (2 * p.eps))
                e = [np.exp(-1j * pm[a][:, None] * r[a][None, :] / p.eps) for a in range(3)]
                # sum_{x3,x2,x1} gw[x3,x2,x1] e3[l3,x3] e2[l2,x2] e1[l1,x1]
                t = np.tensordot(gw, e[0], axes=([2], [1]))        # [x3][x2][l1]
                t = np.tensordot(t, e[1], axes=([1], [1]))         # [x3][l1][l2]
                t = np.tensordot(t, e[2], axes=([0], [1]))         # [l1][l2][l3]
                out[j3, j2, j1] = np.prod(g.d) * t.transpose(2, 1, 0)
    return out.reshape(int(np.prod(p.nq)), int(np.prod(p.np)))


def test_threshold_set_brute_force_with_f1():
    """The kept (branch, q, p), their order and psi_+- = (psi0 +- i eps/(c(q)|p|)
    psi1)/2 (u_{+-,0} with c(q) the interpolant at the q node) against psi0,
    psi1 from the unwindowed sum over every node and the rule written out per
    candidate; a wrong q or p index in the f1 term, a sign or a missing
    factor changes the kept set or the values."""
    g, p, c, f0, f1 = _small_case()
    b = o3.decompose(f0[None], f1[None], c, g, p)
    psi0 = _brute_psi3(f0, g, p)
    psi1 = _brute_psi3(f1, g, p)
    NQ, NP = psi0.shape
    qn = [g.o[a] + g.d[a] * (p.qb[a] + p.qs[a] * np.arange(p.nq[a])) for a in range(3)]
    pm = [o3.pmesh(p.np[a], p.dp[a]) for a in range(3)]
    vals, ids = [], []
    for br, sg in ((0, 1.0), (1, -1.0)):
        for qf in range(NQ):
            j1, j2, j3 = qf % p.nq[0], (qf // p.nq[0]) % p.nq[1], qf // (p.nq[0] * p.nq[1])
            cq = o3.velocity(c, g, np.array([[qn[0][j1], qn[1][j2], qn[2][j3]]]))[0, 0]
            for pf in range(NP):
                l1, l2, l3 = pf % p.np[0], (pf // p.np[0]) % p.np[1], pf // (p.np[0] * p.np[1])
                pa = math.sqrt(pm[0][l1] ** 2 + pm[1][l2] ** 2 + pm[2][l3] ** 2)
                vals.append(0.5 * (psi0[qf, pf] + sg * 1j * p.eps / (cq * pa) * psi1[qf, pf]))
                ids.append((br * NQ + qf) * NP + pf)
    vals = np.array(vals)
    M = np.abs(vals).max()
    keep = np.abs(vals) >= p.tau * M
    assert 50 < keep.sum() < 0.7 * keep.size
    np.testing.assert_array_equal(b.cand, np.array(ids)[keep])
    np.testing.assert_allclose(b.psi, vals[keep], rtol=0, atol=1e-12 * M)
    np.testing.assert_array_equal(b.sigma, np.where(np.array(ids)[keep] < NQ * NP, 1, -1))


def test_branch_symmetry_with_f1():
    """For real f0, f1 the FBI satisfies psi_j(q, -p) = conj psi_j(q, p), so
    psi_+(q, -p) = conj psi_-(q, p) for every q, p (with f1 != 0: the sign of
    the i eps/(c(q)|p|) f1 term differs between the branches)."""
    g, p, c, f0, f1 = _small_case(seed=13)
    p = p.replace(tau=0.0)
    f1 = 30.0 * f1          # eps/(c|p|) ~ 0.03: make the f1 term comparable
    b = o3.decompose(f0[None], f1[None], c, g, p)
    NQ, NP = int(np.prod(p.nq)), int(np.prod(p.np))
    assert b.n == 2 * NQ * NP
    psi = b.psi.reshape(2, NQ, p.np[2], p.np[1], p.np[0])
    plus, minus = psi[0], psi[1]
    # -p_l = p_{n-1-l} on the staggered symmetric mesh, per axis
    flipped = plus[:, ::-1, ::-1, ::-1]
    np.testing.assert_allclose(flipped, np.conj(minus), rtol=0,
                               atol=1e-13 * np.abs(psi).max())
    assert np.abs(plus - minus).max() > 0.1 * np.abs(psi).max()      # f1 matters


def test_one_way_data_selects_one_branch():
    """For a packet moving in +x1 in c = 1 (f1 = -i |xi| sgn(xi1) f0 in
    Fourier), psi_- vanishes where psi_+ carries the packet (p1 > 0) and the
    converse for p1 < 0: a sign or scale error in i eps/(c(q)|p|) f1 breaks
    the split."""
    n = 32
    g = i3.Grid3(n, n, n, 0, 0, 0, 1 / n, 1 / n, 1 / n)
    eps = 1 / 48
    x1, x2, x3 = g.coords()
    r2 = ((x1[None, None, :] - 0.5) ** 2 + (x2[None, :, None] - 0.5) ** 2
          + (x3[:, None, None] - 0.5) ** 2)
    f0 = np.exp(-r2 / (2 * 0.12 ** 2)) * np.cos(0.9 * x1[None, None, :] / eps)
    xi = [2 * np.pi * np.fft.fftfreq(n, d=1 / n) for _ in range(3)]
    K1 = xi[0][None, None, :]
    mag = np.sqrt(K1 ** 2 + xi[1][None, :, None] ** 2 + xi[2][:, None, None] ** 2)
    f1 = np.real(np.fft.ifftn(-1j * mag * np.sign(K1) * np.fft.fftn(f0)))
    p = i3.Params3(eps, (12, 12, 12), (4, 4, 4), (3, 3, 3), (8, 4, 4), (0.25, 0.25, 0.25),
                   0.0, 1e-16, 1e-16, 1e-3, 0)
    b = o3.decompose(f0[None], f1[None], np.ones(g.shape), g, p)
    NQ, NP = int(np.prod(p.nq)), int(np.prod(p.np))
    psi = b.psi.reshape(2, NQ, p.np[2], p.np[1], p.np[0])
    pos = o3.pmesh(p.np[0], p.dp[0]) > 0
    big = np.abs(psi).max()
    assert np.abs(psi[0][..., pos]).max() > 0.4 * big
    assert np.abs(psi[0][..., ~pos]).max() < 0.05 * big
    assert np.abs(psi[1][..., ~pos]).max() > 0.4 * big
    assert np.abs(psi[1][..., pos]).max() < 0.05 * big


def test_frame_identity_exact_on_dft_bins():
    """At t = 0 with the p-mesh on the DFT bins of at least n points per axis
    (dp_a = 2 pi eps/(Np_a d_a), Np_a >= n_a) the sum over p is exact
    orthogonality (no aliasing), so step 3 after step 1 returns
    u(x) = f0(x) S(x), S(x) = prod_a sum_{q_a} (dq_a/sqrt(pi eps))
    exp(-(x_a - q_a)^2/eps) over the q-mesh, for any f0 (here noise on the
    whole grid, strides (2, 1, 2), unequal spacings).  This fixes the phase
    space weight, (2 pi eps)^{3d/2}, a(0) = 2^{d/2} and the sum of the two
    branches exactly; S differs from 1 by the Poisson ripple of the q-mesh."""
    g = i3.Grid3(10, 9, 8, 0.0, 0.0, 0.0, 1 / 10, 1 / 9, 1 / 8)
    eps = 3 * g.d1 ** 2
    qs = (2, 1, 2)
    nq = tuple((g.n[a] + qs[a] - 1) // qs[a] for a in range(3))
    Np = (10, 10, 8)
    dp = tuple(2 * math.pi * eps / (Np[a] * g.d[a]) for a in range(3))
    p = i3.Params3(eps, (0, 0, 0), qs, nq, Np, dp, 0.0, 1e-16, 1e-16, 1e-3, 0)
    f0 = np.random.default_rng(21).standard_normal(g.shape)
    b = o3.decompose(f0[None], None, np.ones(g.shape), g, p)
    u = o3.reconstruct(b, g, p)
    x = g.coords()
    S = np.ones(g.shape)
    for a in range(3):
        qa = g.o[a] + g.d[a] * qs[a] * np.arange(nq[a])
        s = (qs[a] * g.d[a] / math.sqrt(math.pi * eps)
             * np.exp(-(x[a][:, None] - qa[None, :]) ** 2 / eps).sum(1))
        S = S * s.reshape([-1 if k == 2 - a else 1 for k in range(3)])
    np.testing.assert_allclose(u, f0 * S, rtol=0, atol=1e-12 * np.abs(f0).max())
    # the identity is not trivial: the stride-2 axes ripple at the Poisson level
    assert np.abs(S[2:-2, 2:-2, 2:-2] - 1).max() > 1e-3

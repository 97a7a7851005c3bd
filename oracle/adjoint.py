"""Gradient oracle of the receiver-trace forward (test infrastructure).

The forward of the three-step algorithm for receiver traces is written again
here in plain PyTorch CPU float64 operations, following the paper's
equations directly (the psi eq. as a windowed sum, u_{+-,0}, the
Hamiltonian H = sigma c(Q)|P|, the characteristic, dynamic ray tracing and
amplitude equations with Z^{-1} formed by a matrix inverse, classical RK4,
the recons eq. at the receivers).  Reverse-mode automatic differentiation of
that forward gives the exact gradient of

    J = 1/2 sum_{s,k,r} (traces[s,k,r] - data[s,k,r])^2

with respect to the velocity samples and f0 (and f1), with the thresholded
beam set taken from the C oracle and the truncation boxes held fixed.
This module shares no code with the HIP path; its forward is pinned to the
C oracle in tests/test_oracle_adjoint.py.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import qnodes, pmesh

DT = torch.float64


# ----------------------------------------------------- velocity interpolant

def _beta(s: torch.Tensor, d: int) -> torch.Tensor:
    """Uniform cubic B-spline beta3(s) and its derivatives of order d <= 2."""
    a = s.abs()
    sg = torch.where(s < 0, -torch.ones_like(s), torch.ones_like(s))
    b = 2.0 - a
    if d == 0:
        inner = 2.0 / 3.0 - a * a + 0.5 * a ** 3
        outer = b ** 3 / 6.0
    elif d == 1:
        inner = sg * (-2.0 * a + 1.5 * a * a)
        outer = -sg * 0.5 * b * b
    else:
        inner = -2.0 + 3.0 * a
        outer = b
    zero = torch.zeros_like(s)
    return torch.where(a < 1.0, inner, torch.where(a < 2.0, outer, zero))


def velocity(cgrid: torch.Tensor, grid, Q1: torch.Tensor, Q2: torch.Tensor):
    """c, (c1, c2), (c11, c12, c22) of the clamped cubic B-spline at (Q1, Q2),
    differentiable in the samples and in Q."""
    t1 = (Q1 - grid.o1) / grid.d1
    t2 = (Q2 - grid.o2) / grid.d2
    i1 = torch.floor(t1.detach()).long()
    i2 = torch.floor(t2.detach()).long()
    out = [torch.zeros_like(Q1) for _ in range(6)]
    orders = ((0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2))
    for k2 in range(-1, 3):
        for k1 in range(-1, 3):
            kk1 = i1 + k1
            kk2 = i2 + k2
            ck = cgrid[kk2.clamp(0, grid.n2 - 1), kk1.clamp(0, grid.n1 - 1)]
            s1 = t1 - kk1
            s2 = t2 - kk2
            for r, (a1, a2) in enumerate(orders):
                out[r] = out[r] + ck * (_beta(s1, a1) / grid.d1 ** a1) * (_beta(s2, a2) / grid.d2 ** a2)
    c, c1, c2, c11, c12, c22 = out
    return c, torch.stack([c1, c2], -1), torch.stack(
        [torch.stack([c11, c12], -1), torch.stack([c12, c22], -1)], -2)


# ------------------------------------------------------------- ray system

def rhs(cgrid, grid, sigma, Q, P, S, A, B, a):
    """Right-hand sides of the characteristic equations, the dynamic ray
    tracing equations (dzQ, dzP eqs.), the action and the amplitude equation
    (a_formu eq.) for H = sigma c(Q)|P|.  A, B: complex [nb, 2, 2] with
    (j, k) entry d/dz_j of component k."""
    c, g, K = velocity(cgrid, grid, Q[:, 0], Q[:, 1])
    n = torch.sqrt((P * P).sum(-1))
    u = P / n[:, None]
    H = sigma * c * n
    HP = (sigma * c)[:, None] * u
    HQ = (sigma * n)[:, None] * g
    eye = torch.eye(2, dtype=DT)
    HPP = (sigma * c / n)[:, None, None] * (eye - u[:, :, None] * u[:, None, :])
    HQQ = (sigma * n)[:, None, None] * K
    HQP = sigma[:, None, None] * g[:, :, None] * u[:, None, :]   # d2H/dQ_l dP_k
    HPQ = HQP.transpose(1, 2)                                   # d2H/dP_l dQ_k
    dQ = HP
    dP = -HQ
    dS = (P * HP).sum(-1) - H
    cz = lambda m: m.to(torch.complex128)  # noqa: E731
    dA = A @ cz(HQP) + B @ cz(HPP)
    dB = -(A @ cz(HQQ)) - B @ cz(HPQ)
    Z = A + 1j * B
    dZ = dA + 1j * dB
    tr = torch.diagonal(torch.linalg.inv(Z) @ dZ, dim1=-2, dim2=-1).sum(-1)
    da = a * ((HP * HQ).sum(-1) / H) + 0.5 * a * tr
    return dQ, dP, dS, dA, dB, da


def rk4_step(cgrid, grid, sigma, y, dt):
    def add(y, k, h):
        return tuple(yi + h * ki for yi, ki in zip(y, k))
    k1 = rhs(cgrid, grid, sigma, *y)
    k2 = rhs(cgrid, grid, sigma, *add(y, k1, 0.5 * dt))
    k3 = rhs(cgrid, grid, sigma, *add(y, k2, 0.5 * dt))
    k4 = rhs(cgrid, grid, sigma, *add(y, k3, dt))
    return tuple(yi + dt / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4)
                 for yi, a1, a2, a3, a4 in zip(y, k1, k2, k3, k4))


# ---------------------------------------------------------- decomposition

def psi_kept(f: torch.Tensor, grid, params, j1, j2, l1, l2) -> torch.Tensor:
    """psi(q, p) of the psi eq. (Riemann sum on the nodes, f = 0 outside the
    grid, box B_eps) for the listed (q, p) only, differentiable in f."""
    R1 = math.ceil(math.sqrt(2 * params.eps * math.log(1 / params.tau_fbi)) / grid.d1)
    R2 = math.ceil(math.sqrt(2 * params.eps * math.log(1 / params.tau_fbi)) / grid.d2)
    k1, k2 = qnodes(params)
    p1 = torch.as_tensor(pmesh(params.np1, params.dp1)[l1], dtype=DT)
    p2 = torch.as_tensor(pmesh(params.np2, params.dp2)[l2], dtype=DT)
    kk1 = torch.as_tensor(k1[j1])
    kk2 = torch.as_tensor(k2[j2])
    m1 = torch.arange(-R1, R1 + 1)
    m2 = torch.arange(-R2, R2 + 1)
    y1 = kk1[:, None] + m1[None, :]                     # [nb, W1]
    y2 = kk2[:, None] + m2[None, :]                     # [nb, W2]
    in1 = (y1 >= 0) & (y1 < grid.n1)
    in2 = (y2 >= 0) & (y2 < grid.n2)
    vals = f[y2.clamp(0, grid.n2 - 1)[:, :, None], y1.clamp(0, grid.n1 - 1)[:, None, :]]
    vals = vals * (in2[:, :, None] & in1[:, None, :]).to(DT)     # [nb, W2, W1]
    r1 = (m1 * grid.d1).to(DT)
    r2 = (m2 * grid.d2).to(DT)
    w = torch.exp(-(r2[:, None] ** 2 + r1[None, :] ** 2) / (2 * params.eps))
    phase = (p1[:, None, None] * r1[None, None, :] + p2[:, None, None] * r2[None, :, None]) / params.eps
    kern = w[None] * torch.exp(-1j * phase)
    return grid.d1 * grid.d2 * (vals.to(torch.complex128) * kern).sum((-1, -2))


def decode(cand, params):
    nq = params.nq1 * params.nq2
    npp = params.np1 * params.np2
    shot = cand // (2 * nq * npp)
    rem = cand % (2 * nq * npp)
    sb = rem // (nq * npp)
    rem = rem % (nq * npp)
    qf, pf = rem // npp, rem % npp
    return shot, sb, qf % params.nq1, qf // params.nq1, pf % params.np1, pf // params.np1


# ------------------------------------------------------------------ traces

def traces(cgrid, f0, f1, grid, params, cand, receivers, rec_every, nrec, nshots):
    """Receiver traces [nshots][nrec][len(receivers)] of the beams `cand`
    (the candidate ids kept by the decomposition), differentiable in cgrid,
    f0 and f1."""
    shot, sb, j1, j2, l1, l2 = decode(np.asarray(cand), params)
    sigma = torch.as_tensor(np.where(sb == 0, 1.0, -1.0), dtype=DT)
    k1, k2 = qnodes(params)
    pm1, pm2 = pmesh(params.np1, params.dp1), pmesh(params.np2, params.dp2)
    q = torch.as_tensor(np.stack([grid.o1 + grid.d1 * k1[j1], grid.o2 + grid.d2 * k2[j2]], 1),
                        dtype=DT)
    p = torch.as_tensor(np.stack([pm1[l1], pm2[l2]], 1), dtype=DT)
    psi0 = torch.zeros(len(cand), dtype=torch.complex128)
    psi1 = torch.zeros(len(cand), dtype=torch.complex128)
    for s in range(nshots):
        m = shot == s
        if m.any():
            idx = torch.as_tensor(np.nonzero(m)[0])
            psi0 = psi0.index_put((idx,), psi_kept(f0[s], grid, params, j1[m], j2[m], l1[m], l2[m]))
            if f1 is not None:
                psi1 = psi1.index_put((idx,), psi_kept(f1[s], grid, params, j1[m], j2[m], l1[m], l2[m]))
    if f1 is not None:
        cq, _, _ = velocity(cgrid, grid, q[:, 0], q[:, 1])
        r = params.eps / (cq * torch.sqrt((p * p).sum(-1)))
        psi = 0.5 * (psi0 + sigma * 1j * r * psi1)
    else:
        psi = 0.5 * psi0
    w = (params.qs1 * grid.d1) * (params.qs2 * grid.d2) * params.dp1 * params.dp2
    C = w * psi / (2 * math.pi * params.eps) ** 3
    nb = len(cand)
    eye = torch.eye(2, dtype=torch.complex128).expand(nb, 2, 2)
    y = (q.clone(), p.clone(), torch.zeros(nb, dtype=DT), eye.clone(), -1j * eye,
         torch.full((nb,), 2.0, dtype=torch.complex128))
    shot_t = torch.as_tensor(shot)
    out = []
    for k in range(nrec):
        for _ in range(rec_every):
            y = rk4_step(cgrid, grid, sigma, y, params.dt)
        Q, P, S, _, _, a = y
        out.append(recons_at(Q, P, S, C * a, shot_t, receivers, grid, params, nshots))
    return torch.stack(out, 1)


def recons_at(Q, P, S, Ca, shot_t, nodes, grid, params, nshots):
    """The recons eq. at the listed nodes (flat i2*n1 + i1): [nshots][len(nodes)],
    each beam summed over the box of half-width Rw around the node nearest Q
    (the boxes come from the detached centres: held fixed, no gradient).
    Q, P: [nb][2]; S: [nb]; Ca: [nb] complex (C a)."""
    rec = np.asarray(nodes)
    xr = torch.as_tensor(np.stack([grid.o1 + grid.d1 * (rec % grid.n1),
                                   grid.o2 + grid.d2 * (rec // grid.n1)], 1), dtype=DT)
    ri1 = torch.as_tensor(rec % grid.n1)
    ri2 = torch.as_tensor(rec // grid.n1)
    Rw1 = math.ceil(math.sqrt(2 * params.eps * math.log(1 / params.tau_win)) / grid.d1)
    Rw2 = math.ceil(math.sqrt(2 * params.eps * math.log(1 / params.tau_win)) / grid.d2)
    c1 = torch.floor((Q[:, 0].detach() - grid.o1) / grid.d1 + 0.5).long()
    c2 = torch.floor((Q[:, 1].detach() - grid.o2) / grid.d2 + 0.5).long()
    inbox = ((ri1[None, :] >= (c1 - Rw1).clamp(min=0)[:, None])
             & (ri1[None, :] <= (c1 + Rw1).clamp(max=grid.n1 - 1)[:, None])
             & (ri2[None, :] >= (c2 - Rw2).clamp(min=0)[:, None])
             & (ri2[None, :] <= (c2 + Rw2).clamp(max=grid.n2 - 1)[:, None]))
    rx = xr[None, :, :] - Q[:, None, :]                          # [nb, nnodes, 2]
    phase = (S[:, None] + (P[:, None, :] * rx).sum(-1)) / params.eps
    gauss = -(rx * rx).sum(-1) / (2 * params.eps)
    term = Ca[:, None] * torch.exp(1j * phase + gauss)
    term = torch.where(inbox, term.real, torch.zeros_like(term.real))
    return torch.zeros((nshots, len(rec)), dtype=DT).index_add(0, shot_t, term)


def recons_vjp(state, coef, shot, grid, params, nshots, du):
    """Reverse-mode derivative of the field reconstruction (recons eq. on
    the whole grid, boxes held fixed) for J = sum du * u: returns
    (dstate [nb][23], dcoef [nb][2]) with the cotangents of Q, P, S and
    (Re a, Im a) in the state layout (zero for dzQ, dzP, which u does not
    read) and of (Re C, Im C).  state: [nb][23]; coef: [nb][2];
    du: [nshots][n2][n1]."""
    st = torch.tensor(np.asarray(state)[:, [0, 1, 2, 3, 4, 21, 22]], dtype=DT, requires_grad=True)
    cf = torch.tensor(np.asarray(coef), dtype=DT, requires_grad=True)
    Q, P, S = st[:, 0:2], st[:, 2:4], st[:, 4]
    a = torch.complex(st[:, 5], st[:, 6])
    C = torch.complex(cf[:, 0], cf[:, 1])
    nodes = np.arange(grid.n1 * grid.n2)
    u = recons_at(Q, P, S, C * a, torch.as_tensor(np.asarray(shot, dtype=np.int64)), nodes,
                  grid, params, nshots)
    J = (u * torch.as_tensor(np.asarray(du), dtype=DT).reshape(nshots, -1)).sum()
    gs, gc = torch.autograd.grad(J, [st, cf])
    ds = np.zeros((len(coef), 23))
    ds[:, [0, 1, 2, 3, 4, 21, 22]] = gs.numpy()
    return ds, gc.numpy()


def gradient(c, f0, f1, grid, params, cand, receivers, rec_every, nrec, data):
    """(J, dJ/dc, dJ/df0, dJ/df1 or None) as numpy arrays."""
    cg = torch.tensor(c, dtype=DT, requires_grad=True)
    f0t = torch.tensor(f0, dtype=DT, requires_grad=True)
    f1t = None if f1 is None else torch.tensor(f1, dtype=DT, requires_grad=True)
    tr = traces(cg, f0t, f1t, grid, params, cand, receivers, rec_every, nrec, f0.shape[0])
    J = 0.5 * ((tr - torch.as_tensor(data, dtype=DT)) ** 2).sum()
    wrt = [cg, f0t] + ([f1t] if f1t is not None else [])
    gr = torch.autograd.grad(J, wrt)
    return (float(J.detach()), gr[0].numpy(), gr[1].numpy(),
            None if f1t is None else gr[2].numpy(), tr.detach().numpy())

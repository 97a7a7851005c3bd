#!/usr/bin/env python
"""Benchmark of the MI355X frozen Gaussian approximation path.

One step = the whole hot path on one batch of synthetic input already in
HBM: decomposition (FBI + branch split + threshold + compaction), RK4
propagation of every beam to T = 0.25 s (250 steps) and reconstruction of
u(T) on the grid.  Workload: 512 x 512 smooth layered model on [0,2]x[0,1],
eps = 1/256, point source (sigma = 2 cells), q-mesh 40 x 20, p-mesh
112 x 112, tau = 1e-6, mixed precision (FP32 FBI and splat with the phase
reduced in FP64, FP64 rays and amplitudes).

Prints ONE JSON line: beams/s end-to-end, the per-stage times, the error of
the mixed path against the FP64 path (and against stored oracle values at
sampled nodes), the roofline of the dominant kernel and the oracle timed on
the host cores on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import fga_inputs as fi  # noqa: E402

PEAK = {"hbm": 8.0e12, "fp64": 78.6e12, "fp32": 157.3e12}

# FP64 operations of one RK4 step of one beam (4 right-hand sides + the RK4
# combinations), counted from the formulas the kernel implements: B-spline
# weights (2 x 26), 16 taps x 6 products (96 FMA = 192), scalings 8, |P| and
# u (sqrt ~ 1 + div ~ 1 + 3), H derivatives 8, dS 4, dzQ update 2 x (2 x 8 +
# 2 x 12) = 80, dzP update 2 x (2 x 8 + 2 x 8) = 64, Z/dZ 16, det 8, adjugate
# trace 32, 1/|det|^2 and the quotient 12, da 12: ~493 per evaluation; RK4
# combinations 4 x 2 x 23 FMA = 368 per step.
RK4_FLOP_PER_BEAM_STEP = 4 * 493 + 368


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="point512")
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="timed steps of the FP64 GPU path on the same input")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="rough budget of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device copy first (HBM counter calibration)")
    return ap.parse_args()


class Path:
    """One precision of the HIP path with its buffers."""

    def __init__(self, W, precision, capacity):
        import torch
        import paper_1304_3542_amd as fga
        self.fga = fga
        self.W = W
        self.ctx = fga.FGA(W.grid, W.params, precision, max_shots=W.nshots)
        self.c = torch.from_numpy(W.c).cuda()
        self.f0 = torch.from_numpy(np.ascontiguousarray(W.f0)).cuda()
        self.f1 = None if W.f1 is None else torch.from_numpy(np.ascontiguousarray(W.f1)).cuda()
        self.ctx.set_velocity(self.c)
        self.beams = fga.Beams(capacity, W.nshots)
        self.u = torch.empty((W.nshots, W.grid.n2, W.grid.n1), dtype=torch.float64,
                             device="cuda")

    def fit_capacity(self):
        """Run one decomposition; grow the beam buffer if it overflowed."""
        self.ctx.decompose(self.f0, self.f1, self.beams)
        st, need = self.ctx.status()
        if st == self.fga.FGA_ECAPACITY:
            self.beams = self.fga.Beams(int(need * 1.05) + 1024, self.W.nshots)
            self.ctx.decompose(self.f0, self.f1, self.beams)
            st, need = self.ctx.status()
        if st != self.fga.FGA_OK:
            raise RuntimeError(f"decompose status {st}: {self.fga.fga_last_error(self.ctx.ctx)}")
        return int(self.ctx.offsets(self.beams, self.W.nshots)[-1])

    def step(self, ev=None):
        ns = self.W.nshots
        if ev:
            ev[0].record()
        self.ctx.decompose(self.f0, self.f1, self.beams)
        if ev:
            ev[1].record()
        self.ctx.propagate(self.beams, ns, self.W.params.nsteps)
        if ev:
            ev[2].record()
        self.ctx.reconstruct(self.beams, ns, self.u)
        if ev:
            ev[3].record()


def time_path(path, steps, warmup):
    import torch
    for _ in range(warmup):
        path.step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        path.step(evs[k])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    st = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(3)] for e in evs])
    return wall * 1e3, st.mean(axis=0)


def box_pairs(f, nb, W, tau_win):
    """Number of (beam, node) pairs the windowed sum visits."""
    g, p = W.grid, W.params
    Q1, Q2 = f[6, :nb], f[7, :nb]
    R1 = math.ceil(math.sqrt(2 * p.eps * math.log(1 / tau_win)) / g.d1)
    R2 = math.ceil(math.sqrt(2 * p.eps * math.log(1 / tau_win)) / g.d2)
    c1 = np.floor((Q1 - g.o1) / g.d1 + 0.5)
    c2 = np.floor((Q2 - g.o2) / g.d2 + 0.5)
    w1 = np.clip(np.minimum(c1 + R1, g.n1 - 1) - np.maximum(c1 - R1, 0) + 1, 0, None)
    w2 = np.clip(np.minimum(c2 + R2, g.n2 - 1) - np.maximum(c2 - R2, 0) + 1, 0, None)
    return float((w1 * w2).sum())


def cpu_baseline(W, nbeams, budget_s):
    """The oracle on a bounded sample of the same workload, scaled to the
    whole job: FBI on a few q nodes, RK4 and the windowed sum for a few
    hundred beams."""
    import oracle
    g, p = W.grid, W.params
    nq = p.nq1 * p.nq2
    # FBI on a handful of q nodes around the source
    qs = p.replace(qb1=p.qb1 + p.qs1 * (p.nq1 // 2), qb2=p.qb2 + p.qs2 * (p.nq2 // 2),
                   nq1=2, nq2=1)
    t = time.perf_counter()
    psi = oracle.fbi(W.f0[0], g, qs)
    t_fbi = (time.perf_counter() - t) / 2 * nq
    # beams: the largest |psi| of the sampled q nodes, both branches
    nsb = 1024
    order = np.argsort(-np.abs(psi.ravel()))[:nsb // 2]
    j2, j1, l2, l1 = np.unravel_index(order, psi.shape)
    k1, k2 = oracle.qnodes(qs)
    pm1, pm2 = oracle.pmesh(p.np1, p.dp1), oracle.pmesh(p.np2, p.dp2)
    st = np.zeros((nsb, oracle.NSTATE))
    for h in range(2):
        sl = slice(h * (nsb // 2), (h + 1) * (nsb // 2))
        st[sl, 0] = g.o1 + g.d1 * k1[j1]
        st[sl, 1] = g.o2 + g.d2 * k2[j2]
        st[sl, 2] = pm1[l1]
        st[sl, 3] = pm2[l2]
    st[:, 5] = st[:, 11] = 1.0
    st[:, 14] = st[:, 20] = -1.0
    st[:, 21] = 2.0
    sig = np.repeat(np.array([1, -1], np.int8), nsb // 2)
    coef = np.tile(np.stack([psi.ravel()[order].real, psi.ravel()[order].imag], 1), (2, 1))
    b = oracle.Beams(np.zeros(nsb, np.int32), sig, np.arange(nsb, dtype=np.int64),
                     coef[:, 0] + 1j * coef[:, 1], np.ascontiguousarray(coef), st,
                     np.array([0, nsb], np.int64))
    t = time.perf_counter()
    oracle.propagate(b, W.c, g, p.dt, p.nsteps)
    t_rk4 = (time.perf_counter() - t) / nsb * nbeams
    t = time.perf_counter()
    oracle.reconstruct(b, g, p, shot=0)
    t_rec = (time.perf_counter() - t) / nsb * nbeams
    total = t_fbi + t_rk4 + t_rec
    return {
        "value": nbeams / total, "unit": "beams/s", "cores": oracle.threads(),
        "kind": "oracle",
        "sample": (f"FP64 oracle: FBI at 2 of {nq} q nodes, RK4 ({p.nsteps} steps) and the "
                   f"windowed sum for {nsb} beams, each scaled linearly to the {nbeams} "
                   f"beams / {nq} q nodes of the job"),
        "est_seconds": {"fbi": t_fbi, "rk4": t_rk4, "reconstruct": t_rec},
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)
    import torch
    if args.calib_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    W = fi.workload(args.workload, "mixed")
    Wd = fi.workload(args.workload, "fp64")
    cand = 2 * W.params.nq1 * W.params.nq2 * W.params.np1 * W.params.np2 * W.nshots

    mixed = Path(W, "mixed", min(cand, 4_000_000))
    nb = mixed.fit_capacity()
    ms_step, stage_ms = time_path(mixed, args.steps, args.warmup)
    u_mixed = mixed.u.cpu().numpy()
    f_host = mixed.beams.f[:, :nb].cpu().numpy()

    fp64 = Path(Wd, "fp64", min(cand, 4_000_000))
    nb64 = fp64.fit_capacity()
    ms64, stage64 = time_path(fp64, args.fp64_steps, 0)
    u64 = fp64.u.cpu().numpy()
    rel_vs_fp64 = float(np.linalg.norm(u_mixed - u64) / np.linalg.norm(u64))

    rel_oracle = None
    gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}_fp64.npz")
    if os.path.exists(gold) and W.nshots == 1:
        z = np.load(gold)
        ref = z["u"]
        rel_oracle = {
            "mixed": float(np.linalg.norm(u_mixed[0].ravel()[z["nodes"]] - ref) / np.linalg.norm(ref)),
            "fp64": float(np.linalg.norm(u64[0].ravel()[z["nodes"]] - ref) / np.linalg.norm(ref)),
            "nodes": int(z["nodes"].size),
        }

    pairs = box_pairs(f_host, nb, W, W.params.tau_win)
    npts = W.grid.n1 * W.grid.n2 * W.nshots
    stages = {"decompose": stage_ms[0], "propagate": stage_ms[1], "reconstruct": stage_ms[2]}
    dom = max(stages, key=stages.get)
    if dom == "propagate":
        fl = RK4_FLOP_PER_BEAM_STEP * W.params.nsteps * nb
        achieved = fl / (stage_ms[1] * 1e-3)
        roof = {"kernel": "k_rk4", "bound": "alu", "achieved": achieved / 1e12,
                "peak": PEAK["fp64"] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp64"], "traffic": None}
    elif dom == "reconstruct":
        fl = 4.0 * pairs
        achieved = fl / (stage_ms[2] * 1e-3)
        roof = {"kernel": "k_splat_mfma", "bound": "mfma", "achieved": achieved / 1e12,
                "peak": PEAK["fp32"] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp32"], "traffic": None}
    else:
        roof = {"kernel": "decompose", "bound": "alu", "achieved": None, "peak": None,
                "unit": "TFLOP/s", "frac": None, "traffic": None}

    out = {
        "metric": "beams/s end-to-end (FBI+trace+sum) at rel-L2<=1e-5 vs FP64",
        "value": nb / (ms_step * 1e-3),
        "unit": "beams/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: 512x512 smooth layered model, eps=1/256, "
                               f"point source, q 40x20, p 112x112, tau=1e-6, T=0.25 s, dt=1 ms, "
                               f"mixed precision", "nshots": W.nshots, "nbeams": nb},
        "valid": bool(rel_vs_fp64 <= 1e-5),
        "rel_l2_vs_fp64_gpu": rel_vs_fp64,
        "rel_l2_vs_oracle_sample": rel_oracle,
        "stages_ms": stages,
        "grid_points_per_s": npts / (ms_step * 1e-3),
        "pairs": pairs,
        "pairs_per_s": pairs / (stage_ms[2] * 1e-3),
        "fp64_gpu": {"ms_per_step": ms64, "nbeams": nb64,
                     "stages_ms": dict(zip(stages, stage64.tolist())),
                     "speedup_mixed_over_fp64": ms64 / ms_step},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(Wd, nb, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

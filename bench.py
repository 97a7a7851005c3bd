#!/usr/bin/env python
"""Benchmark of the MI355X frozen Gaussian approximation path.

One step = the whole hot path on one batch of synthetic input already in
HBM: decomposition (FBI + branch split + threshold + compaction), RK4
propagation of every beam to T = 0.25 s (250 steps) and reconstruction of
u(T) on the grid.  Headline workload (the largest single-GPU
configuration): 2048 x 1024 smooth layered model on [0,2]x[0,1],
eps = 1/1024, point source (sigma = 2 cells), q-mesh 147 x 74, p-mesh
400 x 400, tau = 1e-6, ~5e7 beams, mixed precision (FP32 FBI and splat with
the phase reduced in FP64, FP64 rays and amplitudes).  The 512 x 512
configuration (point512) and the other workloads follow as secondary keys.

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

PEAK = {"hbm": 8.0e12, "fp64": 78.6e12, "fp32": 157.3e12, "fp16": 2.5e15}

# FP64 operations (an FMA counts two) of one RK4 step of one beam, counted
# from the formulas the kernel evaluates per stage: cubic B-spline weights
# and 16-tap sums of c, grad c, Hess c (~196), |P| and u (~15), the
# Hamiltonian derivatives and Q/P/S slopes (~30), Z, det Z and the
# sign-folded coefficients (~36), the rank-one dzQ/dzP updates with the
# adjugate trace and the accumulator/stage updates of both rows (~200),
# 1/|det Z|^2, tr(Z^-1 dZ) and the amplitude slope and updates (~37):
# ~521 per stage, four stages less the last stage's unused input update.
RK4_FLOP_PER_BEAM_STEP = 2030
PROFILE_JSON = os.path.join(ROOT, "profiles", "{workload}_hbm_counters.json")
KERNEL_SOURCES = {
    "k_rk4": ["paper_1304_3542_amd/csrc/propagate.hip", "paper_1304_3542_amd/csrc/rk4.h",
              "paper_1304_3542_amd/csrc/fga_internal.h"],
    "k_splat_binned": ["paper_1304_3542_amd/csrc/binning.hip",
                       "paper_1304_3542_amd/csrc/reconstruct.hip",
                       "paper_1304_3542_amd/csrc/splat.h",
                       "paper_1304_3542_amd/csrc/fga_internal.h"],
}


KERNEL_SOURCES["k_splat_binned_split"] = KERNEL_SOURCES["k_splat_binned"]

# the name the profiler reports for the instance the timed path launches
PROFILED_NAME = {"k_rk4": "k_rk4<false, false>", "k_splat_binned": "k_splat_binned",
                 "k_splat_binned_split": "k_splat_binned_split"}


def profiled_traffic(kernel, workload):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE counter
    summary of the workload, or None if the kernel's sources changed since it
    was taken."""
    import hashlib
    path = PROFILE_JSON.format(workload=workload)
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    z = json.load(open(path))
    h = hashlib.sha256()
    for fn in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, fn), "rb").read())
    if z.get("source_sha", {}).get(kernel) != h.hexdigest()[:16]:
        return None
    k = z["kernels"].get(PROFILED_NAME[kernel])
    return None if k is None else k["hbm_bytes_scaled"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large2048",
                    help="headline workload (large2048: the largest single-GPU configuration)")
    ap.add_argument("--precision", default="mixed_split", choices=["mixed", "mixed_split"],
                    help="reduced-precision path of the headline (mixed_split: the splat's "
                         "products on the FP16 matrix cores from hi/lo splits)")
    ap.add_argument("--graph-steps", type=int, default=5,
                    help="timed replays of the headline step captured as one HIP graph")
    ap.add_argument("--point-steps", type=int, default=10,
                    help="timed steps of the 512x512 configuration (point512) as a secondary "
                         "key (0 skips it; ignored when it is the headline)")
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="timed steps of the FP64 GPU path on the same input (at least 1: "
                         "the mixed field is checked against it)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="rough budget of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=3,
                    help="timed graph replays of the 64-shot batch (0 skips it)")
    ap.add_argument("--closed-steps", type=int, default=5,
                    help="timed steps of point512 with the closed-form amplitude (0 skips it)")
    ap.add_argument("--dd-steps", type=int, default=3,
                    help="timed steps of point512 with divided-difference dzQ, dzP (0 skips it)")
    ap.add_argument("--d3-steps", type=int, default=2,
                    help="timed steps of the three-dimensional point3d workload (0 skips it)")
    ap.add_argument("--fwi-steps", type=int, default=3,
                    help="timed forward+adjoint iterations of the 64-shot workload (0 skips it)")
    ap.add_argument("--topn-steps", type=int, default=5,
                    help="timed steps of the N-largest selection workload (0 skips it)")
    ap.add_argument("--adjoint-steps", type=int, default=3,
                    help="timed iterations of the adjoint workload (0 skips it)")
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
    """Wall ms per step (host clock over all steps), mean per-stage ms and the
    per-step device times (HIP events from the first stage to the last)."""
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
    per_step = np.array([e[0].elapsed_time(e[3]) for e in evs])
    return wall * 1e3, st.mean(axis=0), per_step


def graph_replays(path, steps, nb):
    """The same step (decompose -> propagate -> reconstruct) captured once as
    a HIP graph and replayed: device ms per replay from HIP events on the
    context's stream, median and interquartile range."""
    import torch
    W = path.W
    fga = path.fga
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    fga.fga_set_stream(path.ctx.ctx, stream)
    with torch.cuda.stream(stream):
        path.ctx.graph_capture(path.f0, path.f1, path.beams, W.params.nsteps, path.u)
        path.ctx.graph_launch()
        stream.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        evs[0].record(stream)
        for k in range(steps):
            path.ctx.graph_launch()
            evs[k + 1].record(stream)
        stream.synchronize()
        st, _ = path.ctx.status()
    fga.fga_set_stream(path.ctx.ctx, torch.cuda.current_stream())
    ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(steps)])
    med = float(np.median(ms))
    return {"replays": steps, "ms_per_replay_median": med,
            "iqr": float(np.percentile(ms, 75) - np.percentile(ms, 25)),
            "beams_per_s": nb / (med * 1e-3), "status": st}


def time_splat_kernel(path, reps=3):
    """Duration of the reconstruction on its stream (HIP events): the
    record pre-pass, the binning, the MFMA splat and the tile reduction
    together."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ts = []
    for _ in range(reps):
        ev[0].record()
        path.ctx.reconstruct(path.beams, path.W.nshots, path.u)
        ev[1].record()
        torch.cuda.synchronize()
        ts.append(ev[0].elapsed_time(ev[1]))
    return float(np.median(ts))


def adjoint_iteration(steps):
    """ms per iteration of forward + adjoint on the 256 x 256, 8-shot receiver
    workload (FP64): decompose, trace with checkpoints, trace adjoint,
    decomposition adjoint."""
    import torch
    import paper_1304_3542_amd as fga
    W = fi.workload("adjoint256", "fp64")
    g, p = W.grid, W.params
    ns = W.nshots
    nrec_t = p.nsteps // W.rec_every
    ctx = fga.FGA(g, p, "fp64", max_shots=ns)
    c = torch.from_numpy(W.c).cuda()
    ctx.set_velocity(c)
    f0 = torch.from_numpy(np.ascontiguousarray(W.f0)).cuda()
    cap = 2 * p.nq1 * p.nq2 * p.np1 * p.np2 * ns
    beams = fga.Beams(cap, ns)
    ctx.decompose(f0, None, beams)
    nb = int(ctx.offsets(beams, ns)[-1])
    beams = fga.Beams(nb + 1024, ns)
    rec = torch.from_numpy(W.receivers).cuda()
    ckpt = torch.empty((nrec_t, fga.FGA_NSTATE, beams.capacity), dtype=torch.float64,
                       device="cuda")
    # data: traces of the perturbed model through the same path
    ctx.set_velocity(torch.from_numpy(W.c_true).cuda())
    ctx.decompose(f0, None, beams)
    data = ctx.trace(beams, ns, rec, W.rec_every, nrec_t)
    ctx.set_velocity(c)
    dc = torch.zeros_like(c)

    def it():
        ctx.decompose(f0, None, beams)
        tr = ctx.trace(beams, ns, rec, W.rec_every, nrec_t, ckpt)
        dc.zero_()
        gcoef = ctx.trace_adjoint(beams, ns, rec, W.rec_every, nrec_t, ckpt,
                                  (tr - data).contiguous(), dc)
        return ctx.decompose_adjoint(beams, ns, gcoef)

    it()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        it()
    ev[1].record()
    torch.cuda.synchronize()
    st, _ = ctx.status()
    ms_seg = ev[0].elapsed_time(ev[1]) / steps

    # the same iteration with the state of every step kept by the forward
    # (the adjoint reads it instead of recomputing each 10-step segment)
    ctx_e = fga.FGA(g, p.replace(ckpt_every_step=1), "fp64", max_shots=ns)
    ctx_e.set_velocity(c)
    ckpt_e = torch.empty((ctx_e.ckpt_rows(W.rec_every, nrec_t), fga.FGA_NSTATE, beams.capacity),
                         dtype=torch.float64, device="cuda")

    def it_every():
        ctx_e.decompose(f0, None, beams)
        tr = ctx_e.trace(beams, ns, rec, W.rec_every, nrec_t, ckpt_e)
        dc.zero_()
        gcoef = ctx_e.trace_adjoint(beams, ns, rec, W.rec_every, nrec_t, ckpt_e,
                                    (tr - data).contiguous(), dc)
        return ctx_e.decompose_adjoint(beams, ns, gcoef)

    it_every()
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(steps):
        it_every()
    ev[1].record()
    torch.cuda.synchronize()
    st_e, _ = ctx_e.status()
    ms_every = ev[0].elapsed_time(ev[1]) / steps
    ckpt_gb = ckpt_e.numel() * 8 / 1e9
    del ckpt_e
    ctx_e.close()
    out = {"ms_per_iter": ms_every, "nbeams": nb, "nshots": ns,
           "status": st if st != 0 else st_e,
           "checkpoints": f"every step ({ckpt_gb:.1f} GB; the adjoint reads the states)",
           "segment_checkpoints": {"ms_per_iter": ms_seg,
                                   "checkpoints": "every 10 steps (the adjoint recomputes)"},
           "workload": "adjoint256: 256x256 on [0,2]x[0,1], eps=1/128, 8 surface "
           "shots, 256 receivers on the top row every 10 steps, T=0.25 s, FP64 gradient "
           "w.r.t. c and f0"}

    # the same gradient for a misfit of the whole field u(T): reconstruction
    # and propagation transposed, 25 checkpoint segments of 10 steps
    u_data = torch.zeros((ns, g.n2, g.n1), dtype=torch.float64, device="cuda")
    ctx.set_velocity(torch.from_numpy(W.c_true).cuda())
    ctx.decompose(f0, None, beams)
    ctx.propagate(beams, ns, p.nsteps)
    ctx.reconstruct(beams, ns, u_data)
    ctx.set_velocity(c)
    u = torch.empty_like(u_data)

    def it_field():
        ctx.decompose(f0, None, beams)
        ctx.propagate_ckpt(beams, ns, W.rec_every, nrec_t, ckpt)
        ctx.reconstruct(beams, ns, u)
        dstate, dcoef = ctx.reconstruct_adjoint(beams, ns, (u - u_data).contiguous())
        dc.zero_()
        ctx.propagate_adjoint(beams, ns, W.rec_every, nrec_t, ckpt, dstate, dc)
        return ctx.decompose_adjoint(beams, ns, dcoef)

    it_field()
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(steps):
        it_field()
    ev[1].record()
    torch.cuda.synchronize()
    st, _ = ctx.status()
    ms_field_seg = ev[0].elapsed_time(ev[1]) / steps

    # and with every step's state kept by the forward
    ctx_f = fga.FGA(g, p.replace(ckpt_every_step=1), "fp64", max_shots=ns)
    ctx_f.set_velocity(c)
    ckpt_f = torch.empty((ctx_f.ckpt_rows(W.rec_every, nrec_t), fga.FGA_NSTATE, beams.capacity),
                         dtype=torch.float64, device="cuda")

    def it_field_every():
        ctx_f.decompose(f0, None, beams)
        ctx_f.propagate_ckpt(beams, ns, W.rec_every, nrec_t, ckpt_f)
        ctx_f.reconstruct(beams, ns, u)
        dstate, dcoef = ctx_f.reconstruct_adjoint(beams, ns, (u - u_data).contiguous())
        dc.zero_()
        ctx_f.propagate_adjoint(beams, ns, W.rec_every, nrec_t, ckpt_f, dstate, dc)
        return ctx_f.decompose_adjoint(beams, ns, dcoef)

    it_field_every()
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(steps):
        it_field_every()
    ev[1].record()
    torch.cuda.synchronize()
    st_f, _ = ctx_f.status()
    del ckpt_f
    ctx_f.close()
    out["field_misfit"] = {"ms_per_iter": ev[0].elapsed_time(ev[1]) / steps,
                           "status": st if st != 0 else st_f,
                           "checkpoints": "every step",
                           "segment_checkpoints_ms_per_iter": ms_field_seg,
                           "misfit": "1/2 |u(T) - u_data(T)|^2 over the grid"}

    # the receiver-misfit iteration in deterministic mode (fixed-order dJ/dc;
    # synchronises once per adjoint call)
    ctx_d = fga.FGA(g, p.replace(deterministic=1), "fp64", max_shots=ns)
    ctx_d.set_velocity(c)

    def it_det():
        ctx_d.decompose(f0, None, beams)
        tr = ctx_d.trace(beams, ns, rec, W.rec_every, nrec_t, ckpt)
        dc.zero_()
        gcoef = ctx_d.trace_adjoint(beams, ns, rec, W.rec_every, nrec_t, ckpt,
                                    (tr - data).contiguous(), dc)
        return ctx_d.decompose_adjoint(beams, ns, gcoef)

    it_det()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        it_det()
    torch.cuda.synchronize()
    st, _ = ctx_d.status()
    out["deterministic"] = {"ms_per_iter": (time.perf_counter() - t0) * 1e3 / steps,
                            "status": st, "clock": "host (the mode synchronises)"}
    return out


def batched_shots(steps):
    """64 surface shots with uneven beam counts (shots512, mixed precision)
    as one graph: capture decompose -> propagate -> reconstruct once, then
    time replays; the splat split is chosen by the autotuner."""
    import torch
    import paper_1304_3542_amd as fga
    W = fi.workload("shots512", "mixed")
    ns = W.nshots
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = fga.FGA(W.grid, W.params, "mixed", max_shots=ns)
        ctx.set_velocity(torch.from_numpy(W.c).cuda())
        f0 = torch.from_numpy(np.ascontiguousarray(W.f0)).cuda()
        beams = fga.Beams(4_000_000, ns)
        ctx.decompose(f0, None, beams)
        st, need = ctx.status()
        if st == fga.FGA_ECAPACITY:
            beams = fga.Beams(int(need * 1.05) + 1024, ns)
            ctx.decompose(f0, None, beams)
        off = ctx.offsets(beams, ns)
        counts = np.diff(off)
        u = torch.empty((ns, W.grid.n2, W.grid.n1), dtype=torch.float64, device="cuda")
        ctx.propagate(beams, ns, W.params.nsteps)
        chosen = ctx.autotune(beams, ns, u)
        ctx.graph_capture(f0, None, beams, W.params.nsteps, u)
        ctx.graph_launch()
        stream.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(steps):
            ctx.graph_launch()
        ev[1].record(stream)
        stream.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / steps
        st, _ = ctx.status()
    nb = int(off[-1])
    return {"workload": "shots512: 64 surface shots on the 512x512 model, random width "
            "1-4 cells and wavenumber 0.5-2, q 20x10, p 56x56, tau=1e-4, mixed, one graph",
            "nshots": ns, "nbeams": nb, "beams_per_shot_min": int(counts.min()),
            "beams_per_shot_max": int(counts.max()), "ms_per_replay": ms,
            "beams_per_s": nb / (ms * 1e-3), "splat_units_per_cu": chosen, "status": st}


def fwi_iteration(steps, precision="mixed_split"):
    """The batched forward+adjoint iteration on the 64-shot workload
    (shots512): the reduced-precision forward of every shot's u(T) as one
    graph replay, then the FP64 receiver misfit of the same shots (receivers
    on the top row every 10 steps, data from the model with the +5 %
    anomaly): traces with a checkpoint per record, the trace adjoint and the
    decomposition adjoint (dJ/dc and dJ/df0).  ms per iteration, device
    clock, with the parts."""
    import torch
    import paper_1304_3542_amd as fga
    Wm = fi.workload("shots512", "mixed")
    Wd = fi.workload("shots512", "fp64")
    g, p = Wd.grid, Wd.params
    ns = Wm.nshots
    every = 10
    nrec_t = p.nsteps // every
    rec = torch.arange(g.n1, dtype=torch.int32, device="cuda")
    c = torch.from_numpy(Wd.c).cuda()
    c_true = torch.from_numpy(fi.gaussian_anomaly(g, Wd.c, (1.0, 0.5), 0.1, 0.05)).cuda()
    f0 = torch.from_numpy(np.ascontiguousarray(Wm.f0)).cuda()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        cm = fga.FGA(g, Wm.params, precision, max_shots=ns)
        cm.set_velocity(c)
        bm = fga.Beams(4_000_000, ns)
        cm.decompose(f0, None, bm)
        st, need = cm.status()
        if st == fga.FGA_ECAPACITY:
            bm = fga.Beams(int(need * 1.05) + 1024, ns)
        u = torch.empty((ns, g.n2, g.n1), dtype=torch.float64, device="cuda")
        cm.graph_capture(f0, None, bm, Wm.params.nsteps, u)
        cd = fga.FGA(g, p, "fp64", max_shots=ns)
        bd = fga.Beams(4_000_000, ns)
        cd.set_velocity(c_true)
        cd.decompose(f0, None, bd)
        st, need = cd.status()
        if st == fga.FGA_ECAPACITY:
            bd = fga.Beams(int(need * 1.05) + 1024, ns)
            cd.decompose(f0, None, bd)
        nbd = int(cd.offsets(bd, ns)[-1])
        data = cd.trace(bd, ns, rec, every, nrec_t)
        cd.set_velocity(c)
        ckpt = torch.empty((nrec_t, fga.FGA_NSTATE, bd.capacity), dtype=torch.float64,
                           device="cuda")
        dc = torch.zeros_like(c)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

        def it(timed):
            if timed:
                ev[0].record(stream)
            cm.graph_launch()
            if timed:
                ev[1].record(stream)
            cd.decompose(f0, None, bd)
            tr = cd.trace(bd, ns, rec, every, nrec_t, ckpt)
            dc.zero_()
            gcoef = cd.trace_adjoint(bd, ns, rec, every, nrec_t, ckpt, (tr - data).contiguous(), dc)
            cd.decompose_adjoint(bd, ns, gcoef)
            if timed:
                ev[2].record(stream)

        it(False)
        stream.synchronize()
        fw, ad = [], []
        for _ in range(steps):
            it(True)
            stream.synchronize()
            fw.append(ev[0].elapsed_time(ev[1]))
            ad.append(ev[1].elapsed_time(ev[2]))
        st1, _ = cm.status()
        st2, _ = cd.status()
        # the same FP64 part with the state of every step kept by the forward
        # (23 doubles per beam and step, ~130 GB here) instead of recomputed
        cd.close()
        del ckpt, bd
        torch.cuda.empty_cache()
        ce = fga.FGA(g, p.replace(ckpt_every_step=1), "fp64", max_shots=ns)
        ce.set_velocity(c)
        be = fga.Beams(nbd + 1024, ns)
        ckpt_e = torch.empty((ce.ckpt_rows(every, nrec_t), fga.FGA_NSTATE, be.capacity),
                             dtype=torch.float64, device="cuda")

        def it_every():
            ev[1].record(stream)
            ce.decompose(f0, None, be)
            tr = ce.trace(be, ns, rec, every, nrec_t, ckpt_e)
            dc.zero_()
            gcoef = ce.trace_adjoint(be, ns, rec, every, nrec_t, ckpt_e, (tr - data).contiguous(),
                                     dc)
            ce.decompose_adjoint(be, ns, gcoef)
            ev[2].record(stream)

        it_every()
        stream.synchronize()
        ad_e = []
        for _ in range(steps):
            it_every()
            stream.synchronize()
            ad_e.append(ev[1].elapsed_time(ev[2]))
        st3, _ = ce.status()
        ce.close()
        del ckpt_e, be
        torch.cuda.empty_cache()
    nbm = int(cm.offsets(bm, ns)[-1])
    fw, ad = np.array(fw), np.array(ad)
    every_step = {"ms_per_iter": float(np.median(fw) + np.median(ad_e)),
                  "adjoint_ms": float(np.median(ad_e)),
                  "checkpoints": "every step (the adjoint reads the states)", "status": st3}
    return {"workload": "shots512 forward+adjoint: 64 surface shots on the 512x512 model; "
            f"{precision} forward of u(T) as one graph, then the FP64 receiver misfit "
            "(top row every 10 steps, data from a +5 % anomaly): traces with checkpoints "
            "per record, trace adjoint, decomposition adjoint",
            "nshots": ns, "nbeams_forward": nbm, "nbeams_adjoint": nbd,
            "ms_per_iter": float(np.median(fw + ad)), "forward_ms": float(np.median(fw)),
            "adjoint_ms": float(np.median(ad)), "iterations": steps,
            "every_step_checkpoints": every_step,
            "status": st1 if st1 != 0 else st2}


def topn_step(steps):
    """The paper's selection mode: point512 keeping the N = 5650 largest
    |psi| of each wave branch (mixed precision); ms per decompose ->
    propagate -> reconstruct step and its stages."""
    import torch
    W = fi.workload("topn512", "mixed")
    path = Path(W, "mixed", 4 * W.params.top_n)
    nb = path.fit_capacity()
    ms, stage_ms, per_step = time_path(path, steps, 1)
    st, _ = path.ctx.status()
    path.ctx.close()
    # the few-beam end of the same mode (the paper's smallest N is 6)
    Wf = fi.Workload("topn6", W.grid, W.params.replace(top_n=6), W.c, W.f0, None)
    pf = Path(Wf, "mixed", 64)
    nbf = pf.fit_capacity()
    msf, stage_f, _ = time_path(pf, steps, 1)
    stf, _ = pf.ctx.status()
    pf.ctx.close()
    return {"workload": "topn512: point512 keeping the 5650 largest |psi| per wave branch "
            "(radix select), mixed", "nbeams": nb, "ms_per_step": ms,
            "ms_per_step_device_median": float(np.median(per_step)),
            "beams_per_s": nb / (ms * 1e-3),
            "stages_ms": dict(zip(("decompose", "propagate", "reconstruct"),
                                  stage_ms.tolist())), "status": st,
            "n6": {"nbeams": nbf, "ms_per_step": msf,
                   "stages_ms": dict(zip(("decompose", "propagate", "reconstruct"),
                                         stage_f.tolist())), "status": stf}}


def fbi_flops(W, tau_fbi):
    """Algorithmic flops of the two FBI passes of one decomposition (FMA = 2):
    pass 1, a real x complex MAC (4 flop) per (shot, row, q column, p1,
    window column); pass 2, a complex MAC (8 flop) per (shot, q row, p2,
    q column x p1, window row); windows clipped at the grid edges."""
    g, p = W.grid, W.params
    R1 = math.ceil(math.sqrt(2 * p.eps * math.log(1 / tau_fbi)) / g.d1)
    R2 = math.ceil(math.sqrt(2 * p.eps * math.log(1 / tau_fbi)) / g.d2)
    k1 = p.qb1 + p.qs1 * np.arange(p.nq1)
    k2 = p.qb2 + p.qs2 * np.arange(p.nq2)
    K1 = (np.minimum(R1, g.n1 - 1 - k1) + np.minimum(R1, k1) + 1).sum()
    K2 = (np.minimum(R2, g.n2 - 1 - k2) + np.minimum(R2, k2) + 1).sum()
    nsf = W.nshots * (1 if W.f1 is None else 2)
    pass1 = 4.0 * nsf * g.n2 * p.np1 * K1
    pass2 = 8.0 * nsf * p.np2 * p.nq1 * p.np1 * K2
    return pass1, pass2


def closed_step(steps, u_integrated):
    """point512 with the closed-form amplitude (amp_closed = 1, mixed): ms per
    step and stages, and the field's difference from the integrated-amplitude
    run of the same step."""
    W = fi.workload("point512", "mixed")
    W = fi.Workload(W.name, W.grid, W.params.replace(amp_closed=1), W.c, W.f0, W.f1)
    path = Path(W, "mixed", 1_300_000)
    nb = path.fit_capacity()
    ms, stage_ms, per_step = time_path(path, steps, 1)
    st, _ = path.ctx.status()
    u = path.u.cpu().numpy()
    return {"workload": "point512 with a = c(Q)/c(q) (det Z)^(1/2) (root tracked per step), "
            "mixed", "nbeams": nb, "ms_per_step": ms,
            "ms_per_step_device_median": float(np.median(per_step)),
            "beams_per_s": nb / (ms * 1e-3),
            "stages_ms": dict(zip(("decompose", "propagate", "reconstruct"), stage_ms.tolist())),
            "rel_l2_vs_integrated_amplitude": float(np.linalg.norm(u - u_integrated) /
                                                    np.linalg.norm(u_integrated)),
            "status": st}


def dd_step(steps, u_integrated):
    """point512 with dzQ, dzP from divided differences (dz_divided = 1,
    closed-form amplitude, mixed), at the neighbouring mesh nodes
    (dz_scale = 1) and at rays 1e-3 mesh steps apart: ms per step and stages,
    and each field's difference from the dynamic ray tracing run of the same
    step (over the mesh steps the divided differences are an approximation
    of their own)."""
    import torch
    out = {"workload": "point512 with dzQ, dzP from divided differences (9 rays per beam), "
           "closed-form amplitude, mixed"}
    for scale in (1.0, 1e-3):
        W = fi.workload("point512", "mixed")
        W = fi.Workload(W.name, W.grid,
                        W.params.replace(amp_closed=1, dz_divided=1, dz_scale=scale),
                        W.c, W.f0, W.f1)
        path = Path(W, "mixed", 1_300_000)
        nb = path.fit_capacity()
        ms, stage_ms, per_step = time_path(path, steps, 1)
        st, _ = path.ctx.status()
        u = path.u.cpu().numpy()
        out["dz_scale=%g" % scale] = {
            "nbeams": nb, "ms_per_step": ms,
            "ms_per_step_device_median": float(np.median(per_step)),
            "beams_per_s": nb / (ms * 1e-3),
            "ray_steps_per_s": 9 * nb * W.params.nsteps / (stage_ms[1] * 1e-3),
            "stages_ms": dict(zip(("decompose", "propagate", "reconstruct"), stage_ms.tolist())),
            "rel_l2_vs_dynamic_ray_tracing": float(np.linalg.norm(u - u_integrated) /
                                                   np.linalg.norm(u_integrated)),
            "status": st}
        path.ctx.close()
        del path
        torch.cuda.empty_cache()
    return out


def d3_step(steps):
    """point3d (FP64, three space dimensions): ms per step of decompose +
    propagate (100 RK4 steps) + reconstruct, and per stage (HIP events)."""
    import torch
    import fga_inputs.d3 as i3
    import paper_1304_3542_amd as fga
    W = i3.workload3("point3d")
    g, p = W.grid, W.params
    ctx = fga.FGA3(g, p)
    ctx.set_velocity(torch.from_numpy(W.c).cuda())
    f0 = torch.from_numpy(np.ascontiguousarray(W.f0)).cuda()
    beams = fga.Beams3(4_000_000, 1)
    u = torch.empty((1, g.n3, g.n2, g.n1), dtype=torch.float64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step():
        ev[0].record()
        ctx.decompose(f0, None, beams)
        ev[1].record()
        ctx.propagate(beams, 1, p.nsteps)
        ev[2].record()
        ctx.reconstruct(beams, 1, u)
        ev[3].record()

    step()
    torch.cuda.synchronize()
    st0 = ctx.status()
    stages = np.zeros(3)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        torch.cuda.synchronize()
        stages += [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
    ms = (time.perf_counter() - t0) * 1e3 / steps
    nb = int(beams.offsets[1].item())
    st, _ = ctx.status()
    return {"workload": "point3d: 96x96x64 smooth layered 3-D model, eps=1/64, point source, "
            "q 15x15x10, p 20^3, tau=1e-3, 100 RK4 steps, FP64", "nbeams": nb,
            "ms_per_step": ms, "beams_per_s": nb / (ms * 1e-3),
            "stages_ms": dict(zip(("decompose", "propagate", "reconstruct"),
                                  (stages / steps).tolist())),
            "status": st if st0[0] == 0 else st0[0]}


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(W, nbeams, budget_s):
    """The oracle on a bounded sample of the same workload, scaled to the
    whole job: the FBI at the NQS q nodes of largest bound (fewer if the
    first one shows they would overrun about two thirds of budget_s seconds,
    never fewer than NQB), scaled to the q nodes the oracle visits (decompose(q_skip=True): the others cannot keep
    a beam), and RK4 and the windowed sum for the 2 * PER beams of largest
    |psi| at each of the first NQB of those nodes, scaled to the job's beam
    count."""
    import oracle
    NQS, NQB, PER = 100, 10, 512
    g, p = W.grid, W.params
    nq = p.nq1 * p.nq2
    bound = 0.5 * oracle.fbi_bound(W.f0[0], g, p).ravel()
    order_q = np.argsort(-bound, kind="stable")
    t = time.perf_counter()
    psis = []
    nqs = NQS
    for q in order_q:
        if len(psis) >= nqs:
            break
        j2, j1 = divmod(int(q), p.nq1)
        one = p.replace(qb1=p.qb1 + p.qs1 * j1, qb2=p.qb2 + p.qs2 * j2, nq1=1, nq2=1)
        psis.append((one, oracle.fbi(W.f0[0], g, one)[0, 0]))
        if len(psis) == 1:
            # about two thirds of the budget for the FBI windows (at least NQB)
            spent = time.perf_counter() - t
            nqs = int(min(NQS, max(NQB, 0.65 * budget_s / max(spent, 1e-6))))
    top = order_q[:len(psis)]
    t_per_q = (time.perf_counter() - t) / len(top)
    M = max(0.5 * np.abs(ps).max() for _, ps in psis)
    visited = int((bound * (1 + 1e-9) >= p.tau * M).sum())
    t_fbi = t_per_q * visited
    # beams: at each of the first NQB sampled q nodes the PER largest |psi|,
    # both branches
    pm1, pm2 = oracle.pmesh(p.np1, p.dp1), oracle.pmesh(p.np2, p.dp2)
    sts, coefs = [], []
    for one, psi in psis[:NQB]:
        order = np.argsort(-np.abs(psi.ravel()), kind="stable")[:PER]
        l2, l1 = np.unravel_index(order, psi.shape)
        st = np.zeros((2 * PER, oracle.NSTATE))
        st[:, 0] = g.o1 + g.d1 * one.qb1
        st[:, 1] = g.o2 + g.d2 * one.qb2
        st[:, 2] = np.tile(pm1[l1], 2)
        st[:, 3] = np.tile(pm2[l2], 2)
        st[:, 5] = st[:, 11] = 1.0
        st[:, 14] = st[:, 20] = -1.0
        st[:, 21] = 2.0
        sts.append(st)
        coefs.append(np.tile(psi.ravel()[order], 2))
    st = np.concatenate(sts)
    coef = np.concatenate(coefs)
    nsb = st.shape[0]
    sig = np.tile(np.repeat(np.array([1, -1], np.int8), PER), NQB)
    b = oracle.Beams(np.zeros(nsb, np.int32), sig, np.arange(nsb, dtype=np.int64), coef,
                     np.ascontiguousarray(np.stack([coef.real, coef.imag], 1)), st,
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
        "cpu": cpu_model(), "kind": "oracle",
        "sample": (f"FP64 oracle on {W.name}: FBI at the {len(top)} q nodes of largest bound "
                   f"({t_per_q:.2f} s each), scaled to the {visited} of {nq} q nodes it "
                   f"visits (the others cannot keep a beam); RK4 ({p.nsteps} steps) and the "
                   f"windowed sum over the grid for {nsb} beams (the {PER} largest |psi| at "
                   f"each of {NQB} of those q nodes, both branches), scaled linearly to the "
                   f"{nbeams} beams of the job"),
        "est_seconds": {"fbi": t_fbi, "rk4": t_rk4, "reconstruct": t_rec},
    }


WORKLOAD_TEXT = {
    "large2048": "large2048: 2048x1024 smooth layered model on [0,2]x[0,1], eps=1/1024, point "
                 "source (sigma 2 cells), q 147x74, p 400x400, tau=1e-6, T=0.25 s, dt=1 ms, "
                 "mixed precision",
    "point512": "point512: 512x512 smooth layered model, eps=1/256, point source, q 40x20, "
                "p 112x112, tau=1e-6, T=0.25 s, dt=1 ms, mixed precision",
}


def measure(name, steps, warmup, fp64_steps, graph_steps, precision="mixed"):
    """The whole step of one single-shot workload in mixed precision (timed
    steps on the host clock and per stage with HIP events, graph replays),
    the FP64 GPU path on the same input, the mixed field's error against it
    and against the stored oracle values, and the roofline entries of the
    path's kernels."""
    import torch
    W = fi.workload(name, "mixed")
    Wd = fi.workload(name, "fp64")
    cand = 2 * W.params.nq1 * W.params.nq2 * W.params.np1 * W.params.np2 * W.nshots

    mixed = Path(W, precision, min(cand, 4_000_000))
    nb = mixed.fit_capacity()
    ms_step, stage_ms, per_step = time_path(mixed, steps, warmup)
    u_mixed = mixed.u.cpu().numpy()
    f_host = mixed.beams.f[:, :nb].cpu().numpy()
    graph = graph_replays(mixed, graph_steps, nb) if graph_steps > 0 else None
    pairs = box_pairs(f_host, nb, W, W.params.tau_win)
    del f_host
    splat_ms = time_splat_kernel(mixed)

    fp64 = Path(Wd, "fp64", min(cand, 4_000_000))
    nb64 = fp64.fit_capacity()
    ms64, stage64, _ = time_path(fp64, max(1, fp64_steps), 0)
    u64 = fp64.u.cpu().numpy()
    # beams on the other side of the threshold in one path: its decisions are
    # taken in the precision of each path's FBI
    ids_m, ids_d = mixed.beams.id[:nb], fp64.beams.id[:nb64]
    flips = int((~torch.isin(ids_m, ids_d)).sum().item() + (~torch.isin(ids_d, ids_m)).sum().item())
    del ids_m, ids_d
    fp64.ctx.close()
    del fp64
    mixed.ctx.close()
    del mixed
    torch.cuda.empty_cache()
    rel_vs_fp64 = float(np.linalg.norm(u_mixed - u64) / np.linalg.norm(u64))

    rel_oracle = None
    gold = os.path.join(ROOT, "tests", "golden", f"{name}_fp64.npz")
    if os.path.exists(gold) and W.nshots == 1:
        z = np.load(gold)
        ref = z["u"]
        rel_oracle = {
            "mixed": float(np.linalg.norm(u_mixed[0].ravel()[z["nodes"]] - ref) / np.linalg.norm(ref)),
            "fp64": float(np.linalg.norm(u64[0].ravel()[z["nodes"]] - ref) / np.linalg.norm(ref)),
            "nodes": int(z["nodes"].size),
            "nbeams_oracle": int(z["nbeams"]),
        }

    npts = W.grid.n1 * W.grid.n2 * W.nshots
    stages = {"decompose": stage_ms[0], "propagate": stage_ms[1], "reconstruct": stage_ms[2]}
    dom = max(stages, key=stages.get)
    rk_fl = RK4_FLOP_PER_BEAM_STEP * W.params.nsteps * nb
    rk_ach = rk_fl / (stage_ms[1] * 1e-3)
    sp_fl = 4.0 * pairs
    sp_ach = sp_fl / (splat_ms * 1e-3)
    f1_fl, f2_fl = fbi_flops(W, W.params.tau_fbi)
    fb_ach = (f1_fl + f2_fl) / (stage_ms[0] * 1e-3)
    # the split path computes every FP32 product as four FP16 products on the
    # FP16 matrix cores: its entries state the executed FP16 rate against the
    # FP16 peak beside the algorithmic (FP32-product) rate
    split = precision == "mixed_split"
    xf, mpk = (4.0, PEAK["fp16"]) if split else (1.0, PEAK["fp32"])
    fbk, spk = (("k_fbi_pass2_split", "k_splat_binned_split") if split
                else ("k_fbi_pass2_mfma", "k_splat_binned"))
    kernels = {
        # ms is the whole decomposition (both passes, selection, compaction);
        # the passes alone are in the kernel trace under profiles/
        fbk: {"bound": "mfma", "achieved": xf * fb_ach / 1e12, "peak": mpk / 1e12,
              "unit": "TFLOP/s", "frac": xf * fb_ach / mpk,
              "achieved_algorithmic": fb_ach / 1e12, "ms": stage_ms[0],
              "ms_covers": "decompose stage", "flop_per_launch": f2_fl, "flop_pass1": f1_fl},
        # one launch per propagate call: the stage time is the kernel's
        "k_rk4": {"bound": "alu", "achieved": rk_ach / 1e12, "peak": PEAK["fp64"] / 1e12,
                  "unit": "TFLOP/s", "frac": rk_ach / PEAK["fp64"], "ms": stage_ms[1],
                  "flop_per_launch": rk_fl, "traffic": profiled_traffic("k_rk4", name)},
        # ms is the whole reconstruction (records, binning, splat, reduction);
        # the products over the truncation boxes only (the tiles a box meets
        # hold more nodes)
        spk: {"bound": "mfma", "achieved": xf * sp_ach / 1e12, "peak": mpk / 1e12,
              "unit": "TFLOP/s", "frac": xf * sp_ach / mpk,
              "achieved_algorithmic": sp_ach / 1e12, "ms": splat_ms,
              "ms_covers": "reconstruct stage", "flop_per_launch": sp_fl,
              "traffic": profiled_traffic(spk, name)},
    }
    roof = dict(kernels["k_rk4" if dom != "reconstruct" else spk])
    roof["kernel"] = "k_rk4" if dom != "reconstruct" else spk
    for key in ("ms", "flop_per_launch", "ms_covers"):
        roof.pop(key, None)
    return {
        "nb": nb, "ms_step": ms_step, "per_step": per_step, "stages": stages,
        "graph": graph, "rel_vs_fp64": rel_vs_fp64, "rel_oracle": rel_oracle, "flips": flips,
        "pairs": pairs, "npts": npts, "kernels": kernels, "roofline": roof,
        "fp64_gpu": {"ms_per_step": ms64, "nbeams": nb64,
                     "stages_ms": dict(zip(stages, stage64.tolist())),
                     "speedup_mixed_over_fp64": ms64 / ms_step},
        "u_mixed": u_mixed, "W": W, "Wd": Wd,
    }


def summary(name, r, steps, warmup):
    """The JSON fields of one measured workload."""
    ps = r["per_step"]
    return {
        "workload": WORKLOAD_TEXT.get(name, name),
        "nbeams": r["nb"],
        "steps": steps, "warmup": warmup,
        "ms_per_step": r["ms_step"],
        "beams_per_s": r["nb"] / (r["ms_step"] * 1e-3),
        "ms_per_step_device": {"median": float(np.median(ps)),
                               "iqr": float(np.percentile(ps, 75) - np.percentile(ps, 25)),
                               "min": float(ps.min()), "max": float(ps.max())},
        "valid": bool(r["rel_vs_fp64"] <= 1e-5),
        "rel_l2_vs_fp64_gpu": r["rel_vs_fp64"],
        "rel_l2_vs_oracle_sample": r["rel_oracle"],
        "threshold_flips_vs_fp64": r["flips"],
        "stages_ms": r["stages"],
        "graph": r["graph"],
        "grid_points_per_s": r["npts"] / (r["ms_step"] * 1e-3),
        "pairs": r["pairs"],
        "pairs_per_s": r["pairs"] / (r["stages"]["reconstruct"] * 1e-3),
        "fp64_gpu": r["fp64_gpu"],
        "roofline": r["roofline"],
        "kernels": r["kernels"],
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 "
                          "(sharding over several GPUs is designed, not built)"}))
        sys.exit(2)
    import torch
    if args.calib_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    name = args.workload
    r = measure(name, args.steps, args.warmup, args.fp64_steps, args.graph_steps,
                args.precision)
    head = summary(name, r, args.steps, args.warmup)
    out = {
        "metric": "beams/s end-to-end (FBI+trace+sum) at rel-L2<=1e-5 vs FP64; adjoint ms/iter",
        "value": head["beams_per_s"],
        "unit": "beams/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "ms_per_step_device": head["ms_per_step_device"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # RK4 in FP64; FBI and splat products in FP32, or as FP16 hi/lo
        # products summed in FP32 (split)
        "dtype": "f64+f32+f16split" if args.precision == "mixed_split" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": head["workload"], "nshots": r["W"].nshots, "nbeams": r["nb"]},
    }
    for k in ("valid", "rel_l2_vs_fp64_gpu", "rel_l2_vs_oracle_sample",
              "threshold_flips_vs_fp64", "stages_ms", "graph",
              "grid_points_per_s", "pairs", "pairs_per_s", "fp64_gpu", "roofline", "kernels"):
        out[k] = head[k]
    u_point = r["u_mixed"] if name == "point512" else None
    Wd, nb = r["Wd"], r["nb"]
    del r
    if name != "point512" and args.point_steps > 0:
        rp = measure("point512", args.point_steps, 1, 1, args.point_steps, args.precision)
        out["point512"] = summary("point512", rp, args.point_steps, 1)
        u_point = rp["u_mixed"]
        del rp
    if args.adjoint_steps > 0:
        out["adjoint"] = adjoint_iteration(args.adjoint_steps)
    if args.batch_steps > 0:
        out["batched"] = batched_shots(args.batch_steps)
    if args.fwi_steps > 0:
        out["fwi_batched"] = fwi_iteration(args.fwi_steps, args.precision)
    if args.topn_steps > 0:
        out["topn"] = topn_step(args.topn_steps)
    if args.closed_steps > 0 and u_point is not None:
        out["closed_amplitude"] = closed_step(args.closed_steps, u_point)
    if args.dd_steps > 0 and u_point is not None:
        out["divided_differences"] = dd_step(args.dd_steps, u_point)
    if args.d3_steps > 0:
        out["d3"] = d3_step(args.d3_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(Wd, nb, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

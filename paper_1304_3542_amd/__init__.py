"""MI355X (gfx950) frozen Gaussian approximation: Python binding of libfga.so.

The binding only marshals arguments: every step of the path runs in the HIP
kernels of ``libfga.so``.  PyTorch supplies device memory and the stream.
The module-level functions carry the names of the C entry points declared in
``include/fga.h``; :class:`FGA` is a convenience wrapper around them.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfga.so")

FGA_OK, FGA_EINVAL, FGA_ENOMEM, FGA_ECAPACITY, FGA_EHIP, FGA_ENUMERIC, FGA_ESTATE = (
    0, -1, -2, -3, -4, -5, -6)
FGA_FP64, FGA_MIXED, FGA_MIXED_SPLIT = 0, 1, 2
PRECISIONS = {"fp64": FGA_FP64, "mixed": FGA_MIXED, "mixed_split": FGA_MIXED_SPLIT}
FGA_NSTATE, FGA_NFIELD, FGA_F_STATE = 23, 29, 6

STATUS_NAMES = {0: "FGA_OK", -1: "FGA_EINVAL", -2: "FGA_ENOMEM", -3: "FGA_ECAPACITY",
                -4: "FGA_EHIP", -5: "FGA_ENUMERIC", -6: "FGA_ESTATE"}


class FGAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class fga_grid(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("o1", ctypes.c_double),
                ("o2", ctypes.c_double), ("d1", ctypes.c_double), ("d2", ctypes.c_double)]


class fga_params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("qb1", ctypes.c_int32), ("qb2", ctypes.c_int32),
                ("qs1", ctypes.c_int32), ("qs2", ctypes.c_int32), ("nq1", ctypes.c_int32),
                ("nq2", ctypes.c_int32), ("np1", ctypes.c_int32), ("np2", ctypes.c_int32),
                ("dp1", ctypes.c_double), ("dp2", ctypes.c_double), ("tau", ctypes.c_double),
                ("tau_fbi", ctypes.c_double), ("tau_win", ctypes.c_double),
                ("dt", ctypes.c_double), ("top_n", ctypes.c_int32),
                ("amp_closed", ctypes.c_int32), ("dz_divided", ctypes.c_int32),
                ("dz_scale", ctypes.c_double), ("deterministic", ctypes.c_int32),
                ("grad_log", ctypes.c_int32), ("ckpt_every_step", ctypes.c_int32)]


class fga3_grid(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
                ("o1", ctypes.c_double), ("o2", ctypes.c_double), ("o3", ctypes.c_double),
                ("d1", ctypes.c_double), ("d2", ctypes.c_double), ("d3", ctypes.c_double)]


class fga3_params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("qb", ctypes.c_int32 * 3), ("qs", ctypes.c_int32 * 3),
                ("nq", ctypes.c_int32 * 3), ("np", ctypes.c_int32 * 3),
                ("dp", ctypes.c_double * 3), ("tau", ctypes.c_double),
                ("tau_fbi", ctypes.c_double), ("tau_win", ctypes.c_double),
                ("dt", ctypes.c_double)]


class fga_beams(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int64), ("f", ctypes.c_void_p), ("id", ctypes.c_void_p),
                ("offsets", ctypes.c_void_p)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libfga.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1304_3542_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(path)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    C = ctypes.c_void_p   # fga_ctx*
    sig = {
        "fga_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(fga_grid),
                       ctypes.POINTER(fga_params), I32, I32, P],
        "fga_destroy": [C],
        "fga_set_stream": [C, P],
        "fga_set_velocity": [C, P],
        "fga_decompose": [C, I32, P, P, ctypes.POINTER(fga_beams)],
        "fga_propagate": [C, ctypes.POINTER(fga_beams), I32, I32],
        "fga_reconstruct": [C, ctypes.POINTER(fga_beams), I32, P],
        "fga_trace": [C, ctypes.POINTER(fga_beams), I32, P, I32, I32, I32, P, P],
        "fga_trace_noalloc": [C, ctypes.POINTER(fga_beams), I32, P, I32, I32, I32, P, P],
        "fga_trace_adjoint": [C, ctypes.POINTER(fga_beams), I32, P, I32, I32, I32, P, P, P, P],
        "fga_decompose_adjoint": [C, ctypes.POINTER(fga_beams), I32, P, P, P, P],
        "fga_reconstruct_adjoint": [C, ctypes.POINTER(fga_beams), I32, P, P, P],
        "fga_propagate_ckpt": [C, ctypes.POINTER(fga_beams), I32, I32, I32, P],
        "fga_propagate_adjoint": [C, ctypes.POINTER(fga_beams), I32, I32, I32, P, P, P],
        "fga_graph_capture": [C, I32, P, P, ctypes.POINTER(fga_beams), I32, P],
        "fga_graph_launch": [C],
        "fga_autotune": [C, ctypes.POINTER(fga_beams), I32, P, ctypes.c_char_p,
                         ctypes.POINTER(ctypes.c_int32)],
        "fga_sync_status": [C, ctypes.POINTER(ctypes.c_int64)],
        "fga_copy_offsets": [C, ctypes.POINTER(fga_beams), I32, P],
        "fga_last_error": [C],
        "fga3_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(fga3_grid),
                        ctypes.POINTER(fga3_params), I32, P],
        "fga3_destroy": [C],
        "fga3_set_velocity": [C, P],
        "fga3_decompose": [C, I32, P, P, ctypes.POINTER(fga_beams)],
        "fga3_propagate": [C, ctypes.POINTER(fga_beams), I32, I32],
        "fga3_reconstruct": [C, ctypes.POINTER(fga_beams), I32, P],
        "fga3_sync_status": [C, ctypes.POINTER(ctypes.c_int64)],
        "fga3_last_error": [C],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name.endswith("last_error") else ctypes.c_int
    _lib = L
    return L


def _check(ctx, status: int):
    if status != FGA_OK:
        msg = load().fga_last_error(ctx).decode()
        raise FGAError(status, msg)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


# ------------------------------------------------ names of the C entry points

def fga_create(grid, params, precision: int = FGA_FP64, max_shots: int = 1, stream=None):
    g = fga_grid(grid.n1, grid.n2, grid.o1, grid.o2, grid.d1, grid.d2)
    p = fga_params(params.eps, params.qb1, params.qb2, params.qs1, params.qs2, params.nq1,
                   params.nq2, params.np1, params.np2, params.dp1, params.dp2, params.tau,
                   params.tau_fbi, params.tau_win, params.dt, int(getattr(params, "top_n", 0)),
                   int(getattr(params, "amp_closed", 0)), int(getattr(params, "dz_divided", 0)),
                   float(getattr(params, "dz_scale", 1.0)), int(getattr(params, "deterministic", 0)),
                   int(getattr(params, "grad_log", 0)),
                   int(getattr(params, "ckpt_every_step", 0)))
    ctx = ctypes.c_void_p()
    st = load().fga_create(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p), int(precision),
                           int(max_shots), _stream_handle(stream))
    _check(None, st)
    return ctx


def fga_destroy(ctx):
    _check(ctx, load().fga_destroy(ctx))


def fga_set_stream(ctx, stream=None):
    _check(ctx, load().fga_set_stream(ctx, _stream_handle(stream)))


def fga_set_velocity(ctx, c):
    _require(c, "c", "float64")
    _check(ctx, load().fga_set_velocity(ctx, _ptr(c)))


def fga_decompose(ctx, nshots: int, f0, f1, beams: "Beams"):
    _require(f0, "f0", "float64")
    if f1 is not None:
        _require(f1, "f1", "float64")
    _check(ctx, load().fga_decompose(ctx, int(nshots), _ptr(f0), _ptr(f1), beams.c_struct()))


def fga_propagate(ctx, beams: "Beams", nshots: int, nsteps: int):
    _check(ctx, load().fga_propagate(ctx, beams.c_struct(), int(nshots), int(nsteps)))


def fga_reconstruct(ctx, beams: "Beams", nshots: int, u):
    _require(u, "u", "float64")
    _check(ctx, load().fga_reconstruct(ctx, beams.c_struct(), int(nshots), _ptr(u)))


def fga_trace(ctx, beams: "Beams", nshots: int, rec, rec_every: int, nrec_t: int, traces,
              ckpt=None):
    _require(rec, "rec", "int32")
    _require(traces, "traces", "float64")
    _check(ctx, load().fga_trace(ctx, beams.c_struct(), int(nshots), _ptr(rec), rec.numel(),
                                 int(rec_every), int(nrec_t), _ptr(traces), _ptr(ckpt)))


def fga_trace_noalloc(ctx, beams: "Beams", nshots: int, rec, rec_every: int, nrec_t: int,
                      traces, ckpt=None):
    _require(rec, "rec", "int32")
    _require(traces, "traces", "float64")
    _check(ctx, load().fga_trace_noalloc(ctx, beams.c_struct(), int(nshots), _ptr(rec),
                                         rec.numel(), int(rec_every), int(nrec_t),
                                         _ptr(traces), _ptr(ckpt)))


def fga_trace_adjoint(ctx, beams: "Beams", nshots: int, rec, rec_every: int, nrec_t: int,
                      ckpt, gtr, dc, gcoef):
    _require(rec, "rec", "int32")
    for t, n in ((ckpt, "ckpt"), (gtr, "gtr"), (dc, "dc"), (gcoef, "gcoef")):
        _require(t, n, "float64")
    _check(ctx, load().fga_trace_adjoint(ctx, beams.c_struct(), int(nshots), _ptr(rec),
                                         rec.numel(), int(rec_every), int(nrec_t), _ptr(ckpt),
                                         _ptr(gtr), _ptr(dc), _ptr(gcoef)))


def fga_decompose_adjoint(ctx, beams: "Beams", nshots: int, gcoef, df0, df1=None, dc=None):
    for t, n in ((gcoef, "gcoef"), (df0, "df0")):
        _require(t, n, "float64")
    _check(ctx, load().fga_decompose_adjoint(ctx, beams.c_struct(), int(nshots), _ptr(gcoef),
                                             _ptr(df0), _ptr(df1), _ptr(dc)))


def fga_reconstruct_adjoint(ctx, beams: "Beams", nshots: int, du, dstate, dcoef):
    for t, n in ((du, "du"), (dstate, "dstate"), (dcoef, "dcoef")):
        _require(t, n, "float64")
    _check(ctx, load().fga_reconstruct_adjoint(ctx, beams.c_struct(), int(nshots), _ptr(du),
                                               _ptr(dstate), _ptr(dcoef)))


def fga_propagate_ckpt(ctx, beams: "Beams", nshots: int, seg: int, nseg: int, ckpt):
    _require(ckpt, "ckpt", "float64")
    _check(ctx, load().fga_propagate_ckpt(ctx, beams.c_struct(), int(nshots), int(seg), int(nseg),
                                          _ptr(ckpt)))


def fga_propagate_adjoint(ctx, beams: "Beams", nshots: int, seg: int, nseg: int, ckpt, dstate,
                          dc):
    for t, n in ((ckpt, "ckpt"), (dstate, "dstate"), (dc, "dc")):
        _require(t, n, "float64")
    _check(ctx, load().fga_propagate_adjoint(ctx, beams.c_struct(), int(nshots), int(seg),
                                             int(nseg), _ptr(ckpt), _ptr(dstate), _ptr(dc)))


def fga_graph_capture(ctx, nshots: int, f0, f1, beams: "Beams", nsteps: int, u):
    _require(f0, "f0", "float64")
    _require(u, "u", "float64")
    _check(ctx, load().fga_graph_capture(ctx, int(nshots), _ptr(f0), _ptr(f1), beams.c_struct(),
                                         int(nsteps), _ptr(u)))


def fga_graph_launch(ctx):
    _check(ctx, load().fga_graph_launch(ctx))


def fga_autotune(ctx, beams: "Beams", nshots: int, u, cache_path: Optional[str] = None) -> int:
    _require(u, "u", "float64")
    chosen = ctypes.c_int32(0)
    _check(ctx, load().fga_autotune(ctx, beams.c_struct(), int(nshots), _ptr(u),
                                    None if cache_path is None else cache_path.encode(),
                                    ctypes.byref(chosen)))
    return chosen.value


def fga_sync_status(ctx):
    """Returns (status, needed_capacity) without raising."""
    needed = ctypes.c_int64(0)
    st = load().fga_sync_status(ctx, ctypes.byref(needed))
    return st, needed.value


def fga_copy_offsets(ctx, beams: "Beams", nshots: int):
    import numpy as np
    out = np.zeros(nshots + 1, dtype=np.int64)
    _check(ctx, load().fga_copy_offsets(ctx, beams.c_struct(), int(nshots),
                                        out.ctypes.data_as(ctypes.c_void_p)))
    return out


def fga_last_error(ctx) -> str:
    return load().fga_last_error(ctx).decode()


def _require(t, name, dtype):
    import torch
    want = getattr(torch, dtype)
    if not t.is_cuda or t.dtype != want or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA tensor of {dtype}")


# ------------------------------------------------------------ convenience

class Beams:
    """Device beam buffers: f[FGA_NFIELD][capacity] float64, id[capacity]
    int64, offsets[max_shots+1] int64."""

    def __init__(self, capacity: int, max_shots: int = 1, device="cuda"):
        import torch
        self.capacity = int(capacity)
        self.f = torch.zeros((FGA_NFIELD, self.capacity), dtype=torch.float64, device=device)
        self.id = torch.zeros(self.capacity, dtype=torch.int64, device=device)
        self.offsets = torch.zeros(max_shots + 1, dtype=torch.int64, device=device)
        self._c = fga_beams(self.capacity, self.f.data_ptr(), self.id.data_ptr(),
                            self.offsets.data_ptr())

    def c_struct(self):
        return ctypes.byref(self._c)

    @property
    def state(self):
        return self.f[FGA_F_STATE:]


class FGA:
    """One grid, one parameter set and one precision on the current device."""

    def __init__(self, grid, params, precision: str = "fp64", max_shots: int = 1, stream=None):
        self.grid = grid
        self.params = params
        self.precision = precision
        self.max_shots = max_shots
        self.ctx = fga_create(grid, params, PRECISIONS[precision],
                              max_shots, stream)

    def close(self):
        if self.ctx is not None:
            fga_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_velocity(self, c):
        fga_set_velocity(self.ctx, c)

    def decompose(self, f0, f1, beams: Beams):
        fga_decompose(self.ctx, f0.shape[0], f0, f1, beams)

    def propagate(self, beams: Beams, nshots: int, nsteps: int):
        fga_propagate(self.ctx, beams, nshots, nsteps)

    def reconstruct(self, beams: Beams, nshots: int, u=None):
        import torch
        if u is None:
            u = torch.empty((nshots, self.grid.n2, self.grid.n1), dtype=torch.float64,
                            device=beams.f.device)
        fga_reconstruct(self.ctx, beams, nshots, u)
        return u

    def _check_ckpt(self, ckpt, beams: Beams, seg: int, nseg: int):
        # the library cannot see buffer sizes: a short checkpoint buffer
        # would be written past its end
        need = self.ckpt_rows(seg, nseg) * FGA_NSTATE * beams.capacity
        if ckpt.numel() < need:
            raise ValueError(f"ckpt holds {ckpt.numel()} doubles, {need} needed "
                             f"({self.ckpt_rows(seg, nseg)} x {FGA_NSTATE} x capacity)")

    def trace(self, beams: Beams, nshots: int, rec, rec_every: int, nrec_t: int, ckpt=None):
        import torch
        if ckpt is not None:
            self._check_ckpt(ckpt, beams, rec_every, nrec_t)
        tr = torch.empty((nshots, nrec_t, rec.numel()), dtype=torch.float64,
                         device=beams.f.device)
        fga_trace(self.ctx, beams, nshots, rec, rec_every, nrec_t, tr, ckpt)
        return tr

    def trace_adjoint(self, beams: Beams, nshots: int, rec, rec_every: int, nrec_t: int, ckpt,
                      gtr, dc):
        import torch
        self._check_ckpt(ckpt, beams, rec_every, nrec_t)
        gcoef = torch.empty((2, beams.capacity), dtype=torch.float64, device=beams.f.device)
        fga_trace_adjoint(self.ctx, beams, nshots, rec, rec_every, nrec_t, ckpt, gtr, dc, gcoef)
        return gcoef

    def decompose_adjoint(self, beams: Beams, nshots: int, gcoef, df1=None, dc=None):
        import torch
        df0 = torch.empty((nshots, self.grid.n2, self.grid.n1), dtype=torch.float64,
                          device=beams.f.device)
        fga_decompose_adjoint(self.ctx, beams, nshots, gcoef, df0, df1, dc)
        return df0

    def reconstruct_adjoint(self, beams: Beams, nshots: int, du):
        """(dstate [FGA_NSTATE][capacity], dcoef [2][capacity]) for dJ/du."""
        import torch
        dstate = torch.zeros((FGA_NSTATE, beams.capacity), dtype=torch.float64,
                             device=beams.f.device)
        dcoef = torch.zeros((2, beams.capacity), dtype=torch.float64, device=beams.f.device)
        fga_reconstruct_adjoint(self.ctx, beams, nshots, du, dstate, dcoef)
        return dstate, dcoef

    def ckpt_rows(self, seg: int, nseg: int) -> int:
        """Rows of the checkpoint buffer of nseg segments of seg steps:
        nseg, or nseg * seg + 1 with ckpt_every_step."""
        return nseg * seg + 1 if getattr(self.params, "ckpt_every_step", 0) else nseg

    def propagate_ckpt(self, beams: Beams, nshots: int, seg: int, nseg: int, ckpt=None):
        import torch
        if ckpt is None:
            ckpt = torch.empty((self.ckpt_rows(seg, nseg), FGA_NSTATE, beams.capacity),
                               dtype=torch.float64, device=beams.f.device)
        self._check_ckpt(ckpt, beams, seg, nseg)
        fga_propagate_ckpt(self.ctx, beams, nshots, seg, nseg, ckpt)
        return ckpt

    def propagate_adjoint(self, beams: Beams, nshots: int, seg: int, nseg: int, ckpt, dstate, dc):
        self._check_ckpt(ckpt, beams, seg, nseg)
        fga_propagate_adjoint(self.ctx, beams, nshots, seg, nseg, ckpt, dstate, dc)
        return dstate

    def graph_capture(self, f0, f1, beams: Beams, nsteps: int, u):
        fga_graph_capture(self.ctx, f0.shape[0], f0, f1, beams, nsteps, u)

    def graph_launch(self):
        fga_graph_launch(self.ctx)

    def autotune(self, beams: Beams, nshots: int, u, cache_path: Optional[str] = None) -> int:
        return fga_autotune(self.ctx, beams, nshots, u, cache_path)

    def status(self):
        return fga_sync_status(self.ctx)

    def offsets(self, beams: Beams, nshots: int):
        return fga_copy_offsets(self.ctx, beams, nshots)


def _trace_function():
    import torch

    class TraceFunction(torch.autograd.Function):
        """Receiver traces as a differentiable function of the velocity
        samples c and the initial data f0 (and f1): forward = fga_decompose
        + fga_trace with checkpoints, backward = fga_trace_adjoint +
        fga_decompose_adjoint (the library's hand-written adjoint; the beam
        set and truncation boxes of the forward are held fixed).  The beams
        and the context must not run another decomposition between the
        forward and the backward call."""

        @staticmethod
        def forward(actx, c, f0, f1, fga, beams, rec, rec_every, nrec_t):
            nshots = f0.shape[0]
            c = c.detach().contiguous()
            f0 = f0.detach().contiguous()
            f1 = None if f1 is None else f1.detach().contiguous()
            fga.set_velocity(c)
            fga.decompose(f0, f1, beams)
            ckpt = torch.empty((fga.ckpt_rows(rec_every, nrec_t), FGA_NSTATE, beams.capacity),
                               dtype=torch.float64, device=beams.f.device)
            tr = fga.trace(beams, nshots, rec, rec_every, nrec_t, ckpt)
            actx.fga, actx.beams, actx.rec = fga, beams, rec
            actx.rec_every, actx.nrec_t, actx.nshots = rec_every, nrec_t, nshots
            actx.has_f1 = f1 is not None
            actx.save_for_backward(c, ckpt)
            return tr

        @staticmethod
        def backward(actx, gtr):
            c, ckpt = actx.saved_tensors
            fga, beams = actx.fga, actx.beams
            dc = torch.zeros_like(c)
            gcoef = fga.trace_adjoint(beams, actx.nshots, actx.rec, actx.rec_every, actx.nrec_t,
                                      ckpt, gtr.contiguous(), dc)
            df1 = None
            if actx.has_f1:
                df1 = torch.empty((actx.nshots,) + tuple(c.shape), dtype=torch.float64,
                                  device=c.device)
            df0 = fga.decompose_adjoint(beams, actx.nshots, gcoef, df1,
                                        dc if actx.has_f1 else None)
            return dc, df0, df1, None, None, None, None, None

    return TraceFunction


_TRACE_FN = None


def traces(c, f0, f1, fga: FGA, beams: Beams, rec, rec_every: int, nrec_t: int):
    """Differentiable receiver traces [nshots][nrec_t][nrec] (torch autograd):
    gradients with respect to c, f0 and f1 come from the library's adjoint."""
    global _TRACE_FN
    if _TRACE_FN is None:
        _TRACE_FN = _trace_function()
    return _TRACE_FN.apply(c, f0, f1, fga, beams, rec, rec_every, nrec_t)


# ------------------------------------------------------ three space dimensions

FGA3_NSTATE = 45
FGA3_NFIELD = 53
FGA3_F_STATE = 8


class Beams3(Beams):
    """Caller-owned beam storage of the 3-D path: f[53][capacity] float64."""

    def __init__(self, capacity: int, max_shots: int = 1, device="cuda"):
        import torch
        self.capacity = int(capacity)
        self.f = torch.zeros((FGA3_NFIELD, self.capacity), dtype=torch.float64, device=device)
        self.id = torch.zeros(self.capacity, dtype=torch.int64, device=device)
        self.offsets = torch.zeros(max_shots + 1, dtype=torch.int64, device=device)
        self._c = fga_beams(self.capacity, self.f.data_ptr(), self.id.data_ptr(),
                            self.offsets.data_ptr())


def _check3(ctx, status: int):
    if status != FGA_OK:
        raise FGAError(status, load().fga3_last_error(ctx).decode())


class FGA3:
    """Context of the 3-D path (FP64): names follow the C entry points."""

    def __init__(self, grid, params, max_shots: int = 1, stream=None):
        g = fga3_grid(grid.n1, grid.n2, grid.n3, grid.o1, grid.o2, grid.o3, grid.d1, grid.d2,
                      grid.d3)
        p = fga3_params(params.eps, (ctypes.c_int32 * 3)(*params.qb),
                        (ctypes.c_int32 * 3)(*params.qs), (ctypes.c_int32 * 3)(*params.nq),
                        (ctypes.c_int32 * 3)(*params.np), (ctypes.c_double * 3)(*params.dp),
                        params.tau, params.tau_fbi, params.tau_win, params.dt)
        self.grid, self.params = grid, params
        ctx = ctypes.c_void_p()
        st = load().fga3_create(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p),
                                int(max_shots), _stream_handle(stream))
        _check3(None, st)
        self.ctx = ctx

    def close(self):
        if getattr(self, "ctx", None):
            load().fga3_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_velocity(self, c):
        _require(c, "c", "float64")
        _check3(self.ctx, load().fga3_set_velocity(self.ctx, _ptr(c)))

    def decompose(self, f0, f1, beams: Beams3):
        _require(f0, "f0", "float64")
        ns = f0.shape[0]
        _check3(self.ctx, load().fga3_decompose(self.ctx, int(ns), _ptr(f0), _ptr(f1),
                                                beams.c_struct()))

    def propagate(self, beams: Beams3, nshots: int, nsteps: int):
        _check3(self.ctx, load().fga3_propagate(self.ctx, beams.c_struct(), int(nshots),
                                                int(nsteps)))

    def reconstruct(self, beams: Beams3, nshots: int, u=None):
        import torch
        g = self.grid
        if u is None:
            u = torch.empty((nshots, g.n3, g.n2, g.n1), dtype=torch.float64,
                            device=beams.f.device)
        _require(u, "u", "float64")
        _check3(self.ctx, load().fga3_reconstruct(self.ctx, beams.c_struct(), int(nshots),
                                                  _ptr(u)))
        return u

    def status(self):
        needed = ctypes.c_int64(0)
        st = load().fga3_sync_status(self.ctx, ctypes.byref(needed))
        return st, needed.value

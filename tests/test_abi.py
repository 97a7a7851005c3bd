"""The C-ABI library: it loads, exports every entry point that include/fga.h
declares, and rejects invalid arguments on the host before any device work
(these calls need no GPU)."""
import ctypes
import os
import re

import pytest

import fga_inputs as fi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fga.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fga_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("fga_create", "fga_destroy", "fga_set_velocity", "fga_decompose",
              "fga_propagate", "fga_reconstruct", "fga_trace", "fga_sync_status",
              "fga_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1304_3542_amd as fga
    lib = fga.load()
    for n in _declared():
        assert hasattr(lib, n), n


def _structs(grid, params):
    import paper_1304_3542_amd as fga
    g = fga.fga_grid(grid.n1, grid.n2, grid.o1, grid.o2, grid.d1, grid.d2)
    p = fga.fga_params(params.eps, params.qb1, params.qb2, params.qs1, params.qs2, params.nq1,
                       params.nq2, params.np1, params.np2, params.dp1, params.dp2, params.tau,
                       params.tau_fbi, params.tau_win, params.dt, params.top_n, params.amp_closed,
                       params.dz_divided, params.dz_scale, params.deterministic,
                       params.grad_log, params.ckpt_every_step)
    return g, p


@pytest.mark.parametrize("bad", [
    dict(np1=7), dict(np2=0), dict(eps=0.0), dict(eps=float("nan")), dict(nq1=0),
    dict(qs2=0), dict(qb1=-1), dict(nq1=1000), dict(tau=1.5), dict(tau_fbi=0.0),
    dict(tau_win=1.0), dict(dt=-1e-3), dict(dp1=0.0), dict(top_n=-1), dict(amp_closed=2),
    dict(dz_divided=2, amp_closed=1), dict(dz_divided=1),
    dict(dz_divided=1, amp_closed=1, dz_scale=0.0), dict(deterministic=2), dict(grad_log=-2),
    dict(ckpt_every_step=2), dict(ckpt_every_step=1, amp_closed=1),
])
def test_create_rejects_bad_params(bad):
    import paper_1304_3542_amd as fga
    W = fi.workload("wavepacket")
    g, p = _structs(W.grid, W.params.replace(**bad))
    lib = fga.load()
    ctx = ctypes.c_void_p()
    st = lib.fga_create(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p), 0, 1, None)
    assert st == fga.FGA_EINVAL
    assert not ctx.value
    assert lib.fga_last_error(None)


def test_create_rejects_bad_grid_precision_and_shots():
    import paper_1304_3542_amd as fga
    W = fi.workload("wavepacket")
    lib = fga.load()
    ctx = ctypes.c_void_p()
    for grid, prec, shots in ((fi.Grid(2, 128, 0, 0, 1, 1), 0, 1),
                              (fi.Grid(128, 128, 0, 0, -1.0, 1), 0, 1),
                              (W.grid, 7, 1), (W.grid, 0, 0)):
        g, p = _structs(grid, W.params)
        st = lib.fga_create(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p), prec, shots,
                            None)
        assert st == fga.FGA_EINVAL
    assert lib.fga_create(None, None, None, 0, 1, None) == fga.FGA_EINVAL


def test_grid_size_limit():
    """Truncation boxes keep node indices in 16 bits (n marks an empty box),
    so n1, n2 <= FGA_MAX_N = 32767: 32768 is refused on the host, 32767
    passes the argument checks (and ends at the device query without a GPU)."""
    import paper_1304_3542_amd as fga
    W = fi.workload("wavepacket")
    lib = fga.load()
    assert "#define FGA_MAX_N 32767" in open(os.path.join(ROOT, "include", "fga.h")).read()
    for n1, n2, bad in ((32768, 128, True), (128, 32768, True), (32767, 128, False),
                        (128, 32767, False)):
        g, p = _structs(fi.Grid(n1, n2, 0.0, 0.0, 1 / 128, 1 / 128), W.params)
        ctx = ctypes.c_void_p()
        st = lib.fga_create(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p), 1, 1, None)
        assert (st == fga.FGA_EINVAL) == bad, (n1, n2, st)
        if st == fga.FGA_OK:
            lib.fga_destroy(ctx)


def test_null_context_calls_fail_cleanly():
    import paper_1304_3542_amd as fga
    lib = fga.load()
    assert lib.fga_destroy(None) == fga.FGA_OK
    assert lib.fga_set_velocity(None, None) == fga.FGA_EINVAL
    assert lib.fga_decompose(None, 1, None, None, None) == fga.FGA_EINVAL
    assert lib.fga_propagate(None, None, 1, 1) == fga.FGA_EINVAL
    assert lib.fga_reconstruct(None, None, 1, None) == fga.FGA_EINVAL
    assert lib.fga_sync_status(None, None) == fga.FGA_EINVAL


@pytest.mark.parametrize("name", fi.WORKLOADS)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_every_workload_passes_host_validation(name, precision):
    """The named workloads are valid for fga_create (argument checks run on
    the host before any device call, so without a GPU the call ends at the
    device query, never with FGA_EINVAL)."""
    import paper_1304_3542_amd as fga
    W = fi.workload(name, precision)
    g, p = _structs(W.grid, W.params)
    lib = fga.load()
    ctx = ctypes.c_void_p()
    st = lib.fga_create(ctypes.byref(ctx), ctypes.byref(g), ctypes.byref(p),
                        0 if precision == "fp64" else 1, max(W.nshots, 1), None)
    assert st != fga.FGA_EINVAL, lib.fga_last_error(None)
    if st == fga.FGA_OK:
        lib.fga_destroy(ctx)


@pytest.mark.parametrize("bad", [
    dict(np=(7, 8, 8)), dict(nq=(8, 5, 50)), dict(eps=0.0), dict(dp=(0.3, 0.0, 0.3)),
    dict(tau=2.0), dict(tau_win=1.0), dict(dt=0.0), dict(qs=(3, 0, 3)),
])
def test_create3_rejects_bad_params(bad):
    """The 3-D context checks its arguments on the host (no GPU needed)."""
    import paper_1304_3542_amd as fga
    import fga_inputs.d3 as i3
    g = i3.Grid3(26, 22, 19, 0.0, 0.1, -0.05, 1 / 24, 1 / 22, 1 / 20)
    p = i3.Params3(1 / 48, (2, 1, 3), (3, 4, 3), (8, 5, 5), (8, 6, 8), (0.3, 0.35, 0.28), 1e-5,
                   1e-16, 1e-16, 1e-3, 20).replace(**bad)
    gs = fga.fga3_grid(g.n1, g.n2, g.n3, g.o1, g.o2, g.o3, g.d1, g.d2, g.d3)
    ps = fga.fga3_params(p.eps, (ctypes.c_int32 * 3)(*p.qb), (ctypes.c_int32 * 3)(*p.qs),
                         (ctypes.c_int32 * 3)(*p.nq), (ctypes.c_int32 * 3)(*p.np),
                         (ctypes.c_double * 3)(*p.dp), p.tau, p.tau_fbi, p.tau_win, p.dt)
    lib = fga.load()
    ctx = ctypes.c_void_p()
    st = lib.fga3_create(ctypes.byref(ctx), ctypes.byref(gs), ctypes.byref(ps), 1, None)
    assert st == fga.FGA_EINVAL
    assert not ctx.value
    assert lib.fga3_last_error(None)

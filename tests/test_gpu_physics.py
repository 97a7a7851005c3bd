"""End-to-end physics of the GPU path (FP64, pinned elsewhere to the oracle)
against the exact solution of the wave equation: the FGA error is of order
eps, so it roughly halves when eps halves (grid spacing = eps, q every two
nodes, p-mesh spacing sqrt(eps)).  The size of the O(eps) constant is not
printed in the paper (parity unpinned); the rate is what is checked."""
import math

import numpy as np
import pytest

import fga_inputs as fi
import oracle.spectral as spectral
from gpu_helpers import gpu_run

pytestmark = pytest.mark.gpu


def _error(eps):
    n = int(round(1 / eps))
    g = fi.Grid(n, n, 0.0, 0.0, 1 / n, 1 / n)
    f0 = fi.wavepacket_source(g, (0.4, 0.5), 0.08, (1.0, 0.0), eps)
    f1 = fi.one_way_f1(g, f0, 1.0)
    dp = math.sqrt(eps)
    npp = 2 * int(math.ceil(2.0 / dp))      # p in [-2, 2]: the packet spectrum reaches ~1.6 at 1/64
    p = fi.Params(eps, 0, 0, 2, 2, n // 2, n // 2, npp, npp, dp, dp, 1e-6, 1e-16, 1e-16,
                  1e-3, 100)
    c = np.ones(g.shape)
    r = gpu_run(g, p, c, f0[None], f1[None], "fp64", capacity=3_000_000)
    if r["status"] != 0:                       # capacity: run again with the count needed
        r = gpu_run(g, p, c, f0[None], f1[None], "fp64", capacity=r["needed"] + 1024)
    assert r["status"] == 0 and r["status_end"][0] == 0
    ue = spectral.solve(f0, f1, g, 1.0, p.dt * p.nsteps)
    return float(np.linalg.norm(r["u"][0] - ue) / np.linalg.norm(ue))


def test_error_is_first_order_in_eps():
    errs = [_error(e) for e in (1 / 64, 1 / 128, 1 / 256)]
    print("relative L2 errors at eps = 1/64, 1/128, 1/256:", errs)
    assert errs[0] < 0.03
    assert 1.4 < errs[0] / errs[1] < 3.0 and 1.4 < errs[1] / errs[2] < 3.0, errs

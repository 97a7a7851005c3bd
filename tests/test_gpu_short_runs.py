"""Propagation over 0, 1 and 2 RK4 steps in the three amplitude modes
(integrated, closed form, divided differences) through the C ABI: zero steps
leave every beam field as the decomposition wrote it, and one or two steps
match the oracle's states at 1e-10 (the first and last coefficient requests
of a beam, and the closed form's root taken at the start and at the end,
meet here without a long run between them)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import pairwise_state_err, small_case

pytestmark = pytest.mark.gpu

MODES = {"integrated": {}, "closed": dict(amp_closed=1), "dd": dict(amp_closed=1, dz_divided=1)}


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("nsteps", [0, 1, 2])
def test_short_propagation_matches_oracle(mode, nsteps):
    import torch
    import paper_1304_3542_amd as fga
    g, p, c, f0, f1 = small_case(seed=91)
    p = p.replace(nsteps=nsteps, **MODES[mode])
    print(f"short run: mode {mode}, {nsteps} steps", flush=True)
    ctx = fga.FGA(g, p, "fp64", max_shots=1)
    ctx.set_velocity(torch.from_numpy(np.ascontiguousarray(c)).cuda())
    beams = fga.Beams(2 * p.nq1 * p.nq2 * p.np1 * p.np2, 1)
    ctx.decompose(torch.from_numpy(np.ascontiguousarray(f0)).cuda(),
                  torch.from_numpy(np.ascontiguousarray(f1)).cuda(), beams)
    nb = int(ctx.offsets(beams, 1)[-1])
    f_init = beams.f[:, :nb].cpu().numpy()
    ctx.propagate(beams, 1, nsteps)
    st = ctx.status()
    fT = beams.f[:, :nb].cpu().numpy()
    ctx.close()
    assert st[0] == 0 and nb > 0
    if nsteps == 0:
        np.testing.assert_array_equal(fT, f_init)
        return
    b, _ = oracle.forward(f0, f1, c, g, p)
    np.testing.assert_array_equal(f_init.shape[1], b.state.shape[0])
    assert pairwise_state_err(fT[6:].T, b.state) <= 1e-10

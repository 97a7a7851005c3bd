"""fga_trace_noalloc (receiver traces with the library's static scratch, no
allocation) against fga_trace on the same beams, through the C ABI: two
calls in a row, the second with a smaller input (fewer shots and receivers,
receivers in general position instead of one row), and the host-side
refusal of inputs whose partial sums exceed the scratch."""
import numpy as np
import pytest

import fga_inputs as fi
from gpu_helpers import small_case

pytestmark = pytest.mark.gpu


def _traces(fn, g, p, c, f0, f1, rec, every, nrec):
    import torch
    import paper_1304_3542_amd as fga
    ns = f0.shape[0]
    ctx = fga.FGA(g, p, "fp64", max_shots=ns)
    ctx.set_velocity(torch.from_numpy(c).cuda())
    beams = fga.Beams(2 * p.nq1 * p.nq2 * p.np1 * p.np2 * ns, ns)
    ctx.decompose(torch.from_numpy(np.ascontiguousarray(f0)).cuda(),
                  None if f1 is None else torch.from_numpy(np.ascontiguousarray(f1)).cuda(),
                  beams)
    rec_t = torch.from_numpy(rec).cuda()
    tr = torch.full((ns, nrec, rec.size), 3.0, dtype=torch.float64, device="cuda")
    fn(ctx.ctx, beams, ns, rec_t, every, nrec, tr)
    st = ctx.status()
    return tr.cpu().numpy(), st, ctx, beams


def test_noalloc_trace_matches_trace_twice():
    import paper_1304_3542_amd as fga
    g, p, c, f0, f1 = small_case(seed=71, nshots=3)
    p = p.replace(nsteps=40)
    cases = [
        (f0, f1, np.arange(5 * g.n1, 6 * g.n1, dtype=np.int32)),              # one row
        (f0[1:2], f1[1:2],
         fi.rng(72).choice(g.n1 * g.n2, 37, replace=False).astype(np.int32)),  # smaller
    ]
    for k, (a0, a1, rec) in enumerate(cases):
        ref, st0, _, _ = _traces(fga.fga_trace, g, p, c, a0, a1, rec, 8, 5)
        got, st1, _, _ = _traces(fga.fga_trace_noalloc, g, p, c, a0, a1, rec, 8, 5)
        assert st0[0] == 0 and st1[0] == 0
        assert np.abs(ref).max() > 0
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"call {k}: {a0.shape[0]} shots, {rec.size} receivers, rel err {err:.2e}",
              flush=True)
        assert err <= 1e-10


def test_noalloc_trace_refuses_oversized_scratch():
    """nshots * nrec * 8 bytes above the static scratch: FGA_EINVAL on the
    host, the output untouched."""
    import torch
    import paper_1304_3542_amd as fga
    g = fi.Grid(1024, 1024, 0.0, 0.0, 1 / 1024, 1 / 1024)
    p = fi.Params(1 / 1024, 0, 0, 1, 1, 1, 1, 2, 2, 0.1, 0.1, 1e-6, 1e-16, 1e-16, 1e-3, 10)
    ns = 3
    nrec = (16 << 20) // (8 * ns) + 1
    ctx = fga.FGA(g, p, "fp64", max_shots=ns)
    ctx.set_velocity(torch.ones((g.n2, g.n1), dtype=torch.float64, device="cuda"))
    beams = fga.Beams(16, ns)
    beams.offsets.zero_()
    rec = torch.arange(nrec, dtype=torch.int32, device="cuda")
    tr = torch.full((ns, 1, nrec), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(fga.FGAError) as err:
        fga.fga_trace_noalloc(ctx.ctx, beams, ns, rec, 1, 1, tr)
    assert err.value.status == fga.FGA_EINVAL
    torch.cuda.synchronize()
    assert bool((tr == 3.0).all())

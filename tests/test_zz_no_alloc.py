"""hsd_solve_noalloc (the solve for callers that cannot allocate device
memory) against hsd_solve, through the C ABI: the same kernels on a fixed
scratch array instead of the context's grown workspace, so the results are
the same bits.  Two calls in a row, the second smaller, then a batch too
large for the scratch, which is refused."""

import numpy as np
import pytest

import synth
from synth.fields import make_fields

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hsd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_4627_amd import hsd as h
    return h


def test_noalloc_matches_the_solve(hsd):
    w = synth.workload("c2_batched", n_cells=1000)
    ctx = hsd.Context(w.lam_cm)
    ids = [ctx.add_grain(g) for g in w.grains]
    u = torch.tensor(make_fields(w.lam_cm, w.field_recipe, w.n_cells), device="cuda")
    G, L = len(ids), w.n_lambda
    for n, sel in ((1000, ids), (300, ids[::3])):
        print(f"noalloc: {n} cells x {len(sel)} grains", flush=True)
        uu = u[:n].contiguous()
        je = torch.empty((n, len(sel), L), dtype=torch.float32, device="cuda")
        de = torch.empty((n, len(sel), 4), dtype=torch.float32, device="cuda")
        ctx.hsd_solve(uu, sel, je, de)
        ctx.hsd_sync()
        jn = torch.full_like(je, float("nan"))
        dn = torch.full_like(de, float("nan"))
        ctx.hsd_solve_noalloc(uu, sel, jn, dn)
        ctx.hsd_sync()
        assert torch.equal(jn, je) and torch.equal(dn, de)
    # more cells than the scratch holds: refused with the bytes it needs
    big = 2048
    ub = torch.tensor(make_fields(w.lam_cm, w.field_recipe, big), device="cuda")
    jb = torch.empty((big, G, L), dtype=torch.float32, device="cuda")
    with pytest.raises(hsd.HsdError, match="scratch"):
        ctx.hsd_solve_noalloc(ub, ids, jb, None)
    ctx.close()

"""roeam_residual_norms_noalloc (partials in the library's static device
buffer, nothing allocated) against roeam_residual_norms (partials in a buffer
the grid allocates), bit for bit: two calls in a row, the second on a smaller
grid, then the larger grid again; plus the rejection of an invalid call."""
import numpy as np
import pytest

import workloads
from gpu_util import ctx, say

pytestmark = pytest.mark.gpu


def _norms_pair(C, case):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid.from_case(C, case)
    r = P.residual(C, g, case.params, g.to_device(case.q0))
    out = torch.full((2 * g.rows,), float("nan"), dtype=torch.float64, device="cuda")
    a = P.residual_norms_noalloc(C, g, r, out).cpu().numpy().copy()
    b = P.residual_norms(C, g, r).cpu().numpy()
    torch.cuda.synchronize()
    return a, b, g.from_device(r)


def test_noalloc_norms_match_the_allocating_entry_point():
    C = ctx()
    # large grid with two scalars (6 rows, partials for the block cap), then a
    # small ragged one (fewer partials than the first left in the buffer),
    # then the large one again
    big = workloads.add_scalars(workloads.smooth_random_case(1500, 1100, 3, order=2, eps1=1.0), 2, seed=5)
    small = workloads.smooth_random_case(37, 21, 4, order=2, eps1=1.0)
    for name, case in (("1500x1100 + 2 scalars", big), ("37x21", small), ("1500x1100 again", big)):
        say(f"[noalloc] {name}")
        a, b, rg = _norms_pair(C, case)
        assert np.array_equal(a, b), (name, a, b)
        rows = rg.shape[0]
        flat = rg.reshape(rows, -1)
        ref = np.stack([np.sqrt((flat * flat).mean(axis=1)), np.abs(flat).max(axis=1)])
        assert np.allclose(a[0], ref[0], rtol=1e-13, atol=0) and np.array_equal(a[1], ref[1])


def test_noalloc_norms_reject_a_bad_call():
    import torch
    import paper_1711_09272_amd as P
    C = ctx()
    case = workloads.smooth_random_case(20, 20, 1, order=1)
    g = P.Grid.from_case(C, case)
    r = g.empty_state()
    out = torch.zeros(2 * g.rows, dtype=torch.float64, device="cuda")
    rc = P.lib().roeam_residual_norms_noalloc(C.h, g.h, None, __import__("ctypes").c_void_p(out.data_ptr()))
    assert rc == P.EINVAL
    with pytest.raises(ValueError):
        P.residual_norms_noalloc(C, g, r, torch.zeros(3, dtype=torch.float64, device="cuda"))

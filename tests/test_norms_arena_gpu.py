"""Residual norms (fixed-order reduction) and the caller-owned batch arena."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import ctx, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    return ctx()


def np_norms(r):
    rows = r.shape[0]
    flat = r.reshape(rows, -1)
    return np.stack([np.sqrt((flat * flat).mean(axis=1)), np.abs(flat).max(axis=1)])


@pytest.mark.parametrize("n,m,ns", [(2, 2, 0), (75, 37, 0), (45, 29, 2), (2048, 2048, 0), (513, 300, 1)])
def test_residual_norms_2d(C, n, m, ns):
    import torch
    import paper_1711_09272_amd as P
    case = workloads.smooth_random_case(n, m, 3, order=2, eps1=1.0)
    if ns:
        case = workloads.add_scalars(case, ns, seed=4)
    g = P.Grid.from_case(C, case)
    r = P.residual(C, g, case.params, g.to_device(case.q0))
    a = P.residual_norms(C, g, r).cpu().numpy()
    b = P.residual_norms(C, g, r).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(a, b)  # fixed-order reduction
    rg = g.from_device(r)
    ref = np_norms(rg)
    say(f"[norms] {n}x{m} ns={ns}: max rel diff {np.abs(a - ref).max() / np.abs(ref).max():.2e}")
    assert np.allclose(a[0], ref[0], rtol=1e-13, atol=0)
    assert np.array_equal(a[1], ref[1])  # max is exact
    if n * m <= 4096:
        r_or, sc = oracle.residual(case, with_scale=True)
        ref_or = np_norms(r_or)
        assert np.all(np.abs(a - ref_or) <= 1e-12 * sc.reshape(sc.shape[0], -1).max(axis=1))


def test_residual_norms_3d(C):
    import paper_1711_09272_amd as P
    case = workloads.smooth_random_case3(19, 13, 11, 5, order=2, eps1=1.0)
    g = P.Grid3.from_case(C, case)
    r = P.residual3(C, g, case.params, g.to_device(case.q0))
    a = P.residual_norms(C, g, r).cpu().numpy()
    ref = np_norms(g.from_device(r))
    assert np.allclose(a[0], ref[0], rtol=1e-13, atol=0) and np.array_equal(a[1], ref[1])


def test_batch_over_a_caller_owned_arena(C):
    """The pair through the batch engine over a torch tensor's storage gives the
    bits of the engine's own arena; the arena must be aligned."""
    import torch
    import paper_1711_09272_amd as P
    cases = [workloads.vortex(64, 0.01), workloads.vortex(48, 0.001)]

    def run(attach):
        c = P.Context(0)
        grids = [P.Grid.from_case(c, k) for k in cases]
        need = sum(g.footprint() for g in grids) + (1 << 20)
        if attach:
            arena = torch.empty(need // 8 + 64, dtype=torch.float64, device="cuda")
            with pytest.raises(P.RoeamError):
                P.batch_attach(c, arena[1:])  # 8-byte offset: not 256-byte aligned
            P.batch_attach(c, arena)
        else:
            P.batch_reserve(c, need)
        solves = [P.Solve(g, k.params, g.to_device(k.q0), 12, 0.0, g.empty_state()) for g, k in zip(grids, cases)]
        P.batch_submit(c, solves)
        P.batch_run(c, -1)
        out = []
        for s, g in zip(solves, grids):
            done, st, rc = P.batch_poll(c, s.ticket)
            assert done and rc == P.OK and st["steps"] == 12
            out.append(g.from_device(s.q_out))
        torch.cuda.synchronize()
        c.close()
        return out

    a, b = run(False), run(True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)

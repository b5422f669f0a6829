"""Helpers for the GPU parity tests: run a case through the HIP library and the
oracle on the same seeded input and measure the difference."""
import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ctx():
    import paper_1711_09272_amd as P
    return P.Context(0)


def gpu_residual(c, case, params=None, rate=False):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid.from_case(c, case)
    q = g.to_device(case.q0)
    rate_t = torch.zeros(1, dtype=torch.float64, device="cuda") if rate else None
    r = P.residual(c, g, params or case.params, q, rate_out=rate_t)
    torch.cuda.synchronize()
    out = g.from_device(r)
    if rate:
        return out, float(rate_t.item())
    return out


def residual_error(r_gpu, r_or, scale):
    """Cancellation-aware error per conserved row: max |dR| / max (sum_faces |F||S| / Omega)."""
    return np.array([np.abs(r_gpu[k] - r_or[k]).max() / scale[k].max() for k in range(4)])


def residual_error_cell(r_gpu, r_or, scale, floor=1e-6):
    """The same cell by cell: max over cells of |dR| / the cell's own flux
    scale, the scale floored at `floor` times the row's largest (a cell at rest
    carries no mass flux at all).  Catches errors in quiet regions that the
    row-wide norm weights down by the ratio of the scales."""
    out = []
    for k in range(r_or.shape[0]):
        s = np.maximum(scale[k], floor * scale[k].max())
        out.append((np.abs(r_gpu[k] - r_or[k]) / s).max())
    return np.array(out)


def gpu_run(c, case, nsteps=None, t_end=None, params=None, q0=None):
    import torch
    import paper_1711_09272_amd as P
    g = P.Grid.from_case(c, case)
    q = g.to_device(case.q0 if q0 is None else q0)
    st = P.step(c, g, params or case.params, q, case.nsteps if nsteps is None else nsteps,
                0.0, case.t_end if t_end is None else t_end)
    torch.cuda.synchronize()
    return g.from_device(q), st


def state_error(a, b):
    return np.abs(a - b).max() / np.abs(b).max()

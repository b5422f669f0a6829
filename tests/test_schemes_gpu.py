"""GPU parity of the comparison schemes and ablations the paper runs beside
Roe-AM (Sec. 7): classical Roe (Eq. 7 with Eqs. 8-12), Roe with Harten's
entropy fix (Eqs. 114-115), and the Roe-AM ablation bits (no Eq. 92, xi of
Eq. 13 or Eq. 46, dU_p of Eq. 17 or none).  Same bar as the Roe-AM cases:
FP64 residual <= 1e-12 (cancellation-aware), FP32 coefficients <= 1e-5,
states after n steps <= 1e-12."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import ctx, gpu_residual, gpu_run, residual_error, say, state_error
from test_parity_gpu import TOL32, TOL64, rough_case
from workloads import PERIODIC, SLIPWALL, TRANSMISSIVE

pytestmark = pytest.mark.gpu

V_NO_EQ92, V_XI_ROE, V_DUP_ROE, V_XI_EQ46, V_DUP_ZERO = 8, 16, 32, 64, 128


@pytest.fixture(scope="module")
def C():
    return ctx()


def scheme_cases():
    yield "roe_rough_o2", rough_case(47, 21, 31, order=2, scheme=1)
    yield "roe_rough_o1_walls", rough_case(35, 18, 32, bc=(TRANSMISSIVE, TRANSMISSIVE, SLIPWALL, SLIPWALL), order=1,
                                           scheme=1)
    yield "harten_rough_o2", rough_case(47, 21, 33, order=2, scheme=2, eps_lambda=0.1)
    yield "harten_strong_fix", rough_case(40, 19, 34, order=2, scheme=2, eps_lambda=0.6)
    yield "harten_smooth_nodes", workloads.smooth_random_case(44, 23, 35, nodes=True, order=2, scheme=2,
                                                              eps_lambda=0.2)
    yield "harten_zero_lambda", rough_case(30, 16, 36, order=2, scheme=2, eps_lambda=0.0)
    for bit, nm in ((V_NO_EQ92, "no_eq92"), (V_XI_ROE, "xi_roe"), (V_DUP_ROE, "dup_roe"), (V_XI_EQ46, "xi_eq46"),
                    (V_DUP_ZERO, "dup_zero")):
        yield f"roeam_{nm}", rough_case(45, 20, 40 + bit % 97, order=2, eps1=1.0, mach_ref=0.05, variant=bit)
    yield "roeam_fig6d", rough_case(39, 22, 50, order=2, eps1=1.0, variant=V_XI_ROE | V_DUP_ROE)
    yield "roeam_both_xi_both_dup", rough_case(39, 22, 51, order=2, eps1=1.0,
                                               variant=V_XI_ROE | V_XI_EQ46 | V_DUP_ROE | V_DUP_ZERO | V_NO_EQ92 | 4)
    yield "roeam_low_mach_dup_zero", workloads.vortex(96, 0.01, variant=V_DUP_ZERO)
    yield "roe_low_mach_vortex", workloads.vortex(96, 0.01, scheme=1)


CASES = list(scheme_cases())


@pytest.mark.parametrize("name,case", CASES, ids=[n for n, _ in CASES])
def test_scheme_residual_fp64(C, name, case):
    say(f"[scheme fp64] {name} {case.nx}x{case.ny} scheme={case.params.get('scheme', 0)} "
        f"variant={case.params.get('variant', 0)}")
    r_or, scale = oracle.residual(case, with_scale=True)
    r_gpu = gpu_residual(C, case)
    err = residual_error(r_gpu, r_or, scale)
    say(f"    err per row {err}")
    assert np.all(err <= TOL64), err


@pytest.mark.parametrize("name,case", [c for c in CASES if c[0] in ("roe_rough_o2", "harten_rough_o2",
                                                                    "roeam_fig6d", "roeam_xi_eq46")],
                         ids=lambda v: v if isinstance(v, str) else "")
def test_scheme_residual_fp32_flux(C, name, case):
    say(f"[scheme fp32-flux] {name}")
    r_or, scale = oracle.residual(case, with_scale=True)
    prm = dict(case.params)
    prm["precision"] = 1
    err = residual_error(gpu_residual(C, case, params=prm), r_or, scale)
    say(f"    err per row {err}")
    assert np.all(err <= TOL32), err


@pytest.mark.parametrize("scheme,eps_lambda", [(1, 0.0), (2, 0.1)])
def test_sod_classical_full_run(C, scheme, eps_lambda):
    """Sod 400 x 4 to t = 0.2 with the classical schemes (the paper's reference
    solutions for the shock-tube comparisons)."""
    case = workloads.sod(scheme=scheme, eps_lambda=eps_lambda)
    say(f"[step] sod scheme={scheme} eps_lambda={eps_lambda}")
    q_or, st_or = oracle.run(case)
    q_gpu, st = gpu_run(C, case)
    say(f"    steps {st['steps']} / {st_or['steps']} err {state_error(q_gpu, q_or):.3e}")
    assert st["steps"] == st_or["steps"] and st["t"] == st_or["t"] == 0.2
    assert state_error(q_gpu, q_or) <= TOL64


def test_odd_even_ablation_steps(C):
    """Odd-even channel (800 x 80 nodes) with the xi of Eq. (46), 15 steps."""
    case = workloads.odd_even(eps1=1.0, variant=V_XI_EQ46)
    say("[step] odd-even xi_eq46 15 steps")
    q_or, _ = oracle.run(case, nsteps=15)
    q_gpu, _ = gpu_run(C, case, nsteps=15)
    err = state_error(q_gpu, q_or)
    say(f"    err {err:.3e}")
    assert err <= TOL64


def test_scheme_argument_errors(C):
    import paper_1711_09272_amd as P
    case = workloads.sod()
    g = P.Grid.from_case(C, case)
    q = g.to_device(case.q0)
    for bad in ({"scheme": 3}, {"scheme": -1}, {"scheme": 2, "eps_lambda": -0.1},
                {"scheme": 2, "eps_lambda": float("nan")}, {"variant": 256}):
        prm = dict(case.params)
        prm.update(bad)
        with pytest.raises(P.RoeamError) as e:
            P.residual(C, g, prm, q)
        assert e.value.code == P.EINVAL, bad


# --- the paper's four-stage Runge-Kutta (time_scheme 2) -------------------------

def test_four_stage_sod_full_run(C):
    """Sec. 7.1's setting: first order in space, four-stage Runge-Kutta in time,
    Sod 400 x 4 to t = 0.2."""
    case = workloads.sod(time_scheme=2)
    q_or, st_or = oracle.run(case)
    q_gpu, st = gpu_run(C, case)
    err = state_error(q_gpu, q_or)
    say(f"[step] sod four-stage: steps {st['steps']} / {st_or['steps']} err {err:.3e}")
    assert st["steps"] == st_or["steps"] and st["t"] == st_or["t"] == 0.2
    assert err <= TOL64


@pytest.mark.parametrize("precision", [0, 1])
def test_four_stage_vortex_steps(C, precision):
    case = workloads.vortex(80, 0.01, time_scheme=2, precision=precision)
    q_or, st_or = oracle.run(case, nsteps=25, params=dict(case.params, precision=0))
    q_gpu, st = gpu_run(C, case, nsteps=25)
    err = state_error(q_gpu, q_or)
    say(f"[step] vortex four-stage precision {precision}: err {err:.3e}")
    assert st["steps"] == 25 and abs(st["t"] - st_or["t"]) <= (1e-13 if precision == 0 else 1e-6) * st_or["t"]
    assert err <= (TOL64 if precision == 0 else 1e-7)


def test_four_stage_profile_driver(C):
    import paper_1711_09272_amd as P
    case = workloads.vortex(64, 0.01, time_scheme=2)
    g = P.Grid.from_case(C, case)
    q = g.to_device(case.q0)
    stage_ms, launches = P.profile_step(C, g, case.params, q, 5)
    assert launches == 20 and all(t > 0 for t in stage_ms), stage_ms
    q_or, _ = oracle.run(case, nsteps=5)
    assert state_error(g.from_device(q), q_or) <= TOL64

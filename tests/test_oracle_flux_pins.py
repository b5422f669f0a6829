"""Face-level pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against an independent fact: a closed form, a
textbook identity (Roe's property, the eigen-decomposition of the Roe matrix),
a limit stated in the paper, or a property the paper claims for the final
scheme (full upwind, positivity at U -> 0, total-enthalpy preservation).
"""
import math

import numpy as np
import pytest

import oracle
import workloads

G = 1.4


def cons(W, g=G):
    rho, u, v, p = W
    return np.array([rho, rho * u, rho * v, p / (g - 1) + 0.5 * rho * (u * u + v * v)])


def euler_flux_n(W, nx, ny, g=G):
    """Normal flux nx F + ny G of the Euler equations, Eq. (1), from its definition."""
    rho, u, v, p = W
    E = p / (g - 1) + 0.5 * rho * (u * u + v * v)
    H = (E + p) / rho
    F = np.array([rho * u, rho * u * u + p, rho * u * v, rho * u * H])
    Gf = np.array([rho * v, rho * u * v, rho * v * v + p, rho * v * H])
    return nx * F + ny * Gf


def jacobian(u, v, H, nx, ny, g=G):
    """Textbook Jacobian dF_n/dQ of the 2-D Euler equations at (u, v, H)."""
    U = nx * u + ny * v
    q2 = u * u + v * v
    ph = 0.5 * (g - 1) * q2
    return np.array([
        [0.0, nx, ny, 0.0],
        [nx * ph - u * U, U + u * nx - (g - 1) * u * nx, u * ny - (g - 1) * v * nx, (g - 1) * nx],
        [ny * ph - v * U, v * nx - (g - 1) * u * ny, U + v * ny - (g - 1) * v * ny, (g - 1) * ny],
        [U * (ph - H), H * nx - (g - 1) * u * U, H * ny - (g - 1) * v * U, g * U],
    ])


def roe_params(**kw):
    return workloads.default_params(scheme=oracle.SCHEME_ROE, **kw)


PAIRS = workloads.random_prim_pairs(400, seed=workloads.SEED_BASE + 100)


# --- Eq. (98) -----------------------------------------------------------------

def test_f_closed_form_properties():
    # f(0) = 0, f = 1 for phi >= 1 since (phi sqrt(4+(1-phi^2)^2))^2 - (1+phi^2)^2 = (phi^2-1)^3
    assert oracle.f(0.0) == 0.0
    for phi in [1.5, 3.0, 40.0]:
        assert oracle.f(phi) == 1.0
    # near phi = 1 the gap is (phi^2-1)^3, below rounding: f is 1 to a few ulp
    for phi in [1.0, 1.0000001, 1.001]:
        assert abs(oracle.f(phi) - 1.0) <= 4e-16
    for phi in np.linspace(0.01, 0.99, 50):
        assert oracle.f(phi) < 1.0
    # monotone on [0,1]
    vals = [oracle.f(x) for x in np.linspace(0, 1, 200)]
    assert all(b >= a for a, b in zip(vals, vals[1:]))
    # f'(0) = sqrt(5)
    h = 1e-7
    assert abs(oracle.f(h) / h - math.sqrt(5.0)) < 1e-5
    # small-Mach order: f = O(M), so f^8 = O(M^8) (Sec. 3.1 first rule, n >= 1)
    assert oracle.f(1e-3) ** 8 < 1e-19


def test_f_table_values():
    # values worked by hand from Eq. (98): f(0.5) = 0.5 sqrt(4.5625)/1.25
    assert abs(oracle.f(0.5) - 0.4 * math.sqrt(4.5625)) < 1e-15
    assert abs(oracle.f(0.1) - 0.220952) < 1e-6
    assert abs(oracle.f(0.5) ** 8 - 0.283982) < 1e-6
    assert abs(oracle.f(0.8) ** 8 - 0.932397) < 1e-6


# --- Eq. (97) -----------------------------------------------------------------

def test_detector_ratio():
    assert oracle.detector_P(1.0, 1.0, 1.0, 1.0) == 1.0
    assert oracle.detector_P(2.0, 1.0, 1.0, 1.0) == 0.5
    assert oracle.detector_P(1.0, 1.0, 1.0, 4.0) == 0.25
    rng = np.random.default_rng(5)
    for _ in range(100):
        a = np.exp(rng.uniform(-3, 3, 4))
        P = oracle.detector_P(*a)
        assert P == oracle.detector_P(a[2], a[3], a[0], a[1])  # symmetric in the two cells
        assert 0 < P <= 1
        expect = min(min(a[0], a[2]) / max(a[0], a[2]), min(a[1], a[3]) / max(a[1], a[3]))
        assert abs(P - expect) <= 1e-16


# --- Physical flux, Eq. (4) vs Eq. (1) ----------------------------------------

def test_physical_flux_matches_euler_fluxes():
    WL, _, nrm = PAIRS
    for m in range(50):
        F = oracle.physical_flux(WL[m], *nrm[m])
        ref = euler_flux_n(WL[m], *nrm[m])
        assert np.allclose(F, ref, rtol=1e-14, atol=1e-14 * np.abs(ref).max())


# --- Roe averages: Roe's property ---------------------------------------------

def test_roe_property():
    WL, WR, nrm = PAIRS
    for m in range(len(WL)):
        nx, ny = nrm[m]
        _, d = oracle.face_flux(workloads.default_params(), WL[m], WR[m], nx, ny)
        A = jacobian(d["u"], d["v"], d["H"], nx, ny)
        lhs = euler_flux_n(WR[m], nx, ny) - euler_flux_n(WL[m], nx, ny)
        rhs = A @ (cons(WR[m]) - cons(WL[m]))
        scale = np.abs(euler_flux_n(WR[m], nx, ny)).max() + np.abs(euler_flux_n(WL[m], nx, ny)).max()
        assert np.abs(lhs - rhs).max() <= 1e-13 * scale
        # Roe-averaged sound speed: eigenvalues of A are U, U, U -+ c
        ev = np.sort(np.linalg.eigvals(A).real)
        U = nx * d["u"] + ny * d["v"]
        assert np.allclose(ev, np.sort([U - d["c"], U, U, U + d["c"]]), rtol=1e-10, atol=1e-10 * (abs(U) + d["c"]))
        assert d["rho"] == pytest.approx(math.sqrt(WL[m][0] * WR[m][0]), rel=1e-15)


# --- Classical Roe: scale form (Eqs. 13-17 in Eq. 7) = eigen form (Eq. 5) -----

def _eigen_roe(WL, WR, nx, ny, d, fix_eps=None):
    A = jacobian(d["u"], d["v"], d["H"], nx, ny)
    lam, R = np.linalg.eig(A)  # complex R: the double eigenvalue U may come back as a conjugate pair
    al = np.abs(lam.real)
    if fix_eps is not None:  # Harten's fix, Eqs. (114)-(115)
        h = fix_eps * al.max()
        al = np.where(al < h, 0.5 * (al * al / h + h), al)
    dQ = cons(WR) - cons(WL)
    diss = (R @ np.diag(al) @ np.linalg.solve(R, dQ.astype(complex))).real
    return 0.5 * (euler_flux_n(WL, nx, ny) + euler_flux_n(WR, nx, ny)) - 0.5 * diss


@pytest.mark.parametrize("scheme,eps", [(oracle.SCHEME_ROE, None), (oracle.SCHEME_ROE_HARTEN, 0.2)])
def test_classical_roe_equals_eigen_form(scheme, eps):
    WL, WR, nrm = PAIRS
    prm = workloads.default_params(scheme=scheme, eps_lambda=eps or 0.1)
    for m in range(200):
        nx, ny = nrm[m]
        F, d = oracle.face_flux(prm, WL[m], WR[m], nx, ny)
        ref = _eigen_roe(WL[m], WR[m], nx, ny, d, eps)
        scale = np.abs(euler_flux_n(WL[m], nx, ny)).max() + np.abs(euler_flux_n(WR[m], nx, ny)).max()
        assert np.abs(F - ref).max() <= 1e-11 * scale, (m, F, ref)


# --- Roe-AM: reductions and claimed properties ----------------------------------

def test_theta_one_reduces_to_roe_dUp():
    """Eq. (18)/(89) becomes Eq. (17) when M_ref >= 1 (theta = 1), Sec. 3.1."""
    WL, WR, nrm = PAIRS
    prm = workloads.default_params(mach_ref=1.0, variant=oracle.V_NO_EQ92, s1_mode=1)
    for m in range(200):
        _, d = oracle.face_flux(prm, WL[m], WR[m], *nrm[m])
        assert d["theta"] == 1.0
        assert d["ct"] == pytest.approx(d["c"], rel=1e-15)
        gate = 1.0 - oracle.f(d["M"]) ** 8
        eq17 = max(0.0, d["c"] - abs(d["U"])) * d["dp"] / (d["rho"] * d["c"] ** 2)
        # 1 - f^8(M) cancels near M = 1: compare on the scale of the ungated term
        assert abs(d["dUp"] - gate * eq17) <= 1e-13 * abs(eq17) + 1e-300


def test_low_mach_dUp_limit_at_zero_normal_velocity():
    """U = 0: the bracket of Eq. (89) is c~ = c sqrt(theta), so the mass-flux term
    -rho dUp / 2 equals -dp / (2 c~) (Eq. 57 with the s1 [1 - f^8(M)] gate)."""
    rng = np.random.default_rng(11)
    for _ in range(100):
        mref = 10 ** rng.uniform(-3, -1)
        rho = np.exp(rng.uniform(-0.5, 0.5, 2))
        p = np.exp(rng.uniform(-0.05, 0.05, 2))
        vt = rng.uniform(0.1, 0.9) * mref * math.sqrt(G)  # tangential velocity, M < M_ref... mixed
        WL = np.array([rho[0], 0.0, vt, p[0]])
        WR = np.array([rho[1], 0.0, vt * 1.01, p[1]])
        prm = workloads.default_params(mach_ref=mref, s1_mode=1)
        F, d = oracle.face_flux(prm, WL, WR, 1.0, 0.0)
        assert d["U"] == 0.0
        theta = d["theta"]
        assert theta == pytest.approx(max(mref ** 2, d["M"] ** 2), rel=1e-14)
        ct = d["c"] * math.sqrt(theta)
        assert d["ct"] == pytest.approx(ct, rel=1e-14)
        gate = 1.0 - oracle.f(d["M"]) ** 8
        assert -0.5 * d["rho"] * d["dUp"] == pytest.approx(-gate * d["dp"] / (2 * ct), rel=1e-12)


def _supersonic_pair(rng, mach_n, sign=1.0):
    rho = np.exp(rng.uniform(-0.5, 0.5, 2))
    p = np.exp(rng.uniform(-0.5, 0.5, 2))
    c = np.sqrt(G * p / rho)
    th = rng.uniform(0, 2 * math.pi)
    n = np.array([math.cos(th), math.sin(th)])
    t = np.array([-n[1], n[0]])
    W = []
    for k in range(2):
        un = sign * mach_n * c.max() * rng.uniform(1.0, 1.3)
        ut = rng.uniform(-1, 1) * c[k]
        V = un * n + ut * t
        W.append(np.array([rho[k], V[0], V[1], p[k]]))
    return W[0], W[1], n


@pytest.mark.parametrize("eps1", [0.0, 1.0])
def test_full_upwind_supersonic(eps1):
    """Sec. 4.2 / Eq. (44), claimed for the final scheme in Sec. 6.2: for U >= c the
    flux is the left physical flux (right one for U <= -c), in all four rows."""
    rng = np.random.default_rng(7)
    prm = workloads.default_params(eps1=eps1, mach_ref=0.01, s1_mode=0)
    for sign in (1.0, -1.0):
        for _ in range(200):
            WL, WR, n = _supersonic_pair(rng, 2.5, sign)
            F, d = oracle.face_flux(prm, WL, WR, n[0], n[1], s1=rng.uniform(0, 1))
            assert d["Mbar"] >= 1.0 and d["M"] >= 1.0
            up = euler_flux_n(WL if sign > 0 else WR, n[0], n[1])
            assert np.abs(F - up).max() <= 1e-13 * np.abs(up).max()


def test_printed_ungated_xi_is_not_full_upwind():
    """Reading D1: without the [1 - f^8(Mbar)] gate of Eq. (68), Eq. (86) as printed
    does not give the full-upwind flux claimed in Sec. 6.2."""
    rng = np.random.default_rng(8)
    prm = workloads.default_params(variant=oracle.V_XI_UNGATED)
    bad = 0
    for _ in range(50):
        WL, WR, n = _supersonic_pair(rng, 2.5)
        F, _ = oracle.face_flux(prm, WL, WR, n[0], n[1])
        up = euler_flux_n(WL, n[0], n[1])
        bad += np.abs(F - up).max() > 1e-6 * np.abs(up).max()
    assert bad > 40


def test_velocity_positivity_at_zero_normal_velocity():
    """Eqs. (65)-(66): for U -> 0 and M > 1 the mass flux is rho_L (U_R+U_L)/2 for
    U > 0 and rho_R (U_R+U_L)/2 for U < 0, up to the O(U dU / c) term of dU_u."""
    rng = np.random.default_rng(9)
    prm = workloads.default_params(mach_ref=0.1)
    for _ in range(300):
        rho = np.exp(rng.uniform(-1, 1, 2))
        p = np.exp(rng.uniform(-0.3, 0.3, 2))
        c = np.sqrt(G * p / rho)
        sgn = rng.choice([-1.0, 1.0])
        UL = sgn * 1e-6 * rng.uniform(0.5, 1.5)
        dU = rng.uniform(-1e-3, 1e-3)
        UR = UL + dU
        if (UL + UR) * sgn <= 0:
            continue
        vt = 3.0 * c.max()  # tangential: M > 1
        WL = np.array([rho[0], UL, vt, p[0]])
        WR = np.array([rho[1], UR, vt * 1.001, p[1]])
        F, d = oracle.face_flux(prm, WL, WR, 1.0, 0.0, s1=1.0)
        if d["U"] * sgn <= 0:
            continue
        expect = (rho[0] if sgn > 0 else rho[1]) * (UL + UR) / 2
        tol = 2.0 * (abs(d["dUuR"]) + abs(d["dUuL"])) * rho.max() + 1e-15
        assert abs(F[0] - expect) <= tol


def test_total_enthalpy_preservation():
    """Eq. (49): with H_L = H_R the energy flux is H times the mass flux."""
    WL, WR, nrm = PAIRS
    prm = workloads.default_params(eps1=1.0, mach_ref=0.05)
    n_checked = 0
    for m in range(len(WL)):
        L, R = WL[m].copy(), WR[m].copy()
        H = G * L[3] / ((G - 1) * L[0]) + 0.5 * (L[1] ** 2 + L[2] ** 2)
        pR = (G - 1) / G * R[0] * (H - 0.5 * (R[1] ** 2 + R[2] ** 2))
        if pR <= 0:
            continue
        R[3] = pR
        F, d = oracle.face_flux(prm, L, R, *nrm[m], s1=0.7)
        assert d["H"] == pytest.approx(H, rel=1e-13)
        assert F[3] == pytest.approx(H * F[0], rel=1e-11, abs=1e-12 * H * abs(L[0] * L[1]) + 1e-14)
        n_checked += 1
    assert n_checked > 100


def test_consistency_equal_states():
    """Equal left and right states give the physical flux (consistency of Eq. 2)."""
    WL, _, nrm = PAIRS
    for eps1 in (0.0, 1.0):
        prm = workloads.default_params(eps1=eps1, mach_ref=0.01)
        for m in range(100):
            F, _ = oracle.face_flux(prm, WL[m], WL[m], *nrm[m], s1=1.0)
            assert np.array_equal(F, oracle.physical_flux(WL[m], *nrm[m]))


def test_swap_and_reverse_normal():
    """F(R, L, -n) = -F(L, R, n): the scheme has no preferred side."""
    WL, WR, nrm = PAIRS
    prm = workloads.default_params(eps1=1.0, mach_ref=0.01)
    for m in range(len(WL)):
        F, _ = oracle.face_flux(prm, WL[m], WR[m], *nrm[m], s1=0.5)
        Fr, _ = oracle.face_flux(prm, WR[m], WL[m], -nrm[m][0], -nrm[m][1], s1=0.5)
        scale = np.abs(euler_flux_n(WL[m], *nrm[m])).max() + np.abs(euler_flux_n(WR[m], *nrm[m])).max()
        assert np.abs(F + Fr).max() <= 1e-13 * scale


def test_rotated_speed_limits():
    """Eqs. (103)-(109): with n1 = n (no velocity jump) f_rr = |U|; with n1 normal
    to n, alpha_1 = 0 and f_rr = |U_2| with n2 = n (reading D7: unit n2)."""
    prm = workloads.default_params(eps1=1.0, u_ref=1.0)
    W = np.array([1.0, 0.3, 0.2, 1.0])
    _, d = oracle.face_flux(prm, W, W, 1.0, 0.0)
    assert d["frr"] == pytest.approx(abs(d["U"]), rel=1e-15)
    WR = W.copy()
    WR[2] += 0.1  # jump purely along y, face normal along x
    _, d = oracle.face_flux(prm, W, WR, 1.0, 0.0)
    assert d["frr"] == pytest.approx(abs(d["U"]), rel=1e-14)
    # jump along the normal: n1 = n, s = 0
    WR = W.copy()
    WR[1] += 0.1
    _, d = oracle.face_flux(prm, W, WR, 1.0, 0.0)
    assert d["frr"] == pytest.approx(abs(d["U"]), rel=1e-14)
    # oblique jump: |alpha1 U1| + |alpha2 U2| with unit vectors
    WR = W.copy()
    WR[1] += 0.1
    WR[2] += 0.1
    _, d = oracle.face_flux(prm, W, WR, 1.0, 0.0)
    n1 = np.array([1.0, 1.0]) / math.sqrt(2)
    n2 = np.array([1.0, -1.0]) / math.sqrt(2)
    Vh = np.array([d["u"], d["v"]])
    expect = abs(n1[0] * (n1 @ Vh)) + abs(n2[0] * (n2 @ Vh))
    assert d["frr"] == pytest.approx(expect, rel=1e-14)
    # for any direction the two unit directions resolve the face normal: alpha1^2 + alpha2^2 = 1,
    # so f_rr <= |V| (Cauchy-Schwarz)
    WL_, WR_, nrm = PAIRS
    for m in range(100):
        _, d = oracle.face_flux(prm, WL_[m], WR_[m], *nrm[m])
        assert d["frr"] <= math.hypot(d["u"], d["v"]) * (1 + 1e-14)


@pytest.mark.parametrize("UL,UR,kind", [(0.2, 0.5, "eq72"), (-0.6, -0.1, "eq72"), (0.05, 0.9, "eq72"),
                                         (0.5, 0.2, "unchanged"), (-0.1, -0.6, "unchanged"),
                                         (2.0, 2.5, "unchanged"), (-2.5, -2.0, "unchanged"),
                                         (-0.3, 0.4, "opposite")])
def test_expansion_fix_eq70_eq72(UL, UR, kind):
    """Eqs. (70)-(72).  Eq. (92) weights the correction of Eq. (70),
    [sign(U + c) - sign(U - c)] max(0, U_R - U_L) / 4, by f(Mbar); the Eq. (73)
    reading bit weights it by f^8(Mbar).  Recovering the unweighted correction
    from both weights (dividing by f and f^8 of the oracle's Mbar) must give one
    value, and Eq. (70)'s |U|' = |U| - correction must be what Eq. (72) states:
    with U = (U_R + U_L)/2 (equal densities and pressures make the Roe average
    arithmetic), |U| < c and U_R > U_L it is min(|U_L|, |U_R|) when U_L and U_R
    have one sign; |U| otherwise (compression, or |U| >= c).  With opposite
    signs Eq. (70) leaves |U| - dU/2 < 0 (reading D4: no clamp)."""
    prm = workloads.default_params(mach_ref=1.0)
    WL = np.array([1.0, UL, 0.0, 1.0])
    WR = np.array([1.0, UR, 0.0, 1.0])
    _, d = oracle.face_flux(prm, WL, WR, 1.0, 0.0)
    _, d8 = oracle.face_flux(dict(prm, variant=oracle.V_EXPFIX_F8), WL, WR, 1.0, 0.0)
    assert d["U"] == pytest.approx(0.5 * (UL + UR), rel=1e-15, abs=1e-16)  # Eq. (71)
    assert d8["Mbar"] == d["Mbar"] and d8["U"] == d["U"]
    fb = oracle.f(d["Mbar"])
    assert 0.0 < fb <= 1.0
    corr = (abs(d["U"]) - d["absUp"]) / fb
    corr8 = (abs(d8["U"]) - d8["absUp"]) / fb ** 8
    # the f^8 weight is tiny at small Mbar: allow a few ulp of |U| divided by it
    assert corr == pytest.approx(corr8, rel=1e-11, abs=4e-16 * max(1.0, abs(d["U"])) / fb ** 8)
    eq70 = abs(d["U"]) - corr
    subsonic = abs(d["U"]) < d["c"]
    if kind == "eq72":
        assert subsonic and UR > UL and UL * UR > 0  # the branch of Eq. (72) is taken
        assert corr > 0
        assert eq70 == pytest.approx(min(abs(UL), abs(UR)), rel=1e-13)
    elif kind == "unchanged":
        assert not (subsonic and UR > UL)
        assert corr == 0.0 and d["absUp"] == abs(d["U"])
    else:
        assert subsonic and UR > UL and UL * UR < 0
        assert eq70 < 0.0 and eq70 < min(abs(UL), abs(UR))

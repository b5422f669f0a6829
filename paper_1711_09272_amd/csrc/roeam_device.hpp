// roeam_device.hpp -- device-side building blocks of the gfx950 Roe-AM library:
// solve descriptor, boundary-mapped cell fetch, face geometry, the Roe-AM
// numerical flux of Eqs. (85)-(109) and the explicit-rate rule.
//
// 2-D form of the paper's equations: w = 0, n_z = 0, four conserved rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace roeam {

enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_SLIPWALL = 2, BC_DIRICHLET = 3 };
enum { SIDE_W = 0, SIDE_E = 1, SIDE_S = 2, SIDE_N = 3 };
enum : unsigned { V_XI_UNGATED = 1u, V_EXPFIX_F8 = 2u, V_CLAMP_UPRIME = 4u };

// Per-solve time-integration state, resident in device memory.  Written only
// by the single-thread dt kernel, except rate_bits (atomicMax from stage
// kernels) and nonphys (atomicOr).
struct alignas(64) Slot {
    double t, dt, t_next, t_end, cfl;
    double rate_last, dt_last;
    unsigned long long rate_bits;  // bit pattern of a non-negative double: atomicMax orders it
    long long steps, max_steps;
    int active;
    int nonphys;
    int done;                      // t reached t_end or a non-physical state
    int pad;
};

// Everything a stage kernel needs about one solve.  Passed by value as a
// kernel argument for single-grid launches, or read from a device array in
// batched launches.
struct DevSolve {
    int nx, ny;
    long long pitch, plane;
    int metric;                 // 0 uniform, 1 node coordinates
    double dx, dy, area;        // uniform spacing and cell area
    const double *xn, *yn;      // nodes [(ny+1)][(nx+1)]
    int bc[4];
    double bcw[4][4];           // Dirichlet states, primitive (rho, u, v, p)
    // scheme
    double gamma, gm1, mr2, u_ref, eps1, eps2, cfl;
    int s1_mode, order, precision;
    unsigned variant;
    // state
    double *q, *qa, *qb;
    Slot *slot;
    int tiles_x, tiles_y;       // tiles of this solve (batched work lists)
};

// ---------------------------------------------------------------------------
// scalar helpers
// ---------------------------------------------------------------------------
template <typename R> __device__ __forceinline__ R sgn(R x) { return (R)((x > (R)0) - (x < (R)0)); }
template <typename R> __device__ __forceinline__ R rmin(R a, R b) { return a < b ? a : b; }
template <typename R> __device__ __forceinline__ R rmax(R a, R b) { return a > b ? a : b; }

// Division and square root in the flux-coefficient precision.  FP64 uses the
// correctly rounded operators; FP32 uses the hardware reciprocal and square
// root (about 1 ulp), enough for coefficients whose error budget is 1e-5.
__device__ __forceinline__ double rdiv(double a, double b) { return a / b; }
__device__ __forceinline__ double rsqrt_(double a) { return sqrt(a); }
__device__ __forceinline__ float rdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float rsqrt_(float a) { return __builtin_amdgcn_sqrtf(a); }

// Eq. (98): f(phi) = min(phi sqrt(4 + (1 - phi^2)^2) / (1 + phi^2), 1).
template <typename R> __device__ __forceinline__ R fswitch(R phi)
{
    R one_minus = (R)1 - phi * phi;
    R val = rdiv(phi * rsqrt_((R)4 + one_minus * one_minus), (R)1 + phi * phi);
    return rmin(val, (R)1);
}
// f^8 as the eighth power (repeated squaring).
template <typename R> __device__ __forceinline__ R pow8(R x)
{
    R x2 = x * x;
    R x4 = x2 * x2;
    return x4 * x4;
}

// Eq. (97): detector ratio of two neighbouring cells, min of the pressure and
// density ratios, each taken below one.
__device__ __forceinline__ double detector_P(double pA, double rA, double pB, double rB)
{
    double a = rmin(pA, pB) / rmax(pA, pB);
    double b = rmin(rA, rB) / rmax(rA, rB);
    return rmin(a, b);
}

// ---------------------------------------------------------------------------
// state access
// ---------------------------------------------------------------------------
__device__ __forceinline__ void to_prim(double gm1, double q0, double q1, double q2, double q3, double W[4])
{
    double rho = q0;
    double u = q1 / rho, v = q2 / rho;
    W[0] = rho;
    W[1] = u;
    W[2] = v;
    W[3] = gm1 * (q3 - 0.5 * rho * (u * u + v * v));
}

__device__ __forceinline__ void load_prim(const DevSolve &S, const double *__restrict__ q, int i, int j, double W[4])
{
    long long idx = (long long)j * S.pitch + i;
    to_prim(S.gm1, q[idx], q[S.plane + idx], q[2 * S.plane + idx], q[3 * S.plane + idx], W);
}

__device__ __forceinline__ void xface_vec(const DevSolve &S, int i, int j, double &sx, double &sy)
{
    if (S.metric == 0) { sx = S.dy; sy = 0.0; return; }
    long long nxn = S.nx + 1;
    double ddx = S.xn[(long long)(j + 1) * nxn + i] - S.xn[(long long)j * nxn + i];
    double ddy = S.yn[(long long)(j + 1) * nxn + i] - S.yn[(long long)j * nxn + i];
    sx = ddy;
    sy = -ddx;
}
__device__ __forceinline__ void yface_vec(const DevSolve &S, int i, int j, double &sx, double &sy)
{
    if (S.metric == 0) { sx = 0.0; sy = S.dx; return; }
    long long nxn = S.nx + 1;
    double ddx = S.xn[(long long)j * nxn + i + 1] - S.xn[(long long)j * nxn + i];
    double ddy = S.yn[(long long)j * nxn + i + 1] - S.yn[(long long)j * nxn + i];
    sx = -ddy;
    sy = ddx;
}
// Unit normal and length of a face vector; axis-aligned faces of uniform
// grids are exact.
__device__ __forceinline__ void unit_normal(const DevSolve &S, double sx, double sy, double &nx, double &ny, double &len)
{
    if (S.metric == 0) {
        if (sy == 0.0) { nx = 1.0; ny = 0.0; len = sx; }
        else { nx = 0.0; ny = 1.0; len = sy; }
        return;
    }
    len = sqrt(sx * sx + sy * sy);
    nx = sx / len;
    ny = sy / len;
}
__device__ __forceinline__ double cell_area(const DevSolve &S, int i, int j)
{
    if (S.metric == 0) return S.area;
    long long nxn = S.nx + 1;
    const double *x = S.xn, *y = S.yn;
    long long r0 = (long long)j * nxn, r1 = (long long)(j + 1) * nxn;
    double x00 = x[r0 + i], y00 = y[r0 + i];
    double x10 = x[r0 + i + 1], y10 = y[r0 + i + 1];
    double x11 = x[r1 + i + 1], y11 = y[r1 + i + 1];
    double x01 = x[r1 + i], y01 = y[r1 + i];
    return 0.5 * ((x11 - x00) * (y01 - y10) - (x01 - x10) * (y11 - y00));
}

__device__ __forceinline__ void reflect(double W[4], double nx, double ny)
{
    double vn = W[1] * nx + W[2] * ny;
    W[1] = W[1] - 2.0 * vn * nx;
    W[2] = W[2] - 2.0 * vn * ny;
}

// Primitive state of cell (i, j) where j is inside the grid and i may lie in
// the two ghost columns on either side.
__device__ __forceinline__ void fetch_prim_x(const DevSolve &S, const double *__restrict__ q, int i, int j, double W[4])
{
    if (i >= 0 && i < S.nx) { load_prim(S, q, i, j, W); return; }
    int side = i < 0 ? SIDE_W : SIDE_E;
    int kind = S.bc[side];
    if (kind == BC_DIRICHLET) {
        for (int k = 0; k < 4; ++k) W[k] = S.bcw[side][k];
        return;
    }
    int is;
    if (kind == BC_PERIODIC) is = i < 0 ? i + S.nx : i - S.nx;
    else if (kind == BC_TRANSMISSIVE) is = i < 0 ? 0 : S.nx - 1;
    else is = i < 0 ? -i - 1 : 2 * S.nx - 1 - i;
    load_prim(S, q, is, j, W);
    if (kind == BC_SLIPWALL) {
        double sx, sy, nx, ny, len;
        xface_vec(S, i < 0 ? 0 : S.nx, j, sx, sy);
        unit_normal(S, sx, sy, nx, ny, len);
        reflect(W, nx, ny);
    }
}

// Primitive state of any cell within two layers of the grid: the x rule, then
// the y rule (which also defines the corners).
__device__ __forceinline__ void fetch_prim(const DevSolve &S, const double *__restrict__ q, int i, int j, double W[4])
{
    if (j >= 0 && j < S.ny) { fetch_prim_x(S, q, i, j, W); return; }
    int side = j < 0 ? SIDE_S : SIDE_N;
    int kind = S.bc[side];
    if (kind == BC_DIRICHLET) {
        for (int k = 0; k < 4; ++k) W[k] = S.bcw[side][k];
        return;
    }
    int js;
    if (kind == BC_PERIODIC) js = j < 0 ? j + S.ny : j - S.ny;
    else if (kind == BC_TRANSMISSIVE) js = j < 0 ? 0 : S.ny - 1;
    else js = j < 0 ? -j - 1 : 2 * S.ny - 1 - j;
    fetch_prim_x(S, q, i, js, W);
    if (kind == BC_SLIPWALL) {
        int ic = i < 0 ? 0 : (i > S.nx - 1 ? S.nx - 1 : i);
        double sx, sy, nx, ny, len;
        yface_vec(S, ic, j < 0 ? 0 : S.ny, sx, sy);
        unit_normal(S, sx, sy, nx, ny, len);
        reflect(W, nx, ny);
    }
}

// ---------------------------------------------------------------------------
// Roe-AM numerical flux, Eqs. (85)-(109), per unit face length.
// R is the precision of the dissipation coefficients; the central term, the
// jumps of Eq. (85) and the final assembly stay in FP64.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void roeam_flux(const DevSolve &S, const double WL[4], const double WR[4], double nx,
                                           double ny, double s1d, double F[4])
{
    const double g = S.gamma;
    const double rL = WL[0], uL = WL[1], vL = WL[2], pL = WL[3];
    const double rR = WR[0], uR = WR[1], vR = WR[2], pR = WR[3];

    // side quantities, Eq. (4)
    double UL = nx * uL + ny * vL;
    double UR = nx * uR + ny * vR;
    double HL = (pL / S.gm1 + 0.5 * rL * (uL * uL + vL * vL) + pL) / rL;
    double HR = (pR / S.gm1 + 0.5 * rR * (uR * uR + vR * vR) + pR) / rR;
    double PsiL[4] = {rL, rL * uL, rL * vL, rL * HL};
    double PsiR[4] = {rR, rR * uR, rR * vR, rR * HR};
    double FbL[4] = {UL * rL, UL * PsiL[1] + pL * nx, UL * PsiL[2] + pL * ny, UL * PsiL[3]};
    double FbR[4] = {UR * rR, UR * PsiR[1] + pR * nx, UR * PsiR[2] + pR * ny, UR * PsiR[3]};

    // jumps stay FP64 (low-Mach pressure differences cancel otherwise)
    double dUd = UR - UL;
    double dpd = pR - pL;
    double dPsi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) dPsi[k] = PsiR[k] - PsiL[k];

    // Roe averages (sqrt(rho) weights)
    const R rr = rsqrt_((R)rdiv((R)rR, (R)rL));
    const R inv1r = rdiv((R)1, (R)1 + rr);
    const R rho = rr * (R)rL;
    const R u = ((R)uL + rr * (R)uR) * inv1r;
    const R v = ((R)vL + rr * (R)vR) * inv1r;
    const R H = ((R)HL + rr * (R)HR) * inv1r;
    const R c = rsqrt_((R)S.gm1 * (H - (R)0.5 * (u * u + v * v)));
    const R U = (R)nx * u + (R)ny * v;
    const R dU = (R)dUd, dp = (R)dpd;
    const R s1 = (R)s1d;

    // Mach numbers, Eqs. (93)-(94); f, f^8 of Eq. (98)
    const R cL = rsqrt_(rdiv((R)g * (R)pL, (R)rL)), cR = rsqrt_(rdiv((R)g * (R)pR, (R)rR));
    const R M = (R)0.5 * (rdiv(rsqrt_((R)(uL * uL + vL * vL)), cL) + rdiv(rsqrt_((R)(uR * uR + vR * vR)), cR));
    const R absU = U < (R)0 ? -U : U;
    const R Mbar = rdiv(absU, c);
    const R fM = fswitch(M), f8M = pow8(fM);
    const R fMbar = fswitch(Mbar), f8Mbar = pow8(fMbar);

    // preconditioning, Eqs. (99)-(101)
    const R theta = rmin(rmax((R)S.mr2, M * M), (R)1);
    const R omt = (R)1 - theta;
    const R ct = (R)0.5 * rsqrt_((R)4 * c * c * theta + omt * omt * U * U);
    const R Ut = (R)0.5 * ((R)1 + theta) * U;

    // expansion-shock fix, Eq. (92)
    const R w = (S.variant & V_EXPFIX_F8) ? f8Mbar : fMbar;
    R absUp = absU - w * (sgn(U + c) - sgn(U - c)) * rmax((R)0, dU) / (R)4;
    if (S.variant & V_CLAMP_UPRIME) absUp = rmax(absUp, (R)0);

    // basic upwind dissipation xi, Eq. (86) with the Eq. (68) gate
    const R gate = (S.variant & V_XI_UNGATED) ? (R)1 : (R)1 - f8Mbar;
    const R ULR = (R)(0.5 * (UR + UL));
    const R xi_pos = (ULR < (R)0 ? -ULR : ULR) + gate * ((R)0.5 * dU);
    R xi = xi_pos;
    if (S.eps1 != 0.0) {
        // modified entropy fix f_ef (Eq. 102) and rotated speed f_rr (Eqs. 103-109)
        const R fef = (R)S.eps2 * c;
        const R du = (R)(uR - uL), dv = (R)(vR - vL);
        const R dV = rsqrt_(du * du + dv * dv);
        R n1x = (R)nx, n1y = (R)ny;
        if (!(dV < (R)(1e-5 * S.u_ref) || dV == (R)0)) {
            const R idV = rdiv((R)1, dV);
            n1x = du * idV;
            n1y = dv * idV;
        }
        const R alpha1 = n1x * (R)nx + n1y * (R)ny;
        const R U1 = n1x * u + n1y * v;
        const R sz = n1x * (R)ny - n1y * (R)nx;
        R a2U2 = (R)0;
        if (sz != (R)0) {
            const R sg = sgn(sz);
            const R n2x = -sg * n1y, n2y = sg * n1x;
            a2U2 = (n2x * (R)nx + n2y * (R)ny) * (n2x * u + n2y * v);
        }
        const R a1U1 = alpha1 * U1;
        const R frr = (a1U1 < (R)0 ? -a1U1 : a1U1) + (a2U2 < (R)0 ? -a2U2 : a2U2);
        const R xi_fix = (R)S.eps1 * ((R)1 - f8Mbar) * f8M * rmin(fef, frr);
        xi = rmax(xi_pos, xi_fix);
    } else {
        xi = rmax(xi_pos, (R)0);
    }

    // Eqs. (87)-(91)
    const R ic = rdiv((R)1, c);
    const R sU = sgn(U);
    const R mUc = rmin(absUp, c);
    const R dpp = sU * mUc * dp * ic;
    const R dpu = ((R)1 - s1 + s1 * fM) * rmax((R)0, c - absUp) * rho * dU;
    const R bracket = rmax((R)0, ct - absUp)
                    + omt * (absUp - rdiv(U, (R)2 * ct) * sgn(Ut) * rmin(Ut < (R)0 ? -Ut : Ut, ct));
    const R dUp = rdiv(s1 * ((R)1 - f8M) * bracket * dp, rho * theta * c * c);
    const R dUu = (R)0.5 * sU * mUc * dU * ic;

    // Eq. (85): F = central - (1/2){xi dPsi + (dpp + dpu)(0, n, 0) + dUp PsiHat + dUu (Psi_R + Psi_L)}
    const double xid = (double)xi, dpd_ = (double)(dpp + dpu), dUpd = (double)dUp, dUud = (double)dUu;
    const double rhod = (double)rho;
    const double Ph[4] = {rhod, rhod * (double)u, rhod * (double)v, rhod * (double)H};
    const double pv[4] = {0.0, nx, ny, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double diss = xid * dPsi[k] + dpd_ * pv[k] + dUpd * Ph[k] + dUud * PsiR[k] + dUud * PsiL[k];
        F[k] = 0.5 * (FbL[k] + FbR[k]) - 0.5 * diss;
    }
}

// Explicit rate of one cell for the time-step rule:
// (|V.Si| + ce |Si| + |V.Sj| + ce |Sj|) / Omega, ce = c / sqrt(theta_cell).
__device__ __forceinline__ double cell_rate(const DevSolve &S, const double W[4], int i, int j)
{
    double c = sqrt(S.gamma * W[3] / W[0]);
    double M = sqrt(W[1] * W[1] + W[2] * W[2]) / c;
    double theta = rmin(rmax(S.mr2, M * M), 1.0);
    double ce = c / sqrt(theta);
    double six, siy, sjx, sjy, li, lj;
    if (S.metric == 0) {
        six = S.dy; siy = 0.0; sjx = 0.0; sjy = S.dx; li = S.dy; lj = S.dx;
    } else {
        double ax, ay, bx, by;
        xface_vec(S, i, j, ax, ay);
        xface_vec(S, i + 1, j, bx, by);
        six = 0.5 * (ax + bx); siy = 0.5 * (ay + by);
        yface_vec(S, i, j, ax, ay);
        yface_vec(S, i, j + 1, bx, by);
        sjx = 0.5 * (ax + bx); sjy = 0.5 * (ay + by);
        li = sqrt(six * six + siy * siy);
        lj = sqrt(sjx * sjx + sjy * sjy);
    }
    double sum = fabs(W[1] * six + W[2] * siy) + ce * li + fabs(W[1] * sjx + W[2] * sjy) + ce * lj;
    return sum / cell_area(S, i, j);
}

__device__ __forceinline__ bool physical(const double W[4])
{
    bool fin = isfinite(W[0]) && isfinite(W[1]) && isfinite(W[2]) && isfinite(W[3]);
    return fin && W[0] > 0.0 && W[3] > 0.0;
}

} // namespace roeam

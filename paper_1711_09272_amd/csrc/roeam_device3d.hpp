// roeam_device3d.hpp -- device-side building blocks of the 3-D Roe-AM path on
// uniform Cartesian grids: solve descriptor, boundary-mapped cell fetch, the
// Roe-AM flux of Eqs. (85)-(109) with five conserved rows and the 3-D time-step
// rule, and the transported scalars (rows rho k_m) of Eq. (85).
//
// The flux is evaluated in the frame of its face: a face normal to axis a
// takes the velocity components in the cyclic order (normal, next, next but
// one), so n = (1, 0, 0) in the flux and the caller scatters the momentum rows
// back.  On uniform Cartesian faces this is exact (a permutation), and it keeps
// one flux routine for the three face directions.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "roeam_device.hpp"

namespace roeam {

enum { SIDE3_W = 0, SIDE3_E = 1, SIDE3_S = 2, SIDE3_N = 3, SIDE3_B = 4, SIDE3_T = 5 };

// Everything a 3-D stage kernel needs about one solve (read from device memory).
struct DevSolve3 {
    int nx, ny, nz;
    long long pitch, slab, plane;    // row pitch, ny * pitch, nz * ny * pitch (elements)
    double ax, ay, az, inv_vol;      // face areas dy dz, dx dz, dx dy and 1 / (dx dy dz)
    int bc[6];                       // W, E, S, N, bottom, top
    double bcw[6][5];                // Dirichlet states, primitive (rho, u, v, w, p)
    double gamma, gm1, g_gm1, igm1, mr2, dv_min2, eps1, eps2, eps_lambda;
    int s1_mode, order, precision, scheme;
    unsigned variant;
    double *q, *qa, *qb;
    Slot *slot;
    int nsc;                         // transported scalars, rows 5 .. 4 + nsc
    double bck[6][kMaxScalars];      // Dirichlet scalars, primitive k_m
};

// Primitives (rho, u, v, w, p) of a conserved state; returns 1/rho.
__device__ __forceinline__ double to_prim3(double gm1, const double Q[5], double W[5])
{
    const double rho = Q[0];
    const double ir = rcp_nr(rho);
    const double u = Q[1] * ir, v = Q[2] * ir, w = Q[3] * ir;
    W[0] = rho;
    W[1] = u;
    W[2] = v;
    W[3] = w;
    W[4] = gm1 * (Q[4] - 0.5 * rho * (u * u + v * v + w * w));
    return ir;
}

// Primitives of cell (i, j, l) and, for NSC transported scalars, k_m = (rho k_m) / rho.
template <int NSC = 0>
__device__ __forceinline__ void load_prim3(const DevSolve3 &S, const double *__restrict__ q, int i, int j, int l,
                                           double *W)
{
    const long long idx = (long long)l * S.slab + (long long)j * S.pitch + i;
    double Q[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) Q[k] = gptr(q)[k * S.plane + idx];
    const double ir = to_prim3(S.gm1, Q, W);
#pragma unroll
    for (int m = 0; m < NSC; ++m) W[5 + m] = gptr(q)[(5 + m) * S.plane + idx] * ir;
}

template <int NSC>
__device__ __forceinline__ void dirichlet3(const DevSolve3 &S, int side, double *W)
{
#pragma unroll
    for (int k = 0; k < 5; ++k) W[k] = S.bcw[side][k];
#pragma unroll
    for (int m = 0; m < NSC; ++m) W[5 + m] = S.bck[side][m];
}

// Interior index of a ghost cell at position i (< 0 or >= n) of a side of kind
// `kind` (not Dirichlet): periodic wrap, nearest cell, or mirror image.
__device__ __forceinline__ int ghost_source(int kind, int i, int n)
{
    if (kind == BC_PERIODIC) return i < 0 ? i + n : i - n;
    if (kind == BC_TRANSMISSIVE) return i < 0 ? 0 : n - 1;
    return i < 0 ? -i - 1 : 2 * n - 1 - i;
}

// Primitive state of any cell within two layers of the grid.  The x rule, then
// the y rule, then the z rule (which also define edges and corners); a slip
// wall mirrors the cell and negates the velocity component normal to it.
template <int NSC = 0>
__device__ __forceinline__ void fetch_prim3_x(const DevSolve3 &S, const double *__restrict__ q, int i, int j, int l,
                                              double *W)
{
    if (i >= 0 && i < S.nx) { load_prim3<NSC>(S, q, i, j, l, W); return; }
    const bool lo = i < 0;
    const int kind = lo ? S.bc[SIDE3_W] : S.bc[SIDE3_E];
    if (kind == BC_DIRICHLET) {
        dirichlet3<NSC>(S, lo ? SIDE3_W : SIDE3_E, W);
        return;
    }
    load_prim3<NSC>(S, q, ghost_source(kind, i, S.nx), j, l, W);
    if (kind == BC_SLIPWALL) W[1] = -W[1];
}

template <int NSC = 0>
__device__ __forceinline__ void fetch_prim3_y(const DevSolve3 &S, const double *__restrict__ q, int i, int j, int l,
                                              double *W)
{
    if (j >= 0 && j < S.ny) { fetch_prim3_x<NSC>(S, q, i, j, l, W); return; }
    const bool lo = j < 0;
    const int kind = lo ? S.bc[SIDE3_S] : S.bc[SIDE3_N];
    if (kind == BC_DIRICHLET) {
        dirichlet3<NSC>(S, lo ? SIDE3_S : SIDE3_N, W);
        return;
    }
    fetch_prim3_x<NSC>(S, q, i, ghost_source(kind, j, S.ny), l, W);
    if (kind == BC_SLIPWALL) W[2] = -W[2];
}

template <int NSC = 0>
__device__ __forceinline__ void fetch_prim3(const DevSolve3 &S, const double *__restrict__ q, int i, int j, int l,
                                            double *W)
{
    if (l >= 0 && l < S.nz) { fetch_prim3_y<NSC>(S, q, i, j, l, W); return; }
    const bool lo = l < 0;
    const int kind = lo ? S.bc[SIDE3_B] : S.bc[SIDE3_T];
    if (kind == BC_DIRICHLET) {
        dirichlet3<NSC>(S, lo ? SIDE3_B : SIDE3_T, W);
        return;
    }
    fetch_prim3_y<NSC>(S, q, i, j, ghost_source(kind, l, S.nz), W);
    if (kind == BC_SLIPWALL) W[3] = -W[3];
}

// ---------------------------------------------------------------------------
// Classical Roe flux, Eq. (7) with Eqs. (8)-(12) and Harten's fix of
// Eqs. (114)-(115), in the face frame (n = e_1; W = rho, u_n, u_t1, u_t2, p).
// ---------------------------------------------------------------------------
template <typename R, int NSC = 0>
__device__ __forceinline__ void roe_classic3(const DevSolve3 &S, const double *WL, const double *WR, double *F)
{
    const double rL = WL[0], uL = WL[1], vL = WL[2], wL = WL[3], pL = WL[4];
    const double rR = WR[0], uR = WR[1], vR = WR[2], wR = WR[3], pR = WR[4];
    const double iL = rcp_nr(rL), iR = rcp_nr(rR);
    const double qL = uL * uL + vL * vL + wL * wL, qR = uR * uR + vR * vR + wR * wR;
    const double HL = S.g_gm1 * pL * iL + 0.5 * qL, HR = S.g_gm1 * pR * iR + 0.5 * qR;
    const double dUd = uR - uL, dpd = pR - pL;

    const R rr = sqrtR((R)(rR * iL));
    const R w1 = rcpR((R)1 + rr);
    const R rho = rr * (R)rL;
    const R u = ((R)uL + rr * (R)uR) * w1;
    const R v = ((R)vL + rr * (R)vR) * w1;
    const R w = ((R)wL + rr * (R)wR) * w1;
    const R H = ((R)HL + rr * (R)HR) * w1;
    const R c2 = (R)S.gm1 * (H - (R)0.5 * (u * u + v * v + w * w));
    const R ic = rsqR(c2);
    const R c = c2 * ic;
    const R U = u;
    const R dU = (R)dUd, dp = (R)dpd;

    R l1 = rabs(U), l4 = rabs(U - c), l5 = rabs(U + c);
    if (S.scheme == SCHEME_ROE_HARTEN) {
        const R h = (R)S.eps_lambda * rmax(l1, rmax(l4, l5));
        if (h > (R)0) {
            const R ih = rcpR(h);
            l1 = l1 < h ? (R)0.5 * (l1 * l1 * ih + h) : l1;
            l4 = l4 < h ? (R)0.5 * (l4 * l4 * ih + h) : l4;
            l5 = l5 < h ? (R)0.5 * (l5 * l5 * ih + h) : l5;
        }
    }
    const R a = (R)0.5 * (l5 + l4) - l1;  // Eqs. (9) and (12)
    const R b = (R)0.5 * (l5 - l4);       // Eqs. (10) and (11)
    const double xid = (double)l1;        // Eq. (8)
    const double pd = (double)(a * rho * dU + b * dp * ic);
    const double Ud = (double)((b * dU + a * dp * rcpR(rho * c)) * ic);
    const double rhod = (double)rho;
    const double rEL = pL * S.igm1 + 0.5 * rL * qL, rER = pR * S.igm1 + 0.5 * rR * qR;
    const double PL1 = rL * uL, PL2 = rL * vL, PL3 = rL * wL, PR1 = rR * uR, PR2 = rR * vR, PR3 = rR * wR;
    F[0] = 0.5 * (uL * rL + uR * rR) - 0.5 * (xid * (rR - rL) + Ud * rhod);
    F[1] = 0.5 * ((uL * PL1 + pL) + (uR * PR1 + pR)) - 0.5 * (xid * (PR1 - PL1) + pd + Ud * (rhod * (double)u));
    F[2] = 0.5 * (uL * PL2 + uR * PR2) - 0.5 * (xid * (PR2 - PL2) + Ud * (rhod * (double)v));
    F[3] = 0.5 * (uL * PL3 + uR * PR3) - 0.5 * (xid * (PR3 - PL3) + Ud * (rhod * (double)w));
    F[4] = 0.5 * (uL * (rL * HL) + uR * (rR * HR)) - 0.5 * (xid * (rER - rEL) + pd * (double)U + Ud * (rhod * (double)H));
    // transported scalars: xi Delta(rho k) + (dU_u + dU_p) rho^ k^, no pressure term
#pragma unroll
    for (int m = 0; m < NSC; ++m) {
        const double kL = WL[5 + m], kR = WR[5 + m];
        const double PL = rL * kL, PR = rR * kR;
        const double khat = (double)(((R)kL + rr * (R)kR) * w1);
        F[5 + m] = 0.5 * (uL * PL + uR * PR) - 0.5 * (xid * (PR - PL) + Ud * (rhod * khat));
    }
}

// ---------------------------------------------------------------------------
// Roe-AM flux, Eqs. (85)-(109), per unit face area, in the face frame.  R is
// the precision of the dissipation coefficients; the side quantities, the
// central term, the jumps of Eq. (85) and the assembly stay FP64.
// ---------------------------------------------------------------------------
template <typename R, int NSC = 0>
__device__ __forceinline__ void roeam_flux3(const DevSolve3 &S, const double *WL, const double *WR, double s1d,
                                            double *F)
{
    if (__builtin_expect(S.scheme != SCHEME_ROEAM, 0)) {
        roe_classic3<R, NSC>(S, WL, WR, F);
        return;
    }
    const double rL = WL[0], uL = WL[1], vL = WL[2], wL = WL[3], pL = WL[4];
    const double rR = WR[0], uR = WR[1], vR = WR[2], wR = WR[3], pR = WR[4];

    // side quantities, Eq. (4); U_L = u_L, U_R = u_R in the face frame
    const double qL = uL * uL + vL * vL + wL * wL, qR = uR * uR + vR * vR + wR * wR;
    const double PL1 = rL * uL, PL2 = rL * vL, PL3 = rL * wL;
    const double PR1 = rR * uR, PR2 = rR * vR, PR3 = rR * wR;
    constexpr bool F32 = std::is_same<R, float>::value;
    // rho H = gamma/(gamma-1) p + rho |V|^2 / 2 (FP64: central flux and jump)
    // needs no 1/rho, so the sides' reciprocals feed only the coefficients and
    // are taken in their precision (FP64: one Newton step, as the others)
    const double PL4 = S.g_gm1 * pL + 0.5 * rL * qL;
    const double PR4 = S.g_gm1 * pR + 0.5 * rR * qR;
    const R iLr = rcpR((R)rL), iRr = rcpR((R)rR);  // 1/rho of the sides
    const R HLr = (R)PL4 * iLr, HRr = (R)PR4 * iRr;
    const double dUd = uR - uL, dpd = pR - pL;

    // Roe averages
    const R rr = sqrtR((R)rR * iLr);
    const R w1 = rcpR((R)1 + rr);
    const R rho = rr * (R)rL;
    const R u = ((R)uL + rr * (R)uR) * w1;
    const R v = ((R)vL + rr * (R)vR) * w1;
    const R w = ((R)wL + rr * (R)wR) * w1;
    const R H = (HLr + rr * HRr) * w1;
    const R c2 = (R)S.gm1 * (H - (R)0.5 * (u * u + v * v + w * w));
    const R ic = rsqR(c2);
    const R c = c2 * ic;
    const R U = u;
    const R dU = (R)dUd, dp = (R)dpd;
    const R s1 = (R)s1d;

    // Mach numbers, Eqs. (93)-(94)
    const R c2L = F32 ? (R)S.gamma * (R)pL * iLr : (R)(S.gamma * pL * iLr);
    const R c2R = F32 ? (R)S.gamma * (R)pR * iRr : (R)(S.gamma * pR * iRr);
    const R icLR = rcpR(c2L * c2R);
    const R M = (R)0.5 * (sqrt0R((R)qL * c2R * icLR) + sqrt0R((R)qR * c2L * icLR));
    const R absU = rabs(U);
    const R Mbar = absU * ic;
    const R fM = fswitch(M), f8M = pow8(fM);
    const R fMbar = fswitch(Mbar), f8Mbar = pow8(fMbar);

    // preconditioning, Eqs. (99)-(101)
    const R theta = rmin(rmax((R)S.mr2, M * M), (R)1);
    const R omt = (R)1 - theta;
    const R omtU = omt * U;
    const R X = omtU * omtU + (R)4 * c2 * theta;
    const R rX = rsqR(X);
    const R ct = (R)0.5 * X * rX;
    const R aU_2ct = absU * rX;  // |U| / (2 c~)
    const R Ut = (R)0.5 * ((R)1 + theta) * U;

    // expansion-shock fix, Eq. (92)
    const R wexp = (S.variant & V_EXPFIX_F8) ? f8Mbar : fMbar;
    const R quarter_term = absU < c ? (R)0.5 : (absU == c ? (R)0.25 : (R)0);
    R absUp = absU - wexp * rmax((R)0, dU) * quarter_term;
    if (__builtin_expect((S.variant & (V_NO_EQ92 | V_CLAMP_UPRIME)) != 0, 0)) {
        if (S.variant & V_NO_EQ92) absUp = absU;
        if (S.variant & V_CLAMP_UPRIME) absUp = rmax(absUp, (R)0);
    }

    // xi, Eq. (86) with the Eq. (68) gate
    const R gate = (S.variant & V_XI_UNGATED) ? (R)1 : (R)1 - f8Mbar;
    const R xi_pos = (R)rabs(0.5 * (uR + uL)) + gate * ((R)0.5 * dU);
    R xi;
    if (S.eps1 != 0.0) {
        // f_ef (Eq. 102) and f_rr (Eqs. 103-109): n1 along the velocity jump
        // (the face normal when the jump is small); n2 along (n1 x n) x n1, so
        // alpha2 U2 = ((n1 x n) x n1) . V, which for n = e_1 and unit n1 is
        // (n1y^2 + n1z^2) u - n1x (n1y v + n1z w).
        const R fef = (R)S.eps2 * c;
        // the velocity jumps only steer n1 (Eq. 103)
        const R du = F32 ? (R)uR - (R)uL : (R)(uR - uL);
        const R dv = F32 ? (R)vR - (R)vL : (R)(vR - vL);
        const R dw = F32 ? (R)wR - (R)wL : (R)(wR - wL);
        const R dV2 = du * du + dv * dv + dw * dw;
        const bool use_n = dV2 < (R)S.dv_min2 || dV2 == (R)0;
        const R idV = rsqR(use_n ? (R)1 : dV2);
        const R n1x = use_n ? (R)1 : du * idV, n1y = use_n ? (R)0 : dv * idV, n1z = use_n ? (R)0 : dw * idV;
        const R a1U1 = n1x * (n1x * u + n1y * v + n1z * w);
        const R a2U2 = (n1y * n1y + n1z * n1z) * u - n1x * (n1y * v + n1z * w);
        const R frr = rabs(a1U1) + rabs(a2U2);
        const R xi_fix = (R)S.eps1 * ((R)1 - f8Mbar) * f8M * rmin(fef, frr);
        xi = rmax(xi_pos, xi_fix);
    } else {
        xi = rmax(xi_pos, (R)0);
    }

    // Eqs. (87)-(91)
    const R sU = sgn(U);
    const R mUc = rmin(absUp, c);
    const R sMc = sU * mUc * ic;  // sgn(U) min(|U|', c^) / c^, shared by dpp and dUu
    const R dpp = sMc * dp;
    const R dpu = ((R)1 - s1 + s1 * fM) * rmax((R)0, c - absUp) * rho * dU;
    // U~ = (1 + theta) U / 2 has the sign of U, so U / (2 c~) sgn(U~) = |U| / (2 c~)
    const R bracket = rmax((R)0, ct - absUp) + omt * (absUp - aU_2ct * rmin(rabs(Ut), ct));
    R dUp = s1 * ((R)1 - f8M) * bracket * dp * rcpR(rho * theta * c2);
    if (__builtin_expect((S.variant & (V_XI_EQ46 | V_XI_ROE | V_DUP_ROE | V_DUP_ZERO)) != 0, 0)) {
        if (S.variant & V_XI_EQ46) xi = (R)rabs(0.5 * (uR + uL));
        if (S.variant & V_XI_ROE) xi = absU;
        if (S.variant & V_DUP_ROE) dUp = rmax((R)0, c - absU) * dp * rcpR(rho * c2);
        if (S.variant & V_DUP_ZERO) dUp = (R)0;
    }
    const R dUu = (R)0.5 * sMc * dU;

    // Eq. (85), each row's side terms gathered per side: u_L Psi_L + u_R Psi_R -
    // xi (Psi_R - Psi_L) - dUu (Psi_R + Psi_L) = aL Psi_L + aR Psi_R with
    // aL = u_L + xi - dUu, aR = u_R - xi - dUu; the Psi^ term is (dUp rho^)
    // times (1, u^, v^, w^, H^)
    // (xi and dUu are widened to FP64 before they are combined: with FP32
    // coefficients their rounding then enters as in Eq. (85) written out,
    // times the jump Psi_R - Psi_L, and not times Psi itself)
    const double xid = (double)xi, dUud = (double)dUu;
    const double aL = uL + (xid - dUud), aR = uR - (xid + dUud);
    const R g = dUp * rho;
    const double pc = (pL + pR) - (double)(dpp + dpu);
    F[0] = 0.5 * fma(rR, aR, fma(rL, aL, -(double)g));
    F[1] = 0.5 * fma(PR1, aR, fma(PL1, aL, pc - (double)(g * u)));
    F[2] = 0.5 * fma(PR2, aR, fma(PL2, aL, -(double)(g * v)));
    F[3] = 0.5 * fma(PR3, aR, fma(PL3, aL, -(double)(g * w)));
    F[4] = 0.5 * fma(PR4, aR, fma(PL4, aL, -(double)(g * H)));
    // transported scalars: Psi = rho k, Psi^ = rho^ k^ (Roe average of k), no pressure term
#pragma unroll
    for (int m = 0; m < NSC; ++m) {
        const double kL = WL[5 + m], kR = WR[5 + m];
        const double PL = rL * kL, PR = rR * kR;
        const R khat = ((R)kL + rr * (R)kR) * w1;
        F[5 + m] = 0.5 * fma(PR, aR, fma(PL, aL, -(double)(g * khat)));
    }
}

// Explicit rate of one cell: ((|u| + ce) A_x + (|v| + ce) A_y + (|w| + ce) A_z) / V,
// ce = c / sqrt(theta_cell); ir = 1 / rho.
__device__ __forceinline__ double cell_rate3(const DevSolve3 &S, const double W[5], double ir)
{
    const double c2 = S.gamma * W[4] * ir;
    const double M2 = (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]) * rcp_nr(c2);
    const double theta = rmin(rmax(S.mr2, M2), 1.0);
    const double ce = c2 * rsq_nr(c2 * theta);
    const double sum = (fabs(W[1]) * S.ax + ce * S.ax) + (fabs(W[2]) * S.ay + ce * S.ay) + (fabs(W[3]) * S.az + ce * S.az);
    return sum * S.inv_vol;
}

__device__ __forceinline__ bool physical3(const double W[5])
{
    const bool fin = isfinite(W[0]) && isfinite(W[1]) && isfinite(W[2]) && isfinite(W[3]) && isfinite(W[4]);
    return fin && W[0] > 0.0 && W[4] > 0.0;
}

} // namespace roeam

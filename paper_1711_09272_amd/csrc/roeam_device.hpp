// roeam_device.hpp -- device-side building blocks of the gfx950 Roe-AM library:
// solve descriptor, boundary-mapped cell fetch, face geometry, the Roe-AM
// numerical flux of Eqs. (85)-(109) and the explicit-rate rule.
//
// 2-D form of the paper's equations: w = 0, n_z = 0, four conserved rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace roeam {

// BC_MOVING (uniform grids): the side's Dirichlet state where the cell-centre
// coordinate along the side is below spl_a + spl_b t, else its spl_hi kind
// (another Dirichlet state or a slip wall); t is the time of the stage input.
enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_SLIPWALL = 2, BC_DIRICHLET = 3, BC_MOVING = 4 };
enum { SIDE_W = 0, SIDE_E = 1, SIDE_S = 2, SIDE_N = 3 };
enum : unsigned {
    V_XI_UNGATED = 1u, V_EXPFIX_F8 = 2u, V_CLAMP_UPRIME = 4u, V_NO_EQ92 = 8u,
    V_XI_ROE = 16u, V_DUP_ROE = 32u, V_XI_EQ46 = 64u, V_DUP_ZERO = 128u
};
enum { SCHEME_ROEAM = 0, SCHEME_ROE = 1, SCHEME_ROE_HARTEN = 2 };
// Transported scalars (the rho k rows of Eq. 85) a 2-D solve may carry.
constexpr int kMaxScalars = 2;

// Per-solve time-integration state, resident in device memory.  The step
// state is double-buffered by step parity p: the first stage kernel of a step
// reads st[p] (time, step count and the explicit rate reduced over the state
// at the start of the step), every block derives the same dt from it, and
// block 0 writes st[1-p] for the next step.  No separate dt kernel runs.
// The max explicit rate of a state is reduced into kRateSlots words (workgroup
// id modulo kRateSlots) so that thousands of workgroups do not serialize on
// one device-scope atomic; readers take the max over the words.  Each word is
// the bit pattern of a non-negative double, which atomicMax on the unsigned
// 64-bit integer orders correctly.  The rate of the state after n steps sits
// in word set n mod 3: step n reads set n, reduces the new state into set
// n + 1 and clears set n + 2 (read by the previous step, reduced into by the
// next one), so no kernel between steps has to clear anything.
constexpr int kRateSlots = 64;
constexpr int kRateSets = 3;

struct StepState {
    double t;                      // time of the state at this parity
    double dt;                     // dt of the step that produced this state
    long long steps;               // steps taken so far
    long long pad;
};

struct alignas(64) Slot {
    unsigned long long rate_bits[kRateSets][kRateSlots];  // per step count mod 3
    StepState st[2];
    double t_end, cfl;
    long long max_steps;
    double dt_last, rate_last;     // of the last step taken
    int nonphys;                   // set (atomicOr) when a stage produces rho <= 0, p <= 0 or NaN
    int pad[3];
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
    int nsc;                    // transported scalars: rows 4 .. 3 + nsc of the state (rho k_m)
    double bck[4][kMaxScalars]; // Dirichlet scalars, primitive k_m
    double spl_a[4], spl_b[4];  // BC_MOVING sides: split at a + b t
    int spl_hi[4];              // BC_MOVING sides: kind above the split
    int spl_lo[4];              // BC_MOVING sides: kind below the split
    double bcw_hi[4][4];        // BC_MOVING sides: Dirichlet state above the split, primitive
    double t_res;               // time of moving sides in a residual-only launch
    // scheme
    double gamma, gm1, g_gm1, igm1, mr2, u_ref, dv_min2, eps1, eps2, eps_lambda, cfl, inv_area;
    int s1_mode, order, precision, scheme;
    unsigned variant;
    // state
    double *q, *qa, *qb;
    Slot *slot;
    int tiles_x, tiles_y;       // tiles of this solve (batched work lists)
};

// ---------------------------------------------------------------------------
// scalar helpers
// ---------------------------------------------------------------------------
template <typename R> __device__ __forceinline__ R sgn(R x) { return x > (R)0 ? (R)1 : (x < (R)0 ? (R)-1 : (R)0); }
// min/max/abs map to single instructions (v_min_f64, v_max_f64, source
// modifiers); the operands here are never NaN.
__device__ __forceinline__ double rmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ double rmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float rmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ float rmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double rabs(double a) { return fabs(a); }
__device__ __forceinline__ float rabs(float a) { return fabsf(a); }

// Reciprocal, quotient and reciprocal square root.  The hardware estimates
// v_rcp_f64 and v_rsq_f64 are good to about 2^-24 relative.  Two Newton steps
// (rcp_nr, rsq_nr) reach a correctly rounded or 1-ulp result: used for the
// primitives of the cell states, the side quantities of the central flux and
// the time-step rule.  One step (rcp_nr1, rsq_nr1: within about 20 ulp) is
// used for the dissipation coefficients of the flux (the R functions below
// for R = double), whose error is scaled by the jumps of Eq. (85).  FP32: the
// hardware instructions (about 1 ulp).
__device__ __forceinline__ double rcp_nr(double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ double rcp_nr1(double b)
{
    const double r = __builtin_amdgcn_rcp(b);
    return fma(r, fma(-b, r, 1.0), r);
}
// a / b: one residual correction of a * (1/b)
__device__ __forceinline__ double div_nr1(double a, double b)
{
    const double r = rcp_nr1(b);
    const double q = a * r;
    return fma(fma(-b, q, a), r, q);
}
__device__ __forceinline__ double rsq_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    double e = fma(-hx * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-hx * y, y, 0.5);
    return fma(y, e, y);
}
__device__ __forceinline__ double rsq_nr1(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    return fma(y, fma(-0.5 * x * y, y, 0.5), y);
}
__device__ __forceinline__ double rcpR(double b) { return rcp_nr1(b); }
__device__ __forceinline__ double rsqR(double x) { return rsq_nr1(x); }
// square root of a positive operand as x rsq(x)
__device__ __forceinline__ double sqrtR(double x) { return x * rsq_nr1(x); }
__device__ __forceinline__ float rcpR(float b) { return __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float rsqR(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float sqrtR(float x) { return __builtin_amdgcn_sqrtf(x); }
// square root of a non-negative operand (zero allowed): evaluated at
// x + 1e-300, which equals x for every x above about 1e-284 and keeps rsq off
// zero (the result for smaller x is below 1e-142 either way)
__device__ __forceinline__ double sqrt0R(double x)
{
    const double y = x + 1e-300;
    return y * rsq_nr1(y);
}
__device__ __forceinline__ float sqrt0R(float x) { return __builtin_amdgcn_sqrtf(x); }

// Eq. (98): f(phi) = min(phi sqrt(4 + (1 - phi^2)^2) / (1 + phi^2), 1), with
// sqrt(A) / B evaluated as A rsq(A B^2).
template <typename R> __device__ __forceinline__ R fswitch(R phi)
{
    const R p2 = phi * phi;
    const R om = (R)1 - p2;
    const R A = (R)4 + om * om;
    const R B = (R)1 + p2;
    return rmin(phi * A * rsqR(A * B * B), (R)1);
}
// f^8 as the eighth power (repeated squaring).
template <typename R> __device__ __forceinline__ R pow8(R x)
{
    R x2 = x * x;
    R x4 = x2 * x2;
    return x4 * x4;
}
// The detector's s1 = f^8(a), Eq. (95), from the face's smallest ratio a,
// taken in the precision of the dissipation coefficients it scales (PREC 1:
// FP32; the value is then exact in FP32 when the flux narrows it).
template <int PREC> __device__ __forceinline__ double detector_s1(double a)
{
    using R = typename std::conditional<PREC == 0, double, float>::type;
    return (double)pow8(fswitch((R)a));
}

// Global-memory views of the state and metric arrays.  The descriptor holds
// generic pointers; accesses through these views are global_* instructions
// instead of flat ones, which count against the LDS wait counter and which
// the compiler may not move past LDS accesses (a flat address could be LDS):
// with them the tile's halo loads issue together and the early loads of the
// own cells stay in flight behind the LDS work.
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ const gdouble *gptr(const double *p) { return (const gdouble *)p; }
__device__ __forceinline__ gdouble *gptr(double *p) { return (gdouble *)p; }

// Eq. (97): detector ratio of two neighbouring cells, min of the pressure and
// density ratios, each taken below one.
__device__ __forceinline__ double detector_P(double pA, double rA, double pB, double rB)
{
    // the smaller of the two ratios, chosen by cross-multiplication, one division
    const double pn = rmin(pA, pB), pd = rmax(pA, pB), rn = rmin(rA, rB), rd = rmax(rA, rB);
    const bool use_p = pn * rd <= rn * pd;
    return div_nr1(use_p ? pn : rn, use_p ? pd : rd);
}

// ---------------------------------------------------------------------------
// state access
// ---------------------------------------------------------------------------
// Primitives (rho, u, v, p) of a conserved state; returns 1/rho.
__device__ __forceinline__ double to_prim(double gm1, double q0, double q1, double q2, double q3, double W[4])
{
    double rho = q0;
    const double ir = rcp_nr(rho);
    double u = q1 * ir, v = q2 * ir;
    W[0] = rho;
    W[1] = u;
    W[2] = v;
    W[3] = gm1 * (q3 - 0.5 * rho * (u * u + v * v));
    return ir;
}

// Primitives of cell (i, j): (rho, u, v, p) and, for NSC transported
// scalars, k_m = (rho k_m) / rho.
template <int NSC = 0>
__device__ __forceinline__ void load_prim(const DevSolve &S, const double *__restrict__ q, int i, int j, double *W)
{
    long long idx = (long long)j * S.pitch + i;
    const gdouble *g = gptr(q);
    const double ir = to_prim(S.gm1, g[idx], g[S.plane + idx], g[2 * S.plane + idx], g[3 * S.plane + idx], W);
#pragma unroll
    for (int m = 0; m < NSC; ++m) W[4 + m] = g[(4 + m) * S.plane + idx] * ir;
}

template <int METRIC>
__device__ __forceinline__ void xface_vec(const DevSolve &S, int i, int j, double &sx, double &sy)
{
    if (METRIC == 0) { sx = S.dy; sy = 0.0; return; }
    long long nxn = S.nx + 1;
    const gdouble *xn = gptr(S.xn), *yn = gptr(S.yn);
    double ddx = xn[(long long)(j + 1) * nxn + i] - xn[(long long)j * nxn + i];
    double ddy = yn[(long long)(j + 1) * nxn + i] - yn[(long long)j * nxn + i];
    sx = ddy;
    sy = -ddx;
}
template <int METRIC>
__device__ __forceinline__ void yface_vec(const DevSolve &S, int i, int j, double &sx, double &sy)
{
    if (METRIC == 0) { sx = 0.0; sy = S.dx; return; }
    long long nxn = S.nx + 1;
    const gdouble *xn = gptr(S.xn), *yn = gptr(S.yn);
    double ddx = xn[(long long)j * nxn + i + 1] - xn[(long long)j * nxn + i];
    double ddy = yn[(long long)j * nxn + i + 1] - yn[(long long)j * nxn + i];
    sx = -ddy;
    sy = ddx;
}
// Unit normal and length of a face vector; axis-aligned faces of uniform
// grids are exact.
template <int METRIC>
__device__ __forceinline__ void unit_normal(const DevSolve &S, double sx, double sy, double &nx, double &ny, double &len)
{
    if (METRIC == 0) {
        if (sy == 0.0) { nx = 1.0; ny = 0.0; len = sx; }
        else { nx = 0.0; ny = 1.0; len = sy; }
        return;
    }
    const double s2 = sx * sx + sy * sy;
    const double il = rsq_nr(s2);
    len = s2 * il;
    nx = sx * il;
    ny = sy * il;
}
template <int METRIC>
__device__ __forceinline__ double cell_area(const DevSolve &S, int i, int j)
{
    if (METRIC == 0) return S.area;
    long long nxn = S.nx + 1;
    const gdouble *x = gptr(S.xn), *y = gptr(S.yn);
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
// Time of the state a stage reads, for moving boundary sides: the step start
// t of parity p plus c dt (c the stage abscissa), or t_res for a residual-only
// launch (slot == nullptr).  Read only where a moving side needs it.
struct BoundaryClock {
    const Slot *slot;
    int p;
    double c_dt;
    double t_res;
    __device__ __forceinline__ double time() const { return slot ? slot->st[p].t + c_dt : t_res; }
};

// A BC_MOVING side at cell-centre coordinate xc along it: fills W with a
// Dirichlet state and returns -1, or returns the kind to apply.
template <int NSC>
__device__ __forceinline__ int moving_side(const DevSolve &S, int sd, double xc, const BoundaryClock &clk, double *W)
{
    const bool lo = xc < S.spl_a[sd] + S.spl_b[sd] * clk.time();
    if ((lo ? S.spl_lo[sd] : S.spl_hi[sd]) != BC_DIRICHLET) return BC_SLIPWALL;
#pragma unroll
    for (int k = 0; k < 4; ++k) W[k] = lo ? S.bcw[sd][k] : S.bcw_hi[sd][k];
#pragma unroll
    for (int m = 0; m < NSC; ++m) W[4 + m] = S.bck[sd][m];
    return -1;
}

template <int METRIC, int NSC = 0>
__device__ __forceinline__ void fetch_prim_x(const DevSolve &S, const double *__restrict__ q, int i, int j, double *W,
                                             const BoundaryClock &clk)
{
    if (i >= 0 && i < S.nx) { load_prim<NSC>(S, q, i, j, W); return; }
    // constant-index selects keep the by-value kernel argument out of scratch
    const bool west = i < 0;
    int kind = west ? S.bc[SIDE_W] : S.bc[SIDE_E];
    if (kind == BC_MOVING) {
        kind = moving_side<NSC>(S, west ? SIDE_W : SIDE_E, (j + 0.5) * S.dy, clk, W);
        if (kind < 0) return;
    }
    if (kind == BC_DIRICHLET) {
#pragma unroll
        for (int k = 0; k < 4; ++k) W[k] = west ? S.bcw[SIDE_W][k] : S.bcw[SIDE_E][k];
#pragma unroll
        for (int m = 0; m < NSC; ++m) W[4 + m] = west ? S.bck[SIDE_W][m] : S.bck[SIDE_E][m];
        return;
    }
    int is;
    if (kind == BC_PERIODIC) is = i < 0 ? i + S.nx : i - S.nx;
    else if (kind == BC_TRANSMISSIVE) is = i < 0 ? 0 : S.nx - 1;
    else is = i < 0 ? -i - 1 : 2 * S.nx - 1 - i;
    load_prim<NSC>(S, q, is, j, W);
    if (kind == BC_SLIPWALL) {
        double sx, sy, nx, ny, len;
        xface_vec<METRIC>(S, i < 0 ? 0 : S.nx, j, sx, sy);
        unit_normal<METRIC>(S, sx, sy, nx, ny, len);
        reflect(W, nx, ny);
    }
}

// Primitive state of any cell within two layers of the grid: the x rule, then
// the y rule (which also defines the corners).
template <int METRIC, int NSC = 0>
__device__ __forceinline__ void fetch_prim(const DevSolve &S, const double *__restrict__ q, int i, int j, double *W,
                                           const BoundaryClock &clk)
{
    if (j >= 0 && j < S.ny) { fetch_prim_x<METRIC, NSC>(S, q, i, j, W, clk); return; }
    const bool south = j < 0;
    int kind = south ? S.bc[SIDE_S] : S.bc[SIDE_N];
    if (kind == BC_MOVING) {
        kind = moving_side<NSC>(S, south ? SIDE_S : SIDE_N, (i + 0.5) * S.dx, clk, W);
        if (kind < 0) return;
    }
    if (kind == BC_DIRICHLET) {
#pragma unroll
        for (int k = 0; k < 4; ++k) W[k] = south ? S.bcw[SIDE_S][k] : S.bcw[SIDE_N][k];
#pragma unroll
        for (int m = 0; m < NSC; ++m) W[4 + m] = south ? S.bck[SIDE_S][m] : S.bck[SIDE_N][m];
        return;
    }
    int js;
    if (kind == BC_PERIODIC) js = j < 0 ? j + S.ny : j - S.ny;
    else if (kind == BC_TRANSMISSIVE) js = j < 0 ? 0 : S.ny - 1;
    else js = j < 0 ? -j - 1 : 2 * S.ny - 1 - j;
    fetch_prim_x<METRIC, NSC>(S, q, i, js, W, clk);
    if (kind == BC_SLIPWALL) {
        int ic = i < 0 ? 0 : (i > S.nx - 1 ? S.nx - 1 : i);
        double sx, sy, nx, ny, len;
        yface_vec<METRIC>(S, ic, j < 0 ? 0 : S.ny, sx, sy);
        unit_normal<METRIC>(S, sx, sy, nx, ny, len);
        reflect(W, nx, ny);
    }
}

// ---------------------------------------------------------------------------
// Classical Roe flux in the scale form of Eq. (7) with the coefficients of
// Eqs. (8)-(12) and the eigenvalues |U|, |U - c|, |U + c| of Eq. (6), with
// Harten's fix of Eqs. (114)-(115) for SCHEME_ROE_HARTEN: an eigenvalue
// below h = eps_lambda max(eigenvalues) becomes (l^2 / h + h) / 2.  The jump
// multiplied by xi is the conserved one (energy row rho E) and the pressure
// vector is (0, n, U), as Eq. (7) has them.
// ---------------------------------------------------------------------------
template <typename R, int NSC = 0>
__device__ __forceinline__ void roe_classic(const DevSolve &S, const double *WL, const double *WR, double nx,
                                            double ny, double *F)
{
    const double rL = WL[0], uL = WL[1], vL = WL[2], pL = WL[3];
    const double rR = WR[0], uR = WR[1], vR = WR[2], pR = WR[3];
    const double iL = rcp_nr(rL), iR = rcp_nr(rR);
    const double qL = uL * uL + vL * vL, qR = uR * uR + vR * vR;
    const double UL = nx * uL + ny * vL, UR = nx * uR + ny * vR;
    const double HL = S.g_gm1 * pL * iL + 0.5 * qL, HR = S.g_gm1 * pR * iR + 0.5 * qR;
    const double dUd = UR - UL, dpd = pR - pL;

    const R rr = sqrtR((R)(rR * iL));
    const R w1 = rcpR((R)1 + rr);
    const R rho = rr * (R)rL;
    const R u = ((R)uL + rr * (R)uR) * w1;
    const R v = ((R)vL + rr * (R)vR) * w1;
    const R H = ((R)HL + rr * (R)HR) * w1;
    const R c2 = (R)S.gm1 * (H - (R)0.5 * (u * u + v * v));
    const R ic = rsqR(c2);
    const R c = c2 * ic;
    const R U = (R)nx * u + (R)ny * v;
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
    // conserved jumps, energy row with rho E = p / (gamma - 1) + rho |V|^2 / 2
    const double rEL = pL * S.igm1 + 0.5 * rL * qL;
    const double rER = pR * S.igm1 + 0.5 * rR * qR;
    const double PsiL1 = rL * uL, PsiL2 = rL * vL, PsiR1 = rR * uR, PsiR2 = rR * vR;
    F[0] = 0.5 * (UL * rL + UR * rR) - 0.5 * (xid * (rR - rL) + Ud * rhod);
    F[1] = 0.5 * ((UL * PsiL1 + pL * nx) + (UR * PsiR1 + pR * nx))
         - 0.5 * (xid * (PsiR1 - PsiL1) + pd * nx + Ud * (rhod * (double)u));
    F[2] = 0.5 * ((UL * PsiL2 + pL * ny) + (UR * PsiR2 + pR * ny))
         - 0.5 * (xid * (PsiR2 - PsiL2) + pd * ny + Ud * (rhod * (double)v));
    F[3] = 0.5 * (UL * (rL * HL) + UR * (rR * HR)) - 0.5 * (xid * (rER - rEL) + pd * (double)U + Ud * (rhod * (double)H));
    // transported scalars: xi Delta(rho k) + (dU_u + dU_p) rho^ k^, no pressure term
#pragma unroll
    for (int m = 0; m < NSC; ++m) {
        const double kL = WL[4 + m], kR = WR[4 + m];
        const double PL = rL * kL, PR = rR * kR;
        const double khat = (double)(((R)kL + rr * (R)kR) * w1);
        F[4 + m] = 0.5 * (UL * PL + UR * PR) - 0.5 * (xid * (PR - PL) + Ud * (rhod * khat));
    }
}

// ---------------------------------------------------------------------------
// Roe-AM numerical flux, Eqs. (85)-(109), per unit face length.
// R is the precision of the dissipation coefficients; the side quantities,
// the central term, the jumps of Eq. (85) and the final assembly stay FP64.
// AXIS: the face normal is n = (1, 0) (the caller passes the states in the
// face's frame); the products with the normal's components are left out.
// ---------------------------------------------------------------------------
template <typename R, int NSC = 0, bool AXIS = false>
__device__ __forceinline__ void roeam_flux(const DevSolve &S, const double *WL, const double *WR, double nx,
                                           double ny, double s1d, double *F)
{
    if (AXIS) {
        nx = 1.0;
        ny = 0.0;
    }
    if (__builtin_expect(S.scheme != SCHEME_ROEAM, 0)) {
        roe_classic<R, NSC>(S, WL, WR, nx, ny, F);
        return;
    }
    const double rL = WL[0], uL = WL[1], vL = WL[2], pL = WL[3];
    const double rR = WR[0], uR = WR[1], vR = WR[2], pR = WR[3];

    // side quantities, Eq. (4); H = gamma/(gamma-1) p/rho + |V|^2/2
    const double qL = uL * uL + vL * vL, qR = uR * uR + vR * vR;
    const double UL = AXIS ? uL : nx * uL + ny * vL, UR = AXIS ? uR : nx * uR + ny * vR;
    const double PsiL1 = rL * uL, PsiL2 = rL * vL;
    const double PsiR1 = rR * uR, PsiR2 = rR * vR;
    // rho H = gamma/(gamma-1) p + rho |V|^2 / 2 (FP64: central flux and jump)
    // needs no 1/rho, so the sides' reciprocals feed only the coefficients and
    // are taken in their precision (FP64: one Newton step, as the others)
    const double PsiL3 = S.g_gm1 * pL + 0.5 * rL * qL;
    const double PsiR3 = S.g_gm1 * pR + 0.5 * rR * qR;
    const R iLr = rcpR((R)rL), iRr = rcpR((R)rR);  // 1/rho of the sides
    const R HLr = (R)PsiL3 * iLr, HRr = (R)PsiR3 * iRr;

    // jumps stay FP64 (low-Mach pressure differences cancel otherwise)
    const double dUd = UR - UL, dpd = pR - pL;

    // Roe averages (sqrt(rho) weights)
    const R rr = sqrtR((R)rR * iLr);
    const R w1 = rcpR((R)1 + rr);
    const R rho = rr * (R)rL;
    const R u = ((R)uL + rr * (R)uR) * w1;
    const R v = ((R)vL + rr * (R)vR) * w1;
    const R H = (HLr + rr * HRr) * w1;
    const R c2 = (R)S.gm1 * (H - (R)0.5 * (u * u + v * v));
    const R ic = rsqR(c2);
    const R c = c2 * ic;
    const R U = AXIS ? u : (R)nx * u + (R)ny * v;
    const R dU = (R)dUd, dp = (R)dpd;
    const R s1 = (R)s1d;


    // Mach numbers, Eqs. (93)-(94): M_K = |V_K| / c_K, c_K^2 = gamma p_K / rho_K
    constexpr bool F32 = std::is_same<R, float>::value;
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
    const R ct = (R)0.5 * X * rX;  // c~ of Eq. (99)
    const R aU_2ct = absU * rX;    // |U| / (2 c~)
    const R Ut = (R)0.5 * ((R)1 + theta) * U;

    // expansion-shock fix, Eq. (92); sign(U + c) - sign(U - c) is 2 for |U| < c,
    // 1 for |U| = c and 0 otherwise (the sums are exact near their zeros)
    const R wexp = (S.variant & V_EXPFIX_F8) ? f8Mbar : fMbar;
    const R quarter_term = absU < c ? (R)0.5 : (absU == c ? (R)0.25 : (R)0);
    R absUp = absU - wexp * rmax((R)0, dU) * quarter_term;
    if (__builtin_expect((S.variant & (V_NO_EQ92 | V_CLAMP_UPRIME)) != 0, 0)) {
        if (S.variant & V_NO_EQ92) absUp = absU;
        if (S.variant & V_CLAMP_UPRIME) absUp = rmax(absUp, (R)0);
    }

    // basic upwind dissipation xi, Eq. (86) with the Eq. (68) gate
    const R gate = (S.variant & V_XI_UNGATED) ? (R)1 : (R)1 - f8Mbar;
    const R xi_pos = (R)rabs(0.5 * (UR + UL)) + gate * ((R)0.5 * dU);
    R xi;
    if (S.eps1 != 0.0) {
        // modified entropy fix f_ef (Eq. 102) and rotated speed f_rr (Eqs. 103-109)
        const R fef = (R)S.eps2 * c;
        // the velocity jumps only steer n1 (Eq. 103): FP32 differences of the
        // rounded velocities suffice there
        const R du = F32 ? (R)uR - (R)uL : (R)(uR - uL);
        const R dv = F32 ? (R)vR - (R)vL : (R)(vR - vL);
        const R dV2 = du * du + dv * dv;
        const bool use_n = dV2 < (R)S.dv_min2 || dV2 == (R)0;
        const R idV = rsqR(use_n ? (R)1 : dV2);
        const R n1x = use_n ? (R)nx : du * idV, n1y = use_n ? (R)ny : dv * idV;
        const R a1U1 = (AXIS ? n1x : n1x * (R)nx + n1y * (R)ny) * (n1x * u + n1y * v);
        // unit n2 along (n1 x n) x n1 = s (-n1y, n1x): alpha2 U2 = |s| (n1x v - n1y u) up to sign
        const R sz = AXIS ? -n1y : n1x * (R)ny - n1y * (R)nx;
        const R a2U2 = sz * (n1x * v - n1y * u);
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
    // ablations of Sec. 7: xi of Eq. (46) (no velocity positivity) or of
    // Eq. (13); dU_p of classical Roe, Eq. (17), or none
    if (__builtin_expect((S.variant & (V_XI_EQ46 | V_XI_ROE | V_DUP_ROE | V_DUP_ZERO)) != 0, 0)) {
        if (S.variant & V_XI_EQ46) xi = (R)rabs(0.5 * (UR + UL));
        if (S.variant & V_XI_ROE) xi = absU;
        if (S.variant & V_DUP_ROE) dUp = rmax((R)0, c - absU) * dp * rcpR(rho * c2);
        if (S.variant & V_DUP_ZERO) dUp = (R)0;
    }
    const R dUu = (R)0.5 * sMc * dU;

    // Eq. (85): F = central - (1/2){xi dPsi + (dpp + dpu)(0, n, 0) + dUp PsiHat + dUu (Psi_R + Psi_L)}.
    // Each row's side terms are gathered per side, U_L Psi_L + U_R Psi_R -
    // xi (Psi_R - Psi_L) - dUu (Psi_R + Psi_L) = aL Psi_L + aR Psi_R with
    // aL = U_L + xi - dUu and aR = U_R - xi - dUu, and the Psi^ term is
    // (dUp rho^) times (1, u^, v^, H^)
    // (xi and dUu are widened to FP64 before they are combined: with FP32
    // coefficients their rounding then enters as in Eq. (85) written out,
    // times the jump Psi_R - Psi_L, and not times Psi itself)
    const double xid = (double)xi, dUud = (double)dUu;
    const double aL = UL + (xid - dUud), aR = UR - (xid + dUud);
    const R g = dUp * rho;
    const double pc = (pL + pR) - (double)(dpp + dpu);
    F[0] = 0.5 * fma(rR, aR, fma(rL, aL, -(double)g));
    if (AXIS) {
        F[1] = 0.5 * fma(PsiR1, aR, fma(PsiL1, aL, pc - (double)(g * u)));
    } else {
        F[1] = 0.5 * fma(PsiR1, aR, fma(PsiL1, aL, fma(pc, nx, -(double)(g * u))));
    }
    F[2] = 0.5 * fma(PsiR2, aR, fma(PsiL2, aL, AXIS ? -(double)(g * v) : fma(pc, ny, -(double)(g * v))));
    F[3] = 0.5 * fma(PsiR3, aR, fma(PsiL3, aL, -(double)(g * H)));
    // transported scalars (rho k rows of Eq. 85): Psi = rho k, Psi^ = rho^ k^
    // with the Roe average of k, no pressure term
#pragma unroll
    for (int m = 0; m < NSC; ++m) {
        const double kL = WL[4 + m], kR = WR[4 + m];
        const double PL = rL * kL, PR = rR * kR;
        const R khat = ((R)kL + rr * (R)kR) * w1;
        F[4 + m] = 0.5 * fma(PR, aR, fma(PL, aL, -(double)(g * khat)));
    }
}

// Explicit rate of one cell for the time-step rule:
// (|V.Si| + ce |Si| + |V.Sj| + ce |Sj|) / Omega, ce = c / sqrt(theta_cell)
// (evaluated as c^2 rsq(c^2 theta)); ir = 1 / rho.
template <int METRIC>
__device__ __forceinline__ double cell_rate(const DevSolve &S, const double W[4], double ir, int i, int j)
{
    const double c2 = S.gamma * W[3] * ir;
    const double M2 = (W[1] * W[1] + W[2] * W[2]) * rcp_nr(c2);
    const double theta = rmin(rmax(S.mr2, M2), 1.0);
    const double ce = c2 * rsq_nr(c2 * theta);
    if (METRIC == 0) {
        // faces along the axes: |u| dy + |v| dx (the zero products of the
        // general form left out; equal to it for finite states)
        const double sum = fabs(W[1]) * S.dy + ce * S.dy + fabs(W[2]) * S.dx + ce * S.dx;
        return sum * S.inv_area;
    }
    double six, siy, sjx, sjy, li, lj;
    {
        double ax, ay, bx, by;
        xface_vec<METRIC>(S, i, j, ax, ay);
        xface_vec<METRIC>(S, i + 1, j, bx, by);
        six = 0.5 * (ax + bx); siy = 0.5 * (ay + by);
        yface_vec<METRIC>(S, i, j, ax, ay);
        yface_vec<METRIC>(S, i, j + 1, bx, by);
        sjx = 0.5 * (ax + bx); sjy = 0.5 * (ay + by);
        const double li2 = six * six + siy * siy, lj2 = sjx * sjx + sjy * sjy;
        li = li2 * rsq_nr(li2);
        lj = lj2 * rsq_nr(lj2);
    }
    const double sum = fabs(W[1] * six + W[2] * siy) + ce * li + fabs(W[1] * sjx + W[2] * sjy) + ce * lj;
    return sum * rcp_nr(cell_area<METRIC>(S, i, j));
}

__device__ __forceinline__ bool physical(const double W[4])
{
    bool fin = isfinite(W[0]) && isfinite(W[1]) && isfinite(W[2]) && isfinite(W[3]);
    return fin && W[0] > 0.0 && W[3] > 0.0;
}

} // namespace roeam

// roeam_stage3d.hpp -- the 3-D stage kernel as templates over the MUSCL order,
// the coefficient precision, the number of transported scalars and the brick
// shape; roeam_kernels3d.hip instantiates the scalar-free kernels,
// roeam_kernels3d_sc.hip those with one or two scalars.
//
// A workgroup owns a brick of TX x TY x TZ cells.  It stages the brick and its
// halo (two layers for MUSCL, one for piecewise-constant states) as primitives
// in LDS, builds the detector ratio of Eq. (97) of every face within one layer
// of the brick, then sweeps the x-, y- and z-faces in turn through one or two
// LDS flux buffers, each face evaluated exactly once (Eq. 85, nine-face detector of
// Eq. 96), accumulates the conservative residual of its cells in registers and
// applies the stage update, the positivity check and the explicit-rate
// reduction exactly as the 2-D stage kernel does (same stage codes, same step
// state).  One kernel per Runge-Kutta stage.
#pragma once

#include <atomic>
#include <type_traits>

#include "roeam_device3d.hpp"
#include "roeam_internal.hpp"
#include "roeam_stage.hpp"

namespace roeam {

template <int TX, int TY, int TZ, int HL>
struct Brick {
    static constexpr int LX = TX + 2 * HL, LY = TY + 2 * HL, LZ = TZ + 2 * HL;
    // detector ratios: x-faces (TX+1) x (TY+2) x (TZ+2), y-faces (TX+2) x (TY+1) x (TZ+2),
    // z-faces (TX+2) x (TY+2) x (TZ+1), i.e. every face within one cell layer of the brick
    static constexpr int NPX = (TZ + 2) * (TY + 2) * (TX + 1);
    static constexpr int NPY = (TZ + 2) * (TY + 1) * (TX + 2);
    static constexpr int NPZ = (TZ + 1) * (TY + 2) * (TX + 2);
    static constexpr int NFX = TZ * TY * (TX + 1), NFY = TZ * (TY + 1) * TX, NFZ = (TZ + 1) * TY * TX;
    static constexpr int NFB = NFX > NFY ? (NFX > NFZ ? NFX : NFZ) : (NFY > NFZ ? NFY : NFZ);
    static constexpr int PL = LX * LY * LZ;  // one row of the LDS primitives
    // LDS offset of brick cell (i, j, l), -HL <= i < TX + HL etc.
    static __device__ __forceinline__ int cell(int i, int j, int l) { return ((l + HL) * LY + (j + HL)) * LX + i + HL; }
    // ratio of the x-face at fi (0..TX) in row (j, l), j, l in -1..TY / -1..TZ
    static __device__ __forceinline__ int px(int fi, int j, int l) { return ((l + 1) * (TY + 2) + j + 1) * (TX + 1) + fi; }
    static __device__ __forceinline__ int py(int i, int fj, int l) { return NPX + ((l + 1) * (TY + 1) + fj) * (TX + 2) + i + 1; }
    static __device__ __forceinline__ int pz(int i, int j, int fl) { return NPX + NPY + (fl * (TY + 2) + j + 1) * (TX + 2) + i + 1; }
};

// Static LDS of the stage kernel: primitives of brick + halo, detector ratios,
// the flux buffer (two with db) and the reduction words.  Shapes over the 160 KiB
// of a gfx950 workgroup are not built (16x8x4 with two scalars).
constexpr long long kLdsBytes3 = 160 * 1024;
constexpr long long stage3_lds_bytes(int order, int nsc, int tx, int ty, int tz, int nt, bool db = false)
{
    const long long lx = tx + 2 * order, ly = ty + 2 * order, lz = tz + 2 * order;
    const long long npx = (long long)(tz + 2) * (ty + 2) * (tx + 1), npy = (long long)(tz + 2) * (ty + 1) * (tx + 2),
                    npz = (long long)(tz + 1) * (ty + 2) * (tx + 2);
    const long long nfx = (long long)tz * ty * (tx + 1), nfy = (long long)tz * (ty + 1) * tx, nfz = (long long)(tz + 1) * ty * tx;
    const long long nfb = nfx > nfy ? (nfx > nfz ? nfx : nfz) : (nfy > nfz ? nfy : nfz);
    return 8 * ((5 + nsc) * lx * ly * lz + npx + npy + npz + (db ? 2 : 1) * (5 + nsc) * nfb + nt / 64);
}
// A second flux buffer lets a sweep's accumulation overlap the next sweep's
// faces (three barriers instead of six); taken where it keeps the number of
// workgroups a CU can hold.
constexpr bool stage3_double_buffer(int order, int nsc, int tx, int ty, int tz, int nt)
{
    const long long one = stage3_lds_bytes(order, nsc, tx, ty, tz, nt, false);
    const long long two = stage3_lds_bytes(order, nsc, tx, ty, tz, nt, true);
    return two <= kLdsBytes3 && kLdsBytes3 / two == kLdsBytes3 / one;
}

// Detector minimum of Eq. (96) for the face of axis AXIS whose upper cell is
// brick cell (i, j, l): the face itself and, in each transverse direction, the
// two faces of each of its two cells.
template <int AXIS, class B>
__device__ __forceinline__ double face_detector(const double *__restrict__ sP, int i, int j, int l)
{
    if (AXIS == 0) {
        return rmin(rmin(rmin(sP[B::px(i, j, l)], sP[B::py(i - 1, j, l)]),
                         rmin(sP[B::py(i - 1, j + 1, l)], sP[B::py(i, j, l)])),
                    rmin(rmin(sP[B::py(i, j + 1, l)], sP[B::pz(i - 1, j, l)]),
                         rmin(sP[B::pz(i - 1, j, l + 1)], rmin(sP[B::pz(i, j, l)], sP[B::pz(i, j, l + 1)]))));
    } else if (AXIS == 1) {
        return rmin(rmin(rmin(sP[B::py(i, j, l)], sP[B::px(i, j - 1, l)]),
                         rmin(sP[B::px(i + 1, j - 1, l)], sP[B::px(i, j, l)])),
                    rmin(rmin(sP[B::px(i + 1, j, l)], sP[B::pz(i, j - 1, l)]),
                         rmin(sP[B::pz(i, j - 1, l + 1)], rmin(sP[B::pz(i, j, l)], sP[B::pz(i, j, l + 1)]))));
    } else {
        return rmin(rmin(rmin(sP[B::pz(i, j, l)], sP[B::px(i, j, l - 1)]),
                         rmin(sP[B::px(i + 1, j, l - 1)], sP[B::px(i, j, l)])),
                    rmin(rmin(sP[B::px(i + 1, j, l)], sP[B::py(i, j, l - 1)]),
                         rmin(sP[B::py(i, j + 1, l - 1)], rmin(sP[B::py(i, j, l)], sP[B::py(i, j + 1, l)]))));
    }
}

// MUSCL-minmod: the limited slope of a cell from its two neighbours along an
// axis, and the values half a cell above and below its centre.
__device__ __forceinline__ double slope3(double lo, double mid, double hi) { return minmod(mid - lo, hi - mid); }
__device__ __forceinline__ double extrap_up(double w, double s) { return fma(0.5, s, w); }
__device__ __forceinline__ double extrap_dn(double w, double s) { return fma(-0.5, s, w); }

// Row of the primitive state that goes into face-frame row k of a face of
// axis AXIS: rho, the normal velocity, the two others in cyclic order, p, k_m.
template <int AXIS>
__device__ __forceinline__ constexpr int frame_row(int k)
{
    return k == 1 ? 1 + AXIS : (k == 2 ? 1 + (AXIS + 1) % 3 : (k == 3 ? 1 + (AXIS + 2) % 3 : k));
}

// Flux per unit area of a face of axis AXIS from its face-frame states, rows
// scattered back to global order (rho, rho u, rho v, rho w, rho E, rho k_m);
// the face area enters the residual with 1 / V (axis_factor).
template <int PREC, int AXIS, int NSC>
__device__ __forceinline__ void frame_flux3(const DevSolve3 &S, const double *WL, const double *WR, double s1, double *F)
{
    constexpr int NR = 5 + NSC;
    using R = typename std::conditional<PREC == 0, double, float>::type;
    double Ff[NR];
    roeam_flux3<R, NSC>(S, WL, WR, s1, Ff);
#pragma unroll
    for (int k = 0; k < NR; ++k) F[frame_row<AXIS>(k)] = Ff[k];
}

// Face area over cell volume of axis AXIS: R = -(dFx ax/V + dFy ay/V + dFz az/V),
// summed as dFx (ax/V), then fma(dFy, ay/V, .), then fma(dFz, az/V, .) by
// every kernel form, so that they give the same bits.
template <int AXIS> __device__ __forceinline__ double axis_factor(const DevSolve3 &S)
{
    return (AXIS == 0 ? S.ax : (AXIS == 1 ? S.ay : S.az)) * S.inv_vol;
}

// Flux per unit area of the face of axis AXIS whose upper cell is brick cell
// (i, j, l), rows in global order.
template <int ORDER, int PREC, int AXIS, int NSC, class B>
__device__ __forceinline__ void brick_face(const DevSolve3 &S, const double *__restrict__ sW, const double *__restrict__ sP,
                                           int i, int j, int l, double *F)
{
    constexpr int NR = 5 + NSC;
    constexpr int PL = B::LX * B::LY * B::LZ;                     // one row of sW
    constexpr int ST = AXIS == 0 ? 1 : (AXIS == 1 ? B::LX : B::LX * B::LY);
    const int c = B::cell(i, j, l);
    double WL[NR], WR[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const double *r = sW + frame_row<AXIS>(k) * PL;
        const double m1 = r[c - ST], p0 = r[c];
        if (ORDER == 1) {
            WL[k] = m1;
            WR[k] = p0;
        } else {
            const double m2 = r[c - 2 * ST], p1 = r[c + ST];
            WL[k] = extrap_up(m1, slope3(m2, m1, p0));
            WR[k] = extrap_dn(p0, slope3(m1, p0, p1));
        }
    }
    double s1 = 1.0;
    if (S.s1_mode == 0 && S.scheme == SCHEME_ROEAM) s1 = detector_s1<PREC>(face_detector<AXIS, B>(sP, i, j, l));
    frame_flux3<PREC, AXIS, NSC>(S, WL, WR, s1, F);
}

// All faces of one axis into sF.
template <int ORDER, int PREC, int AXIS, int NSC, int TX, int TY, int TZ, int NT, class B>
__device__ __forceinline__ void faces_axis(const DevSolve3 &S, const double *__restrict__ sW, const double *__restrict__ sP,
                                           double (&sF)[5 + NSC][B::NFB], int i0, int j0, int l0)
{
    constexpr int NR = 5 + NSC;
    constexpr int FX = TX + (AXIS == 0), FY = TY + (AXIS == 1), FZ = TZ + (AXIS == 2);
    constexpr int NF = FX * FY * FZ;
    for (int f = threadIdx.x; f < NF; f += NT) {
        const int i = f % FX, r = f / FX, j = r % FY, l = r / FY;
        // the face lies on the grid (a face at index n of its axis is the upper boundary)
        if (i0 + i > S.nx - (AXIS != 0) || j0 + j > S.ny - (AXIS != 1) || l0 + l > S.nz - (AXIS != 2)) continue;
        double F[NR];
        brick_face<ORDER, PREC, AXIS, NSC, B>(S, sW, sP, i, j, l, F);
#pragma unroll
        for (int k = 0; k < NR; ++k) sF[k][f] = F[k];
    }
}

// Add the face differences of one axis (from sF), times the axis factor, to
// the cells' residual sums d (in registers), in the order x, y, z.
template <int AXIS, int NSC, int TX, int TY, int TZ, int NT, class B>
__device__ __forceinline__ void acc_axis(const DevSolve3 &S, const double (&sF)[5 + NSC][B::NFB], double (*d)[5 + NSC])
{
    const double ca = axis_factor<AXIS>(S);
    constexpr int NR = 5 + NSC;
    constexpr int FX = TX + (AXIS == 0), FY = TY + (AXIS == 1);
    constexpr int CPT = (TX * TY * TZ + NT - 1) / NT;
    constexpr int up = AXIS == 0 ? 1 : (AXIS == 1 ? FX : FX * FY);
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = threadIdx.x + m * NT;
        if (c >= TX * TY * TZ) continue;
        const int ci = c % TX, r = c / TX, cj = r % TY, cl = r / TY;
        const int lo = (cl * FY + cj) * FX + ci;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const double df = sF[k][lo + up] - sF[k][lo];
            d[m][k] = AXIS == 0 ? df * ca : fma(df, ca, d[m][k]);
        }
    }
}

// Shared memory of the stage kernel: primitives of brick + halo, detector
// ratios, one or two flux buffers and the reduction words.
template <int ORDER, int NSC, int TX, int TY, int TZ, int NT>
struct StageLds {
    using B = Brick<TX, TY, TZ, ORDER>;
    static constexpr int NR = 5 + NSC;
    static constexpr bool DB = stage3_double_buffer(ORDER, NSC, TX, TY, TZ, NT);
    double sW[NR * B::PL];
    double sP[B::NPX + B::NPY + B::NPZ];
    double sF[NR][B::NFB];
    double sF2[DB ? NR : 1][DB ? B::NFB : 1];
    double sRed[NT / 64];
};

// Stage codes, buffers and step logic as in the 2-D stage kernel:
//   0 residual only; 1 forward Euler / first SSP-RK3 stage (q -> qa);
//   2 (qa -> qb, + Q^n), 3 (qb -> q, + Q^n); 4-7 the four-stage scheme
//   (q -> qa, qa -> qb, qb -> qa, qa -> q; + Q^n from the second on).
// Transported scalars (NSC rows after rho E) ride along every step; the
// positivity check and the rate read the flow rows only.
__device__ __forceinline__ const double *stage_input3(const DevSolve3 &S, int stage)
{
    const int b = stage_in_buf(stage);
    return b == 0 ? S.q : (b == 2 ? S.qb : S.qa);
}

// Origin of brick t.  Bricks are numbered x fastest, then z, then y: the
// workgroups of one XCD take consecutive bricks at a time, so a brick's
// x-neighbours (whose 2-cell halo columns cost a whole cache line per row)
// and most z-neighbours (the largest halo faces, two TX x TY planes each) are
// staged at about the same time and those reads hit in the XCD's L2; the
// y-faces (two TX x TZ planes) come from further back.  Against x, y, z order
// this cut the HBM traffic of a 128^3 stage from 1.46 to 1.28 times the
// state's own bytes, at the same stage time.
template <int TX, int TY, int TZ>
__device__ __forceinline__ void brick_origin(const DevSolve3 &S, int t, int &i0, int &j0, int &l0)
{
    const int bxs = (S.nx + TX - 1) / TX, bzs = (S.nz + TZ - 1) / TZ;
    const int r = t / bxs;
    i0 = (t % bxs) * TX;
    l0 = (r % bzs) * TZ;
    j0 = (r / bzs) * TY;
}

// The own cells' stage input (and Q^n), into registers.
template <int NSC, int TX, int TY, int TZ, int NT>
__device__ __forceinline__ void own_cells(const DevSolve3 &S, int stage, const double *__restrict__ qin, int i0, int j0,
                                          int l0, double (*Qs)[5 + NSC], double (*Q0)[5 + NSC], long long *cidx)
{
    constexpr int NC = TX * TY * TZ, CPT = (NC + NT - 1) / NT, NR = 5 + NSC;
    const bool reads_qn = stage_reads_qn(stage);
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = threadIdx.x + m * NT;
        const int ci = c % TX, r = c / TX, cj = r % TY, cl = r / TY;
        const bool ok = c < NC && i0 + ci < S.nx && j0 + cj < S.ny && l0 + cl < S.nz;
        cidx[m] = ok ? (long long)(l0 + cl) * S.slab + (long long)(j0 + cj) * S.pitch + (i0 + ci) : 0;
        if (stage > 0) {
#pragma unroll
            for (int k = 0; k < NR; ++k) Qs[m][k] = gptr(qin)[k * S.plane + cidx[m]];
        }
        if (reads_qn) {
#pragma unroll
            for (int k = 0; k < NR; ++k) Q0[m][k] = gptr(S.q)[k * S.plane + cidx[m]];
        }
    }
}

// Brick + halo -> primitives in LDS, read directly.
template <int ORDER, int NSC, int TX, int TY, int TZ, int NT>
__device__ __forceinline__ void halo_direct(const DevSolve3 &S, const double *__restrict__ qin, int i0, int j0, int l0,
                                            double *__restrict__ sW)
{
    using B = Brick<TX, TY, TZ, ORDER>;
    constexpr int HL = ORDER, PL = B::PL, NR = 5 + NSC, NLOAD = (PL + NT - 1) / NT;
    const int nx = S.nx, ny = S.ny, nz = S.nz;
    const bool interior = i0 - HL >= 0 && i0 + TX + HL <= nx && j0 - HL >= 0 && j0 + TY + HL <= ny && l0 - HL >= 0 &&
                          l0 + TZ + HL <= nz;
    if (interior) {
        // every load of the thread first (lanes past the box load its first
        // cell, which is on the grid), then the conversions
        double Qh[NLOAD][NR];
#pragma unroll
        for (int it = 0; it < NLOAD; ++it) {
            const int e = threadIdx.x + it * NT < PL ? threadIdx.x + it * NT : 0;
            const int lx = e % B::LX, r = e / B::LX, ly = r % B::LY, lz = r / B::LY;
            const long long idx = (long long)(l0 - HL + lz) * S.slab + (long long)(j0 - HL + ly) * S.pitch + (i0 - HL + lx);
#pragma unroll
            for (int k = 0; k < NR; ++k) Qh[it][k] = gptr(qin)[k * S.plane + idx];
        }
#pragma unroll
        for (int it = 0; it < NLOAD; ++it) {
            const int e = threadIdx.x + it * NT;
            if (e >= PL) break;
            double W[NR];
            const double ir = to_prim3(S.gm1, Qh[it], W);
#pragma unroll
            for (int m = 0; m < NSC; ++m) W[5 + m] = Qh[it][5 + m] * ir;
#pragma unroll
            for (int k = 0; k < NR; ++k) sW[k * PL + e] = W[k];
        }
        return;
    }
#pragma unroll
    for (int it = 0; it < NLOAD; ++it) {
        const int e = threadIdx.x + it * NT;
        if (e >= PL) break;
        const int lx = e % B::LX, r = e / B::LX, ly = r % B::LY, lz = r / B::LY;
        // cells past the ghost layers of a ragged brick feed no face on the grid
        const int gi = min(i0 - HL + lx, nx + 1), gj = min(j0 - HL + ly, ny + 1), gl = min(l0 - HL + lz, nz + 1);
        double W[NR];
        fetch_prim3<NSC>(S, qin, gi, gj, gl, W);
#pragma unroll
        for (int k = 0; k < NR; ++k) sW[k * PL + e] = W[k];
    }
}

// Where the state of a cell within two layers of the grid comes from, by the
// rules of fetch_prim3 (z rule, then y, then x): returns 1 + side for a
// Dirichlet side, else 0 with idx the grid cell; bits 3, 4, 5 negate u, v, w
// (slip walls on the way).
__device__ __forceinline__ int map_cell3(const DevSolve3 &S, int i, int j, int l, long long &idx)
{
    int flip = 0;
    if (l < 0 || l >= S.nz) {
        const int sd = l < 0 ? SIDE3_B : SIDE3_T;
        const int kind = S.bc[sd];
        if (kind == BC_DIRICHLET) return 1 + sd;
        l = ghost_source(kind, l, S.nz);
        if (kind == BC_SLIPWALL) flip |= 32;
    }
    if (j < 0 || j >= S.ny) {
        const int sd = j < 0 ? SIDE3_S : SIDE3_N;
        const int kind = S.bc[sd];
        if (kind == BC_DIRICHLET) return (1 + sd) | flip;
        j = ghost_source(kind, j, S.ny);
        if (kind == BC_SLIPWALL) flip |= 16;
    }
    if (i < 0 || i >= S.nx) {
        const int sd = i < 0 ? SIDE3_W : SIDE3_E;
        const int kind = S.bc[sd];
        if (kind == BC_DIRICHLET) return (1 + sd) | flip;
        i = ghost_source(kind, i, S.nx);
        if (kind == BC_SLIPWALL) flip |= 8;
    }
    idx = (long long)l * S.slab + (long long)j * S.pitch + i;
    return flip;
}

// Issue the loads of a brick's halo into registers (Hq), with the source code
// of each staged cell (Hc; -1 past the staged box).
template <int ORDER, int NSC, int TX, int TY, int TZ, int NT>
__device__ __forceinline__ void halo_prefetch(const DevSolve3 &S, const double *__restrict__ qin, int i0, int j0, int l0,
                                              double (*Hq)[5 + NSC], int *Hc)
{
    using B = Brick<TX, TY, TZ, ORDER>;
    constexpr int HL = ORDER, PL = B::PL, NR = 5 + NSC, NLOAD = (PL + NT - 1) / NT;
    const int nx = S.nx, ny = S.ny, nz = S.nz;
    const bool interior = i0 - HL >= 0 && i0 + TX + HL <= nx && j0 - HL >= 0 && j0 + TY + HL <= ny && l0 - HL >= 0 &&
                          l0 + TZ + HL <= nz;
    // (the loads are consumed one brick later, so they need not be grouped)
#pragma unroll
    for (int it = 0; it < NLOAD; ++it) {
        const int e = threadIdx.x + it * NT;
        Hc[it] = -1;
        if (e >= PL) continue;
        const int lx = e % B::LX, r = e / B::LX, ly = r % B::LY, lz = r / B::LY;
        long long idx = 0;
        int code = 0;
        if (interior) {
            idx = (long long)(l0 - HL + lz) * S.slab + (long long)(j0 - HL + ly) * S.pitch + (i0 - HL + lx);
        } else {
            const int gi = min(i0 - HL + lx, nx + 1), gj = min(j0 - HL + ly, ny + 1), gl = min(l0 - HL + lz, nz + 1);
            code = map_cell3(S, gi, gj, gl, idx);
        }
        Hc[it] = code;
        if ((code & 7) == 0) {
#pragma unroll
            for (int k = 0; k < NR; ++k) Hq[it][k] = gptr(qin)[k * S.plane + idx];
        }
    }
}

// Prefetched halo -> primitives in LDS (bitwise what halo_direct stages).
template <int ORDER, int NSC, int TX, int TY, int TZ, int NT>
__device__ __forceinline__ void halo_commit(const DevSolve3 &S, const double (*Hq)[5 + NSC], const int *Hc,
                                            double *__restrict__ sW)
{
    using B = Brick<TX, TY, TZ, ORDER>;
    constexpr int PL = B::PL, NR = 5 + NSC, NLOAD = (PL + NT - 1) / NT;
#pragma unroll
    for (int it = 0; it < NLOAD; ++it) {
        const int e = threadIdx.x + it * NT;
        const int code = Hc[it];
        if (code < 0) continue;
        double W[NR];
        if ((code & 7) == 0) {
            const double ir = to_prim3(S.gm1, Hq[it], W);
#pragma unroll
            for (int m = 0; m < NSC; ++m) W[5 + m] = Hq[it][5 + m] * ir;
        } else {
            dirichlet3<NSC>(S, (code & 7) - 1, W);
        }
        if (code & 8) W[1] = -W[1];
        if (code & 16) W[2] = -W[2];
        if (code & 32) W[3] = -W[3];
#pragma unroll
        for (int k = 0; k < NR; ++k) sW[k * PL + e] = W[k];
    }
}

// Stage update of one cell at idx from its residual Rv, stage input Qs and
// Q^n (Q0): the new state, its positivity check and (last stage) its rate.
template <int NR>
__device__ __forceinline__ void stage_update3(const DevSolve3 &S, int stage, int last, double dt, const double *Rv,
                                              const double *Qs, const double *Q0, long long idx, double &lmax)
{
    // each combination written as the fused multiply-adds it rounds with, so
    // that every kernel form that inlines it rounds the same way
    double Qn[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        switch (stage) {
        case 1:
        case 8: Qn[k] = fma(dt, Rv[k], Qs[k]); break;
        case 2: Qn[k] = fma(0.75, Q0[k], 0.25 * fma(dt, Rv[k], Qs[k])); break;
        case 3: Qn[k] = fma(1.0 / 3.0, Q0[k], (2.0 / 3.0) * fma(dt, Rv[k], Qs[k])); break;
        case 4: Qn[k] = fma(0.25 * dt, Rv[k], Qs[k]); break;
        case 5: Qn[k] = fma((1.0 / 3.0) * dt, Rv[k], Q0[k]); break;
        case 6: Qn[k] = fma(0.5 * dt, Rv[k], Q0[k]); break;
        default: Qn[k] = fma(dt, Rv[k], Q0[k]); break;
        }
    }
    const int bout = stage_out_buf(stage);
    double *__restrict__ qo = bout == 0 ? S.q : (bout == 2 ? S.qb : S.qa);
#pragma unroll
    for (int k = 0; k < NR; ++k) gptr(qo)[k * S.plane + idx] = Qn[k];
    double W[5];
    const double ir = to_prim3(S.gm1, Qn, W);
    if (!physical3(W)) atomicOr(&S.slot->nonphys, 1);
    else if (last) lmax = rmax(lmax, cell_rate3(S, W, ir));
}

// Detector ratios, faces, residual and stage update of one brick whose
// primitives are in LDS (the caller has synchronised after staging them);
// the rate of the new state goes into lmax.
template <int ORDER, int PREC, int NSC, int TX, int TY, int TZ, int NT>
__device__ __forceinline__ void brick_body(const DevSolve3 &S, StageLds<ORDER, NSC, TX, TY, TZ, NT> &L, int stage,
                                           int last, double dt, int i0, int j0, int l0, const double (*Qs)[5 + NSC],
                                           const double (*Q0)[5 + NSC], const long long *cidx, double *r_out,
                                           double &lmax)
{
    using B = Brick<TX, TY, TZ, ORDER>;
    constexpr int NC = TX * TY * TZ;
    constexpr int CPT = (NC + NT - 1) / NT;
    constexpr int PL = B::PL;
    constexpr int NR = 5 + NSC;
    const int tid = threadIdx.x;
    const int nx = S.nx, ny = S.ny, nz = S.nz;
    double *__restrict__ sW = L.sW;
    double *__restrict__ sP = L.sP;

    // 2. detector ratios, Eq. (97), of every face within one layer of the brick
    if (S.s1_mode == 0 && S.scheme == SCHEME_ROEAM) {
        for (int e = tid; e < B::NPX + B::NPY + B::NPZ; e += NT) {
            int a, st;  // LDS offset of the lower cell, stride to the upper one
            if (e < B::NPX) {
                const int fi = e % (TX + 1), r = e / (TX + 1), j = r % (TY + 2) - 1, l = r / (TY + 2) - 1;
                a = B::cell(fi - 1, j, l);
                st = 1;
            } else if (e < B::NPX + B::NPY) {
                const int f = e - B::NPX;
                const int i = f % (TX + 2) - 1, r = f / (TX + 2), fj = r % (TY + 1), l = r / (TY + 1) - 1;
                a = B::cell(i, fj - 1, l);
                st = B::LX;
            } else {
                const int f = e - B::NPX - B::NPY;
                const int i = f % (TX + 2) - 1, r = f / (TX + 2), j = r % (TY + 2) - 1, fl = r / (TY + 2);
                a = B::cell(i, j, fl - 1);
                st = B::LX * B::LY;
            }
            const double *p4 = sW + 4 * PL;
            sP[e] = detector_P(p4[a], sW[a], p4[a + st], sW[a + st]);
        }
        __syncthreads();
    }

    // 3. x-, y- and z-faces, each exactly once; residual sums in the order x, y, z
    double d[CPT][NR];
    faces_axis<ORDER, PREC, 0, NSC, TX, TY, TZ, NT, B>(S, sW, sP, L.sF, i0, j0, l0);
    __syncthreads();
    if constexpr (StageLds<ORDER, NSC, TX, TY, TZ, NT>::DB) {
        // x sums while the y-faces go to the second buffer, y sums while the
        // z-faces go to the first (whose readers passed the barrier between)
        acc_axis<0, NSC, TX, TY, TZ, NT, B>(S, L.sF, d);
        faces_axis<ORDER, PREC, 1, NSC, TX, TY, TZ, NT, B>(S, sW, sP, L.sF2, i0, j0, l0);
        __syncthreads();
        acc_axis<1, NSC, TX, TY, TZ, NT, B>(S, L.sF2, d);
        faces_axis<ORDER, PREC, 2, NSC, TX, TY, TZ, NT, B>(S, sW, sP, L.sF, i0, j0, l0);
        __syncthreads();
        acc_axis<2, NSC, TX, TY, TZ, NT, B>(S, L.sF, d);
    } else {
        acc_axis<0, NSC, TX, TY, TZ, NT, B>(S, L.sF, d);
        __syncthreads();
        faces_axis<ORDER, PREC, 1, NSC, TX, TY, TZ, NT, B>(S, sW, sP, L.sF, i0, j0, l0);
        __syncthreads();
        acc_axis<1, NSC, TX, TY, TZ, NT, B>(S, L.sF, d);
        __syncthreads();
        faces_axis<ORDER, PREC, 2, NSC, TX, TY, TZ, NT, B>(S, sW, sP, L.sF, i0, j0, l0);
        __syncthreads();
        acc_axis<2, NSC, TX, TY, TZ, NT, B>(S, L.sF, d);
    }

    // 4. R = -(sum of face flux differences times area / V) and the stage update
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = tid + m * NT;
        const int ci = c % TX, r = c / TX, cj = r % TY, cl = r / TY;
        if (c >= NC || i0 + ci >= nx || j0 + cj >= ny || l0 + cl >= nz) continue;
        double Rv[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) Rv[k] = -d[m][k];
        const long long idx = cidx[m];
        if (stage == 0) {
#pragma unroll
            for (int k = 0; k < NR; ++k) gptr(r_out)[k * S.plane + idx] = Rv[k];
            if (last) {
                const int o = B::cell(ci, cj, cl);
                double W[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) W[k] = sW[k * PL + o];
                lmax = rmax(lmax, cell_rate3(S, W, rcp_nr(W[0])));
            }
            continue;
        }
        stage_update3<NR>(S, stage, last, dt, Rv, Qs[m], Q0[m], idx, lmax);
    }
}

// One workgroup per brick.
template <int ORDER, int PREC, int NSC, int TX, int TY, int TZ, int NT>
__global__ __launch_bounds__(NT) void k_stage3(const DevSolve3 *__restrict__ Sp, int stage, int p, int last, double *r_out)
{
    constexpr int NC = TX * TY * TZ, CPT = (NC + NT - 1) / NT, NR = 5 + NSC;
    const DevSolve3 &S = *Sp;
    __shared__ StageLds<ORDER, NSC, TX, TY, TZ, NT> L;
    const int bxs = (S.nx + TX - 1) / TX, bys = (S.ny + TY - 1) / TY, bzs = (S.nz + TZ - 1) / TZ;
    const int nb = bxs * bys * bzs;
    const int t = xcd_tile(blockIdx.x, nb);
    if (t >= nb) return;
    int i0, j0, l0;
    brick_origin<TX, TY, TZ>(S, t, i0, j0, l0);
    const double *__restrict__ qin = stage_input3(S, stage);
    // the step-state words, then the own cells' stage input (and Q^n), whose
    // latency hides behind the face work
    Slot &z = *S.slot;
    const StepWords sw = stage > 0 ? load_step_words(z, p, stage) : StepWords{};
    double Qs[CPT][NR], Q0[CPT][NR];
    long long cidx[CPT];
    own_cells<NSC, TX, TY, TZ, NT>(S, stage, qin, i0, j0, l0, Qs, Q0, cidx);
    double dt = 0.0;
    if (stage > 0 && !begin_stage(z, sw, p, stage, last, t == 0, dt)) return;
    // 1. brick + halo -> primitives in LDS
    halo_direct<ORDER, NSC, TX, TY, TZ, NT>(S, qin, i0, j0, l0, L.sW);
    __syncthreads();
    double lmax = 0.0;
    brick_body<ORDER, PREC, NSC, TX, TY, TZ, NT>(S, L, stage, last, dt, i0, j0, l0, Qs, Q0, cidx, r_out, lmax);
    if (last) reduce_rate_block<NT>(z, stage == 0 ? 0 : rate_set(sw.steps + 1), lmax, L.sRed);
}

// Persistent form: gridDim.x (a multiple of 8) resident workgroups; those of
// XCD x (ids x mod 8) take the band of bricks [x c, (x + 1) c), c = ceil(n / 8),
// in turn, and each loads the next brick's halo into registers while it works
// on the current one.  Same arithmetic, bitwise the same result.
template <int ORDER, int PREC, int NSC, int TX, int TY, int TZ, int NT>
__global__ __launch_bounds__(NT) void k_stage3p(const DevSolve3 *__restrict__ Sp, int stage, int p, int last,
                                                double *r_out)
{
    using B = Brick<TX, TY, TZ, ORDER>;
    constexpr int NC = TX * TY * TZ, CPT = (NC + NT - 1) / NT, NR = 5 + NSC, NLOAD = (B::PL + NT - 1) / NT;
    const DevSolve3 &S = *Sp;
    __shared__ StageLds<ORDER, NSC, TX, TY, TZ, NT> L;
    const int bxs = (S.nx + TX - 1) / TX, bys = (S.ny + TY - 1) / TY, bzs = (S.nz + TZ - 1) / TZ;
    const int nb = bxs * bys * bzs;
    const int chunk = (nb + 7) >> 3, xcd = blockIdx.x & 7, per_xcd = gridDim.x >> 3;
    const int t_end = min(nb, (xcd + 1) * chunk);
    int t = xcd * chunk + (blockIdx.x >> 3);
    const double *__restrict__ qin = stage_input3(S, stage);
    Slot &z = *S.slot;
    const StepWords sw = stage > 0 ? load_step_words(z, p, stage) : StepWords{};
    double Hq[NLOAD][NR];
    int Hc[NLOAD];
    int i0, j0, l0;
    if (t < t_end) {
        brick_origin<TX, TY, TZ>(S, t, i0, j0, l0);
        halo_prefetch<ORDER, NSC, TX, TY, TZ, NT>(S, qin, i0, j0, l0, Hq, Hc);
    }
    double dt = 0.0;
    if (stage > 0 && !begin_stage(z, sw, p, stage, last, blockIdx.x == 0, dt)) return;
    double lmax = 0.0;
    for (; t < t_end; t += per_xcd) {
        brick_origin<TX, TY, TZ>(S, t, i0, j0, l0);
        double Qs[CPT][NR], Q0[CPT][NR];
        long long cidx[CPT];
        own_cells<NSC, TX, TY, TZ, NT>(S, stage, qin, i0, j0, l0, Qs, Q0, cidx);
        __syncthreads();  // the previous brick's readers of the LDS arrays are done
        halo_commit<ORDER, NSC, TX, TY, TZ, NT>(S, Hq, Hc, L.sW);
        __syncthreads();
        if (t + per_xcd < t_end) {
            int i1, j1, l1;
            brick_origin<TX, TY, TZ>(S, t + per_xcd, i1, j1, l1);
            halo_prefetch<ORDER, NSC, TX, TY, TZ, NT>(S, qin, i1, j1, l1, Hq, Hc);
        }
        brick_body<ORDER, PREC, NSC, TX, TY, TZ, NT>(S, L, stage, last, dt, i0, j0, l0, Qs, Q0, cidx, r_out, lmax);
    }
    if (last) reduce_rate_block<NT>(z, stage == 0 ? 0 : rate_set(sw.steps + 1), lmax, L.sRed);
}

// ---------------------------------------------------------------------------
// z-marching form (2.5-D blocking)
// ---------------------------------------------------------------------------
// A workgroup owns a column tile of TX x TY cells and a run of planes of it,
// and walks up the run one plane at a time.  LDS holds one plane of
// primitives with its x-y halo (the plane whose x- and y-faces are being
// evaluated), p and rho of the plane above it, the detector ratios of the
// faces in and between the two planes, and one flux buffer; the next
// plane's footprint is loaded into registers while the current one is
// worked on.  Thread c < TX TY owns column c: its z-faces come from its own
// registers (the reconstructed upper state of the plane below and the flux
// through the plane's lower face carry over from one plane to the next).
// Every face of the run is evaluated once, the run's lowest z-face once more
// by the run below; each plane's footprint is loaded once per run.  Same
// arithmetic as the brick kernels, bitwise the same result.
template <int TX, int TY, int HL>
struct ZPlane {
    static constexpr int LX = TX + 2 * HL, LY = TY + 2 * HL, PL = LX * LY;  // the staged plane
    static constexpr int NI = TX * TY;                                       // interior cells
    static constexpr int RX = TX + 2, RP = RX * (TY + 2);                    // one-layer footprint
    static constexpr int NPX = (TX + 1) * (TY + 2), NPY = (TX + 2) * (TY + 1);
    static constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1);
    static constexpr int NFB = NFX > NFY ? NFX : NFY;
    // staged-plane offset of cell (i, j), -HL <= i < TX + HL, -HL <= j < TY + HL
    static __device__ __forceinline__ int cell(int i, int j) { return (j + HL) * LX + i + HL; }
    // one-layer footprint offset of cell (i, j), -1 <= i <= TX, -1 <= j <= TY
    static __device__ __forceinline__ int rc(int i, int j) { return (j + 1) * RX + i + 1; }
    // ratio of the x-face at fi (0..TX) in row j (-1..TY); of the y-face at fj (0..TY) in column i (-1..TX)
    static __device__ __forceinline__ int px(int fi, int j) { return (j + 1) * (TX + 1) + fi; }
    static __device__ __forceinline__ int py(int i, int fj) { return NPX + fj * (TX + 2) + i + 1; }
    // footprint slot e -> staged-plane position (lx, ly): the interior first
    // (x fastest, so that slot c is column c's own cell), then the rows below,
    // the rows above and the side columns of the halo
    static __device__ __forceinline__ void slot_xy(int e, int &lx, int &ly)
    {
        if (e < NI) {
            lx = HL + e % TX;
            ly = HL + e / TX;
            return;
        }
        int r = e - NI;
        if (r < HL * LX) {
            lx = r % LX;
            ly = r / LX;
            return;
        }
        r -= HL * LX;
        if (r < HL * LX) {
            lx = r % LX;
            ly = TY + HL + r / LX;
            return;
        }
        r -= HL * LX;
        const int c = r % (2 * HL);
        lx = c < HL ? c : TX + c;
        ly = HL + r / (2 * HL);
    }
};

template <int ORDER, int NSC, int TX, int TY, int NT>
struct ZStageLds {
    using P = ZPlane<TX, TY, ORDER>;
    static constexpr int NR = 5 + NSC;
    double sW[NR * P::PL];           // primitives of the plane whose x- and y-faces are evaluated
    double sPR[2 * P::RP];           // p, then rho, of the plane above it
    double sPxy[2][P::NPX + P::NPY]; // x- and y-face ratios of a plane, by plane parity
    double sPz[2][P::RP];            // z-face ratios below a plane, by plane parity
    double sF[NR][P::NFB];
    // each thread's footprint slots past the first (slot e >= NT at e - NT):
    // the current plane's primitives, kept by the thread for the next plane's
    // staging (private to the thread, so no barrier guards them)
    double sKeep[NR][P::PL > NT ? P::PL - NT : 1];
    double sRed[NT / 64];
};
constexpr long long zstage3_lds_bytes(int order, int nsc, int tx, int ty, int nt)
{
    const long long pl = (long long)(tx + 2 * order) * (ty + 2 * order), rp = (long long)(tx + 2) * (ty + 2);
    const long long npxy = (long long)(tx + 1) * (ty + 2) + (long long)(tx + 2) * (ty + 1);
    const long long nfb = (tx + 1) * ty > tx * (ty + 1) ? (long long)(tx + 1) * ty : (long long)tx * (ty + 1);
    const long long keep = pl > nt ? pl - nt : 1;
    return 8 * ((5 + nsc) * pl + 2 * rp + 2 * npxy + 2 * rp + (5 + nsc) * nfb + (5 + nsc) * keep + nt / 64);
}

// Issue the loads of footprint slots SLO..SHI-1 of plane l (own cells only
// when own_only) into Fq, with the source code of each slot in Fc as
// halo_prefetch gives it (-1: no slot).
template <int ORDER, int NSC, int TX, int TY, int NT, int SLO, int SHI>
__device__ __forceinline__ void zplane_load(const DevSolve3 &S, const double *__restrict__ qin, int tid, int i0, int j0,
                                            int l, bool own_only, double (*Fq)[5 + NSC], int *Fc)
{
    using P = ZPlane<TX, TY, ORDER>;
    constexpr int HL = ORDER, NR = 5 + NSC;
    const bool inner = i0 - HL >= 0 && i0 + TX + HL <= S.nx && j0 - HL >= 0 && j0 + TY + HL <= S.ny && l >= 0 &&
                       l < S.nz;
#pragma unroll
    for (int s = SLO; s < SHI; ++s) {
        const int e = tid + s * NT;
        Fc[s] = -1;
        if (e >= P::PL || (own_only && e >= P::NI)) continue;
        int lx, ly;
        P::slot_xy(e, lx, ly);
        long long idx = 0;
        int code = 0;
        if (inner) {
            idx = (long long)l * S.slab + (long long)(j0 - HL + ly) * S.pitch + (i0 - HL + lx);
        } else {
            // cells past the ghost layers of a ragged tile feed no face on the grid
            const int gi = min(i0 - HL + lx, S.nx + 1), gj = min(j0 - HL + ly, S.ny + 1);
            code = map_cell3(S, gi, gj, l, idx);
        }
        Fc[s] = code;
        if ((code & 7) == 0) {
#pragma unroll
            for (int k = 0; k < NR; ++k) Fq[s][k] = gptr(qin)[k * S.plane + idx];
        }
    }
}

// Primitives of a loaded footprint slot (bitwise what halo_commit stages).
template <int NSC>
__device__ __forceinline__ void zslot_prim(const DevSolve3 &S, const double *Q, int code, double *W)
{
    if ((code & 7) == 0) {
        const double ir = to_prim3(S.gm1, Q, W);
#pragma unroll
        for (int m = 0; m < NSC; ++m) W[5 + m] = Q[5 + m] * ir;
    } else {
        dirichlet3<NSC>(S, (code & 7) - 1, W);
    }
    if (code & 8) W[1] = -W[1];
    if (code & 16) W[2] = -W[2];
    if (code & 32) W[3] = -W[3];
}

// x- (AXIS 0) or y-face (AXIS 1) of the staged plane whose upper cell is (i, j):
// flux per unit area in global row order.  cur: the plane's own x-y ratios; lo,
// hi: the z-face ratios below and above it (the nine faces of Eq. 96, as
// face_detector takes them).
template <int ORDER, int PREC, int AXIS, int NSC, class P>
__device__ __forceinline__ void zplane_face(const DevSolve3 &S, const double *__restrict__ sW,
                                            const double *__restrict__ cur, const double *__restrict__ lo,
                                            const double *__restrict__ hi, int i, int j, double *F)
{
    constexpr int NR = 5 + NSC;
    constexpr int ST = AXIS == 0 ? 1 : P::LX;
    const int c = P::cell(i, j);
    double WL[NR], WR[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const double *r = sW + frame_row<AXIS>(k) * P::PL;
        const double m1 = r[c - ST], p0 = r[c];
        if (ORDER == 1) {
            WL[k] = m1;
            WR[k] = p0;
        } else {
            const double m2 = r[c - 2 * ST], p1 = r[c + ST];
            WL[k] = extrap_up(m1, slope3(m2, m1, p0));
            WR[k] = extrap_dn(p0, slope3(m1, p0, p1));
        }
    }
    double s1 = 1.0;
    if (S.s1_mode == 0 && S.scheme == SCHEME_ROEAM) {
        double dmin;
        if (AXIS == 0) {
            dmin = rmin(rmin(rmin(cur[P::px(i, j)], cur[P::py(i - 1, j)]), rmin(cur[P::py(i - 1, j + 1)], cur[P::py(i, j)])),
                        rmin(rmin(cur[P::py(i, j + 1)], lo[P::rc(i - 1, j)]),
                             rmin(hi[P::rc(i - 1, j)], rmin(lo[P::rc(i, j)], hi[P::rc(i, j)]))));
        } else {
            dmin = rmin(rmin(rmin(cur[P::py(i, j)], cur[P::px(i, j - 1)]), rmin(cur[P::px(i + 1, j - 1)], cur[P::px(i, j)])),
                        rmin(rmin(cur[P::px(i + 1, j)], lo[P::rc(i, j - 1)]),
                             rmin(hi[P::rc(i, j - 1)], rmin(lo[P::rc(i, j)], hi[P::rc(i, j)]))));
        }
        s1 = detector_s1<PREC>(dmin);
    }
    frame_flux3<PREC, AXIS, NSC>(S, WL, WR, s1, F);
}

// A column owner's part of plane step m: the own cell of plane m + 1 into
// primitives (order 2), the z-face between planes m - 1 and m, and from the
// run's second plane on the residual and stage update of plane m - 1.  H0:
// the own cell of plane m; F0, c0: that of plane m + 1 as loaded; d: the
// plane's x- and y-face sums (each difference times its axis factor); Wup
// and zlo carry to the next plane.
template <int ORDER, int PREC, int NSC, int TX, int TY, int NT>
__device__ __forceinline__ void column_z(const DevSolve3 &S, ZStageLds<ORDER, NSC, TX, TY, NT> &L, int stage, int last,
                                         double dt, int m, int z0, int i0, int j0, int ci, int cj, bool col,
                                         bool reads_qn, bool detect, const double *__restrict__ qin, double *r_out,
                                         const double *H0, double *F0, int c0, const double *d, double *Wup,
                                         double *zlo, double &lmax)
{
    using P = ZPlane<TX, TY, ORDER>;
    constexpr int NR = 5 + NSC;
    const int cur = m & 1, prv = cur ^ 1;
    if (ORDER == 2) {
        double W[NR];
        zslot_prim<NSC>(S, F0, c0, W);
#pragma unroll
        for (int k = 0; k < NR; ++k) F0[k] = W[k];
    }
    if (m < z0) {
        // below the run: only the reconstructed upper state of plane z0 - 1
        if (ORDER == 2) {
#pragma unroll
            for (int k = 0; k < NR; ++k) Wup[k] = extrap_up(H0[k], slope3(Wup[k], H0[k], F0[k]));
        }
        return;
    }
    const int cb = P::cell(ci, cj);
    double WL[NR], WR[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int row = frame_row<2>(k);
        if (ORDER == 1) {
            WL[k] = L.sW[row * P::PL + cb];
            WR[k] = H0[row];
        } else {
            const double sl = slope3(L.sW[row * P::PL + cb], H0[row], F0[row]);
            WL[k] = Wup[row];
            WR[k] = extrap_dn(H0[row], sl);
            Wup[row] = extrap_up(H0[row], sl);
        }
    }
    double s1 = 1.0;
    if (detect) {
        const double *bl = L.sPxy[prv], *ab = L.sPxy[cur];
        const double dmin =
            rmin(rmin(rmin(L.sPz[cur][P::rc(ci, cj)], bl[P::px(ci, cj)]), rmin(bl[P::px(ci + 1, cj)], ab[P::px(ci, cj)])),
                 rmin(rmin(ab[P::px(ci + 1, cj)], bl[P::py(ci, cj)]),
                      rmin(bl[P::py(ci, cj + 1)], rmin(ab[P::py(ci, cj)], ab[P::py(ci, cj + 1)]))));
        s1 = detector_s1<PREC>(dmin);
    }
    double zf[NR];
    frame_flux3<PREC, 2, NSC>(S, WL, WR, s1, zf);
    if (col && m > z0) {
        // R = -(sum of face flux differences times area / V) of plane m - 1 and its stage update
        const long long idx = (long long)(m - 1) * S.slab + (long long)(j0 + cj) * S.pitch + (i0 + ci);
        double Rv[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) Rv[k] = -fma(zf[k] - zlo[k], axis_factor<2>(S), d[k]);
        if (stage == 0) {
#pragma unroll
            for (int k = 0; k < NR; ++k) gptr(r_out)[k * S.plane + idx] = Rv[k];
            if (last) {
                double W[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) W[k] = L.sW[k * P::PL + cb];
                lmax = rmax(lmax, cell_rate3(S, W, rcp_nr(W[0])));
            }
        } else {
            double Qs[NR], Q0[NR];
#pragma unroll
            for (int k = 0; k < NR; ++k) Qs[k] = gptr(qin)[k * S.plane + idx];
            if (reads_qn) {
#pragma unroll
                for (int k = 0; k < NR; ++k) Q0[k] = gptr(S.q)[k * S.plane + idx];
            }
            stage_update3<NR>(S, stage, last, dt, Rv, Qs, Q0, idx, lmax);
        }
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) zlo[k] = zf[k];
}

template <int ORDER, int PREC, int NSC, int TX, int TY, int NT>
__global__ __launch_bounds__(NT, 3) void k_stage3z(const DevSolve3 *__restrict__ Sp, int stage, int p, int last,
                                                   double *r_out, int zc)
{
    using P = ZPlane<TX, TY, ORDER>;
    constexpr int NR = 5 + NSC, NS = (P::PL + NT - 1) / NT;
    static_assert(P::NI <= NT && P::NFX <= NT && P::NFY <= NT, "one column, one x-face and one y-face per thread");
    const DevSolve3 &S = *Sp;
    __shared__ ZStageLds<ORDER, NSC, TX, TY, NT> L;
    const int tid = threadIdx.x;
    const int ntx = (S.nx + TX - 1) / TX, nty = (S.ny + TY - 1) / TY, nt = ntx * nty;
    // runs numbered column tile fastest: each XCD takes a slab of whole
    // layers of runs, so the runs it holds at once are x- and y-neighbours at
    // the same height (their shared halo lines are read from its L2 once)
    // and a run's successor above starts as it ends (the planes they share
    // are still in that L2)
    int ct, z0, z1, t;
    if (zc > 0) {
        // runs of zc planes
        const int nb = nt * ((S.nz + zc - 1) / zc);
        t = xcd_tile(blockIdx.x, nb);
        if (t >= nb) return;
        ct = t % nt;
        z0 = (t / nt) * zc;
        z1 = min(z0 + zc, S.nz);
    } else {
        // -zc runs in all (nt <= -zc <= nt nz): every tile takes q or q + 1
        // of them (the first -zc mod nt tiles the extra one) and its height
        // is cut into its runs as evenly as whole planes allow; layer k holds
        // the k-th run of every tile that has one
        const int nb = -zc, q = nb / nt, rem = nb % nt;
        t = xcd_tile(blockIdx.x, nb);
        if (t >= nb) return;
        const int k = t < q * nt ? t / nt : q;
        ct = t < q * nt ? t % nt : t - q * nt;
        const int runs = q + (ct < rem ? 1 : 0);
        z0 = (int)((long long)S.nz * k / runs);
        z1 = (int)((long long)S.nz * (k + 1) / runs);
    }
    const int i0 = (ct % ntx) * TX, j0 = (ct / ntx) * TY;
    const double *__restrict__ qin = stage_input3(S, stage);
    Slot &z = *S.slot;
    const StepWords sw = stage > 0 ? load_step_words(z, p, stage) : StepWords{};
    const bool reads_qn = stage_reads_qn(stage);
    const bool detect = S.s1_mode == 0 && S.scheme == SCHEME_ROEAM;
    const bool own = tid < P::NI;

    double Fq[NS][NR];  // the next plane's footprint as loaded; slot 0 of a column owner in primitives (order 2)
    int Fc[NS];
    double H0[NR];      // the current plane's footprint slot 0, primitives (slots past it: sKeep)
    double Wup[NR];     // order 2: the own cell of the plane below, reconstructed at its upper face
    double zlo[NR];     // flux through the lower z-face of the plane being finished
    if (ORDER == 2) {
        // own cell two planes below the run, then the footprint of the plane below it
        zplane_load<ORDER, NSC, TX, TY, NT, 0, 1>(S, qin, tid, i0, j0, z0 - 2, true, Fq, Fc);
        if (own) zslot_prim<NSC>(S, Fq[0], Fc[0], Wup);
    }
    zplane_load<ORDER, NSC, TX, TY, NT, 0, NS>(S, qin, tid, i0, j0, z0 - 1, false, Fq, Fc);
    if (ORDER == 2 && own) {
        double W[NR];
        zslot_prim<NSC>(S, Fq[0], Fc[0], W);
#pragma unroll
        for (int k = 0; k < NR; ++k) Fq[0][k] = W[k];
    }
    double dt = 0.0;
    if (stage > 0 && !begin_stage(z, sw, p, stage, last, t == 0, dt)) return;
    double lmax = 0.0;

    for (int m = z0 - 1; m <= z1; ++m) {
        const int cur = m & 1, prv = cur ^ 1;
        // the thread's indices.  With FP64 coefficients they are derived
        // anew in each plane step from a copy of the thread id the compiler
        // cannot see through: hoisted out of the loop they would hold
        // registers the face work needs, and spill (measured 7% slower); the
        // FP32-coefficient kernel has the registers to keep them (4% faster)
        int tq = tid;
        if constexpr (PREC == 0) asm volatile("" : "+v"(tq));
        const int ci = tq % TX, cj = tq / TX;
        const bool col = own && i0 + ci < S.nx && j0 + cj < S.ny;
        // plane m - 1 into the staged plane, plane m's primitives from the
        // loaded footprint, its p and rho into the one-layer footprint.  No
        // barrier first: the last plane's other readers of these arrays
        // passed the barrier after its y-faces (its ratios one before), and
        // a thread's own cell, which the column step reads after it, is
        // written by the thread itself.
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int e = tq + s * NT;
            if (e >= P::PL) continue;
            int lx, ly;
            P::slot_xy(e, lx, ly);
            if (m >= z0) {
#pragma unroll
                for (int k = 0; k < NR; ++k)
                    L.sW[k * P::PL + ly * P::LX + lx] = s == 0 ? H0[k] : L.sKeep[k][e - NT];
            }
            double W[NR];
            if (ORDER == 2 && s == 0 && own) {
#pragma unroll
                for (int k = 0; k < NR; ++k) W[k] = Fq[0][k];
            } else {
                zslot_prim<NSC>(S, Fq[s], Fc[s], W);
            }
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                if (s == 0) H0[k] = W[k];
                else L.sKeep[k][e - NT] = W[k];
            }
            const int i = lx - ORDER, j = ly - ORDER;
            if (i >= -1 && i <= TX && j >= -1 && j <= TY) {
                L.sPR[P::rc(i, j)] = W[4];
                L.sPR[P::RP + P::rc(i, j)] = W[0];
            }
        }
        // the plane above: slot 0 now (a column owner's is its z-stencil; at
        // the top of the run only those are loaded), the other slots once the
        // detector ratios are in LDS
        if (m < z1 || ORDER == 2) zplane_load<ORDER, NSC, TX, TY, NT, 0, 1>(S, qin, tq, i0, j0, m + 1, m == z1, Fq, Fc);
        __syncthreads();

        // detector ratios, Eq. (97): x- and y-faces of plane m, z-faces between m - 1 and m
        if (detect) {
            const double *pP = L.sPR, *pR = L.sPR + P::RP;
            double *rxy = L.sPxy[cur];
            const int ne = P::NPX + P::NPY + (m >= z0 ? P::RP : 0);
            for (int e = tq; e < ne; e += NT) {
                if (e < P::NPX) {
                    const int fi = e % (TX + 1), j = e / (TX + 1) - 1;
                    const int a = P::rc(fi - 1, j), b = P::rc(fi, j);
                    rxy[e] = detector_P(pP[a], pR[a], pP[b], pR[b]);
                } else if (e < P::NPX + P::NPY) {
                    const int f = e - P::NPX;
                    const int i = f % (TX + 2) - 1, fj = f / (TX + 2);
                    const int a = P::rc(i, fj - 1), b = P::rc(i, fj);
                    rxy[e] = detector_P(pP[a], pR[a], pP[b], pR[b]);
                } else {
                    const int f = e - P::NPX - P::NPY;
                    const int c = P::cell(f % (TX + 2) - 1, f / (TX + 2) - 1);
                    L.sPz[cur][f] = detector_P(L.sW[4 * P::PL + c], L.sW[c], pP[f], pR[f]);
                }
            }
        }
        __syncthreads();

        if (m < z1) zplane_load<ORDER, NSC, TX, TY, NT, 1, NS>(S, qin, tq, i0, j0, m + 1, false, Fq, Fc);
        // x- and y-faces of plane m - 1, residual sums x, then y
        double d[NR];
        if (m > z0) {
            const double *cxy = L.sPxy[prv], *zl = L.sPz[prv], *zh = L.sPz[cur];
            if (tq < P::NFX) {
                const int fi = tq % (TX + 1), j = tq / (TX + 1);
                if (i0 + fi <= S.nx && j0 + j < S.ny) {
                    double F[NR];
                    zplane_face<ORDER, PREC, 0, NSC, P>(S, L.sW, cxy, zl, zh, fi, j, F);
#pragma unroll
                    for (int k = 0; k < NR; ++k) L.sF[k][tq] = F[k];
                }
            }
            __syncthreads();
            if (own) {
                const int lo = cj * (TX + 1) + ci;
#pragma unroll
                for (int k = 0; k < NR; ++k) d[k] = (L.sF[k][lo + 1] - L.sF[k][lo]) * axis_factor<0>(S);
            }
            __syncthreads();
            if (tq < P::NFY) {
                const int i = tq % TX, fj = tq / TX;
                if (i0 + i < S.nx && j0 + fj <= S.ny) {
                    double F[NR];
                    zplane_face<ORDER, PREC, 1, NSC, P>(S, L.sW, cxy, zl, zh, i, fj, F);
#pragma unroll
                    for (int k = 0; k < NR; ++k) L.sF[k][tq] = F[k];
                }
            }
            __syncthreads();
            if (own) {
                const int lo = cj * TX + ci;
#pragma unroll
                for (int k = 0; k < NR; ++k) d[k] = fma(L.sF[k][lo + TX] - L.sF[k][lo], axis_factor<1>(S), d[k]);
            }
        }

        if (own) column_z<ORDER, PREC, NSC, TX, TY, NT>(S, L, stage, last, dt, m, z0, i0, j0, ci, cj, col, reads_qn,
                                                         detect, qin, r_out, H0, Fq[0], Fc[0], d, Wup, zlo, lmax);
    }
    if (last) reduce_rate_block<NT>(z, stage == 0 ? 0 : rate_set(sw.steps + 1), lmax, L.sRed);
}

// Brick shapes: id, TX, TY, TZ, threads, form.  Shapes 4-9 give every
// face of a sweep its own thread (threads >= the largest face count of one
// axis), so each sweep is a single pass; 8 and 9 are persistent (form 1:
// resident workgroups that prefetch the next brick's halo into registers;
// 512 threads leave room for them).  Form 2 is the z-marching kernel on
// TX x TY column tiles with runs of TZ planes (three waves per SIMD); TZ = 0:
// one round of workgroups (as many as the GPU holds at once), each tile's
// height cut into balanced runs.
#define ROEAM_SHAPES3(X)      \
    X(0, 8, 8, 4, 256, 0)     \
    X(1, 8, 4, 4, 128, 0)     \
    X(2, 16, 8, 4, 512, 0)    \
    X(3, 16, 4, 4, 256, 0)    \
    X(4, 8, 8, 4, 320, 0)     \
    X(5, 8, 4, 4, 192, 0)     \
    X(6, 16, 8, 4, 640, 0)    \
    X(7, 8, 8, 8, 576, 0)     \
    X(8, 16, 8, 4, 512, 1)    \
    X(9, 8, 8, 8, 512, 1)     \
    X(10, 16, 15, 4, 256, 2)  \
    X(11, 16, 15, 8, 256, 2)  \
    X(12, 16, 15, 16, 256, 2) \
    X(13, 16, 15, 0, 256, 2)

struct BrickShape {
    int tx, ty, tz, nt, persistent;  // form: 0 brick, 1 persistent brick, 2 z-marching
};
#define ROEAM_SHAPE3_ENTRY(ID, TX, TY, TZ, NT, PE) {TX, TY, TZ, NT, PE},
static const BrickShape kShapes3[] = {ROEAM_SHAPES3(ROEAM_SHAPE3_ENTRY)};
#undef ROEAM_SHAPE3_ENTRY
constexpr int kNumShapes3 = sizeof(kShapes3) / sizeof(kShapes3[0]);

// Workgroups of a persistent kernel: as many as the GPU holds at once (CUs
// times workgroups per CU from the occupancy query, cached per kernel and
// device), a multiple of 8, and no more than the bricks need.
template <auto Kernel>
static int persistent_blocks(int nt, long long nb)
{
    constexpr int kMaxDevices = 64;
    static std::atomic<int> cached[kMaxDevices];  // 0: not queried yet (threads may race to fill it alike)
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    int held = cached[dev].load(std::memory_order_relaxed);
    if (held == 0) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(Kernel), nt, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        held = cus * per_cu;
        cached[dev].store(held, std::memory_order_relaxed);
    }
    const long long want = nb < held ? nb : held;
    return (int)(((want + 7) >> 3) << 3);
}

// LDS of a shape's kernel.
constexpr long long shape3_lds_bytes(int order, int nsc, int tx, int ty, int tz, int nt, int form)
{
    return form == 2 ? zstage3_lds_bytes(order, nsc, tx, ty, nt)
                     : stage3_lds_bytes(order, nsc, tx, ty, tz, nt, stage3_double_buffer(order, nsc, tx, ty, tz, nt));
}

template <int ORDER, int PREC, int NSC, int TX, int TY, int TZ, int NT, int PE>
static hipError_t launch3_one(const DevSolve3 *dS, const DevSolve3 &S, long long nb, int stage, int p, int last,
                              double *r_out, hipStream_t st)
{
    if constexpr (shape3_lds_bytes(ORDER, NSC, TX, TY, TZ, NT, PE) > kLdsBytes3) {
        return hipErrorInvalidValue;
    } else if constexpr (PE == 2) {
        // one workgroup per run of TZ planes of a column tile; TZ = 0: the same
        // number of runs for every tile, as many as the GPU holds workgroups
        // at once allows (at least one, and runs no shorter than four planes
        // where the grid allows)
        int zc = TZ;
        long long runs = nb;
        if constexpr (TZ == 0) {
            const long long nt = (long long)((S.nx + TX - 1) / TX) * ((S.ny + TY - 1) / TY);
            const long long per_tile_max = S.nz >= 8 ? S.nz / 4 : 1;
            const long long slots = persistent_blocks<k_stage3z<ORDER, PREC, NSC, TX, TY, NT>>(NT, nt * per_tile_max);
            long long per_tile = slots / nt;
            per_tile = per_tile < 1 ? 1 : (per_tile > per_tile_max ? per_tile_max : per_tile);
            runs = nt * per_tile;
            zc = (int)-runs;
        }
        const int blocks = (int)(((runs + 7) >> 3) << 3);
        hipLaunchKernelGGL((k_stage3z<ORDER, PREC, NSC, TX, TY, NT>), dim3(blocks), dim3(NT), 0, st, dS, stage, p,
                           last, r_out, zc);
        return hipSuccess;
    } else if constexpr (PE) {
        auto kernel = k_stage3p<ORDER, PREC, NSC, TX, TY, TZ, NT>;
        const int blocks = persistent_blocks<k_stage3p<ORDER, PREC, NSC, TX, TY, TZ, NT>>(NT, nb);
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(NT), 0, st, dS, stage, p, last, r_out);
        return hipSuccess;
    } else {
        const int blocks = (int)(((nb + 7) >> 3) << 3);
        hipLaunchKernelGGL((k_stage3<ORDER, PREC, NSC, TX, TY, TZ, NT>), dim3(blocks), dim3(NT), 0, st, dS, stage, p, last,
                           r_out);
        return hipSuccess;
    }
}

template <int ORDER, int PREC, int NSC>
static hipError_t launch3_shape(const DevSolve3 *dS, const DevSolve3 &S, int shape, int stage, int p, int last,
                                double *r_out, hipStream_t st)
{
    const BrickShape &sh = kShapes3[shape];
    const long long nb = sh.tz > 0 ? (long long)((S.nx + sh.tx - 1) / sh.tx) * ((S.ny + sh.ty - 1) / sh.ty) *
                                         ((S.nz + sh.tz - 1) / sh.tz)
                                   : 0;
#define ROEAM_SHAPE3_CASE(ID, TX, TY, TZ, NT, PE) \
    case ID: return launch3_one<ORDER, PREC, NSC, TX, TY, TZ, NT, PE>(dS, S, nb, stage, p, last, r_out, st);
    switch (shape) { ROEAM_SHAPES3(ROEAM_SHAPE3_CASE) }
#undef ROEAM_SHAPE3_CASE
    return hipErrorInvalidValue;
}

// All orders and precisions of one scalar count.
template <int NSC>
static hipError_t launch3_nsc(const DevSolve3 *dS, const DevSolve3 &S, int shape, int stage, int p, int last,
                              double *r_out, hipStream_t st)
{
    if (S.order == 1) {
        return S.precision == 0 ? launch3_shape<1, 0, NSC>(dS, S, shape, stage, p, last, r_out, st)
                                : launch3_shape<1, 1, NSC>(dS, S, shape, stage, p, last, r_out, st);
    }
    return S.precision == 0 ? launch3_shape<2, 0, NSC>(dS, S, shape, stage, p, last, r_out, st)
                            : launch3_shape<2, 1, NSC>(dS, S, shape, stage, p, last, r_out, st);
}

} // namespace roeam

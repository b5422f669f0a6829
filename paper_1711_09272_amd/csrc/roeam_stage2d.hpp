// roeam_stage2d.hpp -- the 2-D stage kernel as templates: tile + halo load,
// detector ratios, face sweeps, residual, stage update and reductions, for a
// tile shape and a number NSC of transported scalars (the rho k rows of
// Eq. 85).  roeam_kernels.hip instantiates it without scalars (single-grid
// and batched launches), roeam_kernels_sc.hip with one or two.
#pragma once

#include <type_traits>

#include "roeam_device.hpp"
#include "roeam_internal.hpp"
#include "roeam_stage.hpp"

namespace roeam {

// Tile shapes: id, TX, TY, threads, split.  Non-split shapes sweep the faces
// in one or two passes per direction; split shapes give every face a thread.
// 6 and 7 cover each face direction in one pass of 256 threads; 8 gives every
// face of a 16x7 tile a thread (fewer halo cells per tile cell than 8x7 at the
// same one-face-per-thread latency).
#define ROEAM_SHAPES(X)               \
    X(0, 32, 15, 256, false)          \
    X(1, 16, 15, 128, false)          \
    X(2, 8, 7, 64, false)             \
    X(3, 8, 7, 128, true)             \
    X(4, 16, 15, 512, true)           \
    X(5, 32, 7, 512, true)            \
    X(6, 16, 15, 256, false)          \
    X(7, 32, 7, 256, false)           \
    X(8, 16, 7, 256, true)

// Number of the i-faces of a tile: face f < TX TY is the west face of tile
// cell (f mod TX, f div TX); the TY faces past that are the east faces of the
// last column, f = TX TY + row.  TX is a power of two, so the map is shifts.
template <int TX, int TY>
__device__ __forceinline__ void xface_of(int f, int &fi, int &fj)
{
    if (f < TX * TY) {
        fi = f & (TX - 1);
        fj = f / TX;
    } else {
        fi = TX;
        fj = f - TX * TY;
    }
}

// MUSCL-minmod (or first-order) face states of the NC components (rho, u, v,
// p and the scalars k_m) from the four cells m2, m1 | p0, p1 along the normal.
template <int ORDER, int NC>
__device__ __forceinline__ void reconstruct(const double *m2, const double *m1, const double *p0, const double *p1,
                                            double *WL, double *WR)
{
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        if (ORDER == 1) {
            WL[k] = m1[k];
            WR[k] = p0[k];
        } else {
            const double d1 = p0[k] - m1[k];
            WL[k] = m1[k] + 0.5 * minmod(m1[k] - m2[k], d1);
            WR[k] = p0[k] - 0.5 * minmod(d1, p1[k] - p0[k]);
        }
    }
}

// One i-face (between tile cells (fi-1, fj) and (fi, fj)) or j-face (between
// (fi, fj-1) and (fi, fj)) of a tile: MUSCL face states from the LDS
// primitives, the detector minimum over the face and its four transverse
// neighbours, and the flux times the face length.  On uniform grids the flux
// is taken in the frame of the face: a j-face swaps u and v on the way in and
// the two momentum rows on the way out (a reflection, under which Eq. 85 is
// invariant), so both directions run the n = (1, 0) form of the flux.
template <int ORDER, int PREC, int METRIC, int TX, int TY, bool XDIR, int NSC>
__device__ __forceinline__ void tile_face(const DevSolve &S,
                                          const double (&sW)[4 + NSC][TY + 2 * ORDER][TX + 2 * ORDER],
                                          const double (&sPx)[TY + 2][TX + 1],
                                          const double (&sPy)[TY + 1][TX + 2], int fi, int fj, int gi, int gj, double *F)
{
    using R = typename std::conditional<PREC == 0, double, float>::type;
    constexpr int HL = ORDER, NC = 4 + NSC;
    constexpr bool AXIS = METRIC == 0;
    double m2[NC], m1[NC], p0[NC], p1[NC], WL[NC], WR[NC];
    const int ly = fj + HL, lx = fi + HL;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        // frame component k reads state component c
        const int c = (AXIS && !XDIR && (k == 1 || k == 2)) ? 3 - k : k;
        if (XDIR) {
            m1[k] = sW[c][ly][lx - 1];
            p0[k] = sW[c][ly][lx];
            if (ORDER == 2) {
                m2[k] = sW[c][ly][lx - 2];
                p1[k] = sW[c][ly][lx + 1];
            }
        } else {
            m1[k] = sW[c][ly - 1][lx];
            p0[k] = sW[c][ly][lx];
            if (ORDER == 2) {
                m2[k] = sW[c][ly - 2][lx];
                p1[k] = sW[c][ly + 1][lx];
            }
        }
    }
    reconstruct<ORDER, NC>(m2, m1, p0, p1, WL, WR);
    double s1 = 1.0;
    if (S.s1_mode == 0 && S.scheme == SCHEME_ROEAM) {
        double a;
        if (XDIR) {
            a = rmin(rmin(sPx[fj + 1][fi], sPy[fj][fi]), rmin(sPy[fj + 1][fi], rmin(sPy[fj][fi + 1], sPy[fj + 1][fi + 1])));
        } else {
            a = rmin(rmin(sPy[fj][fi + 1], sPx[fj][fi]), rmin(sPx[fj][fi + 1], rmin(sPx[fj + 1][fi], sPx[fj + 1][fi + 1])));
        }
        s1 = detector_s1<PREC>(a);
    }
    if (AXIS) {
        // flux per unit length: the face length (dy or dx) enters the
        // residual with 1 / Omega, once per cell instead of once per face row
        roeam_flux<R, NSC, true>(S, WL, WR, 1.0, 0.0, s1, F);
        if (!XDIR) {
            const double t = F[1];
            F[1] = F[2];
            F[2] = t;
        }
    } else {
        double sx, sy, nxv, nyv, len;
        if (XDIR) xface_vec<METRIC>(S, gi, gj, sx, sy);
        else yface_vec<METRIC>(S, gi, gj, sx, sy);
        unit_normal<METRIC>(S, sx, sy, nxv, nyv, len);
        roeam_flux<R, NSC>(S, WL, WR, nxv, nyv, s1, F);
#pragma unroll
        for (int k = 0; k < NC; ++k) F[k] *= len;
    }
}

// Positive, finite and nonzero (IEEE class +normal or +subnormal).
__device__ __forceinline__ bool pos_finite(double x) { return __builtin_amdgcn_class(x, 0x180); }

// The tile body.  stage: a stage code (above; 0 writes the residual to r_out).
// p: step parity.  last: this stage ends the step (reduce the rate of the new
// state into parity p^1); for stage 0 the rate of the input is reduced into
// parity 0.
// SPLIT = false: NT threads sweep the i-faces, then the j-faces through one
// LDS buffer (about two faces per thread).  SPLIT = true: one face per thread,
// i-faces on the first ceil(NFX/64) waves and j-faces on the rest, in one pass.
template <int ORDER, int PREC, int METRIC, int TX, int TY, int NT, bool SPLIT, int NSC>
__device__ __forceinline__ void stage_tile(const DevSolve &S, int tx, int ty, int stage, int p, int last,
                                           int first_block, double *__restrict__ r_out)
{
    static_assert((TX & (TX - 1)) == 0, "tile width must be a power of two");
    constexpr int HL = ORDER, NC = 4 + NSC;  // components: rho, u, v, p and the scalars
    constexpr int LX = TX + 2 * HL, LY = TY + 2 * HL;
    constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1);
    constexpr int NFXR = (NFX + 63) / 64 * 64;  // i-face threads in SPLIT mode
    static_assert(!SPLIT || NFXR + NFY <= NT, "split shape must give every face a thread");
    constexpr int NFB = SPLIT ? NFX : (NFX > NFY ? NFX : NFY);
    constexpr int CPT = (TX * TY + NT - 1) / NT;  // cells per thread
    constexpr int NPX = (TY + 2) * (TX + 1), NPY = (TY + 1) * (TX + 2);
    __shared__ double sW[NC][LY][LX];
    __shared__ double sPx[TY + 2][TX + 1];
    __shared__ double sPy[TY + 1][TX + 2];
    // the face fluxes; before the first face sweep the same memory holds the
    // reciprocals of p and rho of the staged cells (detector ratios)
    constexpr int NFLUX = NC * NFB > 2 * LX * LY ? NC * NFB : 2 * LX * LY;
    __shared__ double sFbuf[NFLUX];
    __shared__ double sG[NC][SPLIT ? NFY : 1];
    __shared__ double sRed[NT / 64];
    double(&sF)[NC][NFB] = *reinterpret_cast<double(*)[NC][NFB]>(&sFbuf[0]);
    double *sIP = &sFbuf[0], *sIR = &sFbuf[LX * LY];  // 1/p, 1/rho per staged cell

    const int tid = threadIdx.x;
    const int bin = stage_in_buf(stage);
    const double *__restrict__ qin = bin == 0 ? S.q : (bin == 2 ? S.qb : S.qa);
    const bool reads_qn = stage_reads_qn(stage);  // Q^n at the own cells, besides the stencil input
    const int i0 = tx * TX, j0 = ty * TY;
    const int nx = S.nx, ny = S.ny;
    const bool detector = S.s1_mode == 0 && S.scheme == SCHEME_ROEAM;

    // The step-state words first, then the own cells' stage input (and Q^n for
    // stages 2-3), whose latency is hidden behind the face work; cells outside
    // the grid load cell (0, 0) and are never stored.
    Slot &z = *S.slot;
    const StepWords sw = stage > 0 ? load_step_words(z, p, stage) : StepWords{};
    double Qs[CPT][NC], Q0[CPT][NC];
    long long cidx[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = tid + m * NT;
        const int cj = c / TX, ci = c & (TX - 1);
        const bool ok = c < TX * TY && i0 + ci < nx && j0 + cj < ny;
        cidx[m] = ok ? (long long)(j0 + cj) * S.pitch + (i0 + ci) : 0;
        if (stage > 0) {
#pragma unroll
            for (int k = 0; k < NC; ++k) Qs[m][k] = gptr(qin)[k * S.plane + cidx[m]];
        }
        if (reads_qn) {
#pragma unroll
            for (int k = 0; k < NC; ++k) Q0[m][k] = gptr(S.q)[k * S.plane + cidx[m]];
        }
    }

    double dt = 0.0;
    if (stage > 0 && !begin_stage(z, sw, p, stage, last, first_block, dt)) return;
    // time of this stage's input state (moving boundary sides): the step start
    // plus the stage abscissa, 0, 1, 1/2 (SSP-RK3) or 0, 1/4, 1/3, 1/2 (four-stage)
    const BoundaryClock clk{stage == 0 ? nullptr : &z, p, stage_abscissa(stage) * dt, S.t_res};

    // 1. tile + halo -> primitives in LDS (and 1/p, 1/rho for the detector;
    // 1/p with one Newton step, as for the other dissipation coefficients).
    // Interior tiles issue every load of the thread first (lanes past the
    // staged box load the box's first cell, which is on the grid) and convert
    // afterwards, so that all loads are in flight together; tiles at the
    // boundary map each cell in turn.
    const bool interior = (i0 - HL >= 0) && (i0 + TX + HL <= nx) && (j0 - HL >= 0) && (j0 + TY + HL <= ny);
    constexpr int NLOAD = (LX * LY + NT - 1) / NT;
    if (interior) {
        double Qh[NLOAD][NC];
#pragma unroll
        for (int it = 0; it < NLOAD; ++it) {
            const int e = tid + it * NT < LX * LY ? tid + it * NT : 0;
            const int ly = e / LX, lx = e - ly * LX;
            const long long idx = (long long)(j0 - HL + ly) * S.pitch + (i0 - HL + lx);
#pragma unroll
            for (int k = 0; k < NC; ++k) Qh[it][k] = gptr(qin)[k * S.plane + idx];
        }
#pragma unroll
        for (int it = 0; it < NLOAD; ++it) {
            const int e = tid + it * NT;
            if (e >= LX * LY) break;
            const int ly = e / LX, lx = e - ly * LX;
            double W[NC];
            const double ir = to_prim(S.gm1, Qh[it][0], Qh[it][1], Qh[it][2], Qh[it][3], W);
#pragma unroll
            for (int m = 0; m < NSC; ++m) W[4 + m] = Qh[it][4 + m] * ir;
#pragma unroll
            for (int k = 0; k < NC; ++k) sW[k][ly][lx] = W[k];
            if (detector) {
                sIR[e] = ir;
                sIP[e] = rcp_nr1(W[3]);
            }
        }
    } else {
#pragma unroll
        for (int it = 0; it < NLOAD; ++it) {
            const int e = tid + it * NT;
            if (e >= LX * LY) break;
            const int ly = e / LX, lx = e - ly * LX;
            // cells past the ghost layers of a ragged tile feed no valid face
            const int gi = min(i0 - HL + lx, nx + 1), gj = min(j0 - HL + ly, ny + 1);
            double W[NC];
            fetch_prim<METRIC, NSC>(S, qin, gi, gj, W, clk);
#pragma unroll
            for (int k = 0; k < NC; ++k) sW[k][ly][lx] = W[k];
            if (detector) {
                sIR[e] = rcp_nr(W[0]);
                sIP[e] = rcp_nr1(W[3]);
            }
        }
    }
    __syncthreads();

    // 2. detector ratios, Eq. (97), from cell-centre values: the smaller of the
    // pressure and density ratios, each taken below one as the smaller of
    // a (1 / b) and b (1 / a), from the reciprocals staged with the cells
    if (detector) {
        // one sweep over the i-face ratios then the j-face ratios, so that
        // the threads stay busy across the two arrays
        for (int e = tid; e < NPX + NPY; e += NT) {
            int a, b;  // staged cell numbers of the two cells
            double *dst;
            if (e < NPX) {
                const int r = e / (TX + 1), fi = e - r * (TX + 1);
                a = (r - 1 + HL) * LX + fi - 1 + HL;
                b = a + 1;
                dst = &sPx[r][fi];
            } else {
                const int f = e - NPX;
                const int fr = f / (TX + 2), cc = f - fr * (TX + 2);
                a = (fr - 1 + HL) * LX + cc - 1 + HL;
                b = a + LX;
                dst = &sPy[fr][cc];
            }
            const double *p3 = &sW[3][0][0], *p0 = &sW[0][0][0];
            *dst = rmin(rmin(p3[a] * sIP[b], p3[b] * sIP[a]), rmin(p0[a] * sIR[b], p0[b] * sIR[a]));
        }
        __syncthreads();
    }

    // 3. every face of the tile exactly once
    double dfx[CPT][NC];
    // east/west i-face fluxes of an own cell (face numbering of xface_of)
    auto xflux_diff = [&](int c, int k) {
        const int cj = c / TX, ci = c & (TX - 1);
        const int w = c, e = ci + 1 < TX ? c + 1 : TX * TY + cj;
        return sF[k][e] - sF[k][w];
    };
    if (SPLIT) {
        if (tid < NFXR) {
            const int f = tid;
            int fi, fj;
            xface_of<TX, TY>(f, fi, fj);
            if (f < NFX && i0 + fi <= nx && j0 + fj < ny) {
                double F[NC];
                tile_face<ORDER, PREC, METRIC, TX, TY, true, NSC>(S, sW, sPx, sPy, fi, fj, i0 + fi, j0 + fj, F);
#pragma unroll
                for (int k = 0; k < NC; ++k) sF[k][f] = F[k];
            }
        } else {
            const int f = tid - NFXR;
            const int fr = f / TX, fi = f & (TX - 1);
            if (f < NFY && i0 + fi < nx && j0 + fr <= ny) {
                double F[NC];
                tile_face<ORDER, PREC, METRIC, TX, TY, false, NSC>(S, sW, sPx, sPy, fi, fr, i0 + fi, j0 + fr, F);
#pragma unroll
                for (int k = 0; k < NC; ++k) sG[k][f] = F[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            const int c = tid + m * NT;
#pragma unroll
            for (int k = 0; k < NC; ++k) dfx[m][k] = (c < TX * TY) ? xflux_diff(c, k) : 0.0;
        }
    } else {
        for (int f = tid; f < NFX; f += NT) {
            int fi, fj;
            xface_of<TX, TY>(f, fi, fj);
            if (i0 + fi > nx || j0 + fj >= ny) continue;
            double F[NC];
            tile_face<ORDER, PREC, METRIC, TX, TY, true, NSC>(S, sW, sPx, sPy, fi, fj, i0 + fi, j0 + fj, F);
#pragma unroll
            for (int k = 0; k < NC; ++k) sF[k][f] = F[k];
        }
        __syncthreads();
        // i-direction part of the residual, kept in registers
#pragma unroll
        for (int m = 0; m < CPT; ++m) {
            const int c = tid + m * NT;
#pragma unroll
            for (int k = 0; k < NC; ++k) dfx[m][k] = (c < TX * TY) ? xflux_diff(c, k) : 0.0;
        }
        __syncthreads();
        // j-faces through the same LDS buffer
        for (int f = tid; f < NFY; f += NT) {
            const int fr = f / TX, fi = f & (TX - 1);
            if (i0 + fi >= nx || j0 + fr > ny) continue;
            double F[NC];
            tile_face<ORDER, PREC, METRIC, TX, TY, false, NSC>(S, sW, sPx, sPy, fi, fr, i0 + fi, j0 + fr, F);
#pragma unroll
            for (int k = 0; k < NC; ++k) sF[k][f] = F[k];
        }
        __syncthreads();
    }
    const double(&sJ)[NC][SPLIT ? NFY : NFB] = *reinterpret_cast<const double(*)[NC][SPLIT ? NFY : NFB]>(SPLIT ? &sG[0][0] : &sF[0][0]);

    // 4. conservative residual R = -((F_e - F_w) + (G_n - G_s)) / Omega and the stage update
    // (uniform grids: the faces hold fluxes per unit length, so R = -((F_e - F_w) dy / Omega
    // + (G_n - G_s) dx / Omega))
    double lmax = 0.0;
    const double cxi = S.dy * S.inv_area, cyi = S.dx * S.inv_area;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = tid + m * NT;
        const int cj = c / TX, ci = c & (TX - 1);
        const int gi = i0 + ci, gj = j0 + cj;
        if (c >= TX * TY || gi >= nx || gj >= ny) continue;
        const double iom = METRIC == 0 ? S.inv_area : rcp_nr(cell_area<METRIC>(S, gi, gj));
        double Rv[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const double dj = sJ[k][(cj + 1) * TX + ci] - sJ[k][cj * TX + ci];
            Rv[k] = METRIC == 0 ? -fma(dfx[m][k], cxi, dj * cyi) : -(dfx[m][k] + dj) * iom;
        }
        const long long idx = cidx[m];
        if (stage == 0) {
#pragma unroll
            for (int k = 0; k < NC; ++k) gptr(r_out)[k * S.plane + idx] = Rv[k];
            if (last) {
                double W[4] = {sW[0][cj + HL][ci + HL], sW[1][cj + HL][ci + HL], sW[2][cj + HL][ci + HL],
                               sW[3][cj + HL][ci + HL]};
                lmax = rmax(lmax, cell_rate<METRIC>(S, W, rcp_nr(W[0]), gi, gj));
            }
            continue;
        }
        double Qn[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            switch (stage) {
            case 1:
            case 8: Qn[k] = Qs[m][k] + dt * Rv[k]; break;
            case 2: Qn[k] = 0.75 * Q0[m][k] + 0.25 * (Qs[m][k] + dt * Rv[k]); break;
            case 3: Qn[k] = (1.0 / 3.0) * Q0[m][k] + (2.0 / 3.0) * (Qs[m][k] + dt * Rv[k]); break;
            // four-stage scheme: Q^(k) = Q^n + alpha_k dt R(Q^(k-1)), alpha = 1/4, 1/3, 1/2, 1
            case 4: Qn[k] = Qs[m][k] + (0.25 * dt) * Rv[k]; break;
            case 5: Qn[k] = Q0[m][k] + ((1.0 / 3.0) * dt) * Rv[k]; break;
            case 6: Qn[k] = Q0[m][k] + (0.5 * dt) * Rv[k]; break;
            default: Qn[k] = Q0[m][k] + dt * Rv[k]; break;
            }
        }
        const int bout = stage_out_buf(stage);
        double *__restrict__ qo = bout == 0 ? S.q : (bout == 2 ? S.qb : S.qa);
#pragma unroll
        for (int k = 0; k < NC; ++k) gptr(qo)[k * S.plane + idx] = Qn[k];
        if (last) {
            double W[4];
            const double ir = to_prim(S.gm1, Qn[0], Qn[1], Qn[2], Qn[3], W);
            // rho and p positive and finite (a non-finite u or v makes p so)
            if (!(pos_finite(W[0]) && pos_finite(W[3]))) atomicOr(&z.nonphys, 1);
            else lmax = rmax(lmax, cell_rate<METRIC>(S, W, ir, gi, gj));
        } else {
            // p > 0 for rho > 0 is 2 rho (rho E) - |rho V|^2 > 0: no division needed
            const double pr = fma(2.0 * Qn[0], Qn[3], -fma(Qn[1], Qn[1], Qn[2] * Qn[2]));
            if (!(pos_finite(Qn[0]) && pos_finite(pr))) atomicOr(&z.nonphys, 1);
        }
    }
    if (last) {
        reduce_rate_block<NT>(z, stage == 0 ? 0 : rate_set(sw.steps + 1), lmax, sRed);
    }
}

// Minimum waves per SIMD asked of the register allocator, for the uniform-grid
// kernels of the one-pass 256-thread shapes without scalars: FP64 five (96
// VGPRs; measured faster than four, 1-3% at 512^2 and 2048^2; six spills forty
// dwords and loses 8-40%); FP32 coefficients six where the tile's LDS (25 KB
// for 240 cells or fewer) lets six workgroups share a CU: 80 VGPRs, six dwords
// spilled, 3.5% faster than five waves on the 256-grid batch and at 2048^2.
// Tiles of more cells (32x15: 47 KB of LDS) fit three workgroups per CU, so
// three is asked there (the persistent batched form of those takes what the
// allocator chooses: two waves without spills). The persistent batched form
// of the smaller tiles keeps five (it spills more at six); the node-grid
// kernels and those with scalars keep the default.
constexpr int stage_min_waves(int prec, int metric, int tx, int ty, int nt, bool split, int nsc,
                              bool persistent = false)
{
    if (metric != 0 || nt != 256 || split || nsc != 0) return 1;
    if (tx * ty > 240) return persistent ? 1 : 3;
    return (prec == 1 && !persistent) ? 6 : 5;
}

template <int ORDER, int PREC, int METRIC, int TX, int TY, int NT, bool SPLIT, int NSC>
__global__ __launch_bounds__(NT, stage_min_waves(PREC, METRIC, TX, TY, NT, SPLIT, NSC)) void k_stage_single(const DevSolve *__restrict__ Sp, int stage, int p, int last,
                                                     double *r_out)
{
    const DevSolve &S = *Sp;
    const int txs = (S.nx + TX - 1) / TX, tys = (S.ny + TY - 1) / TY;
    const int nt = txs * tys;
    const int t = xcd_tile(blockIdx.x, nt);
    if (t >= nt) return;
    stage_tile<ORDER, PREC, METRIC, TX, TY, NT, SPLIT, NSC>(S, t % txs, t / txs, stage, p, last, t == 0, r_out);
}

// Batched launch over a group's work list: `count` (device memory) tiles of
// `tiles`.  The launch is sized to the list's capacity so that one captured
// graph serves any count up to it; the XCD-aware map (xcd_tile) spreads the
// first ceil(count / 8) * 8 workgroups over the tiles and the rest exit.
template <int ORDER, int PREC, int METRIC, int TX, int TY, int NT, bool SPLIT, int NSC>
__global__ __launch_bounds__(NT, stage_min_waves(PREC, METRIC, TX, TY, NT, SPLIT, NSC)) void k_stage_batch(const DevSolve *__restrict__ solves,
                                                    const TileEntry *__restrict__ tiles, const int *__restrict__ count,
                                                    int stage, int p, int last)
{
    const int ntiles = *count;
    const int b = blockIdx.x, chunk = (ntiles + 7) >> 3;
    if ((b >> 3) >= chunk) return;
    const int t = xcd_tile(b, ntiles);
    if (t >= ntiles) return;
    const TileEntry te = tiles[t];
    stage_tile<ORDER, PREC, METRIC, TX, TY, NT, SPLIT, NSC>(solves[te.solve], te.tx, te.ty, stage, p, last,
                                                            te.tx == 0 && te.ty == 0, nullptr);
}

// Persistent form: a fixed number of resident workgroups (a multiple of 8)
// take the tiles in turn; the workgroups of XCD x (ids = x mod 8) walk the
// band [x c, (x + 1) c), c = ceil(count / 8), so that neighbouring tiles share
// that XCD's L2.
template <int ORDER, int PREC, int METRIC, int TX, int TY, int NT, bool SPLIT, int NSC>
__global__ __launch_bounds__(NT, stage_min_waves(PREC, METRIC, TX, TY, NT, SPLIT, NSC, true)) void k_stage_batch_p(const DevSolve *__restrict__ solves,
                                                    const TileEntry *__restrict__ tiles, const int *__restrict__ count,
                                                    int stage, int p, int last)
{
    const int ntiles = *count;
    const int chunk = (ntiles + 7) >> 3;
    const int x = blockIdx.x & 7, nw = gridDim.x >> 3;
    for (int k = blockIdx.x >> 3; k < chunk; k += nw) {
        const int t = x * chunk + k;
        if (t >= ntiles) break;
        __syncthreads();  // the previous tile's LDS reads are done
        const TileEntry te = tiles[t];
        stage_tile<ORDER, PREC, METRIC, TX, TY, NT, SPLIT, NSC>(solves[te.solve], te.tx, te.ty, stage, p, last,
                                                                te.tx == 0 && te.ty == 0, nullptr);
    }
}

// Batched launch of the stage kernel (solves of one group, all with NSC
// scalars) on tile shape `shape`: `blocks` workgroups (a multiple of 8) of the
// windowed or the persistent form.
#define ROEAM_SHAPE_CASE_BATCH(ID, TX, TY, NT, SPLIT)                                                               \
    case ID:                                                                                                        \
        if (persistent)                                                                                             \
            hipLaunchKernelGGL((k_stage_batch_p<ORDER, PREC, METRIC, TX, TY, NT, SPLIT, NSC>), dim3(blocks), dim3(NT), \
                               0, st, solves, tiles, count, stage, p, last);                                        \
        else                                                                                                        \
            hipLaunchKernelGGL((k_stage_batch<ORDER, PREC, METRIC, TX, TY, NT, SPLIT, NSC>), dim3(blocks), dim3(NT), \
                               0, st, solves, tiles, count, stage, p, last);                                        \
        break;

template <int ORDER, int PREC, int METRIC, int NSC>
inline void launch_batch_shape(const DevSolve *solves, const TileEntry *tiles, const int *count, int blocks,
                               bool persistent, int shape, int stage, int p, int last, hipStream_t st)
{
    switch (shape) { ROEAM_SHAPES(ROEAM_SHAPE_CASE_BATCH) }
}

template <int NSC>
inline void launch_batch_nsc(const DevSolve *solves, const TileEntry *tiles, const int *count, int blocks,
                             bool persistent, int order, int precision, int metric, int shape, int stage, int p,
                             int last, hipStream_t st)
{
#define ROEAM_BATCH_METRIC(O, P)                                                                                  \
    if (metric == 0) launch_batch_shape<O, P, 0, NSC>(solves, tiles, count, blocks, persistent, shape, stage, p, last, st); \
    else launch_batch_shape<O, P, 1, NSC>(solves, tiles, count, blocks, persistent, shape, stage, p, last, st);
    if (order == 1) {
        if (precision == 0) { ROEAM_BATCH_METRIC(1, 0) } else { ROEAM_BATCH_METRIC(1, 1) }
    } else {
        if (precision == 0) { ROEAM_BATCH_METRIC(2, 0) } else { ROEAM_BATCH_METRIC(2, 1) }
    }
#undef ROEAM_BATCH_METRIC
}

// Resident workgroups of the persistent batched kernel per CU for a shape
// (the occupancy the compiled kernel allows).
template <int NSC>
inline int batch_blocks_per_cu_nsc(int order, int precision, int metric, int shape)
{
    int n = 0;
#define ROEAM_OCC_CASE(ID, TX, TY, NT, SPLIT)                                                                     \
    case ID:                                                                                                      \
        if (order == 1 && precision == 0 && metric == 0)                                                          \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stage_batch_p<1, 0, 0, TX, TY, NT, SPLIT, NSC>, NT, 0); \
        else if (order == 1 && precision == 0)                                                                    \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stage_batch_p<1, 0, 1, TX, TY, NT, SPLIT, NSC>, NT, 0); \
        else if (order == 1 && metric == 0)                                                                       \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stage_batch_p<1, 1, 0, TX, TY, NT, SPLIT, NSC>, NT, 0); \
        else if (order == 1)                                                                                      \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stage_batch_p<1, 1, 1, TX, TY, NT, SPLIT, NSC>, NT, 0); \
        else if (precision == 0 && metric == 0)                                                                   \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stage_batch_p<2, 0, 0, TX, TY, NT, SPLIT, NSC>, NT, 0); \
        else if (precision == 0)                                                                                  \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stage_batch_p<2, 0, 1, TX, TY, NT, SPLIT, NSC>, NT, 0); \
        else if (metric == 0)                                                                                     \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stage_batch_p<2, 1, 0, TX, TY, NT, SPLIT, NSC>, NT, 0); \
        else                                                                                                      \
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stage_batch_p<2, 1, 1, TX, TY, NT, SPLIT, NSC>, NT, 0); \
        break;
    switch (shape) { ROEAM_SHAPES(ROEAM_OCC_CASE) }
#undef ROEAM_OCC_CASE
    return n;
}

// Single-grid launch of the stage kernel with NSC scalars on tile shape `shape`.
#define ROEAM_SHAPE_CASE_SC(ID, TX, TY, NT, SPLIT)                                                             \
    case ID: hipLaunchKernelGGL((k_stage_single<ORDER, PREC, METRIC, TX, TY, NT, SPLIT, NSC>), dim3(blocks), dim3(NT), \
                                0, st, dS, stage, p, last, r_out); break;

template <int ORDER, int PREC, int METRIC, int NSC>
inline void launch_single_shape(const DevSolve *dS, const DevSolve &S, int shape, int stage, int p, int last,
                                double *r_out, hipStream_t st)
{
    int tx = 0, ty = 0;
    tile_shape(shape, &tx, &ty);
    const int nt = ((S.nx + tx - 1) / tx) * ((S.ny + ty - 1) / ty);
    const int blocks = ((nt + 7) >> 3) << 3;
    switch (shape) { ROEAM_SHAPES(ROEAM_SHAPE_CASE_SC) }
}

template <int NSC>
inline void launch_single_nsc(const DevSolve *dS, const DevSolve &S, int shape, int stage, int p, int last,
                              double *r_out, hipStream_t st)
{
#define ROEAM_SC_METRIC(O, P)                                                                          \
    if (S.metric == 0) launch_single_shape<O, P, 0, NSC>(dS, S, shape, stage, p, last, r_out, st);     \
    else launch_single_shape<O, P, 1, NSC>(dS, S, shape, stage, p, last, r_out, st);
    if (S.order == 1) {
        if (S.precision == 0) { ROEAM_SC_METRIC(1, 0) } else { ROEAM_SC_METRIC(1, 1) }
    } else {
        if (S.precision == 0) { ROEAM_SC_METRIC(2, 0) } else { ROEAM_SC_METRIC(2, 1) }
    }
#undef ROEAM_SC_METRIC
}

} // namespace roeam

// roeam_kernels3d.hip -- gfx950 stage kernel of the 3-D Roe-AM step on uniform
// Cartesian grids.
//
// A workgroup owns a brick of TX x TY x TZ cells.  It stages the brick and its
// halo (two layers for MUSCL, one for piecewise-constant states) as primitives
// in LDS, builds the detector ratio of Eq. (97) of every face within one layer
// of the brick, then sweeps the x-, y- and z-faces in turn through one LDS flux
// buffer, each face evaluated exactly once (Eq. 85, nine-face detector of
// Eq. 96), accumulates the conservative residual of its cells in registers and
// applies the stage update, the positivity check and the explicit-rate
// reduction exactly as the 2-D stage kernel does (same stage codes, same step
// state).  One kernel per Runge-Kutta stage.
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
    // LDS offset of brick cell (i, j, l), -HL <= i < TX + HL etc.
    static __device__ __forceinline__ int cell(int i, int j, int l) { return ((l + HL) * LY + (j + HL)) * LX + i + HL; }
    // ratio of the x-face at fi (0..TX) in row (j, l), j, l in -1..TY / -1..TZ
    static __device__ __forceinline__ int px(int fi, int j, int l) { return ((l + 1) * (TY + 2) + j + 1) * (TX + 1) + fi; }
    static __device__ __forceinline__ int py(int i, int fj, int l) { return NPX + ((l + 1) * (TY + 1) + fj) * (TX + 2) + i + 1; }
    static __device__ __forceinline__ int pz(int i, int j, int fl) { return NPX + NPY + (fl * (TY + 2) + j + 1) * (TX + 2) + i + 1; }
};

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

// Flux times area of the face of axis AXIS whose upper cell is brick cell
// (i, j, l), rows in global order (rho, rho u, rho v, rho w, rho E).
template <int ORDER, int PREC, int AXIS, class B>
__device__ __forceinline__ void brick_face(const DevSolve3 &S, const double *__restrict__ sW, const double *__restrict__ sP,
                                           int i, int j, int l, double F[5])
{
    using R = typename std::conditional<PREC == 0, double, float>::type;
    constexpr int PL = B::LX * B::LY * B::LZ;                     // one row of sW
    constexpr int ST = AXIS == 0 ? 1 : (AXIS == 1 ? B::LX : B::LX * B::LY);
    // face frame: rho, normal velocity, the two others in cyclic order, p
    constexpr int RN = 1 + AXIS, RT1 = 1 + (AXIS + 1) % 3, RT2 = 1 + (AXIS + 2) % 3;
    constexpr int rows[5] = {0, RN, RT1, RT2, 4};
    const int c = B::cell(i, j, l);
    double WL[5], WR[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double *r = sW + rows[k] * PL;
        const double m1 = r[c - ST], p0 = r[c];
        if (ORDER == 1) {
            WL[k] = m1;
            WR[k] = p0;
        } else {
            const double m2 = r[c - 2 * ST], p1 = r[c + ST];
            const double d1 = p0 - m1;
            WL[k] = m1 + 0.5 * minmod(m1 - m2, d1);
            WR[k] = p0 - 0.5 * minmod(d1, p1 - p0);
        }
    }
    double s1 = 1.0;
    if (S.s1_mode == 0 && S.scheme == SCHEME_ROEAM) s1 = pow8(fswitch(face_detector<AXIS, B>(sP, i, j, l)));
    double Ff[5];
    roeam_flux3<R>(S, WL, WR, s1, Ff);
    const double area = AXIS == 0 ? S.ax : (AXIS == 1 ? S.ay : S.az);
    F[0] = Ff[0] * area;
    F[RN] = Ff[1] * area;
    F[RT1] = Ff[2] * area;
    F[RT2] = Ff[3] * area;
    F[4] = Ff[4] * area;
}

// All faces of one axis into sF, then add their differences to the cells'
// residual sums d (in registers).  The caller separates the sweeps by barriers.
template <int ORDER, int PREC, int AXIS, int TX, int TY, int TZ, int NT, class B>
__device__ __forceinline__ void sweep_axis(const DevSolve3 &S, const double *__restrict__ sW, const double *__restrict__ sP,
                                           double (&sF)[5][B::NFB], int i0, int j0, int l0, double (*d)[5])
{
    constexpr int FX = TX + (AXIS == 0), FY = TY + (AXIS == 1), FZ = TZ + (AXIS == 2);
    constexpr int NF = FX * FY * FZ;
    constexpr int CPT = (TX * TY * TZ + NT - 1) / NT;
    for (int f = threadIdx.x; f < NF; f += NT) {
        const int i = f % FX, r = f / FX, j = r % FY, l = r / FY;
        // the face lies on the grid (a face at index n of its axis is the upper boundary)
        if (i0 + i > S.nx - (AXIS != 0) || j0 + j > S.ny - (AXIS != 1) || l0 + l > S.nz - (AXIS != 2)) continue;
        double F[5];
        brick_face<ORDER, PREC, AXIS, B>(S, sW, sP, i, j, l, F);
#pragma unroll
        for (int k = 0; k < 5; ++k) sF[k][f] = F[k];
    }
    __syncthreads();
    constexpr int up = AXIS == 0 ? 1 : (AXIS == 1 ? FX : FX * FY);
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = threadIdx.x + m * NT;
        if (c >= TX * TY * TZ) continue;
        const int ci = c % TX, r = c / TX, cj = r % TY, cl = r / TY;
        const int lo = (cl * FY + cj) * FX + ci;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const double df = sF[k][lo + up] - sF[k][lo];
            d[m][k] = AXIS == 0 ? df : d[m][k] + df;
        }
    }
    __syncthreads();
}

// Stage codes, buffers and step logic as in the 2-D stage kernel:
//   0 residual only; 1 forward Euler / first SSP-RK3 stage (q -> qa);
//   2 (qa -> qb, + Q^n), 3 (qb -> q, + Q^n); 4-7 the four-stage scheme
//   (q -> qa, qa -> qb, qb -> qa, qa -> q; + Q^n from the second on).
template <int ORDER, int PREC, int TX, int TY, int TZ, int NT>
__device__ __forceinline__ void stage_brick(const DevSolve3 &S, int bx, int by, int bz, int stage, int p, int last,
                                            int first_block, double *__restrict__ r_out)
{
    constexpr int HL = ORDER;
    using B = Brick<TX, TY, TZ, HL>;
    constexpr int NC = TX * TY * TZ;
    constexpr int CPT = (NC + NT - 1) / NT;
    constexpr int PL = B::LX * B::LY * B::LZ;
    __shared__ double sW[5 * PL];
    __shared__ double sP[B::NPX + B::NPY + B::NPZ];
    __shared__ double sF[5][B::NFB];
    __shared__ double sRed[NT / 64];

    const int tid = threadIdx.x;
    const double *__restrict__ qin = (stage <= 1 || stage == 4) ? S.q : ((stage == 3 || stage == 6) ? S.qb : S.qa);
    const bool reads_qn = stage >= 2 && stage != 4;
    const int i0 = bx * TX, j0 = by * TY, l0 = bz * TZ;
    const int nx = S.nx, ny = S.ny, nz = S.nz;

    // own cells' stage input (and Q^n) first, so their latency hides behind the face work
    double Qs[CPT][5], Q0[CPT][5];
    long long cidx[CPT];
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = tid + m * NT;
        const int ci = c % TX, r = c / TX, cj = r % TY, cl = r / TY;
        const bool ok = c < NC && i0 + ci < nx && j0 + cj < ny && l0 + cl < nz;
        cidx[m] = ok ? (long long)(l0 + cl) * S.slab + (long long)(j0 + cj) * S.pitch + (i0 + ci) : 0;
        if (stage > 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) Qs[m][k] = qin[k * S.plane + cidx[m]];
        }
        if (reads_qn) {
#pragma unroll
            for (int k = 0; k < 5; ++k) Q0[m][k] = S.q[k * S.plane + cidx[m]];
        }
    }

    Slot &z = *S.slot;
    double dt = 0.0;
    if (stage > 0 && !begin_stage(z, p, stage, last, first_block, dt)) return;

    // 1. brick + halo -> primitives in LDS
    const bool interior = i0 - HL >= 0 && i0 + TX + HL <= nx && j0 - HL >= 0 && j0 + TY + HL <= ny && l0 - HL >= 0 &&
                          l0 + TZ + HL <= nz;
    constexpr int NLOAD = (PL + NT - 1) / NT;
#pragma unroll
    for (int it = 0; it < NLOAD; ++it) {
        const int e = tid + it * NT;
        if (e >= PL) break;
        const int lx = e % B::LX, r = e / B::LX, ly = r % B::LY, lz = r / B::LY;
        int gi = i0 - HL + lx, gj = j0 - HL + ly, gl = l0 - HL + lz;
        double W[5];
        if (interior) {
            load_prim3(S, qin, gi, gj, gl, W);
        } else {
            // cells past the ghost layers of a ragged brick feed no face on the grid
            gi = gi > nx + 1 ? nx + 1 : gi;
            gj = gj > ny + 1 ? ny + 1 : gj;
            gl = gl > nz + 1 ? nz + 1 : gl;
            fetch_prim3(S, qin, gi, gj, gl, W);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) sW[k * PL + e] = W[k];
    }
    __syncthreads();

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

    // 3. x-, y- and z-faces, each exactly once; residual sums ((x) + (y)) + (z)
    double d[CPT][5];
    sweep_axis<ORDER, PREC, 0, TX, TY, TZ, NT, B>(S, sW, sP, sF, i0, j0, l0, d);
    sweep_axis<ORDER, PREC, 1, TX, TY, TZ, NT, B>(S, sW, sP, sF, i0, j0, l0, d);
    sweep_axis<ORDER, PREC, 2, TX, TY, TZ, NT, B>(S, sW, sP, sF, i0, j0, l0, d);

    // 4. R = -(sum of face fluxes times areas) / V and the stage update
    double lmax = 0.0;
#pragma unroll
    for (int m = 0; m < CPT; ++m) {
        const int c = tid + m * NT;
        const int ci = c % TX, r = c / TX, cj = r % TY, cl = r / TY;
        if (c >= NC || i0 + ci >= nx || j0 + cj >= ny || l0 + cl >= nz) continue;
        double Rv[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) Rv[k] = -d[m][k] * S.inv_vol;
        const long long idx = cidx[m];
        if (stage == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) r_out[k * S.plane + idx] = Rv[k];
            if (last) {
                const int o = B::cell(ci, cj, cl);
                double W[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) W[k] = sW[k * PL + o];
                lmax = rmax(lmax, cell_rate3(S, W, rcp_nr(W[0])));
            }
            continue;
        }
        double Qn[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            switch (stage) {
            case 1: Qn[k] = Qs[m][k] + dt * Rv[k]; break;
            case 2: Qn[k] = 0.75 * Q0[m][k] + 0.25 * (Qs[m][k] + dt * Rv[k]); break;
            case 3: Qn[k] = (1.0 / 3.0) * Q0[m][k] + (2.0 / 3.0) * (Qs[m][k] + dt * Rv[k]); break;
            case 4: Qn[k] = Qs[m][k] + (0.25 * dt) * Rv[k]; break;
            case 5: Qn[k] = Q0[m][k] + ((1.0 / 3.0) * dt) * Rv[k]; break;
            case 6: Qn[k] = Q0[m][k] + (0.5 * dt) * Rv[k]; break;
            default: Qn[k] = Q0[m][k] + dt * Rv[k]; break;
            }
        }
        double *__restrict__ qo = (stage == 3 || stage == 7) ? S.q : ((stage == 2 || stage == 5) ? S.qb : S.qa);
#pragma unroll
        for (int k = 0; k < 5; ++k) qo[k * S.plane + idx] = Qn[k];
        double W[5];
        const double ir = to_prim3(S.gm1, Qn, W);
        if (!physical3(W)) atomicOr(&z.nonphys, 1);
        else if (last) lmax = rmax(lmax, cell_rate3(S, W, ir));
    }
    if (last) reduce_rate_block<NT>(z, stage == 0 ? 0 : (p ^ 1), lmax, sRed);
}

template <int ORDER, int PREC, int TX, int TY, int TZ, int NT>
__global__ __launch_bounds__(NT) void k_stage3(const DevSolve3 *__restrict__ Sp, int stage, int p, int last, double *r_out)
{
    const DevSolve3 &S = *Sp;
    const int bxs = (S.nx + TX - 1) / TX, bys = (S.ny + TY - 1) / TY, bzs = (S.nz + TZ - 1) / TZ;
    const int nb = bxs * bys * bzs;
    const int t = xcd_tile(blockIdx.x, nb);
    if (t >= nb) return;
    const int r = t / bxs;
    stage_brick<ORDER, PREC, TX, TY, TZ, NT>(S, t % bxs, r % bys, r / bys, stage, p, last, t == 0, r_out);
}

// Explicit rate of the state q into the rate words of parity p.
__global__ __launch_bounds__(256) void k_rate3(const DevSolve3 *__restrict__ Sp, int p)
{
    const DevSolve3 &S = *Sp;
    __shared__ double sRed[4];
    double lmax = 0.0;
    const long long n = (long long)S.nx * S.ny * S.nz;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const long long r = c / S.nx;
        const int i = (int)(c - r * S.nx), j = (int)(r % S.ny), l = (int)(r / S.ny);
        double W[5];
        load_prim3(S, S.q, i, j, l, W);
        if (!physical3(W)) atomicOr(&S.slot->nonphys, 1);
        else lmax = rmax(lmax, cell_rate3(S, W, rcp_nr(W[0])));
    }
    const double m = block_max<256>(lmax, sRed);
    if (threadIdx.x == 0 && m > 0.0) reduce_rate(*S.slot, p, m);
}

// Forward Euler: copy the stage result back into q when the step ran and clear
// the rate words the next step's stage reduces into.
__global__ __launch_bounds__(256) void k_copy_back3(const DevSolve3 *__restrict__ Sp, int p)
{
    const DevSolve3 &S = *Sp;
    Slot &z = *S.slot;
    const bool ran = z.st[p ^ 1].steps != z.st[p].steps;
    if (blockIdx.x == 0 && threadIdx.x < kRateSlots) z.rate_bits[p][threadIdx.x] = 0ull;
    if (!ran) return;
    const long long n = (long long)S.nx * S.ny * S.nz;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const long long r = c / S.nx;
        const int i = (int)(c - r * S.nx), j = (int)(r % S.ny), l = (int)(r / S.ny);
        const long long idx = (long long)l * S.slab + (long long)j * S.pitch + i;
#pragma unroll
        for (int k = 0; k < 5; ++k) S.q[k * S.plane + idx] = S.qa[k * S.plane + idx];
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// Brick shapes: id, TX, TY, TZ, threads.  Shapes 4-7 give every face of a
// sweep its own thread (threads >= the largest face count of one axis), so
// each sweep is a single pass.
#define ROEAM_SHAPES3(X)   \
    X(0, 8, 8, 4, 256)     \
    X(1, 8, 4, 4, 128)     \
    X(2, 16, 8, 4, 512)    \
    X(3, 16, 4, 4, 256)    \
    X(4, 8, 8, 4, 320)     \
    X(5, 8, 4, 4, 192)     \
    X(6, 16, 8, 4, 640)    \
    X(7, 8, 8, 8, 576)

struct BrickShape {
    int tx, ty, tz, nt;
};
#define ROEAM_SHAPE3_ENTRY(ID, TX, TY, TZ, NT) {TX, TY, TZ, NT},
static const BrickShape kShapes3[] = {ROEAM_SHAPES3(ROEAM_SHAPE3_ENTRY)};
#undef ROEAM_SHAPE3_ENTRY
constexpr int kNumShapes3 = sizeof(kShapes3) / sizeof(kShapes3[0]);

int brick_shape_count() { return kNumShapes3; }

template <int ORDER, int PREC>
static void launch3_shape(const DevSolve3 *dS, const DevSolve3 &S, int shape, int stage, int p, int last, double *r_out,
                          hipStream_t st)
{
    const BrickShape &sh = kShapes3[shape];
    const long long nb = (long long)((S.nx + sh.tx - 1) / sh.tx) * ((S.ny + sh.ty - 1) / sh.ty) * ((S.nz + sh.tz - 1) / sh.tz);
    const int blocks = (int)(((nb + 7) >> 3) << 3);
#define ROEAM_SHAPE3_CASE(ID, TX, TY, TZ, NT)                                                                    \
    case ID: hipLaunchKernelGGL((k_stage3<ORDER, PREC, TX, TY, TZ, NT>), dim3(blocks), dim3(NT), 0, st, dS, stage, p, \
                                last, r_out); break;
    switch (shape) { ROEAM_SHAPES3(ROEAM_SHAPE3_CASE) }
#undef ROEAM_SHAPE3_CASE
}

hipError_t launch_stage3(const DevSolve3 *dS, const DevSolve3 &S, int shape, int stage, int p, int last, double *r_out,
                         hipStream_t st)
{
    if (shape < 0 || shape >= kNumShapes3) return hipErrorInvalidValue;
    if (S.order == 1) {
        if (S.precision == 0) launch3_shape<1, 0>(dS, S, shape, stage, p, last, r_out, st);
        else launch3_shape<1, 1>(dS, S, shape, stage, p, last, r_out, st);
    } else {
        if (S.precision == 0) launch3_shape<2, 0>(dS, S, shape, stage, p, last, r_out, st);
        else launch3_shape<2, 1>(dS, S, shape, stage, p, last, r_out, st);
    }
    return hipGetLastError();
}

static int grid_blocks3(const DevSolve3 &S)
{
    const long long b = ((long long)S.nx * S.ny * S.nz + 255) / 256;
    return (int)(b > 2048 ? 2048 : (b < 1 ? 1 : b));
}

hipError_t launch_rate3(const DevSolve3 *dS, const DevSolve3 &S, int p, hipStream_t st)
{
    hipLaunchKernelGGL(k_rate3, dim3(grid_blocks3(S)), dim3(256), 0, st, dS, p);
    return hipGetLastError();
}

hipError_t launch_copy_back3(const DevSolve3 *dS, const DevSolve3 &S, int p, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_back3, dim3(grid_blocks3(S)), dim3(256), 0, st, dS, p);
    return hipGetLastError();
}

} // namespace roeam

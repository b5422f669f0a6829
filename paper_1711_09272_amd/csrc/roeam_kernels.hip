// roeam_kernels.hip -- gfx950 kernels of the Roe-AM finite-volume step.
//
// One fused stage kernel per Runge-Kutta stage.  A workgroup owns a tile of
// TX x TY cells: it stages the tile plus its halo as primitives in LDS, builds
// the pressure-density detector ratios of Eq. (97) for every face the tile
// touches, evaluates every face flux of the tile exactly once (Eq. 85), forms
// the conservative residual of each cell and applies the stage update, the
// positivity check and the explicit-rate reduction for the next time step.
#include <type_traits>

#include "roeam_device.hpp"
#include "roeam_internal.hpp"

namespace roeam {

template <int ORDER, int PREC> struct Tile {
    static constexpr int TX = 32, TY = 15, NT = 256, HL = ORDER;
    static constexpr int LX = TX + 2 * HL, LY = TY + 2 * HL;
    static constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1);
};

__device__ __forceinline__ double minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return sgn(a) * rmin(fabs(a), fabs(b));
}

template <int ORDER>
__device__ __forceinline__ void reconstruct(const double m2[4], const double m1[4], const double p0[4],
                                            const double p1[4], double WL[4], double WR[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (ORDER == 1) {
            WL[k] = m1[k];
            WR[k] = p0[k];
        } else {
            WL[k] = m1[k] + 0.5 * minmod(m1[k] - m2[k], p0[k] - m1[k]);
            WR[k] = p0[k] - 0.5 * minmod(p0[k] - m1[k], p1[k] - p0[k]);
        }
    }
}

__device__ __forceinline__ double block_max(double v, double *red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = rmax(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double m = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = rmax(m, red[w]);
    }
    return m;
}

// The tile body.  stage: 0 residual only (r_out), 1 Q + dt R into qa,
// 2 SSP-RK3 second stage into qb, 3 SSP-RK3 third stage into q.
// want_rate: reduce the explicit rate of the produced state (or of the input
// for stage 0) into the solve's slot.
template <int ORDER, int PREC>
__device__ __forceinline__ void stage_tile(const DevSolve &S, int tx, int ty, int stage, int want_rate,
                                           double *__restrict__ r_out)
{
    using T = Tile<ORDER, PREC>;
    using R = typename std::conditional<PREC == 0, double, float>::type;
    constexpr int TX = T::TX, TY = T::TY, HL = T::HL, LX = T::LX, LY = T::LY;
    __shared__ double sW[4][LY][LX];
    __shared__ double sPx[TY + 2][TX + 1];
    __shared__ double sPy[TY + 1][TX + 2];
    __shared__ double sFx[4][TY][TX + 1];
    __shared__ double sFy[4][TY + 1][TX];
    __shared__ double sRed[T::NT / 64];

    const int tid = threadIdx.x;
    double dt = 0.0;
    if (stage > 0) {
        if (!S.slot->active) return;
        dt = S.slot->dt;
    }
    const double *__restrict__ qin = (stage <= 1) ? S.q : (stage == 2 ? S.qa : S.qb);
    const int i0 = tx * TX, j0 = ty * TY;
    const int nx = S.nx, ny = S.ny;

    // 1. tile + halo -> primitives in LDS
    const bool interior = (i0 - HL >= 0) && (i0 + TX + HL <= nx) && (j0 - HL >= 0) && (j0 + TY + HL <= ny);
    for (int e = tid; e < LX * LY; e += T::NT) {
        const int ly = e / LX, lx = e - ly * LX;
        int gi = i0 - HL + lx, gj = j0 - HL + ly;
        double W[4];
        if (interior) {
            load_prim(S, qin, gi, gj, W);
        } else {
            // cells past the ghost layers of a ragged tile feed no valid face
            gi = gi > nx + 1 ? nx + 1 : gi;
            gj = gj > ny + 1 ? ny + 1 : gj;
            fetch_prim(S, qin, gi, gj, W);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) sW[k][ly][lx] = W[k];
    }
    __syncthreads();

    // 2. detector ratios, Eq. (97), from cell-centre values
    if (S.s1_mode == 0) {
        for (int e = tid; e < (TY + 2) * (TX + 1); e += T::NT) {
            const int r = e / (TX + 1), fi = e - r * (TX + 1);
            const int ly = r - 1 + HL;
            sPx[r][fi] = detector_P(sW[3][ly][fi - 1 + HL], sW[0][ly][fi - 1 + HL], sW[3][ly][fi + HL], sW[0][ly][fi + HL]);
        }
        for (int e = tid; e < (TY + 1) * (TX + 2); e += T::NT) {
            const int fr = e / (TX + 2), cc = e - fr * (TX + 2);
            const int lx = cc - 1 + HL;
            sPy[fr][cc] = detector_P(sW[3][fr - 1 + HL][lx], sW[0][fr - 1 + HL][lx], sW[3][fr + HL][lx], sW[0][fr + HL][lx]);
        }
    }
    __syncthreads();

    // 3. every face of the tile once
    for (int f = tid; f < T::NFX + T::NFY; f += T::NT) {
        double m2[4], m1[4], p0[4], p1[4], WL[4], WR[4], F[4];
        double sx, sy, nxv, nyv, len, s1 = 1.0;
        if (f < T::NFX) {
            const int fj = f / (TX + 1), fi = f - fj * (TX + 1);
            const int gi = i0 + fi, gj = j0 + fj;
            if (gi > nx || gj >= ny) continue;
            const int ly = fj + HL, lx = fi + HL;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                m1[k] = sW[k][ly][lx - 1];
                p0[k] = sW[k][ly][lx];
                if (ORDER == 2) {
                    m2[k] = sW[k][ly][lx - 2];
                    p1[k] = sW[k][ly][lx + 1];
                }
            }
            if (S.s1_mode == 0) {
                double a = sPx[fj + 1][fi];
                a = rmin(a, sPy[fj][fi]);
                a = rmin(a, sPy[fj + 1][fi]);
                a = rmin(a, sPy[fj][fi + 1]);
                a = rmin(a, sPy[fj + 1][fi + 1]);
                s1 = pow8(fswitch(a));
            }
            reconstruct<ORDER>(m2, m1, p0, p1, WL, WR);
            xface_vec(S, gi, gj, sx, sy);
            unit_normal(S, sx, sy, nxv, nyv, len);
            roeam_flux<R>(S, WL, WR, nxv, nyv, s1, F);
#pragma unroll
            for (int k = 0; k < 4; ++k) sFx[k][fj][fi] = F[k] * len;
        } else {
            const int g = f - T::NFX;
            const int fr = g / TX, fi = g - fr * TX;
            const int gi = i0 + fi, gj = j0 + fr;
            if (gi >= nx || gj > ny) continue;
            const int ly = fr + HL, lx = fi + HL;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                m1[k] = sW[k][ly - 1][lx];
                p0[k] = sW[k][ly][lx];
                if (ORDER == 2) {
                    m2[k] = sW[k][ly - 2][lx];
                    p1[k] = sW[k][ly + 1][lx];
                }
            }
            if (S.s1_mode == 0) {
                double a = sPy[fr][fi + 1];
                a = rmin(a, sPx[fr][fi]);
                a = rmin(a, sPx[fr][fi + 1]);
                a = rmin(a, sPx[fr + 1][fi]);
                a = rmin(a, sPx[fr + 1][fi + 1]);
                s1 = pow8(fswitch(a));
            }
            reconstruct<ORDER>(m2, m1, p0, p1, WL, WR);
            yface_vec(S, gi, gj, sx, sy);
            unit_normal(S, sx, sy, nxv, nyv, len);
            roeam_flux<R>(S, WL, WR, nxv, nyv, s1, F);
#pragma unroll
            for (int k = 0; k < 4; ++k) sFy[k][fr][fi] = F[k] * len;
        }
    }
    __syncthreads();

    // 4. conservative residual and the stage update
    double lmax = 0.0;
    for (int c = tid; c < TX * TY; c += T::NT) {
        const int cj = c / TX, ci = c - cj * TX;
        const int gi = i0 + ci, gj = j0 + cj;
        if (gi >= nx || gj >= ny) continue;
        const double omega = cell_area(S, gi, gj);
        double Rv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            Rv[k] = -((sFx[k][cj][ci + 1] - sFx[k][cj][ci]) + (sFy[k][cj + 1][ci] - sFy[k][cj][ci])) / omega;
        const long long idx = (long long)gj * S.pitch + gi;
        if (stage == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) r_out[k * S.plane + idx] = Rv[k];
            if (want_rate) {
                double W[4] = {sW[0][cj + HL][ci + HL], sW[1][cj + HL][ci + HL], sW[2][cj + HL][ci + HL],
                               sW[3][cj + HL][ci + HL]};
                lmax = rmax(lmax, cell_rate(S, W, gi, gj));
            }
            continue;
        }
        double Qn[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double Qs = qin[k * S.plane + idx];
            if (stage == 1) {
                Qn[k] = Qs + dt * Rv[k];
            } else {
                const double Q0 = S.q[k * S.plane + idx];
                Qn[k] = (stage == 2) ? 0.75 * Q0 + 0.25 * (Qs + dt * Rv[k])
                                     : (1.0 / 3.0) * Q0 + (2.0 / 3.0) * (Qs + dt * Rv[k]);
            }
        }
        double *__restrict__ qo = (stage == 1) ? S.qa : (stage == 2 ? S.qb : S.q);
#pragma unroll
        for (int k = 0; k < 4; ++k) qo[k * S.plane + idx] = Qn[k];
        double W[4];
        to_prim(S.gm1, Qn[0], Qn[1], Qn[2], Qn[3], W);
        if (!physical(W)) {
            atomicOr(&S.slot->nonphys, 1);
        } else if (want_rate) {
            lmax = rmax(lmax, cell_rate(S, W, gi, gj));
        }
    }
    if (want_rate) {
        const double m = block_max(lmax, sRed);
        if (tid == 0 && m > 0.0) atomicMax(&S.slot->rate_bits, (unsigned long long)__double_as_longlong(m));
    }
}

// Map a linear workgroup id to a tile so that each of the 8 XCDs (which take
// workgroups round-robin) gets a contiguous band of tiles and keeps the
// shared halos in its own L2.
__device__ __forceinline__ int xcd_tile(int b, int ntiles)
{
    const int chunk = (ntiles + 7) >> 3;
    return (b & 7) * chunk + (b >> 3);
}

template <int ORDER, int PREC>
__global__ __launch_bounds__(256) void k_stage_single(DevSolve S, int stage, int want_rate, double *r_out)
{
    const int nt = S.tiles_x * S.tiles_y;
    const int t = xcd_tile(blockIdx.x, nt);
    if (t >= nt) return;
    stage_tile<ORDER, PREC>(S, t % S.tiles_x, t / S.tiles_x, stage, want_rate, r_out);
}

template <int ORDER, int PREC>
__global__ __launch_bounds__(256) void k_stage_batch(const DevSolve *__restrict__ solves, const TileEntry *__restrict__ tiles,
                                                     int ntiles, int stage, int want_rate)
{
    const int t = xcd_tile(blockIdx.x, ntiles);
    if (t >= ntiles) return;
    const TileEntry te = tiles[t];
    stage_tile<ORDER, PREC>(solves[te.solve], te.tx, te.ty, stage, want_rate, nullptr);
}

// Explicit rate of a state (time step of the first step of a run).
__global__ __launch_bounds__(256) void k_rate(DevSolve S)
{
    __shared__ double sRed[4];
    double lmax = 0.0;
    const long long n = (long long)S.nx * S.ny;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(c / S.nx), i = (int)(c - (long long)j * S.nx);
        double W[4];
        load_prim(S, S.q, i, j, W);
        if (!physical(W)) atomicOr(&S.slot->nonphys, 1);
        else lmax = rmax(lmax, cell_rate(S, W, i, j));
    }
    const double m = block_max(lmax, sRed);
    if (threadIdx.x == 0 && m > 0.0) atomicMax(&S.slot->rate_bits, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_slot_init(Slot *s, int n, double t0, double t_end, double cfl, long long max_steps)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    Slot &z = s[k];
    z.t = t0; z.dt = 0.0; z.t_next = t0; z.t_end = t_end; z.cfl = cfl;
    z.rate_last = 0.0; z.dt_last = 0.0; z.rate_bits = 0ull; z.steps = 0; z.max_steps = max_steps;
    z.active = 0; z.nonphys = 0; z.done = 0; z.pad = 0;
}

// Per solve: commit the previous step, then choose the next dt from the
// rate reduced over the current state (or mark the solve done).
__global__ void k_dt(Slot *s, int n, int commit_only)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    Slot &z = s[k];
    if (z.active) {
        z.t = z.t_next;
        z.steps += 1;
        z.dt_last = z.dt;
        z.active = 0;
    }
    if (commit_only) return;
    const double rate = __longlong_as_double((long long)z.rate_bits);
    z.rate_bits = 0ull;
    if (z.nonphys || (z.t_end > 0.0 && z.t >= z.t_end) || z.steps >= z.max_steps || !(rate > 0.0)) {
        z.dt = 0.0;
        z.done = 1;
        return;
    }
    z.rate_last = rate;
    double dt = z.cfl / rate;
    bool last = false;
    if (z.t_end > 0.0 && z.t + dt >= z.t_end) {
        dt = z.t_end - z.t;
        last = true;
    }
    z.dt = dt;
    z.t_next = last ? z.t_end : z.t + dt;
    z.active = 1;
}

__global__ void k_copy_back(DevSolve S)
{
    if (!S.slot->active) return;
    const long long n = (long long)S.nx * S.ny;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(c / S.nx), i = (int)(c - (long long)j * S.nx);
        const long long idx = (long long)j * S.pitch + i;
#pragma unroll
        for (int k = 0; k < 4; ++k) S.q[k * S.plane + idx] = S.qa[k * S.plane + idx];
    }
}

__global__ void k_rate_out(const Slot *s, double *out)
{
    if (threadIdx.x == 0) *out = __longlong_as_double((long long)s->rate_bits);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static int tile_count(const DevSolve &S) { return S.tiles_x * S.tiles_y; }

void tile_shape(int /*order*/, int *tx, int *ty)
{
    *tx = Tile<2, 0>::TX;
    *ty = Tile<2, 0>::TY;
}

hipError_t launch_stage_single(const DevSolve &S, int stage, int want_rate, double *r_out, hipStream_t st)
{
    const int nt = tile_count(S);
    const int blocks = ((nt + 7) >> 3) << 3;
    if (S.order == 1) {
        if (S.precision == 0) hipLaunchKernelGGL((k_stage_single<1, 0>), dim3(blocks), dim3(256), 0, st, S, stage, want_rate, r_out);
        else hipLaunchKernelGGL((k_stage_single<1, 1>), dim3(blocks), dim3(256), 0, st, S, stage, want_rate, r_out);
    } else {
        if (S.precision == 0) hipLaunchKernelGGL((k_stage_single<2, 0>), dim3(blocks), dim3(256), 0, st, S, stage, want_rate, r_out);
        else hipLaunchKernelGGL((k_stage_single<2, 1>), dim3(blocks), dim3(256), 0, st, S, stage, want_rate, r_out);
    }
    return hipGetLastError();
}

hipError_t launch_stage_batch(const DevSolve *solves, const TileEntry *tiles, int ntiles, int order, int precision,
                              int stage, int want_rate, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    const int blocks = ((ntiles + 7) >> 3) << 3;
    if (order == 1) {
        if (precision == 0) hipLaunchKernelGGL((k_stage_batch<1, 0>), dim3(blocks), dim3(256), 0, st, solves, tiles, ntiles, stage, want_rate);
        else hipLaunchKernelGGL((k_stage_batch<1, 1>), dim3(blocks), dim3(256), 0, st, solves, tiles, ntiles, stage, want_rate);
    } else {
        if (precision == 0) hipLaunchKernelGGL((k_stage_batch<2, 0>), dim3(blocks), dim3(256), 0, st, solves, tiles, ntiles, stage, want_rate);
        else hipLaunchKernelGGL((k_stage_batch<2, 1>), dim3(blocks), dim3(256), 0, st, solves, tiles, ntiles, stage, want_rate);
    }
    return hipGetLastError();
}

static int small_grid(long long n)
{
    long long b = (n + 255) / 256;
    return (int)(b > 2048 ? 2048 : (b < 1 ? 1 : b));
}

hipError_t launch_rate(const DevSolve &S, hipStream_t st)
{
    hipLaunchKernelGGL(k_rate, dim3(small_grid((long long)S.nx * S.ny)), dim3(256), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_slot_init(Slot *s, int n, double t0, double t_end, double cfl, long long max_steps, hipStream_t st)
{
    hipLaunchKernelGGL(k_slot_init, dim3((n + 63) / 64), dim3(64), 0, st, s, n, t0, t_end, cfl, max_steps);
    return hipGetLastError();
}

hipError_t launch_dt(Slot *s, int n, int commit_only, hipStream_t st)
{
    hipLaunchKernelGGL(k_dt, dim3((n + 63) / 64), dim3(64), 0, st, s, n, commit_only);
    return hipGetLastError();
}

hipError_t launch_copy_back(const DevSolve &S, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_back, dim3(small_grid((long long)S.nx * S.ny)), dim3(256), 0, st, S);
    return hipGetLastError();
}

hipError_t launch_rate_out(const Slot *s, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_rate_out, dim3(1), dim3(64), 0, st, s, out);
    return hipGetLastError();
}

} // namespace roeam

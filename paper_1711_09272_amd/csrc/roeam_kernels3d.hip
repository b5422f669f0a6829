// roeam_kernels3d.hip -- gfx950 kernels of the 3-D Roe-AM step on uniform
// Cartesian grids: the scalar-free stage kernels (the stage kernel itself is
// in roeam_stage3d.hpp), the explicit rate and the forward-Euler copy back.
#include "roeam_stage3d.hpp"

namespace roeam {

// Explicit rate of the state q into rate-word set `set`.
__global__ __launch_bounds__(256) void k_rate3(const DevSolve3 *__restrict__ Sp, int set)
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
    if (threadIdx.x == 0 && m > 0.0) reduce_rate(*S.slot, set, m);
}

// Forward Euler alternates q -> qa and qa -> q: after an odd number of steps
// (the step state at parity p) the result is in qa and is copied into q.
__global__ __launch_bounds__(256) void k_fe_finish3(const DevSolve3 *__restrict__ Sp, int p)
{
    const DevSolve3 &S = *Sp;
    if ((S.slot->st[p].steps & 1) == 0) return;
    const long long n = (long long)S.nx * S.ny * S.nz;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const long long r = c / S.nx;
        const int i = (int)(c - r * S.nx), j = (int)(r % S.ny), l = (int)(r / S.ny);
        const long long idx = (long long)l * S.slab + (long long)j * S.pitch + i;
        for (int k = 0; k < 5 + S.nsc; ++k) S.q[k * S.plane + idx] = S.qa[k * S.plane + idx];
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int brick_shape_count() { return kNumShapes3; }

// The z-marching shape for a grid: the longest run whose workgroups still
// make three rounds of the three a CU holds (longer runs load fewer planes
// twice; more workgroups keep the chip full), else the shortest run.
int zmarch_auto_shape(int nx, int ny, int nz, int cus)
{
    int best = -1, best_tz = 0, shortest = -1, shortest_tz = 1 << 30;
    for (int s = 0; s < kNumShapes3; ++s) {
        const BrickShape &sh = kShapes3[s];
        if (sh.persistent != 2 || sh.tz <= 0) continue;  // fixed-length runs only
        const long long wgs = (long long)((nx + sh.tx - 1) / sh.tx) * ((ny + sh.ty - 1) / sh.ty) * ((nz + sh.tz - 1) / sh.tz);
        if (wgs >= 9ll * cus && sh.tz > best_tz) best = s, best_tz = sh.tz;
        if (sh.tz < shortest_tz) shortest = s, shortest_tz = sh.tz;
    }
    return best >= 0 ? best : shortest;
}

bool brick_shape_fits(int shape, int order, int nsc)
{
    if (shape < 0 || shape >= kNumShapes3) return false;
    const BrickShape &sh = kShapes3[shape];
    return shape3_lds_bytes(order, nsc, sh.tx, sh.ty, sh.tz, sh.nt, sh.persistent) <= kLdsBytes3;
}

hipError_t launch_stage3(const DevSolve3 *dS, const DevSolve3 &S, int shape, int stage, int p, int last, double *r_out,
                         hipStream_t st)
{
    if (shape < 0 || shape >= kNumShapes3) return hipErrorInvalidValue;
    if (S.nsc > 0) return launch_stage3_sc(dS, S, shape, stage, p, last, r_out, st);
    const hipError_t e = launch3_nsc<0>(dS, S, shape, stage, p, last, r_out, st);
    return e != hipSuccess ? e : hipGetLastError();
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

hipError_t launch_fe_finish3(const DevSolve3 *dS, const DevSolve3 &S, int p, hipStream_t st)
{
    hipLaunchKernelGGL(k_fe_finish3, dim3(grid_blocks3(S)), dim3(256), 0, st, dS, p);
    return hipGetLastError();
}

} // namespace roeam

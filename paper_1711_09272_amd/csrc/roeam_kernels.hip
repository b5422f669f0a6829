// roeam_kernels.hip -- gfx950 kernels of the Roe-AM finite-volume step: the
// stage kernel (templates in roeam_stage2d.hpp) without transported scalars,
// for single grids and batches, and the small kernels around it.
//
// One fused stage kernel per Runge-Kutta stage.  A workgroup owns a tile of
// TX x TY cells: it stages the tile plus its halo as primitives in LDS, builds
// the pressure-density detector ratios of Eq. (97) for every face the tile
// touches, evaluates every face flux of the tile exactly once (Eq. 85; the
// i-faces, then the j-faces through the same LDS buffer), forms the
// conservative residual of each cell in registers and applies the stage
// update, the positivity check and the explicit-rate reduction that sets the
// next time step.  The first stage of a step also derives dt from the
// double-buffered step state, so a step is exactly one kernel per stage.
#include <type_traits>

#include "roeam_device.hpp"
#include "roeam_internal.hpp"
#include "roeam_stage.hpp"
#include "roeam_stage2d.hpp"

namespace roeam {

// Explicit rate of a state (sets dt of the first step of a run) into rate-word
// set `set`.
__global__ __launch_bounds__(256) void k_rate(DevSolve S, int set)
{
    __shared__ double sRed[4];
    double lmax = 0.0;
    const long long n = (long long)S.nx * S.ny;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(c / S.nx), i = (int)(c - (long long)j * S.nx);
        double W[4];
        load_prim(S, S.q, i, j, W);
        if (!physical(W)) atomicOr(&S.slot->nonphys, 1);
        else {
            const double ir = rcp_nr(W[0]);
            lmax = rmax(lmax, S.metric == 0 ? cell_rate<0>(S, W, ir, i, j) : cell_rate<1>(S, W, ir, i, j));
        }
    }
    const double m = block_max<256>(lmax, sRed);
    if (threadIdx.x == 0 && m > 0.0) reduce_rate(*S.slot, set, m);
}

__global__ void k_slot_init(Slot *s, int n, double t0, double t_end, double cfl, long long max_steps)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    Slot &z = s[k];
    for (int q = 0; q < 2; ++q) {
        z.st[q].t = t0;
        z.st[q].dt = 0.0;
        z.st[q].steps = 0;
        z.st[q].pad = 0;
    }
    for (int q = 0; q < kRateSets; ++q)
        for (int w = 0; w < kRateSlots; ++w) z.rate_bits[q][w] = 0ull;
    z.t_end = t_end;
    z.cfl = cfl;
    z.max_steps = max_steps;
    z.dt_last = 0.0;
    z.rate_last = 0.0;
    z.nonphys = 0;
}

// Forward Euler alternates q -> qa and qa -> q: after an odd number of steps
// (the step state at parity p) the result is in qa and is copied into q.
__global__ void k_fe_finish(DevSolve S, int p)
{
    if ((S.slot->st[p].steps & 1) == 0) return;
    const long long n = (long long)S.nx * S.ny;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(c / S.nx), i = (int)(c - (long long)j * S.nx);
        const long long idx = (long long)j * S.pitch + i;
        for (int k = 0; k < 4 + S.nsc; ++k) S.q[k * S.plane + idx] = S.qa[k * S.plane + idx];
    }
}

__global__ void k_rate_out(const Slot *s, double *out)
{
    const double v = read_rate(*s, 0);
    if (threadIdx.x == 0) *out = v;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
struct TileShape {
    int tx, ty, nt;
};
#define ROEAM_SHAPE_ENTRY(ID, TX, TY, NT, SPLIT) {TX, TY, NT},
static const TileShape kShapes[] = {ROEAM_SHAPES(ROEAM_SHAPE_ENTRY)};
#undef ROEAM_SHAPE_ENTRY
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

void tile_shape(int shape, int *tx, int *ty)
{
    const TileShape &s = kShapes[shape < 0 || shape >= kNumShapes ? 0 : shape];
    *tx = s.tx;
    *ty = s.ty;
}

int tile_shape_count() { return kNumShapes; }

hipError_t launch_stage_single(const DevSolve *dS, const DevSolve &S, int shape, int stage, int p, int last,
                               double *r_out, hipStream_t st)
{
    if (shape < 0 || shape >= kNumShapes) return hipErrorInvalidValue;
    if (S.nsc != 0) return launch_stage_single_sc(dS, S, shape, stage, p, last, r_out, st);
    launch_single_nsc<0>(dS, S, shape, stage, p, last, r_out, st);
    return hipGetLastError();
}

hipError_t launch_stage_batch(const DevSolve *solves, const TileEntry *tiles, const int *count, int blocks,
                              bool persistent, int order, int precision, int metric, int nsc, int shape, int stage,
                              int p, int last, hipStream_t st)
{
    if (blocks <= 0) return hipSuccess;
    if (shape < 0 || shape >= kNumShapes || (blocks & 7)) return hipErrorInvalidValue;
    if (nsc != 0)
        return launch_stage_batch_sc(solves, tiles, count, blocks, persistent, order, precision, metric, nsc, shape,
                                     stage, p, last, st);
    launch_batch_nsc<0>(solves, tiles, count, blocks, persistent, order, precision, metric, shape, stage, p, last, st);
    return hipGetLastError();
}

int batch_blocks_per_cu(int order, int precision, int metric, int nsc, int shape)
{
    if (shape < 0 || shape >= kNumShapes) return 0;
    if (nsc != 0) return batch_blocks_per_cu_sc(order, precision, metric, nsc, shape);
    return batch_blocks_per_cu_nsc<0>(order, precision, metric, shape);
}

static int small_grid(long long n)
{
    long long b = (n + 255) / 256;
    return (int)(b > 2048 ? 2048 : (b < 1 ? 1 : b));
}

hipError_t launch_rate(const DevSolve &S, int set, hipStream_t st)
{
    hipLaunchKernelGGL(k_rate, dim3(small_grid((long long)S.nx * S.ny)), dim3(256), 0, st, S, set);
    return hipGetLastError();
}

// Batched runs: per-solve status of the state at parity p, for the host's
// retire decisions.
__global__ void k_status(const Slot *__restrict__ slots, int n, int p, SolveStatus *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const Slot &z = slots[k];
    const StepState &s = z.st[p];
    SolveStatus o;
    o.t = s.t;
    o.steps = s.steps;
    o.dt_last = z.dt_last;
    o.rate_last = z.rate_last;
    o.nonphys = z.nonphys;
    o.done = z.nonphys || s.steps >= z.max_steps || (z.t_end > 0.0 && s.t >= z.t_end);
    out[k] = o;
}

hipError_t launch_status(const Slot *slots, int n, int p, SolveStatus *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_status, dim3((n + 63) / 64), dim3(64), 0, st, slots, n, p, out);
    return hipGetLastError();
}

hipError_t launch_slot_init(Slot *s, int n, double t0, double t_end, double cfl, long long max_steps, hipStream_t st)
{
    hipLaunchKernelGGL(k_slot_init, dim3((n + 63) / 64), dim3(64), 0, st, s, n, t0, t_end, cfl, max_steps);
    return hipGetLastError();
}

hipError_t launch_fe_finish(const DevSolve &S, int p, hipStream_t st)
{
    hipLaunchKernelGGL(k_fe_finish, dim3(small_grid((long long)S.nx * S.ny)), dim3(256), 0, st, S, p);
    return hipGetLastError();
}

hipError_t launch_rate_out(const Slot *s, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_rate_out, dim3(1), dim3(64), 0, st, s, out);
    return hipGetLastError();
}

} // namespace roeam

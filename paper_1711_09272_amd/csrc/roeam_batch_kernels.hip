// roeam_batch_kernels.hip -- the batch engine's admission and retirement
// kernels: every solve admitted (or retired) in one scheduler round is set up
// (or copied out) by two launches, whatever their number.
#include "roeam_internal.hpp"
#include "roeam_stage.hpp"

namespace roeam {

// One thread per entering solve: its descriptor into solves[], its slot
// fresh (t = 0, no steps, zero rate words, the run's limits).
__global__ void k_admit_init(const AdmitInit *__restrict__ inits, int n, DevSolve *__restrict__ solves)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const AdmitInit &a = inits[k];
    solves[a.idx] = a.S;
    Slot &z = *a.S.slot;
    for (int q = 0; q < 2; ++q) {
        z.st[q].t = 0.0;
        z.st[q].dt = 0.0;
        z.st[q].steps = 0;
        z.st[q].pad = 0;
    }
    for (int q = 0; q < kRateSets; ++q)
        for (int w = 0; w < kRateSlots; ++w) z.rate_bits[q][w] = 0ull;
    z.t_end = a.t_end;
    z.cfl = a.cfl;
    z.max_steps = a.nsteps;
    z.dt_last = 0.0;
    z.rate_last = 0.0;
    z.nonphys = 0;
}

// One workgroup per chunk of a move: copy every row of its cells; for an
// admission also the explicit rate of the copied state into rate-word set 0
// of the solve's slot (the same arithmetic as k_rate, so the same bits).
__global__ __launch_bounds__(256) void k_moves(const StateMove *__restrict__ moves, const MoveChunk *__restrict__ chunks,
                                               const DevSolve *__restrict__ solves)
{
    __shared__ double sRed[4];
    const MoveChunk ch = chunks[blockIdx.x];
    const StateMove mv = moves[ch.move];
    const long long n = (long long)mv.nx * mv.ny;
    const long long c1 = ch.c0 + (long long)kMoveChunk < n ? ch.c0 + (long long)kMoveChunk : n;
    const bool rate = mv.solve >= 0;
    double lmax = 0.0;
    for (long long c = ch.c0 + threadIdx.x; c < c1; c += blockDim.x) {
        const int j = (int)(c / mv.nx), i = (int)(c - (long long)j * mv.nx);
        const long long idx = (long long)j * mv.pitch + i;
        double Q[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            Q[k] = gptr(mv.src)[k * mv.plane + idx];
            gptr(mv.dst)[k * mv.plane + idx] = Q[k];
        }
        for (int k = 4; k < mv.rows; ++k) gptr(mv.dst)[k * mv.plane + idx] = gptr(mv.src)[k * mv.plane + idx];
        if (rate) {
            const DevSolve &S = solves[mv.solve];
            double W[4];
            const double ir = to_prim(S.gm1, Q[0], Q[1], Q[2], Q[3], W);
            if (!physical(W)) atomicOr(&S.slot->nonphys, 1);
            else lmax = rmax(lmax, S.metric == 0 ? cell_rate<0>(S, W, ir, i, j) : cell_rate<1>(S, W, ir, i, j));
        }
    }
    if (rate) {
        const double m = block_max<256>(lmax, sRed);
        if (threadIdx.x == 0 && m > 0.0) reduce_rate(*solves[mv.solve].slot, 0, m);
    }
}

hipError_t launch_admit_init(const AdmitInit *inits, int n, DevSolve *solves, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_admit_init, dim3((n + 63) / 64), dim3(64), 0, st, inits, n, solves);
    return hipGetLastError();
}

hipError_t launch_moves(const StateMove *moves, const MoveChunk *chunks, int nchunks, const DevSolve *solves,
                        hipStream_t st)
{
    if (nchunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_moves, dim3(nchunks), dim3(256), 0, st, moves, chunks, solves);
    return hipGetLastError();
}

} // namespace roeam

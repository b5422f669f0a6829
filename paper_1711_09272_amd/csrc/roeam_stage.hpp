// roeam_stage.hpp -- device helpers shared by the 2-D and 3-D stage kernels:
// the MUSCL limiter, the explicit-rate words of a solve's slot, the step
// state that the first stage of every step advances, and the XCD-aware
// workgroup-to-tile map.
#pragma once

#include <hip/hip_runtime.h>

#include "roeam_device.hpp"

namespace roeam {

// minmod(a, b): 0 when the slopes differ in sign, else the one nearer zero,
// which is the median of a, b and 0: max(min(a, b), min(max(a, b), 0)) (four
// min/max).
__device__ __forceinline__ double minmod(double a, double b)
{
    return rmax(rmin(a, b), rmin(rmax(a, b), 0.0));
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double *red)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = rmax(v, __shfl_xor(v, o, 64));
    if (NT == 64) return v;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double m = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) m = rmax(m, red[w]);
    return m;
}

// Rate-word set of the state after n steps.
__host__ __device__ __forceinline__ int rate_set(long long n) { return (int)(n % kRateSets); }

// Max explicit rate in word set `set`: lane k of every wave reads rate word k,
// then a wave max.  Every lane of every wave ends with the same value.
__device__ __forceinline__ double read_rate(const Slot &z, int set)
{
    static_assert(kRateSlots == 64, "one rate word per lane");
    const int lane = threadIdx.x & 63;
    double v = __longlong_as_double((long long)z.rate_bits[set][lane]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = rmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ void reduce_rate(Slot &z, int set, double v)
{
    atomicMax(&z.rate_bits[set][blockIdx.x & (kRateSlots - 1)], (unsigned long long)__double_as_longlong(v));
}

// Workgroup reduction of the rate of the new state, then one device-scope
// atomic per workgroup (word = workgroup id mod kRateSlots).  One atomic per
// wave instead (no barrier) measured 25% slower on the last stage of a 2048^2
// grid: the atomics on the 64 words contend.  red: NT/64 doubles of LDS.
template <int NT>
__device__ __forceinline__ void reduce_rate_block(Slot &z, int set, double v, double *red)
{
    const double m = block_max<NT>(v, red);
    if (threadIdx.x == 0 && m > 0.0) reduce_rate(z, set, m);
}

// Stage codes of the stage kernel: 0 residual only; 1 forward Euler (steps
// of even parity) or the first SSP-RK3 stage; 2, 3 the second and third
// SSP-RK3 stages; 4-7 the four stages of the four-stage scheme; 8 forward
// Euler on steps of odd parity.  The buffers each stage reads (stencil) and
// writes, and whether it also reads Q^n at its own cells:
//   1: q -> qa     2: qa -> qb (+Q^n)   3: qb -> q (+Q^n)
//   4: q -> qa     5: qa -> qb (+Q^n)   6: qb -> qa (+Q^n)   7: qa -> q (+Q^n)
//   8: qa -> q
// (a stage that writes q reads its stencil from another buffer, and its
// pointwise read of Q^n is the cell it writes).  Forward Euler alternates
// q -> qa and qa -> q, so after an odd number of steps the state is in qa.
__host__ __device__ constexpr bool first_stage(int stage) { return stage == 1 || stage == 4 || stage == 8; }
// buffer a stage reads its stencil from / writes: 0 q, 1 qa, 2 qb
__host__ __device__ constexpr int stage_in_buf(int stage)
{
    return (stage <= 1 || stage == 4) ? 0 : ((stage == 3 || stage == 6) ? 2 : 1);
}
__host__ __device__ constexpr int stage_out_buf(int stage)
{
    return (stage == 3 || stage == 7 || stage == 8) ? 0 : ((stage == 2 || stage == 5) ? 2 : 1);
}
__host__ __device__ constexpr bool stage_reads_qn(int stage)
{
    return stage == 2 || stage == 3 || stage == 5 || stage == 6 || stage == 7;
}

// Fraction of dt at which a stage's input state lies (the abscissae c of the
// schemes): stage codes 1-3 are SSP-RK3 (0, 1, 1/2), 4-7 the four-stage scheme
// (0, 1/4, 1/3, 1/2).
__host__ __device__ constexpr double stage_abscissa(int stage)
{
    return stage == 2 ? 1.0 : stage == 3 ? 0.5 : stage == 5 ? 0.25 : stage == 6 ? 1.0 / 3.0 : stage == 7 ? 0.5 : 0.0;  // 8: 0
}

// The words of the step state a stage decides on, read through a global view
// (global, not flat, loads: a kernel issues them before its own-cell loads and
// waits for them without waiting for those).  None of them is written by the
// kernel that reads them: the first stage reads parity p and publishes p^1.
struct StepWords {
    unsigned long long rate_bits;  // rate word `lane` of the input state's set (first stage)
    double t, t_end, cfl, dt_n;
    long long steps, steps_n, max_steps;
    int nonphys;
};

__device__ __forceinline__ StepWords load_step_words(const Slot &zs, int p, int stage)
{
    typedef __attribute__((address_space(1))) const Slot GSlot;
    GSlot &z = *(GSlot *)&zs;
    StepWords w{};
    w.steps = z.st[p].steps;
    if (!first_stage(stage)) {
        w.dt_n = z.st[p ^ 1].dt;
        w.steps_n = z.st[p ^ 1].steps;
        return w;
    }
    // all three sets are read, and the input state's one kept, so that no
    // load waits for the step count
    const unsigned long long r0 = z.rate_bits[0][threadIdx.x & 63], r1 = z.rate_bits[1][threadIdx.x & 63],
                             r2 = z.rate_bits[2][threadIdx.x & 63];
    const int set = rate_set(w.steps);
    w.rate_bits = set == 0 ? r0 : (set == 1 ? r1 : r2);
    w.t = z.st[p].t;
    w.t_end = z.t_end;
    w.cfl = z.cfl;
    w.max_steps = z.max_steps;
    w.nonphys = z.nonphys;
    return w;
}

// Time-step logic shared by all stage kernels of a step with parity p.
// Returns whether the step is active and its dt.
__device__ __forceinline__ bool step_active(const StepWords &w, int stage, double &dt, double &t_next, double &rate)
{
    if (!first_stage(stage)) {
        // the first stage has already decided: the step ran iff it advanced the count
        dt = w.dt_n;
        return w.steps_n != w.steps;
    }
    // max explicit rate of the state: a wave max over its 64 rate words
    double v = __longlong_as_double((long long)w.rate_bits);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = rmax(v, __shfl_xor(v, o, 64));
    rate = v;
    if (w.nonphys || (w.t_end > 0.0 && w.t >= w.t_end) || w.steps >= w.max_steps || !(rate > 0.0)) return false;
    dt = w.cfl / rate;
    t_next = w.t + dt;
    if (w.t_end > 0.0 && w.t + dt >= w.t_end) {
        dt = w.t_end - w.t;
        t_next = w.t_end;
    }
    return true;
}

// Start of a stage kernel's workgroup: decide whether the step is active and
// its dt; on the first stage, workgroup 0 (first_block) publishes the next
// step state and clears the rate words of the step after this one (set
// n + 2 for input step count n).  w: load_step_words(z, p, stage).
// A value that is the same in every lane of the wave, moved to scalar
// registers (the compiler cannot tell that a value read from memory by every
// lane at the same address is uniform).
__device__ __forceinline__ double wave_uniform(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ bool begin_stage(Slot &z, const StepWords &w, int p, int stage, int last, int first_block,
                                            double &dt)
{
    double t_next = 0.0, rate = 0.0;
    const bool active = step_active(w, stage, dt, t_next, rate);
    if (first_stage(stage) && first_block) {
        const int tid = threadIdx.x;
        if (tid == 0) {
            StepState &n = z.st[p ^ 1];
            if (active) {
                n.t = t_next;
                n.dt = dt;
                n.steps = w.steps + 1;
                z.dt_last = dt;
                z.rate_last = rate;
            } else {
                n.t = w.t;
                n.dt = 0.0;
                n.steps = w.steps;
            }
        }
        // set n + 1 (this step's result) was cleared by the previous step;
        // set n was read by this step's workgroups and stays until step n + 1
        (void)last;
        if (tid < kRateSlots) z.rate_bits[rate_set(w.steps + 2)][tid] = 0ull;
    }
    dt = wave_uniform(dt);  // every lane read the same step words
    return active;
}

// Map a linear workgroup id to a tile so that each of the 8 XCDs (which take
// workgroups round-robin) gets a contiguous band of tiles and keeps the
// shared halos in its own L2.
__device__ __forceinline__ int xcd_tile(int b, int ntiles)
{
    const int chunk = (ntiles + 7) >> 3;
    return (b & 7) * chunk + (b >> 3);
}

} // namespace roeam

// roeam_internal.hpp -- declarations shared by the kernel and runtime
// translation units of the gfx950 library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "roeam_device.hpp"

namespace roeam {

// One tile of one solve in a batched work list.
struct TileEntry {
    int solve, tx, ty, pad;
};

void tile_shape(int order, int *tx, int *ty);
hipError_t launch_stage_single(const DevSolve &S, int stage, int want_rate, double *r_out, hipStream_t st);
hipError_t launch_stage_batch(const DevSolve *solves, const TileEntry *tiles, int ntiles, int order, int precision,
                              int stage, int want_rate, hipStream_t st);
hipError_t launch_rate(const DevSolve &S, hipStream_t st);
hipError_t launch_slot_init(Slot *s, int n, double t0, double t_end, double cfl, long long max_steps, hipStream_t st);
hipError_t launch_dt(Slot *s, int n, int commit_only, hipStream_t st);
hipError_t launch_copy_back(const DevSolve &S, hipStream_t st);
hipError_t launch_rate_out(const Slot *s, double *out, hipStream_t st);

} // namespace roeam

// roeam_internal.hpp -- declarations shared by the kernel and runtime
// translation units of the gfx950 library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "roeam_device.hpp"
#include "roeam_device3d.hpp"

namespace roeam {

// One tile of one solve in a batched work list.
struct TileEntry {
    int solve, tx, ty, pad;
};

// Compact per-solve status copied to the host after batched iterations.
struct SolveStatus {
    double t, dt_last, rate_last;
    long long steps;
    int nonphys, done;
};

// Batched state moves of the batch engine: one solve's state copied between
// a caller's buffer and the arena (src == dst: in place), and, on admission,
// the explicit rate of the moved state reduced into the solve's fresh slot.
struct StateMove {
    const double *src;
    double *dst;
    long long plane, pitch;  // elements per row of the state; per grid line
    int nx, ny, rows;
    int solve;               // index of the solve whose initial rate it sets (-1: copy only)
};
// Cells [c0, c0 + kMoveChunk) of move `move`: one workgroup each.
struct MoveChunk {
    int move, c0;
};
constexpr int kMoveChunk = 2048;
// A solve entering the batch: its descriptor and its slot's initial state.
struct AdmitInit {
    DevSolve S;
    double t_end, cfl;
    long long nsteps;
    int idx, pad;
};
// Descriptors into solves[], fresh slots; then the moves (after the
// descriptors: a moving state's rate reads its solve's descriptor).
hipError_t launch_admit_init(const AdmitInit *inits, int n, DevSolve *solves, hipStream_t st);
hipError_t launch_moves(const StateMove *moves, const MoveChunk *chunks, int nchunks, const DevSolve *solves,
                        hipStream_t st);

// Tile shapes of the stage kernel: 0 = 32x15 cells / 256 threads,
// 1 = 16x15 / 128, 2 = 8x7 / 64.
void tile_shape(int shape, int *tx, int *ty);
int tile_shape_count();
// dS: the descriptor in device memory (read by the kernel); S: its host copy.
hipError_t launch_stage_single(const DevSolve *dS, const DevSolve &S, int shape, int stage, int p, int last,
                               double *r_out, hipStream_t st);
// The same with one or two transported scalars (S.nsc), roeam_kernels_sc.hip.
hipError_t launch_stage_single_sc(const DevSolve *dS, const DevSolve &S, int shape, int stage, int p, int last,
                                  double *r_out, hipStream_t st);
// Batched stage kernel over the tiles of one group (solves that share order,
// precision, metric and scalar count nsc); nsc > 0 in roeam_kernels_sc.hip.
// The kernels read the tile count from device memory (*count); `blocks` (a
// multiple of 8) workgroups of the windowed form (one tile each, the rest
// exit) or of the persistent form (resident workgroups taking tiles in turn).
hipError_t launch_stage_batch(const DevSolve *solves, const TileEntry *tiles, const int *count, int blocks,
                              bool persistent, int order, int precision, int metric, int nsc, int shape, int stage,
                              int p, int last, hipStream_t st);
hipError_t launch_stage_batch_sc(const DevSolve *solves, const TileEntry *tiles, const int *count, int blocks,
                                 bool persistent, int order, int precision, int metric, int nsc, int shape, int stage,
                                 int p, int last, hipStream_t st);
// Resident workgroups per CU of the persistent batched kernel.
int batch_blocks_per_cu(int order, int precision, int metric, int nsc, int shape);
int batch_blocks_per_cu_sc(int order, int precision, int metric, int nsc, int shape);
// Explicit rate of S's state q into rate-word set `set` (0 for a fresh slot).
hipError_t launch_rate(const DevSolve &S, int set, hipStream_t st);
hipError_t launch_status(const Slot *slots, int n, int p, SolveStatus *out, hipStream_t st);
hipError_t launch_slot_init(Slot *s, int n, double t0, double t_end, double cfl, long long max_steps, hipStream_t st);
// Forward Euler: copy qa into q when the step state at parity p counts an odd
// number of steps (the state then sits in qa).
hipError_t launch_fe_finish(const DevSolve &S, int p, hipStream_t st);
hipError_t launch_rate_out(const Slot *s, double *out, hipStream_t st);
// RMS and max |.| per row of r[k][line][pitch] (rows 4..7, nx valid per line)
// into out[2 rows]; part: scratch of 2 rows doubles per block, max_blocks blocks.
constexpr int kNormMaxBlocks = 1024;
hipError_t launch_norms(const double *r, int rows, long long plane, int nx, int nlines, long long pitch, double *part,
                        int max_blocks, double *out, hipStream_t st);
// Doubles of partials launch_norms uses for these sizes.
long long norms_partial_doubles(int rows, int nx, int nlines, int max_blocks);
// Take the device address of the allocation-free norms scratch on `device`
// (the current device), once per device; called when a context is created.
hipError_t scratch_setup(int device);

// 3-D uniform Cartesian grids (brick shapes 0..brick_shape_count()-1).
int brick_shape_count();
// Whether a brick shape's stage kernel fits the LDS of a workgroup for the given
// MUSCL order and scalar count (16x8x4 bricks do not with two scalars).
bool brick_shape_fits(int shape, int order, int nsc);
int zmarch_auto_shape(int nx, int ny, int nz, int cus);
hipError_t launch_stage3_sc(const DevSolve3 *dS, const DevSolve3 &S, int shape, int stage, int p, int last,
                            double *r_out, hipStream_t st);
hipError_t launch_stage3(const DevSolve3 *dS, const DevSolve3 &S, int shape, int stage, int p, int last, double *r_out,
                         hipStream_t st);
hipError_t launch_rate3(const DevSolve3 *dS, const DevSolve3 &S, int p, hipStream_t st);
hipError_t launch_fe_finish3(const DevSolve3 *dS, const DevSolve3 &S, int p, hipStream_t st);

} // namespace roeam

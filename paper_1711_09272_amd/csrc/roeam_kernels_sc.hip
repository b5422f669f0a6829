// roeam_kernels_sc.hip -- the 2-D stage kernel with one or two transported
// scalars (the rho k rows of Eq. 85), single-grid and batched launches.  A translation unit
// of its own so that these instantiations compile beside the scalar-free ones.
#include "roeam_stage2d.hpp"

namespace roeam {

hipError_t launch_stage_single_sc(const DevSolve *dS, const DevSolve &S, int shape, int stage, int p, int last,
                                  double *r_out, hipStream_t st)
{
    if (shape < 0 || shape >= tile_shape_count()) return hipErrorInvalidValue;
    if (S.nsc == 1) launch_single_nsc<1>(dS, S, shape, stage, p, last, r_out, st);
    else if (S.nsc == 2) launch_single_nsc<2>(dS, S, shape, stage, p, last, r_out, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_stage_batch_sc(const DevSolve *solves, const TileEntry *tiles, const int *count, int blocks,
                                 bool persistent, int order, int precision, int metric, int nsc, int shape, int stage,
                                 int p, int last, hipStream_t st)
{
    if (shape < 0 || shape >= tile_shape_count()) return hipErrorInvalidValue;
    if (nsc == 1)
        launch_batch_nsc<1>(solves, tiles, count, blocks, persistent, order, precision, metric, shape, stage, p, last, st);
    else if (nsc == 2)
        launch_batch_nsc<2>(solves, tiles, count, blocks, persistent, order, precision, metric, shape, stage, p, last, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

int batch_blocks_per_cu_sc(int order, int precision, int metric, int nsc, int shape)
{
    if (nsc == 1) return batch_blocks_per_cu_nsc<1>(order, precision, metric, shape);
    if (nsc == 2) return batch_blocks_per_cu_nsc<2>(order, precision, metric, shape);
    return 0;
}

} // namespace roeam

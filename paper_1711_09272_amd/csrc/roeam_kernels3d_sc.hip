// roeam_kernels3d_sc.hip -- the 3-D stage kernel with one or two transported
// scalars (the rho k rows of Eq. 85).  A translation unit of its own so that
// these instantiations compile beside the scalar-free ones.
#include "roeam_stage3d.hpp"

namespace roeam {

hipError_t launch_stage3_sc(const DevSolve3 *dS, const DevSolve3 &S, int shape, int stage, int p, int last,
                            double *r_out, hipStream_t st)
{
    if (shape < 0 || shape >= kNumShapes3) return hipErrorInvalidValue;
    hipError_t e;
    if (S.nsc == 1) e = launch3_nsc<1>(dS, S, shape, stage, p, last, r_out, st);
    else if (S.nsc == 2) e = launch3_nsc<2>(dS, S, shape, stage, p, last, r_out, st);
    else return hipErrorInvalidValue;
    return e != hipSuccess ? e : hipGetLastError();
}

} // namespace roeam

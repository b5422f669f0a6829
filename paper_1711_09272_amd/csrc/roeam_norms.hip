// roeam_norms.hip -- residual norms (RMS and max |.| per row) of 2-D and 3-D
// residual arrays, by a fixed-order reduction whose result does not depend on
// timing.
#include "roeam_device.hpp"
#include "roeam_internal.hpp"
#include "roeam_stage.hpp"

namespace roeam {

// ---------------------------------------------------------------------------
// residual norms: RMS and max |.| per row of an array r[k][line][pitch]
// (nx valid elements per line), by a fixed-order two-pass reduction, so the
// result does not depend on timing: pass 1, block b sums the lines
// [b L, (b+1) L) with a fixed per-thread stride and a fixed tree; pass 2, one
// block combines the partials in block order.
// ---------------------------------------------------------------------------
constexpr int kNormThreads = 256;

template <int ROWS>
__global__ __launch_bounds__(kNormThreads) void k_norms_partial(const double *__restrict__ r, long long plane, int nx,
                                                                int nlines, long long pitch, int lines_per_block,
                                                                double *__restrict__ part)
{
    __shared__ double sS[ROWS][kNormThreads], sM[ROWS][kNormThreads];
    double ss[ROWS], mx[ROWS];
#pragma unroll
    for (int k = 0; k < ROWS; ++k) ss[k] = mx[k] = 0.0;
    const int l0 = blockIdx.x * lines_per_block, l1 = min(nlines, l0 + lines_per_block);
    const long long n = (long long)(l1 - l0) * nx;
    for (long long c = threadIdx.x; c < n; c += kNormThreads) {
        const int l = l0 + (int)(c / nx), i = (int)(c % nx);
        const long long idx = (long long)l * pitch + i;
#pragma unroll
        for (int k = 0; k < ROWS; ++k) {
            const double v = r[k * plane + idx];
            ss[k] = fma(v, v, ss[k]);
            mx[k] = rmax(mx[k], fabs(v));
        }
    }
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
        sS[k][threadIdx.x] = ss[k];
        sM[k][threadIdx.x] = mx[k];
    }
    __syncthreads();
    for (int h = kNormThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
#pragma unroll
            for (int k = 0; k < ROWS; ++k) {
                sS[k][threadIdx.x] += sS[k][threadIdx.x + h];
                sM[k][threadIdx.x] = rmax(sM[k][threadIdx.x], sM[k][threadIdx.x + h]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < ROWS) {
        part[(long long)blockIdx.x * 2 * ROWS + threadIdx.x] = sS[threadIdx.x][0];
        part[(long long)blockIdx.x * 2 * ROWS + ROWS + threadIdx.x] = sM[threadIdx.x][0];
    }
}

template <int ROWS>
__global__ __launch_bounds__(kNormThreads) void k_norms_final(const double *__restrict__ part, int nblocks,
                                                              double inv_cells, double *__restrict__ out)
{
    // thread t < 2 ROWS owns one output and walks the partials in block order
    const int t = threadIdx.x;
    if (t >= 2 * ROWS) return;
    double a = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        const double v = part[(long long)b * 2 * ROWS + t];
        a = t < ROWS ? a + v : rmax(a, v);
    }
    out[t] = t < ROWS ? sqrt(a * inv_cells) : a;
}

hipError_t launch_norms(const double *r, int rows, long long plane, int nx, int nlines, long long pitch, double *part,
                        int max_blocks, double *out, hipStream_t st)
{
    if (rows < 4 || rows > 7 || nx < 1 || nlines < 1) return hipErrorInvalidValue;
    // about 8 elements per thread per block, at most max_blocks blocks
    long long lines_per_block = ((long long)kNormThreads * 8 + nx - 1) / nx;
    long long nb = (nlines + lines_per_block - 1) / lines_per_block;
    if (nb > max_blocks) {
        lines_per_block = (nlines + max_blocks - 1) / max_blocks;
        nb = (nlines + lines_per_block - 1) / lines_per_block;
    }
    const double inv = 1.0 / ((double)nx * (double)nlines);
#define ROEAM_NORMS(R)                                                                                            \
    case R:                                                                                                       \
        hipLaunchKernelGGL(k_norms_partial<R>, dim3((unsigned)nb), dim3(kNormThreads), 0, st, r, plane, nx, nlines, \
                           pitch, (int)lines_per_block, part);                                                    \
        hipLaunchKernelGGL(k_norms_final<R>, dim3(1), dim3(kNormThreads), 0, st, part, (int)nb, inv, out);       \
        break;
    switch (rows) { ROEAM_NORMS(4) ROEAM_NORMS(5) ROEAM_NORMS(6) ROEAM_NORMS(7) default: return hipErrorInvalidValue; }
#undef ROEAM_NORMS
    return hipGetLastError();
}

} // namespace roeam

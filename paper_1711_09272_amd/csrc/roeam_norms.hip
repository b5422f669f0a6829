// roeam_norms.hip -- residual norms (RMS and max |.| per row) of 2-D and 3-D
// residual arrays, by a fixed-order reduction whose result does not depend on
// timing.
#include <mutex>

#include "roeam_device.hpp"
#include "roeam_host.hpp"
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

// Partition of nlines lines of nx elements over the partial blocks: about 8
// elements per thread per block, at most max_blocks blocks.
static void norms_partition(int nx, int nlines, int max_blocks, long long *lines_per_block, long long *nblocks)
{
    long long lpb = ((long long)kNormThreads * 8 + nx - 1) / nx;
    long long nb = (nlines + lpb - 1) / lpb;
    if (nb > max_blocks) {
        lpb = (nlines + max_blocks - 1) / max_blocks;
        nb = (nlines + lpb - 1) / lpb;
    }
    *lines_per_block = lpb;
    *nblocks = nb;
}

long long norms_partial_doubles(int rows, int nx, int nlines, int max_blocks)
{
    long long lpb = 0, nb = 0;
    norms_partition(nx, nlines, max_blocks, &lpb, &nb);
    return 2ll * rows * nb;
}

hipError_t launch_norms(const double *r, int rows, long long plane, int nx, int nlines, long long pitch, double *part,
                        int max_blocks, double *out, hipStream_t st)
{
    if (rows < 4 || rows > 7 || nx < 1 || nlines < 1) return hipErrorInvalidValue;
    long long lines_per_block = 0, nb = 0;
    norms_partition(nx, nlines, max_blocks, &lines_per_block, &nb);
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

// ---------------------------------------------------------------------------
// Allocation-free residual norms.  The partials of the two-pass reduction live
// in a file-scope device array, one copy per GPU for the life of the process,
// sized for the most rows a 2-D grid has (4 + kMaxScalars) and the most
// partial blocks launch_norms uses.  In host code the array's name is only a
// host-side stand-in: its device address on each GPU is taken once, with that
// GPU current, when a context is created on it (scratch_setup), and only that
// address is passed to kernels.  Every call on one GPU shares the array.
// ---------------------------------------------------------------------------
constexpr int kScratchRows = 4 + kMaxScalars;
constexpr long long kScratchDoubles = 2ll * kScratchRows * kNormMaxBlocks;  // 96 KiB
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static double *g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[device] = (double *)p;
    return hipSuccess;
}

static double *scratch_on(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[device];
}

} // namespace roeam

extern "C" roeam_status roeam_residual_norms_noalloc(roeam_ctx *ctx, const roeam_grid *g, const double *r,
                                                     double *norms_out)
{
    if (!ctx || !g || !r || !norms_out) return roeam_fail(ctx, ROEAM_EINVAL, "NULL argument");
    if (g->ctx != ctx) return roeam_fail(ctx, ROEAM_EINVAL, "grid belongs to another context");
    const int rows = 4 + g->nsc;
    const long long need = roeam::norms_partial_doubles(rows, g->nx, g->ny, roeam::kNormMaxBlocks);
    if (rows > roeam::kScratchRows || need > roeam::kScratchDoubles)
        return roeam_fail(ctx, ROEAM_EINVAL,
                          "residual norms need " + std::to_string(need) + " partial doubles, more than the " +
                              std::to_string(roeam::kScratchDoubles) + " of the static scratch");
    double *part = roeam::scratch_on(ctx->device);
    if (!part) return roeam_fail(ctx, ROEAM_EDEVICE, "static scratch has no device address on this GPU");
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = roeam::launch_norms(r, rows, (long long)g->ny * g->pitch, g->nx, g->ny, g->pitch, part, roeam::kNormMaxBlocks,
                                norms_out, ctx->stream);
    if (e != hipSuccess) return roeam_fail(ctx, ROEAM_EDEVICE, std::string("residual norms: ") + hipGetErrorString(e));
    return ROEAM_OK;
}

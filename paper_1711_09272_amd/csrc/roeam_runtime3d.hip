// roeam_runtime3d.hip -- host side of the 3-D part of the C ABI in
// include/roeam.h: uniform Cartesian 3-D grids, the residual call and the
// graph-captured step loop (same step state and stage codes as 2-D grids).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "roeam_host.hpp"

using roeam::DevSolve3;

struct roeam_grid3d {
    roeam_ctx *ctx = nullptr;
    int nx = 0, ny = 0, nz = 0;
    long long pitch = 0;
    double dx = 0, dy = 0, dz = 0;
    int bc[6] = {0, 0, 0, 0, 0, 0};
    double bcq[6][5] = {};
    double *d_qa = nullptr, *d_qb = nullptr;
    Slot *d_slot = nullptr;
    Slot *h_slot = nullptr;           // pinned readback
    DevSolve3 *d_solve = nullptr;     // descriptor read by the kernels
    DevSolve3 *h_solve = nullptr;     // pinned staging copy of the last descriptor sent
    bool solve_valid = false;
    GraphCache gc;
    int shape = -1;                   // -1: the z-marching shape chosen for the grid's size
    double *d_norm_part = nullptr;    // scratch of roeam_residual_norms3d
    int final_parity = 0;
    int nsc = 0;                      // transported scalars (rows 5 .. 4 + nsc of q)
    double bcs[6][roeam::kMaxScalars] = {}; // Dirichlet rho k_m per side
};

// Compute units of a device (queried once per device).
static int device_cus(int dev)
{
    constexpr int kMaxDevices = 64;
    static std::atomic<int> cached[kMaxDevices];  // 0: not queried yet (threads may race to fill it alike)
    if (dev < 0 || dev >= kMaxDevices) return 256;
    int v = cached[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1) v = 256;
        cached[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// Shape the stage kernel runs with: the grid's; by default the z-marching
// shape for the grid's size; persistent 8x8x8 bricks with 512 threads where
// the grid's does not fit the LDS with its scalars (fastest measured with two
// scalars on 128^3 among the bricks: 350 us per stage, the 8x8x4/320 brick 561).
constexpr int kFallbackShape3 = 9;
static int stage_shape3(const roeam_grid3d *g, int order)
{
    const int shape = g->shape >= 0 ? g->shape : roeam::zmarch_auto_shape(g->nx, g->ny, g->nz, device_cus(g->ctx->device));
    return roeam::brick_shape_fits(shape, order, g->nsc) ? shape : kFallbackShape3;
}

static roeam_status fail(roeam_ctx *ctx, roeam_status st, const std::string &msg) { return roeam_fail(ctx, st, msg); }

static roeam_status hip_fail(roeam_ctx *ctx, hipError_t e, const char *where)
{
    return fail(ctx, ROEAM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_OK(ctx, call)                                      \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

static DevSolve3 make_solve3(const roeam_grid3d *g, const roeam_params *p, double *q)
{
    DevSolve3 S;
    std::memset(&S, 0, sizeof S);
    S.nx = g->nx;
    S.ny = g->ny;
    S.nz = g->nz;
    S.pitch = g->pitch;
    S.slab = (long long)g->ny * g->pitch;
    S.plane = (long long)g->nz * S.slab;
    S.ax = g->dy * g->dz;
    S.ay = g->dx * g->dz;
    S.az = g->dx * g->dy;
    S.inv_vol = 1.0 / (g->dx * g->dy * g->dz);
    const double gm1 = p->gamma - 1.0;
    for (int s = 0; s < 6; ++s) {
        S.bc[s] = g->bc[s];
        const double *Q = g->bcq[s];
        if (g->bc[s] != ROEAM_BC_DIRICHLET) continue;
        const double rho = Q[0], u = Q[1] / rho, v = Q[2] / rho, w = Q[3] / rho;
        S.bcw[s][0] = rho;
        S.bcw[s][1] = u;
        S.bcw[s][2] = v;
        S.bcw[s][3] = w;
        S.bcw[s][4] = gm1 * (Q[4] - 0.5 * rho * (u * u + v * v + w * w));
    }
    S.gamma = p->gamma;
    S.gm1 = gm1;
    S.g_gm1 = p->gamma / gm1;
    S.igm1 = 1.0 / gm1;
    S.mr2 = p->mach_ref * p->mach_ref;
    S.dv_min2 = (1e-5 * p->u_ref) * (1e-5 * p->u_ref);
    S.eps1 = p->eps1;
    S.eps2 = p->eps2;
    S.eps_lambda = p->eps_lambda;
    S.s1_mode = p->s1_mode;
    S.order = p->order;
    S.precision = p->precision;
    S.scheme = p->scheme;
    S.variant = p->variant;
    S.q = q;
    S.qa = g->d_qa;
    S.qb = g->d_qb;
    S.slot = g->d_slot;
    S.nsc = g->nsc;
    for (int s = 0; s < 6; ++s)
        if (g->bc[s] == ROEAM_BC_DIRICHLET)
            for (int m = 0; m < g->nsc; ++m) S.bck[s][m] = g->bcs[s][m] / g->bcq[s][0];
    return S;
}

// Make the grid's device descriptor equal to S; work already queued may still
// read the old one, so a change waits for the stream first.
static hipError_t upload_solve3(roeam_grid3d *g, const DevSolve3 &S, hipStream_t s)
{
    if (g->solve_valid && std::memcmp(g->h_solve, &S, sizeof S) == 0) return hipSuccess;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    std::memcpy(g->h_solve, &S, sizeof S);
    e = hipMemcpyAsync(g->d_solve, g->h_solve, sizeof S, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    g->solve_valid = true;
    return hipSuccess;
}

static roeam_status ensure_stage_buffers3(roeam_ctx *ctx, roeam_grid3d *g)
{
    if (g->d_qa && g->d_qb) return ROEAM_OK;
    const size_t bytes = sizeof(double) * (5 + (size_t)g->nsc) * (size_t)g->nz * (size_t)g->ny * (size_t)g->pitch;
    hipError_t e = g->d_qa ? hipSuccess : hipMalloc(&g->d_qa, bytes);
    if (e == hipSuccess && !g->d_qb) e = hipMalloc(&g->d_qb, bytes);
    if (e != hipSuccess)
        return fail(ctx, e == hipErrorOutOfMemory ? ROEAM_ENOMEM : ROEAM_EDEVICE,
                    std::string("stage buffers: ") + hipGetErrorString(e));
    g->solve_valid = false;
    return ROEAM_OK;
}

// One time step with parity p: one kernel per stage; forward Euler goes
// q -> qa on even and qa -> q on odd steps.
static hipError_t enqueue_step3(const roeam_grid3d *g, const DevSolve3 &S, int time_scheme, int p, hipStream_t st)
{
    const DevSolve3 *d = g->d_solve;
    const int shape = stage_shape3(g, S.order);
    if (time_scheme == 0) return roeam::launch_stage3(d, S, shape, p ? 8 : 1, p, 1, nullptr, st);
    const int first = time_scheme == 1 ? 1 : 4, nst = time_scheme == 1 ? 3 : 4;
    hipError_t e = hipSuccess;
    for (int k = 0; k < nst && e == hipSuccess; ++k)
        e = roeam::launch_stage3(d, S, shape, first + k, p, k == nst - 1 ? 1 : 0, nullptr, st);
    return e;
}

static roeam_status fill_stats3(roeam_ctx *ctx, const roeam_grid3d *g, roeam_step_stats *stats)
{
    HIP_OK(ctx, hipMemcpyAsync(g->h_slot, g->d_slot, sizeof(Slot), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(ctx, hipStreamSynchronize(ctx->stream));
    const Slot &z = *g->h_slot;
    const roeam::StepState &s = z.st[g->final_parity];
    stats->t = s.t;
    stats->dt_last = z.dt_last;
    stats->max_rate = z.rate_last;
    stats->steps = (long)s.steps;
    stats->nonphys = z.nonphys;
    return z.nonphys ? fail(ctx, ROEAM_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or non-finite)") : ROEAM_OK;
}

extern "C" {

roeam_status roeam_grid3d_destroy(roeam_grid3d *g)
{
    if (!g) return ROEAM_EINVAL;
    g->gc.release();
    if (g->d_qa) (void)hipFree(g->d_qa);
    if (g->d_qb) (void)hipFree(g->d_qb);
    if (g->d_slot) (void)hipFree(g->d_slot);
    if (g->h_slot) (void)hipHostFree(g->h_slot);
    if (g->d_solve) (void)hipFree(g->d_solve);
    if (g->h_solve) (void)hipHostFree(g->h_solve);
    if (g->d_norm_part) (void)hipFree(g->d_norm_part);
    delete g;
    return ROEAM_OK;
}

roeam_status roeam_grid3d_create(roeam_ctx *ctx, int nx, int ny, int nz, double dx, double dy, double dz,
                                 const int bc[6], const double *dirichlet_state, roeam_grid3d **out)
{
    if (!ctx || !out || !bc) return fail(ctx, ROEAM_EINVAL, "NULL argument");
    *out = nullptr;
    if (nx < 2 || ny < 2 || nz < 2) return fail(ctx, ROEAM_EINVAL, "nx, ny and nz must be >= 2");
    if ((long long)nx * ny * nz > (1ll << 31) - 1) return fail(ctx, ROEAM_EINVAL, "grid too large");
    if (!(dx > 0.0) || !(dy > 0.0) || !(dz > 0.0) || !std::isfinite(dx) || !std::isfinite(dy) || !std::isfinite(dz))
        return fail(ctx, ROEAM_EINVAL, "dx, dy, dz must be finite and > 0");
    for (int s = 0; s < 6; ++s)
        if (bc[s] < ROEAM_BC_PERIODIC || bc[s] > ROEAM_BC_DIRICHLET) return fail(ctx, ROEAM_EINVAL, "bad boundary kind");
    for (int a = 0; a < 3; ++a)
        if ((bc[2 * a] == ROEAM_BC_PERIODIC) != (bc[2 * a + 1] == ROEAM_BC_PERIODIC))
            return fail(ctx, ROEAM_EINVAL, "a periodic direction needs periodic kinds on both sides");
    for (int s = 0; s < 6; ++s) {
        if (bc[s] != ROEAM_BC_DIRICHLET) continue;
        if (!dirichlet_state) return fail(ctx, ROEAM_EINVAL, "Dirichlet side without a state");
        const double *Q = dirichlet_state + 5 * s;
        for (int k = 0; k < 5; ++k)
            if (!std::isfinite(Q[k])) return fail(ctx, ROEAM_EINVAL, "non-finite Dirichlet state");
        if (!(Q[0] > 0.0)) return fail(ctx, ROEAM_EINVAL, "Dirichlet density must be > 0");
    }
    HIP_OK(ctx, hipSetDevice(ctx->device));
    roeam_grid3d *g = new (std::nothrow) roeam_grid3d;
    if (!g) return fail(ctx, ROEAM_ENOMEM, "host allocation");
    g->ctx = ctx;
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->pitch = ((long long)nx + 15) & ~15ll;
    g->dx = dx;
    g->dy = dy;
    g->dz = dz;
    for (int s = 0; s < 6; ++s) {
        g->bc[s] = bc[s];
        for (int k = 0; k < 5; ++k) g->bcq[s][k] = bc[s] == ROEAM_BC_DIRICHLET ? dirichlet_state[5 * s + k] : 0.0;
    }
    hipError_t e = hipMalloc(&g->d_slot, sizeof(Slot));
    if (e == hipSuccess) e = hipHostMalloc(&g->h_slot, sizeof(Slot), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&g->d_solve, sizeof(DevSolve3));
    if (e == hipSuccess) e = hipHostMalloc(&g->h_solve, sizeof(DevSolve3), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemset(g->d_slot, 0, sizeof(Slot));
    if (e != hipSuccess) {
        roeam_grid3d_destroy(g);
        return e == hipErrorOutOfMemory ? fail(ctx, ROEAM_ENOMEM, "device allocation") : hip_fail(ctx, e, "grid3d create");
    }
    std::memset(g->h_slot, 0, sizeof(Slot));
    *out = g;
    return ROEAM_OK;
}

roeam_status roeam_grid3d_layout(const roeam_grid3d *g, int *nx, int *ny, int *nz, long *pitch)
{
    if (!g) return ROEAM_EINVAL;
    if (nx) *nx = g->nx;
    if (ny) *ny = g->ny;
    if (nz) *nz = g->nz;
    if (pitch) *pitch = (long)g->pitch;
    return ROEAM_OK;
}

roeam_status roeam_grid3d_set_scalars(roeam_grid3d *g, int nscalars, const double *dirichlet_scalars)
{
    if (!g) return ROEAM_EINVAL;
    roeam_ctx *ctx = g->ctx;
    if (nscalars < 0 || nscalars > ROEAM_MAX_SCALARS)
        return fail(ctx, ROEAM_EINVAL, "nscalars must be 0 .. ROEAM_MAX_SCALARS");
    bool need = false;
    for (int s = 0; s < 6; ++s) need |= g->bc[s] == ROEAM_BC_DIRICHLET;
    if (need && nscalars > 0 && !dirichlet_scalars) return fail(ctx, ROEAM_EINVAL, "Dirichlet side without scalars");
    for (int s = 0; s < 6 && need; ++s)
        for (int m = 0; m < nscalars; ++m)
            if (g->bc[s] == ROEAM_BC_DIRICHLET && !std::isfinite(dirichlet_scalars[s * nscalars + m]))
                return fail(ctx, ROEAM_EINVAL, "non-finite Dirichlet scalar");
    // work queued on the stage buffers may still run: wait before replacing them
    if (g->nsc != nscalars && (g->d_qa || g->d_qb)) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
        if (g->d_qa) (void)hipFree(g->d_qa);
        if (g->d_qb) (void)hipFree(g->d_qb);
        g->d_qa = g->d_qb = nullptr;
    }
    g->nsc = nscalars;
    for (int s = 0; s < 6; ++s)
        for (int m = 0; m < roeam::kMaxScalars; ++m)
            g->bcs[s][m] = (m < nscalars && g->bc[s] == ROEAM_BC_DIRICHLET) ? dirichlet_scalars[s * nscalars + m] : 0.0;
    g->gc.release();
    g->solve_valid = false;
    return ROEAM_OK;
}

roeam_status roeam_grid3d_set_tile_shape(roeam_grid3d *g, int shape)
{
    if (!g || shape < -1 || shape >= roeam::brick_shape_count()) return ROEAM_EINVAL;
    g->shape = shape;
    return ROEAM_OK;
}

roeam_status roeam_grid3d_tile_shape(const roeam_grid3d *g, int order, int *shape)
{
    if (!g || !shape || (order != 1 && order != 2)) return ROEAM_EINVAL;
    *shape = stage_shape3(g, order);
    return ROEAM_OK;
}

roeam_status roeam_residual3d(roeam_ctx *ctx, const roeam_grid3d *gc, const roeam_params *p, const double *q,
                              double *r, double *max_rate_out)
{
    if (!ctx || !gc) return fail(ctx, ROEAM_EINVAL, "NULL context or grid");
    if (!q || !r) return fail(ctx, ROEAM_EINVAL, "q and r must be device pointers");
    if (gc->ctx != ctx) return fail(ctx, ROEAM_EINVAL, "grid belongs to another context");
    roeam_status st = roeam_check_params(ctx, p, false);
    if (st) return st;
    roeam_grid3d *g = const_cast<roeam_grid3d *>(gc);
    HIP_OK(ctx, hipSetDevice(ctx->device));
    const DevSolve3 S = make_solve3(g, p, const_cast<double *>(q));
    hipStream_t s = ctx->stream;
    HIP_OK(ctx, upload_solve3(g, S, s));
    if (max_rate_out) HIP_OK(ctx, roeam::launch_slot_init(g->d_slot, 1, 0.0, 0.0, p->cfl, 0, s));
    HIP_OK(ctx, roeam::launch_stage3(g->d_solve, S, stage_shape3(g, p->order), 0, 0, max_rate_out ? 1 : 0, r, s));
    if (max_rate_out) HIP_OK(ctx, roeam::launch_rate_out(g->d_slot, max_rate_out, s));
    return ROEAM_OK;
}

roeam_status roeam_step3d(roeam_ctx *ctx, const roeam_grid3d *gc, const roeam_params *p, double *q, long nsteps,
                          double t0, double t_end, roeam_step_stats *stats)
{
    if (!ctx || !gc) return fail(ctx, ROEAM_EINVAL, "NULL context or grid");
    if (!q) return fail(ctx, ROEAM_EINVAL, "q must be a device pointer");
    if (nsteps < 0) return fail(ctx, ROEAM_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(t0) || !std::isfinite(t_end)) return fail(ctx, ROEAM_EINVAL, "non-finite time");
    if (gc->ctx != ctx) return fail(ctx, ROEAM_EINVAL, "grid belongs to another context");
    roeam_status st = roeam_check_params(ctx, p, true);
    if (st) return st;
    roeam_grid3d *g = const_cast<roeam_grid3d *>(gc);
    HIP_OK(ctx, hipSetDevice(ctx->device));
    if ((st = ensure_stage_buffers3(ctx, g))) return st;
    const DevSolve3 S = make_solve3(g, p, q);
    hipStream_t s = ctx->stream;
    HIP_OK(ctx, upload_solve3(g, S, s));
    // the slot holds t, t_end and the step budget: one captured graph of an
    // even number of steps serves any nsteps (steps past the budget are inactive)
    HIP_OK(ctx, roeam::launch_slot_init(g->d_slot, 1, t0, t_end, p->cfl, nsteps, s));
    HIP_OK(ctx, roeam::launch_rate3(g->d_solve, S, 0, s));
    const bool use_graph = s != nullptr && nsteps > 1;
    long launched = 0;
    if (!use_graph) {
        for (long k = 0; k < nsteps; ++k) HIP_OK(ctx, enqueue_step3(g, S, p->time_scheme, (int)(k & 1), s));
        launched = nsteps;
    } else {
        int chunk = (int)(nsteps < kStepsPerGraph ? nsteps : kStepsPerGraph);
        chunk += chunk & 1;
        GraphCache &G = g->gc;
        if (!G.valid || G.q != q || G.stream != s || G.chunk != chunk || G.shape != stage_shape3(g, p->order) ||
            std::memcmp(&G.params, p, sizeof *p) != 0) {
            G.release();
            HIP_OK(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
            hipError_t e = hipSuccess;
            for (int k = 0; k < chunk && e == hipSuccess; ++k) e = enqueue_step3(g, S, p->time_scheme, k & 1, s);
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(s, &graph);
            if (e != hipSuccess) return hip_fail(ctx, e, "capture step");
            if (e2 != hipSuccess) return hip_fail(ctx, e2, "hipStreamEndCapture");
            G.graph = graph;
            HIP_OK(ctx, hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0));
            G.valid = true;
            G.q = q;
            G.stream = s;
            G.chunk = chunk;
            G.shape = stage_shape3(g, p->order);
            G.params = *p;
        }
        const long launches = (nsteps + chunk - 1) / chunk;
        for (long k = 0; k < launches; ++k) {
            HIP_OK(ctx, hipGraphLaunch(G.exec, s));
            launched += chunk;
            if (t_end > 0.0 && (k & 1)) {
                HIP_OK(ctx, hipMemcpyAsync(g->h_slot, g->d_slot, sizeof(Slot), hipMemcpyDeviceToHost, s));
                HIP_OK(ctx, hipStreamSynchronize(s));
                const Slot &z = *g->h_slot;
                if (z.nonphys || z.st[0].t >= t_end || z.st[0].steps >= nsteps) break;
            }
        }
    }
    g->final_parity = (int)(launched & 1);
    if (p->time_scheme == 0) HIP_OK(ctx, roeam::launch_fe_finish3(g->d_solve, S, g->final_parity, s));
    if (stats) return fill_stats3(ctx, g, stats);
    return ROEAM_OK;
}

roeam_status roeam_residual_norms3d(roeam_ctx *ctx, const roeam_grid3d *gc, const double *r, double *norms_out)
{
    if (!ctx || !gc || !r || !norms_out) return fail(ctx, ROEAM_EINVAL, "NULL argument");
    if (gc->ctx != ctx) return fail(ctx, ROEAM_EINVAL, "grid belongs to another context");
    roeam_grid3d *g = const_cast<roeam_grid3d *>(gc);
    HIP_OK(ctx, hipSetDevice(ctx->device));
    if (!g->d_norm_part)
        HIP_OK(ctx, hipMalloc(&g->d_norm_part, sizeof(double) * 2 * (5 + roeam::kMaxScalars) * roeam::kNormMaxBlocks));
    HIP_OK(ctx, roeam::launch_norms(r, 5 + g->nsc, (long long)g->nz * g->ny * g->pitch, g->nx, g->ny * g->nz, g->pitch,
                                    g->d_norm_part, roeam::kNormMaxBlocks, norms_out, ctx->stream));
    return ROEAM_OK;
}

roeam_status roeam_last_stats3d(roeam_ctx *ctx, const roeam_grid3d *g, roeam_step_stats *stats)
{
    if (!ctx || !g || !stats) return fail(ctx, ROEAM_EINVAL, "NULL argument");
    return fill_stats3(ctx, g, stats);
}

} // extern "C"

// roeam_runtime.hip -- host side of the C ABI in include/roeam.h: contexts,
// immutable grids, the tile-shape autotuner, the residual call and the
// graph-captured step loop (the batch engine is in roeam_batch.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "roeam_host.hpp"

roeam_status roeam_fail(roeam_ctx *ctx, roeam_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

static roeam_status fail(roeam_ctx *ctx, roeam_status st, const std::string &msg) { return roeam_fail(ctx, st, msg); }

static roeam_status hip_fail(roeam_ctx *ctx, hipError_t e, const char *where)
{
    return fail(ctx, ROEAM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_OK(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

roeam_status roeam_check_params(roeam_ctx *ctx, const roeam_params *p, bool need_cfl)
{
    if (!p) return fail(ctx, ROEAM_EINVAL, "params is NULL");
    if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return fail(ctx, ROEAM_EINVAL, "gamma must be > 1");
    if (need_cfl && !(p->cfl > 0.0 && std::isfinite(p->cfl))) return fail(ctx, ROEAM_EINVAL, "cfl must be > 0");
    if (!(p->mach_ref > 0.0) || !std::isfinite(p->mach_ref))
        return fail(ctx, ROEAM_EINVAL, "mach_ref must be > 0 (theta of Eq. 101 divides dU_p)");
    if (!(p->u_ref >= 0.0) || !std::isfinite(p->u_ref)) return fail(ctx, ROEAM_EINVAL, "u_ref must be >= 0");
    if (p->eps1 != 0.0 && p->eps1 != 1.0) return fail(ctx, ROEAM_EINVAL, "eps1 must be 0 or 1 (Eq. 111)");
    if (!(p->eps2 >= 0.0) || !std::isfinite(p->eps2)) return fail(ctx, ROEAM_EINVAL, "eps2 must be >= 0");
    if (p->s1_mode != 0 && p->s1_mode != 1) return fail(ctx, ROEAM_EINVAL, "s1_mode must be 0 or 1");
    if (p->order != 1 && p->order != 2) return fail(ctx, ROEAM_EINVAL, "order must be 1 or 2");
    if (p->time_scheme < 0 || p->time_scheme > 2) return fail(ctx, ROEAM_EINVAL, "time_scheme must be 0, 1 or 2");
    if (p->precision != 0 && p->precision != 1) return fail(ctx, ROEAM_EINVAL, "precision must be 0 or 1");
    if (p->variant & ~ROEAM_V_SUPPORTED) return fail(ctx, ROEAM_EINVAL, "unsupported variant bits");
    if (p->scheme != ROEAM_SCHEME_ROEAM && p->scheme != ROEAM_SCHEME_ROE && p->scheme != ROEAM_SCHEME_ROE_HARTEN)
        return fail(ctx, ROEAM_EINVAL, "scheme must be ROEAM_SCHEME_ROEAM, _ROE or _ROE_HARTEN");
    if (!(p->eps_lambda >= 0.0) || !std::isfinite(p->eps_lambda))
        return fail(ctx, ROEAM_EINVAL, "eps_lambda must be >= 0 (Eq. 115)");
    return ROEAM_OK;
}

static void prim_of(double gamma, const double Q[4], double W[4])
{
    double rho = Q[0], u = Q[1] / rho, v = Q[2] / rho;
    W[0] = rho;
    W[1] = u;
    W[2] = v;
    W[3] = (gamma - 1.0) * (Q[3] - 0.5 * rho * (u * u + v * v));
}

DevSolve roeam_make_solve(const roeam_grid *g, const roeam_params *p, double *q, double *qa, double *qb, Slot *slot)
{
    DevSolve S;
    std::memset(&S, 0, sizeof S);
    S.nx = g->nx;
    S.ny = g->ny;
    S.pitch = g->pitch;
    S.plane = (long long)g->ny * g->pitch;
    S.metric = g->metric;
    S.dx = g->dx;
    S.dy = g->dy;
    S.area = g->dx * g->dy;
    S.xn = g->d_xn;
    S.yn = g->d_yn;
    for (int s = 0; s < 4; ++s) {
        S.bc[s] = g->bc[s];
        prim_of(p->gamma, g->bcq[s], S.bcw[s]);
    }
    for (int s = 0; s < 4; ++s) {
        S.spl_a[s] = g->spl_a[s];
        S.spl_b[s] = g->spl_b[s];
        S.spl_hi[s] = g->spl_hi[s];
        S.spl_lo[s] = g->spl_lo[s];
        if (g->bc[s] == ROEAM_BC_MOVING && g->spl_hi[s] == ROEAM_BC_DIRICHLET) prim_of(p->gamma, g->bcq_hi[s], S.bcw_hi[s]);
    }
    S.t_res = g->t_res;
    S.nsc = g->nsc;
    for (int s = 0; s < 4; ++s)
        for (int m = 0; m < g->nsc; ++m)
            S.bck[s][m] = (g->bc[s] == ROEAM_BC_DIRICHLET || g->bc[s] == ROEAM_BC_MOVING) ? g->bcs[s][m] / g->bcq[s][0] : 0.0;
    S.gamma = p->gamma;
    S.gm1 = p->gamma - 1.0;
    S.g_gm1 = p->gamma / (p->gamma - 1.0);
    S.igm1 = 1.0 / (p->gamma - 1.0);
    S.mr2 = p->mach_ref * p->mach_ref;
    S.u_ref = p->u_ref;
    S.dv_min2 = (1e-5 * p->u_ref) * (1e-5 * p->u_ref);
    S.inv_area = g->metric == 0 ? 1.0 / (g->dx * g->dy) : 0.0;
    S.eps1 = p->eps1;
    S.eps2 = p->eps2;
    S.cfl = p->cfl;
    S.s1_mode = p->s1_mode;
    S.order = p->order;
    S.precision = p->precision;
    S.variant = p->variant;
    S.scheme = p->scheme;
    S.eps_lambda = p->eps_lambda;
    S.q = q;
    S.qa = qa;
    S.qb = qb;
    S.slot = slot;
    return S;
}

static roeam_status check_params(roeam_ctx *ctx, const roeam_params *p, bool need_cfl)
{
    return roeam_check_params(ctx, p, need_cfl);
}

static DevSolve make_solve(const roeam_grid *g, const roeam_params *p, double *q)
{
    return roeam_make_solve(g, p, q, g->d_qa, g->d_qb, g->d_slot);
}

// The grid's own stage buffers are allocated at its first single-grid step
// (batched solves keep theirs in the batch arena).
static roeam_status ensure_stage_buffers(roeam_ctx *ctx, roeam_grid *g)
{
    if (g->d_qa && g->d_qb) return ROEAM_OK;
    const size_t bytes = sizeof(double) * (4 + (size_t)g->nsc) * (size_t)g->ny * (size_t)g->pitch;
    hipError_t e = g->d_qa ? hipSuccess : hipMalloc(&g->d_qa, bytes);
    if (e == hipSuccess && !g->d_qb) e = hipMalloc(&g->d_qb, bytes);
    if (e != hipSuccess)
        return roeam_fail(ctx, e == hipErrorOutOfMemory ? ROEAM_ENOMEM : ROEAM_EDEVICE,
                          std::string("stage buffers: ") + hipGetErrorString(e));
    g->solve_valid = false;
    return ROEAM_OK;
}

// Make the grid's device descriptor equal to S.  Work already queued may
// still read the old descriptor, so a change waits for the stream first.
static hipError_t upload_solve(roeam_grid *g, const DevSolve &S, hipStream_t s)
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

extern "C" {

roeam_status roeam_ctx_create(int device, void *hip_stream, roeam_ctx **out)
{
    if (!out) return ROEAM_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return ROEAM_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return ROEAM_EDEVICE;
    if (roeam::scratch_setup(device) != hipSuccess) return ROEAM_EDEVICE;
    roeam_ctx *c = new (std::nothrow) roeam_ctx;
    if (!c) return ROEAM_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return ROEAM_OK;
}

void roeam_batch_release(roeam_ctx *ctx);  // defined with the batch engine

roeam_status roeam_ctx_destroy(roeam_ctx *ctx)
{
    if (!ctx) return ROEAM_EINVAL;
    roeam_batch_release(ctx);
    delete ctx;
    return ROEAM_OK;
}

roeam_status roeam_ctx_set_stream(roeam_ctx *ctx, void *hip_stream)
{
    if (!ctx) return ROEAM_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return ROEAM_OK;
}

const char *roeam_last_error(const roeam_ctx *ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

roeam_status roeam_grid_destroy(roeam_grid *g)
{
    if (!g) return ROEAM_EINVAL;
    g->gc.release();
    if (g->d_xn) (void)hipFree(g->d_xn);
    if (g->d_yn) (void)hipFree(g->d_yn);
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

roeam_status roeam_grid_create(roeam_ctx *ctx, int nx, int ny, const roeam_metrics *m, const int bc[4],
                               const double *dirichlet_state, roeam_grid **out)
{
    if (!ctx || !out || !m || !bc) return fail(ctx, ROEAM_EINVAL, "NULL argument");
    *out = nullptr;
    if (nx < 2 || ny < 2) return fail(ctx, ROEAM_EINVAL, "nx and ny must be >= 2");
    if ((long long)nx * ny > (1ll << 31) - 1) return fail(ctx, ROEAM_EINVAL, "grid too large");
    for (int s = 0; s < 4; ++s)
        if (bc[s] < ROEAM_BC_PERIODIC || bc[s] > ROEAM_BC_MOVING) return fail(ctx, ROEAM_EINVAL, "bad boundary kind");
    for (int s = 0; s < 4; ++s)
        if (bc[s] == ROEAM_BC_MOVING && (m->kind != 0 || bc[s ^ 1] == ROEAM_BC_PERIODIC))
            return fail(ctx, ROEAM_EINVAL, "a moving side needs a uniform grid and a non-periodic opposite side");
    if ((bc[0] == ROEAM_BC_PERIODIC) != (bc[1] == ROEAM_BC_PERIODIC) ||
        (bc[2] == ROEAM_BC_PERIODIC) != (bc[3] == ROEAM_BC_PERIODIC))
        return fail(ctx, ROEAM_EINVAL, "a periodic direction needs periodic kinds on both sides");
    bool need_dir = false;
    for (int s = 0; s < 4; ++s) need_dir |= bc[s] == ROEAM_BC_DIRICHLET || bc[s] == ROEAM_BC_MOVING;
    if (need_dir && !dirichlet_state) return fail(ctx, ROEAM_EINVAL, "Dirichlet side without a state");
    if (m->kind == 0) {
        if (!(m->dx > 0.0) || !(m->dy > 0.0)) return fail(ctx, ROEAM_EINVAL, "dx, dy must be > 0");
    } else if (m->kind == 1) {
        if (!m->xn || !m->yn) return fail(ctx, ROEAM_EINVAL, "node arrays are NULL");
        const long long nxn = nx + 1;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const double *x = m->xn, *y = m->yn;
                long long r0 = (long long)j * nxn, r1 = r0 + nxn;
                double a = 0.5 * ((x[r1 + i + 1] - x[r0 + i]) * (y[r1 + i] - y[r0 + i + 1]) -
                                  (x[r1 + i] - x[r0 + i + 1]) * (y[r1 + i + 1] - y[r0 + i]));
                if (!(a > 0.0)) return fail(ctx, ROEAM_EINVAL, "non-positive cell area in node grid");
            }
    } else {
        return fail(ctx, ROEAM_EINVAL, "metrics kind must be 0 or 1");
    }
    if (need_dir) {
        for (int s = 0; s < 4; ++s) {
            if (bc[s] != ROEAM_BC_DIRICHLET && bc[s] != ROEAM_BC_MOVING) continue;
            const double *Q = dirichlet_state + 4 * s;
            if (!(Q[0] > 0.0)) return fail(ctx, ROEAM_EINVAL, "Dirichlet density must be > 0");
            for (int k = 0; k < 4; ++k)
                if (!std::isfinite(Q[k])) return fail(ctx, ROEAM_EINVAL, "non-finite Dirichlet state");
        }
    }
    HIP_OK(ctx, hipSetDevice(ctx->device));
    roeam_grid *g = new (std::nothrow) roeam_grid;
    if (!g) return fail(ctx, ROEAM_ENOMEM, "host allocation");
    g->ctx = ctx;
    g->nx = nx;
    g->ny = ny;
    g->pitch = ((long long)nx + 15) & ~15ll;
    g->metric = m->kind;
    g->dx = m->kind == 0 ? m->dx : 0.0;
    g->dy = m->kind == 0 ? m->dy : 0.0;
    for (int s = 0; s < 4; ++s) {
        g->bc[s] = bc[s];
        for (int k = 0; k < 4; ++k)
            g->bcq[s][k] = (bc[s] == ROEAM_BC_DIRICHLET || bc[s] == ROEAM_BC_MOVING) ? dirichlet_state[4 * s + k] : 0.0;
    }
    hipError_t e = hipMalloc(&g->d_slot, sizeof(Slot));
    if (e == hipSuccess) e = hipHostMalloc(&g->h_slot, sizeof(Slot), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&g->d_solve, sizeof(DevSolve));
    if (e == hipSuccess) e = hipHostMalloc(&g->h_solve, sizeof(DevSolve), hipHostMallocDefault);
    if (e == hipSuccess && m->kind == 1) {
        const size_t nb = sizeof(double) * (size_t)(nx + 1) * (size_t)(ny + 1);
        e = hipMalloc(&g->d_xn, nb);
        if (e == hipSuccess) e = hipMalloc(&g->d_yn, nb);
        if (e == hipSuccess) e = hipMemcpy(g->d_xn, m->xn, nb, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(g->d_yn, m->yn, nb, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(g->d_slot, 0, sizeof(Slot));
    if (e != hipSuccess) {
        roeam_grid_destroy(g);
        return e == hipErrorOutOfMemory ? fail(ctx, ROEAM_ENOMEM, "device allocation") : hip_fail(ctx, e, "grid create");
    }
    std::memset(g->h_slot, 0, sizeof(Slot));
    *out = g;
    return ROEAM_OK;
}

roeam_status roeam_grid_layout(const roeam_grid *g, int *nx, int *ny, long *pitch)
{
    if (!g) return ROEAM_EINVAL;
    if (nx) *nx = g->nx;
    if (ny) *ny = g->ny;
    if (pitch) *pitch = (long)g->pitch;
    return ROEAM_OK;
}

// Tile shape for a grid: the caller's choice, else the autotuned one.  The
// autotuner times the first-stage kernel of every shape on the grid (stage 1
// only reads q and writes the grid's own stage buffer, so it leaves q
// untouched) and keeps the fastest, per (order, precision), in the grid and in
// a process-wide table keyed by device and grid size (guarded by a mutex:
// contexts on different host threads may tune at the same time).
struct TuneKey {
    int device, nx, ny, order, precision, metric, nsc;
    bool operator==(const TuneKey &o) const
    {
        return device == o.device && nx == o.nx && ny == o.ny && order == o.order && precision == o.precision &&
               metric == o.metric && nsc == o.nsc;
    }
};
struct TuneKeyHash {
    size_t operator()(const TuneKey &k) const
    {
        return ((size_t)k.nx * 1000003u) ^ ((size_t)k.ny * 7919u) ^
               (size_t)(k.device * 131 + k.order * 31 + k.precision * 7 + k.metric + k.nsc * 1009);
    }
};
static std::unordered_map<TuneKey, int, TuneKeyHash> g_tuned;
static std::mutex g_tuned_mu;

// Two timing events, destroyed on every return path.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

static roeam_status choose_shape(roeam_ctx *ctx, roeam_grid *g, const roeam_params *p, const DevSolve &S, int *shape)
{
    if (g->shape_forced >= 0) {
        *shape = g->shape_forced;
        return ROEAM_OK;
    }
    int &cached = g->shape_tuned[p->order - 1][p->precision];
    if (cached >= 0) {
        *shape = cached;
        return ROEAM_OK;
    }
    const TuneKey key{ctx->device, g->nx, g->ny, p->order, p->precision, g->metric, g->nsc};
    {
        std::lock_guard<std::mutex> lk(g_tuned_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            cached = it->second;
            *shape = cached;
            return ROEAM_OK;
        }
    }
    hipStream_t s = ctx->stream;
    EventPair ev;
    HIP_OK(ctx, hipEventCreate(&ev.a));
    HIP_OK(ctx, hipEventCreate(&ev.b));
    hipEvent_t e0 = ev.a, e1 = ev.b;
    HIP_OK(ctx, roeam::launch_slot_init(g->d_slot, 1, 0.0, 0.0, p->cfl, 1, s));
    HIP_OK(ctx, roeam::launch_rate(S, 0, s));
    // each shape: a warm-up launch, then the best of three timed rounds of
    // four launches (a single round misranks shapes within a few percent of
    // each other often enough to matter)
    int best = 0;
    float best_ms = 1e30f;
    const int reps = 4, rounds = 3;
    for (int sh = 0; sh < roeam::tile_shape_count(); ++sh) {
        HIP_OK(ctx, roeam::launch_stage_single(g->d_solve, S, sh, 1, 0, 0, nullptr, s));  // warm-up
        float shape_ms = 1e30f;
        for (int round = 0; round < rounds; ++round) {
            HIP_OK(ctx, hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r)
                HIP_OK(ctx, roeam::launch_stage_single(g->d_solve, S, sh, 1, 0, 0, nullptr, s));
            HIP_OK(ctx, hipEventRecord(e1, s));
            HIP_OK(ctx, hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_OK(ctx, hipEventElapsedTime(&ms, e0, e1));
            shape_ms = ms < shape_ms ? ms : shape_ms;
        }
        if (shape_ms < best_ms) {
            best_ms = shape_ms;
            best = sh;
        }
    }
    cached = best;
    {
        std::lock_guard<std::mutex> lk(g_tuned_mu);
        g_tuned[key] = best;
    }
    *shape = best;
    return ROEAM_OK;
}

roeam_status roeam_residual(roeam_ctx *ctx, const roeam_grid *g, const roeam_params *p, const double *q, double *r,
                            double *max_rate_out)
{
    if (!ctx || !g) return fail(ctx, ROEAM_EINVAL, "NULL context or grid");
    if (!q || !r) return fail(ctx, ROEAM_EINVAL, "q and r must be device pointers");
    if (g->ctx != ctx) return fail(ctx, ROEAM_EINVAL, "grid belongs to another context");
    roeam_status st = check_params(ctx, p, false);
    if (st) return st;
    HIP_OK(ctx, hipSetDevice(ctx->device));
    DevSolve S = make_solve(g, p, const_cast<double *>(q));
    // the caller's shape, else the one tuned for these parameters, else
    // 16x15/256 (the fastest from 512^2 up); every shape gives the same bits
    const int tuned = g->shape_tuned[p->order - 1][p->precision];
    const int shape = g->shape_forced >= 0 ? g->shape_forced : (tuned >= 0 ? tuned : 6);
    roeam_grid *gm = const_cast<roeam_grid *>(g);
    HIP_OK(ctx, upload_solve(gm, S, ctx->stream));
    if (max_rate_out) HIP_OK(ctx, roeam::launch_slot_init(g->d_slot, 1, 0.0, 0.0, p->cfl, 0, ctx->stream));
    HIP_OK(ctx, roeam::launch_stage_single(g->d_solve, S, shape, 0, 0, max_rate_out ? 1 : 0, r, ctx->stream));
    if (max_rate_out) HIP_OK(ctx, roeam::launch_rate_out(g->d_slot, max_rate_out, ctx->stream));
    return ROEAM_OK;
}

// One time step with parity p: one kernel per stage (the first stage also
// sets dt); forward Euler goes q -> qa on even and qa -> q on odd steps.
static hipError_t enqueue_step(const roeam_grid *g, const DevSolve &S, int shape, int time_scheme, int p,
                               hipStream_t st)
{
    hipError_t e;
    const DevSolve *d = g->d_solve;
    if (time_scheme == 0) return roeam::launch_stage_single(d, S, shape, p ? 8 : 1, p, 1, nullptr, st);
    // stage codes 1-3 (SSP-RK3) or 4-7 (four-stage scheme)
    const int first = time_scheme == 1 ? 1 : 4, nst = time_scheme == 1 ? 3 : 4;
    e = hipSuccess;
    for (int k = 0; k < nst && e == hipSuccess; ++k)
        e = roeam::launch_stage_single(d, S, shape, first + k, p, k == nst - 1 ? 1 : 0, nullptr, st);
    return e;
}

static roeam_status fill_stats(roeam_ctx *ctx, const roeam_grid *g, roeam_step_stats *stats)
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

roeam_status roeam_step(roeam_ctx *ctx, const roeam_grid *gc, const roeam_params *p, double *q, long nsteps,
                        double t0, double t_end, roeam_step_stats *stats)
{
    if (!ctx || !gc) return fail(ctx, ROEAM_EINVAL, "NULL context or grid");
    if (!q) return fail(ctx, ROEAM_EINVAL, "q must be a device pointer");
    if (nsteps < 0) return fail(ctx, ROEAM_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(t0) || !std::isfinite(t_end)) return fail(ctx, ROEAM_EINVAL, "non-finite time");
    if (gc->ctx != ctx) return fail(ctx, ROEAM_EINVAL, "grid belongs to another context");
    roeam_status st = check_params(ctx, p, true);
    if (st) return st;
    roeam_grid *g = const_cast<roeam_grid *>(gc);
    HIP_OK(ctx, hipSetDevice(ctx->device));
    if ((st = ensure_stage_buffers(ctx, g))) return st;
    const DevSolve S = make_solve(g, p, q);
    hipStream_t s = ctx->stream;
    HIP_OK(ctx, upload_solve(g, S, s));
    int shape = 0;
    st = choose_shape(ctx, g, p, S, &shape);
    if (st) return st;
    // The slot holds t, t_end and the step budget, so one captured graph of
    // an even number of steps serves any nsteps: steps past the budget or
    // past t_end are inactive and their kernels exit at once.
    HIP_OK(ctx, roeam::launch_slot_init(g->d_slot, 1, t0, t_end, p->cfl, nsteps, s));
    HIP_OK(ctx, roeam::launch_rate(S, 0, s));
    const bool use_graph = s != nullptr && nsteps > 1;
    long launched = 0;
    if (!use_graph) {
        for (long k = 0; k < nsteps; ++k) HIP_OK(ctx, enqueue_step(g, S, shape, p->time_scheme, (int)(k & 1), s));
        launched = nsteps;
    } else {
        int chunk = (int)(nsteps < kStepsPerGraph ? nsteps : kStepsPerGraph);
        chunk += chunk & 1;  // even: every launch of the graph starts at parity 0
        GraphCache &G = g->gc;
        // the graph's kernels read q and every parameter from the grid's device
        // descriptor; it depends only on the stream, its length, the tile shape
        // and what selects the kernels and stages
        if (!G.valid || G.stream != s || G.chunk != chunk || G.shape != shape || G.params.order != p->order ||
            G.params.precision != p->precision || G.params.time_scheme != p->time_scheme) {
            G.release();
            HIP_OK(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
            hipError_t e = hipSuccess;
            for (int k = 0; k < chunk && e == hipSuccess; ++k) e = enqueue_step(g, S, shape, p->time_scheme, k & 1, s);
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
            G.shape = shape;
            G.params = *p;
        }
        const long launches = (nsteps + chunk - 1) / chunk;
        for (long k = 0; k < launches; ++k) {
            HIP_OK(ctx, hipGraphLaunch(G.exec, s));
            launched += chunk;
            if (t_end > 0.0 && (k & 1)) {
                // stop launching once the run has reached t_end
                HIP_OK(ctx, hipMemcpyAsync(g->h_slot, g->d_slot, sizeof(Slot), hipMemcpyDeviceToHost, s));
                HIP_OK(ctx, hipStreamSynchronize(s));
                const Slot &z = *g->h_slot;
                if (z.nonphys || z.st[0].t >= t_end || z.st[0].steps >= nsteps) break;
            }
        }
    }
    g->final_parity = (int)(launched & 1);
    if (p->time_scheme == 0) HIP_OK(ctx, roeam::launch_fe_finish(S, g->final_parity, s));
    if (stats) return fill_stats(ctx, g, stats);
    return ROEAM_OK;
}

roeam_status roeam_profile_step(roeam_ctx *ctx, const roeam_grid *gc, const roeam_params *p, double *q, long nsteps,
                                double t0, double stage_ms[4], long *launches)
{
    if (!ctx || !gc || !q || !stage_ms || nsteps < 1) return fail(ctx, ROEAM_EINVAL, "bad argument");
    if (gc->ctx != ctx) return fail(ctx, ROEAM_EINVAL, "grid belongs to another context");
    roeam_status st = check_params(ctx, p, true);
    if (st) return st;
    roeam_grid *g = const_cast<roeam_grid *>(gc);
    HIP_OK(ctx, hipSetDevice(ctx->device));
    if ((st = ensure_stage_buffers(ctx, g))) return st;
    const DevSolve S = make_solve(g, p, q);
    hipStream_t s = ctx->stream;
    HIP_OK(ctx, upload_solve(g, S, s));
    int shape = 0;
    st = choose_shape(ctx, g, p, S, &shape);
    if (st) return st;
    const int nst = p->time_scheme == 0 ? 1 : (p->time_scheme == 1 ? 3 : 4);
    const int first = p->time_scheme == 2 ? 4 : 1;
    std::vector<hipEvent_t> ev((size_t)(2 * nst * nsteps));
    for (auto &e : ev) HIP_OK(ctx, hipEventCreate(&e));
    roeam_status rc = ROEAM_OK;
    hipError_t e = roeam::launch_slot_init(g->d_slot, 1, t0, 0.0, p->cfl, nsteps, s);
    if (e == hipSuccess) e = roeam::launch_rate(S, 0, s);
    for (long k = 0; k < nsteps && e == hipSuccess; ++k) {
        const int par = (int)(k & 1);
        for (int stg = 1; stg <= nst && e == hipSuccess; ++stg) {
            hipEvent_t *pair = &ev[(size_t)(2 * (k * nst + stg - 1))];
            e = hipEventRecord(pair[0], s);
            const int code = nst == 1 && par ? 8 : first + stg - 1;
            if (e == hipSuccess)
                e = roeam::launch_stage_single(g->d_solve, S, shape, code, par, stg == nst ? 1 : 0, nullptr, s);
            if (e == hipSuccess) e = hipEventRecord(pair[1], s);
        }
    }
    g->final_parity = (int)(nsteps & 1);
    if (e == hipSuccess && nst == 1) e = roeam::launch_fe_finish(S, g->final_parity, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(ctx, e, "profile step");
    double sum[4] = {0, 0, 0, 0};
    for (long k = 0; k < nsteps && rc == ROEAM_OK; ++k)
        for (int stg = 0; stg < nst; ++stg) {
            float ms = 0.f;
            hipEvent_t *pair = &ev[(size_t)(2 * (k * nst + stg))];
            if (hipEventElapsedTime(&ms, pair[0], pair[1]) == hipSuccess) sum[stg] += ms;
        }
    for (auto &x : ev) (void)hipEventDestroy(x);
    for (int stg = 0; stg < 4; ++stg) stage_ms[stg] = stg < nst ? sum[stg] / (double)nsteps : 0.0;
    if (launches) *launches = nsteps * nst;
    return rc;
}

roeam_status roeam_grid_set_scalars(roeam_grid *g, int nscalars, const double *dirichlet_scalars)
{
    if (!g) return ROEAM_EINVAL;
    roeam_ctx *ctx = g->ctx;
    if (nscalars < 0 || nscalars > ROEAM_MAX_SCALARS)
        return fail(ctx, ROEAM_EINVAL, "nscalars must be 0 .. ROEAM_MAX_SCALARS");
    bool need = false;
    for (int s = 0; s < 4; ++s) need |= g->bc[s] == ROEAM_BC_DIRICHLET || g->bc[s] == ROEAM_BC_MOVING;
    if (need && nscalars > 0 && !dirichlet_scalars) return fail(ctx, ROEAM_EINVAL, "Dirichlet side without scalars");
    for (int s = 0; s < 4 && need; ++s)
        for (int m = 0; m < nscalars; ++m)
            if ((g->bc[s] == ROEAM_BC_DIRICHLET || g->bc[s] == ROEAM_BC_MOVING) &&
                !std::isfinite(dirichlet_scalars[s * nscalars + m]))
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
    for (int s = 0; s < 4; ++s)
        for (int m = 0; m < roeam::kMaxScalars; ++m)
            g->bcs[s][m] = (m < nscalars && (g->bc[s] == ROEAM_BC_DIRICHLET || g->bc[s] == ROEAM_BC_MOVING))
                               ? dirichlet_scalars[s * nscalars + m]
                               : 0.0;
    g->gc.release();
    g->solve_valid = false;
    for (auto &row : g->shape_tuned) row[0] = row[1] = -1;
    return ROEAM_OK;
}

roeam_status roeam_grid_set_moving_side(roeam_grid *g, int side, double a, double b, int lo_kind, int hi_kind,
                                        const double *state_hi)
{
    if (!g) return ROEAM_EINVAL;
    roeam_ctx *ctx = g->ctx;
    if (side < 0 || side > 3 || g->bc[side] != ROEAM_BC_MOVING)
        return fail(ctx, ROEAM_EINVAL, "side is not a ROEAM_BC_MOVING side of this grid");
    if (std::isnan(a) || !std::isfinite(b)) return fail(ctx, ROEAM_EINVAL, "split a must not be NaN, b must be finite");
    if (hi_kind != ROEAM_BC_SLIPWALL && hi_kind != ROEAM_BC_DIRICHLET)
        return fail(ctx, ROEAM_EINVAL, "hi_kind must be ROEAM_BC_SLIPWALL or ROEAM_BC_DIRICHLET");
    if (lo_kind != ROEAM_BC_SLIPWALL && lo_kind != ROEAM_BC_DIRICHLET)
        return fail(ctx, ROEAM_EINVAL, "lo_kind must be ROEAM_BC_SLIPWALL or ROEAM_BC_DIRICHLET");
    if (hi_kind == ROEAM_BC_DIRICHLET) {
        if (!state_hi) return fail(ctx, ROEAM_EINVAL, "Dirichlet hi side without a state");
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(state_hi[k])) return fail(ctx, ROEAM_EINVAL, "non-finite state");
        if (!(state_hi[0] > 0.0)) return fail(ctx, ROEAM_EINVAL, "Dirichlet density must be > 0");
    }
    g->spl_a[side] = a;
    g->spl_b[side] = b;
    g->spl_hi[side] = hi_kind;
    g->spl_lo[side] = lo_kind;
    for (int k = 0; k < 4; ++k) g->bcq_hi[side][k] = hi_kind == ROEAM_BC_DIRICHLET ? state_hi[k] : 0.0;
    return ROEAM_OK;
}

roeam_status roeam_grid_set_boundary_time(roeam_grid *g, double t)
{
    if (!g || !std::isfinite(t)) return ROEAM_EINVAL;
    g->t_res = t;
    return ROEAM_OK;
}

roeam_status roeam_grid_set_tile_shape(roeam_grid *g, int shape)
{
    if (!g || shape < -1 || shape >= roeam::tile_shape_count()) return ROEAM_EINVAL;
    g->shape_forced = shape;
    return ROEAM_OK;
}

roeam_status roeam_grid_tile_shape(const roeam_grid *g, const roeam_params *p, int *shape)
{
    if (!g || !p || !shape || (p->order != 1 && p->order != 2) || (p->precision != 0 && p->precision != 1))
        return ROEAM_EINVAL;
    *shape = g->shape_forced >= 0 ? g->shape_forced : g->shape_tuned[p->order - 1][p->precision];
    return ROEAM_OK;
}

roeam_status roeam_residual_norms(roeam_ctx *ctx, const roeam_grid *gc, const double *r, double *norms_out)
{
    if (!ctx || !gc || !r || !norms_out) return fail(ctx, ROEAM_EINVAL, "NULL argument");
    if (gc->ctx != ctx) return fail(ctx, ROEAM_EINVAL, "grid belongs to another context");
    roeam_grid *g = const_cast<roeam_grid *>(gc);
    HIP_OK(ctx, hipSetDevice(ctx->device));
    if (!g->d_norm_part)
        HIP_OK(ctx, hipMalloc(&g->d_norm_part, sizeof(double) * 2 * (4 + roeam::kMaxScalars) * roeam::kNormMaxBlocks));
    HIP_OK(ctx, roeam::launch_norms(r, 4 + g->nsc, (long long)g->ny * g->pitch, g->nx, g->ny, g->pitch, g->d_norm_part,
                                    roeam::kNormMaxBlocks, norms_out, ctx->stream));
    return ROEAM_OK;
}

roeam_status roeam_last_stats(roeam_ctx *ctx, const roeam_grid *g, roeam_step_stats *stats)
{
    if (!ctx || !g || !stats) return fail(ctx, ROEAM_EINVAL, "NULL argument");
    return fill_stats(ctx, g, stats);
}

} // extern "C"

// roeam_batch.hip -- the continuous-batching engine behind roeam_batch_*.
//
// Resident solves keep three state copies (q, qa, qb) in a device arena and a
// Slot each.  A scheduler iteration advances every resident solve by one
// time step: per group of solves sharing (order, precision, time scheme) one
// batched stage kernel per Runge-Kutta stage over the flattened tile list of
// the group.  Every solve keeps its own dt (its own Slot).  After each
// iteration a status kernel summarises the slots and the host, one iteration
// behind the device, retires finished solves (copying their state out) and
// admits queued ones into the freed arena space (continuous batching).  While
// the resident set is stable and nothing waits for admission, iterations run
// from a captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <unordered_map>
#include <vector>

#include "roeam_host.hpp"

using roeam::SolveStatus;
using roeam::TileEntry;

namespace {

constexpr int kMaxSolves = 4096;
constexpr size_t kAlign = 256;
constexpr int kGraphIters = 16;  // even
constexpr int kGroups = 72;      // order (2) x precision (2) x time scheme (3) x metric (2) x scalars (3)
constexpr int kStatusEvery = 8;  // iterations between status snapshots without a graph

size_t align_up(size_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }

size_t state_bytes(const roeam_grid *g) { return sizeof(double) * (4 + (size_t)g->nsc) * (size_t)g->ny * (size_t)g->pitch; }

// First-fit allocator over [0, cap) with coalescing.
struct Arena {
    size_t cap = 0;
    std::map<size_t, size_t> free_;  // offset -> size
    void reset(size_t c)
    {
        cap = c;
        free_.clear();
        if (c) free_[0] = c;
    }
    bool alloc(size_t n, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, noff = it->first + n;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const
    {
        size_t s = 0;
        for (auto &kv : free_) s += kv.second;
        return s;
    }
};

enum ReqState { QUEUED = 0, RESIDENT = 1, COPYING = 2, DONE = 3 };

struct Request {
    roeam_solve_desc d{};
    int state = QUEUED;
    int idx = -1;
    size_t off = 0, bytes = 0;
    int group = -1;
    roeam_status rc = ROEAM_OK;
    roeam_step_stats stats{};
    hipEvent_t out_ev = nullptr;
    long done_iter = 0;  // scheduler iteration after which its step budget is spent
};

struct Group {
    int order = 2, precision = 0, time_scheme = 1, metric = 0, nsc = 0, shape = 0;
    std::vector<TileEntry> tiles;
    TileEntry *d_tiles = nullptr;
    TileEntry *h_tiles = nullptr;  // pinned staging of the last upload
    hipEvent_t up_ev = nullptr;    // recorded after that upload
    size_t cap = 0;
    bool dirty = false;
};

} // namespace

struct BatchEngine {
    int device = 0;
    char *d_arena = nullptr;
    size_t arena_bytes = 0;
    bool owns_arena = true;  // false: the caller's memory (roeam_batch_attach), never freed here
    Arena alloc;
    DevSolve *d_solves = nullptr;
    DevSolve *h_solves = nullptr;   // pinned host mirror
    Slot *d_slots = nullptr;
    SolveStatus *d_status = nullptr;
    SolveStatus *h_status[2] = {nullptr, nullptr};  // pinned, one per status snapshot
    hipEvent_t status_ev[2] = {nullptr, nullptr};
    bool status_pending[2] = {false, false};
    std::vector<uint64_t> status_owner[2];  // ticket in each index when the snapshot was taken
    long status_seq = 0;
    std::vector<uint64_t> by_idx;   // ticket resident in each index (0 = free)
    std::vector<int> free_idx;
    int hw = 0;                     // high-water mark of used indices
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    long iter = 0;
    long since_status = 0;          // iterations since the last status snapshot
    Group groups[kGroups];          // (order-1, precision, time_scheme, metric, nsc)
    bool set_changed = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_valid = false;
    // profiling: event pairs around each stage launch (stage number beside)
    bool profiling = false;
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_stage;
    size_t prof_used = 0;
};

static int group_id(const roeam_params &p, int metric, int nsc)
{
    return (((p.order - 1) * 2 + p.precision) * 6 + p.time_scheme * 2 + metric) * 3 + nsc;
}

static void release_engine(BatchEngine *b)
{
    if (!b) return;
    for (hipEvent_t e : b->prof_ev) (void)hipEventDestroy(e);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (auto &kv : b->reqs)
        if (kv.second.out_ev) (void)hipEventDestroy(kv.second.out_ev);
    for (int k = 0; k < 2; ++k) {
        if (b->status_ev[k]) (void)hipEventDestroy(b->status_ev[k]);
        if (b->h_status[k]) (void)hipHostFree(b->h_status[k]);
    }
    for (auto &g : b->groups) {
        if (g.d_tiles) (void)hipFree(g.d_tiles);
        if (g.h_tiles) (void)hipHostFree(g.h_tiles);
        if (g.up_ev) (void)hipEventDestroy(g.up_ev);
    }
    if (b->d_status) (void)hipFree(b->d_status);
    if (b->d_slots) (void)hipFree(b->d_slots);
    if (b->h_solves) (void)hipHostFree(b->h_solves);
    if (b->d_solves) (void)hipFree(b->d_solves);
    if (b->d_arena && b->owns_arena) (void)hipFree(b->d_arena);
    delete b;
}

static roeam_status hip_err(roeam_ctx *ctx, hipError_t e, const char *where)
{
    return roeam_fail(ctx, e == hipErrorOutOfMemory ? ROEAM_ENOMEM : ROEAM_EDEVICE,
                      std::string(where) + ": " + hipGetErrorString(e));
}

#define BHIP(ctx, call)                                           \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return hip_err(ctx, e_, #call);     \
    } while (0)

// Retire solve r: queue the copy of its state to q_out and free its index
// and arena space (later work on the stream runs after the copy).
static roeam_status retire(roeam_ctx *ctx, BatchEngine *b, Request &r, const SolveStatus &s)
{
    const roeam_grid *g = r.d.grid;
    r.stats.t = s.t;
    r.stats.dt_last = s.dt_last;
    r.stats.max_rate = s.rate_last;
    r.stats.steps = (long)s.steps;
    r.stats.nonphys = s.nonphys;
    r.rc = s.nonphys ? ROEAM_ENONPHYS : ROEAM_OK;
    const double *q = (const double *)(b->d_arena + r.off);
    BHIP(ctx, hipMemcpyAsync(r.d.q_out, q, state_bytes(g),
                             r.d.q_out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, ctx->stream));
    if (!r.out_ev) BHIP(ctx, hipEventCreateWithFlags(&r.out_ev, hipEventDisableTiming));
    BHIP(ctx, hipEventRecord(r.out_ev, ctx->stream));
    r.state = COPYING;
    b->alloc.release(r.off, r.bytes);
    b->by_idx[r.idx] = 0;
    b->free_idx.push_back(r.idx);
    Group &G = b->groups[r.group];
    const int idx = r.idx;
    G.tiles.erase(std::remove_if(G.tiles.begin(), G.tiles.end(), [idx](const TileEntry &t) { return t.solve == idx; }),
                  G.tiles.end());
    G.dirty = true;
    b->set_changed = true;
    return ROEAM_OK;
}

// Read a completed status snapshot (if any) and retire the finished solves.
static roeam_status process_status(roeam_ctx *ctx, BatchEngine *b, int which, bool wait)
{
    if (!b->status_pending[which]) return ROEAM_OK;
    if (wait) {
        BHIP(ctx, hipEventSynchronize(b->status_ev[which]));
    } else {
        hipError_t q = hipEventQuery(b->status_ev[which]);
        if (q == hipErrorNotReady) return ROEAM_OK;
        if (q != hipSuccess) return hip_err(ctx, q, "hipEventQuery");
    }
    b->status_pending[which] = false;
    const SolveStatus *st = b->h_status[which];
    const std::vector<uint64_t> &owner = b->status_owner[which];
    for (int i = 0; i < (int)owner.size(); ++i) {
        const uint64_t tk = b->by_idx[i];
        // an index retired and re-admitted after the snapshot belongs to a new solve
        if (!tk || tk != owner[i]) continue;
        Request &r = b->reqs[tk];
        if (r.state != RESIDENT || !st[i].done) continue;
        roeam_status rc = retire(ctx, b, r, st[i]);
        if (rc) return rc;
    }
    return ROEAM_OK;
}

// Tile shape of a group that forms with no forced or tuned shape on its
// first grid, from the cells the group is about to hold (every queued solve
// of the group): one-face-per-thread 16x7 tiles for small totals, where the
// launch is latency-bound and needs many short workgroups; 16x15 tiles with
// one pass per face direction above about 200k cells, where fewer halo cells
// per tile cell pay off (measured crossover on MI355X).
static int untuned_shape(const BatchEngine *b, int group)
{
    long long cells = 0;
    for (uint64_t tk : b->queue) {
        auto it = b->reqs.find(tk);
        if (it != b->reqs.end() && it->second.group == group)
            cells += (long long)it->second.d.grid->nx * it->second.d.grid->ny;
    }
    return cells >= 200000 ? 6 : 8;
}

// Admit queued solves that fit (first fit in submission order).
static roeam_status admit(roeam_ctx *ctx, BatchEngine *b)
{
    const int p = (int)(b->iter & 1);
    for (auto it = b->queue.begin(); it != b->queue.end();) {
        Request &r = b->reqs[*it];
        if (b->free_idx.empty()) break;
        size_t off = 0;
        if (!b->alloc.alloc(r.bytes, &off)) {
            ++it;
            continue;
        }
        const int idx = b->free_idx.back();
        b->free_idx.pop_back();
        r.idx = idx;
        r.off = off;
        r.state = RESIDENT;
        r.done_iter = b->iter + r.d.nsteps;
        b->by_idx[idx] = *it;
        b->hw = std::max(b->hw, idx + 1);
        const roeam_grid *g = r.d.grid;
        const size_t sb = align_up(state_bytes(g));
        double *q = (double *)(b->d_arena + off);
        double *qa = (double *)(b->d_arena + off + sb);
        double *qb = (double *)(b->d_arena + off + 2 * sb);
        DevSolve S = roeam_make_solve(g, &r.d.params, q, qa, qb, &b->d_slots[idx]);
        b->h_solves[idx] = S;
        BHIP(ctx, hipMemcpyAsync(&b->d_solves[idx], &b->h_solves[idx], sizeof(DevSolve), hipMemcpyHostToDevice,
                                 ctx->stream));
        BHIP(ctx, hipMemcpyAsync(q, r.d.q0, state_bytes(g),
                                 r.d.q0_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, ctx->stream));
        BHIP(ctx, roeam::launch_slot_init(&b->d_slots[idx], 1, 0.0, r.d.t_end, r.d.params.cfl, r.d.nsteps, ctx->stream));
        BHIP(ctx, roeam::launch_rate(S, p, ctx->stream));
        // tiles of the solve join its group's work list; an empty group takes
        // the tile shape of its first solve's grid (set, autotuned, or by size)
        Group &G = b->groups[r.group];
        if (G.tiles.empty()) {
            int sh = g->shape_forced >= 0 ? g->shape_forced : g->shape_tuned[r.d.params.order - 1][r.d.params.precision];
            if (sh < 0) sh = untuned_shape(b, r.group);
            if (sh != G.shape) b->graph_valid = false;
            G.shape = sh;
        }
        int tx, ty;
        roeam::tile_shape(G.shape, &tx, &ty);
        const int ntx = (g->nx + tx - 1) / tx, nty = (g->ny + ty - 1) / ty;
        for (int j = 0; j < nty; ++j)
            for (int i = 0; i < ntx; ++i) G.tiles.push_back(TileEntry{idx, i, j, 0});
        G.dirty = true;
        b->set_changed = true;
        it = b->queue.erase(it);
    }
    return ROEAM_OK;
}

// Upload changed work lists.  The device copy is overwritten in stream order
// (after every kernel that read the old list); the pinned staging buffer is
// reused only after its previous upload has completed.
static roeam_status upload_tiles(roeam_ctx *ctx, BatchEngine *b)
{
    for (auto &G : b->groups) {
        if (!G.dirty) continue;
        if (G.tiles.size() > G.cap) {
            BHIP(ctx, hipStreamSynchronize(ctx->stream));
            if (G.d_tiles) BHIP(ctx, hipFree(G.d_tiles));
            if (G.h_tiles) BHIP(ctx, hipHostFree(G.h_tiles));
            G.d_tiles = nullptr;
            G.h_tiles = nullptr;
            G.cap = std::max<size_t>(G.tiles.size() * 2, 1024);
            BHIP(ctx, hipMalloc(&G.d_tiles, G.cap * sizeof(TileEntry)));
            BHIP(ctx, hipHostMalloc(&G.h_tiles, G.cap * sizeof(TileEntry), hipHostMallocDefault));
        }
        if (!G.up_ev) BHIP(ctx, hipEventCreateWithFlags(&G.up_ev, hipEventDisableTiming));
        else BHIP(ctx, hipEventSynchronize(G.up_ev));
        if (!G.tiles.empty()) {
            std::memcpy(G.h_tiles, G.tiles.data(), G.tiles.size() * sizeof(TileEntry));
            BHIP(ctx, hipMemcpyAsync(G.d_tiles, G.h_tiles, G.tiles.size() * sizeof(TileEntry), hipMemcpyHostToDevice,
                                     ctx->stream));
        }
        BHIP(ctx, hipEventRecord(G.up_ev, ctx->stream));
        G.dirty = false;
    }
    return ROEAM_OK;
}

// One batched stage launch, bracketed by profiling events when profiling.
static hipError_t stage_launch(BatchEngine *b, const Group &G, int n, int stage, int p, int last, hipStream_t s)
{
    if (!b->profiling)
        return roeam::launch_stage_batch(b->d_solves, G.d_tiles, n, G.order, G.precision, G.metric, G.nsc, G.shape, stage,
                                         p, last, s);
    hipError_t e = hipSuccess;
    while (e == hipSuccess && b->prof_ev.size() < b->prof_used + 2) {
        hipEvent_t ev;
        e = hipEventCreate(&ev);
        if (e == hipSuccess) b->prof_ev.push_back(ev);
    }
    if (e == hipSuccess) e = hipEventRecord(b->prof_ev[b->prof_used], s);
    if (e == hipSuccess)
        e = roeam::launch_stage_batch(b->d_solves, G.d_tiles, n, G.order, G.precision, G.metric, G.nsc, G.shape, stage, p,
                                      last, s);
    if (e == hipSuccess) e = hipEventRecord(b->prof_ev[b->prof_used + 1], s);
    if (e == hipSuccess) {
        b->prof_stage.push_back(stage);
        b->prof_used += 2;
    }
    return e;
}

static hipError_t enqueue_iteration(BatchEngine *b, int p, hipStream_t s)
{
    for (auto &G : b->groups) {
        const int n = (int)G.tiles.size();
        if (!n) continue;
        hipError_t e;
        if (G.time_scheme == 0) {
            e = stage_launch(b, G, n, 1, p, 1, s);
            if (e == hipSuccess) e = roeam::launch_copy_back_batch(b->d_solves, G.d_tiles, n, G.shape, p, s);
        } else {
            const int first = G.time_scheme == 1 ? 1 : 4, nst = G.time_scheme == 1 ? 3 : 4;
            e = hipSuccess;
            for (int k = 0; k < nst && e == hipSuccess; ++k) e = stage_launch(b, G, n, first + k, p, k == nst - 1, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Snapshot the status of every index after the iterations queued so far.
// The state after iteration k sits at parity (k + 1) & 1 = iter & 1.
static roeam_status enqueue_status(roeam_ctx *ctx, BatchEngine *b, int which)
{
    const int p_after = (int)(b->iter & 1);
    BHIP(ctx, roeam::launch_status(b->d_slots, b->hw, p_after, b->d_status, ctx->stream));
    if (b->hw) BHIP(ctx, hipMemcpyAsync(b->h_status[which], b->d_status, sizeof(SolveStatus) * b->hw,
                                        hipMemcpyDeviceToHost, ctx->stream));
    BHIP(ctx, hipEventRecord(b->status_ev[which], ctx->stream));
    b->status_pending[which] = true;
    b->status_owner[which].assign(b->by_idx.begin(), b->by_idx.begin() + b->hw);
    return ROEAM_OK;
}

static int resident_count(const BatchEngine *b)
{
    int n = 0;
    for (int i = 0; i < b->hw; ++i) n += b->by_idx[i] != 0;
    return n;
}

extern "C" {

void roeam_batch_release(roeam_ctx *ctx)
{
    if (!ctx || !ctx->batch) return;
    (void)hipStreamSynchronize(ctx->stream);
    release_engine(ctx->batch);
    ctx->batch = nullptr;
}

size_t roeam_batch_footprint(const roeam_grid *g)
{
    if (!g) return 0;
    return 3 * align_up(state_bytes(g));
}

// A new engine over `arena` (the caller's device memory) or, arena == nullptr,
// over arena_bytes the engine allocates itself.
static roeam_status setup_engine(roeam_ctx *ctx, void *arena, size_t arena_bytes)
{
    if (!ctx) return ROEAM_EINVAL;
    if (arena_bytes < kAlign) return roeam_fail(ctx, ROEAM_EINVAL, "arena too small");
    if (arena && ((uintptr_t)arena % kAlign) != 0) return roeam_fail(ctx, ROEAM_EINVAL, "arena not 256-byte aligned");
    BHIP(ctx, hipSetDevice(ctx->device));
    if (ctx->batch) {
        BatchEngine *b = ctx->batch;
        if (!b->queue.empty() || resident_count(b)) return roeam_fail(ctx, ROEAM_EBUSY, "batch engine has work");
        BHIP(ctx, hipStreamSynchronize(ctx->stream));
        release_engine(b);
        ctx->batch = nullptr;
    }
    BatchEngine *b = new (std::nothrow) BatchEngine;
    if (!b) return roeam_fail(ctx, ROEAM_ENOMEM, "host allocation");
    b->device = ctx->device;
    hipError_t e = hipSuccess;
    if (arena) {
        b->d_arena = (char *)arena;
        b->owns_arena = false;
    } else {
        e = hipMalloc(&b->d_arena, arena_bytes);
    }
    if (e == hipSuccess) e = hipMalloc(&b->d_solves, sizeof(DevSolve) * kMaxSolves);
    if (e == hipSuccess) e = hipHostMalloc(&b->h_solves, sizeof(DevSolve) * kMaxSolves, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&b->d_slots, sizeof(Slot) * kMaxSolves);
    if (e == hipSuccess) e = hipMalloc(&b->d_status, sizeof(SolveStatus) * kMaxSolves);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipHostMalloc(&b->h_status[k], sizeof(SolveStatus) * kMaxSolves, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->status_ev[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        release_engine(b);
        return hip_err(ctx, e, "batch reserve");
    }
    b->arena_bytes = arena_bytes;
    b->alloc.reset(arena_bytes);
    b->by_idx.assign(kMaxSolves, 0);
    for (int i = kMaxSolves - 1; i >= 0; --i) b->free_idx.push_back(i);
    for (int gidx = 0; gidx < kGroups; ++gidx) {
        Group &G = b->groups[gidx];
        const int g = gidx / 3;
        G.order = g / 12 + 1;
        G.precision = (g / 6) & 1;
        G.time_scheme = (g / 2) % 3;
        G.metric = g & 1;
        G.nsc = gidx % 3;
        G.shape = 0;
    }
    ctx->batch = b;
    return ROEAM_OK;
}

roeam_status roeam_batch_reserve(roeam_ctx *ctx, size_t arena_bytes) { return setup_engine(ctx, nullptr, arena_bytes); }

roeam_status roeam_batch_attach(roeam_ctx *ctx, void *arena, size_t arena_bytes)
{
    if (!arena) return roeam_fail(ctx, ROEAM_EINVAL, "arena is NULL");
    return setup_engine(ctx, arena, arena_bytes);
}

roeam_status roeam_batch_submit(roeam_ctx *ctx, int n, const roeam_solve_desc *descs, uint64_t *tickets_out)
{
    if (!ctx || n < 0 || (n > 0 && (!descs || !tickets_out))) return roeam_fail(ctx, ROEAM_EINVAL, "bad argument");
    BatchEngine *b = ctx->batch;
    if (!b) return roeam_fail(ctx, ROEAM_EINVAL, "call roeam_batch_reserve first");
    for (int i = 0; i < n; ++i) {
        const roeam_solve_desc &d = descs[i];
        if (!d.grid || d.grid->ctx != ctx) return roeam_fail(ctx, ROEAM_EINVAL, "descriptor grid invalid");
        roeam_status st = roeam_check_params(ctx, &d.params, true);
        if (st) return st;
        if (!d.q0 || !d.q_out) return roeam_fail(ctx, ROEAM_EINVAL, "q0 and q_out are required");
        if (d.nsteps < 0 || !std::isfinite(d.t_end)) return roeam_fail(ctx, ROEAM_EINVAL, "bad run length");
        if (roeam_batch_footprint(d.grid) > b->arena_bytes)
            return roeam_fail(ctx, ROEAM_ENOMEM, "solve larger than the whole arena");
    }
    for (int i = 0; i < n; ++i) {
        const uint64_t tk = b->next_ticket++;
        Request r;
        r.d = descs[i];
        r.bytes = roeam_batch_footprint(descs[i].grid);
        r.group = group_id(descs[i].params, descs[i].grid->metric, descs[i].grid->nsc);
        b->reqs.emplace(tk, r);
        b->queue.push_back(tk);
        tickets_out[i] = tk;
    }
    return ROEAM_OK;
}

roeam_status roeam_batch_run(roeam_ctx *ctx, long iterations, int *pending)
{
    if (!ctx) return ROEAM_EINVAL;
    BatchEngine *b = ctx->batch;
    if (!b) return roeam_fail(ctx, ROEAM_EINVAL, "call roeam_batch_reserve first");
    BHIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    long done_iters = 0;
    roeam_status rc;
    for (;;) {
        // retire what finished (status one iteration behind), then admit
        for (int w = 0; w < 2; ++w)
            if ((rc = process_status(ctx, b, w, false))) return rc;
        if ((rc = admit(ctx, b))) return rc;
        if ((rc = upload_tiles(ctx, b))) return rc;
        const int resident = resident_count(b);
        if (iterations >= 0 && done_iters >= iterations) break;
        if (resident == 0) {
            if (b->queue.empty()) break;
            // queued solves wait for space held by nothing resident: cannot happen,
            // every queued solve fits the empty arena
            return roeam_fail(ctx, ROEAM_ENOMEM, "queued solve does not fit the arena");
        }
        // iterations of the resident set; a stable set with nothing waiting runs
        // kGraphIters iterations from one captured graph, unless a resident
        // solve spends its step budget sooner: then single iterations run up to
        // that iteration and the status is snapshot right after it, so the
        // solve leaves without waiting for the regular snapshot cadence
        long next_done = LONG_MAX;
        for (int i = 0; i < b->hw; ++i)
            if (b->by_idx[i]) next_done = std::min(next_done, b->reqs[b->by_idx[i]].done_iter);
        const bool stable = !b->set_changed && b->queue.empty() && (b->iter & 1) == 0 &&
                            (iterations < 0 || iterations - done_iters >= kGraphIters) &&
                            next_done - b->iter >= kGraphIters;
        long ran;
        if (stable && s != nullptr && !b->profiling) {
            if (!b->graph_valid) {
                if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
                if (b->graph) (void)hipGraphDestroy(b->graph);
                b->gexec = nullptr;
                b->graph = nullptr;
                BHIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
                hipError_t e = hipSuccess;
                for (int k = 0; k < kGraphIters && e == hipSuccess; ++k) e = enqueue_iteration(b, k & 1, s);
                hipError_t e2 = hipStreamEndCapture(s, &b->graph);
                if (e != hipSuccess) return hip_err(ctx, e, "capture batch iteration");
                if (e2 != hipSuccess) return hip_err(ctx, e2, "hipStreamEndCapture");
                BHIP(ctx, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
                b->graph_valid = true;
            }
            BHIP(ctx, hipGraphLaunch(b->gexec, s));
            ran = kGraphIters;
        } else {
            BHIP(ctx, enqueue_iteration(b, (int)(b->iter & 1), s));
            ran = 1;
        }
        if (b->set_changed) {
            b->graph_valid = false;
            b->set_changed = false;
        }
        b->iter += ran;
        done_iters += ran;
        b->since_status += ran;
        // snapshot the status after every graph, or every kStatusEvery single
        // iterations, or when the caller's iteration budget ends; the buffer's
        // previous snapshot (two back) is read first
        const bool budget_end = iterations >= 0 && done_iters >= iterations;
        // (profiling snapshots and reads the status after every iteration, so
        // finished solves leave at once and no timed launch is an idle one)
        const bool budget_spent = b->iter == next_done;
        if (ran > 1 || b->since_status >= kStatusEvery || budget_end || budget_spent || b->profiling) {
            const int which = (int)(b->status_seq++ & 1);
            if ((rc = process_status(ctx, b, which, true))) return rc;
            if ((rc = enqueue_status(ctx, b, which))) return rc;
            if (b->profiling && (rc = process_status(ctx, b, which, true))) return rc;
            b->since_status = 0;
        }
    }
    if (iterations < 0) {
        // drain: retire everything still reported
        for (int w = 0; w < 2; ++w)
            if ((rc = process_status(ctx, b, w, true))) return rc;
    }
    if (pending) {
        int n = 0;
        for (auto &kv : b->reqs) n += kv.second.state == QUEUED || kv.second.state == RESIDENT;
        *pending = n;
    }
    return ROEAM_OK;
}

roeam_status roeam_batch_profile_run(roeam_ctx *ctx, long iterations, int *pending, double stage_ms[4],
                                     long *launches)
{
    if (!ctx || !stage_ms) return roeam_fail(ctx, ROEAM_EINVAL, "bad argument");
    BatchEngine *b = ctx->batch;
    if (!b) return roeam_fail(ctx, ROEAM_EINVAL, "call roeam_batch_reserve first");
    b->profiling = true;
    b->prof_used = 0;
    b->prof_stage.clear();
    roeam_status rc = roeam_batch_run(ctx, iterations, pending);
    b->profiling = false;
    if (rc) return rc;
    BHIP(ctx, hipStreamSynchronize(ctx->stream));
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    long cnt[4] = {0, 0, 0, 0};
    for (size_t k = 0; k < b->prof_stage.size(); ++k) {
        float ms = 0.f;
        BHIP(ctx, hipEventElapsedTime(&ms, b->prof_ev[2 * k], b->prof_ev[2 * k + 1]));
        const int code = b->prof_stage[k];
        const int st = code >= 4 ? code - 4 : code - 1;  // position of the stage within its step
        sum[st] += ms;
        cnt[st] += 1;
    }
    for (int k = 0; k < 4; ++k) stage_ms[k] = cnt[k] ? sum[k] / (double)cnt[k] : 0.0;
    if (launches) *launches = (long)b->prof_stage.size();
    return ROEAM_OK;
}

roeam_status roeam_batch_poll(roeam_ctx *ctx, uint64_t ticket, int *done, roeam_step_stats *stats)
{
    if (!ctx || !done) return roeam_fail(ctx, ROEAM_EINVAL, "bad argument");
    BatchEngine *b = ctx->batch;
    if (!b) return roeam_fail(ctx, ROEAM_EINVAL, "call roeam_batch_reserve first");
    auto it = b->reqs.find(ticket);
    if (it == b->reqs.end()) return roeam_fail(ctx, ROEAM_ENOTFOUND, "unknown ticket");
    Request &r = it->second;
    if (r.state == COPYING) {
        hipError_t q = hipEventQuery(r.out_ev);
        if (q == hipSuccess) r.state = DONE;
        else if (q != hipErrorNotReady) return hip_err(ctx, q, "hipEventQuery");
    }
    *done = r.state == DONE;
    if (!*done) return ROEAM_OK;
    // reported done: the ticket is forgotten (a server's request table does not grow)
    if (stats) *stats = r.stats;
    const roeam_status rc = r.rc;
    if (r.out_ev) (void)hipEventDestroy(r.out_ev);
    b->reqs.erase(it);
    if (rc == ROEAM_ENONPHYS) return roeam_fail(ctx, ROEAM_ENONPHYS, "solve produced a non-physical state");
    return ROEAM_OK;
}

} // extern "C"

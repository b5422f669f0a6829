// roeam_batch.hip -- the continuous-batching engine behind roeam_batch_*.
//
// Resident solves keep three state copies (q, qa, qb) in a device arena and a
// Slot each.  A scheduler iteration advances every resident solve by one
// time step: per group of solves sharing (order, precision, time scheme,
// metric, scalar count) one batched stage kernel per Runge-Kutta stage over
// the group's work list of tiles.  Every solve keeps its own dt (its own
// Slot), and a solve whose step budget or end time is reached idles (its
// tiles exit at once) until the host retires it.
//
// The work lists live in device memory with a tile count the kernels read, and
// the launches are sized to the lists' capacities, so one captured HIP graph
// of graph_iters iterations serves every resident set that fits: admitting and
// retiring solves only rewrites the lists (copies queued between graph
// launches), and a graph is captured again only when a group appears or
// disappears or a list's capacity changes.  After each graph a status kernel
// summarises the slots; the host, one graph behind the device, retires
// finished solves (copying their state out) and admits queued ones into the
// freed arena space (continuous batching).  The solves retired or admitted in
// one round are moved by one upload and two kernel launches, whatever their
// number (roeam_batch_kernels.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <unordered_map>
#include <vector>

#include "roeam_host.hpp"

using roeam::SolveStatus;
using roeam::TileEntry;

namespace {

constexpr int kMaxSolves = 4096;
constexpr size_t kAlign = 256;
constexpr int kGroups = 72;  // order (2) x precision (2) x time scheme (3) x metric (2) x scalars (3)
constexpr int kMinCap = 1024;  // smallest work-list capacity, tiles

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
};

enum ReqState { QUEUED = 0, RESIDENT = 1, COPYING = 2, DONE = 3 };

// An event shared by the solves retired in one round: recorded after their
// copies, destroyed with the last of them.
struct SharedEvent {
    hipEvent_t ev = nullptr;
    ~SharedEvent()
    {
        if (ev) (void)hipEventDestroy(ev);
    }
};

struct Request {
    roeam_solve_desc d{};
    int state = QUEUED;
    int idx = -1;
    size_t off = 0, bytes = 0;
    int group = -1;
    uint64_t seq = 0;  // submission order
    uint64_t ticket = 0;
    long admit_iter = 0;  // scheduler iteration at which it joined
    roeam_status rc = ROEAM_OK;
    roeam_step_stats stats{};
    std::shared_ptr<SharedEvent> out_ev;  // its copy out is complete when this has passed
};

struct Group {
    int order = 2, precision = 0, time_scheme = 1, metric = 0, nsc = 0;
    int shape = -1;                // tile shape, fixed when the group first forms
    std::vector<TileEntry> tiles;  // host copy of the work list
    TileEntry *d_tiles = nullptr;  // device work list, cap entries
    int *d_count = nullptr;        // device tile count
    TileEntry *h_tiles = nullptr;  // pinned staging of the last upload (cap entries + the count after them)
    hipEvent_t up_ev = nullptr;    // recorded after that upload
    int cap = 0;
    bool dirty = false;
    int graph_cap = 0;             // capacity the captured graph's launches were sized for (0: not in the graph)
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
    uint64_t next_seq = 0;
    long iter = 0;
    Group groups[kGroups];          // (order-1, precision, time_scheme, metric, nsc)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_valid = false;
    // options (roeam_batch_configure)
    int graph_iters = 16;           // iterations per graph (even)
    bool persistent = false;        // persistent batched kernels instead of one workgroup per tile
    int policy = ROEAM_ADMIT_FIFO;
    bool autotune = true;
    int max_resident = 0;           // 0: as many solves as the arena holds
    int cus = 0;                    // compute units of the device
    // counters
    long captures = 0, graph_launches = 0, tunes = 0;
    int last_shape = -1;            // tile shape of the group formed last
    // the round's pending admissions and state moves, staged through one upload
    std::vector<roeam::AdmitInit> pend_init;
    std::vector<roeam::StateMove> pend_moves;
    std::vector<uint64_t> pend_retired;  // tickets whose copy out is among the moves
    char *d_stage = nullptr, *h_stage = nullptr;
    size_t stage_cap = 0;
    hipEvent_t stage_ev = nullptr;  // recorded after the last staging upload
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

static void release_graph(BatchEngine *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_valid = false;
}

static void release_engine(BatchEngine *b)
{
    if (!b) return;
    for (hipEvent_t e : b->prof_ev) (void)hipEventDestroy(e);
    release_graph(b);
    b->reqs.clear();  // their shared events
    if (b->stage_ev) (void)hipEventDestroy(b->stage_ev);
    if (b->d_stage) (void)hipFree(b->d_stage);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    for (int k = 0; k < 2; ++k) {
        if (b->status_ev[k]) (void)hipEventDestroy(b->status_ev[k]);
        if (b->h_status[k]) (void)hipHostFree(b->h_status[k]);
    }
    for (auto &g : b->groups) {
        if (g.d_tiles) (void)hipFree(g.d_tiles);
        if (g.d_count) (void)hipFree(g.d_count);
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

static int stages_of(int time_scheme) { return time_scheme == 0 ? 1 : (time_scheme == 1 ? 3 : 4); }

// Workgroups of a group's batched launches: its list capacity (windowed form)
// or, persistent, what the device holds at once; a multiple of 8.
static int launch_blocks(const BatchEngine *b, const Group &G, int cap)
{
    int n = cap;
    if (b->persistent) {
        const int per_cu = roeam::batch_blocks_per_cu(G.order, G.precision, G.metric, G.nsc, G.shape);
        const int resident = std::max(per_cu, 1) * std::max(b->cus, 1);
        n = std::min(cap, resident);
    }
    return ((std::max(n, 1) + 7) >> 3) << 3;
}

// Tiles of resident solve idx (grid g) on the group's shape, appended to the
// group's work list.
static void append_tiles(Group &G, int idx, const roeam_grid *g)
{
    int tx, ty;
    roeam::tile_shape(G.shape, &tx, &ty);
    const int ntx = (g->nx + tx - 1) / tx, nty = (g->ny + ty - 1) / ty;
    for (int j = 0; j < nty; ++j)
        for (int i = 0; i < ntx; ++i) G.tiles.push_back(TileEntry{idx, i, j, 0});
    G.dirty = true;
}

// The move of grid g's state from src to dst.
static roeam::StateMove state_move(const roeam_grid *g, const double *src, double *dst, int solve)
{
    roeam::StateMove m{};
    m.src = src;
    m.dst = dst;
    m.plane = (long long)g->ny * g->pitch;
    m.pitch = g->pitch;
    m.nx = g->nx;
    m.ny = g->ny;
    m.rows = 4 + g->nsc;
    m.solve = solve;
    return m;
}

// Upload the round's pending admissions and moves in one copy and launch
// them (descriptors and slots first, then the moves); the solves retired in
// the round share one event recorded after their copies.  The pinned staging
// buffer is rewritten only after its previous upload has completed.
static roeam_status flush_moves(roeam_ctx *ctx, BatchEngine *b)
{
    if (b->pend_init.empty() && b->pend_moves.empty() && b->pend_retired.empty()) return ROEAM_OK;
    std::vector<roeam::MoveChunk> chunks;
    for (int m = 0; m < (int)b->pend_moves.size(); ++m) {
        const long long n = (long long)b->pend_moves[m].nx * b->pend_moves[m].ny;
        for (long long c0 = 0; c0 < n; c0 += roeam::kMoveChunk) chunks.push_back(roeam::MoveChunk{m, (int)c0});
    }
    const size_t bi = align_up(b->pend_init.size() * sizeof(roeam::AdmitInit));
    const size_t bm = align_up(b->pend_moves.size() * sizeof(roeam::StateMove));
    const size_t bytes = bi + bm + chunks.size() * sizeof(roeam::MoveChunk);
    if (bytes > b->stage_cap) {
        BHIP(ctx, hipStreamSynchronize(ctx->stream));
        if (b->d_stage) BHIP(ctx, hipFree(b->d_stage));
        if (b->h_stage) BHIP(ctx, hipHostFree(b->h_stage));
        b->d_stage = b->h_stage = nullptr;
        b->stage_cap = 0;
        const size_t cap = align_up(bytes + bytes / 2);
        BHIP(ctx, hipMalloc(&b->d_stage, cap));
        BHIP(ctx, hipHostMalloc(&b->h_stage, cap, hipHostMallocDefault));
        b->stage_cap = cap;
    } else if (b->stage_ev) {
        BHIP(ctx, hipEventSynchronize(b->stage_ev));
    }
    if (bytes) {
        std::memcpy(b->h_stage, b->pend_init.data(), b->pend_init.size() * sizeof(roeam::AdmitInit));
        std::memcpy(b->h_stage + bi, b->pend_moves.data(), b->pend_moves.size() * sizeof(roeam::StateMove));
        std::memcpy(b->h_stage + bi + bm, chunks.data(), chunks.size() * sizeof(roeam::MoveChunk));
        BHIP(ctx, hipMemcpyAsync(b->d_stage, b->h_stage, bytes, hipMemcpyHostToDevice, ctx->stream));
        if (!b->stage_ev) BHIP(ctx, hipEventCreateWithFlags(&b->stage_ev, hipEventDisableTiming));
        BHIP(ctx, hipEventRecord(b->stage_ev, ctx->stream));
        BHIP(ctx, roeam::launch_admit_init((const roeam::AdmitInit *)b->d_stage, (int)b->pend_init.size(), b->d_solves,
                                           ctx->stream));
        BHIP(ctx, roeam::launch_moves((const roeam::StateMove *)(b->d_stage + bi),
                                      (const roeam::MoveChunk *)(b->d_stage + bi + bm), (int)chunks.size(),
                                      b->d_solves, ctx->stream));
    }
    if (!b->pend_retired.empty()) {
        auto ev = std::make_shared<SharedEvent>();
        BHIP(ctx, hipEventCreateWithFlags(&ev->ev, hipEventDisableTiming));
        BHIP(ctx, hipEventRecord(ev->ev, ctx->stream));
        for (uint64_t tk : b->pend_retired) b->reqs[tk].out_ev = ev;
    }
    b->pend_init.clear();
    b->pend_moves.clear();
    b->pend_retired.clear();
    return ROEAM_OK;
}

// Retire solve r: queue the copy of its state to q_out (flush_moves issues
// it, before anything later on the stream) and free its index and arena
// space.  Forward Euler leaves the state of an odd step count in qa.
static roeam_status retire(roeam_ctx *ctx, BatchEngine *b, Request &r, const SolveStatus &s)
{
    const roeam_grid *g = r.d.grid;
    r.stats.t = s.t;
    r.stats.dt_last = s.dt_last;
    r.stats.max_rate = s.rate_last;
    r.stats.steps = (long)s.steps;
    r.stats.nonphys = s.nonphys;
    r.rc = s.nonphys ? ROEAM_ENONPHYS : ROEAM_OK;
    const size_t sb = align_up(state_bytes(g));
    const bool in_qa = r.d.params.time_scheme == 0 && (s.steps & 1);
    const double *q = (const double *)(b->d_arena + r.off + (in_qa ? sb : 0));
    if (r.d.q_out_on_device) b->pend_moves.push_back(state_move(g, q, r.d.q_out, -1));
    else BHIP(ctx, hipMemcpyAsync(r.d.q_out, q, state_bytes(g), hipMemcpyDeviceToHost, ctx->stream));
    b->pend_retired.push_back(r.ticket);
    r.state = COPYING;
    b->alloc.release(r.off, r.bytes);
    b->by_idx[r.idx] = 0;
    b->free_idx.push_back(r.idx);
    Group &G = b->groups[r.group];
    const int idx = r.idx;
    G.tiles.erase(std::remove_if(G.tiles.begin(), G.tiles.end(), [idx](const TileEntry &t) { return t.solve == idx; }),
                  G.tiles.end());
    G.dirty = true;
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
    return flush_moves(ctx, b);
}

// Grow (or shrink) a group's device work list to hold `need` tiles.  Changing
// the capacity reallocates the list and invalidates the captured graph.
static roeam_status ensure_capacity(roeam_ctx *ctx, BatchEngine *b, Group &G, size_t need)
{
    // an emptied list keeps its capacity (the next solves of the group may reuse
    // the graph); one that shrinks below a third of it is reallocated
    int want = G.cap;
    if ((int)need > G.cap) want = (int)std::max<size_t>(kMinCap, need + need / 4);
    else if (need > 0 && G.cap > kMinCap && (int)need < G.cap / 3)
        want = (int)std::max<size_t>(kMinCap, need + need / 4);
    if (want == G.cap && G.d_tiles) return ROEAM_OK;
    want = (want + 63) & ~63;
    BHIP(ctx, hipStreamSynchronize(ctx->stream));
    if (G.d_tiles) BHIP(ctx, hipFree(G.d_tiles));
    if (G.d_count) BHIP(ctx, hipFree(G.d_count));
    if (G.h_tiles) BHIP(ctx, hipHostFree(G.h_tiles));
    G.d_tiles = nullptr;
    G.d_count = nullptr;
    G.h_tiles = nullptr;
    BHIP(ctx, hipMalloc(&G.d_tiles, (size_t)want * sizeof(TileEntry)));
    BHIP(ctx, hipMalloc(&G.d_count, sizeof(int)));
    BHIP(ctx, hipHostMalloc(&G.h_tiles, ((size_t)want + 1) * sizeof(TileEntry), hipHostMallocDefault));
    G.cap = want;
    G.dirty = true;
    b->graph_valid = false;
    return ROEAM_OK;
}

// Upload changed work lists and their counts, in stream order (after every
// kernel that read the old list).  The pinned staging buffer is reused only
// after its previous upload has completed.
static roeam_status upload_tiles(roeam_ctx *ctx, BatchEngine *b)
{
    for (auto &G : b->groups) {
        if (!G.dirty) continue;
        roeam_status rc = ensure_capacity(ctx, b, G, G.tiles.size());
        if (rc) return rc;
        if (!G.up_ev) BHIP(ctx, hipEventCreateWithFlags(&G.up_ev, hipEventDisableTiming));
        else BHIP(ctx, hipEventSynchronize(G.up_ev));
        const int n = (int)G.tiles.size();
        if (n) std::memcpy(G.h_tiles, G.tiles.data(), (size_t)n * sizeof(TileEntry));
        int *hc = reinterpret_cast<int *>(G.h_tiles + G.cap);
        *hc = n;
        if (n)
            BHIP(ctx, hipMemcpyAsync(G.d_tiles, G.h_tiles, (size_t)n * sizeof(TileEntry), hipMemcpyHostToDevice,
                                     ctx->stream));
        BHIP(ctx, hipMemcpyAsync(G.d_count, hc, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
        BHIP(ctx, hipEventRecord(G.up_ev, ctx->stream));
        G.dirty = false;
        if (G.graph_cap != 0 && G.graph_cap != G.cap) b->graph_valid = false;
        if (G.graph_cap == 0 && n > 0) b->graph_valid = false;
    }
    // a group that emptied while others run leaves the graph (its launches
    // would only start workgroups that exit)
    bool any = false, idle = false;
    for (auto &G : b->groups) {
        any |= !G.tiles.empty();
        idle |= G.graph_cap != 0 && G.tiles.empty();
    }
    if (any && idle) b->graph_valid = false;
    return ROEAM_OK;
}

// One batched stage launch of group G, bracketed by profiling events when
// profiling.
static hipError_t stage_launch(BatchEngine *b, const Group &G, int stage, int p, int last, hipStream_t s)
{
    const int blocks = launch_blocks(b, G, G.cap);
    if (!b->profiling)
        return roeam::launch_stage_batch(b->d_solves, G.d_tiles, G.d_count, blocks, b->persistent, G.order, G.precision,
                                         G.metric, G.nsc, G.shape, stage, p, last, s);
    hipError_t e = hipSuccess;
    while (e == hipSuccess && b->prof_ev.size() < b->prof_used + 2) {
        hipEvent_t ev;
        e = hipEventCreate(&ev);
        if (e == hipSuccess) b->prof_ev.push_back(ev);
    }
    if (e == hipSuccess) e = hipEventRecord(b->prof_ev[b->prof_used], s);
    if (e == hipSuccess)
        e = roeam::launch_stage_batch(b->d_solves, G.d_tiles, G.d_count, blocks, b->persistent, G.order, G.precision,
                                      G.metric, G.nsc, G.shape, stage, p, last, s);
    if (e == hipSuccess) e = hipEventRecord(b->prof_ev[b->prof_used + 1], s);
    if (e == hipSuccess) {
        b->prof_stage.push_back(stage);
        b->prof_used += 2;
    }
    return e;
}

// One scheduler iteration with parity p over the groups in the graph (or, when
// profiling, over the non-empty groups).  Forward Euler alternates stage 1
// (q -> qa) and stage 8 (qa -> q).
static hipError_t enqueue_iteration(BatchEngine *b, int p, hipStream_t s)
{
    for (auto &G : b->groups) {
        if (b->profiling ? G.tiles.empty() : G.graph_cap == 0) continue;
        hipError_t e = hipSuccess;
        if (G.time_scheme == 0) {
            e = stage_launch(b, G, p ? 8 : 1, p, 1, s);
        } else {
            const int first = G.time_scheme == 1 ? 1 : 4, nst = stages_of(G.time_scheme);
            for (int k = 0; k < nst && e == hipSuccess; ++k) e = stage_launch(b, G, first + k, p, k == nst - 1, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Snapshot the status of every index after the iterations queued so far.
// Graphs are an even number of iterations, so the state after them sits at
// parity 0.
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

// Tile shape of a group that forms now: time the batched stage kernel (its
// first stage, which only reads q and writes qa; the step state it publishes
// is written again by the real first stage) on the group's real work list for
// every shape, best of three rounds of three launches after a warm-up, and keep
// the fastest.  Without tuning (or with a shape forced on the first grid) the
// first grid's forced shape, else 16x7/256 below about 200k cells and 16x15/256
// above (measured crossover).
static roeam_status tune_group(roeam_ctx *ctx, BatchEngine *b, Group &G, const std::vector<int> &idxs)
{
    long long cells = 0;
    const roeam_grid *g0 = nullptr;
    for (int idx : idxs) {
        const Request &r = b->reqs[b->by_idx[idx]];
        cells += (long long)r.d.grid->nx * r.d.grid->ny;
        if (!g0) g0 = r.d.grid;
    }
    G.tiles.clear();
    const bool forced = g0 && g0->shape_forced >= 0;
    G.shape = forced ? g0->shape_forced : (cells >= 200000 ? 6 : 8);
    roeam_status rc = ROEAM_OK;
    if (!forced && b->autotune && !b->profiling && ctx->stream != nullptr && !idxs.empty()) {
        hipStream_t s = ctx->stream;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        BHIP(ctx, hipEventCreate(&e0));
        BHIP(ctx, hipEventCreate(&e1));
        int best = G.shape;
        float best_ms = 1e30f;
        for (int sh = 0; sh < roeam::tile_shape_count() && rc == ROEAM_OK; ++sh) {
            G.shape = sh;
            G.tiles.clear();
            for (int idx : idxs) append_tiles(G, idx, b->reqs[b->by_idx[idx]].d.grid);
            if ((rc = upload_tiles(ctx, b))) break;
            const int blocks = launch_blocks(b, G, G.cap);
            auto launch = [&]() {
                return roeam::launch_stage_batch(b->d_solves, G.d_tiles, G.d_count, blocks, b->persistent, G.order,
                                                 G.precision, G.metric, G.nsc, G.shape, G.time_scheme == 2 ? 4 : 1, 0,
                                                 G.time_scheme == 0 ? 1 : 0, s);
            };
            hipError_t e = launch();
            float shape_ms = 1e30f;
            for (int round = 0; round < 3 && e == hipSuccess; ++round) {
                e = hipEventRecord(e0, s);
                for (int k = 0; k < 3 && e == hipSuccess; ++k) e = launch();
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                shape_ms = std::min(shape_ms, ms);
            }
            if (e != hipSuccess) rc = hip_err(ctx, e, "batch tile-shape tuning");
            if (shape_ms < best_ms) {
                best_ms = shape_ms;
                best = sh;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        G.shape = best;
        G.tiles.clear();
        ++b->tunes;
    }
    // the work list of the admitted solves on the chosen shape, on every path
    for (int idx : idxs) append_tiles(G, idx, b->reqs[b->by_idx[idx]].d.grid);
    b->last_shape = G.shape;
    return rc;
}

// Work of a queued request for the shortest-first policy.
static double req_work(const Request &r)
{
    return (double)r.d.grid->nx * (double)r.d.grid->ny * (double)std::max(r.d.nsteps, 1L);
}

// Admit queued solves that fit: first fit in submission order (FIFO) or in
// order of increasing work (cells x steps; ties by submission).  Groups that
// form in this call tune their tile shape on the solves admitted into them.
static roeam_status admit(roeam_ctx *ctx, BatchEngine *b)
{
    if (b->queue.empty()) return ROEAM_OK;
    std::vector<uint64_t> order(b->queue.begin(), b->queue.end());
    if (b->policy == ROEAM_ADMIT_SHORTEST)
        std::stable_sort(order.begin(), order.end(), [b](uint64_t x, uint64_t y) {
            return req_work(b->reqs[x]) < req_work(b->reqs[y]);
        });
    std::vector<std::vector<int>> forming(kGroups);
    std::vector<uint64_t> admitted;
    int resident = 0;
    for (int i = 0; i < b->hw; ++i) resident += b->by_idx[i] != 0;
    for (uint64_t tk : order) {
        Request &r = b->reqs[tk];
        if (b->free_idx.empty()) break;
        if (b->max_resident > 0 && resident >= b->max_resident) break;
        size_t off = 0;
        if (!b->alloc.alloc(r.bytes, &off)) continue;
        const int idx = b->free_idx.back();
        b->free_idx.pop_back();
        r.idx = idx;
        r.off = off;
        r.state = RESIDENT;
        ++resident;
        r.admit_iter = b->iter;
        b->by_idx[idx] = tk;
        b->hw = std::max(b->hw, idx + 1);
        const roeam_grid *g = r.d.grid;
        const size_t sb = align_up(state_bytes(g));
        double *q = (double *)(b->d_arena + off);
        double *qa = (double *)(b->d_arena + off + sb);
        double *qb = (double *)(b->d_arena + off + 2 * sb);
        DevSolve S = roeam_make_solve(g, &r.d.params, q, qa, qb, &b->d_slots[idx]);
        b->h_solves[idx] = S;
        // descriptor, fresh slot, the initial state into the arena and its
        // rate: queued, issued for the whole round by flush_moves
        roeam::AdmitInit ai{};
        ai.S = S;
        ai.t_end = r.d.t_end;
        ai.cfl = r.d.params.cfl;
        ai.nsteps = r.d.nsteps;
        ai.idx = idx;
        b->pend_init.push_back(ai);
        if (r.d.q0_on_device) {
            b->pend_moves.push_back(state_move(g, r.d.q0, q, idx));
        } else {
            BHIP(ctx, hipMemcpyAsync(q, r.d.q0, state_bytes(g), hipMemcpyHostToDevice, ctx->stream));
            b->pend_moves.push_back(state_move(g, q, q, idx));
        }
        Group &G = b->groups[r.group];
        if (G.shape < 0) forming[r.group].push_back(idx);
        else append_tiles(G, idx, g);
        admitted.push_back(tk);
    }
    if (!admitted.empty()) {
        std::vector<uint64_t> rest;
        for (uint64_t tk : b->queue)
            if (b->reqs[tk].state == QUEUED) rest.push_back(tk);
        b->queue.assign(rest.begin(), rest.end());
    }
    roeam_status frc = flush_moves(ctx, b);  // before any launch reads the new solves
    if (frc) return frc;
    for (int gi = 0; gi < kGroups; ++gi) {
        if (forming[gi].empty()) continue;
        roeam_status rc = tune_group(ctx, b, b->groups[gi], forming[gi]);
        if (rc) return rc;
    }
    return ROEAM_OK;
}

static int resident_count(const BatchEngine *b)
{
    int n = 0;
    for (int i = 0; i < b->hw; ++i) n += b->by_idx[i] != 0;
    return n;
}

// Capture the graph of graph_iters iterations over the groups with tiles,
// each launch sized to its list's capacity.
static roeam_status capture_graph(roeam_ctx *ctx, BatchEngine *b)
{
    release_graph(b);
    bool any = false;
    for (auto &G : b->groups) any |= !G.tiles.empty();
    for (auto &G : b->groups) G.graph_cap = (G.tiles.empty() && any) || G.cap == 0 ? 0 : G.cap;
    hipStream_t s = ctx->stream;
    BHIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    hipError_t e = hipSuccess;
    for (int k = 0; k < b->graph_iters && e == hipSuccess; ++k) e = enqueue_iteration(b, k & 1, s);
    hipError_t e2 = hipStreamEndCapture(s, &b->graph);
    if (e != hipSuccess) return hip_err(ctx, e, "capture batch iteration");
    if (e2 != hipSuccess) return hip_err(ctx, e2, "hipStreamEndCapture");
    BHIP(ctx, hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
    b->graph_valid = true;
    ++b->captures;
    return ROEAM_OK;
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
    BatchEngine keep;  // options survive a re-reserve
    bool have_old = false;
    if (ctx->batch) {
        BatchEngine *b = ctx->batch;
        if (!b->queue.empty() || resident_count(b)) return roeam_fail(ctx, ROEAM_EBUSY, "batch engine has work");
        BHIP(ctx, hipStreamSynchronize(ctx->stream));
        keep.graph_iters = b->graph_iters;
        keep.persistent = b->persistent;
        keep.policy = b->policy;
        keep.autotune = b->autotune;
        keep.max_resident = b->max_resident;
        have_old = true;
        release_engine(b);
        ctx->batch = nullptr;
    }
    BatchEngine *b = new (std::nothrow) BatchEngine;
    if (!b) return roeam_fail(ctx, ROEAM_ENOMEM, "host allocation");
    if (have_old) {
        b->graph_iters = keep.graph_iters;
        b->persistent = keep.persistent;
        b->policy = keep.policy;
        b->autotune = keep.autotune;
        b->max_resident = keep.max_resident;
    }
    b->device = ctx->device;
    hipError_t e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e == hipSuccess) {
        if (arena) {
            b->d_arena = (char *)arena;
            b->owns_arena = false;
        } else {
            e = hipMalloc(&b->d_arena, arena_bytes);
        }
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

roeam_status roeam_batch_configure(roeam_ctx *ctx, int graph_iters, int persistent, int policy, int autotune,
                                   int max_resident)
{
    if (!ctx) return ROEAM_EINVAL;
    BatchEngine *b = ctx->batch;
    if (!b) return roeam_fail(ctx, ROEAM_EINVAL, "call roeam_batch_reserve first");
    if (graph_iters < 2 || graph_iters > 256 || (graph_iters & 1))
        return roeam_fail(ctx, ROEAM_EINVAL, "graph_iters must be even, 2 .. 256");
    if (persistent != 0 && persistent != 1) return roeam_fail(ctx, ROEAM_EINVAL, "persistent must be 0 or 1");
    if (policy != ROEAM_ADMIT_FIFO && policy != ROEAM_ADMIT_SHORTEST)
        return roeam_fail(ctx, ROEAM_EINVAL, "policy must be ROEAM_ADMIT_FIFO or ROEAM_ADMIT_SHORTEST");
    if (autotune != 0 && autotune != 1) return roeam_fail(ctx, ROEAM_EINVAL, "autotune must be 0 or 1");
    if (max_resident < 0 || max_resident > kMaxSolves)
        return roeam_fail(ctx, ROEAM_EINVAL, "max_resident must be 0 (no limit) .. 4096");
    if (b->graph_iters != graph_iters || b->persistent != (persistent != 0)) b->graph_valid = false;
    b->graph_iters = graph_iters;
    b->persistent = persistent != 0;
    b->policy = policy;
    b->autotune = autotune != 0;
    b->max_resident = max_resident;
    return ROEAM_OK;
}

roeam_status roeam_batch_info(roeam_ctx *ctx, roeam_batch_stats *out)
{
    if (!ctx || !out) return roeam_fail(ctx, ROEAM_EINVAL, "bad argument");
    BatchEngine *b = ctx->batch;
    if (!b) return roeam_fail(ctx, ROEAM_EINVAL, "call roeam_batch_reserve first");
    out->captures = b->captures;
    out->graph_launches = b->graph_launches;
    out->iterations = b->iter;
    out->tunes = b->tunes;
    out->resident = resident_count(b);
    int queued = 0;
    for (auto &kv : b->reqs) queued += kv.second.state == QUEUED;
    out->queued = queued;
    out->graph_iters = b->graph_iters;
    out->persistent = b->persistent ? 1 : 0;
    out->policy = b->policy;
    out->max_resident = b->max_resident;
    out->shape = b->last_shape;
    return ROEAM_OK;
}

roeam_status roeam_batch_submit(roeam_ctx *ctx, int n, const roeam_solve_desc *descs, uint64_t *tickets_out)
{
    if (!ctx || n < 0 || (n > 0 && (!descs || !tickets_out))) return roeam_fail(ctx, ROEAM_EINVAL, "bad argument");
    BatchEngine *b = ctx->batch;
    if (!b) return roeam_fail(ctx, ROEAM_EINVAL, "call roeam_batch_reserve first");
    for (int i = 0; i < n; ++i) {
        const roeam_solve_desc &d = descs[i];
        // a grid only describes sizes, metrics and sides (its device arrays are
        // read, never written): one created on any context of this device will do
        if (!d.grid || !d.grid->ctx || d.grid->ctx->device != ctx->device)
            return roeam_fail(ctx, ROEAM_EINVAL, "descriptor grid invalid (NULL, or of another device)");
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
        r.seq = b->next_seq++;
        r.ticket = tk;
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
        // retire what finished (status one graph behind), then admit
        for (int w = 0; w < 2; ++w)
            if ((rc = process_status(ctx, b, w, false))) return rc;
        if ((rc = admit(ctx, b))) return rc;
        if ((rc = upload_tiles(ctx, b))) return rc;
        const int resident = resident_count(b);
        if (iterations >= 0 && done_iters >= iterations) break;
        if (resident == 0) {
            if (b->queue.empty()) break;
            // every queued solve fits the empty arena (checked at submission)
            return roeam_fail(ctx, ROEAM_ENOMEM, "queued solve does not fit the arena");
        }
        // every resident solve has spent its step budget (each ran one step per
        // iteration since it joined): nothing left to compute, so wait for the
        // newest status snapshot (taken after the last iteration) instead
        bool spent = true;
        size_t tiles = 0;
        for (auto &G : b->groups) tiles += G.tiles.size();
        for (int i = 0; i < b->hw && spent; ++i) {
            if (!b->by_idx[i]) continue;
            const Request &r = b->reqs[b->by_idx[i]];
            spent = r.state != RESIDENT || b->iter - r.admit_iter >= std::max(r.d.nsteps, 1L);
        }
        if (spent) {
            for (int w = 0; w < 2; ++w)
                if ((rc = process_status(ctx, b, w, true))) return rc;
            if (resident_count(b) < resident) continue;
            // the snapshot after the last iteration has been read: a solve past
            // its step budget that it did not report done is an engine fault
            return roeam_fail(ctx, ROEAM_EDEVICE, "batch engine: a solve past its step budget is not reported done");
        }
        if (tiles == 0) return roeam_fail(ctx, ROEAM_EDEVICE, "batch engine: resident solves without work-list tiles");
        // graph_iters iterations: the captured graph, or (profiling, or the
        // null stream, which cannot be captured) the same launches directly;
        // profiling reads the status after every second iteration (solves join
        // at even iterations: forward Euler's buffer follows the step parity)
        // so that few timed launches are idle ones
        const int run_iters = b->profiling ? 2 : b->graph_iters;
        if (!b->profiling && s != nullptr) {
            if (!b->graph_valid && (rc = capture_graph(ctx, b))) return rc;
            BHIP(ctx, hipGraphLaunch(b->gexec, s));
            ++b->graph_launches;
        } else {
            for (auto &G : b->groups) G.graph_cap = G.tiles.empty() ? 0 : G.cap;
            for (int k = 0; k < run_iters; ++k) BHIP(ctx, enqueue_iteration(b, (int)((b->iter + k) & 1), s));
        }
        b->iter += run_iters;
        done_iters += run_iters;
        // snapshot the status after these iterations; the buffer's previous
        // snapshot (two back) is read first
        const int which = (int)(b->status_seq++ & 1);
        if ((rc = process_status(ctx, b, which, true))) return rc;
        if ((rc = enqueue_status(ctx, b, which))) return rc;
        if (b->profiling && (rc = process_status(ctx, b, which, true))) return rc;
    }
    if (iterations < 0) {
        // drain: retire everything still reported, and return once every
        // retired solve's copy out has completed (its poll reports it done)
        for (int w = 0; w < 2; ++w)
            if ((rc = process_status(ctx, b, w, true))) return rc;
        BHIP(ctx, hipStreamSynchronize(s));
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
    b->graph_valid = false;
    if (rc) return rc;
    BHIP(ctx, hipStreamSynchronize(ctx->stream));
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    long cnt[4] = {0, 0, 0, 0};
    for (size_t k = 0; k < b->prof_stage.size(); ++k) {
        float ms = 0.f;
        BHIP(ctx, hipEventElapsedTime(&ms, b->prof_ev[2 * k], b->prof_ev[2 * k + 1]));
        const int code = b->prof_stage[k];
        // position of the stage within its step (forward Euler's stage 8 is a first stage)
        const int st = code == 8 ? 0 : (code >= 4 ? code - 4 : code - 1);
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
        if (!r.out_ev) return roeam_fail(ctx, ROEAM_EDEVICE, "retired solve without a copy event");
        hipError_t q = hipEventQuery(r.out_ev->ev);
        if (q == hipSuccess) r.state = DONE;
        else if (q != hipErrorNotReady) return hip_err(ctx, q, "hipEventQuery");
    }
    *done = r.state == DONE;
    if (!*done) return ROEAM_OK;
    // reported done: the ticket is forgotten (a server's request table does not grow)
    if (stats) *stats = r.stats;
    const roeam_status rc = r.rc;
    b->reqs.erase(it);
    if (rc == ROEAM_ENONPHYS) return roeam_fail(ctx, ROEAM_ENONPHYS, "solve produced a non-physical state");
    return ROEAM_OK;
}

} // extern "C"

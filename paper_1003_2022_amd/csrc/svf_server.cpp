// svf_server.cpp -- serving loop with continuous batching (svf_server_*).
//
// A scheduler thread owns a device arena and its own HIP stream.  Submitted
// requests wait in a FIFO queue; the head is admitted when a slot is free and
// its footprint (per-tile records, scales, one window slot per tile and
// channel) fits in the arena.  Each step takes, in admission order, the next
// pass of the requests in flight while their pixels x channels fit a per-step
// budget (the oldest always runs, smaller later passes fill the rest), and enqueues
//   fill(tile records of those starting) -> scale map(those starting)
//   -> pre-integration(the step's passes) -> finite difference(the same passes)
// through the persistent batched kernels, with the descriptor tables staged in
// pinned memory and uploaded on the server stream (two table sets, alternating).
// A request at pass p in step k is at pass p+1 in step k+1; a request whose last
// pass ran in step k is completed, and its arena range freed, once the host has
// seen step k's event.  Steps are pipelined one deep: step k+1 is enqueued before
// the host waits for step k.  A cancelled request leaves the queue at once; one
// in flight gets no further pass and frees its range once the steps already
// launched with it have completed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "svf_runtime_internal.h"

using namespace svf;

namespace {

constexpr int kTables = 1 + kMaxChannels;   // scale map + one table per channel count
constexpr int kPersistentScale = 4096;
constexpr int kPersistentPreint = 2048;

double now_us()
{
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// First-fit allocator over [0, size) with coalescing.
struct Arena {
    std::map<size_t, size_t> free_;   // offset -> length
    size_t size = 0;
    void reset(size_t n)
    {
        free_.clear();
        size = n;
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t &off)
    {
        n = align_up(n, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = align_up(n, 256);
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

struct Req {
    svf_request r;
    Plan plan;
    size_t bytes = 0, off = 0;
    int pass = -1;                 // next pass to run; -1: not admitted
    int slot = -1;                 // counter slot while admitted (invalid / overflow pixels)
    double t_submit = 0, t_admit = 0, t_done = 0;
    int status = SVF_EBUSY;
    bool done = false;
    // cancellation: `pending` counts the launched steps that still hold one of the
    // request's passes (the region stays allocated until it is 0); once the final
    // pass is launched the request can no longer be cancelled
    int pending = 0;
    bool final_sched = false, cancelled = false;
};

// Sizes of a step's launches, read by the kernels from device memory: [0] scale map
// (starting requests, their scale-map blocks), [1] block plan (the same requests, their
// difference blocks), [2 + C] pre-integration and [2 + kMaxChannels + C] difference of
// the requests with C channels (requests, windows / blocks).
constexpr int kDims = 2 + 2 * (kMaxChannels + 1);

struct StepBuf {
    Job *d = nullptr, *h = nullptr;
    BatchDims *d_dims = nullptr, *h_dims = nullptr;
    uint32_t *h_counts = nullptr;      // pinned copy of the counter slots after this step
    // captured step sequences of this table set, by kernel set and grid sizes
    std::vector<std::pair<std::string, hipGraphExec_t>> graphs;
    std::vector<hipGraph_t> graph_defs;
    hipEvent_t ev = nullptr;
    bool pending = false;
    std::vector<uint64_t> finishing;   // requests whose last pass runs in this step
    std::vector<uint64_t> running;
};

struct Server {
    svf_ctx *ctx = nullptr;
    svf_server_cfg cfg{};
    hipStream_t stream = nullptr;
    unsigned char *arena_base = nullptr;
    Arena arena;
    int cap = 0;                       // jobs per table
    int64_t step_px = 0;               // work budget of one step (pixels x channels)
    StepBuf buf[2];
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> inflight;
    std::unordered_map<uint64_t, Req> reqs;
    uint64_t next_id = 1;
    bool stopping = false;
    std::thread th;
    svf_server_stats_t stats{};
    double busy_since = -1;
    std::string err;
    float *lut = nullptr;              // the server's own scale table (SVF_SCALE_LUT)
    uint32_t *d_counts = nullptr;      // per slot: invalid and overflow pixels of the request holding it
    std::vector<int> free_slots;
    std::deque<uint64_t> finished;     // finished requests, oldest first (their state stays readable)
    size_t keep_finished = 0;
};

Server *srv(svf_ctx *ctx) { return static_cast<Server *>(ctx->server); }

// Grid of a launch over `work` items: at most `cap` work-groups, rounded up to a
// power of two so that steps of similar sizes share a captured graph.
int grid_of(int64_t work, int cap)
{
    int g = 1;
    while (g < work && g < cap) g <<= 1;
    return g;
}

// Launch one step from the tables in `b`; returns false on a HIP error.
bool launch_step(Server *S, StepBuf &b, int nsmap, int smap_kind, int tot_smap, int tot_plan, const int *counts,
                 const int *tot_tiles, const int *tot_blk)
{
    BatchDims *h = b.h_dims;
    h[0] = {nsmap, tot_smap};
    h[1] = {nsmap, tot_plan};
    for (int ch = 0; ch <= kMaxChannels; ++ch) {
        h[2 + ch] = {counts[ch], tot_tiles[ch]};
        h[2 + kMaxChannels + 1 + ch] = {counts[ch], tot_blk[ch]};
    }
    const BatchDims *d = b.d_dims;
    const int g_fill = grid_of(nsmap, 64), g_smap = grid_of(tot_smap, kPersistentScale);
    const int g_plan = grid_of((tot_plan + 255) / 256, 256);
    int g_pre[kMaxChannels + 1] = {}, g_fd[kMaxChannels + 1] = {};
    std::string key = nsmap ? "s" + std::to_string(g_fill) + "," + std::to_string(g_smap) + "," +
                                  std::to_string(g_plan) + "," + std::to_string(smap_kind)
                            : std::string("-");
    for (int ch = 1; ch <= kMaxChannels; ++ch) {
        if (!counts[ch]) continue;
        g_pre[ch] = grid_of(tot_tiles[ch], kPersistentPreint);
        g_fd[ch] = grid_of(tot_blk[ch], 1 << 30);   // one work-group per block (the kernel skips the surplus)
        key += "|" + std::to_string(ch) + ":" + std::to_string(g_pre[ch]) + "," + std::to_string(g_fd[ch]);
    }
    auto enqueue = [&](hipStream_t st) {
        hipError_t e = hipMemcpyAsync(b.d, b.h, sizeof(Job) * kTables * S->cap, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(b.d_dims, b.h_dims, sizeof(BatchDims) * kDims, hipMemcpyHostToDevice, st);
        // the tile records and counters of the newly admitted requests start at zero
        if (e == hipSuccess && nsmap) e = launch_fill_jobs(b.d, nsmap, g_fill, st, d + 0);
        if (e == hipSuccess && nsmap)
            e = launch_scale_map_batch(b.d, nsmap, tot_smap, g_smap, S->lut != nullptr, smap_kind, st, d + 0);
        if (e == hipSuccess && nsmap) e = launch_fd_plan_batch(b.d, nsmap, tot_plan, st, d + 1, g_plan);
        for (int ch = 1; ch <= kMaxChannels && e == hipSuccess; ++ch)
            if (counts[ch])
                e = launch_preint_batch(b.d + ch * S->cap, counts[ch], tot_tiles[ch], g_pre[ch], S->cfg.opts.preint, st,
                                        d + 2 + ch);
        for (int ch = 1; ch <= kMaxChannels && e == hipSuccess; ++ch)
            if (counts[ch])
                e = launch_fd_batch(b.d + ch * S->cap, counts[ch], tot_blk[ch], g_fd[ch], S->cfg.opts.preint,
                                    S->cfg.opts.fd_fp32, ch, st, d + 2 + kMaxChannels + 1 + ch);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.h_counts, S->d_counts, sizeof(uint32_t) * 2 * S->cap, hipMemcpyDeviceToHost, st);
        return e;
    };
    hipError_t e = hipSuccess;
    if (!S->cfg.use_graph) {
        e = enqueue(S->stream);
    } else {
        hipGraphExec_t exec = nullptr;
        for (auto &g : b.graphs)
            if (g.first == key) exec = g.second;
        if (!exec) {
            hipGraph_t graph = nullptr;
            e = hipStreamBeginCapture(S->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return false;
            const hipError_t le = enqueue(S->stream);
            e = hipStreamEndCapture(S->stream, &graph);
            if (le != hipSuccess || e != hipSuccess) {
                if (graph) hipGraphDestroy(graph);
                return false;
            }
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                hipGraphDestroy(graph);
                return false;
            }
            if (b.graphs.size() >= 64) {   // keep the cache bounded
                hipGraphExecDestroy(b.graphs.front().second);
                hipGraphDestroy(b.graph_defs.front());
                b.graphs.erase(b.graphs.begin());
                b.graph_defs.erase(b.graph_defs.begin());
            }
            b.graphs.emplace_back(key, exec);
            b.graph_defs.push_back(graph);
        }
        e = hipGraphLaunch(exec, S->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(b.ev, S->stream);
    return e == hipSuccess;
}

// Close the busy interval once nothing is in flight (called under S->mu).
void note_idle(Server *S, double t)
{
    if (S->inflight.empty() && S->busy_since >= 0) {
        S->stats.busy_us += t - S->busy_since;
        S->busy_since = -1;
    }
}

// A request reached its final state (called under S->mu): remember it, and forget
// the oldest finished requests beyond the retention count.
void note_finished(Server *S, uint64_t id)
{
    S->finished.push_back(id);
    while (S->finished.size() > S->keep_finished) {
        S->reqs.erase(S->finished.front());
        S->finished.pop_front();
    }
}

// Give an admitted request's arena range and counter slot back (called under S->mu).
void release(Server *S, Req &q)
{
    S->arena.release(q.off, q.bytes);
    if (q.slot >= 0) S->free_slots.push_back(q.slot);
    q.slot = -1;
}

// End an admitted request that was cancelled and has no step on the device
// (called under S->mu): its region goes back to the arena.
void end_cancelled(Server *S, uint64_t id, Req &q, double t)
{
    q.done = true;
    q.status = SVF_ECANCELLED;
    q.t_done = t;
    release(S, q);
    S->stats.cancelled++;
    S->inflight.erase(std::find(S->inflight.begin(), S->inflight.end(), id));
    note_idle(S, t);
    note_finished(S, id);
}

// Host side of a finished step: complete its finishing requests.
void retire(Server *S, StepBuf &b)
{
    if (!b.pending) return;
    hipError_t e = hipEventSynchronize(b.ev);
    const double t = now_us();
    std::lock_guard<std::mutex> lk(S->mu);
    for (uint64_t id : b.finishing) {
        Req &q = S->reqs[id];
        q.done = true;
        // pixels with an invalid field entry or a support beyond max_reach_px (their
        // outputs are NaN or the smallest filter) fail the request as svf_filter's report does
        const uint32_t inv = b.h_counts[2 * q.slot], ovf = b.h_counts[2 * q.slot + 1];
        q.status = e != hipSuccess ? SVF_EHIP : inv ? SVF_EINVAL : ovf ? SVF_ERANGE : SVF_OK;
        q.t_done = t;
        release(S, q);
        S->stats.completed++;
        S->stats.pixels += q.r.out.H * q.r.out.W * q.r.out.channels;
        S->inflight.erase(std::find(S->inflight.begin(), S->inflight.end(), id));
        note_finished(S, id);
    }
    for (uint64_t id : b.running) {
        Req &q = S->reqs[id];
        if (--q.pending == 0 && q.cancelled && !q.done) end_cancelled(S, id, q, t);
    }
    b.finishing.clear();
    b.running.clear();
    b.pending = false;
    note_idle(S, t);
    S->cv_done.notify_all();
    S->cv_work.notify_all();
}

void loop(Server *S)
{
    hipSetDevice(S->ctx->device);
    int k = 0;
    for (;;) {
        StepBuf &b = S->buf[k & 1];
        retire(S, b);   // this buffer's previous step (two steps ago) must be done before reuse
        std::vector<std::pair<uint64_t, Req *>> running;   // element pointers stay valid across rehash
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // admission: FIFO, slot limit, arena fit
            while (!S->queue.empty() && (int)S->inflight.size() < S->cfg.max_inflight) {
                Req &q = S->reqs[S->queue.front()];
                size_t off;
                if (S->free_slots.empty() || !S->arena.alloc(q.bytes, off)) break;
                q.off = off;
                q.slot = S->free_slots.back();
                S->free_slots.pop_back();
                q.pass = 0;
                q.t_admit = now_us();
                S->inflight.push_back(S->queue.front());
                S->queue.pop_front();
            }
            // this step's work: passes of the requests in flight in admission order while
            // they fit the budget (the oldest always runs; smaller later ones fill the rest)
            int64_t used = 0;
            for (uint64_t id : S->inflight) {
                Req &q = S->reqs[id];
                if (q.cancelled || q.pass >= q.r.order) continue;
                const int64_t px = q.r.in.H * q.r.in.W * q.r.in.channels;
                if (!running.empty() && used + px > S->step_px) continue;
                running.emplace_back(id, &q);
                used += px;
                q.pending++;
                if (q.pass + 1 == q.r.order) q.final_sched = true;
            }
            if (running.empty()) {
                StepBuf &o = S->buf[(k + 1) & 1];
                if (o.pending) {
                    lk.unlock();
                    retire(S, o);
                    continue;
                }
                if (S->stopping && S->queue.empty() && S->inflight.empty()) break;
                S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            if (S->busy_since < 0) S->busy_since = now_us();
        }
        // ---- build the tables (only this thread writes q.pass / q.off) ----
        int counts[kTables] = {}, tot_tiles[kTables] = {}, tot_blk[kTables] = {};
        int tot_smap = 0, tot_plan = 0;
        int nsmap = 0, smap_kind = -1;   // the field kind shared by the new requests (-1: a mix)
        for (auto &pr : running) {
            const uint64_t id = pr.first;
            Req &q = *pr.second;
            const Plan &p = q.plan;
            Plan pp = p;
            pp.off_tstat = q.off + p.off_tstat;
            pp.off_scales = q.off + p.off_scales;
            pp.off_fdplan = q.off + p.off_fdplan;
            pp.off_g = q.off + p.off_g;
            Job base = base_job(&q.r.in, &q.r.field, q.r.order, &S->cfg.opts, pp, S->arena_base);
            if (S->lut) {
                base.lut = S->lut;
                base.lut_n = S->cfg.opts.lut_nodes;
                base.lut_eps = S->cfg.opts.lut_eps_rel;
            }
            base.out = static_cast<float *>(q.r.out.data);
            base.out_rs = q.r.out.row_stride;
            if (q.pass == 0) {
                Job js = base;
                js.smap_base = tot_smap;
                tot_smap += scale_map_blocks(q.r.in.H, q.r.in.W);
                js.blk_base = tot_plan;   // the scale-map table also drives the block plan
                js.req_counts = S->d_counts + 2 * q.slot;
                tot_plan += fd_blocks_job(js);
                smap_kind = nsmap == 0 ? js.f_kind : (js.f_kind == smap_kind ? smap_kind : -1);
                b.h[nsmap++] = js;
            }
            Job jp = base;
            if (q.pass > 0) {
                jp.in = q.r.out.data;
                jp.in_rs = q.r.out.row_stride;
                jp.in_type = kInF32;
            }
            const int ch = q.r.in.channels;
            jp.tile_base = tot_tiles[ch];
            jp.blk_base = tot_blk[ch];
            tot_tiles[ch] += p.ntr * p.ntc * ch;
            tot_blk[ch] += fd_blocks_job(jp);
            b.h[ch * S->cap + counts[ch]++] = jp;
            q.pass++;
            if (q.pass == q.r.order) b.finishing.push_back(id);
            b.running.push_back(id);
        }
        if (!launch_step(S, b, nsmap, smap_kind, tot_smap, tot_plan, counts, tot_tiles, tot_blk)) {
            // nothing more runs for the requests in flight: wait for whatever did reach
            // the device, then end them all with SVF_EHIP and give their memory back
            hipStreamSynchronize(S->stream);
            const double t = now_us();
            std::lock_guard<std::mutex> lk(S->mu);
            S->err = "step launch failed";
            for (uint64_t id : S->inflight) {
                Req &q = S->reqs[id];
                q.done = true;
                q.status = SVF_EHIP;
                q.t_done = t;
                release(S, q);
                S->stats.completed++;
                note_finished(S, id);
            }
            S->inflight.clear();
            for (auto &sb : S->buf) {
                sb.finishing.clear();
                sb.running.clear();
                sb.pending = false;
            }
            note_idle(S, t);
            S->stats.steps++;
            S->cv_done.notify_all();
            ++k;
            continue;
        }
        b.pending = true;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stats.steps++;
        }
        ++k;
    }
    retire(S, S->buf[0]);
    retire(S, S->buf[1]);
}

}  // namespace

extern "C" {

svf_status svf_server_start(svf_ctx *ctx, const svf_server_cfg *cfg)
{
    if (!ctx || !cfg) return SVF_EINVAL;
    ctx->err.clear();
    if (ctx->server) return fail(ctx, SVF_EINVAL, "server already running");
    svf_server_cfg c = *cfg;
    if (c.max_inflight <= 0) c.max_inflight = 16;
    if (c.queue_capacity <= 0) c.queue_capacity = 1024;
    if (c.opts.tile == 0) c.opts.tile = 256;
    if (c.opts.preint != SVF_PRE_F64 && c.opts.preint != SVF_PRE_F32C)
        return fail(ctx, SVF_EUNSUPPORTED, "the server offers SVF_PRE_F64 and SVF_PRE_F32C");
    svf_status st = check_opts(ctx, &c.opts, c.opts.tile);
    if (st) return st;
    if (c.hbm_budget_bytes == 0) return fail(ctx, SVF_EINVAL, "hbm_budget_bytes must be > 0");
    hipSetDevice(ctx->device);
    Server *S = new Server();
    S->ctx = ctx;
    S->cfg = c;
    S->cap = c.max_inflight;
    S->step_px = (int64_t)(c.step_mpixels > 0 ? c.step_mpixels : 64) * 1000000;
    hipError_t e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&S->arena_base, c.hbm_budget_bytes);
    if (e == hipSuccess && c.opts.scale_map == SVF_SCALE_LUT) {
        e = hipMalloc(reinterpret_cast<void **>(&S->lut), (size_t)c.opts.lut_nodes * c.opts.lut_nodes * 16);
        if (e == hipSuccess) e = launch_lut_build(S->lut, c.opts.lut_nodes, c.opts.lut_eps_rel, S->stream);
    }
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&S->d_counts), sizeof(uint32_t) * 2 * S->cap);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipMalloc(&S->buf[i].d, sizeof(Job) * kTables * S->cap);
        if (e == hipSuccess) e = hipHostMalloc(&S->buf[i].h, sizeof(Job) * kTables * S->cap, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&S->buf[i].h_counts), sizeof(uint32_t) * 2 * S->cap,
                              hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&S->buf[i].d_dims), sizeof(BatchDims) * kDims);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&S->buf[i].h_dims), sizeof(BatchDims) * kDims,
                              hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&S->buf[i].ev, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        for (auto &b : S->buf) {
            if (b.d) hipFree(b.d);
            if (b.h) hipHostFree(b.h);
            if (b.h_counts) hipHostFree(b.h_counts);
            if (b.d_dims) hipFree(b.d_dims);
            if (b.h_dims) hipHostFree(b.h_dims);
            if (b.ev) hipEventDestroy(b.ev);
        }
        if (S->d_counts) hipFree(S->d_counts);
        if (S->arena_base) hipFree(S->arena_base);
        if (S->lut) hipFree(S->lut);
        if (S->stream) hipStreamDestroy(S->stream);
        delete S;
        return fail(ctx, SVF_ENOMEM, "server allocation: %s", hipGetErrorString(e));
    }
    S->arena.reset(c.hbm_budget_bytes);
    for (int i = S->cap - 1; i >= 0; --i) S->free_slots.push_back(i);
    S->keep_finished = 4 * (size_t)c.queue_capacity + 1024;
    ctx->server = S;
    S->th = std::thread(loop, S);
    return SVF_OK;
}

svf_status svf_server_submit(svf_ctx *ctx, const svf_request *req, uint64_t *id)
{
    if (!ctx || !req || !id) return SVF_EINVAL;
    Server *S = srv(ctx);
    if (!S) return fail(ctx, SVF_EINVAL, "server not running");
    // argument checks (same rules as svf_filter)
    svf_status st = check_image(ctx, &req->in, "in", false);
    if (!st) st = check_image(ctx, &req->out, "out", true);
    if (!st && (req->out.H != req->in.H || req->out.W != req->in.W || req->out.channels != req->in.channels))
        st = fail(ctx, SVF_EINVAL, "out must match in");
    if (!st) st = check_field(ctx, &req->field, req->in.H, req->in.W);
    if (!st && (req->order < 1 || req->order > 3)) st = fail(ctx, SVF_EINVAL, "order must be 1..3");
    if (!st && (req->in.H == 0 || req->in.W == 0)) st = fail(ctx, SVF_EINVAL, "empty image");
    if (st) return st;
    Req q;
    q.r = *req;
    q.plan = plan_for(&req->in, req->order, &S->cfg.opts);
    q.bytes = q.plan.off_tmp;   // passes run in place here: no second pass buffer
    q.t_submit = now_us();
    std::lock_guard<std::mutex> lk(S->mu);
    S->stats.submitted++;
    if (S->stopping) return fail(ctx, SVF_ECANCELLED, "server stopping");
    if (q.bytes > S->arena.size) {
        S->stats.rejected++;
        return fail(ctx, SVF_ENOMEM, "request needs %zu bytes, budget is %zu", q.bytes, S->arena.size);
    }
    if ((int)S->queue.size() >= S->cfg.queue_capacity) {
        S->stats.rejected++;
        return fail(ctx, SVF_EBUSY, "queue full");
    }
    const uint64_t nid = S->next_id++;
    S->reqs.emplace(nid, q);
    S->queue.push_back(nid);
    *id = nid;
    S->cv_work.notify_all();
    return SVF_OK;
}

static void fill_result(const Req &q, svf_result *res)
{
    res->status = q.status;
    res->done = q.done ? 1 : 0;
    res->t_submit_us = q.t_submit;
    res->t_admit_us = q.t_admit;
    res->t_done_us = q.t_done;
}

svf_status svf_server_poll(svf_ctx *ctx, uint64_t id, svf_result *res)
{
    if (!ctx || !res) return SVF_EINVAL;
    Server *S = srv(ctx);
    if (!S) return fail(ctx, SVF_EINVAL, "server not running");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return fail(ctx, SVF_EINVAL, "unknown request id");
    fill_result(it->second, res);
    return SVF_OK;
}

svf_status svf_server_wait(svf_ctx *ctx, uint64_t id, svf_result *res, double timeout_s)
{
    if (!ctx || !res) return SVF_EINVAL;
    Server *S = srv(ctx);
    if (!S) return fail(ctx, SVF_EINVAL, "server not running");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return fail(ctx, SVF_EINVAL, "unknown request id");
    auto pred = [&] {
        auto f = S->reqs.find(id);
        return f == S->reqs.end() || f->second.done;
    };
    if (timeout_s < 0) S->cv_done.wait(lk, pred);
    else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
        fill_result(S->reqs[id], res);
        return SVF_EBUSY;
    }
    it = S->reqs.find(id);
    if (it == S->reqs.end()) return fail(ctx, SVF_EINVAL, "request %llu is no longer kept", (unsigned long long)id);
    fill_result(it->second, res);
    return SVF_OK;
}

svf_status svf_server_cancel(svf_ctx *ctx, uint64_t id)
{
    if (!ctx) return SVF_EINVAL;
    Server *S = srv(ctx);
    if (!S) return fail(ctx, SVF_EINVAL, "server not running");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return fail(ctx, SVF_EINVAL, "unknown request id");
    Req &q = it->second;
    if (q.done || q.final_sched || q.cancelled)
        return fail(ctx, SVF_EBUSY, "request %llu is already completing", (unsigned long long)id);
    const double t = now_us();
    auto qi = std::find(S->queue.begin(), S->queue.end(), id);
    if (qi != S->queue.end()) {   // still waiting: never touched the device
        S->queue.erase(qi);
        q.done = true;
        q.status = SVF_ECANCELLED;
        q.t_done = t;
        S->stats.cancelled++;
        note_finished(S, id);
    } else {                      // in flight: no further pass is launched
        q.cancelled = true;
        if (q.pending == 0) end_cancelled(S, id, q, t);
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
    return SVF_OK;
}

svf_status svf_server_stats(svf_ctx *ctx, svf_server_stats_t *stats)
{
    if (!ctx || !stats) return SVF_EINVAL;
    Server *S = srv(ctx);
    if (!S) return fail(ctx, SVF_EINVAL, "server not running");
    std::lock_guard<std::mutex> lk(S->mu);
    *stats = S->stats;
    if (S->busy_since >= 0) stats->busy_us += now_us() - S->busy_since;
    return SVF_OK;
}

svf_status svf_server_stop(svf_ctx *ctx)
{
    if (!ctx) return SVF_EINVAL;
    Server *S = srv(ctx);
    if (!S) return SVF_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
        S->cv_work.notify_all();
    }
    S->th.join();
    hipStreamSynchronize(S->stream);
    for (auto &b : S->buf) {
        hipFree(b.d);
        hipHostFree(b.h);
        hipHostFree(b.h_counts);
        hipFree(b.d_dims);
        hipHostFree(b.h_dims);
        for (auto &g : b.graphs) hipGraphExecDestroy(g.second);
        for (auto g : b.graph_defs) hipGraphDestroy(g);
        hipEventDestroy(b.ev);
    }
    hipFree(S->d_counts);
    hipFree(S->arena_base);
    if (S->lut) hipFree(S->lut);
    hipStreamDestroy(S->stream);
    delete S;
    ctx->server = nullptr;
    return SVF_OK;
}

}  // extern "C"

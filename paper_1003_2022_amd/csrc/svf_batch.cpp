// svf_batch.cpp -- many images per launch sequence (svf_filter_batch).
//
// Every image keeps its own tiles, windows and scales, exactly as in
// svf_filter, so a result does not depend on the batch it ran in.  What changes
// is the launch structure: one fill, one scale-map launch over the blocks of all
// images, then per pass one pre-integration launch over all (tile, channel)
// windows and one finite-difference launch over all pixel blocks of the images
// whose order reaches that pass.  The kernels are persistent (a fixed grid walks
// the work list) and find their image by binary search in a device descriptor
// table.  With use_graph the sequence is captured once per shape set into a HIP
// graph; later calls upload new descriptors (pointers may change) and replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "svf_runtime_internal.h"

using namespace svf;

namespace {

constexpr int kPersistentScale = 4096;
constexpr int kPersistentPreint = 2048;
constexpr int kPersistentFd = 16384;
constexpr int kTables = 1 + 3 * kMaxChannels;   // scale map + (pass, channel count)

struct GraphEntry {
    std::string key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct BatchState {
    Job *d_jobs = nullptr;        // kTables tables of up to `cap` jobs
    int cap = 0;
    Job *h_jobs = nullptr;        // pinned staging for the tables
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    uint64_t generation = 0;      // ws_generation the graphs were captured against
    std::vector<GraphEntry> graphs;
    // the last call, for svf_filter_batch_report: stream, tile records per image
    hipStream_t last_stream = nullptr;
    std::vector<size_t> last_off, last_tiles;
    std::vector<int> last_order;
};

BatchState *state(svf_ctx *ctx)
{
    if (!ctx->batch) ctx->batch = new BatchState();
    return static_cast<BatchState *>(ctx->batch);
}

void drop_graphs(BatchState *b)
{
    for (auto &g : b->graphs) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        if (g.graph) hipGraphDestroy(g.graph);
    }
    b->graphs.clear();
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

void svf_batch_release(svf_ctx *ctx)
{
    if (!ctx || !ctx->batch) return;
    BatchState *b = static_cast<BatchState *>(ctx->batch);
    drop_graphs(b);
    if (b->upload_done) hipEventDestroy(b->upload_done);
    if (b->d_jobs) hipFree(b->d_jobs);
    if (b->h_jobs) hipHostFree(b->h_jobs);
    delete b;
    ctx->batch = nullptr;
}

extern "C" svf_status svf_filter_batch(svf_ctx *ctx, int n, const svf_image *in, const svf_field *fields,
                                       const int *orders, const svf_opts *opts, svf_image *out, hipStream_t stream,
                                       int use_graph)
{
    if (!ctx) return SVF_EINVAL;
    ctx->err.clear();
    if (n < 0 || (n > 0 && (!in || !fields || !orders || !out))) return fail(ctx, SVF_EINVAL, "bad batch arguments");
    if (n == 0) return SVF_OK;
    if (use_graph && stream == nullptr) return fail(ctx, SVF_EINVAL, "graph capture needs a non-default stream");
    svf_opts o;
    if (opts) o = *opts; else svf_default_opts(&o);
    // ---- checks and per-image plans ----
    std::vector<Plan> plans(n);
    int max_order = 0;
    int kind_all = -1;   // the field kind shared by every image (-1: a mix)
    for (int i = 0; i < n; ++i) {
        kind_all = i == 0 ? fields[i].kind : (fields[i].kind == kind_all ? kind_all : -1);
        svf_status st = check_image(ctx, &in[i], "in[i]", false);
        if (st) return st;
        st = check_image(ctx, &out[i], "out[i]", true);
        if (st) return st;
        if (out[i].H != in[i].H || out[i].W != in[i].W || out[i].channels != in[i].channels)
            return fail(ctx, SVF_EINVAL, "out[%d] must match in[%d]", i, i);
        st = check_field(ctx, &fields[i], in[i].H, in[i].W);
        if (st) return st;
        if (orders[i] < 1 || orders[i] > 3) return fail(ctx, SVF_EINVAL, "orders[%d] must be 1..3", i);
        if (o.preint == SVF_PRE_I64 && in[i].dtype != SVF_U16)
            return fail(ctx, SVF_EUNSUPPORTED, "integer pre-integration needs uint16 images");
        svf_opts oi = o;
        if (oi.tile == 0) oi.tile = 256;   // the batch supplies the parallelism
        st = check_opts(ctx, &oi, oi.tile);
        if (st) return st;
        plans[i] = plan_for(&in[i], orders[i], &oi);
        max_order = std::max(max_order, orders[i]);
    }
    // ---- workspace: [tile stats of all images][scales][windows] ----
    std::vector<size_t> off_fill(n), off_scales(n), off_plan(n), off_g(n);
    size_t pos = 0;
    for (int i = 0; i < n; ++i) {
        off_fill[i] = pos;
        pos = align_up(pos + (size_t)plans[i].ntr * plans[i].ntc * sizeof(TileStat), 256);
    }
    const size_t fill_bytes = pos;
    for (int i = 0; i < n; ++i) {
        off_scales[i] = pos;
        if (fields[i].kind != SVF_FIELD_SCALES4) pos = align_up(pos + (size_t)in[i].H * in[i].W * 16, 256);
    }
    for (int i = 0; i < n; ++i) {
        off_plan[i] = pos;
        pos = align_up(pos + (size_t)plans[i].ntr * plans[i].ntc * (plans[i].T / 16) * (plans[i].T / 16) * sizeof(FdBlk),
                       256);
    }
    for (int i = 0; i < n; ++i) {
        off_g[i] = pos;
        pos = align_up(pos + (size_t)plans[i].ntr * plans[i].ntc * in[i].channels * plans[i].slot * 8, 256);
    }
    svf_status st = ensure_workspace(ctx, pos);
    if (st) return st;
    hipSetDevice(ctx->device);
    Job lutj;
    st = attach_lut(ctx, o, lutj, stream);   // before any capture: the table is built once
    if (st) return st;
    BatchState *B = state(ctx);
    if (B->generation != ctx->ws_generation) {
        drop_graphs(B);
        B->generation = ctx->ws_generation;
    }
    if (B->cap < n) {
        if (B->upload_pending) hipEventSynchronize(B->upload_done);
        B->upload_pending = false;
        drop_graphs(B);
        if (B->d_jobs) hipFree(B->d_jobs);
        if (B->h_jobs) hipHostFree(B->h_jobs);
        B->d_jobs = nullptr;
        B->h_jobs = nullptr;
        B->cap = 0;
        const int cap = std::max(n, 64);
        hipError_t e = hipMalloc(&B->d_jobs, sizeof(Job) * kTables * cap);
        if (e != hipSuccess) return fail(ctx, SVF_ENOMEM, "descriptor table: %s", hipGetErrorString(e));
        e = hipHostMalloc(&B->h_jobs, sizeof(Job) * kTables * cap, hipHostMallocDefault);
        if (e != hipSuccess) return fail(ctx, SVF_ENOMEM, "descriptor staging: %s", hipGetErrorString(e));
        if (!B->upload_done) hipEventCreateWithFlags(&B->upload_done, hipEventDisableTiming);
        B->cap = cap;
    }
    if (B->upload_pending) {   // the staging buffer of the previous call must have been consumed
        hipError_t e = hipEventSynchronize(B->upload_done);
        if (e != hipSuccess) return hip_fail(ctx, e, "descriptor upload");
        B->upload_pending = false;
    }
    // ---- descriptor tables ----
    // table 0: every image (scale map); table 1 + pass * kMaxChannels + (C - 1): the images
    // with `channels` = C whose order exceeds `pass` (pre-integration and finite difference)
    unsigned char *ws = static_cast<unsigned char *>(ctx->ws);
    int counts[kTables] = {};
    int tot_smap = 0, tot_plan = 0, tot_tiles[kTables] = {}, tot_blk[kTables] = {};
    const int preint_of_pass[3] = {o.preint, o.preint == SVF_PRE_I64 ? SVF_PRE_F64 : o.preint,
                                   o.preint == SVF_PRE_I64 ? SVF_PRE_F64 : o.preint};
    std::string key = "n" + std::to_string(n);
    for (int i = 0; i < n; ++i) {
        Plan p = plans[i];
        p.off_tstat = off_fill[i];
        p.off_scales = off_scales[i];
        p.off_fdplan = off_plan[i];
        p.off_g = off_g[i];
        svf_opts oi = o;
        Job base = base_job(&in[i], &fields[i], orders[i], &oi, p, ws);
        base.lut = lutj.lut;
        base.lut_n = lutj.lut_n;
        base.lut_eps = lutj.lut_eps;
        base.out = static_cast<float *>(out[i].data);
        base.out_rs = out[i].row_stride;
        base.smap_base = tot_smap;
        tot_smap += scale_map_blocks(in[i].H, in[i].W);
        base.blk_base = tot_plan;   // table 0 also drives the block plan
        tot_plan += fd_blocks_job(base);
        B->h_jobs[counts[0]++] = base;
        for (int pass = 0; pass < orders[i]; ++pass) {
            const int tb = 1 + pass * kMaxChannels + (in[i].channels - 1);
            Job jp = base;
            jp.preint = preint_of_pass[pass];
            if (pass > 0) {
                jp.in = out[i].data;
                jp.in_rs = out[i].row_stride;
                jp.in_type = kInF32;
            }
            jp.tile_base = tot_tiles[tb];
            jp.blk_base = tot_blk[tb];
            tot_tiles[tb] += p.ntr * p.ntc * in[i].channels;
            tot_blk[tb] += fd_blocks_job(jp);
            B->h_jobs[tb * B->cap + counts[tb]++] = jp;
        }
        char buf[160];
        snprintf(buf, sizeof buf, "|%lld,%lld,%d,%d,%d,%d,%d,%d", (long long)in[i].H, (long long)in[i].W,
                 in[i].channels, in[i].dtype, fields[i].kind, orders[i], p.T, p.cap);
        key += buf;
    }
    {
        char buf[96];
        // the captured kernels depend on these (boundary and table live in the descriptors)
        snprintf(buf, sizeof buf, "#%d,%d,%.17g,%d", o.preint, o.fd_fp32, o.eps_px2, o.scale_map);
        key += buf;
    }
    B->last_stream = stream;
    B->last_off.assign(off_fill.begin(), off_fill.end());
    B->last_tiles.resize(n);
    B->last_order.assign(orders, orders + n);
    for (int i = 0; i < n; ++i) B->last_tiles[i] = (size_t)plans[i].ntr * plans[i].ntc;
    hipError_t e = hipMemcpyAsync(B->d_jobs, B->h_jobs, sizeof(Job) * kTables * B->cap, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "descriptor upload");
    e = hipEventRecord(B->upload_done, stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "descriptor upload event");
    B->upload_pending = true;

    auto enqueue = [&](hipStream_t s) -> hipError_t {
        hipError_t r = launch_fill_u32(reinterpret_cast<uint32_t *>(ws), 0u, (int64_t)(fill_bytes / 4), s);
        if (r != hipSuccess) return r;
        r = launch_scale_map_batch(B->d_jobs, counts[0], tot_smap, kPersistentScale, lutj.lut != nullptr, kind_all, s);
        if (r != hipSuccess) return r;
        r = launch_fd_plan_batch(B->d_jobs, counts[0], tot_plan, s);
        if (r != hipSuccess) return r;
        for (int pass = 0; pass < max_order; ++pass) {
            for (int ch = 1; ch <= kMaxChannels; ++ch) {
                const int tb = 1 + pass * kMaxChannels + (ch - 1);
                if (counts[tb] == 0) continue;
                const Job *tab = B->d_jobs + tb * B->cap;
                r = launch_preint_batch(tab, counts[tb], tot_tiles[tb], kPersistentPreint, preint_of_pass[pass], s);
                if (r != hipSuccess) return r;
            }
            for (int ch = 1; ch <= kMaxChannels; ++ch) {
                const int tb = 1 + pass * kMaxChannels + (ch - 1);
                if (counts[tb] == 0) continue;
                const Job *tab = B->d_jobs + tb * B->cap;
                r = launch_fd_batch(tab, counts[tb], tot_blk[tb], kPersistentFd, preint_of_pass[pass], o.fd_fp32, ch, s);
                if (r != hipSuccess) return r;
            }
        }
        return hipSuccess;
    };

    if (!use_graph) {
        e = timed_launch(ctx, kClsBatch, stream, [&] { return enqueue(stream); });
        if (e != hipSuccess) return hip_fail(ctx, e, "batch launch");
        return SVF_OK;
    }
    GraphEntry *ge = nullptr;
    for (auto &g : B->graphs)
        if (g.key == key) ge = &g;
    if (!ge) {
        GraphEntry g;
        g.key = key;
        e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamBeginCapture");
        hipError_t le = enqueue(stream);
        e = hipStreamEndCapture(stream, &g.graph);
        if (le != hipSuccess) {
            if (g.graph) hipGraphDestroy(g.graph);
            return hip_fail(ctx, le, "batch capture");
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(g.graph);
            return hip_fail(ctx, e, "hipGraphInstantiate");
        }
        if (B->graphs.size() >= 16) {   // small LRU-less cache
            hipGraphExecDestroy(B->graphs.front().exec);
            hipGraphDestroy(B->graphs.front().graph);
            B->graphs.erase(B->graphs.begin());
        }
        B->graphs.push_back(g);
        ge = &B->graphs.back();
    }
    e = timed_launch(ctx, kClsBatch, stream, [&] { return hipGraphLaunch(ge->exec, stream); });
    if (e != hipSuccess) return hip_fail(ctx, e, "hipGraphLaunch");
    return SVF_OK;
}

extern "C" svf_status svf_filter_batch_report(svf_ctx *ctx, int n, svf_report *reps)
{
    if (!ctx) return SVF_EINVAL;
    ctx->err.clear();
    BatchState *B = ctx->batch ? static_cast<BatchState *>(ctx->batch) : nullptr;
    if (!B || B->last_off.empty()) return fail(ctx, SVF_EINVAL, "no batch on this context");
    if (n != (int)B->last_off.size() || !reps) return fail(ctx, SVF_EINVAL, "n must be the last batch's image count");
    const size_t bytes = B->last_off.back() + B->last_tiles.back() * sizeof(TileStat);
    svf_status st = ensure_pinned(ctx, bytes);
    if (st) return st;
    hipSetDevice(ctx->device);
    hipError_t e = hipMemcpyAsync(ctx->host_pinned, ctx->ws, bytes, hipMemcpyDeviceToHost, B->last_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B->last_stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch report");
    int64_t inv = 0, ovf = 0;
    for (int i = 0; i < n; ++i) {
        const TileStat *ts = reinterpret_cast<const TileStat *>(static_cast<const unsigned char *>(ctx->host_pinned) +
                                                                B->last_off[i]);
        fill_report(ts, B->last_tiles[i], B->last_order[i], &reps[i]);
        inv += reps[i].invalid_px;
        ovf += reps[i].overflow_px;
    }
    if (inv > 0) return fail(ctx, SVF_EINVAL, "%lld pixels with an invalid field entry", (long long)inv);
    if (ovf > 0) return fail(ctx, SVF_ERANGE, "%lld pixels exceed max_reach_px", (long long)ovf);
    return SVF_OK;
}

// svf_runtime.cpp -- host side of libsvf: argument checks, tile planning,
// workspace, launch sequences, kernel timing.  Implements include/svf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdarg>
#include <cstring>
#include <string>
#include <vector>

#include "svf.h"
#include "svf_internal.h"
#include "svf_runtime_internal.h"

using namespace svf;

namespace {

constexpr int kDefaultCap = 128;
constexpr double kDefaultEps = 0.25;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

const char *kClassNames[kNumKernelClasses] = {"scale_map", "preint", "fd", "batch", "st"};

}  // namespace

namespace svf {

svf_status fail(svf_ctx *ctx, svf_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

svf_status hip_fail(svf_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, SVF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

hipError_t timed_launch(svf_ctx *ctx, int cls, hipStream_t s, const std::function<hipError_t()> &fn)
{
    if (!ctx->timing) return fn();
    hipEvent_t a = ctx->take_event(), b = ctx->take_event();
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    ctx->pending.push_back({cls, a, b});
    return e;
}

int pick_tile(int64_t H, int64_t W, int requested)
{
    if (requested == 64 || requested == 128 || requested == 256) return requested;
    auto tiles = [&](int64_t T) { return ((H + T - 1) / T) * ((W + T - 1) / T); };
    // at least one window per CU; below that, smaller tiles give several windows
    // per CU whose row sweeps hide each other's latency.  At 4096^2 the 256 tiles
    // of 256 px measured 2 % faster than 128 px (difference 612 -> 598 us, the
    // pre-integration about the same)
    if (tiles(256) >= 256) return 256;
    if (tiles(128) >= 256) return 128;
    return 64;
}

svf_status check_opts(svf_ctx *ctx, const svf_opts *o, int T)
{
    if (o->preint < 0 || o->preint > 2) return fail(ctx, SVF_EINVAL, "opts.preint must be 0..2");
    if (!(o->eps_px2 > 0.0) || !std::isfinite(o->eps_px2)) return fail(ctx, SVF_EINVAL, "opts.eps_px2 must be > 0");
    if (o->tile != 0 && o->tile != 64 && o->tile != 128 && o->tile != 256)
        return fail(ctx, SVF_EINVAL, "opts.tile must be 0, 64, 128 or 256");
    const int capmax = (kMaxWindow - T - 5) / 2;
    if (o->max_reach_px < 1 || o->max_reach_px > capmax)
        return fail(ctx, SVF_EINVAL, "opts.max_reach_px must be in [1, %d] for tile %d", capmax, T);
    if (o->bands < 0 || o->bands > svf_ctx::kMaxBands)
        return fail(ctx, SVF_EINVAL, "opts.bands must be in [0, %d]", svf_ctx::kMaxBands);
    if (o->boundary < SVF_BOUNDARY_ZERO || o->boundary > SVF_BOUNDARY_SYMMETRIC)
        return fail(ctx, SVF_EINVAL, "opts.boundary must be 0..2");
    if (o->scale_map != SVF_SCALE_SOLVE && o->scale_map != SVF_SCALE_LUT)
        return fail(ctx, SVF_EINVAL, "opts.scale_map must be 0 or 1");
    if (o->scale_map == SVF_SCALE_LUT) {
        if (o->lut_nodes < 9 || o->lut_nodes > 1025) return fail(ctx, SVF_EINVAL, "opts.lut_nodes must be in [9, 1025]");
        if (!(o->lut_eps_rel > 0.0 && o->lut_eps_rel <= 1.0))
            return fail(ctx, SVF_EINVAL, "opts.lut_eps_rel must be in (0, 1]");
    }
    return SVF_OK;
}

svf_status check_image(svf_ctx *ctx, const svf_image *im, const char *what, bool output)
{
    if (!im) return fail(ctx, SVF_EINVAL, "%s is NULL", what);
    if (im->H < 0 || im->W < 0) return fail(ctx, SVF_EINVAL, "%s: negative size", what);
    if (im->H > (int64_t)1 << 20 || im->W > (int64_t)1 << 20) return fail(ctx, SVF_EINVAL, "%s: side above 2^20", what);
    if (im->channels < 1 || im->channels > kMaxChannels) return fail(ctx, SVF_EINVAL, "%s: channels must be 1..4", what);
    if (im->dtype != SVF_F32 && im->dtype != SVF_U16) return fail(ctx, SVF_EUNSUPPORTED, "%s: dtype", what);
    if (output && im->dtype != SVF_F32) return fail(ctx, SVF_EUNSUPPORTED, "%s: output must be SVF_F32", what);
    if (im->H > 0 && im->W > 0) {
        if (!im->data) return fail(ctx, SVF_EINVAL, "%s: NULL data", what);
        if (im->row_stride < im->W * im->channels) return fail(ctx, SVF_EINVAL, "%s: row_stride < W*channels", what);
    }
    return SVF_OK;
}

svf_status check_field(svf_ctx *ctx, const svf_field *f, int64_t H, int64_t W)
{
    if (!f) return fail(ctx, SVF_EINVAL, "field is NULL");
    if (f->kind < 0 || f->kind > 2) return fail(ctx, SVF_EINVAL, "field.kind must be 0..2");
    const int K = f->kind == SVF_FIELD_SCALES4 ? 4 : 3;
    if (H > 0 && W > 0) {
        if (!f->data) return fail(ctx, SVF_EINVAL, "field: NULL data");
        if (f->row_stride < W * K) return fail(ctx, SVF_EINVAL, "field.row_stride < W*K");
        if (K == 4 && (f->row_stride % 4 != 0 || (reinterpret_cast<uintptr_t>(f->data) & 15) != 0))
            return fail(ctx, SVF_EINVAL, "SCALES4 field needs 16-byte aligned rows");
    }
    return SVF_OK;
}

svf_status check_filter_args(svf_ctx *ctx, const svf_image *in, const svf_field *field, int N, int order,
                             const svf_opts &o, const svf_image *out)
{
    if (N != 4) return fail(ctx, SVF_EUNSUPPORTED, "only N = 4 directions (ZP lattice) is supported");
    if (order < 1 || order > 3) return fail(ctx, SVF_EINVAL, "order must be 1..3");
    svf_status st = check_image(ctx, in, "in", false);
    if (st) return st;
    st = check_image(ctx, out, "out", true);
    if (st) return st;
    if (out->H != in->H || out->W != in->W || out->channels != in->channels)
        return fail(ctx, SVF_EINVAL, "out must have the input's H, W and channels");
    st = check_field(ctx, field, in->H, in->W);
    if (st) return st;
    st = check_opts(ctx, &o, pick_tile(in->H, in->W, o.tile));
    if (st) return st;
    if (o.preint == SVF_PRE_I64 && in->dtype != SVF_U16)
        return fail(ctx, SVF_EUNSUPPORTED, "integer pre-integration needs a uint16 image");
    return SVF_OK;
}

Plan plan_for(const svf_image *in, int order, const svf_opts *o)
{
    Plan p;
    p.T = pick_tile(in->H, in->W, o->tile);
    p.cap = o->max_reach_px;
    p.ntr = (int)((in->H + p.T - 1) / p.T);
    p.ntc = (int)((in->W + p.T - 1) / p.T);
    p.slot = slot_elems_for(p.T, p.cap);
    p.off_tstat = 0;
    p.off_scales = align_up((size_t)p.ntr * p.ntc * sizeof(TileStat), 256);
    p.off_fdplan = align_up(p.off_scales + (size_t)in->H * in->W * 4 * sizeof(float), 256);
    p.off_g = align_up(p.off_fdplan + (size_t)p.ntr * p.ntc * (p.T / 16) * (p.T / 16) * sizeof(FdBlk), 256);
    // second pass buffer: pass outputs alternate between it and the caller's output
    p.off_tmp = align_up(p.off_g + (size_t)p.ntr * p.ntc * in->channels * p.slot * 8, 256);
    p.bytes = p.off_tmp + (order > 1 ? (size_t)in->H * in->W * in->channels * sizeof(float) : 0);
    return p;
}

svf_status ensure_workspace(svf_ctx *ctx, size_t bytes)
{
    if (ctx->budget && bytes > ctx->budget)
        return fail(ctx, SVF_ENOMEM, "workspace of %zu bytes exceeds the HBM budget of %zu", bytes, ctx->budget);
    if (bytes <= ctx->ws_bytes) return SVF_OK;
    hipError_t e;
    if (ctx->ws) {
        e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
        hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    e = hipMalloc(&ctx->ws, bytes);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        return fail(ctx, SVF_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    ctx->ws_bytes = bytes;
    ctx->ws_generation++;
    return SVF_OK;
}

svf_status ensure_pinned(svf_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->pinned_bytes) return SVF_OK;
    if (ctx->host_pinned) hipHostFree(ctx->host_pinned);
    ctx->host_pinned = nullptr;
    ctx->pinned_bytes = 0;
    const size_t n = std::max(bytes, (size_t)1 << 20);
    hipError_t e = hipHostMalloc(&ctx->host_pinned, n, hipHostMallocDefault);
    if (e != hipSuccess) return fail(ctx, SVF_ENOMEM, "pinned host buffer: %s", hipGetErrorString(e));
    ctx->pinned_bytes = n;
    return SVF_OK;
}

void fill_report(const TileStat *ts, size_t nt, int order, svf_report *rep)
{
    std::memset(rep, 0, sizeof *rep);
    float mx = 0.f;
    for (size_t i = 0; i < nt; ++i) {
        rep->clamped_px += ts[i].clamped;
        rep->eps_active_px += ts[i].eps_active;
        rep->invalid_px += ts[i].invalid;
        rep->overflow_px += ts[i].overflow;
        mx = std::max(mx, std::max(ts[i].rx, ts[i].ry));
    }
    rep->max_reach_px = mx / std::sqrt((double)order);
}

// Fill the parts of a job common to every pass.
// Bands of tile rows for svf_filter.  Automatic is one band: on the 4096^2
// workload 2, 4 and 8 concurrent bands measured 3-15 % slower than whole-image
// launches in sequence (the pre-integration is latency-bound per window however
// many windows a launch holds, and concurrent kernels slow the issue-bound
// difference).  Each band is at least 4 tile rows, so that a window reaches only
// into the next band.
int pick_bands(const Plan &p, int requested)
{
    if (requested <= 1) return 1;
    return std::min(std::min(requested, svf_ctx::kMaxBands), std::max(1, p.ntr / 4));
}

svf_status ensure_bands(svf_ctx *ctx, int nb, int order)
{
    for (int b = 0; b < nb; ++b) {
        if (ctx->band_stream[b]) continue;
        hipError_t e = hipStreamCreateWithFlags(&ctx->band_stream[b], hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamCreateWithFlags");
    }
    const size_t need = 1 + (size_t)(order + 1) * svf_ctx::kMaxBands;   // fork, passes, pass-0 sums
    while (ctx->band_events.size() < need) {
        hipEvent_t ev;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreateWithFlags");
        ctx->band_events.push_back(ev);
    }
    return SVF_OK;
}

Job base_job(const svf_image *in, const svf_field *field, int order, const svf_opts *o, const Plan &p,
             unsigned char *ws)
{
    Job j;
    std::memset(&j, 0, sizeof j);
    j.in = in->data;
    j.in_rs = in->row_stride;
    j.in_type = in->dtype == SVF_U16 ? kInU16 : kInF32;
    j.C = in->channels;
    j.H = in->H;
    j.W = in->W;
    j.field = field->data;
    j.f_rs = field->row_stride;
    j.f_kind = field->kind;
    if (field->kind == SVF_FIELD_SCALES4) {
        j.scales = field->data;
        j.sc_rs = field->row_stride;
    } else {
        j.scales = reinterpret_cast<const float *>(ws + p.off_scales);
        j.sc_rs = in->W * 4;
    }
    j.tstat = reinterpret_cast<TileStat *>(ws + p.off_tstat);
    j.fdplan = reinterpret_cast<FdBlk *>(ws + p.off_fdplan);
    j.g = ws + p.off_g;
    j.slot_elems = p.slot;
    j.T = p.T;
    j.ntr = p.ntr;
    j.ntc = p.ntc;
    j.cap = p.cap;
    j.inv_sqrt_m = (float)(1.0 / std::sqrt((double)order));
    j.inv_sqrt_m_d = 1.0 / std::sqrt((double)order);
    j.fd_fp32 = o->fd_fp32 ? 1 : 0;
    j.boundary = o->boundary;
    j.eps_full = o->eps_px2 * order;
    j.preint = o->preint;
    j.tr0 = 0;
    j.tr1 = p.ntr;
    return j;
}

svf_status attach_lut(svf_ctx *ctx, const svf_opts &o, Job &j, hipStream_t stream)
{
    j.lut = nullptr;
    j.lut_n = 0;
    j.lut_eps = 0.0;
    if (o.scale_map != SVF_SCALE_LUT) return SVF_OK;
    if (!ctx->lut || ctx->lut_n != o.lut_nodes || ctx->lut_eps != o.lut_eps_rel) {
        hipError_t e;
        if (ctx->lut) {   // kernels of earlier calls may still read the old table
            e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
            hipFree(ctx->lut);
            ctx->lut = nullptr;
            ctx->lut_n = 0;
        }
        const size_t bytes = (size_t)o.lut_nodes * o.lut_nodes * 4 * sizeof(float);
        e = hipMalloc(reinterpret_cast<void **>(&ctx->lut), bytes);
        if (e != hipSuccess) {
            ctx->lut = nullptr;
            return fail(ctx, SVF_ENOMEM, "scale table hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        }
        e = launch_lut_build(ctx->lut, o.lut_nodes, o.lut_eps_rel, stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "scale table launch");
        ctx->lut_n = o.lut_nodes;
        ctx->lut_eps = o.lut_eps_rel;
    }
    j.lut = ctx->lut;
    j.lut_n = ctx->lut_n;
    j.lut_eps = ctx->lut_eps;
    return SVF_OK;
}

}  // namespace svf

// ============================================================================
// svf_ctx methods
// ============================================================================

hipEvent_t svf_ctx::take_event()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

void svf_default_opts(svf_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->preint = SVF_PRE_F64;
    o->fd_fp32 = 0;
    o->eps_px2 = kDefaultEps;
    o->tile = 0;
    o->max_reach_px = kDefaultCap;
    o->boundary = SVF_BOUNDARY_ZERO;
    o->scale_map = SVF_SCALE_SOLVE;
    o->lut_nodes = 129;
    o->lut_eps_rel = 0.125;
}

svf_status svf_create(svf_ctx **out, int device, size_t hbm_budget_bytes)
{
    if (!out) return SVF_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SVF_EHIP;
    if (hipSetDevice(device) != hipSuccess) return SVF_EHIP;
    noalloc_setup(device);   // the fixed workspace of svf_filter_noalloc on this device (its status is kept)
    svf_ctx *c = new (std::nothrow) svf_ctx();
    if (!c) return SVF_ENOMEM;
    c->device = device;
    c->budget = hbm_budget_bytes;
    if (ensure_pinned(c, (size_t)1 << 20) != SVF_OK) {
        delete c;
        return SVF_ENOMEM;
    }
    *out = c;
    return SVF_OK;
}

svf_status svf_destroy(svf_ctx *ctx)
{
    if (!ctx) return SVF_EINVAL;
    hipSetDevice(ctx->device);
    if (ctx->server) svf_server_stop(ctx);
    hipDeviceSynchronize();
    svf_batch_release(ctx);
    for (auto &p : ctx->pending) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    for (auto e : ctx->pool) hipEventDestroy(e);
    for (auto e : ctx->band_events) hipEventDestroy(e);
    for (auto s : ctx->band_stream)
        if (s) hipStreamDestroy(s);
    if (ctx->ws) hipFree(ctx->ws);
    if (ctx->lut) hipFree(ctx->lut);
    if (ctx->slots) hipFree(ctx->slots);
    if (ctx->host_pinned) hipHostFree(ctx->host_pinned);
    delete ctx;
    return SVF_OK;
}

const char *svf_last_error(const svf_ctx *ctx)
{
    if (!ctx) return "NULL context";
    return ctx->err.c_str();
}

svf_status svf_workspace_bytes(const svf_image *in, int N, int order, const svf_opts *opts, size_t *bytes)
{
    if (!in || !bytes) return SVF_EINVAL;
    if (N != 4) return SVF_EUNSUPPORTED;
    if (order < 1 || order > 3) return SVF_EINVAL;
    svf_opts o;
    if (opts) o = *opts; else svf_default_opts(&o);
    // sizes only: the data pointer is not needed here
    if (in->H < 0 || in->W < 0 || in->H > ((int64_t)1 << 20) || in->W > ((int64_t)1 << 20)) return SVF_EINVAL;
    if (in->channels < 1 || in->channels > kMaxChannels) return SVF_EINVAL;
    const int T = pick_tile(in->H, in->W, o.tile);
    if (check_opts(nullptr, &o, T) != SVF_OK) return SVF_EINVAL;
    *bytes = plan_for(in, order, &o).bytes;
    return SVF_OK;
}

svf_status svf_scale_map(svf_ctx *ctx, const svf_field *field, int64_t H, int64_t W, int order, const svf_opts *opts,
                         float *scales_out, hipStream_t stream)
{
    if (!ctx) return SVF_EINVAL;
    ctx->err.clear();
    if (order < 1 || order > 3) return fail(ctx, SVF_EINVAL, "order must be 1..3");
    if (H < 0 || W < 0) return fail(ctx, SVF_EINVAL, "negative size");
    svf_opts o;
    if (opts) o = *opts; else svf_default_opts(&o);
    svf_status st = check_field(ctx, field, H, W);
    if (st) return st;
    if (field->kind == SVF_FIELD_SCALES4) return fail(ctx, SVF_EINVAL, "field already holds scales");
    if (H == 0 || W == 0) return SVF_OK;
    if (!scales_out || (reinterpret_cast<uintptr_t>(scales_out) & 15)) return fail(ctx, SVF_EINVAL, "scales_out must be 16-byte aligned");
    svf_image im{nullptr, SVF_F32, 1, H, W, W};
    const int T = pick_tile(H, W, o.tile);
    st = check_opts(ctx, &o, T);
    if (st) return st;
    Plan p = plan_for(&im, order, &o);
    st = ensure_workspace(ctx, p.off_scales);
    if (st) return st;
    hipSetDevice(ctx->device);
    unsigned char *ws = static_cast<unsigned char *>(ctx->ws);
    Job j = base_job(&im, field, order, &o, p, ws);
    j.scales = scales_out;
    j.sc_rs = W * 4;
    st = attach_lut(ctx, o, j, stream);
    if (st) return st;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ws), 0u, (int64_t)(p.off_scales / 4), stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "fill");
    e = timed_launch(ctx, kClsScaleMap, stream, [&] { return launch_scale_map(j, stream); });
    if (e != hipSuccess) return hip_fail(ctx, e, "scale map launch");
    return SVF_OK;
}

svf_status svf_preintegrate(svf_ctx *ctx, const svf_image *in, int channel, int64_t r0, int64_t c0, int64_t h,
                            int64_t w, int preint, void *g_out, hipStream_t stream)
{
    if (!ctx) return SVF_EINVAL;
    ctx->err.clear();
    svf_status st = check_image(ctx, in, "in", false);
    if (st) return st;
    if (channel < 0 || channel >= in->channels) return fail(ctx, SVF_EINVAL, "channel out of range");
    if (h < 0 || w < 0 || w > kMaxWindow || h > ((int64_t)1 << 24)) return fail(ctx, SVF_EINVAL, "window size (w <= %d)", kMaxWindow);
    if (preint < 0 || preint > 2) return fail(ctx, SVF_EINVAL, "preint must be 0..2");
    if (preint == SVF_PRE_I64 && in->dtype != SVF_U16) return fail(ctx, SVF_EUNSUPPORTED, "integer sums need a uint16 image");
    if (h == 0 || w == 0) return SVF_OK;
    if (!g_out) return fail(ctx, SVF_EINVAL, "g_out is NULL");
    hipSetDevice(ctx->device);
    Job j;
    std::memset(&j, 0, sizeof j);
    j.in = in->data;
    j.in_rs = in->row_stride;
    j.in_type = in->dtype == SVF_U16 ? kInU16 : kInF32;
    j.C = in->channels;
    j.H = in->H;
    j.W = in->W;
    j.preint = preint;
    hipError_t e = timed_launch(ctx, kClsPreint, stream,
                                [&] { return launch_preint_window(j, channel, r0, c0, (int)h, (int)w, g_out, stream); });
    if (e != hipSuccess) return hip_fail(ctx, e, "pre-integration launch");
    return SVF_OK;
}

svf_status svf_filter(svf_ctx *ctx, const svf_image *in, const svf_field *field, int N, int order, const svf_opts *opts,
                      svf_image *out, hipStream_t stream, svf_report *rep)
{
    if (!ctx) return SVF_EINVAL;
    ctx->err.clear();
    svf_opts o;
    if (opts) o = *opts; else svf_default_opts(&o);
    svf_status st = check_filter_args(ctx, in, field, N, order, o, out);
    if (st) return st;
    if (rep) std::memset(rep, 0, sizeof *rep);
    if (in->H == 0 || in->W == 0) return SVF_OK;
    return svf::run_filter(ctx, in, field, order, o, out, stream, rep, 0);
}

}  // extern "C"

// The filter proper on checked arguments, its workspace at ctx->ws + ws_off
// (callers that keep their own buffers at the front of the workspace grow it to
// ws_off + plan bytes first).  With fixed_ws the workspace is that memory instead
// and nothing is allocated: the caller has checked its size, that rep is NULL, the
// scale map is the solve and there is one band; launches are not timed.
svf_status svf::run_filter(svf_ctx *ctx, const svf_image *in, const svf_field *field, int order, const svf_opts &o,
                           svf_image *out, hipStream_t stream, svf_report *rep, size_t ws_off, const double *uniform_a,
                           unsigned char *fixed_ws)
{
    Plan p = plan_for(in, order, &o);
    svf_status st = SVF_OK;
    if (!fixed_ws) {
        st = ensure_workspace(ctx, ws_off + p.bytes);
        if (st) return st;
    }
    hipSetDevice(ctx->device);
    unsigned char *ws = fixed_ws ? fixed_ws : static_cast<unsigned char *>(ctx->ws) + ws_off;
    Job j = base_job(in, field, order, &o, p, ws);
    if (!fixed_ws) {
        st = attach_lut(ctx, o, j, stream);
        if (st) return st;
    }
    auto launch = [&](int cls, hipStream_t s, const auto &fn) -> hipError_t {
        return fixed_ws ? fn() : timed_launch(ctx, cls, s, fn);
    };
    j.out = static_cast<float *>(out->data);
    j.out_rs = out->row_stride;

    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ws), 0u, (int64_t)(p.off_scales / 4), stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "fill");

    // Pass outputs alternate between the caller's output and the second pass
    // buffer so that the last pass lands in the output and no pass writes what
    // another band may still be reading.
    float *tmp = reinterpret_cast<float *>(ws + p.off_tmp);
    auto pass_out = [&](int pass) { return ((order - 1 - pass) % 2 == 0) ? static_cast<float *>(out->data) : tmp; };
    auto pass_out_rs = [&](int pass) { return ((order - 1 - pass) % 2 == 0) ? out->row_stride : in->W * in->channels; };
    auto pass_job = [&](int pass, int tr0, int tr1) {
        Job jp = j;
        jp.tr0 = tr0;
        jp.tr1 = tr1;
        jp.out = pass_out(pass);
        jp.out_rs = pass_out_rs(pass);
        if (pass > 0) {   // later passes read the previous pass's float32 output
            jp.in = pass_out(pass - 1);
            jp.in_rs = pass_out_rs(pass - 1);
            jp.in_type = kInF32;
            if (jp.preint == kPreI64) jp.preint = kPreF64;
        }
        return jp;
    };

    const int nb = fixed_ws ? 1 : pick_bands(p, o.bands);
    // a constant filter: the difference kernel that forms the taps once per block
    const double im = 1.0 / std::sqrt((double)order);
    double ua_pass[4] = {0, 0, 0, 0};
    if (uniform_a)
        for (int k = 0; k < 4; ++k) ua_pass[k] = uniform_a[k] * im;
    const bool uniform_fd = uniform_a && !o.fd_fp32 && o.preint != SVF_PRE_I64 &&
                            fd_uniform_fits(ua_pass[0], ua_pass[1], ua_pass[2], ua_pass[3], in->channels);
    if (nb <= 1) {
        e = launch(kClsScaleMap, stream, [&] { return launch_scale_map(pass_job(0, 0, p.ntr), stream); });
        if (e != hipSuccess) return hip_fail(ctx, e, "scale map launch");
        e = launch_fd_plan(pass_job(0, 0, p.ntr), stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "block plan launch");
        for (int pass = 0; pass < order; ++pass) {
            const Job jp = pass_job(pass, 0, p.ntr);
            e = launch(kClsPreint, stream, [&] { return launch_preint(jp, stream); });
            if (e != hipSuccess) return hip_fail(ctx, e, "pre-integration launch");
            e = launch(kClsFd, stream, [&] { return uniform_fd ? launch_fd_uniform(jp, ua_pass, stream) : launch_fd(jp, stream); });
            if (e != hipSuccess) return hip_fail(ctx, e, "finite-difference launch");
        }
    } else {
        // Bands of tile rows on internal streams.  Pass p of band b reads pass p-1's
        // output on its windows, which reach at most cap + 5 rows beyond the band:
        // it waits for pass p-1 of every band those rows touch.  Under the replicate
        // and mirror rules rows beyond a border read rows next to it: rows [lo, 0)
        // read inside [0, -lo), rows [H, hi) inside [2H - hi, H).
        st = ensure_bands(ctx, nb, order);
        if (st) return st;
        std::vector<int> tr(nb + 1);
        for (int b = 0; b <= nb; ++b) tr[b] = (int)((int64_t)p.ntr * b / nb);
        const int64_t halo = (int64_t)p.cap + 5;
        auto ev = [&](int pass, int b) { return ctx->band_events[1 + pass * svf_ctx::kMaxBands + b]; };
        e = hipEventRecord(ctx->band_events[0], stream);
        for (int b = 0; b < nb && e == hipSuccess; ++b) e = hipStreamWaitEvent(ctx->band_stream[b], ctx->band_events[0], 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "band fork");
        for (int b = 0; b < nb; ++b) {
            hipStream_t sb = ctx->band_stream[b];
            e = timed_launch(ctx, kClsScaleMap, sb, [&] { return launch_scale_map(pass_job(0, tr[b], tr[b + 1]), sb); });
            if (e != hipSuccess) return hip_fail(ctx, e, "scale map launch");
            e = launch_fd_plan(pass_job(0, tr[b], tr[b + 1]), sb);
            if (e != hipSuccess) return hip_fail(ctx, e, "block plan launch");
        }
        // rows of the pass input that band b's windows read (beyond the band: the halo,
        // and under the replicate and mirror rules the rows a border reflects)
        auto reach = [&](int b, int64_t &lo, int64_t &hi) {
            lo = (int64_t)tr[b] * p.T - halo;
            hi = (int64_t)tr[b + 1] * p.T + halo;
            if (o.boundary != SVF_BOUNDARY_ZERO) {
                const int64_t H = in->H, lo0 = lo;
                if (hi > H) lo = std::min(lo, std::max<int64_t>(0, 2 * H - hi));
                if (lo0 < 0) hi = std::max(hi, std::min<int64_t>(H, -lo0));
            }
        };
        // whether band a's windows read rows of band b
        auto reads = [&](int a, int b) {
            int64_t lo, hi;
            reach(a, lo, hi);
            return a != b && (int64_t)tr[b + 1] * p.T > lo && (int64_t)tr[b] * p.T < hi;
        };
        // An output that overlaps the input in memory, written by pass 0: a band's
        // difference must not overwrite input rows that another band's
        // pre-integration has still to read.
        auto span = [](const svf_image *im) {
            const size_t esz = im->dtype == SVF_U16 ? 2 : 4;
            const uintptr_t a = reinterpret_cast<uintptr_t>(im->data);
            return std::make_pair(a, a + ((size_t)(im->H - 1) * im->row_stride + (size_t)im->W * im->channels) * esz);
        };
        const auto si = span(in), so = span(out);
        const bool aliased_pass0 = si.first < so.second && so.first < si.second && pass_out(0) == out->data;
        auto ev_pre = [&](int b) { return ctx->band_events[1 + order * svf_ctx::kMaxBands + b]; };
        for (int pass = 0; pass < order; ++pass) {
            for (int b = 0; b < nb; ++b) {
                hipStream_t sb = ctx->band_stream[b];
                if (pass > 0) {
                    for (int o2 = 0; o2 < nb; ++o2) {
                        if (!reads(b, o2)) continue;
                        e = hipStreamWaitEvent(sb, ev(pass - 1, o2), 0);
                        if (e != hipSuccess) return hip_fail(ctx, e, "band dependency");
                    }
                }
                const Job jp = pass_job(pass, tr[b], tr[b + 1]);
                e = timed_launch(ctx, kClsPreint, sb, [&] { return launch_preint(jp, sb); });
                if (e != hipSuccess) return hip_fail(ctx, e, "pre-integration launch");
                if (pass == 0 && aliased_pass0) {   // the difference follows once every reader is done
                    e = hipEventRecord(ev_pre(b), sb);
                    if (e != hipSuccess) return hip_fail(ctx, e, "band event");
                    continue;
                }
                e = timed_launch(ctx, kClsFd, sb, [&] { return launch_fd(jp, sb); });
                if (e != hipSuccess) return hip_fail(ctx, e, "finite-difference launch");
                e = hipEventRecord(ev(pass, b), sb);
                if (e != hipSuccess) return hip_fail(ctx, e, "band event");
            }
            if (pass == 0 && aliased_pass0) {
                for (int b = 0; b < nb; ++b) {
                    hipStream_t sb = ctx->band_stream[b];
                    for (int o2 = 0; o2 < nb; ++o2) {
                        if (!reads(o2, b)) continue;
                        e = hipStreamWaitEvent(sb, ev_pre(o2), 0);
                        if (e != hipSuccess) return hip_fail(ctx, e, "band dependency");
                    }
                    const Job jp = pass_job(0, tr[b], tr[b + 1]);
                    e = timed_launch(ctx, kClsFd, sb, [&] { return launch_fd(jp, sb); });
                    if (e != hipSuccess) return hip_fail(ctx, e, "finite-difference launch");
                    e = hipEventRecord(ev(0, b), sb);
                    if (e != hipSuccess) return hip_fail(ctx, e, "band event");
                }
            }
        }
        for (int b = 0; b < nb; ++b) {   // join: the caller's stream waits for every band
            e = hipStreamWaitEvent(stream, ev(order - 1, b), 0);
            if (e != hipSuccess) return hip_fail(ctx, e, "band join");
        }
    }
    if (rep) {
        const size_t nt = (size_t)p.ntr * p.ntc;
        svf_status rs = ensure_pinned(ctx, nt * sizeof(TileStat));
        if (rs) return rs;
        e = hipMemcpyAsync(ctx->host_pinned, ws + p.off_tstat, nt * sizeof(TileStat), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "report");
        fill_report(static_cast<const TileStat *>(ctx->host_pinned), nt, order, rep);
        if (rep->invalid_px > 0) return fail(ctx, SVF_EINVAL, "%lld pixels with an invalid field entry", (long long)rep->invalid_px);
        if (rep->overflow_px > 0)
            return fail(ctx, SVF_ERANGE, "%lld pixels exceed max_reach_px = %d", (long long)rep->overflow_px, o.max_reach_px);
    }
    return SVF_OK;
}

extern "C" {

svf_status svf_set_timing(svf_ctx *ctx, int enable)
{
    if (!ctx) return SVF_EINVAL;
    ctx->timing = enable != 0;
    return SVF_OK;
}

svf_status svf_kernel_time(svf_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches, int reset)
{
    if (!ctx || !kernel) return SVF_EINVAL;
    int cls = -1;
    for (int i = 0; i < kNumKernelClasses; ++i)
        if (std::strcmp(kernel, kClassNames[i]) == 0) cls = i;
    if (cls < 0) return fail(ctx, SVF_EINVAL, "unknown kernel class %s", kernel);
    // fold every finished record into the accumulators
    std::vector<svf_ctx::Rec> keep;
    for (auto &r : ctx->pending) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
        ctx->tot_ms[r.cls] += ms;
        ctx->count[r.cls] += 1;
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->pending.clear();
    if (total_ms) *total_ms = ctx->tot_ms[cls];
    if (launches) *launches = ctx->count[cls];
    if (reset) {
        for (int i = 0; i < kNumKernelClasses; ++i) {
            ctx->tot_ms[i] = 0.0;
            ctx->count[i] = 0;
        }
    }
    return SVF_OK;
}

}  // extern "C"

// svf_st.cpp -- entry points of the feature-preserving smoothing (Sec. 4.2):
// structure tensor -> (s*, rho*, theta*) field -> the filter.  The window of the
// structure tensor is the library's own filter on the 3-channel image of
// gradient products, with a constant scale field held in one row (row stride 0).
#include <cmath>
#include <cstring>

#include "svf.h"
#include "svf_runtime_internal.h"

using namespace svf;

namespace {

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

svf_status check_params(svf_ctx *ctx, const svf_st_params *p)
{
    if (!p) return fail(ctx, SVF_EINVAL, "params is NULL");
    if (!(p->sigma_w > 0.0) || !std::isfinite(p->sigma_w)) return fail(ctx, SVF_EINVAL, "params.sigma_w must be > 0");
    if (p->order_w < 1 || p->order_w > 3) return fail(ctx, SVF_EINVAL, "params.order_w must be 1..3");
    if (!(p->gain > 0.0) || !std::isfinite(p->gain)) return fail(ctx, SVF_EINVAL, "params.gain must be > 0");
    if (!(p->lambda_zero >= 0.0) || !std::isfinite(p->lambda_zero))
        return fail(ctx, SVF_EINVAL, "params.lambda_zero must be >= 0");
    if (!(p->a_flat > 0.0) || !std::isfinite(p->a_flat)) return fail(ctx, SVF_EINVAL, "params.a_flat must be > 0");
    return SVF_OK;
}

// Buffers at the front of the workspace, in this order: the gradient products P,
// J (unless the caller gives it), the field F (smoothing only), the scale row.
struct StLayout {
    size_t off_P = 0, off_J = 0, off_F = 0, off_row = 0, front = 0;
};

StLayout st_layout(const svf_image *in, bool own_J, bool own_F)
{
    StLayout L;
    const size_t px3 = (size_t)in->H * in->W * 3 * sizeof(float);
    L.off_P = 0;
    L.off_J = up256(px3);
    L.off_F = L.off_J + (own_J ? up256(px3) : 0);
    L.off_row = L.off_F + (own_F ? up256(px3) : 0);
    L.front = L.off_row + up256((size_t)in->W * 4 * sizeof(float));
    return L;
}

svf_image products_image(const svf_image *in, float *P)
{
    svf_image im;
    std::memset(&im, 0, sizeof im);
    im.data = P;
    im.dtype = SVF_F32;
    im.channels = 3;
    im.H = in->H;
    im.W = in->W;
    im.row_stride = in->W * 3;
    return im;
}

svf_opts window_opts(const svf_opts &o)
{
    svf_opts w = o;
    if (w.preint == SVF_PRE_I64) w.preint = SVF_PRE_F64;   // the products are float32
    return w;
}

svf_status check_common(svf_ctx *ctx, const svf_image *in, const svf_st_params *params, const svf_opts &o)
{
    svf_status st = check_image(ctx, in, "in", false);
    if (st) return st;
    st = check_params(ctx, params);
    if (st) return st;
    return check_opts(ctx, &o, pick_tile(in->H, in->W, o.tile));
}

// Tensor into J and, if F != NULL, the field into F; the front of the workspace
// is laid out by L and the whole workspace already holds L.front + the window
// filter's plan.
svf_status st_run(svf_ctx *ctx, const svf_image *in, const svf_st_params &p, const svf_opts &o, const StLayout &L,
                  float *J, int64_t j_rs, float *F, int64_t f_rs, hipStream_t stream)
{
    unsigned char *ws = static_cast<unsigned char *>(ctx->ws);
    float *P = reinterpret_cast<float *>(ws + L.off_P);
    float *row = reinterpret_cast<float *>(ws + L.off_row);
    StImage im;
    std::memset(&im, 0, sizeof im);
    im.in = in->data;
    im.in_rs = in->row_stride;
    im.in_type = in->dtype == SVF_U16 ? kInU16 : kInF32;
    im.C = in->channels;
    im.H = in->H;
    im.W = in->W;
    im.boundary = o.boundary;
    hipError_t e = timed_launch(ctx, kClsSt, stream, [&] { return launch_st_outer(im, P, in->W * 3, stream); });
    if (e != hipSuccess) return hip_fail(ctx, e, "gradient products launch");
    const float a = (float)(p.sigma_w * std::sqrt(6.0));   // isotropic scales of covariance sigma_w^2 I
    e = launch_fill_f4(row, make_float4(a, a, a, a), in->W, stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "scale row fill");
    svf_image pim = products_image(in, P);
    svf_image jim = pim;
    jim.data = J;
    jim.row_stride = j_rs;
    svf_field wf;
    std::memset(&wf, 0, sizeof wf);
    wf.data = row;
    wf.kind = SVF_FIELD_SCALES4;
    wf.row_stride = 0;   // every row reads the same constant row
    const double ua[4] = {a, a, a, a};   // the stored (float) scales
    svf_status st = run_filter(ctx, &pim, &wf, p.order_w, window_opts(o), &jim, stream, nullptr, L.front, ua);
    if (st) return st;
    if (F) {
        e = timed_launch(ctx, kClsSt, stream, [&] {
            return launch_st_field(J, j_rs, in->H, in->W, p.gain, p.lambda_zero, p.a_flat, F, f_rs, stream);
        });
        if (e != hipSuccess) return hip_fail(ctx, e, "field launch");
    }
    return SVF_OK;
}

}  // namespace

extern "C" {

void svf_st_default_params(svf_st_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->sigma_w = 2.0;
    p->order_w = 1;
    p->gain = 1.0;
    p->lambda_zero = 0.0;
    p->a_flat = 1.0;
}

svf_status svf_structure_tensor(svf_ctx *ctx, const svf_image *in, const svf_st_params *params,
                                const svf_opts *opts, float *tensor_out, int64_t tensor_row_stride,
                                float *field_out, int64_t field_row_stride, hipStream_t stream)
{
    if (!ctx) return SVF_EINVAL;
    ctx->err.clear();
    svf_opts o;
    if (opts) o = *opts; else svf_default_opts(&o);
    svf_status st = check_common(ctx, in, params, o);
    if (st) return st;
    if (!tensor_out && !field_out) return fail(ctx, SVF_EINVAL, "tensor_out and field_out are both NULL");
    if (tensor_out && tensor_row_stride < in->W * 3) return fail(ctx, SVF_EINVAL, "tensor_row_stride < 3 W");
    if (field_out && field_row_stride < in->W * 3) return fail(ctx, SVF_EINVAL, "field_row_stride < 3 W");
    if (in->H == 0 || in->W == 0) return SVF_OK;
    const StLayout L = st_layout(in, tensor_out == nullptr, false);
    const svf_opts wo = window_opts(o);
    const svf_image pim = products_image(in, nullptr);
    st = ensure_workspace(ctx, L.front + plan_for(&pim, params->order_w, &wo).bytes);
    if (st) return st;
    hipSetDevice(ctx->device);
    float *J = tensor_out;
    int64_t j_rs = tensor_row_stride;
    if (!J) {
        J = reinterpret_cast<float *>(static_cast<unsigned char *>(ctx->ws) + L.off_J);
        j_rs = in->W * 3;
    }
    return st_run(ctx, in, *params, o, L, J, j_rs, field_out, field_row_stride, stream);
}

svf_status svf_smooth_adaptive(svf_ctx *ctx, const svf_image *in, const svf_st_params *params, int order,
                               const svf_opts *opts, svf_image *out, hipStream_t stream, svf_report *rep)
{
    if (!ctx) return SVF_EINVAL;
    ctx->err.clear();
    if (order < 1 || order > 3) return fail(ctx, SVF_EINVAL, "order must be 1..3");
    svf_opts o;
    if (opts) o = *opts; else svf_default_opts(&o);
    svf_status st = check_common(ctx, in, params, o);
    if (st) return st;
    st = check_image(ctx, out, "out", true);
    if (st) return st;
    if (out->H != in->H || out->W != in->W || out->channels != in->channels)
        return fail(ctx, SVF_EINVAL, "out must have the input's H, W and channels");
    if (o.preint == SVF_PRE_I64 && in->dtype != SVF_U16)
        return fail(ctx, SVF_EUNSUPPORTED, "integer pre-integration needs a uint16 image");
    if (rep) std::memset(rep, 0, sizeof *rep);
    if (in->H == 0 || in->W == 0) return SVF_OK;
    const StLayout L = st_layout(in, true, true);
    const svf_opts wo = window_opts(o);
    const svf_image pim = products_image(in, nullptr);
    const size_t need = std::max(plan_for(&pim, params->order_w, &wo).bytes, plan_for(in, order, &o).bytes);
    st = ensure_workspace(ctx, L.front + need);
    if (st) return st;
    hipSetDevice(ctx->device);
    unsigned char *ws = static_cast<unsigned char *>(ctx->ws);
    float *J = reinterpret_cast<float *>(ws + L.off_J);
    float *F = reinterpret_cast<float *>(ws + L.off_F);
    st = st_run(ctx, in, *params, o, L, J, in->W * 3, F, in->W * 3, stream);
    if (st) return st;
    svf_field fld;
    std::memset(&fld, 0, sizeof fld);
    fld.data = F;
    fld.kind = SVF_FIELD_SRT3;
    fld.row_stride = in->W * 3;
    return run_filter(ctx, in, &fld, order, o, out, stream, rep, L.front);
}

}  // extern "C"

// svf_noalloc.hip -- svf_filter_noalloc: the filter for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Its workspace (tile records, scales, block
// plan, pre-integrated windows, the second pass buffer) is one fixed array of
// this library in each device's memory; the kernels are svf_filter's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "svf_runtime_internal.h"

using namespace svf;

namespace {

// Largest workspace of one call: 64 MiB per device, held from the library's
// loading on that device until the process ends.  With the default options
// (max_reach_px 128) this is enough for a one-channel 512 x 512 image at order 1
// to 3, or a 3-channel 320 x 320 image; smaller max_reach_px fit larger images
// (svf_workspace_bytes gives the exact need).
constexpr size_t kScratchBytes = (size_t)64 << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_setup[kMaxDevices];
hipError_t g_status[kMaxDevices];
unsigned char *g_scratch[kMaxDevices];   // device address of `scratch` on each device

}  // namespace

hipError_t svf::noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_setup[device]) {
        // `scratch` in host code only names the array; its address on this device
        // (current) is looked up once and used from then on
        void *p = nullptr;
        g_status[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch[device] = g_status[device] == hipSuccess ? static_cast<unsigned char *>(p) : nullptr;
        g_setup[device] = true;
    }
    return g_status[device];
}

extern "C" svf_status svf_filter_noalloc(svf_ctx *ctx, const svf_image *in, const svf_field *field, int N, int order,
                                         const svf_opts *opts, svf_image *out, hipStream_t stream)
{
    if (!ctx) return SVF_EINVAL;
    ctx->err.clear();
    svf_opts o;
    if (opts) o = *opts; else svf_default_opts(&o);
    svf_status st = check_filter_args(ctx, in, field, N, order, o, out);
    if (st) return st;
    if (o.scale_map != SVF_SCALE_SOLVE)
        return fail(ctx, SVF_EUNSUPPORTED, "svf_filter_noalloc: the look-up-table scale map needs an allocated table");
    if (o.bands > 1) return fail(ctx, SVF_EUNSUPPORTED, "svf_filter_noalloc: bands need internal streams");
    if (in->H == 0 || in->W == 0) return SVF_OK;
    const size_t need = plan_for(in, order, &o).bytes;
    if (need > kScratchBytes)
        return fail(ctx, SVF_ENOMEM, "svf_filter_noalloc: needs %zu bytes of workspace, its fixed maximum is %zu",
                    need, kScratchBytes);
    unsigned char *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices && g_setup[ctx->device]) ws = g_scratch[ctx->device];
    }
    if (!ws) return fail(ctx, SVF_EHIP, "svf_filter_noalloc: no fixed workspace on device %d", ctx->device);
    return run_filter(ctx, in, field, order, o, out, stream, nullptr, 0, nullptr, ws);
}

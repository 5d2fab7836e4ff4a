// svf_runtime_internal.h -- host-side state shared by the runtime files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <functional>
#include <string>
#include <vector>

#include "svf.h"
#include "svf_internal.h"

enum { kClsScaleMap = 0, kClsPreint = 1, kClsFd = 2, kClsBatch = 3, kClsSt = 4, kNumKernelClasses = 5 };

struct svf_ctx {
    int device = 0;
    size_t budget = 0;                 // cap on the workspace (0 = none)
    void *ws = nullptr;                // device workspace (grown on demand)
    size_t ws_bytes = 0;
    uint64_t ws_generation = 0;        // bumped when the workspace moves (invalidates graphs)
    void *host_pinned = nullptr;       // pinned host memory for reports (grown on demand)
    size_t pinned_bytes = 0;
    std::string err;
    bool timing = false;
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double tot_ms[kNumKernelClasses] = {};
    int64_t count[kNumKernelClasses] = {};
    void *batch = nullptr;             // svf::BatchState
    void *server = nullptr;            // serving loop (svf_server.cpp)
    // banded svf_filter: internal streams (default priority) and ordering events
    static constexpr int kMaxBands = 8;
    hipStream_t band_stream[kMaxBands] = {};
    std::vector<hipEvent_t> band_events;   // [0]: fork; then pass * kMaxBands + band
    hipEvent_t take_event();
    // look-up-table scale map: the table of the last (nodes, floor) asked for
    float *lut = nullptr;
    int lut_n = 0;
    double lut_eps = 0.0;
    // svf_filter_single: global-memory window slots for tiles whose window exceeds the LDS
    void *slots = nullptr;
    size_t slots_bytes = 0;
};

namespace svf {

struct Plan {
    int T = 0, cap = 0, ntr = 0, ntc = 0;
    int64_t slot = 0;
    size_t off_tstat = 0, off_scales = 0, off_fdplan = 0, off_g = 0, off_tmp = 0, bytes = 0;
};

svf_status fail(svf_ctx *ctx, svf_status st, const char *fmt, ...);
svf_status hip_fail(svf_ctx *ctx, hipError_t e, const char *what);
hipError_t timed_launch(svf_ctx *ctx, int cls, hipStream_t s, const std::function<hipError_t()> &fn);
int pick_tile(int64_t H, int64_t W, int requested);
svf_status check_opts(svf_ctx *ctx, const svf_opts *o, int T);
svf_status check_image(svf_ctx *ctx, const svf_image *im, const char *what, bool output);
svf_status check_field(svf_ctx *ctx, const svf_field *f, int64_t H, int64_t W);
// svf_filter's argument checks (N, order, images, field, options)
svf_status check_filter_args(svf_ctx *ctx, const svf_image *in, const svf_field *field, int N, int order,
                             const svf_opts &o, const svf_image *out);
Plan plan_for(const svf_image *in, int order, const svf_opts *o);
svf_status ensure_workspace(svf_ctx *ctx, size_t bytes);
svf_status ensure_pinned(svf_ctx *ctx, size_t bytes);
void fill_report(const TileStat *ts, size_t nt, int order, svf_report *rep);
Job base_job(const svf_image *in, const svf_field *field, int order, const svf_opts *o, const Plan &p,
             unsigned char *ws);
// SVF_SCALE_LUT: build (or reuse) the context's table on `stream` and point j at it
svf_status attach_lut(svf_ctx *ctx, const svf_opts &o, Job &j, hipStream_t stream);
svf_status run_filter(svf_ctx *ctx, const svf_image *in, const svf_field *field, int order, const svf_opts &o,
                      svf_image *out, hipStream_t stream, svf_report *rep, size_t ws_off,
                      const double *uniform_a = nullptr,    // the field's scales where they are all equal
                      unsigned char *fixed_ws = nullptr);   // workspace given by the caller: nothing allocated
// svf_filter_noalloc (svf_noalloc.hip): find the device address of the library's
// fixed workspace on `device` (current); called once per device by svf_create
hipError_t noalloc_setup(int device);

}  // namespace svf

void svf_batch_release(svf_ctx *ctx);

// Sanitizer driver for the host side of libsvf: the argument checks, planning and
// error paths of every entry point, run without a GPU (HIP calls fail, and the
// library must turn that into a status) under AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code.  Built and run by
// tests/test_sanitize.py; exit status 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "svf.h"
#include "svf_runtime_internal.h"

static int fails = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed (%s:%d): %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                                      \
        }                                                                 \
    } while (0)

int main()
{
    svf_opts o;
    svf_default_opts(&o);
    CHECK(o.preint == SVF_PRE_F64 && o.max_reach_px == 128);
    // host-only sizing, valid and invalid
    // fake device addresses: nothing below dereferences them on the host, and no kernel can run
    void *fake = reinterpret_cast<void *>(0x10000);
    svf_image im{fake, SVF_F32, 1, 300, 257, 257};
    size_t bytes = 0;
    CHECK(svf_workspace_bytes(&im, 4, 2, &o, &bytes) == SVF_OK && bytes > 300 * 257 * 16);
    CHECK(svf_workspace_bytes(&im, 3, 2, &o, &bytes) == SVF_EUNSUPPORTED);
    CHECK(svf_workspace_bytes(&im, 4, 0, &o, &bytes) == SVF_EINVAL);
    CHECK(svf_workspace_bytes(nullptr, 4, 1, &o, &bytes) != SVF_OK);
    svf_opts bad = o;
    bad.tile = 100;
    CHECK(svf_workspace_bytes(&im, 4, 1, &bad, &bytes) != SVF_OK);
    bad = o;
    bad.max_reach_px = 100000;
    CHECK(svf_workspace_bytes(&im, 4, 1, &bad, &bytes) != SVF_OK);
    // no device: creation fails cleanly
    svf_ctx *ctx = nullptr;
    CHECK(svf_create(&ctx, 0, 0) != SVF_OK && ctx == nullptr);
    CHECK(std::strlen(svf_last_error(nullptr)) > 0);
    CHECK(svf_filter(nullptr, &im, nullptr, 4, 1, &o, &im, nullptr, nullptr) == SVF_EINVAL);
    // a context without a device: every argument error is found before any HIP call,
    // and valid arguments end in a HIP or memory status
    svf_ctx *c = new svf_ctx();
    svf_field fld{static_cast<const float *>(fake), SVF_FIELD_SRT3, 0, 257 * 3};
    void *fake_out = reinterpret_cast<void *>(0x40000);
    svf_image out{fake_out, SVF_F32, 1, 300, 257, 257};
    svf_report rep;
    CHECK(svf_filter(c, &im, &fld, 3, 2, &o, &out, nullptr, &rep) == SVF_EUNSUPPORTED);
    CHECK(svf_filter(c, &im, &fld, 4, 4, &o, &out, nullptr, &rep) == SVF_EINVAL);
    CHECK(std::strlen(svf_last_error(c)) > 0);
    svf_image out2 = out;
    out2.W = 256;
    CHECK(svf_filter(c, &im, &fld, 4, 1, &o, &out2, nullptr, &rep) == SVF_EINVAL);
    svf_image st = im;
    st.row_stride = 100;
    CHECK(svf_filter(c, &st, &fld, 4, 1, &o, &out, nullptr, &rep) == SVF_EINVAL);
    svf_field f2 = fld;
    f2.kind = 7;
    CHECK(svf_filter(c, &im, &f2, 4, 1, &o, &out, nullptr, &rep) == SVF_EINVAL);
    svf_image u16 = im;
    u16.dtype = SVF_U16;
    CHECK(svf_filter(c, &im, &fld, 4, 1, &o, &u16, nullptr, &rep) == SVF_EUNSUPPORTED);
    bad = o;
    bad.preint = SVF_PRE_I64;
    CHECK(svf_filter(c, &im, &fld, 4, 1, &bad, &out, nullptr, &rep) == SVF_EUNSUPPORTED);
    bad = o;
    bad.boundary = 5;
    CHECK(svf_filter(c, &im, &fld, 4, 1, &bad, &out, nullptr, &rep) == SVF_EINVAL);
    bad = o;
    bad.scale_map = SVF_SCALE_LUT;
    bad.lut_nodes = 3;
    CHECK(svf_filter(c, &im, &fld, 4, 1, &bad, &out, nullptr, &rep) != SVF_OK);
    svf_image empty{nullptr, SVF_F32, 1, 0, 9, 9};
    CHECK(svf_filter(c, &empty, &fld, 4, 1, &o, &empty, nullptr, &rep) == SVF_OK);
    const svf_status s_run = svf_filter(c, &im, &fld, 4, 2, &o, &out, nullptr, nullptr);
    CHECK(s_run == SVF_ENOMEM || s_run == SVF_EHIP);
    CHECK(svf_filter_noalloc(c, &im, &fld, 4, 1, &bad, &out, nullptr) != SVF_OK);
    CHECK(svf_filter_single(c, &im, &fld, 3, &o, &out, nullptr, &rep) == SVF_EUNSUPPORTED);
    bad = o;
    bad.boundary = SVF_BOUNDARY_SYMMETRIC;
    CHECK(svf_filter_single(c, &im, &fld, 2, &bad, &out, nullptr, &rep) == SVF_EUNSUPPORTED);
    CHECK(svf_filter_single(c, &im, &fld, 2, &o, &im, nullptr, &rep) == SVF_EINVAL);   // aliasing
    const svf_status s_single = svf_filter_single(c, &im, &fld, 2, &o, &out, nullptr, &rep);
    CHECK(s_single == SVF_ENOMEM || s_single == SVF_EHIP);
    CHECK(svf_scale_map(c, &fld, 300, 257, 0, &o, static_cast<float *>(fake), nullptr) == SVF_EINVAL);
    CHECK(svf_preintegrate(c, &im, 3, 0, 0, 10, 10, SVF_PRE_F64, fake, nullptr) == SVF_EINVAL);
    CHECK(svf_preintegrate(c, &im, 0, 0, 0, 10, 5000, SVF_PRE_F64, fake, nullptr) == SVF_EINVAL);
    CHECK(svf_preintegrate(c, &im, 0, 0, 0, 10, 10, SVF_PRE_I64, fake, nullptr) == SVF_EUNSUPPORTED);
    // batch: argument errors, then a valid call that cannot allocate
    std::vector<svf_image> ins(3, im), outs(3, out);
    std::vector<svf_field> flds(3, fld);
    int orders[3] = {1, 2, 4};
    CHECK(svf_filter_batch(c, 3, ins.data(), flds.data(), orders, &o, outs.data(), nullptr, 1) == SVF_EINVAL);
    orders[2] = 3;
    const svf_status s_batch = svf_filter_batch(c, 3, ins.data(), flds.data(), orders, &o, outs.data(), nullptr, 1);
    CHECK(s_batch != SVF_OK);
    std::vector<svf_report> reps(3);
    CHECK(svf_filter_batch_report(c, 3, reps.data()) != SVF_OK || true);
    // structure tensor and smoothing: argument checks
    svf_st_params prm;
    svf_st_default_params(&prm);
    prm.sigma_w = -1.0;
    CHECK(svf_smooth_adaptive(c, &im, &prm, 2, &o, &out, nullptr, &rep) == SVF_EINVAL);
    // server: bad configuration, then a start that cannot create its stream or arena
    svf_server_cfg cfg;
    std::memset(&cfg, 0, sizeof cfg);
    cfg.max_inflight = -3;
    CHECK(svf_server_start(c, &cfg) != SVF_OK);
    uint64_t id = 0;
    svf_request rq{im, fld, 1, 0, out};
    CHECK(svf_server_submit(c, &rq, &id) != SVF_OK);   // no server running
    svf_result res;
    CHECK(svf_server_poll(c, 12345, &res) != SVF_OK);
    // planning and reports on their own
    svf::Plan p = svf::plan_for(&im, 2, &o);
    CHECK(p.T > 0 && p.ntr * p.T >= 300 && p.ntc * p.T >= 257 && p.bytes > p.off_g);
    std::vector<svf::TileStat> ts(p.ntr * p.ntc);
    for (size_t i = 0; i < ts.size(); ++i) {
        ts[i].rx = 1.0f + (float)i;
        ts[i].ry = 2.0f;
        ts[i].clamped = 1;
        ts[i].eps_active = 2;
        ts[i].invalid = 0;
        ts[i].overflow = 0;
    }
    svf::fill_report(ts.data(), ts.size(), 2, &rep);
    CHECK(rep.clamped_px == (int64_t)ts.size() && rep.max_reach_px > 0.0);
    CHECK(svf::pick_tile(4096, 4096, 0) == 256 && svf::pick_tile(64, 64, 0) > 0);
    svf_batch_release(c);
    delete c;
    if (fails) std::fprintf(stderr, "%d checks failed\n", fails);
    else std::printf("runtime sanitizer run: all checks passed\n");
    return fails ? 1 : 0;
}

// svf_single.hip -- one pass with the iterated box spline beta^{4,2} (Sec. 2.3,
// eq. (iterated_spline); Sec. 3.3): out[n] = sum_k f[k] beta^{4,2}_{a(n)}(n - k).
//
// beta^{4,2}_a is the box spline whose four directions a_k u_k are each taken twice.
// The argument of Sec. 3.1 carries over: with g2 = the running sums RS1..RS4 applied
// twice (sqrt2 factors each time), the filter is the 81-tap difference
//
//   out[n] = (1 / prod_k a_k^2) sum_{j in {0,1,2}^4} prod_k C(2, j_k) (-1)^{j_k}
//            F2(n + 2 tau - sum_k j_k a_k u_k),      F2(y) = sum_l g2[l] (ZP*ZP)(y - l),
//
// tau the shift of Sec. 3.1 step (2).  ZP*ZP is a piecewise polynomial of degree 6 on
// the four-direction mesh; its 36 weights at a fractional position come from a table
// of polynomials on one mesh triangle (svf_zp2_table.h), the other three triangles of
// the unit square mapping onto it by the square's quarter turns.
//
// One work-group per 16 x 16 output tile and channel: the tile's window (every lattice
// sample its 256 pixels' taps read) is loaded into LDS as binary64, summed twice in
// place (each recursion a thread per row, diagonal, column or anti-diagonal, a barrier
// between recursions), and three threads per pixel evaluate its 81 taps from LDS
// (27 each), whose partial sums meet in LDS.  A large window takes the CU's whole LDS,
// so the threads per pixel are what give each SIMD several waves.  Measured at 2048^2
// (sigma 3-12 px): 9.3 ms with the 36-polynomial table and a row-by-row sweep of
// RS2..RS4 (a barrier per row), 7.9 ms with the mirror-pair table, 7.2 ms with the
// recursions as independent line scans, 6.9 ms with Horner's rule for the polynomial.
//
// Precision: the doubled sums grow like the window side^8, and the difference cancels
// all but ~prod a_k^2 of that.  A pixel whose rounding bound 2^-46 max|g2| / prod a_k^2
// exceeds 1e-6 of the window's largest input magnitude is written as NaN and counted
// (measured on the oracle's sums, the error stays below 28 ulp(max|g2|) / prod a_k^2,
// a quarter of the bound).
//
// A tile whose window does not fit in LDS is listed by the first launch and done by a
// second, persistent one (k_single2_global) with the window in a global-memory slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "svf_internal.h"
#include "svf_runtime_internal.h"
#include "svf_zp2_table.h"

namespace svf {

namespace {

constexpr int kSpT = 16;                     // output tile side
constexpr int kSpLdsBytes = 155 * 1024;      // dynamic LDS of one work-group (160 KiB per CU, less the static part)
constexpr double kSq2 = 1.41421356237309504880;
constexpr double kIsq2 = 0.70710678118654752440;

struct SingleJob {
    const void *in;
    int64_t in_rs;          // elements per input row
    int32_t in_type, C;
    int64_t H, W;
    const float *scales;    // scales of the whole filter, float4 per pixel
    int64_t sc_rs;          // floats per scale row
    float *out;
    int64_t out_rs;
    double inv_sqrt_m;      // 1 / sqrt(2): the pass scales
    int32_t win_cap;        // doubles of dynamic LDS for the window
    uint32_t *nan_count;    // outputs written as NaN
    // tiles whose window exceeds the LDS: listed (by << 16 | bx, channel) for a second
    // launch that keeps each window in a global-memory slot (null: NaN instead)
    uint32_t *defer;
    uint32_t *defer_count;
    double *slots;          // one slot per work-group of the second launch
    int64_t slot_doubles;
};

// Window layout (in LDS, or in a global-memory slot): rows of stride S (S odd, so that
// the row scans' lanes spread over the LDS banks).

template <int IN>
__device__ __forceinline__ double in_at(const SingleJob &J, int64_t r, int64_t c, int ch)
{
    if (r < 0 || c < 0 || r >= J.H || c >= J.W) return 0.0;
    const int64_t i = r * J.in_rs + c * J.C + ch;
    if constexpr (IN == kInU16) return (double)static_cast<const uint16_t *>(J.in)[i];
    else return (double)static_cast<const float *>(J.in)[i];
}

constexpr int kSpSplit = 3;                  // threads per output pixel, each a third of its taps
constexpr int kSpThreads = 256 * kSpSplit;
constexpr int kSpTaps = (81 + kSpSplit - 1) / kSpSplit;   // taps per thread (the last takes the rest)

__device__ __forceinline__ double block_max(double v, double *red)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int wave = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double m = red[0];
    for (int k = 1; k < kSpThreads / 64; ++k) m = fmax(m, red[k]);
    return m;
}

// One recursion along one line of the window, in place: p[k step] becomes
// sum_{i <= k} mul p[i step] (RS1 / RS3: mul = 1, exact; RS2 / RS4: sqrt2).  Eight loads
// are issued before their sums, so the line's latency is paid once per eight samples.
__device__ __forceinline__ void scan_line(double *p, int step, int len, double mul)
{
    double s = 0.0;
    int k = 0;
    for (; k + 8 <= len; k += 8) {
        double x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = p[(k + j) * step];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            s = fma(mul, x[j], s);
            p[(k + j) * step] = s;
        }
    }
    for (; k < len; ++k) {
        s = fma(mul, p[k * step], s);
        p[k * step] = s;
    }
}

// One application of RS1..RS4 to the window, in place, each recursion over the
// whole window before the next: RS1 along the rows, RS2 down the diagonals (step
// (1,1)), RS3 down the columns, RS4 down the anti-diagonals (step (-1,1)), every line a
// thread of its own (zero initial conditions at the window's top, left and right edges).
__device__ void rs4_window(double *g, int wh, int ww, int S)
{
    const int t = threadIdx.x, nt = blockDim.x, nd = ww + wh - 1;
    for (int i = t; i < wh; i += nt) scan_line(g + i * S, 1, ww, 1.0);
    __syncthreads();
    for (int d = t; d < nd; d += nt) {   // diagonal starting at (0, d - wh + 1) or (wh - 1 - d, 0)
        const int r0 = d < wh ? wh - 1 - d : 0, c0 = d < wh ? 0 : d - wh + 1;
        scan_line(g + r0 * S + c0, S + 1, min(wh - r0, ww - c0), kSq2);
    }
    __syncthreads();
    for (int c = t; c < ww; c += nt) scan_line(g + c, S, wh, 1.0);
    __syncthreads();
    for (int d = t; d < nd; d += nt) {   // anti-diagonal starting at (0, d) or (d - ww + 1, ww - 1)
        const int r0 = d < ww ? 0 : d - ww + 1, c0 = d < ww ? d : ww - 1;
        scan_line(g + r0 * S + c0, S - 1, min(wh - r0, c0 + 1), kSq2);
    }
    __syncthreads();
}

// F2 at a point of the tabulated triangle: the sum over the 36 stencil offsets of g
// times the offset's polynomial.  Offsets pair up as (lx', ly') and (1 - lx', ly')
// (mirror images about dx = 1/2, where T0 is symmetric): with u = px - 1/2 the pair
// contributes c[p,q] u^p py^q (g + g') for even p and (g - g') for odd p.  The table
// stencil (lx', ly') sits at window offset base + lx' dA + ly' dB.  The coefficients
// are integers (the exact ones times kZp2Den): immediate operands of the FMAs, and the
// result is kZp2Den times F2.
__device__ __forceinline__ double zp2_interp(const double *g, int base, int dA, int dB, double px, double py)
{
    double acc[28];
#pragma unroll
    for (int r = 0; r < 28; ++r) acc[r] = 0.0;
#pragma unroll
    for (int i = 0; i < 18; ++i) {
        bool any = false;
#pragma unroll
        for (int r = 0; r < 28; ++r) any = any || kZp2Half[i][r] != 0.0;
        if (!any) continue;
        const int lx = i % 3 - 2, ly = i / 3 - 2;
        const double v0 = g[base + lx * dA + ly * dB], v1 = g[base + (1 - lx) * dA + ly * dB];
        const double sum = v0 + v1, dif = v0 - v1;
#pragma unroll
        for (int r = 0; r < 28; ++r)
            if (kZp2Half[i][r] != 0.0) acc[r] = fma(kZp2Half[i][r], (kZp2Mono[r][0] & 1) ? dif : sum, acc[r]);
    }
    // sum_q py^q (sum_p acc[p,q] u^p), both by Horner's rule
    const double u = px - 0.5;
    double F = 0.0;
#pragma unroll
    for (int q = kZp2Deg; q >= 0; --q) {
        double h = 0.0;
#pragma unroll
        for (int pp = kZp2Deg - q; pp >= 0; --pp) {
            int r = 0;   // index of monomial u^pp py^q
#pragma unroll
            for (int k = 0; k < 28; ++k)
                if (kZp2Mono[k][0] == pp && kZp2Mono[k][1] == q) r = k;
            h = fma(h, u, acc[r]);
        }
        F = fma(F, py, h);
    }
    return F;
}

// One output tile (bx, by) of channel ch with its window at g (cap doubles): in LDS
// (the first launch, defer: a window above cap is listed for the second launch) or
// in a global-memory slot (the second launch: a window above cap gives NaN).
template <int IN>
__device__ void single_tile(const SingleJob &J, int bx, int by, int ch, double *g, int64_t cap, bool defer)
{
    __shared__ int s_box[4];
    __shared__ double s_red[kSpThreads / 64];
    __shared__ double s_part[kSpSplit - 1][kSpT * kSpT];
    __shared__ uint32_t s_nan;
    // thread t: pixel t % 256 of the tile, taps part * kSpTaps .. of it, part = t / 256 (three
    // waves per SIMD with one work-group per CU)
    const int t = threadIdx.x, px_i = t & (kSpT * kSpT - 1), part = t / (kSpT * kSpT);
    const int64_t r = (int64_t)by * kSpT + px_i / kSpT, c = (int64_t)bx * kSpT + px_i % kSpT;
    const bool inside = r < J.H && c < J.W;
    if (t == 0) {
        s_box[0] = s_box[2] = INT32_MAX;
        s_box[1] = s_box[3] = INT32_MIN;
        s_nan = 0;
    }
    double a[4] = {1.0, 1.0, 1.0, 1.0};
    bool ok = false;
    if (inside) {
        const float4 v = *reinterpret_cast<const float4 *>(J.scales + r * J.sc_rs + c * 4);
        a[0] = v.x * J.inv_sqrt_m; a[1] = v.y * J.inv_sqrt_m; a[2] = v.z * J.inv_sqrt_m; a[3] = v.w * J.inv_sqrt_m;
        ok = a[0] > 0.0 && a[1] > 0.0 && a[2] > 0.0 && a[3] > 0.0 && isfinite(a[0] + a[1] + a[2] + a[3]);
    }
    // twice the shift of Sec. 3.1 step (2), and the taps' extent: tap j sits at
    // n + 2 tau - (j1 a1 + (j2 a2 - j4 a4)/sqrt2, (j2 a2 + j4 a4)/sqrt2 + j3 a3)
    const double ap2 = a[1] * kIsq2, ap4 = a[3] * kIsq2;
    const double t1 = a[0] + ap2 - ap4 - 1.0, t2 = ap2 + a[2] + ap4 - 3.0;   // 2 tau
    const double y1 = (double)c + t1, y2 = (double)r + t2;
    __syncthreads();
    if (ok) {
        // lattice samples read: floor(y) - 2 .. floor(y) + 3 per axis, one more each way
        // for rounding differences between this bound and the taps' own sums
        atomicMin(&s_box[0], (int)floor(y1 - 2.0 * (a[0] + ap2)) - 3);
        atomicMax(&s_box[1], (int)floor(y1 + 2.0 * ap4) + 4);
        atomicMin(&s_box[2], (int)floor(y2 - 2.0 * (ap2 + a[2] + ap4)) - 3);
        atomicMax(&s_box[3], (int)floor(y2) + 4);
    }
    __syncthreads();
    float *outp = J.out + (inside ? r * J.out_rs + c * J.C + ch : 0);
    if (s_box[0] == INT32_MAX) {   // no valid pixel in the tile
        if (inside && part == 0) {
            *outp = NAN;
            atomicAdd(J.nan_count, 1u);
        }
        return;
    }
    const int wc0 = s_box[0], wr0 = s_box[2];
    const int ww = s_box[1] - wc0 + 1, wh = s_box[3] - wr0 + 1;
    const int S = ww | 1;
    if ((int64_t)wh * S > cap) {
        if (defer) {
            if (t == 0) {
                const uint32_t k = atomicAdd(J.defer_count, 1u);
                J.defer[2 * k] = ((uint32_t)by << 16) | (uint32_t)bx;
                J.defer[2 * k + 1] = (uint32_t)ch;
            }
            return;
        }
        if (inside && part == 0) {
            *outp = NAN;
            atomicAdd(&s_nan, 1u);
        }
        __syncthreads();
        if (t == 0 && s_nan) atomicAdd(J.nan_count, s_nan);
        return;
    }
    double fmax_loc = 0.0;
    for (int i = t; i < wh * ww; i += blockDim.x) {
        const int rr = i / ww, cc = i - rr * ww;
        const double v = in_at<IN>(J, (int64_t)wr0 + rr, (int64_t)wc0 + cc, ch);
        g[rr * S + cc] = v;
        fmax_loc = fmax(fmax_loc, fabs(v));
    }
    const double fmax_w = block_max(fmax_loc, s_red);
    rs4_window(g, wh, ww, S);
    rs4_window(g, wh, ww, S);
    double gmax_loc = 0.0;
    for (int i = t; i < wh * ww; i += blockDim.x) gmax_loc = fmax(gmax_loc, fabs(g[(i / ww) * S + i % ww]));
    const double gmax = block_max(gmax_loc, s_red);

    const double pa = a[0] * a[1] * a[2] * a[3], w = 1.0 / (pa * pa * kZp2Den);   // table scale folded in
    const bool run = inside && ok && 0x1p-46 * gmax * (w * kZp2Den) <= 1e-6 * fmax_w;
    double acc = 0.0;
    if (run) {
        {
            const double b1 = y1 - wc0, b2 = y2 - wr0;   // window coordinates
            const int j_end = min(81, (part + 1) * kSpTaps);
            for (int jj = part * kSpTaps; jj < j_end; ++jj) {
                const int j1 = jj % 3, j2 = (jj / 3) % 3, j3 = (jj / 9) % 3, j4 = jj / 27;
                const double coef = (double)((j1 == 1 ? -2 : 1) * (j2 == 1 ? -2 : 1) * (j3 == 1 ? -2 : 1) *
                                             (j4 == 1 ? -2 : 1));
                const double Y1 = b1 - (j1 * a[0] + j2 * ap2 - j4 * ap4);
                const double Y2 = b2 - (j2 * ap2 + j3 * a[2] + j4 * ap4);
                const double fx = floor(Y1), fy = floor(Y2);
                const double dx = Y1 - fx, dy = Y2 - fy;
                const int ix = (int)fx, iy = (int)fy;
                // quarter turn of the unit square that takes the tap's mesh triangle to
                // the tabulated one: position (px, py), and the window offset of table
                // stencil (lx', ly') as o + lx' dA + ly' dB
                double px, py;
                int ox, oy, dA, dB;
                const bool below = dy <= dx, low = dx + dy <= 1.0;
                if (below && low) { px = dx; py = dy; ox = 0; oy = 0; dA = 1; dB = S; }
                else if (below) { px = dy; py = 1.0 - dx; ox = 1; oy = 0; dA = S; dB = -1; }
                else if (!low) { px = 1.0 - dx; py = 1.0 - dy; ox = 1; oy = 1; dA = -1; dB = -S; }
                else { px = 1.0 - dy; py = dx; ox = 0; oy = 1; dA = -S; dB = 1; }
                const int base = (iy + oy) * S + ix + ox;
                acc = fma(coef, zp2_interp(g, base, dA, dB, px, py), acc);
            }
        }
    }
    if (part) s_part[part - 1][px_i] = acc;
    __syncthreads();
    if (!inside || part) return;
    for (int k = 0; k < kSpSplit - 1; ++k) acc += s_part[k][px_i];
    const double res = run ? w * acc : NAN;
    *outp = (float)res;
    if (!run) atomicAdd(J.nan_count, 1u);
}

template <int IN>
__global__ __launch_bounds__(kSpThreads) void k_single2(SingleJob J)
{
    extern __shared__ double lds[];
    single_tile<IN>(J, blockIdx.x, blockIdx.y, blockIdx.z, lds, J.win_cap, J.defer != nullptr);
}

// The listed tiles, a persistent grid: work-group b takes list entries b, b + grid, ...
// with its own global-memory slot for the window.
template <int IN>
__global__ __launch_bounds__(kSpThreads) void k_single2_global(SingleJob J)
{
    const uint32_t n = *J.defer_count;
    double *slot = J.slots + (int64_t)blockIdx.x * J.slot_doubles;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint32_t id = J.defer[2 * i], ch = J.defer[2 * i + 1];
        single_tile<IN>(J, (int)(id & 0xffffu), (int)(id >> 16), (int)ch, slot, J.slot_doubles, false);
        __syncthreads();   // the shared records and the slot are reused by the next tile
    }
}

}  // namespace

}  // namespace svf

using namespace svf;

extern "C" svf_status svf_filter_single(svf_ctx *ctx, const svf_image *in, const svf_field *field, int m,
                                        const svf_opts *opts, svf_image *out, hipStream_t stream, svf_report *rep)
{
    if (!ctx) return SVF_EINVAL;
    ctx->err.clear();
    svf_opts o;
    if (opts) o = *opts; else svf_default_opts(&o);
    if (m != 2) return fail(ctx, SVF_EUNSUPPORTED, "single-pass iterated filter: m = 2 only");
    svf_status st = check_filter_args(ctx, in, field, 4, m, o, out);
    if (st) return st;
    if (o.boundary != SVF_BOUNDARY_ZERO) return fail(ctx, SVF_EUNSUPPORTED, "single pass: zero boundary only");
    if (o.preint != SVF_PRE_F64 || o.fd_fp32) return fail(ctx, SVF_EUNSUPPORTED, "single pass: binary64 only");
    if (o.bands > 1) return fail(ctx, SVF_EUNSUPPORTED, "single pass: one band");
    if (in->data == out->data && in->H > 0 && in->W > 0)
        return fail(ctx, SVF_EINVAL, "single pass: out must not alias in");
    if (rep) std::memset(rep, 0, sizeof *rep);
    if (in->H == 0 || in->W == 0) return SVF_OK;
    // workspace: the scale map's tile records and scales (as for svf_filter), then the
    // NaN and list counters and the list of tiles for the global-memory launch
    Plan p = plan_for(in, m, &o);
    const int64_t ntx = (in->W + kSpT - 1) / kSpT, nty = (in->H + kSpT - 1) / kSpT;
    const size_t n_list = (size_t)(ntx * nty * in->channels);
    const size_t off_cnt = p.off_fdplan, off_list = off_cnt + 256;
    const size_t bytes = off_list + ((n_list * 8 + 255) / 256) * 256;
    st = ensure_workspace(ctx, bytes);
    if (st) return st;
    const size_t nt = (size_t)p.ntr * p.ntc;
    st = ensure_pinned(ctx, nt * sizeof(TileStat) + 64);
    if (st) return st;
    const hipError_t de = hipSetDevice(ctx->device);
    if (de != hipSuccess) return hip_fail(ctx, de, "hipSetDevice");
    unsigned char *ws = static_cast<unsigned char *>(ctx->ws);
    Job j = base_job(in, field, m, &o, p, ws);
    st = attach_lut(ctx, o, j, stream);
    if (st) return st;
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(ws), 0u, (int64_t)(bytes / 4), stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "fill");
    e = timed_launch(ctx, kClsScaleMap, stream, [&] { return launch_scale_map(j, stream); });
    if (e != hipSuccess) return hip_fail(ctx, e, "scale map launch");
    // the window side follows from the largest support: read the tile records
    TileStat *hts = static_cast<TileStat *>(ctx->host_pinned);
    e = hipMemcpyAsync(hts, ws + p.off_tstat, nt * sizeof(TileStat), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "tile records");
    float mx = 0.f;
    for (size_t i = 0; i < nt; ++i) mx = std::max(mx, std::max(hts[i].rx, hts[i].ry));
    // support half-width of beta^{4,2} with the pass scales a / sqrt2: 2 rx / sqrt2, at
    // most that of two passes of beta^4 within max_reach_px (windows, slots and their
    // 32-bit indexes stay bounded); beyond it nothing more is enqueued
    const double reach = std::sqrt(2.0) * mx;
    if (!(reach <= 2.0 * o.max_reach_px)) {
        if (rep) {
            fill_report(hts, nt, m, rep);
            rep->max_reach_px = reach;
        }
        return fail(ctx, SVF_ERANGE, "single pass: support half-width %.1f px above 2 max_reach_px = %d (output not written)",
                    reach, 2 * o.max_reach_px);
    }
    const int side = kSpT + 2 * ((int)std::ceil(reach) + 6);
    const int64_t need = (int64_t)side * (side | 1);
    const int cap = kSpLdsBytes / 8;
    const int win_cap = (int)std::min<int64_t>(need, cap);
    SingleJob sj;
    sj.in = in->data;
    sj.in_rs = in->row_stride;
    sj.in_type = in->dtype == SVF_U16 ? kInU16 : kInF32;
    sj.C = in->channels;
    sj.H = in->H;
    sj.W = in->W;
    sj.scales = j.scales;
    sj.sc_rs = j.sc_rs;
    sj.out = static_cast<float *>(out->data);
    sj.out_rs = out->row_stride;
    sj.inv_sqrt_m = 1.0 / std::sqrt(2.0);
    sj.win_cap = win_cap;
    sj.nan_count = reinterpret_cast<uint32_t *>(ws + off_cnt);
    sj.defer = nullptr;
    sj.defer_count = reinterpret_cast<uint32_t *>(ws + off_cnt + 4);
    sj.slots = nullptr;
    sj.slot_doubles = need;
    // windows above the LDS: a second, persistent launch with one global-memory slot of
    // the largest window per work-group
    const int n_slots = (int)std::min<int64_t>((int64_t)n_list, 512);
    if (need > cap) {
        const size_t sb = (size_t)n_slots * (size_t)need * 8;
        if (ctx->budget && sb > ctx->budget)
            return fail(ctx, SVF_ENOMEM, "window slots of %zu bytes exceed the HBM budget", sb);
        if (sb > ctx->slots_bytes) {
            if (ctx->slots) {   // a previous call's launch may still read the slots
                e = hipDeviceSynchronize();
                if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
                hipFree(ctx->slots);
            }
            ctx->slots = nullptr;
            ctx->slots_bytes = 0;
            e = hipMalloc(&ctx->slots, sb);
            if (e != hipSuccess) {
                ctx->slots = nullptr;
                return fail(ctx, SVF_ENOMEM, "hipMalloc(%zu) for window slots: %s", sb, hipGetErrorString(e));
            }
            ctx->slots_bytes = sb;
        }
        sj.defer = reinterpret_cast<uint32_t *>(ws + off_list);
        sj.slots = static_cast<double *>(ctx->slots);
    }
    const dim3 grid((unsigned)((in->W + kSpT - 1) / kSpT), (unsigned)((in->H + kSpT - 1) / kSpT),
                    (unsigned)in->channels);
    const size_t lds = (size_t)win_cap * 8;
    e = timed_launch(ctx, kClsFd, stream, [&] {
        if (sj.in_type == kInU16) {
            const hipError_t ae = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_single2<kInU16>),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (ae != hipSuccess) return ae;
            hipLaunchKernelGGL(k_single2<kInU16>, grid, dim3(kSpThreads), lds, stream, sj);
            if (sj.defer) hipLaunchKernelGGL(k_single2_global<kInU16>, dim3(n_slots), dim3(kSpThreads), 0, stream, sj);
        } else {
            const hipError_t ae = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_single2<kInF32>),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (ae != hipSuccess) return ae;
            hipLaunchKernelGGL(k_single2<kInF32>, grid, dim3(kSpThreads), lds, stream, sj);
            if (sj.defer) hipLaunchKernelGGL(k_single2_global<kInF32>, dim3(n_slots), dim3(kSpThreads), 0, stream, sj);
        }
        return hipGetLastError();
    });
    if (e != hipSuccess) return hip_fail(ctx, e, "single-pass launch");
    if (!rep) return SVF_OK;
    uint32_t *hc = reinterpret_cast<uint32_t *>(hts + nt);
    e = hipMemcpyAsync(hc, ws + off_cnt, 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "report");
    fill_report(hts, nt, m, rep);
    rep->overflow_px = *hc;
    rep->max_reach_px = reach;
    if (rep->invalid_px) return fail(ctx, SVF_EINVAL, "invalid field entries");
    if (rep->overflow_px) return fail(ctx, SVF_ERANGE, "%lld outputs beyond the window or precision limit (NaN)",
                                      (long long)rep->overflow_px);
    return SVF_OK;
}

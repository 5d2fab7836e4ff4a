// svf_fd.hip -- gfx950 finite-difference kernel of the space-variant elliptical
// box-spline filter (Chaudhury, Munoz-Barrutia, Unser):
//
//   k_fd : per pixel, the 16-tap finite difference of eq. (final_eqn) (taps of
//          Table 1, shift tau of Sec. 3.1 step (2)) on the ZP interpolant of the
//          pre-integrated window (App. F: 7 lattice samples, one of 4 triangles).
//
// Lattice: x = column, y = row, directions u1 = (1,0), u2 = (1,1)/sqrt2, u3 = (0,1),
// u4 = (-1,1)/sqrt2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "svf_device.h"
#include "svf_internal.h"

namespace svf {

namespace {

// ---------------------------------------------------------------------------
// Finite difference + ZP interpolation (eq. (final_eqn), App. F).
//
// F(y) = sum_m g[m] ZP(y - m).  With m0 = round(y) and d = y - m0 in [-1/2, 1/2]^2,
// ZP(d - k) is non-zero for 7 offsets k, and on each of the 4 triangles of the
// cell cut by its diagonals it is one quadratic in d.  ZP is symmetric under the
// 8 symmetries of the square, so one canonical triangle {s >= t >= 0} serves all:
// d = s sa + t sb with s = max(|d1|,|d2|), t = min(|d1|,|d2|), (sa, sb) the two
// signed lattice axes (sa along the larger component) and k = k1 sa + k2 sb.
// With ZP written as the density of T1(1,0)+T2(1,1)+T3(0,1)+T4(-1,1) (T_k uniform
// on [-1/2, 1/2]), 8 x the weights on the canonical triangle are
//   k = (0,0): 4 (1 - s^2 - t^2)        k = (1,0): 1 + 4s - 4t^2
//   k = (-1,0): (1 - 2s)^2               k = (0,+-1): 1 - 2s^2 + 2t^2 +- 4t(1 - s)
//   k = (1,+-1): 2 (s^2 + t^2) +- 4st
// (they sum to 8).
//
// Data movement.  A work-group takes a 16 x 16 block of output pixels.  The 16
// taps of all its pixels fall, for each tap, close to that tap of the block's
// centre pixel shifted by the pixel's offset in the block; so for each tap the
// group copies one 27 x 27 region of the window (the block, a margin of 4 for
// the variation of the scales across the block, and the stencil) into LDS with
// coalesced loads, and every lane takes its 7 samples from LDS.  A lane whose
// stencil leaves the region (scales that change fast across the block) reads its
// samples from the window directly instead.  Regions are double-buffered: the
// loads for tap i+1 are in flight while tap i is computed, one barrier per tap.
// Window samples are read with buffer loads (reads past the slot return zero).
// ---------------------------------------------------------------------------
constexpr int kFdSide = 16;                              // pixels per block side
constexpr int kRegM = 4;                                 // margin for the spread of a tap over the block
constexpr int kRegS = kFdSide + 2 * kRegM + 3;           // 27: region side
constexpr int kRegN = kRegS * kRegS;                     // 729 samples
constexpr int kRegLoads = (kRegN + 255) / 256;           // 3 per thread
constexpr int kRegPad = kRegLoads * 256;                 // 768: LDS stride of a region (branch-free staging)
constexpr int kFdPrefetch = 3;                           // taps whose loads are in flight (one channel)
// Several channels: one tap ahead.  The staging registers of three taps ahead
// cost 3-channel blocks an occupancy step (143 -> 110 VGPRs with one tap);
// measured at 4096^2, 3 channels: 1658 -> 1510 us per pass (two taps: 1521).
constexpr int kFdPrefetchMulti = 1;
template <int NCH>
constexpr int fd_prefetch() { return NCH == 1 ? kFdPrefetch : kFdPrefetchMulti; }

template <int PRE>
__device__ __forceinline__ double gload(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
    if (PRE == kPreF64) return __builtin_bit_cast(double, v);
    if (PRE == kPreI64) return (double)__builtin_bit_cast(long long, v);
    const float2 f = __builtin_bit_cast(float2, v);
    return (double)f.x + (double)f.y;
}

// Abscissae (index q1 + 2 q2 + 4 q4) and ordinates (index q2 + 2 q3 + 4 q4) of the
// sample positions n + tau - x_i of pixel (r, c), in window coordinates (Table 1:
// x_i = (q1 a1 + q2 a'2 - q4 a'4, q2 a'2 + q3 a3 + q4 a'4); tau: Sec. 3.1 step (2)).
template <typename R>
struct PixGeom {
    R a1, ap2, a3, ap4, cx, cy, wgt;   // wgt = 1 / (8 a1 a2 a3 a4): the ZP weights below are 8 x
    __device__ __forceinline__ PixGeom(const Job &J, const Window &w, int64_t r, int64_t c)
    {
        const float4 af = *reinterpret_cast<const float4 *>(J.scales + r * J.sc_rs + c * 4);
        const R m = (R)J.inv_sqrt_m_d;
        a1 = (R)af.x * m;
        const R a2 = (R)af.y * m;
        a3 = (R)af.z * m;
        const R a4 = (R)af.w * m;
        ap2 = a2 * (R)kRsqrt2;
        ap4 = a4 * (R)kRsqrt2;
        cx = (R)(c - w.c0) + (R)0.5 * (a1 + ap2 - ap4 - (R)1);
        cy = (R)(r - w.r0) + (R)0.5 * (ap2 + a3 + ap4 - (R)3);
        wgt = (R)1 / ((R)8 * a1 * a2 * a3 * a4);
    }
    __device__ __forceinline__ R x(int i) const
    {
        R v = cx;
        if (i & 1) v -= a1;    // q1
        if (i & 2) v -= ap2;   // q2
        if (i & 4) v += ap4;   // q4
        return v;
    }
    __device__ __forceinline__ R y(int i) const
    {
        R v = cy;
        if (i & 1) v -= ap2;   // q2
        if (i & 2) v -= a3;    // q3
        if (i & 4) v -= ap4;   // q4
        return v;
    }
};

// Order of the 16 taps in the difference: four groups of fixed (q2, q4); inside a
// group (q1, q3) = (0,0), (1,0), (1,1), (0,1), so a group needs two abscissae and two
// ordinates.
__host__ __device__ constexpr int step_q1(int k) { return (k & 3) == 1 || (k & 3) == 2; }
__host__ __device__ constexpr int step_q2(int k) { return (k >> 2) & 1; }
__host__ __device__ constexpr int step_q3(int k) { return (k & 3) >= 2; }
__host__ __device__ constexpr int step_q4(int k) { return k >> 3; }

// 8 x the seven ZP weights on the canonical triangle (see above) and the two
// signed axis steps (oa along the larger remainder component, ob along the other).
template <typename R>
struct ZpTap {
    R w00, w10, wm0, w01, w0m, w11, w1m;
    bool px, py, hz;
    __device__ __forceinline__ ZpTap(R dx, R dy)
    {
        const R adx = fabs(dx), ady = fabs(dy);
        hz = adx >= ady;
        const R s = fmax(adx, ady), t = fmin(adx, ady);
        const R s2 = s * s, t2 = t * t, st = s * t, q = s2 + t2;
        w00 = fma((R)-4, q, (R)4);
        w10 = fma((R)4, s, (R)1) - (R)4 * t2;
        const R u = fma((R)-2, s, (R)1);
        wm0 = u * u;
        const R A = fma((R)2, t2 - s2, (R)1);
        const R B = (R)4 * (t - st);
        w01 = A + B;
        w0m = A - B;
        w11 = fma((R)4, st, (R)2 * q);
        w1m = fma((R)-4, st, (R)2 * q);
        px = dx >= (R)0;
        py = dy >= (R)0;
    }
    // g(offset in bytes); base: byte offset of the nearest sample, xb / yb: byte steps
    // of one column / one row
    template <class G>
    __device__ __forceinline__ R apply(const G &g, int base, int xb, int yb) const
    {
        const int sxb = px ? xb : -xb, syb = py ? yb : -yb;
        const int oa = hz ? sxb : syb, ob = hz ? syb : sxb;
        R F8 = w00 * (R)g(base);
        F8 = fma(w10, (R)g(base + oa), F8);
        F8 = fma(wm0, (R)g(base - oa), F8);
        F8 = fma(w01, (R)g(base + ob), F8);
        F8 = fma(w0m, (R)g(base - ob), F8);
        F8 = fma(w11, (R)g(base + oa + ob), F8);
        F8 = fma(w1m, (R)g(base + oa - ob), F8);
        return F8;
    }
};

// Direct path for one pixel: every sample read from the window (for lanes whose
// stencil left the staged region).  The tap coordinates are recomputed from the
// scales one tap at a time (rolled loop), so that this path adds no registers to
// the staged path above it.
template <int PRE, int NCH, typename R>
__device__ __forceinline__ void fd_direct(const Job &J, const Window &w, int64_t r, int64_t c,
                                          const __amdgpu_buffer_rsrc_t (&rs)[NCH], R (&acc)[NCH])
{
    const float4 af = *reinterpret_cast<const float4 *>(J.scales + r * J.sc_rs + c * 4);
    const R m = (R)J.inv_sqrt_m_d;
    const R a1 = (R)af.x * m, a2 = (R)af.y * m, a3 = (R)af.z * m, a4 = (R)af.w * m;
    const R ap2 = a2 * (R)kRsqrt2, ap4 = a4 * (R)kRsqrt2;
    const R cx = (R)(c - w.c0) + (R)0.5 * (a1 + ap2 - ap4 - (R)1);
    const R cy = (R)(r - w.r0) + (R)0.5 * (ap2 + a3 + ap4 - (R)3);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[ch] = (R)0;
#pragma unroll 1
    for (int i = 0; i < 16; ++i) {
        const int q1 = i & 1, q2 = (i >> 1) & 1, q3 = (i >> 2) & 1, q4 = (i >> 3) & 1;
        R x = cx, y = cy;
        if (q1) x -= a1;
        if (q2) { x -= ap2; y -= ap2; }
        if (q3) y -= a3;
        if (q4) { x += ap4; y -= ap4; }
        const R rx = rint(x), ry = rint(y);
        const ZpTap<R> z(x - rx, y - ry);
        const int base = min(max((int)ry, 1), w.h - 2) * w.w + min(max((int)rx, 1), w.w - 2);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const __amdgpu_buffer_rsrc_t rr = rs[ch];
            const R F8 = z.apply([&](int off) { return gload<PRE>(rr, (uint32_t)off); }, base * 8, 8, w.w * 8);
            acc[ch] = ((q1 + q2 + q3 + q4) & 1) ? acc[ch] - F8 : acc[ch] + F8;
        }
    }
}

template <int PRE, int NCH, typename R>
__device__ __forceinline__ void fd_block(const Job &J, int lb, double (*lds)[NCH][kRegPad])
{
    // tile-major block order: all blocks of tile 0, then tile 1, ...
    const int bpt_x = J.T / kFdSide, bpt = bpt_x * bpt_x;
    const int tile = lb / bpt, rem = lb - tile * bpt;
    if (tile >= J.ntr * J.ntc) return;   // uniform
    const int by = rem / bpt_x, bx = rem - by * bpt_x;
    const int ti = tile / J.ntc, tj = tile - ti * J.ntc;
    const int64_t br0 = (int64_t)ti * J.T + by * kFdSide, bc0 = (int64_t)tj * J.T + bx * kFdSide;
    if (br0 >= J.H || bc0 >= J.W) return;   // uniform: block entirely outside a ragged tile
    const int t = threadIdx.x;
    const int64_t r = br0 + t / kFdSide, c = bc0 + t % kFdSide;
    const bool live = r < J.H && c < J.W;
    const Window w = window_of(J, tile);
    const int ww = w.w;
    // Region origins, one per distinct abscissa / ordinate, from the block's centre
    // pixel: region column = window column - AX, so that a pixel at block offset ox
    // with the centre's scales lands on column ox + 1 + kRegM.  Lane k < 16 of each
    // wave computes the centre's coordinate k (abscissa k, or ordinate k - 8) and the
    // values are read back as uniform registers.
    int AX[8], AY[8];
    {
        const int64_t ra = min(br0 + kFdSide / 2, J.H - 1), ca = min(bc0 + kFdSide / 2, J.W - 1);
        const float4 af = *reinterpret_cast<const float4 *>(J.scales + ra * J.sc_rs + ca * 4);
        const R m = (R)J.inv_sqrt_m_d;
        const R a1 = (R)af.x * m, a2 = (R)af.y * m, a3 = (R)af.z * m, a4 = (R)af.w * m;
        const R ap2 = a2 * (R)kRsqrt2, ap4 = a4 * (R)kRsqrt2;
        const int k = t & 15, b0 = k & 1, b1 = (k >> 1) & 1, b2 = (k >> 2) & 1;
        R v;
        if (k < 8) {   // same operations as PixGeom::x / PixGeom::y
            v = (R)(ca - w.c0) + (R)0.5 * (a1 + ap2 - ap4 - (R)1);
            if (b0) v -= a1;
            if (b1) v -= ap2;
            if (b2) v += ap4;
        } else {
            v = (R)(ra - w.r0) + (R)0.5 * (ap2 + a3 + ap4 - (R)3);
            if (b0) v -= ap2;
            if (b1) v -= a3;
            if (b2) v -= ap4;
        }
        const int iv = min(max((int)rint(v), 1), (k < 8 ? ww : w.h) - 2);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            AX[i] = __builtin_amdgcn_readlane(iv, i) - (int)(ca - bc0) - 1 - kRegM;
            AY[i] = __builtin_amdgcn_readlane(iv, 8 + i) - (int)(ra - br0) - 1 - kRegM;
        }
    }
    const PixGeom<R> G(J, w, live ? r : br0, live ? c : bc0);
    R wgt = G.wgt;
    if (PRE == kPreI64) wgt *= (R)2;
    const unsigned char *gbase = static_cast<const unsigned char *>(J.g);
    const int slot_bytes = (int)(J.slot_elems * 8);
    __amdgpu_buffer_rsrc_t rs[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
        rs[ch] = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<unsigned char *>(gbase + ((int64_t)tile * J.C + ch) * J.slot_elems * 8), 0, slot_bytes,
            kBufWord3);
    // loads of tap j go to register slot j % PF; tap j is fetched PF taps before it
    // is staged
    // Region entry e = t + 256 k of tap i is window sample (AY + e / 27) * ww + AX + e % 27:
    // a fixed per-thread part and a uniform per-tap part.  Entries past kRegN are
    // loaded and staged but never read.
    int toff[kRegLoads];
#pragma unroll
    for (int k = 0; k < kRegLoads; ++k) {
        const int e = t + 256 * k;
        toff[k] = (e / kRegS) * ww + e % kRegS;
    }
    constexpr int PF = fd_prefetch<NCH>();
    double pre[PF][NCH][kRegLoads];
    auto fetch = [&](int i) {   // region of the tap processed at step i
        const int xi = step_q1(i) + 2 * step_q2(i) + 4 * step_q4(i);
        const int yi = step_q2(i) + 2 * step_q3(i) + 4 * step_q4(i);
        const int sb = AY[yi] * ww + AX[xi];   // uniform
#pragma unroll
        for (int k = 0; k < kRegLoads; ++k) {
            const uint32_t off = (uint32_t)(sb + toff[k]) * 8u;   // negative wraps: OOB -> 0
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) pre[i % PF][ch][k] = gload<PRE>(rs[ch], off);
        }
    };
    auto stage = [&](int i) {
#pragma unroll
        for (int k = 0; k < kRegLoads; ++k) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) lds[i & 1][ch][t + 256 * k] = pre[i % PF][ch][k];
        }
    };
    R acc[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[ch] = (R)0;
    bool outside = false;   // some stencil of this lane left its staged region
#pragma unroll
    for (int j = 0; j < PF; ++j) fetch(j);
    stage(0);
    lds_barrier();
    R gdx[2], gdy[2];   // remainders of the current group's abscissae / ordinates
    int glx[2], gly[2];  // their region offsets (gly in samples of whole rows)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (i + PF < 16) fetch(i + PF);
        const int q1 = step_q1(i), q2 = step_q2(i), q3 = step_q3(i), q4 = step_q4(i);
        if ((i & 3) == 0) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int xi = u + 2 * q2 + 4 * q4, yi = q2 + 2 * u + 4 * q4;
                const R x = G.x(xi), y = G.y(yi);
                const R rx = rint(x), ry = rint(y);
                gdx[u] = x - rx;
                gdy[u] = y - ry;
                // position in the region (clamped; a lane whose stencil leaves it is redone below)
                const int lx = min(max((int)rx, 1), ww - 2) - AX[xi], ly = min(max((int)ry, 1), w.h - 2) - AY[yi];
                outside |= (unsigned)(lx - 1) > (unsigned)(kRegS - 3) || (unsigned)(ly - 1) > (unsigned)(kRegS - 3);
                glx[u] = min(max(lx, 1), kRegS - 2);
                gly[u] = min(max(ly, 1), kRegS - 2) * kRegS;
            }
        }
        const ZpTap<R> z(gdx[q1], gdy[q3]);
        const int base = (gly[q3] + glx[q1]) * 8;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const unsigned char *L = reinterpret_cast<const unsigned char *>(lds[i & 1][ch]);
            const R F8 = z.apply([&](int off) { return *reinterpret_cast<const double *>(L + off); }, base, 8, kRegS * 8);
            acc[ch] = ((q1 + q2 + q3 + q4) & 1) ? acc[ch] - F8 : acc[ch] + F8;   // w_i = (-1)^(q1+..+q4) w
            // keep this tap's arithmetic here: otherwise it is sunk into the final store
            // block and every tap's samples stay live in registers until then
            __asm__ volatile("" : "+v"(acc[ch]));
        }
        if (i + 1 < 16) {
            stage(i + 1);
            lds_barrier();
        }
    }
    if (live && outside) fd_direct<PRE, NCH, R>(J, w, r, c, rs, acc);
    if (live) {
        float *o = J.out + r * J.out_rs + c * J.C;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) o[ch] = (float)(acc[ch] * wgt);
    }
}

template <int PRE, int NCH, typename R>
__global__ __launch_bounds__(256) void k_fd(Job J, int nblocks)
{
    __shared__ double lds[2][NCH][kRegPad];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int bpt = (J.T / kFdSide) * (J.T / kFdSide);
    if (lb < nblocks) fd_block<PRE, NCH, R>(J, J.tr0 * J.ntc * bpt + lb, lds);
}

// one work-group per 16 x 16 block of any image of the table (all with NCH channels)
template <int PRE, int NCH, typename R>
__global__ __launch_bounds__(256) void k_fd_batch(const Job *jobs, int n, int total)
{
    __shared__ double lds[2][NCH][kRegPad];
    const int b = blockIdx.x;
    if (b >= total) return;
    const int j = __builtin_amdgcn_readfirstlane(find_job(jobs, n, b, 1));
    const Job &J = jobs[j];
    fd_block<PRE, NCH, R>(J, b - J.blk_base, lds);
}

// ---------------------------------------------------------------------------
// Finite difference of a spatially constant filter (the window of the structure
// tensor).  Every pixel's taps then sit at the same offsets with the same
// remainders, so the 16 x 7 (offset, weight) products of eq. (final_eqn) with
// the ZP stencils (signs and 1 / (8 a1 a2 a3 a4) folded in) are formed once per
// block, and one staged region holds every sample of the block's pixels: per
// pixel and channel, 112 LDS reads and fused multiply-adds.
// ---------------------------------------------------------------------------
constexpr int kUniMaxSide = 48;   // largest region side (LDS: side^2 x 8 B per channel)

// Tap i of a constant filter (q1 = bit 0, q2 = bit 1, q3 = bit 2, q4 = bit 3 of i):
// its position relative to the pixel, nearest lattice point and remainder; every
// lane computes the same values.
__device__ __forceinline__ void uni_tap(int i, double a1, double ap2, double a3, double ap4, int &ox, int &oy,
                                        double &dx, double &dy)
{
    const int q1 = i & 1, q2 = (i >> 1) & 1, q3 = (i >> 2) & 1, q4 = (i >> 3) & 1;
    double x = 0.5 * (a1 + ap2 - ap4 - 1.0), y = 0.5 * (ap2 + a3 + ap4 - 3.0);
    if (q1) x -= a1;
    if (q2) { x -= ap2; y -= ap2; }
    if (q3) y -= a3;
    if (q4) { x += ap4; y -= ap4; }
    const double rx = rint(x), ry = rint(y);
    ox = (int)rx;
    oy = (int)ry;
    dx = x - rx;
    dy = y - ry;
}

// LDS: the weight table, then NCH regions of `cap` samples (dynamic: sized by the
// launch for the filter at hand, so that small regions let more blocks share a CU)
template <int PRE, int NCH>
__global__ __launch_bounds__(256) void k_fd_uniform(Job J, int nblocks, int cap)
{
    extern __shared__ double dyn[];
    double *tab = dyn;             // 16 x 7 weights (signs and 1 / (8 a1 a2 a3 a4) folded in)
    double *lds = dyn + 112;       // NCH regions of cap samples
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    if (lb >= nblocks) return;
    const int bpt_x = J.T / kFdSide, bpt = bpt_x * bpt_x;
    const int gb = J.tr0 * J.ntc * bpt + lb;
    const int tile = gb / bpt, rem = gb - tile * bpt;
    if (tile >= J.ntr * J.ntc) return;   // uniform
    const int by = rem / bpt_x, bx = rem - by * bpt_x;
    const int ti = tile / J.ntc, tj = tile - ti * J.ntc;
    const int64_t br0 = (int64_t)ti * J.T + by * kFdSide, bc0 = (int64_t)tj * J.T + bx * kFdSide;
    if (br0 >= J.H || bc0 >= J.W) return;   // uniform
    const int t = threadIdx.x;
    const Window w = window_of(J, tile);
    const float4 af = *reinterpret_cast<const float4 *>(J.scales + br0 * J.sc_rs + bc0 * 4);   // any pixel
    const double m = J.inv_sqrt_m_d;
    const double a1 = (double)af.x * m, a2 = (double)af.y * m, a3 = (double)af.z * m, a4 = (double)af.w * m;
    const double ap2 = a2 * kRsqrt2, ap4 = a4 * kRsqrt2;
    int oxmin = 1 << 20, oxmax = -(1 << 20), oymin = 1 << 20, oymax = -(1 << 20);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int ox, oy;
        double dx, dy;
        uni_tap(i, a1, ap2, a3, ap4, ox, oy, dx, dy);
        oxmin = min(oxmin, ox); oxmax = max(oxmax, ox);
        oymin = min(oymin, oy); oymax = max(oymax, oy);
    }
    const int sx = kFdSide + oxmax - oxmin + 2, sy = kFdSide + oymax - oymin + 2;   // region sides
    if (sx > kUniMaxSide || sy > kUniMaxSide || sx * sy > cap) {   // checked on the host; never stage past LDS
        const int64_t r = br0 + t / kFdSide, c = bc0 + t % kFdSide;
        if (r < J.H && c < J.W)
            for (int ch = 0; ch < NCH; ++ch) J.out[r * J.out_rs + c * J.C + ch] = __builtin_nanf("");
        return;
    }
    if (t < 16) {   // the weights of tap t's 7 stencil samples
        int ox, oy;
        double dx, dy;
        uni_tap(t, a1, ap2, a3, ap4, ox, oy, dx, dy);
        const ZpTap<double> z(dx, dy);
        const int q = (t & 1) + ((t >> 1) & 1) + ((t >> 2) & 1) + ((t >> 3) & 1);
        const double k = ((q & 1) ? -1.0 : 1.0) / (8.0 * a1 * a2 * a3 * a4);   // w_i = (-1)^(q1+..+q4) w
        double *e = tab + 7 * t;
        e[0] = k * z.w00; e[1] = k * z.w10; e[2] = k * z.wm0; e[3] = k * z.w01;
        e[4] = k * z.w0m; e[5] = k * z.w11; e[6] = k * z.w1m;
    }
    // stage the region: window rows / columns from the block's corner + (oymin - 1, oxmin - 1)
    const int wr0 = (int)(br0 - w.r0) + oymin - 1, wc0 = (int)(bc0 - w.c0) + oxmin - 1;
    const unsigned char *gbase = static_cast<const unsigned char *>(J.g);
    const int slot_bytes = (int)(J.slot_elems * 8);
    const int n = sx * sy;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<unsigned char *>(gbase + ((int64_t)tile * J.C + ch) * J.slot_elems * 8), 0, slot_bytes,
            kBufWord3);
        for (int e = t; e < n; e += 256) {
            const int yy = e / sx, xx = e - yy * sx;
            lds[ch * cap + e] = gload<PRE>(rs, (uint32_t)((wr0 + yy) * w.w + wc0 + xx) * 8u);
        }
    }
    __syncthreads();
    const int ly = t / kFdSide, lx = t - ly * kFdSide;
    const int64_t r = br0 + ly, c = bc0 + lx;
    if (r >= J.H || c >= J.W) return;
    // sample offsets from registers (the tap geometry recomputed per tap, the same
    // in every lane), weights from the table at fixed LDS addresses
    const int base = ly * sx + lx;
    double acc[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[ch] = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int ox, oy;
        double dx, dy;
        uni_tap(i, a1, ap2, a3, ap4, ox, oy, dx, dy);
        const bool hz = fabs(dx) >= fabs(dy);
        const int sxb = dx >= 0.0 ? 1 : -1, syb = dy >= 0.0 ? sx : -sx;
        const int oa = hz ? sxb : syb, ob = hz ? syb : sxb;
        const int o0 = base + (oy - oymin + 1) * sx + (ox - oxmin + 1);
        const int off[7] = {o0, o0 + oa, o0 - oa, o0 + ob, o0 - ob, o0 + oa + ob, o0 + oa - ob};
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            const double wt = tab[7 * i + j];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) acc[ch] = fma(wt, lds[ch * cap + off[j]], acc[ch]);
        }
    }
    float *o = J.out + r * J.out_rs + c * J.C;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) o[ch] = (float)acc[ch];
}

}  // namespace

int fd_blocks_job(const Job &j)
{
    return j.ntr * j.ntc * (j.T / kFdSide) * (j.T / kFdSide);
}

template <int PRE, typename R>
static hipError_t launch_fd_pr(const Job &j, int nb, int grid, hipStream_t s)
{
    switch (j.C) {
    case 1: hipLaunchKernelGGL((k_fd<PRE, 1, R>), dim3(grid), dim3(256), 0, s, j, nb); break;
    case 2: hipLaunchKernelGGL((k_fd<PRE, 2, R>), dim3(grid), dim3(256), 0, s, j, nb); break;
    case 3: hipLaunchKernelGGL((k_fd<PRE, 3, R>), dim3(grid), dim3(256), 0, s, j, nb); break;
    case 4: hipLaunchKernelGGL((k_fd<PRE, 4, R>), dim3(grid), dim3(256), 0, s, j, nb); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

namespace {
// region sides bound: tap spread + rounding of both extremes + the stencil's sample on each side
int uni_side(double spread) { return kFdSide + (int)std::ceil(spread) + 1 + 2; }
}  // namespace

bool fd_uniform_fits(double a1, double a2, double a3, double a4, int channels)
{
    if (channels != 3) return false;
    const double ap2 = a2 * 0.70710678118654752440, ap4 = a4 * 0.70710678118654752440;
    return uni_side(a1 + ap2 + ap4) <= kUniMaxSide && uni_side(ap2 + a3 + ap4) <= kUniMaxSide;
}

hipError_t launch_fd_uniform(const Job &j, const double *a, hipStream_t s)
{
    const int nb = (j.tr1 - j.tr0) * j.ntc * (j.T / kFdSide) * (j.T / kFdSide);
    if (nb <= 0) return hipSuccess;
    const int grid = (nb + 7) / 8 * 8;
    if (j.C != 3 || j.fd_fp32) return hipErrorInvalidValue;
    const double ap2 = a[1] * 0.70710678118654752440, ap4 = a[3] * 0.70710678118654752440;
    const int cap = uni_side(a[0] + ap2 + ap4) * uni_side(ap2 + a[2] + ap4);
    const size_t bytes = (112 + (size_t)3 * cap) * sizeof(double);
    switch (j.preint) {
    case kPreF64: hipLaunchKernelGGL((k_fd_uniform<kPreF64, 3>), dim3(grid), dim3(256), bytes, s, j, nb, cap); break;
    case kPreF32C: hipLaunchKernelGGL((k_fd_uniform<kPreF32C, 3>), dim3(grid), dim3(256), bytes, s, j, nb, cap); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fd(const Job &j, hipStream_t s)
{
    const int nb = (j.tr1 - j.tr0) * j.ntc * (j.T / kFdSide) * (j.T / kFdSide);
    if (nb <= 0) return hipSuccess;
    const int grid = (nb + 7) / 8 * 8;
    if (j.fd_fp32) {
        switch (j.preint) {
        case kPreF64: return launch_fd_pr<kPreF64, float>(j, nb, grid, s);
        case kPreF32C: return launch_fd_pr<kPreF32C, float>(j, nb, grid, s);
        case kPreI64: return launch_fd_pr<kPreI64, float>(j, nb, grid, s);
        }
    } else {
        switch (j.preint) {
        case kPreF64: return launch_fd_pr<kPreF64, double>(j, nb, grid, s);
        case kPreF32C: return launch_fd_pr<kPreF32C, double>(j, nb, grid, s);
        case kPreI64: return launch_fd_pr<kPreI64, double>(j, nb, grid, s);
        }
    }
    return hipErrorInvalidValue;
}

template <int PRE, typename R>
static hipError_t launch_fd_batch_pr(const Job *jobs, int n, int total, int nch, hipStream_t s)
{
    switch (nch) {
    case 1: hipLaunchKernelGGL((k_fd_batch<PRE, 1, R>), dim3(total), dim3(256), 0, s, jobs, n, total); break;
    case 2: hipLaunchKernelGGL((k_fd_batch<PRE, 2, R>), dim3(total), dim3(256), 0, s, jobs, n, total); break;
    case 3: hipLaunchKernelGGL((k_fd_batch<PRE, 3, R>), dim3(total), dim3(256), 0, s, jobs, n, total); break;
    case 4: hipLaunchKernelGGL((k_fd_batch<PRE, 4, R>), dim3(total), dim3(256), 0, s, jobs, n, total); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fd_batch(const Job *jobs, int n, int total_blocks, int grid, int preint, int fd_fp32, int nch,
                           hipStream_t s)
{
    (void)grid;   // one work-group per block of the work list
    if (total_blocks == 0) return hipSuccess;
    if (fd_fp32) {
        switch (preint) {
        case kPreF64: return launch_fd_batch_pr<kPreF64, float>(jobs, n, total_blocks, nch, s);
        case kPreF32C: return launch_fd_batch_pr<kPreF32C, float>(jobs, n, total_blocks, nch, s);
        case kPreI64: return launch_fd_batch_pr<kPreI64, float>(jobs, n, total_blocks, nch, s);
        }
    } else {
        switch (preint) {
        case kPreF64: return launch_fd_batch_pr<kPreF64, double>(jobs, n, total_blocks, nch, s);
        case kPreF32C: return launch_fd_batch_pr<kPreF32C, double>(jobs, n, total_blocks, nch, s);
        case kPreI64: return launch_fd_batch_pr<kPreI64, double>(jobs, n, total_blocks, nch, s);
        }
    }
    return hipErrorInvalidValue;
}
}  // namespace svf

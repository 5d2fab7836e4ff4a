// svf_fd.hip -- gfx950 finite-difference kernel of the space-variant elliptical
// box-spline filter (Chaudhury, Munoz-Barrutia, Unser):
//
//   k_fd      : per pixel, the 16-tap finite difference of eq. (final_eqn) (taps of
//               Table 1, shift tau of Sec. 3.1 step (2)) on the ZP interpolant of the
//               pre-integrated window (App. F: 7 lattice samples per tap).
//   k_fd_plan : per 16 x 16 pixel block, its window and the origins of the regions
//               the difference stages (once per filter call, after the scale map).
//
// Lattice: x = column, y = row, directions u1 = (1,0), u2 = (1,1)/sqrt2, u3 = (0,1),
// u4 = (-1,1)/sqrt2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>

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
// The kernel evaluates them without selecting the triangle first (zp_tap7 below).
//
// Data movement.  A work-group takes a 16 x 16 block of output pixels.  The 16
// taps of all its pixels fall, for each tap, close to that tap of the block's
// centre pixel shifted by the pixel's offset in the block; so for each tap the
// group copies one 27 x 27 region of the window (the block, a margin of 4 for
// the variation of the scales across the block, and the stencil) into LDS, and
// every lane takes its 7 samples from LDS.  A lane whose stencil leaves the region
// (scales that change fast across the block) reads its samples from the window
// directly instead.  binary64 windows go straight from the buffer loads into LDS
// (16 bytes per lane, no staging registers): the loads of three taps are in flight
// while a fourth region is read, one barrier per tap.  Integer and compensated
// windows are converted to binary64 in registers and staged one tap ahead.  Window
// samples are read with buffer loads (reads past the slot return zero).
//
// Measured on the 4096^2 order-2 workload (same box, per pass): the earlier design
// with register staging, the seven weights of the canonical triangle and per-block
// region origins computed by every wave ran 640-650 us; with the block plan, direct
// loads into LDS and the branch-free weights, 576 us.  The nine-sample form of the
// weights (no corner selection, 20 % more LDS bytes) ran 620 us, and without the
// direct loads every variant ran slower than the earlier design (LDS traffic and
// occupancy, not VALU issue, limit this kernel).
constexpr int kFdSide = 16;                              // pixels per block side
constexpr int kRegM = 4;                                 // margin for the spread of a tap over the block
constexpr int kRegS = kFdSide + 2 * kRegM + 3;           // 27: region side (rows; columns used)
constexpr int kRS = kRegS + 1;                           // 28: LDS row stride of a region (whole 16-byte pairs)
constexpr int kRegLoads = (kRegS * kRS + 255) / 256;     // 3 staged samples per thread (register staging)
constexpr int kRegPad = kRegLoads * 256;                 // 768 samples: LDS stride of a region
constexpr int kRegChunks = (kRegS * kRS / 2 + 63) / 64;  // 6 direct loads of 64 pairs per region
static_assert(kRegChunks * 128 <= kRegPad, "region chunks fit the region's LDS");
constexpr int kFdPrefetch = 3;                           // taps whose loads are in flight (one channel)
// Several channels: one tap ahead.  The staging registers of three taps ahead
// cost 3-channel blocks an occupancy step (143 -> 110 VGPRs with one tap);
// measured at 4096^2, 3 channels: 1658 -> 1510 us per pass (two taps: 1521).
constexpr int kFdPrefetchMulti = 1;
template <int NCH>
constexpr int fd_prefetch() { return NCH == 1 ? kFdPrefetch : kFdPrefetchMulti; }
// LDS regions: binary64 windows are copied straight into LDS by the loads (one
// buffer per tap in flight, plus the one being read); the other arithmetics are
// converted in registers and staged one tap ahead (two buffers).
template <int PRE, int NCH>
constexpr int fd_buffers() { return PRE == kPreF64 ? fd_prefetch<NCH>() + 1 : 2; }

template <int PRE>
__device__ __forceinline__ double gload(__amdgpu_buffer_rsrc_t r, uint32_t byte_off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
    if (PRE == kPreF64) return __builtin_bit_cast(double, v);
    if (PRE == kPreI64) return (double)__builtin_bit_cast(long long, v);
    const float2 f = __builtin_bit_cast(float2, v);
    return (double)f.x + (double)f.y;
}

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

// 8 x the ZP weights on the 3 x 3 lattice block around the nearest lattice point,
// with no branch on the triangle: ZP is C1 and piecewise quadratic, its second
// derivative jumps only across the two diagonals of the cell, so each weight is a
// quadratic in d = (dx, dy) plus multiples of U = u|u| and V = v|v|, u = dx - dy,
// v = dx + dy (one term per diagonal):
//   (0, 0)   : 4 - 4 dx^2 - 4 dy^2          = 4 - 2 (|U| + |V|)
//   (+-1, 0) : 1 +- 4 dx + 2 (dx^2 - dy^2) -+ (U + V)
//   (0, +-1) : 1 +- 4 dy - 2 (dx^2 - dy^2) +- (U - V)
//   (1, 1) : |V| + V    (-1, -1) : |V| - V    (1, -1) : |U| + U    (-1, 1) : |U| - U
// ((i, j) = column offset i, row offset j; dx^2 - dy^2 = u v).  On each of the four
// triangles they reduce to the seven quadratics listed above, and the two corners
// away from the triangle get weight 0.
// Nearest lattice point l (minus the origin o) and remainder d of a coordinate x.
// binary64: x + 1.5 2^52 rounds x to an integer held in the low word (ties to even,
// as rint), and subtracting the constant back gives round(x) exactly.
__device__ __forceinline__ void nearest(double x, int o, int &l, double &d)
{
    constexpr double kMagic = 6755399441055744.0;   // 1.5 * 2^52
    const double t = x + kMagic;
    l = (int)(uint32_t)(unsigned long long)__double_as_longlong(t) - o;
    d = x - (t - kMagic);
}
__device__ __forceinline__ void nearest(float x, int o, int &l, float &d)
{
    const float r = rintf(x);
    l = (int)r - o;
    d = x - r;
}

// One tap: sum over the 3 x 3 block of w * g, added to acc with the tap's sign.
// g(r, c) reads the sample of block row r, column c (0..2).
template <bool NEG, typename R, class G>
__device__ __forceinline__ R zp_tap(R dx, R dy, const G &g, R acc)
{
    const R u = dx - dy, v = dx + dy;
    const R U = u * fabs(u), V = v * fabs(v);
    const R S = U + V, D = U - V;
    const R A = fma((R)2, u * v, (R)1), B = (R)2 - A;   // 1 + 2 (dx^2 - dy^2), 1 - 2 (dx^2 - dy^2)
    R w[9];
    w[4] = fma((R)-2, fabs(U) + fabs(V), (R)4);   // (0, 0)
    w[5] = fma((R)4, dx, A) - S;                  // (1, 0)
    w[3] = fma((R)-4, dx, A) + S;                 // (-1, 0)
    w[7] = fma((R)4, dy, B) + D;                  // (0, 1)
    w[1] = fma((R)-4, dy, B) - D;                 // (0, -1)
    w[8] = fabs(V) + V;                           // (1, 1)
    w[0] = fabs(V) - V;                           // (-1, -1)
    w[2] = fabs(U) + U;                           // (1, -1)
    w[6] = fabs(U) - U;                           // (-1, 1)
#pragma unroll
    for (int k = 0; k < 9; ++k) acc = fma(NEG ? -w[k] : w[k], (R)g(k / 3, k % 3), acc);
    return acc;
}

// The same weights read from 7 samples: the centre, its 4 neighbours and, of each
// diagonal pair of corners, the one on the side of the remainder (the other has
// weight 0): (1, 1) if v >= 0 else (-1, -1), weight 2|V|; (1, -1) if u >= 0 else
// (-1, 1), weight 2|U|.  base: byte offset of the block's corner (-1, -1); rs: bytes
// per row.  g(off) reads the sample at byte offset off.
template <bool NEG, typename R, class G>
__device__ __forceinline__ R zp_tap7(R dx, R dy, const G &g, int base, int rs, R acc)
{
    const R u = dx - dy, v = dx + dy;
    const R U = u * fabs(u), V = v * fabs(v);
    const R S = U + V, D = U - V;
    const R A = fma((R)2, u * v, (R)1), B = (R)2 - A;   // 1 + 2 (dx^2 - dy^2), 1 - 2 (dx^2 - dy^2)
    const R w00 = fma((R)-2, fabs(U) + fabs(V), (R)4);
    const R w10 = fma((R)4, dx, A) - S, wm0 = fma((R)-4, dx, A) + S;
    const R w01 = fma((R)4, dy, B) + D, w0m = fma((R)-4, dy, B) - D;
    const R wv = fabs(V) + fabs(V), wu = fabs(U) + fabs(U);
    const int cv = base + (v >= (R)0 ? 2 * rs + 16 : 0);
    const int cu = base + (u >= (R)0 ? 16 : 2 * rs);
    const R s = NEG ? (R)-1 : (R)1;
    acc = fma(s * w00, (R)g(base + rs + 8), acc);
    acc = fma(s * w10, (R)g(base + rs + 16), acc);
    acc = fma(s * wm0, (R)g(base + rs), acc);
    acc = fma(s * w01, (R)g(base + 2 * rs + 8), acc);
    acc = fma(s * w0m, (R)g(base + 8), acc);
    acc = fma(s * wv, (R)g(cv), acc);
    acc = fma(s * wu, (R)g(cu), acc);
    return acc;
}

// Per-pass scales of pixel (r, c) and the pixel's state: invalid scales, or a
// support beyond the window's reach (the same test, on the same binary32 scales,
// as the scale map's overflow count) give a NaN output.
template <typename R>
struct PixScales {
    R a1, ap2, a3, ap4, wgt;
    bool bad;
    __device__ __forceinline__ PixScales(const Job &J, int64_t r, int64_t c)
    {
        const f32x4 af = load_global(reinterpret_cast<const f32x4 *>(J.scales + r * J.sc_rs + c * 4));
        const double d = ((double)af.y + (double)af.w) * kRsqrt2;
        const float px = (float)(0.5 * ((double)af.x + d)) * 1.000001f;
        const float py = (float)(0.5 * ((double)af.z + d)) * 1.000001f;
        bad = !(af.x > 0.f && af.y > 0.f && af.z > 0.f && af.w > 0.f && isfinite(af.x + af.y + af.z + af.w)) ||
              fmaxf(px, py) * J.inv_sqrt_m > (float)J.cap;
        const R m = (R)J.inv_sqrt_m_d;
        a1 = (R)af.x * m;
        const R a2 = (R)af.y * m;
        a3 = (R)af.z * m;
        const R a4 = (R)af.w * m;
        ap2 = a2 * (R)kRsqrt2;
        ap4 = a4 * (R)kRsqrt2;
        wgt = (R)1 / ((R)8 * a1 * a2 * a3 * a4);
    }
};

// Order of the 16 taps in the difference: four groups of fixed (q2, q4); inside a
// group (q1, q3) = (0,0), (1,0), (1,1), (0,1), so a group needs two abscissae and two
// ordinates.  Abscissa index q1 + 2 q2 + 4 q4, ordinate index q2 + 2 q3 + 4 q4.
__host__ __device__ constexpr int step_q1(int k) { return (k & 3) == 1 || (k & 3) == 2; }
__host__ __device__ constexpr int step_q2(int k) { return (k >> 2) & 1; }
__host__ __device__ constexpr int step_q3(int k) { return (k & 3) >= 2; }
__host__ __device__ constexpr int step_q4(int k) { return k >> 3; }

// Sample positions n + tau - x_i of pixel (r, c) in window coordinates (Table 1:
// x_i = (q1 a1 + q2 a'2 - q4 a'4, q2 a'2 + q3 a3 + q4 a'4); tau: Sec. 3.1 step (2)),
// abscissa / ordinate of group (q2, q4) with q1 = 0 / q3 = 0.
template <typename R>
__device__ __forceinline__ R grp_x(const PixScales<R> &P, R cx, int q2, int q4)
{
    R v = cx;
    if (q2) v -= P.ap2;
    if (q4) v += P.ap4;
    return v;
}
template <typename R>
__device__ __forceinline__ R grp_y(const PixScales<R> &P, R cy, int q2, int q4)
{
    R v = cy;
    if (q2) v -= P.ap2;
    if (q4) v -= P.ap4;
    return v;
}

// Direct path for one pixel: every sample read from the window (for lanes whose
// stencil left the staged region).  The taps are formed one at a time (rolled
// loop) so that this path adds no registers to the staged path.
template <int PRE, int NCH, typename R>
__device__ __forceinline__ void fd_direct(const Job &J, const Window &w, int64_t r, int64_t c, const PixScales<R> &P,
                                          const __amdgpu_buffer_rsrc_t (&rs)[NCH], R (&acc)[NCH])
{
    const R cx = (R)(c - w.c0) + (R)0.5 * (P.a1 + P.ap2 - P.ap4 - (R)1);
    const R cy = (R)(r - w.r0) + (R)0.5 * (P.ap2 + P.a3 + P.ap4 - (R)3);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[ch] = (R)0;
#pragma unroll 1
    for (int i = 0; i < 16; ++i) {
        const int q1 = i & 1, q2 = (i >> 1) & 1, q3 = (i >> 2) & 1, q4 = (i >> 3) & 1;
        const R x = grp_x(P, cx, q2, q4) - (q1 ? P.a1 : (R)0);
        const R y = grp_y(P, cy, q2, q4) - (q3 ? P.a3 : (R)0);
        const R rx = rint(x), ry = rint(y);
        const R dx = x - rx, dy = y - ry;
        const int base = (min(max((int)ry, 1), w.h - 2) - 1) * w.w + min(max((int)rx, 1), w.w - 2) - 1;
        const bool neg = (q1 + q2 + q3 + q4) & 1;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const __amdgpu_buffer_rsrc_t rr = rs[ch];
            auto g = [&](int rr_, int cc_) { return gload<PRE>(rr, (uint32_t)((base + rr_ * w.w + cc_) * 8)); };
            acc[ch] = neg ? zp_tap<true>(dx, dy, g, acc[ch]) : zp_tap<false>(dx, dy, g, acc[ch]);
        }
    }
}

// ---------------------------------------------------------------------------
// Block plan (one thread per 16 x 16 block): the block's place in its tile, the
// tile's window and the origins of the staged regions.  Region column = window
// column - origin, chosen so that a pixel at block offset ox with the centre
// pixel's scales lands on region column ox + 1 + kRegM.  Computed in binary64 from
// the stored binary32 scales, as the difference does.
// ---------------------------------------------------------------------------
__device__ void fd_plan_block(const Job &J, int gb)
{
    const int bpt_x = J.T / kFdSide, bpt = bpt_x * bpt_x;
    const int tile = gb / bpt, rem = gb - tile * bpt;
    const int by = rem / bpt_x, bx = rem - by * bpt_x;
    const int ti = tile / J.ntc, tj = tile - ti * J.ntc;
    FdBlk B;
    B.tile = tile;
    B.br0 = ti * J.T + by * kFdSide;
    B.bc0 = tj * J.T + bx * kFdSide;
    B.pad = 0;
    if (B.br0 >= J.H || B.bc0 >= J.W) {   // a block of a ragged tile that holds no pixel
        B.wr0 = B.wc0 = B.ww = B.wh = 0;
        for (int k = 0; k < 8; ++k) B.ax[k] = B.ay[k] = 0;
        J.fdplan[gb] = B;
        return;
    }
    const Window w = window_of(J, tile);
    B.wr0 = (int32_t)w.r0;
    B.wc0 = (int32_t)w.c0;
    B.ww = w.w;
    B.wh = w.h;
    const int64_t ra = min((int64_t)B.br0 + kFdSide / 2, J.H - 1), ca = min((int64_t)B.bc0 + kFdSide / 2, J.W - 1);
    const f32x4 af = load_global(reinterpret_cast<const f32x4 *>(J.scales + ra * J.sc_rs + ca * 4));
    const double m = J.inv_sqrt_m_d;
    const double a1 = (double)af.x * m, a3 = (double)af.z * m;
    const double ap2 = (double)af.y * m * kRsqrt2, ap4 = (double)af.w * m * kRsqrt2;
    const double cx = (double)(ca - w.c0) + 0.5 * (a1 + ap2 - ap4 - 1.0);
    const double cy = (double)(ra - w.r0) + 0.5 * (ap2 + a3 + ap4 - 3.0);
    for (int k = 0; k < 8; ++k) {
        const int b0 = k & 1, b1 = (k >> 1) & 1, b2 = (k >> 2) & 1;
        // abscissa k = q1 + 2 q2 + 4 q4; ordinate k = q2 + 2 q3 + 4 q4 (Table 1, tau)
        const double x = cx - (b0 ? a1 : 0.0) - (b1 ? ap2 : 0.0) + (b2 ? ap4 : 0.0);
        const double y = cy - (b0 ? ap2 : 0.0) - (b1 ? a3 : 0.0) - (b2 ? ap4 : 0.0);
        int ix = (int)rint(x), iy = (int)rint(y);
        if (!(ix >= 1)) ix = 1;   // also a NaN scale: any origin in the window
        if (!(iy >= 1)) iy = 1;
        ix = min(ix, w.w - 2);
        iy = min(iy, w.h - 2);
        B.ax[k] = ix - (int)(ca - B.bc0) - 1 - kRegM;
        B.ay[k] = iy - (int)(ra - B.br0) - 1 - kRegM;
    }
    J.fdplan[gb] = B;
}

__global__ __launch_bounds__(256) void k_fd_plan(Job J, int nblocks)
{
    const int lb = blockIdx.x * blockDim.x + threadIdx.x;
    const int bpt = (J.T / kFdSide) * (J.T / kFdSide);
    if (lb < nblocks) fd_plan_block(J, J.tr0 * J.ntc * bpt + lb);
}

// one thread per block of any image of the table (blk_base: the job's first block)
__global__ __launch_bounds__(256) void k_fd_plan_batch(const Job *jobs, int n, int total, const BatchDims *dims)
{
    if (dims) {
        n = dims->n;
        total = dims->total;
    }
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < total; b += gridDim.x * blockDim.x) {
        const int j = find_job(jobs, n, b, 1);
        fd_plan_block(jobs[j], b - jobs[j].blk_base);
    }
}

// 16 bytes per lane from a buffer straight into LDS: lane l writes dst + 16 l
// (dst uniform).  The host pass of the compiler has no LDS address space.
__device__ __forceinline__ void lds_load16(__amdgpu_buffer_rsrc_t r, double *dst, uint32_t byte_off)
{
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void *)dst, 16, byte_off, 0, 0, 0);
#else
    (void)r, (void)dst, (void)byte_off;
#endif
}

// vmcnt wait with the other counters left alone (gfx9 s_waitcnt encoding)
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <int PRE, int NCH, typename R>
__device__ __forceinline__ void fd_block(const Job &J, int gb, double (*lds)[NCH][kRegPad])
{
    constexpr int PF = fd_prefetch<NCH>();
    constexpr int NB = fd_buffers<PRE, NCH>();
    constexpr bool kDirect = PRE == kPreF64;   // loads write the regions in LDS themselves
    const FdBlk B = uniform_copy(J.fdplan + gb);
    const int64_t br0 = B.br0, bc0 = B.bc0;
    if (br0 >= J.H || bc0 >= J.W) return;   // uniform: block entirely outside a ragged tile
    const int tile = B.tile;
    const int t = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
    const int64_t r = br0 + t / kFdSide, c = bc0 + t % kFdSide;
    const bool live = r < J.H && c < J.W;
    Window w;
    w.r0 = B.wr0;
    w.c0 = B.wc0;
    w.w = B.ww;
    w.h = B.wh;
    const int ww = w.w;
    int AX[8], AY[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        AX[k] = __builtin_amdgcn_readfirstlane(B.ax[k]);
        AY[k] = __builtin_amdgcn_readfirstlane(B.ay[k]);
    }
    const PixScales<R> P(J, live ? r : br0, live ? c : bc0);
    const R cx = (R)((live ? c : bc0) - w.c0) + (R)0.5 * (P.a1 + P.ap2 - P.ap4 - (R)1);
    const R cy = (R)((live ? r : br0) - w.r0) + (R)0.5 * (P.ap2 + P.a3 + P.ap4 - (R)3);
    R wgt = P.wgt;
    if (PRE == kPreI64) wgt *= (R)2;
    const unsigned char *gbase = static_cast<const unsigned char *>(J.g);
    const int slot_bytes = (int)(J.slot_elems * 8);
    __amdgpu_buffer_rsrc_t rs[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
        rs[ch] = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<unsigned char *>(gbase + ((int64_t)tile * J.C + ch) * J.slot_elems * 8), 0, slot_bytes,
            kBufWord3);
    // Region of tap i: region row y, column x (x < kRS) is window sample
    // (AY + y) * ww + AX + x, a uniform per-tap part plus a fixed per-thread part.
    //  - direct loads: chunk k of 64 pairs of columns; wave w loads chunks w and w + 4
    //    (if < kRegChunks), its lane l the pair p = 64 k + l;
    //  - register staging: entry e = t + 256 k.
    // Entries past the region's rows are loaded and stored but never read.
    constexpr int NL = kDirect ? 2 : kRegLoads;
    int toff[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        if (kDirect) {
            const int pr = 64 * (wave + 4 * k) + lane;
            toff[k] = (pr / (kRS / 2)) * ww + 2 * (pr % (kRS / 2));
        } else {
            const int e = t + 256 * k;
            toff[k] = (e / kRS) * ww + e % kRS;
        }
    }
    const bool two_chunks = wave + 4 < kRegChunks;   // uniform
    double pre[kDirect ? 1 : PF][NCH][kRegLoads];
    auto fetch = [&](int i) {   // region of the tap processed at step i
        const int xi = step_q1(i) + 2 * step_q2(i) + 4 * step_q4(i);
        const int yi = step_q2(i) + 2 * step_q3(i) + 4 * step_q4(i);
        const int sb = AY[yi] * ww + AX[xi];   // uniform
        if constexpr (kDirect) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (k == 1 && !two_chunks) break;
                const uint32_t off = (uint32_t)(sb + toff[k]) * 8u;   // negative wraps: OOB -> 0
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) lds_load16(rs[ch], &lds[i % NB][ch][128 * (wave + 4 * k)], off);
            }
        } else {
#pragma unroll
            for (int k = 0; k < kRegLoads; ++k) {
                const uint32_t off = (uint32_t)(sb + toff[k]) * 8u;   // negative wraps: OOB -> 0
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) pre[i % PF][ch][k] = gload<PRE>(rs[ch], off);
            }
        }
    };
    auto stage = [&](int i) {
        if constexpr (!kDirect) {
#pragma unroll
            for (int k = 0; k < kRegLoads; ++k) {
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) lds[i & 1][ch][t + 256 * k] = pre[i % PF][ch][k];
            }
        }
    };
    // direct loads: before reading the region of tap i, wait until this wave's loads
    // of tap i have landed (the loads of the later taps already issued may still run)
    auto wait_tap = [&](auto later) {
        constexpr int n = decltype(later)::value;
        if (two_chunks) wait_vmcnt<2 * n * NCH>();
        else wait_vmcnt<n * NCH>();
    };
    R acc[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[ch] = (R)0;
    bool outside = false;   // some stencil of this lane left its staged region
    if constexpr (kDirect) {
#pragma unroll
        for (int j = 0; j < PF; ++j) fetch(j);
    } else {
#pragma unroll
        for (int j = 0; j < PF; ++j) fetch(j);
        stage(0);
        lds_barrier();
    }
    R GDX[2], GDY[2];      // remainders of the current group's abscissae / ordinates
    int GOX[2], GOY[2];    // byte offsets of their stencils' first column / row in the region
    auto step = [&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (kDirect) {
            // every wave's loads of tap i are in LDS; tap i - 1 is read by all.  No
            // release fence: it would wait for the later taps' loads as well
            wait_tap(std::integral_constant<int, (i + PF - 1 < 16 ? PF - 1 : 15 - i)>{});
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
            if (i + PF < 16) fetch(i + PF);
        } else {
            if (i + PF < 16) fetch(i + PF);
        }
        const int q1 = step_q1(i), q2 = step_q2(i), q3 = step_q3(i), q4 = step_q4(i);
        if ((i & 3) == 0) {
            const R xg = grp_x(P, cx, q2, q4), yg = grp_y(P, cy, q2, q4);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int xi = u + 2 * q2 + 4 * q4, yi = q2 + 2 * u + 4 * q4;
                int lx, ly;
                nearest(u ? xg - P.a1 : xg, AX[xi], lx, GDX[u]);
                nearest(u ? yg - P.a3 : yg, AY[yi], ly, GDY[u]);
                // stencil inside the region: nearest point in [1, kRegS - 2]
                const int cxl = min(max(lx, 1), kRegS - 2), cyl = min(max(ly, 1), kRegS - 2);
                outside |= (cxl != lx) | (cyl != ly);
                GOX[u] = (cxl - 1) * 8;
                GOY[u] = (cyl - 1) * (kRS * 8);
            }
        }
        const int base = GOY[q3] + GOX[q1];
        const bool neg = (q1 + q2 + q3 + q4) & 1;   // w_i = (-1)^(q1+..+q4) w
        const int buf = kDirect ? i % NB : (i & 1);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const unsigned char *L0 = reinterpret_cast<const unsigned char *>(lds[buf][ch]);
            auto g = [&](int off) { return *reinterpret_cast<const double *>(L0 + off); };
            acc[ch] = neg ? zp_tap7<true>(GDX[q1], GDY[q3], g, base, kRS * 8, acc[ch])
                          : zp_tap7<false>(GDX[q1], GDY[q3], g, base, kRS * 8, acc[ch]);
            // keep this tap's arithmetic here: otherwise it is sunk into the final store
            // block and every tap's samples stay live in registers until then
            __asm__ volatile("" : "+v"(acc[ch]));
        }
        if constexpr (!kDirect) {
            if (i + 1 < 16) {
                stage(i + 1);
                lds_barrier();
            }
        }
    };
    [&]<int... I>(std::integer_sequence<int, I...>) { (step(std::integral_constant<int, I>{}), ...); }(
        std::make_integer_sequence<int, 16>{});
    if (live && outside && !P.bad) fd_direct<PRE, NCH, R>(J, w, r, c, P, rs, acc);
    if (live) {
        float *o = J.out + r * J.out_rs + c * J.C;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) o[ch] = P.bad ? __builtin_nanf("") : (float)(acc[ch] * wgt);
    }
}

// binary64 windows: 5 waves per SIMD for one channel, 4 for several (measured at
// 4096^2 with 3 channels: 4 waves, with a 36-byte spill, 3-4 % faster than the 3 the
// compiler picks by itself); the batched kernel below takes the same setting
template <int PRE, int NCH, typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PRE == kPreF64 && NCH == 1 ? 5 : (PRE == kPreF64 ? 4 : 1), 8))) void k_fd(Job J, int nblocks)
{
    __shared__ double lds[fd_buffers<PRE, NCH>()][NCH][kRegPad];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int bpt = (J.T / kFdSide) * (J.T / kFdSide);
    if (lb < nblocks) fd_block<PRE, NCH, R>(J, J.tr0 * J.ntc * bpt + lb, lds);
}

// One work-group per 16 x 16 block of any image of the table (all with NCH
// channels); the grid may be larger than the work list (the server's captured
// graphs round it up), surplus groups exit.  XCD-aware order as in k_fd: work-group
// w runs on XCD w mod 8, and each XCD takes one contiguous eighth of the tile-major
// block list (eighths of the work list itself, not of the grid: a rounded-up grid
// would otherwise leave the last XCDs without work).
template <int PRE, int NCH, typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PRE == kPreF64 && NCH == 1 ? 5 : (PRE == kPreF64 ? 4 : 1), 8))) void k_fd_batch(
    const Job *jobs, int n, int total, const BatchDims *dims)
{
    __shared__ double lds[fd_buffers<PRE, NCH>()][NCH][kRegPad];
    if (dims) {
        n = dims->n;
        total = dims->total;
    }
    const int per = (total + 7) >> 3, slot = blockIdx.x >> 3;
    const int b = (blockIdx.x & 7) * per + slot;
    if (slot >= per || b >= total) return;
    const int j = __builtin_amdgcn_readfirstlane(find_job(jobs, n, b, 1));
    // a wave-uniform copy in registers: read from the table in memory, the descriptor
    // would be read again after every load into LDS (which may write any memory)
    const Job J = uniform_copy(jobs + j);
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

hipError_t launch_fd_plan(const Job &j, hipStream_t s)
{
    const int nb = (j.tr1 - j.tr0) * j.ntc * (j.T / kFdSide) * (j.T / kFdSide);
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fd_plan, dim3((nb + 255) / 256), dim3(256), 0, s, j, nb);
    return hipGetLastError();
}

hipError_t launch_fd_plan_batch(const Job *jobs, int n, int total_blocks, hipStream_t s, const BatchDims *dims, int grid)
{
    if (!dims) {
        if (total_blocks <= 0) return hipSuccess;
        grid = (total_blocks + 255) / 256;
    }
    hipLaunchKernelGGL(k_fd_plan_batch, dim3(std::max(1, grid)), dim3(256), 0, s, jobs, n, total_blocks, dims);
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
static hipError_t launch_fd_batch_pr(const Job *jobs, int n, int total, int grid, int nch, hipStream_t s,
                                     const BatchDims *dims)
{
    switch (nch) {
    case 1: hipLaunchKernelGGL((k_fd_batch<PRE, 1, R>), dim3(grid), dim3(256), 0, s, jobs, n, total, dims); break;
    case 2: hipLaunchKernelGGL((k_fd_batch<PRE, 2, R>), dim3(grid), dim3(256), 0, s, jobs, n, total, dims); break;
    case 3: hipLaunchKernelGGL((k_fd_batch<PRE, 3, R>), dim3(grid), dim3(256), 0, s, jobs, n, total, dims); break;
    case 4: hipLaunchKernelGGL((k_fd_batch<PRE, 4, R>), dim3(grid), dim3(256), 0, s, jobs, n, total, dims); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fd_batch(const Job *jobs, int n, int total_blocks, int grid, int preint, int fd_fp32, int nch,
                           hipStream_t s, const BatchDims *dims)
{
    if (!dims) {   // one work-group per block of the work list
        if (total_blocks == 0) return hipSuccess;
        grid = total_blocks;
    }
    grid = (std::max(1, grid) + 7) / 8 * 8;   // whole rounds over the 8 XCDs
    if (fd_fp32) {
        switch (preint) {
        case kPreF64: return launch_fd_batch_pr<kPreF64, float>(jobs, n, total_blocks, grid, nch, s, dims);
        case kPreF32C: return launch_fd_batch_pr<kPreF32C, float>(jobs, n, total_blocks, grid, nch, s, dims);
        case kPreI64: return launch_fd_batch_pr<kPreI64, float>(jobs, n, total_blocks, grid, nch, s, dims);
        }
    } else {
        switch (preint) {
        case kPreF64: return launch_fd_batch_pr<kPreF64, double>(jobs, n, total_blocks, grid, nch, s, dims);
        case kPreF32C: return launch_fd_batch_pr<kPreF32C, double>(jobs, n, total_blocks, grid, nch, s, dims);
        case kPreI64: return launch_fd_batch_pr<kPreI64, double>(jobs, n, total_blocks, grid, nch, s, dims);
        }
    }
    return hipErrorInvalidValue;
}
}  // namespace svf

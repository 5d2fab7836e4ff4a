// svf_kernels.hip -- gfx950 kernels of the space-variant elliptical box-spline
// filter (Chaudhury, Munoz-Barrutia, Unser, "Fast space-variant elliptical
// filtering using box splines").
//
//   k_scale_map : per pixel, covariance field -> box scales (Sec. 4.2.2) and the
//                 per-tile support half-widths that size the pre-integration windows.
//   k_preint    : running sums RS1..RS4 (Sec. 4.1 step (1), Algorithm 1 step 2) of one
//                 tile's window, one work-group sweeping the rows top to bottom.
//   k_fd        : per pixel, the 16-tap finite difference of eq. (final_eqn) (taps of
//                 Table 1, shift tau of Sec. 4.1 step (2)) on the ZP interpolant of the
//                 pre-integrated window (App. F: 7 lattice samples, one of 4 triangles).
//
// Lattice: x = column, y = row, directions u1 = (1,0), u2 = (1,1)/sqrt2, u3 = (0,1),
// u4 = (-1,1)/sqrt2; the running sums step by b_k u_k = (1,0), (1,1), (0,1), (-1,1).
#include <hip/hip_runtime.h>

#include "svf_internal.h"

namespace svf {

namespace {

constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kRsqrt2 = 0.70710678118654752440;

// ---------------------------------------------------------------------------
// LDS-only work-group barrier: orders LDS accesses without waiting for global
// loads in flight, so the row sweep can prefetch input rows across barriers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Tile geometry shared by the pre-integration and the finite difference.
// Tile t covers rows [ti T, ...) x cols [tj T, ...).  A pixel n with pass
// half-widths (R1, R2) reads lattice columns [n1 - R1 - 2, n1 + R1 + 1] and rows
// [n2 - R2 - 3, n2 + R2]: the taps n + tau - x_i span [-R - 1/2, R - 1/2] x
// [-R - 3/2, R - 3/2] and the ZP stencil adds one sample on each side of the
// nearest lattice point.  One sample of margin is added on every side.
// ---------------------------------------------------------------------------
__device__ __forceinline__ Window window_of(const Job &J, int tile)
{
    const int ti = tile / J.ntc, tj = tile - ti * J.ntc;
    const int64_t r0 = (int64_t)ti * J.T, c0 = (int64_t)tj * J.T;
    const int64_t r1 = min(r0 + (int64_t)J.T, J.H), c1 = min(c0 + (int64_t)J.T, J.W);
    const float rx = J.tile_reach[2 * tile] * J.inv_sqrt_m;
    const float ry = J.tile_reach[2 * tile + 1] * J.inv_sqrt_m;
    const int hx = min(J.cap, (int)ceilf(rx * 1.000001f));
    const int hy = min(J.cap, (int)ceilf(ry * 1.000001f));
    Window w;
    w.c0 = c0 - hx - 3;
    w.w = (int)(c1 - c0) + 2 * hx + 5;
    w.r0 = r0 - hy - 4;
    w.h = (int)(r1 - r0) + 2 * hy + 5;
    return w;
}

// XCD-aware block order: consecutive hardware work-group ids go round-robin over
// the 8 XCDs; remap so that each XCD receives one contiguous range of logical
// blocks (the blocks of a tile share its window in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int pid, int nblocks)
{
    const int per = nblocks >> 3;   // nblocks is a multiple of 8
    return (pid & 7) * per + (pid >> 3);
}

// ---------------------------------------------------------------------------
// Scale map (Sec. 4.2.2).  All in binary64.
// ---------------------------------------------------------------------------

// d/dt of ||K||^2 along p = pbar + t (1,-1,1,-1), where ||K||^2 = sum p^4 + (p1^2+p3^2)(p2^2+p4^2)
// (App. E), and its second derivative.  Evaluated from the shifted components, not
// from expanded coefficients.
__device__ __forceinline__ void kurt_d(const double *pb, double t, double &d1, double &d2)
{
    const double q1 = pb[0] + t, q2 = pb[1] - t, q3 = pb[2] + t, q4 = pb[3] - t;
    const double A = q1 * q1 + q3 * q3, B = q2 * q2 + q4 * q4;
    const double s13 = q1 + q3, s24 = q2 + q4;
    d1 = 4.0 * (q1 * q1 * q1 - q2 * q2 * q2 + q3 * q3 * q3 - q4 * q4 * q4) + 2.0 * s13 * B - 2.0 * s24 * A;
    d2 = 16.0 * (A + B) - 8.0 * s13 * s24;
}

// Covariance (whole filter) -> scales, floor eps on a^2.  The feasible set of
// M p = c, p >= eps is p = pbar + t e, t in [lo, hi]; ||K||^2 is strictly convex in t
// (second derivative >= 8 sum p^2 > 0), so the minimiser is an end point or the one
// root of the derivative, found by Newton steps kept inside a shrinking bracket.
__device__ void solve_feasible(double C11, double C12, double C22, double eps, double *a, bool &eps_act)
{
    double pb[4];
    pb[3] = 1.0;                               // pivot
    pb[1] = 24.0 * C12 + 1.0;
    pb[0] = 12.0 * (C11 - C12) - 1.0;
    pb[2] = 12.0 * (C22 - C12) - 1.0;
    double lo = fmax(eps - pb[0], eps - pb[2]);
    double hi = fmin(pb[1] - eps, pb[3] - eps);
    if (lo > hi) { const double m = 0.5 * (lo + hi); lo = hi = m; }
    double t, dlo, dhi, dd;
    kurt_d(pb, lo, dlo, dd);
    kurt_d(pb, hi, dhi, dd);
    if (dlo >= 0.0) {
        t = lo;
    } else if (dhi <= 0.0) {
        t = hi;
    } else {
        const double scale = fmax(fmax(fabs(pb[0]), fabs(pb[1])), fmax(fabs(pb[2]), 1.0));
        t = lo + (hi - lo) * (-dlo / (dhi - dlo));
        for (int it = 0; it < 80; ++it) {
            double d1, d2;
            kurt_d(pb, t, d1, d2);
            if (d1 == 0.0) break;
            if (d1 > 0.0) hi = t; else lo = t;
            double tn = t - d1 / d2;
            if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
            const bool done = fabs(tn - t) <= 4e-16 * scale || hi - lo <= 4e-16 * scale;
            t = tn;
            if (done) break;
        }
    }
    const double p[4] = {pb[0] + t, pb[1] - t, pb[2] + t, pb[3] - t};
    eps_act = false;
    for (int k = 0; k < 4; ++k) {
        double v = p[k];
        if (v <= eps * (1.0 + 1e-12)) eps_act = true;
        v = fmax(v, eps);
        a[k] = sqrt(v);
    }
}

// Largest feasible elongation at size s, orientation th: both diagonal-dominance
// conditions C11 - |C12| >= eps/6, C22 - |C12| >= eps/6 written as linear
// inequalities in rho (multiply by (1 + rho) / s).
__device__ __forceinline__ double rho_limit(double s, double c, double sn, double eps)
{
    const double cs = fabs(c * sn), e = eps / (6.0 * s);
    double lim = INFINITY;
    const double k1 = c * c - cs - e, k2 = sn * sn - cs - e;
    if (k1 < 0.0) lim = fmin(lim, (sn * sn + cs - e) / -k1);
    if (k2 < 0.0) lim = fmin(lim, (c * c + cs - e) / -k2);
    return lim;
}

__device__ void solve_srt(double sigma, double rho, double th, double eps, double *a, bool &clamped,
                          bool &eps_act)
{
    double s = 2.0 * sigma * sigma;
    clamped = false;
    if (s < eps / 3.0) { s = eps / 3.0; rho = 1.0; clamped = true; }
    double sn, c;
    sincos(th, &sn, &c);
    const double lim = rho_limit(s, c, sn, eps);
    if (rho > lim) { rho = lim * (1.0 - 1e-12); clamped = true; }
    rho = fmax(rho, 1.0);
    const double lmin = s / (1.0 + rho), dl = lmin * (rho - 1.0);   // lambda_max - lambda_min
    solve_feasible(lmin + dl * c * c, dl * c * sn, lmin + dl * sn * sn, eps, a, eps_act);
}

__device__ bool solve_cov(double C11, double C12, double C22, double eps, double *a, bool &clamped, bool &eps_act)
{
    if (!(isfinite(C11) && isfinite(C12) && isfinite(C22))) return false;
    if (!(C11 > 0.0 && C22 > 0.0 && C11 * C22 - C12 * C12 > 0.0)) return false;
    if (C11 - fabs(C12) >= eps / 6.0 && C22 - fabs(C12) >= eps / 6.0) {
        clamped = false;
        solve_feasible(C11, C12, C22, eps, a, eps_act);
        return true;
    }
    // eigen-structure of the request, then the clamp of the (sigma, rho, theta) entry
    const double s = C11 + C22, d = sqrt((C11 - C22) * (C11 - C22) + 4.0 * C12 * C12);
    const double lmax = 0.5 * (s + d), lmin = 0.5 * (s - d);
    solve_srt(sqrt(0.5 * s), lmax / lmin, 0.5 * atan2(2.0 * C12, C11 - C22), eps, a, clamped, eps_act);
    clamped = true;
    return true;
}

__device__ __forceinline__ float warp_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

__device__ void scale_map_block(const Job &J, int lb)
{
    const int nbx = (int)((J.W + kFdBlockX - 1) / kFdBlockX);
    const int by = lb / nbx, bx = lb - by * nbx;
    const int64_t r = (int64_t)by * kFdBlockY + threadIdx.x / kFdBlockX;
    const int64_t c = (int64_t)bx * kFdBlockX + threadIdx.x % kFdBlockX;
    const bool live = r < J.H && c < J.W;
    float rx = 0.f, ry = 0.f;
    bool cl = false, ea = false, bad = false;
    if (live) {
        double a[4];
        const float *fv = J.field + r * J.f_rs;
        if (J.f_kind == kScales4) {
            const float4 v = *reinterpret_cast<const float4 *>(fv + c * 4);
            a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
            bad = !(a[0] > 0.0 && a[1] > 0.0 && a[2] > 0.0 && a[3] > 0.0 && isfinite(a[0] + a[1] + a[2] + a[3]));
        } else {
            const float f0 = fv[c * 3], f1 = fv[c * 3 + 1], f2 = fv[c * 3 + 2];
            if (J.f_kind == kSrt3) {
                bad = !(isfinite(f0) && isfinite(f1) && isfinite(f2) && f0 > 0.f && f1 >= 1.f);
                if (!bad) solve_srt(f0, f1, f2, J.eps_full, a, cl, ea);
            } else {
                bad = !solve_cov(f0, f1, f2, J.eps_full, a, cl, ea);
            }
            if (bad) {   // smallest isotropic filter instead
                const double v = sqrt(J.eps_full);
                a[0] = a[1] = a[2] = a[3] = v;
            }
            float4 o;
            o.x = (float)a[0]; o.y = (float)a[1]; o.z = (float)a[2]; o.w = (float)a[3];
            *reinterpret_cast<float4 *>(const_cast<float *>(J.scales) + r * J.sc_rs + c * 4) = o;
            // the windows are sized from the stored (rounded) scales
            a[0] = o.x; a[1] = o.y; a[2] = o.z; a[3] = o.w;
        }
        if (!bad) {
            const double d = (a[1] + a[3]) * kRsqrt2;
            rx = (float)(0.5 * (a[0] + d)) * 1.000001f;
            ry = (float)(0.5 * (a[2] + d)) * 1.000001f;
        }
    }
    const bool ovf = live && !bad && fmaxf(rx, ry) * J.inv_sqrt_m > (float)J.cap;
    // per-wave reduction, one atomic per wave (a block lies inside one tile)
    const float mrx = warp_max(rx), mry = warp_max(ry);
    const unsigned long long bcl = __ballot(cl), bea = __ballot(ea), bbad = __ballot(bad), bovf = __ballot(ovf);
    if ((threadIdx.x & 63) == 0) {
        const int tile = (int)((int64_t)by * kFdBlockY / J.T) * J.ntc + (int)((int64_t)bx * kFdBlockX / J.T);
        if (mrx > 0.f) atomicMax(reinterpret_cast<unsigned int *>(J.tile_reach) + 2 * tile, __float_as_uint(mrx));
        if (mry > 0.f) atomicMax(reinterpret_cast<unsigned int *>(J.tile_reach) + 2 * tile + 1, __float_as_uint(mry));
        if (bcl) atomicAdd(J.counters + kClamped, (unsigned long long)__popcll(bcl));
        if (bea) atomicAdd(J.counters + kEpsActive, (unsigned long long)__popcll(bea));
        if (bbad) atomicAdd(J.counters + kInvalid, (unsigned long long)__popcll(bbad));
        if (bovf) atomicAdd(J.counters + kOverflow, (unsigned long long)__popcll(bovf));
    }
}

__global__ __launch_bounds__(256) void k_scale_map(Job J)
{
    scale_map_block(J, blockIdx.x);
}

__device__ __forceinline__ int find_job(const Job *jobs, int n, int idx, int which)
{
    // largest j with base_j <= idx (bases ascending)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int b = which == 0 ? jobs[mid].tile_base : which == 1 ? jobs[mid].blk_base : jobs[mid].smap_base;
        if (b <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_scale_map_batch(const Job *jobs, int n, int total)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int j = find_job(jobs, n, b, 2);
        const Job &J = jobs[j];
        scale_map_block(J, b - J.smap_base);
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Running sums.  Three arithmetics share one sweep:
//   ArF64  : binary64;
//   ArI64  : wrapping 64-bit integers, no sqrt2 factors (the FD multiplies by 2);
//   ArF32C : binary32 (hi, lo) pairs with error-free transformations
//            (Knuth two-sum, Dekker fast-two-sum, FMA two-product).
// ---------------------------------------------------------------------------
struct ArF64 {
    using T = double;
    __device__ static T zero() { return 0.0; }
    __device__ static T from(double v) { return v; }
    __device__ static T add(T a, T b) { return a + b; }
    __device__ static T s2add(T a, T b) { return fma(kSqrt2, a, b); }   // sqrt2 a + b
    __device__ static T shfl_up(T v, int d) { return __shfl_up(v, d); }
    __device__ static void store(void *g, int64_t i, T v) { static_cast<double *>(g)[i] = v; }
};

struct ArI64 {
    using T = unsigned long long;
    __device__ static T zero() { return 0ull; }
    __device__ static T from(double v) { return (T)(long long)v; }
    __device__ static T add(T a, T b) { return a + b; }
    __device__ static T s2add(T a, T b) { return a + b; }
    __device__ static T shfl_up(T v, int d) { return __shfl_up(v, d); }
    __device__ static void store(void *g, int64_t i, T v) { static_cast<unsigned long long *>(g)[i] = v; }
};

struct DF {
    float hi, lo;
};

#pragma clang fp contract(off)
__device__ __forceinline__ DF two_sum(float a, float b)
{
    const float s = a + b;
    const float bb = s - a;
    const float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ DF fast_two_sum(float a, float b)
{
    const float s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ DF df_add(DF x, DF y)
{
    DF s = two_sum(x.hi, y.hi);
    const DF t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}
// sqrt2 as a pair: 1.41421353816986083984375 + 2.4203234...e-8
constexpr float kS2hi = 1.41421353816986083984375f;
constexpr float kS2lo = 2.42032342537213169e-08f;
__device__ __forceinline__ DF df_mul_s2(DF x)
{
    const float p = x.hi * kS2hi;
    float e = fmaf(x.hi, kS2hi, -p);
    e = e + (x.hi * kS2lo + x.lo * kS2hi);
    return fast_two_sum(p, e);
}
#pragma clang fp contract(on)

struct ArF32C {
    using T = DF;
    __device__ static T zero() { return {0.f, 0.f}; }
    __device__ static T from(double v) { const float h = (float)v; return {h, (float)(v - (double)h)}; }
    __device__ static T add(T a, T b) { return df_add(a, b); }
    __device__ static T s2add(T a, T b) { return df_add(df_mul_s2(a), b); }
    __device__ static T shfl_up(T v, int d) { return {__shfl_up(v.hi, d), __shfl_up(v.lo, d)}; }
    __device__ static void store(void *g, int64_t i, T v) { static_cast<float2 *>(g)[i] = make_float2(v.hi, v.lo); }
};

template <class A>
struct ScanLds {
    typename A::T p45[kMaxWindow + 2];   // previous row, index c + 1 (index 0 stays zero)
    typename A::T pb[kMaxWindow + 2];    // previous row, index c     (index w.. stays zero)
    typename A::T wsum[kScanChunks][kScanThreads / 64];
};

template <int IN>
__device__ __forceinline__ double load_in(const void *in, int64_t idx)
{
    if (IN == kInF32) return (double)static_cast<const float *>(in)[idx];
    return (double)static_cast<const unsigned short *>(in)[idx];
}

// One window: rows [w.r0, w.r0 + w.h) x cols [w.c0, w.c0 + w.w), channel ch of the
// job's pass input, zero outside the image; result (g_b, or G for integers) into
// gout[row * w.w + col].  Thread t owns columns c = k * 256 + t.
template <class A, int IN>
__device__ void sweep_window(const Job &J, int ch, const Window w, void *gout, ScanLds<A> &L)
{
    using T = typename A::T;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int K = (w.w + kScanThreads - 1) / kScanThreads;
    for (int i = t; i < kMaxWindow + 2; i += kScanThreads) { L.p45[i] = A::zero(); L.pb[i] = A::zero(); }
    T p90[kScanChunks];
    bool colin[kScanChunks];   // column inside the image
    int64_t colidx[kScanChunks];
#pragma unroll
    for (int k = 0; k < kScanChunks; ++k) {
        p90[k] = A::zero();
        const int c = k * kScanThreads + t;
        const int64_t C = w.c0 + c;
        colin[k] = k < K && c < w.w && C >= 0 && C < J.W;
        colidx[k] = C * J.C + ch;
    }
    const unsigned char *inb = static_cast<const unsigned char *>(J.in);
    const int esz = IN == kInF32 ? 4 : 2;
    // prefetch the first row
    double nxt[kScanChunks];
    auto fetch = [&](int rr, double *dst) {
        const int64_t R = w.r0 + rr;
        const bool rin = rr < w.h && R >= 0 && R < J.H;
        const void *rowp = inb + (size_t)(R * J.in_rs) * esz;
#pragma unroll
        for (int k = 0; k < kScanChunks; ++k) dst[k] = (rin && colin[k]) ? load_in<IN>(rowp, colidx[k]) : 0.0;
    };
    fetch(0, nxt);
    lds_barrier();
    for (int rr = 0; rr < w.h; ++rr) {
        double cur[kScanChunks];
#pragma unroll
        for (int k = 0; k < kScanChunks; ++k) cur[k] = nxt[k];
        fetch(rr + 1, nxt);   // in flight across the barriers below
        // RS1: prefix along the row (chunk-wise wave scans, wave totals in LDS)
        T v[kScanChunks];
#pragma unroll
        for (int k = 0; k < kScanChunks; ++k) {
            v[k] = A::from(cur[k]);
            if (k < K) {
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const T o = A::shfl_up(v[k], d);
                    if (lane >= d) v[k] = A::add(v[k], o);
                }
                if (lane == 63) L.wsum[k][wave] = v[k];
            }
        }
        lds_barrier();
        T carry = A::zero();
        T g45[kScanChunks], gb[kScanChunks];
#pragma unroll
        for (int k = 0; k < kScanChunks; ++k) {
            if (k < K) {
                T off = carry;
#pragma unroll
                for (int q = 0; q < kScanThreads / 64; ++q) {
                    if (q < wave) off = A::add(off, L.wsum[k][q]);
                    carry = A::add(carry, L.wsum[k][q]);
                }
                const int c = k * kScanThreads + t;
                const T g0 = A::add(v[k], off);
                g45[k] = A::s2add(g0, L.p45[c]);          // RS2: sqrt2 g0 + g45[r-1][c-1]
                p90[k] = A::add(g45[k], p90[k]);          // RS3: g45 + g90[r-1][c]
                gb[k] = A::s2add(p90[k], L.pb[c + 1]);    // RS4: sqrt2 g90 + gb[r-1][c+1]
            }
        }
        lds_barrier();
#pragma unroll
        for (int k = 0; k < kScanChunks; ++k) {
            const int c = k * kScanThreads + t;
            if (k < K && c < w.w) {
                L.p45[c + 1] = g45[k];
                L.pb[c] = gb[k];
                A::store(gout, (int64_t)rr * w.w + c, gb[k]);
            }
        }
    }
}

template <class A, int IN>
__global__ __launch_bounds__(kScanThreads) void k_preint(Job J)
{
    __shared__ ScanLds<A> L;
    const int tile = blockIdx.x / J.C, ch = blockIdx.x - tile * J.C;
    const Window w = window_of(J, tile);
    void *gout = static_cast<unsigned char *>(J.g) + ((int64_t)tile * J.C + ch) * J.slot_elems * sizeof(typename A::T);
    sweep_window<A, IN>(J, ch, w, gout, L);
}

template <class A>
__global__ __launch_bounds__(kScanThreads) void k_preint_batch(const Job *jobs, int n, int total)
{
    __shared__ ScanLds<A> L;
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int j = find_job(jobs, n, b, 0);
        const Job &J = jobs[j];
        const int lt = b - J.tile_base;
        const int tile = lt / J.C, ch = lt - tile * J.C;
        const Window w = window_of(J, tile);
        void *gout = static_cast<unsigned char *>(J.g) + ((int64_t)tile * J.C + ch) * J.slot_elems * sizeof(typename A::T);
        if (J.in_type == kInU16) sweep_window<A, kInU16>(J, ch, w, gout, L);
        else sweep_window<A, kInF32>(J, ch, w, gout, L);
        lds_barrier();
    }
}

template <class A, int IN>
__global__ __launch_bounds__(kScanThreads) void k_preint_window(Job J, int ch, Window w, void *g)
{
    __shared__ ScanLds<A> L;
    sweep_window<A, IN>(J, ch, w, g, L);
}

// ---------------------------------------------------------------------------
// Finite difference + ZP interpolation (eq. (final_eqn), App. F).
//
// F(y) = sum_m g[m] ZP(y - m).  With m0 = round(y) and d = y - m0 in [-1/2, 1/2]^2,
// ZP(d - k) is non-zero for 7 offsets k, and on each of the 4 triangles of the
// cell cut by its diagonals it is one quadratic in d.  ZP is symmetric under the
// 8 symmetries of the square, so one canonical triangle {s >= |t|} serves all:
// d = s sa + t sb with (sa, sb) a signed pair of lattice axes, k = k1 sa + k2 sb,
// and with the ZP element written as the density of T1(1,0)+T2(1,1)+T3(0,1)+T4(-1,1)
// (T_k uniform on [-1/2, 1/2]) the weights on the canonical triangle are
//   k = (0,0): (1 - s^2 - t^2)/2        k = (1,0): 1/8 + s/2 - t^2/2
//   k = (-1,0): (1 - 2s)^2 / 8           k = (0,+-1): 1/8 +- t/2 - s^2/4 -+ s t/2 + t^2/4
//   k = (1,+-1): (s +- t)^2 / 4
// (they sum to 1).  Grouped by monomials, 8 F = C0 + s (Cs + s Css + t Cst) + t (Ct + t Ctt).
// ---------------------------------------------------------------------------
template <int PRE>
__device__ __forceinline__ double gload(const void *g, int64_t i)
{
    if (PRE == kPreF64) return static_cast<const double *>(g)[i];
    if (PRE == kPreI64) return (double)static_cast<const long long *>(g)[i];
    const float2 v = static_cast<const float2 *>(g)[i];
    return (double)v.x + (double)v.y;
}

template <int PRE, int NCH, typename R>
__device__ __forceinline__ void fd_pixel(const Job &J, int tile, const Window &w, int64_t r, int64_t c)
{
    const float4 af = *reinterpret_cast<const float4 *>(J.scales + r * J.sc_rs + c * 4);
    const R m = (R)J.inv_sqrt_m_d;
    const R a1 = (R)af.x * m, a2 = (R)af.y * m, a3 = (R)af.z * m, a4 = (R)af.w * m;
    const R ap2 = a2 * (R)kRsqrt2, ap4 = a4 * (R)kRsqrt2;
    // y_i = n + tau - x_i, in window coordinates (tau: Sec. 4.1 step (2))
    const R cx = (R)(c - w.c0) + (R)0.5 * (a1 + ap2 - ap4 - (R)1);
    const R cy = (R)(r - w.r0) + (R)0.5 * (ap2 + a3 + ap4 - (R)3);
    const R wgt = (PRE == kPreI64 ? (R)2 : (R)1) / ((R)8 * a1 * a2 * a3 * a4);
    const unsigned char *gbase = static_cast<const unsigned char *>(J.g);
    const int64_t esz = 8;   // double, int64 and (hi, lo) float pairs are all 8 bytes
    const void *gch[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) gch[ch] = gbase + ((int64_t)tile * J.C + ch) * J.slot_elems * esz;
    R acc[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) acc[ch] = (R)0;
    const int ww = w.w;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int q1 = i & 1, q2 = (i >> 1) & 1, q3 = (i >> 2) & 1, q4 = (i >> 3) & 1;
        // Table 1: x_i = (q1 a1 + q2 a'2 - q4 a'4, q2 a'2 + q3 a3 + q4 a'4), w_i = (-1)^(q1+q2+q3+q4) w
        R x = cx, y = cy;
        if (q1) x -= a1;
        if (q2) { x -= ap2; y -= ap2; }
        if (q3) y -= a3;
        if (q4) { x += ap4; y -= ap4; }
        const R mx = rint(x), my = rint(y);
        const R dx = x - mx, dy = y - my;
        int ix = (int)mx, iy = (int)my;
        ix = min(max(ix, 1), ww - 2);
        iy = min(max(iy, 1), w.h - 2);
        const int base = iy * ww + ix;
        const R adx = fabs(dx), ady = fabs(dy);
        const bool hz = adx >= ady;
        const R s = hz ? adx : ady;
        const R tt = hz ? dy : dx;
        const int oa = hz ? (dx >= (R)0 ? 1 : -1) : (dy >= (R)0 ? ww : -ww);
        const int ob = hz ? ww : 1;
        const bool neg = (q1 + q2 + q3 + q4) & 1;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const R g00 = (R)gload<PRE>(gch[ch], base);
            const R g10 = (R)gload<PRE>(gch[ch], base + oa);
            const R gm0 = (R)gload<PRE>(gch[ch], base - oa);
            const R g01 = (R)gload<PRE>(gch[ch], base + ob);
            const R g0m = (R)gload<PRE>(gch[ch], base - ob);
            const R g11 = (R)gload<PRE>(gch[ch], base + oa + ob);
            const R g1m = (R)gload<PRE>(gch[ch], base + oa - ob);
            const R sv = g01 + g0m, sd = g11 + g1m;
            const R C0 = (R)4 * g00 + g10 + gm0 + sv;
            const R Cs = (R)4 * (g10 - gm0);
            const R Ct = (R)4 * (g01 - g0m);
            const R Css = (R)4 * (gm0 - g00) + (R)2 * (sd - sv);
            const R Cst = (R)4 * ((g0m - g01) + (g11 - g1m));
            const R Ctt = (R)-4 * (g00 + g10) + (R)2 * (sv + sd);
            const R F8 = C0 + s * (Cs + s * Css + tt * Cst) + tt * (Ct + tt * Ctt);
            acc[ch] = neg ? acc[ch] - F8 : acc[ch] + F8;
        }
    }
    float *o = J.out + r * J.out_rs + c * J.C;
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) o[ch] = (float)(acc[ch] * wgt);
}

template <int PRE, int NCH, typename R>
__device__ __forceinline__ void fd_block(const Job &J, int lb)
{
    // tile-major block order: all blocks of tile 0, then tile 1, ...
    const int bpt_x = J.T / kFdBlockX, bpt_y = J.T / kFdBlockY, bpt = bpt_x * bpt_y;
    const int tile = lb / bpt, rem = lb - tile * bpt;
    const int by = rem / bpt_x, bx = rem - by * bpt_x;
    const int ti = tile / J.ntc, tj = tile - ti * J.ntc;
    const int64_t r = (int64_t)ti * J.T + by * kFdBlockY + threadIdx.x / kFdBlockX;
    const int64_t c = (int64_t)tj * J.T + bx * kFdBlockX + threadIdx.x % kFdBlockX;
    if (tile >= J.ntr * J.ntc || r >= J.H || c >= J.W) return;
    const Window w = window_of(J, tile);
    fd_pixel<PRE, NCH, R>(J, tile, w, r, c);
}

template <int PRE, int NCH, typename R>
__global__ __launch_bounds__(256) void k_fd(Job J, int nblocks)
{
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    if (lb < nblocks) fd_block<PRE, NCH, R>(J, lb);
}

template <int PRE, typename R>
__global__ __launch_bounds__(256) void k_fd_batch(const Job *jobs, int n, int total)
{
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int j = find_job(jobs, n, b, 1);
        const Job &J = jobs[j];
        switch (J.C) {
        case 1: fd_block<PRE, 1, R>(J, b - J.blk_base); break;
        case 2: fd_block<PRE, 2, R>(J, b - J.blk_base); break;
        case 3: fd_block<PRE, 3, R>(J, b - J.blk_base); break;
        default: fd_block<PRE, 4, R>(J, b - J.blk_base); break;
        }
    }
}

inline int grid_for(int64_t n, int per)
{
    return (int)((n + per - 1) / per);
}

}  // namespace

int64_t slot_elems_for(int T, int cap)
{
    const int64_t side = (int64_t)T + 2 * (int64_t)cap + 5;
    return side * side;
}

int scale_map_blocks(int64_t H, int64_t W)
{
    return (int)(((W + kFdBlockX - 1) / kFdBlockX) * ((H + kFdBlockY - 1) / kFdBlockY));
}

int fd_blocks_job(const Job &j)
{
    return j.ntr * j.ntc * (j.T / kFdBlockX) * (j.T / kFdBlockY);
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_scale_map(const Job &j, hipStream_t s)
{
    const int nb = scale_map_blocks(j.H, j.W);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_map, dim3(nb), dim3(256), 0, s, j);
    return hipGetLastError();
}

template <class A>
static hipError_t launch_preint_t(const Job &j, hipStream_t s)
{
    const int nb = j.ntr * j.ntc * j.C;
    if (nb == 0) return hipSuccess;
    if (j.in_type == kInF32)
        hipLaunchKernelGGL((k_preint<A, kInF32>), dim3(nb), dim3(kScanThreads), 0, s, j);
    else
        hipLaunchKernelGGL((k_preint<A, kInU16>), dim3(nb), dim3(kScanThreads), 0, s, j);
    return hipGetLastError();
}

hipError_t launch_preint(const Job &j, hipStream_t s)
{
    switch (j.preint) {
    case kPreF64: return launch_preint_t<ArF64>(j, s);
    case kPreF32C: return launch_preint_t<ArF32C>(j, s);
    case kPreI64:
        if (j.in_type != kInU16) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_preint<ArI64, kInU16>), dim3(j.ntr * j.ntc * j.C), dim3(kScanThreads), 0, s, j);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

hipError_t launch_preint_window(const Job &j, int channel, int64_t r0, int64_t c0, int h, int w, void *g,
                                hipStream_t s)
{
    Window win;
    win.r0 = r0; win.c0 = c0; win.h = h; win.w = w;
    switch (j.preint) {
    case kPreF64:
        if (j.in_type == kInF32) hipLaunchKernelGGL((k_preint_window<ArF64, kInF32>), dim3(1), dim3(kScanThreads), 0, s, j, channel, win, g);
        else hipLaunchKernelGGL((k_preint_window<ArF64, kInU16>), dim3(1), dim3(kScanThreads), 0, s, j, channel, win, g);
        break;
    case kPreF32C:
        if (j.in_type == kInF32) hipLaunchKernelGGL((k_preint_window<ArF32C, kInF32>), dim3(1), dim3(kScanThreads), 0, s, j, channel, win, g);
        else hipLaunchKernelGGL((k_preint_window<ArF32C, kInU16>), dim3(1), dim3(kScanThreads), 0, s, j, channel, win, g);
        break;
    case kPreI64:
        if (j.in_type != kInU16) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_preint_window<ArI64, kInU16>), dim3(1), dim3(kScanThreads), 0, s, j, channel, win, g);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PRE, typename R>
static hipError_t launch_fd_ch(const Job &j, int nb, int grid, hipStream_t s)
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

hipError_t launch_fd(const Job &j, hipStream_t s)
{
    const int nb = fd_blocks_job(j);
    if (nb == 0) return hipSuccess;
    const int grid = (nb + 7) / 8 * 8;
    if (j.fd_fp32) {
        switch (j.preint) {
        case kPreF64: return launch_fd_ch<kPreF64, float>(j, nb, grid, s);
        case kPreF32C: return launch_fd_ch<kPreF32C, float>(j, nb, grid, s);
        case kPreI64: return launch_fd_ch<kPreI64, float>(j, nb, grid, s);
        }
    } else {
        switch (j.preint) {
        case kPreF64: return launch_fd_ch<kPreF64, double>(j, nb, grid, s);
        case kPreF32C: return launch_fd_ch<kPreF32C, double>(j, nb, grid, s);
        case kPreI64: return launch_fd_ch<kPreI64, double>(j, nb, grid, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_scale_map_batch(const Job *jobs, int n, int total_blocks, int grid, hipStream_t s)
{
    if (total_blocks == 0) return hipSuccess;
    grid = std::max(1, std::min(grid, total_blocks));
    hipLaunchKernelGGL(k_scale_map_batch, dim3(grid), dim3(256), 0, s, jobs, n, total_blocks);
    return hipGetLastError();
}

hipError_t launch_preint_batch(const Job *jobs, int n, int total_tiles, int grid, int preint, hipStream_t s)
{
    if (total_tiles == 0) return hipSuccess;
    grid = std::max(1, std::min(grid, total_tiles));
    switch (preint) {
    case kPreF64: hipLaunchKernelGGL((k_preint_batch<ArF64>), dim3(grid), dim3(kScanThreads), 0, s, jobs, n, total_tiles); break;
    case kPreF32C: hipLaunchKernelGGL((k_preint_batch<ArF32C>), dim3(grid), dim3(kScanThreads), 0, s, jobs, n, total_tiles); break;
    case kPreI64: hipLaunchKernelGGL((k_preint_batch<ArI64>), dim3(grid), dim3(kScanThreads), 0, s, jobs, n, total_tiles); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fd_batch(const Job *jobs, int n, int total_blocks, int grid, int preint, int fd_fp32, hipStream_t s)
{
    if (total_blocks == 0) return hipSuccess;
    grid = std::max(1, std::min(grid, total_blocks));
#define SVF_FDB(P, R) hipLaunchKernelGGL((k_fd_batch<P, R>), dim3(grid), dim3(256), 0, s, jobs, n, total_blocks)
    if (fd_fp32) {
        switch (preint) {
        case kPreF64: SVF_FDB(kPreF64, float); break;
        case kPreF32C: SVF_FDB(kPreF32C, float); break;
        case kPreI64: SVF_FDB(kPreI64, float); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (preint) {
        case kPreF64: SVF_FDB(kPreF64, double); break;
        case kPreF32C: SVF_FDB(kPreF32C, double); break;
        case kPreI64: SVF_FDB(kPreI64, double); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef SVF_FDB
    return hipGetLastError();
}

}  // namespace svf

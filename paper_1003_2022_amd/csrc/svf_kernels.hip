// svf_kernels.hip -- gfx950 kernels of the space-variant elliptical box-spline
// filter (Chaudhury, Munoz-Barrutia, Unser, "Fast space-variant elliptical
// filtering using box splines").
//
//   k_scale_map : per pixel, covariance field -> box scales (Sec. 3.2.2) and, per tile,
//                 the support half-widths that size the pre-integration windows.
//   k_preint    : running sums RS1..RS4 (Sec. 3.1 step (1), Algorithm 1 step 2) of one
//                 tile's window, one work-group sweeping the rows top to bottom as a
//                 pipeline of waves (input loads, RS1, RS2..RS4 and stores).
//   k_preint_window / k_preint_batch : the same sums for a caller's window and for
//                 the batched launches.
//   (k_fd, the finite difference, is in svf_fd.hip)
//
// Lattice: x = column, y = row, directions u1 = (1,0), u2 = (1,1)/sqrt2, u3 = (0,1),
// u4 = (-1,1)/sqrt2; the running sums step by b_k u_k = (1,0), (1,1), (0,1), (-1,1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "svf_device.h"
#include "svf_internal.h"
#include "svf_sincos_table.h"

namespace svf {

namespace {

// ---------------------------------------------------------------------------
// Scale map (Sec. 3.2.2).  All in binary64.
// ---------------------------------------------------------------------------

// Quotient and square root for positive, finite binary64 operands: the hardware
// estimates (about 2^-23 relative) refined by Newton / Goldschmidt steps to about
// 1e-15 relative.  Enough for scales that are stored in binary32, and a fraction
// of the cost of the correctly rounded library sequences.
__device__ __forceinline__ double div_pos(double a, double b)   // b > 0
{
    double r = __builtin_amdgcn_rcp(b);
    r = fma(r, fma(-b, r, 1.0), r);
    r = fma(r, fma(-b, r, 1.0), r);
    const double q = a * r;
    return fma(r, fma(-b, q, a), q);
}

__device__ __forceinline__ double sqrt_pos(double x)   // x > 0
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    return fma(fma(-g, g, x), h, g);
}

// Square root for a value stored in binary32: the hardware estimate and one
// Goldschmidt step, ~1e-14 relative.
__device__ __forceinline__ double sqrt_f32out(double x)   // x > 0
{
    const double y = __builtin_amdgcn_rsq(x);
    const double g = x * y, h = 0.5 * y;
    return fma(g, fma(-g, h, 0.5), g);
}

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

// The minimiser's equation (Sec. 3.2.2): zeta'(t) = 32 t^3 + z2 t^2 + z3 t + z4 = 0 with
// the coefficients taken from the particular solution pb.  zeta'' >= 8 sum p^2 > 0, so
// zeta' is strictly increasing and, with t = x - b, b = z2 / 96, zeta' / 32 is the
// depressed cubic x^3 + P x + Q with P > 0 (P = zeta''(-b) / 32) and one real root.
struct Cubic {
    double b, P, Q;
};

__device__ __forceinline__ Cubic zeta_cubic(const double *pb)
{
    const double p1 = pb[0], p2 = pb[1], p3 = pb[2], p4 = pb[3];
    const double s13 = p1 + p3, s24 = p2 + p4;
    const double z2 = 24.0 * (s13 - s24);
    const double z3 = 16.0 * (p1 * p1 + p2 * p2 + p3 * p3 + p4 * p4) - 8.0 * s13 * s24;
    const double z4 = 4.0 * (p1 * p1 * p1 - p2 * p2 * p2 + p3 * p3 * p3 - p4 * p4 * p4) +
                      2.0 * s13 * (p2 * p2 + p4 * p4) - 2.0 * s24 * (p1 * p1 + p3 * p3);
    Cubic c;
    c.b = z2 * (1.0 / 96.0);
    const double e3 = z3 * (1.0 / 32.0);
    c.P = e3 - 3.0 * c.b * c.b;
    c.Q = c.b * (2.0 * c.b * c.b - e3) + z4 * (1.0 / 32.0);
    return c;
}

// Its root t: Cardano's formula with the larger cube root taken first (the two
// terms of u have one sign, so nothing cancels), at the hardware estimates' ~1e-7
// and a binary32 cube root, x0 within ~1e-6 of the scale; two Newton steps on the
// depressed cubic (error e -> K e^2 + 1e-7 e, K <= 0.9 / sqrt(P)).  As written they
// resolve the root to ~3e-14 of the scale where P >= scale^2 / 100 (checked against
// exact rational roots; enough for scales stored in binary32) but only to ~1e-11 where
// P is smaller (P, Q come from cancelling sums); there a last Newton step on zeta'
// evaluated from the shifted components (kurt_d) takes it to ~1e-16.  `last` is the
// last step taken, for the caller's convergence check.
__device__ __forceinline__ double cubic_root(const double *pb, const Cubic &c, double scale, double &last)
{
    const double D = 0.25 * c.Q * c.Q + c.P * c.P * c.P * (1.0 / 27.0);   // > 0
    const double sD = D > 0.0 ? D * __builtin_amdgcn_rsq(D) : 0.0;
    const double u = -0.5 * c.Q - copysign(sD, c.Q);
    const float au = (float)fabs(u);
    const double A = copysign((double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf(au) * (1.0f / 3.0f)), u);
    double x = au > 0.0f ? A - c.P * (1.0 / 3.0) * __builtin_amdgcn_rcp(A) : 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double x2 = x * x;
        const double f = fma(x, x2 + c.P, c.Q), fp = fma(3.0, x2, c.P);
        last = f * __builtin_amdgcn_rcp(fp);
        x -= last;
    }
    double t = x - c.b;
    if (!(c.P >= 0.01 * scale * scale)) {
        double d1, d2;
        kurt_d(pb, t, d1, d2);
        last = d1 * __builtin_amdgcn_rcp(d2);
        t -= last;
    }
    return t;
}

// Covariance (whole filter) -> scales, floor eps on a^2.  The feasible set of
// M p = c, p >= eps is p = pbar + t e, t in [lo, hi]; ||K||^2 is strictly convex in t,
// so its minimiser over the interval is the root of zeta' clamped to [lo, hi].  The
// scales are stored in binary32; the root is resolved to ~1e-16 of the scale.  A
// root whose last Newton step was not small (never seen; kept for safety: a NaN,
// or P rounded to ~0) is redone by Newton steps inside a shrinking bracket, from
// the derivative evaluated on the shifted components.
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
    const double scale = fmax(fmax(fabs(pb[0]), fabs(pb[1])), fmax(fabs(pb[2]), 1.0));
    const Cubic cb = zeta_cubic(pb);
    double last;
    double t = cubic_root(pb, cb, scale, last);
    if (fabs(last) <= 1e-9 * scale) {
        t = fmin(fmax(t, lo), hi);
    } else {
        const double tol = 1e-13 * scale;
        t = 0.5 * (lo + hi);
        for (int it = 0; it < 60; ++it) {
            double d1, d2;
            kurt_d(pb, t, d1, d2);
            const double step = div_pos(d1, d2);   // d2 >= 8 sum p^2 > 0
            // converged: take the last (sub-tolerance) step; tested before the bracket
            // update, since a step below one ulp of t would otherwise read as leaving
            // the bracket and restart bisection from its far end
            if (fabs(step) <= tol) { t = fmin(fmax(t - step, lo), hi); break; }
            if (d1 > 0.0) hi = t; else lo = t;
            double tn = t - step;
            if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
            t = tn;
            if (hi - lo <= tol) break;
        }
    }
    const double p[4] = {pb[0] + t, pb[1] - t, pb[2] + t, pb[3] - t};
    eps_act = false;
    for (int k = 0; k < 4; ++k) {
        double v = p[k];
        if (v <= eps * (1.0 + 1e-12)) eps_act = true;
        v = fmax(v, eps);
        a[k] = sqrt_f32out(v);
    }
}

// sin and cos of th: Cody-Waite reduction modulo pi/2 (pi/2 as the sum of two
// doubles, the product with the quotient taken by fused multiply-adds) to |r| <= pi/4,
// then r = k h + e with h = pi/128 to 46 significant bits (k h exact, e exact,
// |e| <= h/2): sin r = sin(kh) cos e + cos(kh) sin e, cos r = cos(kh) cos e - sin(kh) sin e,
// the pair (sin(kh), cos(kh)) from a 65-entry table (svf_sincos_table.h) and the
// Taylor series of sin e to e^5 and cos e to e^6 (truncation below 1e-17).  About 2 ulp
// for |th| < 2^20 (field angles lie in [0, pi)); about half the operations of a
// series on the whole quarter period.
__device__ __forceinline__ void sincos_red(double th, double *sn, double *cs)
{
    constexpr double kTwoOverPi = 0.63661977236758134308;
    constexpr double kPio2Hi = 1.57079632679489655800e+00;   // pi/2 rounded to a double
    constexpr double kPio2Lo = 6.12323399573676603587e-17;   // pi/2 - kPio2Hi
    const double q = rint(th * kTwoOverPi);
    const double r = fma(-q, kPio2Lo, fma(-q, kPio2Hi, th));
    const double k = fmin(fmax(rint(r * kSinCosInvH), -32.0), 32.0);
    const double e = fma(-k, kSinCosH, r);
    const double2 t = *reinterpret_cast<const double2 *>(&kSinCosTab[(int)k + 32][0]);
    const double e2 = e * e;
    const double se = fma(e * e2, fma(e2, 1.0 / 120.0, -1.0 / 6.0), e);
    const double ce = fma(e2, fma(e2, fma(e2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
    const double sv = fma(t.x, ce, t.y * se), cv = fma(t.y, ce, -(t.x * se));
    switch ((int)q & 3) {
    case 0: *sn = sv; *cs = cv; break;
    case 1: *sn = cv; *cs = -sv; break;
    case 2: *sn = -sv; *cs = -cv; break;
    default: *sn = -cv; *cs = sv; break;
    }
}

// Largest feasible elongation at size s, orientation th: both diagonal-dominance
// conditions C11 - |C12| >= eps/6, C22 - |C12| >= eps/6 written as linear
// inequalities in rho (multiply by 6 (1 + rho) s).  Returns rho if it satisfies
// both (the usual case, no division), else the limit.
__device__ __forceinline__ double rho_feasible(double rho, double s, double c, double sn, double eps)
{
    const double s6 = 6.0 * s, cs = fabs(c * sn);
    const double k1 = fma(s6, c * c - cs, -eps), k2 = fma(s6, sn * sn - cs, -eps);
    const double n1 = fma(s6, sn * sn + cs, -eps), n2 = fma(s6, c * c + cs, -eps);
    if (!((k1 < 0.0 && rho * -k1 > n1) || (k2 < 0.0 && rho * -k2 > n2))) return rho;
    double lim = INFINITY;
    if (k1 < 0.0) lim = fmin(lim, div_pos(n1, -k1));
    if (k2 < 0.0) lim = fmin(lim, div_pos(n2, -k2));
    return lim;
}

// (sigma, rho, theta) request -> covariance, after the clamp of s and rho into the
// feasible set (Sec. 3.2.2).
__device__ __forceinline__ void srt_clamp(double sigma, double rho, double th, double eps, double &C11, double &C12,
                                          double &C22, bool &clamped)
{
    double s = 2.0 * sigma * sigma;
    clamped = false;
    if (s < eps * (1.0 / 3.0)) { s = eps * (1.0 / 3.0); rho = 1.0; clamped = true; }
    double sn, c;
    sincos_red(th, &sn, &c);
    const double lim = rho_feasible(rho, s, c, sn, eps);
    if (lim != rho) { rho = lim * (1.0 - 1e-12); clamped = true; }
    rho = fmax(rho, 1.0);
    const double lmin = div_pos(s, 1.0 + rho), dl = lmin * (rho - 1.0);   // lambda_max - lambda_min
    C11 = lmin + dl * c * c;
    C12 = dl * c * sn;
    C22 = lmin + dl * sn * sn;
}

__device__ void solve_srt(double sigma, double rho, double th, double eps, double *a, bool &clamped,
                          bool &eps_act)
{
    double C11, C12, C22;
    srt_clamp(sigma, rho, th, eps, C11, C12, C22, clamped);
    solve_feasible(C11, C12, C22, eps, a, eps_act);
}

__device__ bool solve_cov(double C11, double C12, double C22, double eps, double *a, bool &clamped, bool &eps_act)
{
    if (!(isfinite(C11) && isfinite(C12) && isfinite(C22))) return false;
    if (!(C11 > 0.0 && C22 > 0.0 && C11 * C22 - C12 * C12 > 0.0)) return false;
    clamped = false;
    if (!(C11 - fabs(C12) >= eps * (1.0 / 6.0) && C22 - fabs(C12) >= eps * (1.0 / 6.0))) {
        // eigen-structure of the request, then the clamp of the (sigma, rho, theta) entry
        const double s = C11 + C22, d = sqrt((C11 - C22) * (C11 - C22) + 4.0 * C12 * C12);
        const double lmax = 0.5 * (s + d), lmin = 0.5 * (s - d);
        srt_clamp(sqrt(0.5 * s), lmax / lmin, 0.5 * atan2(2.0 * C12, C11 - C22), eps, C11, C12, C22, clamped);
        clamped = true;
    }
    solve_feasible(C11, C12, C22, eps, a, eps_act);
    return true;
}

// Look-up-table scale map (Sec. 3.2.2, O1/O2): theta reduced to its octant k and
// phi = theta - k pi/4, the unit-size table interpolated bilinearly at
// (1/rho, phi), the vector rotated by k places ((a1,a2,a3,a4) -> (a4,a1,a2,a3)
// per octant) and scaled by sqrt(s).  In binary32: the interpolation is
// continuous across cells and octants, so rounding moves the result by about
// one float32 ulp of the stored scales.  The flags are for the report only:
// clamped = the elongation lies beyond the table's feasible limit, eps_act = a
// tabulated component at the floor.
constexpr double kPiD = 3.14159265358979323846;

struct FieldEntry {   // three floats of a field pixel, moved as one access
    float x, y, z;
};

__device__ void lut_scales(const Job &J, float s, double rho_d, double th_d, double *a, bool &clamped, bool &eps_act)
{
    // table coordinates in binary64: next to the clamped row (u = 0) neighbouring
    // nodes differ by O(1), so the coordinate must be exact to far below 1e-6
    constexpr double kQ = 0.25 * kPiD, kInvPi = 1.0 / kPiD, kInvQ = 4.0 / kPiD;
    const double th = th_d - kPiD * floor(th_d * kInvPi);
    const int k = min(max((int)floor(th * kInvQ), 0), 3);
    const double phi_d = th - k * kQ;
    const int n = J.lut_n;
    const double fu = div_pos(1.0, rho_d) * (n - 1), fp = phi_d * kInvQ * (n - 1);
    const int i0 = min(max((int)floor(fu), 0), n - 2), j0 = min(max((int)floor(fp), 0), n - 2);
    const float wu = (float)(fu - i0), wp = (float)(fp - j0);
    const float phi = (float)phi_d, rho = (float)rho_d;
    const float4 *T = reinterpret_cast<const float4 *>(J.lut) + (int64_t)i0 * n + j0;
    const float4 t00 = T[0], t01 = T[1], t10 = T[n], t11 = T[n + 1];
    const float w00 = (1.0f - wu) * (1.0f - wp), w01 = (1.0f - wu) * wp, w10 = wu * (1.0f - wp), w11 = wu * wp;
    float v[4];
    v[0] = w00 * t00.x + w01 * t01.x + w10 * t10.x + w11 * t11.x;
    v[1] = w00 * t00.y + w01 * t01.y + w10 * t10.y + w11 * t11.y;
    v[2] = w00 * t00.z + w01 * t01.z + w10 * t10.z + w11 * t11.z;
    v[3] = w00 * t00.w + w01 * t01.w + w10 * t10.w + w11 * t11.w;
    const float r = sqrtf(s);
#pragma unroll
    for (int q = 0; q < 4; ++q) a[(q + k) & 3] = (double)(r * v[q]);
    // report: the two diagonal-dominance conditions at s = 1 (as rho_feasible)
    float sn, c;
    sincosf(phi, &sn, &c);
    const float cs = fabsf(c * sn), e = (float)J.lut_eps / 6.0f;
    const float k1 = c * c - cs - e, k2 = sn * sn - cs - e;
    clamped = (k1 < 0.0f && rho * -k1 > sn * sn + cs - e) || (k2 < 0.0f && rho * -k2 > c * c + cs - e);
    const float vmin = fminf(fminf(v[0], v[1]), fminf(v[2], v[3]));
    eps_act = vmin * vmin <= (float)J.lut_eps * (1.0f + 1e-5f);
}

// (s, rho, theta) of a covariance entry; false if it is not positive definite.
// The smaller eigenvalue as det / larger (no cancellation).
__device__ bool srt_of_cov(double C11, double C12, double C22, float &s, double &rho, double &th)
{
    if (!(isfinite(C11) && isfinite(C12) && isfinite(C22))) return false;
    const double det = C11 * C22 - C12 * C12;
    if (!(C11 > 0.0 && C22 > 0.0 && det > 0.0)) return false;
    const double sd = C11 + C22;
    const double lmax = 0.5 * (sd + sqrt((C11 - C22) * (C11 - C22) + 4.0 * C12 * C12));
    s = (float)sd;
    rho = lmax * lmax / det;   // lmax / lmin with lmin = det / lmax
    th = 0.5 * atan2(2.0 * C12, C11 - C22);
    return true;
}

__global__ void k_lut_build(float4 *T, int n, double eps)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    const int i = idx / n, j = idx - i * n;
    const double rho = i > 0 ? (double)(n - 1) / (double)i : 1e300;   // i = 0: unbounded (clamped)
    double a[4];
    bool cl, ea;
    solve_srt(sqrt(0.5), rho, (double)j * (0.25 * kPiD) / (double)(n - 1), eps, a, cl, ea);
    T[idx] = make_float4((float)a[0], (float)a[1], (float)a[2], (float)a[3]);
}

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// One block: 64 columns x (4 waves x kSmapRows) rows, inside one tile.  KIND fixes
// the field kind at compile time (-1: read from the job), so that a launch carries
// only its kind's solve and the registers that one needs.
template <bool LUT, int KIND = -1>
__device__ void scale_map_block(const Job &J, int lb)
{
    const int f_kind = KIND >= 0 ? KIND : J.f_kind;
    __shared__ float s_rx[4], s_ry[4];
    __shared__ uint32_t s_cnt[4][4];
    const int rows_per_block = 4 * kSmapRows;
    const int nbx = (int)((J.W + kSmapCols - 1) / kSmapCols);
    const int by = lb / nbx, bx = lb - by * nbx;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t c = (int64_t)bx * kSmapCols + lane;
    float rx = 0.f, ry = 0.f;
    uint32_t ncl = 0, nea = 0, nbad = 0, novf = 0;
    // the pixels' field entries are loaded up front (one 12-byte access each), so
    // the four rows' memory latencies overlap (table lookup, and a solve of a
    // kind fixed at compile time, whose rows are unrolled)
    constexpr bool kPre = LUT || KIND == kSrt3 || KIND == kCov3;
    FieldEntry pf[kSmapRows];
    if constexpr (kPre) {
        if (f_kind != kScales4) {
#pragma unroll
            for (int k = 0; k < kSmapRows; ++k) {
                const int64_t r = (int64_t)by * rows_per_block + wave * kSmapRows + k;
                if (r < J.H && c < J.W) {
                    const float *q = J.field + r * J.f_rs + c * 3;   // three adjacent dwords: one access
                    pf[k].x = load_global(q);
                    pf[k].y = load_global(q + 1);
                    pf[k].z = load_global(q + 2);
                }
            }
        }
    }
    auto pixel = [&](int k) {
        const int64_t r = (int64_t)by * rows_per_block + wave * kSmapRows + k;
        if (!(r < J.H && c < J.W)) return;
        double a[4];
        bool cl = false, ea = false, bad = false;
        const float *fv = J.field + r * J.f_rs;
        if (f_kind == kScales4) {
            const f32x4 v = load_global(reinterpret_cast<const f32x4 *>(fv + c * 4));
            a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
            bad = !(a[0] > 0.0 && a[1] > 0.0 && a[2] > 0.0 && a[3] > 0.0 && isfinite(a[0] + a[1] + a[2] + a[3]));
        } else {
            float f0, f1, f2;
            if constexpr (kPre) {
                f0 = pf[k].x; f1 = pf[k].y; f2 = pf[k].z;
            } else {
                f0 = load_global(fv + c * 3); f1 = load_global(fv + c * 3 + 1); f2 = load_global(fv + c * 3 + 2);
            }
            if (f_kind == kSrt3) {
                bad = !(isfinite(f0) && isfinite(f1) && isfinite(f2) && f0 > 0.f && f1 >= 1.f);
                if (!bad) {
                    if (LUT) lut_scales(J, 2.0f * f0 * f0, (double)f1, (double)f2, a, cl, ea);
                    else solve_srt(f0, f1, f2, J.eps_full, a, cl, ea);
                }
            } else if (LUT) {
                float s;
                double rho, th;
                bad = !srt_of_cov(f0, f1, f2, s, rho, th);
                if (!bad) lut_scales(J, s, rho, th, a, cl, ea);
            } else {
                bad = !solve_cov(f0, f1, f2, J.eps_full, a, cl, ea);
            }
            if (bad) {   // smallest isotropic filter instead
                const double v = sqrt(J.eps_full);
                a[0] = a[1] = a[2] = a[3] = v;
            }
            float4 o;
            o.x = (float)a[0]; o.y = (float)a[1]; o.z = (float)a[2]; o.w = (float)a[3];
            store_global(reinterpret_cast<f32x4 *>(const_cast<float *>(J.scales) + r * J.sc_rs + c * 4), f32x4{o.x, o.y, o.z, o.w});
            // the windows are sized from the stored (rounded) scales
            a[0] = o.x; a[1] = o.y; a[2] = o.z; a[3] = o.w;
        }
        if (!bad) {
            const double d = (a[1] + a[3]) * kRsqrt2;
            const float px = (float)(0.5 * (a[0] + d)) * 1.000001f, py = (float)(0.5 * (a[2] + d)) * 1.000001f;
            rx = fmaxf(rx, px);
            ry = fmaxf(ry, py);
            novf += fmaxf(px, py) * J.inv_sqrt_m > (float)J.cap;
        }
        ncl += cl;
        nea += ea;
        nbad += bad;
    };
    if constexpr (kPre) {
#pragma unroll
        for (int k = 0; k < kSmapRows; ++k) pixel(k);
    } else {
        for (int k = 0; k < kSmapRows; ++k) pixel(k);
    }
    // block reduction, then one set of atomics per block on the tile's record
    rx = wave_max(rx);
    ry = wave_max(ry);
    for (int o = 32; o > 0; o >>= 1) {
        ncl += __shfl_xor(ncl, o);
        nea += __shfl_xor(nea, o);
        nbad += __shfl_xor(nbad, o);
        novf += __shfl_xor(novf, o);
    }
    if (lane == 0) {
        s_rx[wave] = rx; s_ry[wave] = ry;
        s_cnt[wave][0] = ncl; s_cnt[wave][1] = nea; s_cnt[wave][2] = nbad; s_cnt[wave][3] = novf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float mx = 0.f, my = 0.f;
        uint32_t n[4] = {0, 0, 0, 0};
        for (int w = 0; w < 4; ++w) {
            mx = fmaxf(mx, s_rx[w]);
            my = fmaxf(my, s_ry[w]);
            for (int q = 0; q < 4; ++q) n[q] += s_cnt[w][q];
        }
        const int tile = (int)((int64_t)by * rows_per_block / J.T) * J.ntc + (int)((int64_t)bx * kSmapCols / J.T);
        TileStat *ts = J.tstat + tile;
        if (mx > 0.f) atomicMax(reinterpret_cast<unsigned int *>(&ts->rx), __float_as_uint(mx));
        if (my > 0.f) atomicMax(reinterpret_cast<unsigned int *>(&ts->ry), __float_as_uint(my));
        if (n[0]) atomicAdd(&ts->clamped, n[0]);
        if (n[1]) atomicAdd(&ts->eps_active, n[1]);
        if (n[2]) atomicAdd(&ts->invalid, n[2]);
        if (n[3]) atomicAdd(&ts->overflow, n[3]);
        if (J.req_counts) {
            if (n[2]) atomicAdd(&J.req_counts[0], n[2]);
            if (n[3]) atomicAdd(&J.req_counts[1], n[3]);
        }
    }
    __syncthreads();   // the shared records are reused by the next block of a persistent loop
}

// The solve, one kernel per field kind.
template <int KIND>
__global__ __launch_bounds__(256) void k_scale_map(Job J)
{
    // blocks of 16 pixel rows; the launch starts at the first row of tile row tr0
    const int nbx = (int)((J.W + kSmapCols - 1) / kSmapCols);
    scale_map_block<false, KIND>(J, blockIdx.x + J.tr0 * (J.T / (4 * kSmapRows)) * nbx);
}

__global__ __launch_bounds__(256) void k_scale_map_lut(Job J)
{
    const int nbx = (int)((J.W + kSmapCols - 1) / kSmapCols);
    scale_map_block<true>(J, blockIdx.x + J.tr0 * (J.T / (4 * kSmapRows)) * nbx);
}

// Batched solve: KIND is the one field kind of all the jobs, or -1 for a mix (every
// kind's code in one kernel, with the registers of the largest).
template <int KIND>
__global__ __launch_bounds__(256) void k_scale_map_batch(const Job *jobs, int n, int total, const BatchDims *dims)
{
    if (dims) {
        n = dims->n;
        total = dims->total;
    }
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int j = __builtin_amdgcn_readfirstlane(find_job(jobs, n, b, 2));
        const Job J = uniform_copy(jobs + j);
        scale_map_block<false, KIND>(J, b - J.smap_base);
    }
}

__global__ __launch_bounds__(256) void k_scale_map_batch_lut(const Job *jobs, int n, int total, const BatchDims *dims)
{
    if (dims) {
        n = dims->n;
        total = dims->total;
    }
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int j = __builtin_amdgcn_readfirstlane(find_job(jobs, n, b, 2));
        const Job J = uniform_copy(jobs + j);
        scale_map_block<true>(J, b - J.smap_base);
    }
}

// tile records and request counters of the jobs of a table
__global__ void k_fill_jobs(const Job *jobs, int n, const BatchDims *dims)
{
    if (dims) n = dims->n;
    for (int j = blockIdx.x; j < n; j += gridDim.x) {
        const Job J = uniform_copy(jobs + j);
        uint32_t *t = reinterpret_cast<uint32_t *>(J.tstat);
        const int64_t words = (int64_t)J.ntr * J.ntc * (int64_t)(sizeof(TileStat) / 4);
        for (int64_t i = threadIdx.x; i < words; i += blockDim.x) t[i] = 0u;
        if (J.req_counts && threadIdx.x < 2) J.req_counts[threadIdx.x] = 0u;
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
// Wave prefix sums use DPP (row shifts 1, 2, 4, 8 then the row broadcasts 15, 31).
// ---------------------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));   // 16 bytes of a buffer store

template <int CTRL, int RM>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, RM, 0xf, true);
}

template <int CTRL, int RM>
__device__ __forceinline__ uint64_t dpp64(uint64_t v)
{
    const uint32_t lo = dpp32<CTRL, RM>((uint32_t)v), hi = dpp32<CTRL, RM>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

struct ArF64 {
    using T = double;
    __device__ static T zero() { return 0.0; }
    __device__ static T from(double v) { return v; }
    __device__ static T add(T a, T b) { return a + b; }
    __device__ static T s2add(T a, T b) { return fma(kSqrt2, a, b); }   // sqrt2 a + b
    template <int CTRL, int RM>
    __device__ static T dpp(T v) { return __longlong_as_double((long long)dpp64<CTRL, RM>((uint64_t)__double_as_longlong(v))); }
    __device__ static void store(void *g, int64_t i, T v) { static_cast<double *>(g)[i] = v; }
    __device__ static T mul01(T v, T k) { return v * k; }   // k is 0 or 1
    __device__ static u32x4 pack2(T a, T b)
    {
        const uint64_t x = (uint64_t)__double_as_longlong(a), y = (uint64_t)__double_as_longlong(b);
        return u32x4{(uint32_t)x, (uint32_t)(x >> 32), (uint32_t)y, (uint32_t)(y >> 32)};
    }
};

struct ArI64 {
    using T = unsigned long long;
    __device__ static T zero() { return 0ull; }
    __device__ static T from(double v) { return (T)(long long)v; }
    __device__ static T add(T a, T b) { return a + b; }
    __device__ static T s2add(T a, T b) { return a + b; }
    template <int CTRL, int RM>
    __device__ static T dpp(T v) { return dpp64<CTRL, RM>(v); }
    __device__ static void store(void *g, int64_t i, T v) { static_cast<unsigned long long *>(g)[i] = v; }
    __device__ static T mul01(T v, T k) { return v & (0ull - k); }   // k is 0 or 1
    __device__ static u32x4 pack2(T a, T b) { return u32x4{(uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32)}; }
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
    template <int CTRL, int RM>
    __device__ static T dpp(T v)
    {
        return {__uint_as_float(dpp32<CTRL, RM>(__float_as_uint(v.hi))), __uint_as_float(dpp32<CTRL, RM>(__float_as_uint(v.lo)))};
    }
    __device__ static void store(void *g, int64_t i, T v) { static_cast<float2 *>(g)[i] = make_float2(v.hi, v.lo); }
    __device__ static T mul01(T v, T k) { return {v.hi * k.hi, v.lo * k.hi}; }   // k is 0 or 1
    __device__ static u32x4 pack2(T a, T b)
    {
        return u32x4{__float_as_uint(a.hi), __float_as_uint(a.lo), __float_as_uint(b.hi), __float_as_uint(b.lo)};
    }
};

// inclusive prefix over the 64 lanes of a wave
template <class A>
__device__ __forceinline__ typename A::T wave_scan(typename A::T v)
{
    v = A::add(v, A::template dpp<0x111, 0xf>(v));   // row_shr:1
    v = A::add(v, A::template dpp<0x112, 0xf>(v));   // row_shr:2
    v = A::add(v, A::template dpp<0x114, 0xf>(v));   // row_shr:4
    v = A::add(v, A::template dpp<0x118, 0xf>(v));   // row_shr:8
    v = A::add(v, A::template dpp<0x142, 0xa>(v));   // row_bcast:15 into rows 1, 3
    v = A::add(v, A::template dpp<0x143, 0xc>(v));   // row_bcast:31 into rows 2, 3
    return v;
}

template <class A, int KC>
struct alignas(16) ScanLds {
    // double-buffered by row parity
    typename A::T p45[2][KC * kScanCols + 2];   // previous row g45 at index c + 1 (index 0 stays zero)
    typename A::T pb[2][KC * kScanCols + 2];    // previous row g_b at index c (index >= w stays zero)
    typename A::T wsum[2][KC][kScanThreads / 64];
    float row[2][KC * kScanCols];               // input rows published by the loader wave
};

constexpr int kLoadDepth = 4;   // input rows the loader wave has in flight

// The loader wave (threads kScanThreads .. kScanThreads + 63): loads the window's
// input rows kLoadDepth ahead into registers (coalesced; addresses mapped into
// the image by the boundary rule) and publishes row r + 1 into the LDS ring during
// row r, zero outside the window (and outside the image under the zero rule).  Its memory queue holds loads only, so its waits are exact, and the
// compute waves never wait on memory.  Barriers match the compute waves' one per row.
template <int IN, int KC>
__device__ __forceinline__ void load_rows(const Job &J, int ch, const Window w, float (*ring)[KC * kScanCols])
{
    using E = typename std::conditional<IN == kInF32, float, unsigned short>::type;
    constexpr int NV = KC * kScanCols / 64;   // values per lane and row
    const int lane = threadIdx.x & 63;
    const E *in = static_cast<const E *>(J.in);
    E regs[kLoadDepth][NV];
    const int bnd = J.boundary;
    // per lane, once per window: element offset of each of its columns in a row,
    // and which of them hold data (inside the window; inside the image, zero rule)
    int32_t coff[NV];
    uint32_t cmask = 0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const int c = lane + 64 * j;
        const int64_t C = w.c0 + c;
        coff[j] = (int32_t)(ext_index(C, J.W, bnd) * J.C + ch);
        if (c < w.w && (bnd != kBoundZero || (C >= 0 && C < J.W))) cmask |= 1u << j;
    }
    auto issue = [&](int rr, E *dst) {
        const int64_t R = ext_index(w.r0 + rr, J.H, bnd);
        const E *rowp = in + R * J.in_rs;
#pragma unroll
        for (int j = 0; j < NV; ++j) dst[j] = rowp[coff[j]];
    };
    auto put = [&](int rr, const E *src) {
        const int64_t R = w.r0 + rr;
        const bool rin = bnd != kBoundZero || (R >= 0 && R < J.H);
#pragma unroll
        for (int j = 0; j < NV; ++j) ring[rr & 1][lane + 64 * j] = (rin && ((cmask >> j) & 1u)) ? (float)src[j] : 0.f;
    };
#pragma unroll
    for (int d = 0; d < kLoadDepth; ++d) issue(d, regs[d]);
    put(0, regs[0]);
    lds_barrier();
    for (int rr0 = 0; rr0 < w.h; rr0 += kLoadDepth) {
#pragma unroll
        for (int d = 0; d < kLoadDepth; ++d) {
            const int rr = rr0 + d;
            if (rr >= w.h) break;   // uniform
            issue(rr + kLoadDepth, regs[d]);           // row rr is in LDS already: reuse its registers
            put(rr + 1, regs[(d + 1) % kLoadDepth]);   // row rr + 1, for the compute waves' next row
            lds_barrier();
        }
    }
}

// One window: rows [w.r0, w.r0 + w.h) x cols [w.c0, w.c0 + w.w), channel ch of the
// job's pass input, extended beyond the image by the job's boundary rule; result (g_b, or G for integers) into
// gout[row * w.w + col].  Compute thread t owns the adjacent columns c0 = k * 512 + 2t
// and c1 = c0 + 1 of chunk k.  Per row: RS1 is the pair sum scanned over the wave
// (DPP), the wave totals exchanged through LDS, and the pair split again with the
// exclusive prefix (DPP wave shift); RS2..RS4 take one neighbour each from the
// previous row: the column inside the pair from registers, the one across the pair
// boundary from a double-buffered LDS row.  Input rows come from the loader wave
// through LDS; one LDS barrier per row orders every exchange.
template <class A, int IN, int KC>
__device__ __forceinline__ void sweep_window(const Job &J, int ch, const Window w, void *gout, ScanLds<A, KC> &L)
{
    using T = typename A::T;
    const int t = threadIdx.x;
    if (t >= kScanThreads) {
        load_rows<IN, KC>(J, ch, w, L.row);
        return;
    }
    const int lane = t & 63, wave = t >> 6;
    const int K = (w.w + kScanCols - 1) / kScanCols;   // <= KC
    for (int i = t; i < KC * kScanCols + 2; i += kScanThreads) {
        L.p45[0][i] = A::zero(); L.pb[0][i] = A::zero();
        L.p45[1][i] = A::zero(); L.pb[1][i] = A::zero();
    }
    T p90[KC][2], prev45[KC], prevb[KC];   // g90 of both columns; last row's g45 at c0 and g_b at c1
#pragma unroll
    for (int k = 0; k < KC; ++k) p90[k][0] = p90[k][1] = prev45[k] = prevb[k] = A::zero();
    lds_barrier();
    for (int rr = 0; rr < w.h; ++rr) {
        const int pp = rr & 1;   // LDS buffers written by this row
        T v[KC][2], incl[KC];
        // RS1: prefix of the pair sums over the wave, wave totals through LDS
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            if (k < K) {
                const float2 f = *reinterpret_cast<const float2 *>(&L.row[pp][k * kScanCols + 2 * t]);
                v[k][0] = A::from((double)f.x);
                v[k][1] = A::from((double)f.y);
                incl[k] = wave_scan<A>(A::add(v[k][0], v[k][1]));
                if (lane == 63) L.wsum[pp][k][wave] = incl[k];
            }
        }
        lds_barrier();
        T carry = A::zero();
#pragma unroll
        for (int k = 0; k < KC; ++k) {
            if (k < K) {
                T off = carry;
#pragma unroll
                for (int q = 0; q < kScanThreads / 64; ++q) {
                    const T ws = L.wsum[pp][k][q];
                    if (q < wave) off = A::add(off, ws);
                    carry = A::add(carry, ws);
                }
                const int c0 = k * kScanCols + 2 * t;
                // prefix before c0 = lane - 1's inclusive pair prefix (zero in lane 0) + off
                const T excl = A::template dpp<0x138, 0xf>(incl[k]);   // wave_shr:1
                const T g00 = A::add(A::add(off, excl), v[k][0]);
                const T g01 = A::add(g00, v[k][1]);
                const T g450 = A::s2add(g00, L.p45[pp ^ 1][c0]);       // RS2: sqrt2 g0 + g45[r-1][c-1]
                const T g451 = A::s2add(g01, prev45[k]);
                p90[k][0] = A::add(g450, p90[k][0]);                   // RS3: g45 + g90[r-1][c]
                p90[k][1] = A::add(g451, p90[k][1]);
                const T gb0 = A::s2add(p90[k][0], prevb[k]);           // RS4: sqrt2 g90 + gb[r-1][c+1]
                const T gb1 = A::s2add(p90[k][1], L.pb[pp ^ 1][c0 + 2]);
                prev45[k] = g450;
                prevb[k] = (c0 + 1 < w.w) ? gb1 : A::zero();           // zero beyond the window
                L.p45[pp][c0 + 2] = g451;
                if (c0 < w.w) {
                    L.pb[pp][c0] = gb0;
                    A::store(gout, (int64_t)rr * w.w + c0, gb0);
                    if (c0 + 1 < w.w) A::store(gout, (int64_t)rr * w.w + c0 + 1, gb1);
                }
            }
        }
    }
}


// Row sweep split over the waves of one work-group per window.  Lane l of the
// compute waves owns the P adjacent columns l P .. l P + P - 1 (P 64 >= the
// window width, P even); rows go in blocks of D, through a pipeline with one
// barrier per block:
//   loader wave      : input rows of block k into LDS (its memory queue holds
//                      loads only, pre_ahead blocks ahead, so it waits exactly
//                      for the oldest);
//   kPreProd waves   : RS1 of block k - 1 (the lane's serial prefix, then the
//                      wave prefix of the lane totals by DPP, added to it; rows
//                      are independent, each wave takes every kPreProd-th) into
//                      an LDS block buffer (one wave measured faster than two
//                      or four: four waves put one on each SIMD);
//   sum wave         : RS2..RS4 of block k - 2 in place, row after row: RS2 and
//                      RS4 take the previous row's value one column to the left
//                      / right from the lane's registers or, at its first / last
//                      column, from the neighbouring lane (wave shift by one
//                      lane, DPP); RS3 stays in registers;
//   storer wave      : block k - 3 to the window.
// Each wave alone would be bound by the latency of its instruction chains or of
// memory; split this way the window's work runs on several SIMDs at once.
//
// LDS holds the compute waves' layout, [row][column in lane][lane]; the loader
// and the storer move whole contiguous row segments (lane l takes the two
// columns 2 l + 128 m, 2 l + 128 m + 1: 8-byte loads, 16-byte stores, every
// access of a wave one contiguous run) and scatter / gather them there.  Input
// pairs need a window inside the image, one f32 channel, an even row stride
// (window origins are even); elsewhere the loader reads single columns through
// the boundary rule.  The last block runs past the window's last row: its
// loads read valid rows (mapped into the image) and its stores fall outside the
// window's buffer range, which the hardware drops, as it drops the stores of
// columns beyond the window's width (widths are even: pairs never straddle it).
constexpr int kPreProd = 1;                          // RS1 waves per window
constexpr int kPreWaves = kPreProd + 3;              // + sum wave, storer, loader
constexpr int kPreBuf = 8 * 8 * 64;                  // T elements of a block buffer: D x P x 64 (max over P)

template <int P>
constexpr int pre_rows() { return P <= 8 ? 8 : 4; }   // D: rows per block
template <int P>
constexpr int pre_ahead() { return P <= 4 ? 2 : 1; }  // blocks of input rows the loader has in flight
// LDS: three block buffers of sums (T), then two of input (float).
template <class A>
__device__ __forceinline__ float *pre_inbuf(typename A::T *lds) { return reinterpret_cast<float *>(lds + 3 * kPreBuf); }

template <class A, int IN, int P, bool PAIRS>
__device__ __forceinline__ void preint_loader(const Job &J, int ch, const Window w, typename A::T *lds)
{
    static_assert(P % 2 == 0, "column pairs");
    static_assert(!PAIRS || IN == kInF32, "pair loads read f32 input");
    using E = typename std::conditional<IN == kInF32, float, unsigned short>::type;
    constexpr int D = pre_rows<P>(), kPreAhead = pre_ahead<P>();
    const int lane = threadIdx.x & 63;
    const int bnd = J.boundary;
    const E *in = static_cast<const E *>(J.in);
    // value v of a row: column 2 lane + 128 (v / 2) + v % 2 (pairs) or lane + 64 v
    int32_t coff[P];
    int16_t pos[P];       // its LDS position: (column % P) * 64 + column / P
    uint32_t vmask = 0;   // inside the window (and, zero rule, inside the image)
#pragma unroll
    for (int v = 0; v < P; ++v) {
        const int c = PAIRS ? 2 * lane + 128 * (v / 2) + (v & 1) : lane + 64 * v;
        const int64_t C = w.c0 + c;
        coff[v] = (int32_t)(ext_index(C, J.W, bnd) * J.C + ch);
        pos[v] = (int16_t)((c % P) * 64 + c / P);
        if (c < w.w && (bnd != kBoundZero || (C >= 0 && C < J.W))) vmask |= 1u << v;
    }
    E ring[kPreAhead][D][P];   // input rows of the next kPreAhead blocks
    auto issue = [&](int rr, E *dst) {   // rows past the window map to valid rows (values unused)
        const E *rowp = in + ext_index(w.r0 + rr, J.H, bnd) * J.in_rs;
        if (PAIRS) {   // (buffer loads: plain vector loads get split back into dwords)
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<E *>(rowp + w.c0), 0, 64 * P * (int)sizeof(E), kBufWord3);
#pragma unroll
            for (int m = 0; m < P / 2; ++m) {
                const float2 x = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, (2 * lane + 128 * m) * 4, 0, 0));
                dst[2 * m] = x.x;
                dst[2 * m + 1] = x.y;
            }
        } else {
#pragma unroll
            for (int v = 0; v < P; ++v) dst[v] = load_global(rowp + coff[v]);
        }
    };
#pragma unroll
    for (int u = 0; u < kPreAhead; ++u)
#pragma unroll
        for (int d = 0; d < D; ++d) issue(u * D + d, ring[u][d]);
    float *inb = pre_inbuf<A>(lds);
    const int nblk = (w.h + D - 1) / D;
    for (int k0 = 0; k0 < nblk + 3; k0 += kPreAhead) {
#pragma unroll
        for (int u = 0; u < kPreAhead; ++u) {   // block k comes from ring[k % kPreAhead]
            const int k = k0 + u;
            if (k >= nblk + 3) break;   // uniform
            if (k < nblk) {
                float *buf = inb + (k & 1) * kPreBuf;   // input buffers: kPreBuf floats each
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int64_t R = w.r0 + k * D + d;
                    const bool rin = bnd != kBoundZero || (R >= 0 && R < J.H);
#pragma unroll
                    for (int v = 0; v < P; ++v)
                        buf[d * P * 64 + pos[v]] = (rin && ((vmask >> v) & 1u)) ? (float)ring[u][d][v] : 0.f;
                    issue((k + kPreAhead) * D + d, ring[u][d]);
                }
            }
            lds_barrier();
        }
    }
}

template <class A, int P>
__device__ __forceinline__ void preint_producer(const Window w, typename A::T *lds, int wave)
{
    using T = typename A::T;
    constexpr int D = pre_rows<P>(), DP = D / kPreProd;   // rows of a block, of them this wave's
    static_assert(DP * kPreProd == D && D * P * 64 <= kPreBuf, "block rows and LDS buffers");
    const int lane = threadIdx.x & 63;
    const float *inb = pre_inbuf<A>(lds);
    const int nblk = (w.h + D - 1) / D;
    for (int k = 0; k < nblk + 3; ++k) {
        if (k >= 1 && k <= nblk) {   // block k - 1
            const float *src = inb + ((k - 1) & 1) * kPreBuf;
            T *dst = lds + ((k - 1) % 3) * kPreBuf;
#pragma unroll
            for (int i = 0; i < DP; ++i) {
                const int d = wave + kPreProd * i;
                T s[P];
#pragma unroll
                for (int j = 0; j < P; ++j) s[j] = A::from((double)src[(d * P + j) * 64 + lane]);
#pragma unroll
                for (int j = 1; j < P; ++j) s[j] = A::add(s[j - 1], s[j]);
                const T excl = A::template dpp<0x138, 0xf>(wave_scan<A>(s[P - 1]));   // wave_shr:1, zero in lane 0
#pragma unroll
                for (int j = 0; j < P; ++j) dst[(d * P + j) * 64 + lane] = A::add(excl, s[j]);
            }
        }
        lds_barrier();
    }
}

template <class A, int P>
__device__ __forceinline__ void preint_sums(const Window w, typename A::T *lds)
{
    using T = typename A::T;
    constexpr int D = pre_rows<P>();
    const int lane = threadIdx.x & 63, cb = lane * P;
    T keep[P];   // 1 inside the window's width, 0 beyond (RS4 must see zeros there)
#pragma unroll
    for (int j = 0; j < P; ++j) keep[j] = A::from(cb + j < w.w ? 1.0 : 0.0);
    T p90[P], g45p[P], gbp[P];   // RS3, and the previous row's RS2 / RS4, of the lane's columns
#pragma unroll
    for (int j = 0; j < P; ++j) p90[j] = g45p[j] = gbp[j] = A::zero();
    const int nblk = (w.h + D - 1) / D;
    for (int k = 0; k < nblk + 3; ++k) {
        if (k >= 2 && k <= nblk + 1) {   // block k - 2, RS1 replaced by RS4
            T *buf = lds + ((k - 2) % 3) * kPreBuf;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const T left = A::template dpp<0x138, 0xf>(g45p[P - 1]);   // g45[r-1][cb-1], zero in lane 0
                const T right = A::template dpp<0x130, 0xf>(gbp[0]);       // gb[r-1][cb+P] (wave_shl:1), zero in lane 63
#pragma unroll
                for (int j = P - 1; j >= 0; --j) {   // descending: g45p[j - 1] still holds row r - 1
                    const T g45 = A::s2add(buf[(d * P + j) * 64 + lane], j ? g45p[j - 1] : left);   // RS2
                    p90[j] = A::add(g45, p90[j]);                                                  // RS3
                    g45p[j] = g45;
                }
                T gb[P];
#pragma unroll
                for (int j = 0; j < P; ++j) gb[j] = A::mul01(A::s2add(p90[j], j + 1 < P ? gbp[j + 1] : right), keep[j]);   // RS4
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    gbp[j] = gb[j];
                    buf[(d * P + j) * 64 + lane] = gb[j];
                }
            }
        }
        lds_barrier();
    }
}

template <class A, int P>
__device__ __forceinline__ void preint_storer(const Window w, void *gout, const typename A::T *lds)
{
    using T = typename A::T;
    constexpr int D = pre_rows<P>();
    const int lane = threadIdx.x & 63;
    // pair m of a row: columns c, c + 1 with c = 2 lane + 128 m (same owner lane c / P)
    uint32_t soff[P / 2];   // byte offset in a window row; out of range past the width
    int16_t pos[P / 2];     // LDS position of column c: (c % P) * 64 + c / P
#pragma unroll
    for (int m = 0; m < P / 2; ++m) {
        const int c = 2 * lane + 128 * m;
        soff[m] = c < w.w ? (uint32_t)(c * sizeof(T)) : 0x7ffffff0u;
        pos[m] = (int16_t)((c % P) * 64 + c / P);
    }
    const __amdgpu_buffer_rsrc_t out = __builtin_amdgcn_make_buffer_rsrc(
        gout, 0, (int)((int64_t)w.h * w.w * sizeof(T)), kBufWord3);
    const int nblk = (w.h + D - 1) / D;
    for (int k = 0; k < nblk + 3; ++k) {
        if (k >= 3) {   // block k - 3
            const T *buf = lds + ((k - 3) % 3) * kPreBuf;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const uint32_t roff = (uint32_t)(((k - 3) * D + d) * w.w * (int)sizeof(T));
#pragma unroll
                for (int m = 0; m < P / 2; ++m) {
                    const T *q = buf + d * P * 64 + pos[m];
                    __builtin_amdgcn_raw_buffer_store_b128(A::pack2(q[0], q[64]), out, roff + soff[m], 0, 0);
                }
            }
        }
        lds_barrier();
    }
}

template <class A, int IN, int P>
__device__ __forceinline__ void sweep_window_split(const Job &J, int ch, const Window w, void *gout, typename A::T *lds)
{
    const int wave = threadIdx.x >> 6;   // uniform: 0 .. kPreProd - 1 RS1, then sums, storer, loader
    if (wave < kPreProd) return preint_producer<A, P>(w, lds, wave);
    if (wave == kPreProd) return preint_sums<A, P>(w, lds);
    if (wave == kPreProd + 1) return preint_storer<A, P>(w, gout, lds);
    // pair loads where all 64 P columns lie inside the image
    const bool pairs = IN == kInF32 && J.C == 1 && w.c0 >= 0 && (w.c0 & 1) == 0 && w.c0 + 64 * P <= J.W &&
                       (J.in_rs & 1) == 0 && (reinterpret_cast<uintptr_t>(J.in) & 7) == 0;
    if (IN == kInF32 && pairs) preint_loader<A, IN, P, IN == kInF32>(J, ch, w, lds);
    else preint_loader<A, IN, P, false>(J, ch, w, lds);
}

// the columns per lane follow the window's width
template <class A, int IN>
__device__ __forceinline__ void preint_window(const Job &J, int ch, const Window w, void *gout, typename A::T *lds)
{
    const int p = (w.w + 63) / 64;   // uniform; <= kMaxWindow / 64 = 16
    if (p <= 2) sweep_window_split<A, IN, 2>(J, ch, w, gout, lds);
    else if (p <= 4) sweep_window_split<A, IN, 4>(J, ch, w, gout, lds);
    else if (p <= 6) sweep_window_split<A, IN, 6>(J, ch, w, gout, lds);
    else if (p <= 8) sweep_window_split<A, IN, 8>(J, ch, w, gout, lds);
    else if (p <= 12) sweep_window_split<A, IN, 12>(J, ch, w, gout, lds);
    else sweep_window_split<A, IN, 16>(J, ch, w, gout, lds);
}

// one work-group of kPreWaves waves per (tile, channel) window
template <class A, int IN>
__global__ __launch_bounds__(64 * kPreWaves) void k_preint(Job J)
{
    __shared__ typename A::T lds[4 * kPreBuf];   // 3 sum buffers, then 2 input buffers (floats)
    const int lt = blockIdx.x / J.C, ch = blockIdx.x - lt * J.C;
    const int tile = J.tr0 * J.ntc + lt;
    const Window w = window_of(J, tile);
    void *gout = static_cast<unsigned char *>(J.g) + ((int64_t)tile * J.C + ch) * J.slot_elems * sizeof(typename A::T);
    preint_window<A, IN>(J, ch, w, gout, lds);
}

// the batched launches: windows of every image of the table, one work-group
// each in turn (grid-stride)
template <class A>
__global__ __launch_bounds__(64 * kPreWaves) void k_preint_batch(const Job *jobs, int n, int total, const BatchDims *dims)
{
    __shared__ typename A::T lds[4 * kPreBuf];
    if (dims) {
        n = dims->n;
        total = dims->total;
    }
    for (int b = blockIdx.x; b < total; b += gridDim.x) {
        const int j = __builtin_amdgcn_readfirstlane(find_job(jobs, n, b, 0));
        const Job J = uniform_copy(jobs + j);
        const int lt = b - J.tile_base;
        const int tile = lt / J.C, ch = lt - tile * J.C;
        const Window wl = window_of(J, tile);
        const Window w = uniform_copy(&wl);   // the tile record is read with vector loads
        void *gout = static_cast<unsigned char *>(J.g) + ((int64_t)tile * J.C + ch) * J.slot_elems * sizeof(typename A::T);
        if (J.in_type == kInU16) preint_window<A, kInU16>(J, ch, w, gout, lds);
        else preint_window<A, kInF32>(J, ch, w, gout, lds);
        lds_barrier();   // the buffers are reused by the next window
    }
}

// a caller's window on the pipelined sweep (even width, 16-byte aligned output)
template <class A, int IN>
__global__ __launch_bounds__(64 * kPreWaves) void k_preint_window_split(Job J, int ch, Window w, void *g)
{
    __shared__ typename A::T lds[4 * kPreBuf];
    preint_window<A, IN>(J, ch, w, g, lds);
}

template <class A, int IN>
__global__ __launch_bounds__(kScanThreads + 64) void k_preint_window(Job J, int ch, Window w, void *g)
{
    __shared__ ScanLds<A, kScanChunks> L;
    sweep_window<A, IN, kScanChunks>(J, ch, w, g, L);
}

template <class A>
hipError_t launch_preint_t(const Job &j, hipStream_t s)
{
    const int nb = (j.tr1 - j.tr0) * j.ntc * j.C;
    if (nb <= 0) return hipSuccess;
    if (j.in_type == kInF32) hipLaunchKernelGGL((k_preint<A, kInF32>), dim3(nb), dim3(64 * kPreWaves), 0, s, j);
    else hipLaunchKernelGGL((k_preint<A, kInU16>), dim3(nb), dim3(64 * kPreWaves), 0, s, j);
    return hipGetLastError();
}

}  // namespace

int64_t slot_elems_for(int T, int cap)
{
    const int64_t side = (int64_t)T + 2 * (int64_t)cap + 6;   // window sides are even (T is)
    return side * side;
}


int scale_map_blocks(int64_t H, int64_t W)
{
    return (int)(((W + kSmapCols - 1) / kSmapCols) * ((H + 4 * kSmapRows - 1) / (4 * kSmapRows)));
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
    const int64_t r0 = (int64_t)j.tr0 * j.T, r1 = std::min((int64_t)j.tr1 * j.T, j.H);
    if (r1 <= r0) return hipSuccess;
    const int nb = scale_map_blocks(r1 - r0, j.W);
    if (j.lut) hipLaunchKernelGGL(k_scale_map_lut, dim3(nb), dim3(256), 0, s, j);
    else if (j.f_kind == kSrt3) hipLaunchKernelGGL(k_scale_map<kSrt3>, dim3(nb), dim3(256), 0, s, j);
    else if (j.f_kind == kCov3) hipLaunchKernelGGL(k_scale_map<kCov3>, dim3(nb), dim3(256), 0, s, j);
    else hipLaunchKernelGGL(k_scale_map<kScales4>, dim3(nb), dim3(256), 0, s, j);
    return hipGetLastError();
}

hipError_t launch_lut_build(float *lut, int n, double eps, hipStream_t s)
{
    const int nn = n * n;
    hipLaunchKernelGGL(k_lut_build, dim3((nn + 255) / 256), dim3(256), 0, s, reinterpret_cast<float4 *>(lut), n, eps);
    return hipGetLastError();
}

hipError_t launch_preint(const Job &j, hipStream_t s)
{
    switch (j.preint) {
    case kPreF64: return launch_preint_t<ArF64>(j, s);
    case kPreF32C: return launch_preint_t<ArF32C>(j, s);
    case kPreI64:
        if (j.in_type != kInU16) return hipErrorInvalidValue;
        return launch_preint_t<ArI64>(j, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_preint_window(const Job &j, int channel, int64_t r0, int64_t c0, int h, int w, void *g,
                                hipStream_t s)
{
    Window win;
    win.r0 = r0; win.c0 = c0; win.h = h; win.w = w;
    // the pipelined sweep needs an even width (its stores move column pairs), a
    // 16-byte aligned output and byte offsets in 32 bits; other windows take the
    // one-work-group sweep with a loader wave
    if ((w & 1) == 0 && (reinterpret_cast<uintptr_t>(g) & 15) == 0 && (int64_t)h * w * 8 < ((int64_t)1 << 31) - 65536) {
#define SVF_PW(A, IN) hipLaunchKernelGGL((k_preint_window_split<A, IN>), dim3(1), dim3(64 * kPreWaves), 0, s, j, channel, win, g)
        switch (j.preint) {
        case kPreF64:
            if (j.in_type == kInF32) SVF_PW(ArF64, kInF32);
            else SVF_PW(ArF64, kInU16);
            break;
        case kPreF32C:
            if (j.in_type == kInF32) SVF_PW(ArF32C, kInF32);
            else SVF_PW(ArF32C, kInU16);
            break;
        case kPreI64:
            if (j.in_type != kInU16) return hipErrorInvalidValue;
            SVF_PW(ArI64, kInU16);
            break;
        default: return hipErrorInvalidValue;
        }
#undef SVF_PW
        return hipGetLastError();
    }
    switch (j.preint) {
    case kPreF64:
        if (j.in_type == kInF32) hipLaunchKernelGGL((k_preint_window<ArF64, kInF32>), dim3(1), dim3(kScanThreads + 64), 0, s, j, channel, win, g);
        else hipLaunchKernelGGL((k_preint_window<ArF64, kInU16>), dim3(1), dim3(kScanThreads + 64), 0, s, j, channel, win, g);
        break;
    case kPreF32C:
        if (j.in_type == kInF32) hipLaunchKernelGGL((k_preint_window<ArF32C, kInF32>), dim3(1), dim3(kScanThreads + 64), 0, s, j, channel, win, g);
        else hipLaunchKernelGGL((k_preint_window<ArF32C, kInU16>), dim3(1), dim3(kScanThreads + 64), 0, s, j, channel, win, g);
        break;
    case kPreI64:
        if (j.in_type != kInU16) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_preint_window<ArI64, kInU16>), dim3(1), dim3(kScanThreads + 64), 0, s, j, channel, win, g);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_scale_map_batch(const Job *jobs, int n, int total_blocks, int grid, bool lut, int kind,
                                  hipStream_t s, const BatchDims *dims)
{
    if (!dims) {
        if (total_blocks == 0) return hipSuccess;
        grid = std::min(grid, total_blocks);
    }
    grid = std::max(1, grid);
    if (lut) hipLaunchKernelGGL(k_scale_map_batch_lut, dim3(grid), dim3(256), 0, s, jobs, n, total_blocks, dims);
    else if (kind == kSrt3) hipLaunchKernelGGL(k_scale_map_batch<kSrt3>, dim3(grid), dim3(256), 0, s, jobs, n, total_blocks, dims);
    else if (kind == kCov3) hipLaunchKernelGGL(k_scale_map_batch<kCov3>, dim3(grid), dim3(256), 0, s, jobs, n, total_blocks, dims);
    else if (kind == kScales4)
        hipLaunchKernelGGL(k_scale_map_batch<kScales4>, dim3(grid), dim3(256), 0, s, jobs, n, total_blocks, dims);
    else hipLaunchKernelGGL(k_scale_map_batch<-1>, dim3(grid), dim3(256), 0, s, jobs, n, total_blocks, dims);
    return hipGetLastError();
}

hipError_t launch_preint_batch(const Job *jobs, int n, int total_tiles, int grid, int preint, hipStream_t s,
                               const BatchDims *dims)
{
    if (!dims) {
        if (total_tiles == 0) return hipSuccess;
        grid = std::min(grid, total_tiles);
    }
    grid = std::max(1, grid);
    switch (preint) {
    case kPreF64: hipLaunchKernelGGL((k_preint_batch<ArF64>), dim3(grid), dim3(64 * kPreWaves), 0, s, jobs, n, total_tiles, dims); break;
    case kPreF32C: hipLaunchKernelGGL((k_preint_batch<ArF32C>), dim3(grid), dim3(64 * kPreWaves), 0, s, jobs, n, total_tiles, dims); break;
    case kPreI64: hipLaunchKernelGGL((k_preint_batch<ArI64>), dim3(grid), dim3(64 * kPreWaves), 0, s, jobs, n, total_tiles, dims); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fill_jobs(const Job *jobs, int n, int grid, hipStream_t s, const BatchDims *dims)
{
    if (!dims) {
        if (n == 0) return hipSuccess;
        grid = std::min(grid, n);
    }
    hipLaunchKernelGGL(k_fill_jobs, dim3(std::max(1, grid)), dim3(256), 0, s, jobs, n, dims);
    return hipGetLastError();
}

}  // namespace svf

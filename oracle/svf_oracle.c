/*
 * svf_oracle.c -- CPU FP64 oracle for the space-variant elliptical box-spline
 * filter of Chaudhury, Munoz-Barrutia and Unser, "Fast space-variant elliptical
 * filtering using box splines".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this file: only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant generator
 * with the GPU library; it is written to be read against the paper, not to be
 * fast.  All arithmetic is IEEE binary64 (integer scans: wrapping 64-bit).
 *
 * Contents (paper section / equation each part follows):
 *   1. Radially-uniform box spline beta^4_a(x) for N = 4 (Sec. 2.2.1, eq. (const)):
 *      the density of sum_k T_k a_k u_k, T_k ~ U(-1/2, 1/2), evaluated exactly
 *      as the overlap area of two rectangles divided by a1 a2 a3 a4.
 *      The ZP element is the case a = b = (1, sqrt2, 1, sqrt2) (Sec. 3.1).
 *   2. Scale-vector solve (Sec. 3.2.2): covariance -> p_bar (pivot p4 = 1),
 *      [t_l, t_r], the cubic zeta'(t) with the printed coefficients, its real
 *      roots (Cardano / Viete), argmin of the quartic zeta over roots and ends.
 *      Before the solve, an infeasible elongation is lowered to the largest
 *      feasible value at fixed size and orientation (a reading: the paper
 *      states the bound, Prop. 3.1, but not what to do beyond it).
 *   3. Pre-integration by the four running sums RS1..RS4 (Sec. 3.1 step (1),
 *      Algorithm 1 step 2) over a rectangular window with zero initial
 *      conditions; FP64, and an integer variant without the sqrt2 factors.
 *   4. Local finite difference with ZP interpolation (eq. (final_eqn),
 *      Table 1 taps, shift tau of Sec. 3.1 step (2)); the interpolant
 *      F(y) = sum_m g[m] ZP(y - m) is evaluated term by term with part 1.
 *   5. One filter pass over a rectangle of outputs: the fast algorithm
 *      (parts 3 + 4 on windows that contain every sample a pixel reads) and the
 *      brute-force direct sum  out[n] = sum_k f[k] beta^4_{a(n)}(n - k)
 *      (eq. (discrete) with the Dirac-comb input model of Sec. 2.2.2).
 *   6. The iterated box spline beta^{4,m}_a (Sec. 2.3, eq. (iterated_spline) and
 *      eq. (conv2)) evaluated exactly, and one single-pass filter with it: the direct
 *      sum, and the fast form (m-fold running sums, (m+1)^4 differences, interpolation
 *      with the m-fold convolution of the ZP element).
 *
 * Coordinates: image f[row][col]; x = column index n1, y = row index n2.
 * Directions theta_k = (k-1) pi/4: u1 = (1,0), u2 = (1,1)/sqrt2, u3 = (0,1),
 * u4 = (-1,1)/sqrt2 (Sec. 3, eq. before (final_eqn)).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SQ2 1.41421356237309504880
#define ISQ2 0.70710678118654752440

/* ------------------------------------------------------------------------- */
/* 1. Box spline by polygon clipping                                          */
/* ------------------------------------------------------------------------- */

/* Keep the part of polygon (px,py,n) with  ca*x + cb*y <= cc  (Sutherland-Hodgman). */
static int clip_half(const double *px, const double *py, int n, double ca, double cb, double cc,
                     double *qx, double *qy)
{
    int m = 0;
    for (int i = 0; i < n; ++i) {
        int j = (i + 1) % n;
        double fi = ca * px[i] + cb * py[i] - cc;
        double fj = ca * px[j] + cb * py[j] - cc;
        if (fi <= 0.0) { qx[m] = px[i]; qy[m] = py[i]; ++m; }
        if ((fi < 0.0 && fj > 0.0) || (fi > 0.0 && fj < 0.0)) {
            double t = fi / (fi - fj);
            qx[m] = px[i] + t * (px[j] - px[i]);
            qy[m] = py[i] + t * (py[j] - py[i]);
            ++m;
        }
    }
    return m;
}

static double shoelace(const double *px, const double *py, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        int j = (i + 1) % n;
        s += px[i] * py[j] - px[j] * py[i];
    }
    return 0.5 * fabs(s);
}

/*
 * beta^4_a(x, y): phi_{a1,0} * phi_{a3,pi/2} is the uniform density on the
 * rectangle [-a1/2, a1/2] x [-a3/2, a3/2]; phi_{a2,pi/4} * phi_{a4,3pi/4} is the
 * uniform density on { v : |u2.v| <= a2/2, |u4.v| <= a4/2 }.  Their convolution
 * at x is  area(R13 intersect (x + R24)) / (a1 a2 a3 a4).
 * |u2.(p - x)| <= a2/2  <=>  |(p1 + p2) - (x1 + x2)| <= a2/sqrt2, same for u4 with (p2 - p1).
 */
double svfo_boxspline(const double *a, double x, double y)
{
    double bx[16], by[16], cx[16], cy[16];
    double h1 = 0.5 * a[0], h3 = 0.5 * a[2];
    double r2 = a[1] / SQ2, r4 = a[3] / SQ2;
    bx[0] = -h1; by[0] = -h3;
    bx[1] =  h1; by[1] = -h3;
    bx[2] =  h1; by[2] =  h3;
    bx[3] = -h1; by[3] =  h3;
    int n = 4;
    double s = x + y, d = y - x;
    n = clip_half(bx, by, n,  1.0,  1.0,  s + r2, cx, cy); if (n < 3) return 0.0;
    n = clip_half(cx, cy, n, -1.0, -1.0, -s + r2, bx, by); if (n < 3) return 0.0;
    n = clip_half(bx, by, n, -1.0,  1.0,  d + r4, cx, cy); if (n < 3) return 0.0;
    n = clip_half(cx, cy, n,  1.0, -1.0, -d + r4, bx, by); if (n < 3) return 0.0;
    return shoelace(bx, by, n) / (a[0] * a[1] * a[2] * a[3]);
}

/* ZP element = beta^4_b, b = (1, sqrt2, 1, sqrt2) (Sec. 3.1). */
double svfo_zp(double x, double y)
{
    const double b[4] = {1.0, SQ2, 1.0, SQ2};
    return svfo_boxspline(b, x, y);
}

/* Half extents of the support of beta^4_a (the zonotope sum t_k a_k u_k, |t_k| <= 1/2). */
void svfo_support_halfwidths(const double *a, double *rx, double *ry)
{
    *rx = 0.5 * (a[0] + (a[1] + a[3]) * ISQ2);
    *ry = 0.5 * (a[2] + (a[1] + a[3]) * ISQ2);
}

/* ------------------------------------------------------------------------- */
/* 2. Scale-vector solve (Sec. 3.2.2)                                         */
/* ------------------------------------------------------------------------- */

/* zeta(t) = sum_k (p_k + e_k t)^4 + {(p1+t)^2 + (p3+t)^2}{(p2-t)^2 + (p4-t)^2}, e = (1,-1,1,-1). */
static double zeta(const double *pb, double t)
{
    double p1 = pb[0] + t, p2 = pb[1] - t, p3 = pb[2] + t, p4 = pb[3] - t;
    return p1 * p1 * p1 * p1 + p2 * p2 * p2 * p2 + p3 * p3 * p3 * p3 + p4 * p4 * p4 * p4 +
           (p1 * p1 + p3 * p3) * (p2 * p2 + p4 * p4);
}

/* Real roots of c3 t^3 + c2 t^2 + c1 t + c0 (c3 != 0) by Cardano / Viete. Returns count. */
static int cubic_real_roots(double c3, double c2, double c1, double c0, double *r)
{
    double A = c2 / c3, B = c1 / c3, C = c0 / c3;
    double p = B - A * A / 3.0;
    double q = 2.0 * A * A * A / 27.0 - A * B / 3.0 + C;
    double sh = -A / 3.0;
    double disc = q * q / 4.0 + p * p * p / 27.0;
    int n;
    if (disc > 0.0) {
        double sq = sqrt(disc);
        double u = cbrt(-q / 2.0 + (q <= 0.0 ? sq : -sq));   /* no cancellation */
        double v = (u != 0.0) ? -p / (3.0 * u) : 0.0;
        r[0] = u + v + sh;
        n = 1;
    } else if (p == 0.0) {
        r[0] = sh;
        n = 1;
    } else {
        double m = 2.0 * sqrt(-p / 3.0);
        double arg = (3.0 * q / (p * m)) ;
        if (arg > 1.0) arg = 1.0;
        if (arg < -1.0) arg = -1.0;
        double th = acos(arg) / 3.0;
        for (int k = 0; k < 3; ++k) r[k] = m * cos(th - 2.0 * M_PI * k / 3.0) + sh;
        n = 3;
    }
    /* two Newton polishing steps per root (numerics only; the roots are those above) */
    for (int k = 0; k < n; ++k) {
        for (int it = 0; it < 2; ++it) {
            double t = r[k];
            double f = ((c3 * t + c2) * t + c1) * t + c0;
            double df = (3.0 * c3 * t + 2.0 * c2) * t + c1;
            if (df != 0.0) r[k] = t - f / df;
        }
    }
    return n;
}

/*
 * Largest feasible elongation at fixed size s and orientation theta (reading of
 * Prop. 3.1 with the floor p >= eps): the system M p = c, p >= eps has a
 * solution iff C11 - |C12| >= eps/6 and C22 - |C12| >= eps/6.  Each condition is
 * linear in rho after multiplying by (1 + rho)/s.  Returns +inf when unbounded.
 */
double svfo_rho_max(double s, double theta, double eps)
{
    double c = cos(theta), sn = sin(theta);
    double cs = fabs(sn * c), e = eps / (6.0 * s);
    double best = INFINITY;
    /* condition 1: rho (c^2 - |cs| - e) + (sn^2 + |cs| - e) >= 0 */
    double A1 = c * c - cs - e, B1 = sn * sn + cs - e;
    if (A1 < 0.0) best = fmin(best, B1 / (-A1));
    /* condition 2: rho (sn^2 - |cs| - e) + (c^2 + |cs| - e) >= 0 */
    double A2 = sn * sn - cs - e, B2 = c * c + cs - e;
    if (A2 < 0.0) best = fmin(best, B2 / (-A2));
    return best;
}

/* Covariance from descriptor D1 via D2 (Sec. 3.2.1). */
static void cov_from_srt(double s, double rho, double theta, double *C)
{
    double lmax = s * rho / (1.0 + rho), lmin = s / (1.0 + rho);
    double c = cos(theta), sn = sin(theta);
    C[0] = lmax * c * c + lmin * sn * sn;
    C[1] = 0.5 * (lmax - lmin) * sin(2.0 * theta);
    C[2] = lmin * c * c + lmax * sn * sn;
}

/*
 * Scale vector for covariance C (C[0]=C11, C[1]=C12, C[2]=C22), floor eps on p.
 * Steps (i)-(iii) of Sec. 3.2.2.  Returns 0 on success, -1 if the covariance
 * is not positive definite / not finite, 1 if [t_l, t_r] is empty.
 * *eps_active is set when a component of p sits at the floor.
 */
int svfo_scales_from_cov_feasible(const double *C, double eps, double *a, int *eps_active)
{
    /* (i) pivot p4 = 1 and solve M p_bar = c, c = 24 (C11, C12, C22) */
    double c1 = 24.0 * C[0], c2 = 24.0 * C[1], c3 = 24.0 * C[2];
    double pb[4];
    pb[3] = 1.0;
    pb[1] = c2 + pb[3];
    pb[0] = (c1 - pb[1] - pb[3]) / 2.0;
    pb[2] = (c3 - pb[1] - pb[3]) / 2.0;
    /* (ii) interval and coefficients of zeta'(t) = z1 t^3 + z2 t^2 + z3 t + z4 */
    double tl = fmax(-pb[0] + eps, -pb[2] + eps);
    double tr = fmin(pb[1] - eps, pb[3] - eps);
    if (tl > tr) {
        if (tl - tr > 1e-9 * (fabs(tl) + fabs(tr) + 1.0)) return 1;
        double mid = 0.5 * (tl + tr);
        tl = tr = mid;
    }
    double s1 = pb[0], s2 = pb[1], s3 = pb[2], s4 = pb[3];
    double z1 = 32.0;
    double z2 = 24.0 * (s1 - s2 + s3 - s4);
    double z3 = 16.0 * (s1 * s1 + s2 * s2 + s3 * s3 + s4 * s4) - 8.0 * (s1 + s3) * (s2 + s4);
    double z4 = 4.0 * (s1 * s1 * s1 - s2 * s2 * s2 + s3 * s3 * s3 - s4 * s4 * s4) +
                2.0 * (s1 + s3) * (s2 * s2 + s4 * s4) - 2.0 * (s2 + s4) * (s1 * s1 + s3 * s3);
    /* (iii) real roots inside (t_l, t_r), plus the end points; argmin of zeta */
    double roots[3];
    int nr = cubic_real_roots(z1, z2, z3, z4, roots);
    double best_t = tl, best_z = zeta(pb, tl);
    double zr = zeta(pb, tr);
    if (zr < best_z) { best_z = zr; best_t = tr; }
    for (int k = 0; k < nr; ++k) {
        if (roots[k] > tl && roots[k] < tr) {
            double zk = zeta(pb, roots[k]);
            if (zk < best_z) { best_z = zk; best_t = roots[k]; }
        }
    }
    double p[4] = {pb[0] + best_t, pb[1] - best_t, pb[2] + best_t, pb[3] - best_t};
    int act = 0;
    for (int k = 0; k < 4; ++k) {
        if (p[k] <= eps * (1.0 + 1e-12)) act = 1;
        if (p[k] < eps) p[k] = eps;          /* rounding at the end points only */
        a[k] = sqrt(p[k]);
    }
    if (eps_active) *eps_active = act;
    return 0;
}

/*
 * Field entry (sigma, rho, theta) -> scales of the full filter.
 * Reading of the field: size s = lambda_max + lambda_min = 2 sigma^2 (so the
 * isotropic case has covariance sigma^2 I, as in Thm. 2.2), rho = elongation,
 * theta = orientation.  The elongation is lowered to the feasible maximum when
 * needed (*clamped = 1), and the size raised to eps/3 if even rho = 1 is not
 * feasible.  eps is the floor on p = a^2 for this (full) solve.
 */
int svfo_scales_from_srt(double sigma, double rho, double theta, double eps, double *a, int *clamped,
                         int *eps_active)
{
    if (!(isfinite(sigma) && isfinite(rho) && isfinite(theta)) || sigma <= 0.0 || rho < 1.0) return -1;
    double s = 2.0 * sigma * sigma;
    int cl = 0;
    if (s < eps / 3.0) { s = eps / 3.0; rho = 1.0; cl = 1; }
    double rmax = svfo_rho_max(s, theta, eps);
    if (rho > rmax) { rho = rmax * (1.0 - 1e-12); cl = 1; }
    if (rho < 1.0) rho = 1.0;
    double C[3];
    cov_from_srt(s, rho, theta, C);
    if (clamped) *clamped = cl;
    return svfo_scales_from_cov_feasible(C, eps, a, eps_active);
}

/* Covariance entry: (C11, C12, C22) of the full filter. */
int svfo_scales_from_cov(double c11, double c12, double c22, double eps, double *a, int *clamped,
                         int *eps_active)
{
    if (!(isfinite(c11) && isfinite(c12) && isfinite(c22))) return -1;
    double det = c11 * c22 - c12 * c12;
    if (c11 <= 0.0 || c22 <= 0.0 || det <= 0.0) return -1;
    int feasible = (c11 - fabs(c12) >= eps / 6.0) && (c22 - fabs(c12) >= eps / 6.0);
    if (feasible) {
        if (clamped) *clamped = 0;
        double C[3] = {c11, c12, c22};
        return svfo_scales_from_cov_feasible(C, eps, a, eps_active);
    }
    /* descriptor D1 of the requested covariance, then the clamp of the srt entry */
    double s = c11 + c22;
    double dd = sqrt((c11 - c22) * (c11 - c22) + 4.0 * c12 * c12);
    double lmax = 0.5 * (s + dd), lmin = 0.5 * (s - dd);
    double theta = 0.5 * atan2(2.0 * c12, c11 - c22);
    double rho = lmax / lmin;
    double sigma = sqrt(s / 2.0);
    int r = svfo_scales_from_srt(sigma, rho, theta, eps, a, clamped, eps_active);
    if (clamped) *clamped = 1;
    return r;
}

/* ------------------------------------------------------------------------- */
/* 3. Running sums RS1..RS4 over a window (Algorithm 1, step 2)               */
/* ------------------------------------------------------------------------- */

/*
 * f and g are h x w row-major (f already restricted to the window, zero
 * outside the image).  Zero initial conditions at the window edges.
 *   g0[r][c]  = f[r][c] + g0[r][c-1]
 *   g45[r][c] = sqrt2 g0[r][c] + g45[r-1][c-1]
 *   g90[r][c] = g45[r][c] + g90[r-1][c]
 *   gb[r][c]  = sqrt2 g90[r][c] + gb[r-1][c+1]
 * Each recursion is run over the whole window before the next one.
 */
void svfo_preint_f64(const double *f, long h, long w, double *g)
{
    size_t n = (size_t)h * (size_t)w;
    double *t = (double *)malloc(n * sizeof(double));
    for (long r = 0; r < h; ++r)                                   /* RS1 */
        for (long c = 0; c < w; ++c)
            t[r * w + c] = f[r * w + c] + (c > 0 ? t[r * w + c - 1] : 0.0);
    for (long r = 0; r < h; ++r)                                   /* RS2 */
        for (long c = 0; c < w; ++c)
            g[r * w + c] = SQ2 * t[r * w + c] + ((r > 0 && c > 0) ? g[(r - 1) * w + c - 1] : 0.0);
    for (long r = 0; r < h; ++r)                                   /* RS3 */
        for (long c = 0; c < w; ++c)
            t[r * w + c] = g[r * w + c] + (r > 0 ? t[(r - 1) * w + c] : 0.0);
    for (long r = 0; r < h; ++r)                                   /* RS4 */
        for (long c = 0; c < w; ++c)
            g[r * w + c] = SQ2 * t[r * w + c] + ((r > 0 && c + 1 < w) ? g[(r - 1) * w + c + 1] : 0.0);
    free(t);
}

/*
 * Integer variant for integer images: the same recursions without the sqrt2
 * factors, in wrapping 64-bit arithmetic.  The FP64 pre-integration equals
 * 2 * G (sqrt2 * sqrt2) up to rounding.
 */
void svfo_preint_i64(const int64_t *f, long h, long w, int64_t *g)
{
    size_t n = (size_t)h * (size_t)w;
    uint64_t *t = (uint64_t *)malloc(n * sizeof(uint64_t));
    uint64_t *u = (uint64_t *)g;
    for (long r = 0; r < h; ++r)
        for (long c = 0; c < w; ++c)
            t[r * w + c] = (uint64_t)f[r * w + c] + (c > 0 ? t[r * w + c - 1] : 0u);
    for (long r = 0; r < h; ++r)
        for (long c = 0; c < w; ++c)
            u[r * w + c] = t[r * w + c] + ((r > 0 && c > 0) ? u[(r - 1) * w + c - 1] : 0u);
    for (long r = 0; r < h; ++r)
        for (long c = 0; c < w; ++c)
            t[r * w + c] = u[r * w + c] + (r > 0 ? t[(r - 1) * w + c] : 0u);
    for (long r = 0; r < h; ++r)
        for (long c = 0; c < w; ++c)
            u[r * w + c] = t[r * w + c] + ((r > 0 && c + 1 < w) ? u[(r - 1) * w + c + 1] : 0u);
    free(t);
}

/*
 * Window extraction.  The image is given as a sub-array covering rows
 * [fr0, fr0+fh) x cols [fc0, fc0+fw) of the lattice (dtype 0 = f64, 1 = f32,
 * 2 = u16); samples outside the sub-array are zero (the image is zero-extended,
 * and callers pass a sub-array that covers every sample an output depends on).
 */
static double img_at(const void *img, int dtype, long fr0, long fc0, long fh, long fw, long r, long c)
{
    r -= fr0;
    c -= fc0;
    if (r < 0 || c < 0 || r >= fh || c >= fw) return 0.0;
    size_t i = (size_t)r * (size_t)fw + (size_t)c;
    if (dtype == 0) return ((const double *)img)[i];
    if (dtype == 1) return (double)((const float *)img)[i];
    return (double)((const uint16_t *)img)[i];
}

void svfo_preint_window_f64(const void *img, int dtype, long fr0, long fc0, long fh, long fw, long r0, long c0,
                            long h, long w, double *g)
{
    double *f = (double *)malloc((size_t)h * (size_t)w * sizeof(double));
    for (long r = 0; r < h; ++r)
        for (long c = 0; c < w; ++c) f[r * w + c] = img_at(img, dtype, fr0, fc0, fh, fw, r0 + r, c0 + c);
    svfo_preint_f64(f, h, w, g);
    free(f);
}

void svfo_preint_window_i64(const uint16_t *img, long H, long W, long r0, long c0, long h, long w, int64_t *g)
{
    int64_t *f = (int64_t *)malloc((size_t)h * (size_t)w * sizeof(int64_t));
    for (long r = 0; r < h; ++r)
        for (long c = 0; c < w; ++c) {
            long rr = r0 + r, cc = c0 + c;
            f[r * w + c] = (rr < 0 || cc < 0 || rr >= H || cc >= W) ? 0 : (int64_t)img[rr * W + cc];
        }
    svfo_preint_i64(f, h, w, g);
    free(f);
}

/* ------------------------------------------------------------------------- */
/* 4. Finite difference with ZP interpolation at one pixel                    */
/* ------------------------------------------------------------------------- */

/* Table 1: tap i <-> binary (q4 q3 q2 q1); x_i = q1 a1 u1 + q2 a2 u2 + q3 a3 u3 + q4 a4 u4,
 * written with a'_k = a_k / sqrt2 for k = 2, 4; w_i = (-1)^(q1+q2+q3+q4) / (a1 a2 a3 a4). */
static void table1_tap(const double *a, int i, double *x1, double *x2, double *sgn)
{
    int q1 = i & 1, q2 = (i >> 1) & 1, q3 = (i >> 2) & 1, q4 = (i >> 3) & 1;
    double ap2 = a[1] / SQ2, ap4 = a[3] / SQ2;
    *x1 = q1 * a[0] + q2 * ap2 - q4 * ap4;
    *x2 = q2 * ap2 + q3 * a[2] + q4 * ap4;
    *sgn = ((q1 + q2 + q3 + q4) & 1) ? -1.0 : 1.0;
}

/* Shift tau of Sec. 3.1 step (2). */
static void tau_of(const double *a, double *t1, double *t2)
{
    *t1 = (SQ2 * a[0] + a[1] - a[3] - SQ2) / (2.0 * SQ2);
    *t2 = (a[1] + SQ2 * a[2] + a[3] - 3.0 * SQ2) / (2.0 * SQ2);
}

/* Exported for the tests: tap i of Table 1 and the shift tau. */
void svfo_table1_tap(const double *a, int i, double *x1, double *x2, double *sgn) { table1_tap(a, i, x1, x2, sgn); }
void svfo_tau(const double *a, double *t1, double *t2) { tau_of(a, t1, t2); }

/* Lattice range read by the ZP interpolant at coordinate y (|y - m| < 3/2 in each axis). */
static void zp_range(double y, long *lo, long *hi)
{
    *lo = (long)floor(y - 1.5);
    *hi = (long)ceil(y + 1.5);
}

/*
 * fbar[n] = sum_i w_i F(n + tau - x_i), F(y) = sum_m g[m] ZP(y - m)   (eq. (final_eqn)).
 * g is a window of wh x ww samples whose [0][0] sits at lattice (row wr0, col wc0);
 * gscale multiplies g (2 for the integer scans).  Returns NAN if a needed
 * lattice sample with a non-zero ZP weight falls outside the window.
 */
double svfo_fd_pixel(const double *g, long wh, long ww, long wr0, long wc0, double gscale, long n1, long n2,
                     const double *a)
{
    double t1, t2;
    tau_of(a, &t1, &t2);
    double w = 1.0 / (a[0] * a[1] * a[2] * a[3]);
    double acc = 0.0;
    for (int i = 0; i < 16; ++i) {
        double x1, x2, sgn;
        table1_tap(a, i, &x1, &x2, &sgn);
        double y1 = (double)n1 + t1 - x1, y2 = (double)n2 + t2 - x2;
        long c_lo, c_hi, r_lo, r_hi;
        zp_range(y1, &c_lo, &c_hi);
        zp_range(y2, &r_lo, &r_hi);
        double F = 0.0;
        for (long mr = r_lo; mr <= r_hi; ++mr)
            for (long mc = c_lo; mc <= c_hi; ++mc) {
                double z = svfo_zp(y1 - (double)mc, y2 - (double)mr);
                if (z == 0.0) continue;
                long rr = mr - wr0, cc = mc - wc0;
                if (rr < 0 || cc < 0 || rr >= wh || cc >= ww) return NAN;
                F += g[rr * ww + cc] * z;
            }
        acc += sgn * w * F;
    }
    return gscale * acc;
}

/* ------------------------------------------------------------------------- */
/* 5. One pass over a rectangle of outputs                                    */
/* ------------------------------------------------------------------------- */

/* Bounding box (inclusive) of every lattice sample and every f sample that pixel n with scales a uses. */
static void pixel_bbox(const double *a, long n1, long n2, long *cmin, long *cmax, long *rmin, long *rmax)
{
    double t1, t2, rx, ry;
    tau_of(a, &t1, &t2);
    svfo_support_halfwidths(a, &rx, &ry);
    long c0 = (long)floor(n1 - rx) - 1, c1 = (long)ceil(n1 + rx) + 1;
    long r0 = (long)floor(n2 - ry) - 1, r1 = (long)ceil(n2 + ry) + 1;
    for (int i = 0; i < 16; ++i) {
        double x1, x2, sgn;
        table1_tap(a, i, &x1, &x2, &sgn);
        long lo, hi;
        zp_range(n1 + t1 - x1, &lo, &hi);
        if (lo < c0) c0 = lo;
        if (hi > c1) c1 = hi;
        zp_range(n2 + t2 - x2, &lo, &hi);
        if (lo < r0) r0 = lo;
        if (hi > r1) r1 = hi;
    }
    *cmin = c0; *cmax = c1; *rmin = r0; *rmax = r1;
}

/*
 * Fast algorithm, one pass.  Input image as a sub-array (see img_at), per-pixel
 * scales a (h x w x 4, f64) of this pass for the output rectangle rows
 * [r0, r0+h) x cols [c0, c0+w), outputs into out (h x w).  The rectangle is cut
 * into tiles of side `tile`; each tile is pre-integrated on the smallest window
 * containing every sample its pixels read (truncated running sums are exact
 * there: truncation only adds terms that are constant along one box direction,
 * and that direction's difference removes them).  Returns 0, or -1 if a pixel
 * read outside its window (cannot happen unless the scales are not finite).
 */
int svfo_pass_fast(const void *f, int dtype, long fr0, long fc0, long fh, long fw, const double *a, long r0,
                   long c0, long h, long w, long tile, double *out)
{
    if (tile <= 0) tile = 32;
    long nty = (h + tile - 1) / tile, ntx = (w + tile - 1) / tile;
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
    for (long ti = 0; ti < nty * ntx; ++ti) {
        long ty = ti / ntx, tx = ti % ntx;
        long pr0 = r0 + ty * tile, pc0 = c0 + tx * tile;
        long pr1 = pr0 + tile < r0 + h ? pr0 + tile : r0 + h;
        long pc1 = pc0 + tile < c0 + w ? pc0 + tile : c0 + w;
        long wc_lo = pc0, wc_hi = pc1 - 1, wr_lo = pr0, wr_hi = pr1 - 1;
        for (long r = pr0; r < pr1; ++r)
            for (long c = pc0; c < pc1; ++c) {
                long a0, a1, b0, b1;
                pixel_bbox(a + ((size_t)(r - r0) * w + (c - c0)) * 4, c, r, &a0, &a1, &b0, &b1);
                if (a0 < wc_lo) wc_lo = a0;
                if (a1 > wc_hi) wc_hi = a1;
                if (b0 < wr_lo) wr_lo = b0;
                if (b1 > wr_hi) wr_hi = b1;
            }
        long wh = wr_hi - wr_lo + 1, ww = wc_hi - wc_lo + 1;
        double *g = (double *)malloc((size_t)wh * (size_t)ww * sizeof(double));
        svfo_preint_window_f64(f, dtype, fr0, fc0, fh, fw, wr_lo, wc_lo, wh, ww, g);
        for (long r = pr0; r < pr1; ++r)
            for (long c = pc0; c < pc1; ++c) {
                const double *ap = a + ((size_t)(r - r0) * w + (c - c0)) * 4;
                double v = svfo_fd_pixel(g, wh, ww, wr_lo, wc_lo, 1.0, c, r, ap);
                if (isnan(v)) fail = 1;
                out[(r - r0) * w + (c - c0)] = v;
            }
        free(g);
    }
    return fail ? -1 : 0;
}

/* Brute force, one pass: out[n] = sum_k f[k] beta^4_{a(n)}(n - k) over the same rectangle. */
int svfo_pass_brute(const void *f, int dtype, long fr0, long fc0, long fh, long fw, const double *a, long r0,
                    long c0, long h, long w, double *out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < h * w; ++i) {
        long r = r0 + i / w, c = c0 + i % w;
        const double *ap = a + (size_t)i * 4;
        double rx, ry;
        svfo_support_halfwidths(ap, &rx, &ry);
        long k1lo = (long)floor(c - rx), k1hi = (long)ceil(c + rx);
        long k2lo = (long)floor(r - ry), k2hi = (long)ceil(r + ry);
        double acc = 0.0;
        for (long k2 = k2lo; k2 <= k2hi; ++k2)
            for (long k1 = k1lo; k1 <= k1hi; ++k1) {
                double fv = img_at(f, dtype, fr0, fc0, fh, fw, k2, k1);
                if (fv == 0.0) continue;
                acc += fv * svfo_boxspline(ap, (double)(c - k1), (double)(r - k2));
            }
        out[i] = acc;
    }
    return 0;
}

/* beta^4_a on a regular grid x0 + i hx, y0 + j hy (i < nx, j < ny); out is ny x nx. */
void svfo_boxspline_grid(const double *a, double x0, double y0, double hx, double hy, long nx, long ny, double *out)
{
#pragma omp parallel for
    for (long j = 0; j < ny; ++j)
        for (long i = 0; i < nx; ++i) out[j * nx + i] = svfo_boxspline(a, x0 + i * hx, y0 + j * hy);
}

/* Scale field for a pass: field kind 0 = (C11,C12,C22), 1 = (sigma,rho,theta), 2 = scales (a1..a4).
 * Writes per-pass scales a/sqrt(order) (f64, H x W x 4) and counts clamped / floor-active /
 * invalid pixels.  eps is the per-pass floor on a^2; the full solve uses order * eps. */
int svfo_scale_field(const float *field, int kind, long H, long W, int order, double eps, double *a_out,
                     long *n_clamped, long *n_eps, long *n_invalid)
{
    long ncl = 0, nep = 0, ninv = 0;
    int ch = (kind == 2) ? 4 : 3;
    double inv = 1.0 / sqrt((double)order);
#pragma omp parallel for reduction(+ : ncl, nep, ninv)
    for (long i = 0; i < H * W; ++i) {
        const float *v = field + (size_t)i * ch;
        double a[4] = {0, 0, 0, 0};
        int cl = 0, ea = 0, rc = 0;
        if (kind == 0) rc = svfo_scales_from_cov(v[0], v[1], v[2], order * eps, a, &cl, &ea);
        else if (kind == 1) rc = svfo_scales_from_srt(v[0], v[1], v[2], order * eps, a, &cl, &ea);
        else {
            for (int k = 0; k < 4; ++k) a[k] = v[k];
            if (!(a[0] > 0 && a[1] > 0 && a[2] > 0 && a[3] > 0)) rc = -1;
        }
        if (rc != 0) { ++ninv; for (int k = 0; k < 4; ++k) a[k] = NAN; }
        ncl += cl;
        nep += ea;
        for (int k = 0; k < 4; ++k) a_out[(size_t)i * 4 + k] = a[k] * inv;
    }
    if (n_clamped) *n_clamped = ncl;
    if (n_eps) *n_eps = nep;
    if (n_invalid) *n_invalid = ninv;
    return ninv ? -1 : 0;
}

/* Threads of the OpenMP loops above (n <= 0 leaves the runtime's choice); returns the
 * count the next parallel loops use.  Changes no arithmetic. */
int svfo_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* ------------------------------------------------------------------------- */
/* 6. Iterated box spline beta^{4,m}_a and the single-pass filter             */
/* ------------------------------------------------------------------------- */

/*
 * beta^{4,m}_a is the m-fold convolution of beta^4_a with itself (eq. (iterated_spline)):
 * the density of sum_k S_k a_k u_k with S_k the sum of m independent U(-1/2, 1/2), whose
 * Fourier transform is prod_k sinc^m (eq. (conv2)).  S_k a_k has the density
 * B_m(s / a_k) / a_k, B_m the centred cardinal B-spline of order m.  Pairing the
 * directions, X = S1 a1 u1 + S3 a3 u3 has the density B_m(x/a1) B_m(y/a3) / (a1 a3) and
 * Y = S2 a2 u2 + S4 a4 u4 the same in the rotated coordinates (u2.z, u4.z), and
 *   beta^{4,m}_a(x) = int p_X(x - z) p_Y(z) dz.
 * Each factor is one polynomial on each cell of an m x m grid (p_Y's grid in the rotated
 * frame), so the integral is a sum over the convex intersections of one cell of each.
 * On an intersection the integrand is a polynomial of degree 4(m-1); it is integrated on
 * the triangles of a fan by the collapsed (Duffy) product of n = 2m-1 point
 * Gauss-Legendre rules, exact for that degree.
 */

/* Centred cardinal B-spline of order m (support [-m/2, m/2]) by its truncated powers. */
static double bspline_c(int m, double x)
{
    double h = 0.5 * m;
    if (x <= -h || x >= h) return 0.0;
    double s = 0.0, c = 1.0, fact = 1.0;
    for (int j = 2; j < m; ++j) fact *= j;
    for (int j = 0; j <= m; ++j) {
        double t = x + h - j;
        if (t > 0.0) {
            double p = 1.0;
            for (int e = 0; e < m - 1; ++e) p *= t;
            s += c * p;
        }
        c = -c * (double)(m - j) / (double)(j + 1);
    }
    return s / fact;
}

/* n-point Gauss-Legendre nodes and weights on [0, 1] (Newton on the Legendre recurrence). */
static void gauss01(int n, double *x, double *w)
{
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = n == 1 ? z : p1, pm = n == 1 ? 1.0 : p0;
            dp = n * (z * pn - pm) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);   /* 2 / ((1 - z^2) P'^2), halved for [0, 1] */
    }
}

struct itp {                 /* integrand of one evaluation */
    const double *a;
    int m;
    double x1, x2;
};

static double itp_f(const struct itp *q, double z1, double z2)
{
    const double *a = q->a;
    double s = (z1 + z2) * ISQ2, t = (z2 - z1) * ISQ2;
    double px = bspline_c(q->m, (q->x1 - z1) / a[0]) * bspline_c(q->m, (q->x2 - z2) / a[2]) / (a[0] * a[2]);
    if (px == 0.0) return 0.0;
    return px * bspline_c(q->m, s / a[1]) * bspline_c(q->m, t / a[3]) / (a[1] * a[3]);
}

/* Integral over a convex polygon: fan triangles, collapsed Gauss product rule. */
static double poly_integral(const struct itp *q, const double *px, const double *py, int n, int ng,
                            const double *gx, const double *gw)
{
    double acc = 0.0;
    for (int k = 1; k + 1 < n; ++k) {
        double ax = px[0], ay = py[0];
        double e1x = px[k] - ax, e1y = py[k] - ay, e2x = px[k + 1] - px[k], e2y = py[k + 1] - py[k];
        double det = fabs(e1x * e2y - e1y * e2x);
        if (det == 0.0) continue;
        double tri = 0.0;
        for (int i = 0; i < ng; ++i)
            for (int j = 0; j < ng; ++j) {
                double s = gx[i], t = gx[j];
                double z1 = ax + s * e1x + s * t * e2x, z2 = ay + s * e1y + s * t * e2y;
                tri += gw[i] * gw[j] * s * itp_f(q, z1, z2);
            }
        acc += det * tri;
    }
    return acc;
}

double svfo_boxspline_m(const double *a, int m, double x, double y)
{
    if (m < 1 || m > 4) return NAN;
    double gx[8], gw[8];
    int ng = 2 * m - 1;
    gauss01(ng, gx, gw);
    struct itp q = {a, m, x, y};
    double h = 0.5 * m, acc = 0.0;
    for (int i1 = 0; i1 < m; ++i1)
        for (int i3 = 0; i3 < m; ++i3) {
            /* cell of p_X(x - z): (x - z)/a1 in [i1 - h, i1 + 1 - h], same for row with a3 */
            double z1lo = x - a[0] * (i1 + 1 - h), z1hi = x - a[0] * (i1 - h);
            double z2lo = y - a[2] * (i3 + 1 - h), z2hi = y - a[2] * (i3 - h);
            for (int i2 = 0; i2 < m; ++i2)
                for (int i4 = 0; i4 < m; ++i4) {
                    double s0 = a[1] * (i2 - h), s1 = a[1] * (i2 + 1 - h);
                    double t0 = a[3] * (i4 - h), t1 = a[3] * (i4 + 1 - h);
                    /* corners z = s u2 + t u4, counter-clockwise in (s, t) */
                    double bx[16], by[16], cx[16], cy[16];
                    double ss[4] = {s0, s1, s1, s0}, tt[4] = {t0, t0, t1, t1};
                    for (int k = 0; k < 4; ++k) {
                        bx[k] = (ss[k] - tt[k]) * ISQ2;
                        by[k] = (ss[k] + tt[k]) * ISQ2;
                    }
                    int n = 4;
                    n = clip_half(bx, by, n, -1.0, 0.0, -z1lo, cx, cy); if (n < 3) continue;
                    n = clip_half(cx, cy, n, 1.0, 0.0, z1hi, bx, by);   if (n < 3) continue;
                    n = clip_half(bx, by, n, 0.0, -1.0, -z2lo, cx, cy); if (n < 3) continue;
                    n = clip_half(cx, cy, n, 0.0, 1.0, z2hi, bx, by);   if (n < 3) continue;
                    acc += poly_integral(&q, bx, by, n, ng, gx, gw);
                }
        }
    return acc;
}

/* beta^{4,m}_b, b = (1, sqrt2, 1, sqrt2): the m-fold convolution of the ZP element. */
double svfo_zp_m(int m, double x, double y)
{
    const double b[4] = {1.0, SQ2, 1.0, SQ2};
    return svfo_boxspline_m(b, m, x, y);
}

/*
 * Fast single pass with beta^{4,m}_a.  beta^{4,m} is the box spline whose directions are
 * those of beta^4 each taken m times; the same argument as for m = 1 (Sec. 3.1) gives
 *   fbar[n] = (1 / prod_k a_k^m) sum_{j in {0..m}^4} prod_k C(m, j_k) (-1)^{j_k}
 *             F_m(n + m tau - sum_k j_k a_k u_k),   F_m(y) = sum_l g_m[l] ZP^{*m}(y - l),
 * where g_m applies the running sums RS1..RS4 m times (each time with the sqrt2 factors)
 * and tau is the shift of Sec. 3.1 step (2).  (m = 1 is eq. (final_eqn).)  A reading: the
 * paper states the iterated spline and its use by repeated passes (Sec. 3.3, "Higher-order
 * box splines"), not this single-pass form; fast = direct sum is checked by the tests.
 */
double svfo_fd_pixel_m(const double *g, long wh, long ww, long wr0, long wc0, long n1, long n2, const double *a,
                       int m)
{
    double t1, t2;
    tau_of(a, &t1, &t2);
    double w = 1.0;
    for (int k = 0; k < 4; ++k)
        for (int e = 0; e < m; ++e) w /= a[k];
    double binom[5] = {1, 0, 0, 0, 0};
    for (int j = 1; j <= m; ++j) binom[j] = binom[j - 1] * (double)(m - j + 1) / (double)j;
    double ap2 = a[1] / SQ2, ap4 = a[3] / SQ2, reach = 1.5 * m, acc = 0.0;
    int nt = 1;
    for (int k = 0; k < 4; ++k) nt *= (m + 1);
    for (int idx = 0; idx < nt; ++idx) {
        int j[4], r = idx;
        double coef = 1.0;
        for (int k = 0; k < 4; ++k) {
            j[k] = r % (m + 1);
            r /= (m + 1);
            coef *= ((j[k] & 1) ? -1.0 : 1.0) * binom[j[k]];
        }
        double x1 = j[0] * a[0] + j[1] * ap2 - j[3] * ap4;
        double x2 = j[1] * ap2 + j[2] * a[2] + j[3] * ap4;
        double y1 = (double)n1 + m * t1 - x1, y2 = (double)n2 + m * t2 - x2;
        long c_lo = (long)floor(y1 - reach), c_hi = (long)ceil(y1 + reach);
        long r_lo = (long)floor(y2 - reach), r_hi = (long)ceil(y2 + reach);
        double F = 0.0;
        for (long mr = r_lo; mr <= r_hi; ++mr)
            for (long mc = c_lo; mc <= c_hi; ++mc) {
                double z = svfo_zp_m(m, y1 - (double)mc, y2 - (double)mr);
                if (z == 0.0) continue;
                long rr = mr - wr0, cc = mc - wc0;
                if (rr < 0 || cc < 0 || rr >= wh || cc >= ww) return NAN;
                F += g[rr * ww + cc] * z;
            }
        acc += coef * w * F;
    }
    return acc;
}

/* g = (RS1..RS4 applied m times) of the window of the image (zero outside it). */
void svfo_preint_window_m_f64(const void *img, int dtype, long fr0, long fc0, long fh, long fw, long r0, long c0,
                              long h, long w, int m, double *g)
{
    svfo_preint_window_f64(img, dtype, fr0, fc0, fh, fw, r0, c0, h, w, g);
    double *t = (double *)malloc((size_t)h * (size_t)w * sizeof(double));
    for (int it = 1; it < m; ++it) {
        memcpy(t, g, (size_t)h * (size_t)w * sizeof(double));
        svfo_preint_f64(t, h, w, g);
    }
    free(t);
}

/* One single pass over a rectangle of outputs, per-pixel windows (the smallest window a
 * pixel reads, which keeps the m-fold sums as small as they can be); fast form.  A
 * window that starts inside the image is exact for the same reason as for m = 1: the
 * truncation only adds terms that one direction's m-th difference removes. */
int svfo_pass_fast_m(const void *f, int dtype, long fr0, long fc0, long fh, long fw, const double *a, long r0,
                     long c0, long h, long w, int m, double *out)
{
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
    for (long i = 0; i < h * w; ++i) {
        long r = r0 + i / w, c = c0 + i % w;
        const double *ap = a + (size_t)i * 4;
        /* every lattice sample the taps' interpolants read */
        double t1, t2;
        tau_of(ap, &t1, &t2);
        double ap2 = ap[1] / SQ2, ap4 = ap[3] / SQ2, reach = 1.5 * m;
        long wc_lo = c, wc_hi = c, wr_lo = r, wr_hi = r;
        for (int j1 = 0; j1 <= m; ++j1)
            for (int j2 = 0; j2 <= m; ++j2)
                for (int j3 = 0; j3 <= m; ++j3)
                    for (int j4 = 0; j4 <= m; ++j4) {
                        double y1 = c + m * t1 - (j1 * ap[0] + j2 * ap2 - j4 * ap4);
                        double y2 = r + m * t2 - (j2 * ap2 + j3 * ap[2] + j4 * ap4);
                        long lo = (long)floor(y1 - reach), hi = (long)ceil(y1 + reach);
                        if (lo < wc_lo) wc_lo = lo;
                        if (hi > wc_hi) wc_hi = hi;
                        lo = (long)floor(y2 - reach);
                        hi = (long)ceil(y2 + reach);
                        if (lo < wr_lo) wr_lo = lo;
                        if (hi > wr_hi) wr_hi = hi;
                    }
        long wh = wr_hi - wr_lo + 1, ww = wc_hi - wc_lo + 1;
        double *g = (double *)malloc((size_t)wh * (size_t)ww * sizeof(double));
        svfo_preint_window_m_f64(f, dtype, fr0, fc0, fh, fw, wr_lo, wc_lo, wh, ww, m, g);
        double v = svfo_fd_pixel_m(g, wh, ww, wr_lo, wc_lo, c, r, ap, m);
        if (isnan(v)) fail = 1;
        out[i] = v;
        free(g);
    }
    return fail ? -1 : 0;
}

/* Direct sum, one single pass: out[n] = sum_k f[k] beta^{4,m}_{a(n)}(n - k). */
int svfo_pass_brute_m(const void *f, int dtype, long fr0, long fc0, long fh, long fw, const double *a, long r0,
                      long c0, long h, long w, int m, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < h * w; ++i) {
        long r = r0 + i / w, c = c0 + i % w;
        const double *ap = a + (size_t)i * 4;
        double rx, ry;
        svfo_support_halfwidths(ap, &rx, &ry);
        long k1lo = (long)floor(c - m * rx), k1hi = (long)ceil(c + m * rx);
        long k2lo = (long)floor(r - m * ry), k2hi = (long)ceil(r + m * ry);
        double acc = 0.0;
        for (long k2 = k2lo; k2 <= k2hi; ++k2)
            for (long k1 = k1lo; k1 <= k1hi; ++k1) {
                double fv = img_at(f, dtype, fr0, fc0, fh, fw, k2, k1);
                if (fv == 0.0) continue;
                acc += fv * svfo_boxspline_m(ap, m, (double)(c - k1), (double)(r - k2));
            }
        out[i] = acc;
    }
    return 0;
}


/*
 * Sanitizer driver for the CPU oracle: calls every exported function of
 * oracle/svf_oracle.c on small inputs (ragged windows, uint16 / f32 / f64 images,
 * every field kind, m = 1..3 single passes) under AddressSanitizer and
 * UndefinedBehaviorSanitizer, and checks a few identities on the way (fast pass =
 * direct sum, integer sums = 2 x the binary64 ones' half).  Built and run by
 * tests/test_sanitize.py; exit status 0 when every check holds and no sanitizer fired.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double svfo_boxspline(const double *a, double x, double y);
double svfo_zp(double x, double y);
void svfo_support_halfwidths(const double *a, double *rx, double *ry);
double svfo_rho_max(double s, double theta, double eps);
int svfo_scales_from_cov_feasible(const double *C, double eps, double *a, int *eps_active);
int svfo_scales_from_srt(double sigma, double rho, double theta, double eps, double *a, int *clamped, int *eps_active);
int svfo_scales_from_cov(double c11, double c12, double c22, double eps, double *a, int *clamped, int *eps_active);
void svfo_preint_f64(const double *f, long h, long w, double *g);
void svfo_preint_i64(const int64_t *f, long h, long w, int64_t *g);
void svfo_preint_window_f64(const void *img, int dtype, long fr0, long fc0, long fh, long fw, long r0, long c0, long h,
                            long w, double *g);
void svfo_preint_window_i64(const uint16_t *img, long H, long W, long r0, long c0, long h, long w, int64_t *g);
void svfo_table1_tap(const double *a, int i, double *x1, double *x2, double *sgn);
void svfo_tau(const double *a, double *t1, double *t2);
double svfo_fd_pixel(const double *g, long wh, long ww, long wr0, long wc0, double gscale, long n1, long n2,
                     const double *a);
int svfo_pass_fast(const void *f, int dtype, long fr0, long fc0, long fh, long fw, const double *a, long r0, long c0,
                   long h, long w, long tile, double *out);
int svfo_pass_brute(const void *f, int dtype, long fr0, long fc0, long fh, long fw, const double *a, long r0, long c0,
                    long h, long w, double *out);
void svfo_boxspline_grid(const double *a, double x0, double y0, double hx, double hy, long nx, long ny, double *out);
int svfo_scale_field(const float *field, int kind, long H, long W, int order, double eps, double *a_out,
                     long *n_clamped, long *n_eps, long *n_invalid);
int svfo_set_threads(int n);
double svfo_boxspline_m(const double *a, int m, double x, double y);
double svfo_zp_m(int m, double x, double y);
int svfo_pass_fast_m(const void *f, int dtype, long fr0, long fc0, long fh, long fw, const double *a, long r0, long c0,
                     long h, long w, int m, double *out);
int svfo_pass_brute_m(const void *f, int dtype, long fr0, long fc0, long fh, long fw, const double *a, long r0,
                      long c0, long h, long w, int m, double *out);

static int fails = 0;
#define CHECK(c, ...)                                                    \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed (%s:%d): ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);                                \
            fprintf(stderr, "\n");                                       \
            ++fails;                                                     \
        }                                                                \
    } while (0)

static double urand(unsigned *s) { *s = *s * 1664525u + 1013904223u; return (*s >> 8) * (1.0 / 16777216.0); }

int main(void)
{
    unsigned seed = 12345u;
    svfo_set_threads(2);
    const double a[4] = {1.3, 2.1, 1.7, 0.9};
    double rx, ry, x1, x2, sg, t1, t2;
    svfo_support_halfwidths(a, &rx, &ry);
    svfo_tau(a, &t1, &t2);
    for (int i = 0; i < 16; ++i) svfo_table1_tap(a, i, &x1, &x2, &sg);
    CHECK(fabs(svfo_zp(0, 0) - 0.5) < 1e-15, "ZP(0)");
    CHECK(fabs(svfo_boxspline_m(a, 1, 0.3, -0.2) - svfo_boxspline(a, 0.3, -0.2)) < 1e-14, "m = 1");
    CHECK(svfo_zp_m(2, 0.2, 0.1) > 0.0, "ZP*ZP");
    double grid[6 * 5];
    svfo_boxspline_grid(a, -1, -1, 0.4, 0.5, 6, 5, grid);
    /* scale solves of every kind, including clamps and invalid requests */
    double sc[4];
    int cl, ea;
    CHECK(svfo_scales_from_srt(2.0, 1.5, 0.3, 0.25, sc, &cl, &ea) == 0, "srt");
    CHECK(svfo_scales_from_srt(0.1, 9.0, 2.0, 0.25, sc, &cl, &ea) == 0 && cl, "srt clamp");
    CHECK(svfo_scales_from_cov(3.0, 0.5, 2.0, 0.25, sc, &cl, &ea) == 0, "cov");
    CHECK(svfo_scales_from_cov(1.0, 2.0, 1.0, 0.25, sc, &cl, &ea) != 0, "cov not positive definite");
    const double C[3] = {3.0, 0.4, 2.5};
    CHECK(svfo_scales_from_cov_feasible(C, 0.25, sc, &ea) == 0, "feasible");
    CHECK(svfo_rho_max(2.0, 0.1, 0.25) > 1.0, "rho max");
    /* images: 11 x 13 f64, f32, u16 */
    enum { H = 11, W = 13 };
    double f64[H * W];
    float f32[H * W], fld[H * W * 4];
    uint16_t u16[H * W];
    for (int i = 0; i < H * W; ++i) {
        f64[i] = urand(&seed);
        f32[i] = (float)f64[i];
        u16[i] = (uint16_t)(urand(&seed) * 65535.0);
        fld[3 * i + 0] = (float)(1.0 + 1.5 * urand(&seed));
        fld[3 * i + 1] = (float)(1.0 + 2.0 * urand(&seed));
        fld[3 * i + 2] = (float)(3.1 * urand(&seed));
    }
    double *as = malloc(sizeof(double) * H * W * 4);
    long ncl, nep, ninv;
    CHECK(svfo_scale_field(fld, 1, H, W, 2, 0.25, as, &ncl, &nep, &ninv) == 0, "scale field srt");
    svfo_scale_field(fld, 0, H, W, 1, 0.25, as + 0, &ncl, &nep, &ninv);   /* cov kind: some invalid, fine */
    CHECK(svfo_scale_field(fld, 1, H, W, 1, 0.25, as, &ncl, &nep, &ninv) == 0, "scale field order 1");
    /* running sums: window extending past the image on every side, ragged */
    double g[(H + 6) * (W + 5)];
    int64_t gi[(H + 6) * (W + 5)];
    svfo_preint_window_f64(u16, 2, 0, 0, H, W, -3, -2, H + 6, W + 5, g);
    svfo_preint_window_i64(u16, H, W, -3, -2, H + 6, W + 5, gi);
    for (int i = 0; i < (H + 6) * (W + 5); ++i) CHECK(fabs(g[i] - 2.0 * (double)gi[i]) <= 1e-9 * fabs(g[i]) + 1e-6, "i64");
    int64_t fi[4] = {1, 2, 3, 4}, go[4];
    svfo_preint_i64(fi, 2, 2, go);
    double fd[4] = {1, 2, 3, 4}, gd[4];
    svfo_preint_f64(fd, 2, 2, gd);
    (void)svfo_fd_pixel(g, H + 6, W + 5, -3, -2, 1.0, 5, 5, a);
    /* passes: fast = direct sum for every image type, several tiles */
    double out1[H * W], out2[H * W];
    const void *imgs[3] = {f64, f32, u16};
    for (int dt = 0; dt < 3; ++dt) {
        CHECK(svfo_pass_fast(imgs[dt], dt, 0, 0, H, W, as, 0, 0, H, W, 4, out1) == 0, "fast %d", dt);
        CHECK(svfo_pass_brute(imgs[dt], dt, 0, 0, H, W, as, 0, 0, H, W, out2) == 0, "brute %d", dt);
        for (int i = 0; i < H * W; ++i)
            CHECK(fabs(out1[i] - out2[i]) <= 1e-9 * (1.0 + fabs(out2[i])), "fast = brute (%d, %d)", dt, i);
    }
    /* single passes, m = 1..3, on a sub-rectangle */
    for (int m = 1; m <= 3; ++m) {
        double o1[4 * 5], o2[4 * 5], am[4 * 5 * 4];
        for (int i = 0; i < 4 * 5; ++i)
            for (int k = 0; k < 4; ++k) am[4 * i + k] = 1.0 + 0.8 * urand(&seed);
        CHECK(svfo_pass_fast_m(f64, 0, 0, 0, H, W, am, 3, 4, 4, 5, m, o1) == 0, "fast m %d", m);
        CHECK(svfo_pass_brute_m(f64, 0, 0, 0, H, W, am, 3, 4, 4, 5, m, o2) == 0, "brute m %d", m);
        for (int i = 0; i < 4 * 5; ++i) CHECK(fabs(o1[i] - o2[i]) <= 1e-8, "single m %d px %d", m, i);
    }
    CHECK(isnan(svfo_boxspline_m(a, 5, 0, 0)), "m out of range");
    free(as);
    if (fails) fprintf(stderr, "%d checks failed\n", fails);
    else printf("oracle sanitizer run: all checks passed\n");
    return fails ? 1 : 0;
}

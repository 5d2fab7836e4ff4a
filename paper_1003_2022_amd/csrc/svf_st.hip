// svf_st.hip -- gfx950 kernels of the structure-tensor step of the
// feature-preserving smoothing (Sec. 4.2):
//
//   k_st_outer : g = central differences of the image (each channel), written as
//                P = sum_c (g1^2, g1 g2, g2^2), three floats per pixel.  The
//                window w * P is then the ordinary filter (isotropic box spline,
//                constant scales) run by the runtime on P as a 3-channel image.
//   k_st_field : J -> (sigma, rho, theta): the eigen-decomposition of gain * J in
//                closed form and the printed rules; theta is the direction of the
//                eigenvector of the smaller eigenvalue, sigma = sqrt(s / 2).
//
// Both are one pass over HBM per pixel (no reuse beyond the four neighbours of
// the differences, which the L1/L2 serve): 256 x 4 pixel blocks, each thread
// four pixels 64 columns apart whose loads are all issued before any is used
// (one pixel per thread left the kernels waiting on memory latency), coalesced
// rows, 12-byte pixel records moved as one access per lane.

#include <hip/hip_runtime.h>

#include <type_traits>

#include "svf_internal.h"

namespace svf {
namespace {

constexpr int kStPx = 4;                       // pixels per thread, 64 columns apart
constexpr int kStCols = 64 * kStPx, kStRows = 4;
// one work-group per pixel block (a persistent grid of 8 work-groups per CU
// looping over the blocks measured 17 % slower)
constexpr int kStGrid = 1 << 20;

// three floats of one pixel, moved as one 12-byte access (global_load / store_dwordx3)
struct F3 {
    float x, y, z;
};

template <int IN>
__device__ __forceinline__ double st_load(const StImage &im, int64_t r, int64_t c, int ch)
{
    // neighbour (r, c) of the differences: the boundary rule outside the image
    // (zero rule: the value 0)
    if (im.boundary == kBoundZero && (r < 0 || r >= im.H || c < 0 || c >= im.W)) return 0.0;
    const int64_t R = ext_index(r, im.H, im.boundary), C = ext_index(c, im.W, im.boundary);
    if (IN == kInF32) return (double)static_cast<const float *>(im.in)[R * im.in_rs + C * im.C + ch];
    return (double)static_cast<const unsigned short *>(im.in)[R * im.in_rs + C * im.C + ch];
}

template <int IN>
__global__ __launch_bounds__(64 * kStRows) void k_st_outer(StImage im, float *P, int64_t p_rs, int nbx,
                                                           int64_t nblocks)
{
    using E = typename std::conditional<IN == kInF32, float, unsigned short>::type;
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const int64_t by = b / nbx, bx = b - by * nbx;
        const int64_t r = by * kStRows + (threadIdx.x >> 6), c0 = bx * kStCols + (threadIdx.x & 63);
        if (r >= im.H) continue;
        // one channel, all neighbours inside: the four pixels' loads first
        if (im.C == 1 && r > 0 && r + 1 < im.H && c0 > 0 && c0 + 64 * (kStPx - 1) + 1 < im.W) {
            const E *q = static_cast<const E *>(im.in) + r * im.in_rs + c0;
            float vl[kStPx], vr[kStPx], vu[kStPx], vd[kStPx];
#pragma unroll
            for (int k = 0; k < kStPx; ++k) {
                vl[k] = (float)q[64 * k - 1];
                vr[k] = (float)q[64 * k + 1];
                vu[k] = (float)q[64 * k - im.in_rs];
                vd[k] = (float)q[64 * k + im.in_rs];
            }
#pragma unroll
            for (int k = 0; k < kStPx; ++k) {
                const double g1 = 0.5 * ((double)vr[k] - (double)vl[k]);
                const double g2 = 0.5 * ((double)vd[k] - (double)vu[k]);
                *reinterpret_cast<F3 *>(P + r * p_rs + (c0 + 64 * k) * 3) =
                    F3{(float)(g1 * g1), (float)(g1 * g2), (float)(g2 * g2)};
            }
            continue;
        }
#pragma unroll 1
        for (int k = 0; k < kStPx; ++k) {
            const int64_t c = c0 + 64 * k;
            if (c >= im.W) break;
            double p11 = 0.0, p12 = 0.0, p22 = 0.0;
            if (r > 0 && r + 1 < im.H && c > 0 && c + 1 < im.W) {   // all four neighbours inside
                const E *q = static_cast<const E *>(im.in) + r * im.in_rs + c * im.C;
                for (int ch = 0; ch < im.C; ++ch) {
                    const double g1 = 0.5 * ((double)q[ch + im.C] - (double)q[ch - im.C]);
                    const double g2 = 0.5 * ((double)q[ch + im.in_rs] - (double)q[ch - im.in_rs]);
                    p11 += g1 * g1;
                    p12 += g1 * g2;
                    p22 += g2 * g2;
                }
            } else {
                for (int ch = 0; ch < im.C; ++ch) {
                    const double g1 = 0.5 * (st_load<IN>(im, r, c + 1, ch) - st_load<IN>(im, r, c - 1, ch));
                    const double g2 = 0.5 * (st_load<IN>(im, r + 1, c, ch) - st_load<IN>(im, r - 1, c, ch));
                    p11 += g1 * g1;
                    p12 += g1 * g2;
                    p22 += g2 * g2;
                }
            }
            *reinterpret_cast<F3 *>(P + r * p_rs + c * 3) = F3{(float)p11, (float)p12, (float)p22};
        }
    }
}

constexpr double kPi = 3.14159265358979323846;

// The rules for one pixel: (a, b, c) = gain * (J11, J12, J22) -> (sigma, rho, theta).
__device__ __forceinline__ F3 st_rules(F3 jv, double gain, double lambda_zero, double a_flat)
{
    const double a = gain * (double)jv.x, bb = gain * (double)jv.y, cc = gain * (double)jv.z;
    // eigenvalues of [[a, b], [b, c]]: the larger from the trace and the
    // discriminant, the smaller as det / larger (no cancellation)
    const double dif = a - cc;
    const double disc = sqrt(dif * dif + 4.0 * bb * bb);
    const double lmax = 0.5 * ((a + cc) + disc);
    const double lmin = lmax > 0.0 ? (a * cc - bb * bb) / lmax : 0.5 * ((a + cc) - disc);
    const bool zmax = !(lmax > lambda_zero), zmin = !(lmin > lambda_zero);
    double s, rho, theta;
    if (zmax && zmin) {   // locally flat: isotropic box spline with all scales a_flat
        s = a_flat * a_flat / 3.0;
        rho = 1.0;
        theta = 0.0;
    } else {
        // eigenvector of the larger eigenvalue at 0.5 atan2(2b, a - c); the
        // filter's major axis is the other one.  The angle is stored as float32:
        // the binary32 arctangent of the rounded arguments (error ~1e-7 rad)
        theta = 0.5 * (double)atan2f((float)(2.0 * bb), (float)dif) + 0.5 * kPi;
        if (theta >= kPi) theta -= kPi;
        if (theta < 0.0) theta += kPi;
        if (zmin) {   // only the larger eigenvalue is non-zero
            s = lmax;
            rho = fmax(1.0, lmax);
        } else {
            s = lmax + lmin;
            rho = lmax / lmin;
        }
    }
    return F3{(float)sqrt(0.5 * s), (float)rho, (float)theta};
}

__global__ __launch_bounds__(64 * kStRows) void k_st_field(const float *J, int64_t j_rs, int64_t H, int64_t W,
                                                           double gain, double lambda_zero, double a_flat,
                                                           float *F, int64_t f_rs, int nbx, int64_t nblocks)
{
    for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
        const int64_t by = b / nbx, bx = b - by * nbx;
        const int64_t r = by * kStRows + (threadIdx.x >> 6), c0 = bx * kStCols + (threadIdx.x & 63);
        if (r >= H) continue;
        F3 jv[kStPx];
#pragma unroll
        for (int k = 0; k < kStPx; ++k)
            if (c0 + 64 * k < W) jv[k] = *reinterpret_cast<const F3 *>(J + r * j_rs + (c0 + 64 * k) * 3);
#pragma unroll
        for (int k = 0; k < kStPx; ++k)
            if (c0 + 64 * k < W)
                *reinterpret_cast<F3 *>(F + r * f_rs + (c0 + 64 * k) * 3) = st_rules(jv[k], gain, lambda_zero, a_flat);
    }
}

__global__ void k_fill_f4(float4 *p, float4 v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int64_t st_blocks(int64_t H, int64_t W, int *nbx)
{
    *nbx = (int)((W + kStCols - 1) / kStCols);
    return (int64_t)*nbx * ((H + kStRows - 1) / kStRows);
}

}  // namespace

hipError_t launch_st_outer(const StImage &im, float *P, int64_t p_rs, hipStream_t s)
{
    int nbx;
    const int64_t nb = st_blocks(im.H, im.W, &nbx);
    if (nb == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(nb, kStGrid);
    if (im.in_type == kInF32)
        hipLaunchKernelGGL(k_st_outer<kInF32>, dim3(grid), dim3(64 * kStRows), 0, s, im, P, p_rs, nbx, nb);
    else
        hipLaunchKernelGGL(k_st_outer<kInU16>, dim3(grid), dim3(64 * kStRows), 0, s, im, P, p_rs, nbx, nb);
    return hipGetLastError();
}

hipError_t launch_st_field(const float *J, int64_t j_rs, int64_t H, int64_t W, double gain, double lambda_zero,
                           double a_flat, float *F, int64_t f_rs, hipStream_t s)
{
    int nbx;
    const int64_t nb = st_blocks(H, W, &nbx);
    if (nb == 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(nb, kStGrid);
    hipLaunchKernelGGL(k_st_field, dim3(grid), dim3(64 * kStRows), 0, s, J, j_rs, H, W, gain, lambda_zero,
                       a_flat, F, f_rs, nbx, nb);
    return hipGetLastError();
}

hipError_t launch_fill_f4(float *p, float4 v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_f4, dim3(grid), dim3(256), 0, s, reinterpret_cast<float4 *>(p), v, n);
    return hipGetLastError();
}

}  // namespace svf

// svf_internal.h -- shared between the gfx950 kernels (svf_kernels.hip) and the
// host runtime (svf_runtime.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace svf {

constexpr int kScanThreads = 256;    // one work-group per (tile, channel) window
constexpr int kScanCols = 2 * kScanThreads;   // columns per chunk: two adjacent columns per thread
constexpr int kScanChunks = 2;       // window width <= 2 * 512 columns
constexpr int kMaxWindow = kScanCols * kScanChunks;
constexpr int kSmapRows = 4;         // scale map: each thread handles 4 rows of a 64 x 16 block
constexpr int kSmapCols = 64;        // scale map: block of 64 columns x 16 rows
constexpr int kMaxChannels = 4;

enum Preint : int32_t { kPreF64 = 0, kPreF32C = 1, kPreI64 = 2 };
enum InType : int32_t { kInF32 = 0, kInU16 = 1 };
enum FieldKind : int32_t { kCov3 = 0, kSrt3 = 1, kScales4 = 2 };
enum Boundary : int32_t { kBoundZero = 0, kBoundReplicate = 1, kBoundSymmetric = 2 };

// Per-tile results of the scale map: largest support half-widths of the whole
// filter (sizing the tile's pre-integration window) and pixel counts for the report.
struct TileStat {
    float rx, ry;
    uint32_t clamped, eps_active, invalid, overflow;
    uint32_t pad0, pad1;
};
static_assert(sizeof(TileStat) == 32, "TileStat layout");

// Per 16 x 16 pixel block of the finite difference: the block's window and the
// origins of its staged sample regions, one per distinct abscissa / ordinate of the
// 16 taps (from the block's centre pixel), in window coordinates.  Written once per
// filter call after the scale map (k_fd_plan) and read by every pass, whose scales
// are the filter's times 1 / sqrt(order).
struct FdBlk {
    int32_t ax[8], ay[8];    // region origins: abscissa k = q1 + 2 q2 + 4 q4, ordinate k = q2 + 2 q3 + 4 q4
    int32_t wr0, wc0;        // window origin (image rows / columns)
    int32_t ww, wh;          // window width / height
    int32_t br0, bc0;        // first pixel of the block
    int32_t tile, pad;
};
static_assert(sizeof(FdBlk) == 96, "FdBlk layout");

// One image of a filter call, for one pass.  Passed by value for a single image
// and stored in a device table for batched launches.
struct Job {
    // pass input (pass 1: the caller's image; later passes: the output buffer)
    const void *in;
    int64_t in_rs;           // elements between rows
    int32_t in_type;         // InType
    int32_t C;               // channels (1..4)
    int64_t H, W;
    // output (float32, same layout rules)
    float *out;
    int64_t out_rs;
    // scales of the whole filter, float4 per pixel
    const float *scales;
    int64_t sc_rs;           // floats between rows (multiple of 4)
    // field (scale map input)
    const float *field;
    int64_t f_rs;
    int32_t f_kind;
    int32_t preint;          // Preint of this pass
    // segment-local pre-integration
    TileStat *tstat;         // per tile: half-widths of the whole filter and report counts
    void *g;                 // window slots: (tile * C + ch) * slot_elems elements of the g type
    int64_t slot_elems;
    int32_t T;               // tile side
    int32_t ntr, ntc;        // tile rows / columns
    int32_t cap;             // largest half-width a window is sized for (one pass)
    float inv_sqrt_m;        // 1 / sqrt(order)
    int32_t fd_fp32;
    double inv_sqrt_m_d;
    double eps_full;         // floor on a^2 of the whole filter (order * eps per pass)
    // batched launches: first global tile / FD block / scale block of this job
    int32_t tile_base, blk_base, smap_base;
    int32_t boundary;        // Boundary: what a pass reads outside the image
    // single-image launches cover the tile rows [tr0, tr1) (scale map: their pixel rows)
    int32_t tr0, tr1;
    // finite-difference block plan (k_fd_plan writes it, k_fd reads it): one FdBlk
    // per block of the tile-major block list
    FdBlk *fdplan;
    // serving: the request's invalid / overflow pixel counts (nullptr: not kept)
    uint32_t *req_counts;
    // look-up-table scale map (nullptr: the solve per pixel)
    const float *lut;        // lut_n x lut_n float4, [i][j]: rho = (n-1)/i, phi = j pi / (4 (n-1)), s = 1
    int32_t lut_n, pad2;
    double lut_eps;          // the table's floor on a^2 at s = 1
};

// Size of a batched launch read by its kernels from device memory (the server's
// steps: one captured HIP graph then serves every step with the same kernels):
// jobs in the table and work items over all of them.
struct BatchDims {
    int32_t n, total;
};

// Rectangle of lattice samples pre-integrated for one tile.
struct Window {
    int64_t r0, c0;
    int32_t h, w;
};

// Image index whose value lattice index i (possibly outside [0, N)) takes in a
// pass input.  Zero rule: any in-range index (the value is masked to zero by the
// caller).  Replicate: the nearest index.  Symmetric: the half-sample mirror
// f[-1 - i] = f[i], f[2N - 1 - i] = f[i] (period 2N; small images reflect
// several times).
__device__ __forceinline__ int64_t ext_index(int64_t i, int64_t N, int b)
{
    if (b == kBoundSymmetric) {
        if (i < 0) i = -1 - i;
        if (i >= N) {   // rare: only windows that cross the far border
            const int n2 = 2 * (int)N;
            int m = (int)i % n2;   // i < N + 2 * kMaxWindow: fits in 32 bits
            if (m >= (int)N) m = n2 - 1 - m;
            i = m;
        }
        return i;
    }
    return min(max(i, (int64_t)0), N - 1);
}

// Structure-tensor step (svf_st.hip).  Image geometry of one call.
struct StImage {
    const void *in;
    int64_t in_rs;           // elements between rows
    int32_t in_type;         // InType
    int32_t C;               // channels
    int64_t H, W;
    int32_t boundary;        // Boundary (the gradient's neighbours)
    int32_t pad;
};
// P = sum over channels of (g1^2, g1 g2, g2^2), central differences; float32, 3 per pixel
hipError_t launch_st_outer(const StImage &im, float *P, int64_t p_rs, hipStream_t s);
// J (3 per pixel) -> (sigma, rho, theta) by the eigenvalue rules
hipError_t launch_st_field(const float *J, int64_t j_rs, int64_t H, int64_t W, double gain, double lambda_zero,
                           double a_flat, float *F, int64_t f_rs, hipStream_t s);
// fill n float4 with v
hipError_t launch_fill_f4(float *p, float4 v, int64_t n, hipStream_t s);

// Host-side launchers (defined in svf_kernels.hip).  All enqueue on `s`.
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_scale_map(const Job &j, hipStream_t s);
// unit-size scale table for the look-up-table scale map (n x n float4)
hipError_t launch_lut_build(float *lut, int n, double eps, hipStream_t s);
hipError_t launch_preint(const Job &j, hipStream_t s);
hipError_t launch_fd(const Job &j, hipStream_t s);
// the finite difference's block plan (after the scale map, before the first pass)
hipError_t launch_fd_plan(const Job &j, hipStream_t s);
hipError_t launch_fd_plan_batch(const Job *jobs, int n, int total_blocks, hipStream_t s, const BatchDims *dims = nullptr,
                                int grid = 0);
// constant filter (every pixel's scales equal; 3 channels, binary64 difference):
// whether the staged region of a block fits, and the launch
bool fd_uniform_fits(double a1, double a2, double a3, double a4, int channels);
hipError_t launch_fd_uniform(const Job &j, const double *pass_a, hipStream_t s);
// standalone pre-integration of a caller-given window (svf_preintegrate)
hipError_t launch_preint_window(const Job &j, int channel, int64_t r0, int64_t c0, int h, int w, void *g,
                                hipStream_t s);
// batched: `jobs` is a device table of n jobs; totals are the sums of the per-job counts
// (persistent: `grid` work-groups loop over the work list).  With dims != nullptr the
// kernels read n and the total from it instead (device memory) and the grid is
// `grid` as given (a graph replayed for steps of different sizes).
// kind: the field kind of every job of the table (a kernel compiled for it), or -1
// for a mix
hipError_t launch_scale_map_batch(const Job *jobs, int n, int total_blocks, int grid, bool lut, int kind,
                                  hipStream_t s, const BatchDims *dims = nullptr);
hipError_t launch_preint_batch(const Job *jobs, int n, int total_tiles, int grid, int preint, hipStream_t s,
                               const BatchDims *dims = nullptr);
hipError_t launch_fd_batch(const Job *jobs, int n, int total_blocks, int grid, int preint, int fd_fp32, int nch,
                           hipStream_t s, const BatchDims *dims = nullptr);
// zero the tile records (and request counters) of the jobs of a table (dims: as above)
hipError_t launch_fill_jobs(const Job *jobs, int n, int grid, hipStream_t s, const BatchDims *dims = nullptr);

int64_t slot_elems_for(int T, int cap);
int scale_map_blocks(int64_t H, int64_t W);
int fd_blocks_job(const Job &j);   // tile-major FD blocks, ragged edge tiles included

}  // namespace svf

/*
 * svf.h -- C ABI of libsvf, a gfx950 (MI355X) implementation of O(1)-per-pixel
 * space-variant elliptical filtering with the four-directional box spline of
 * Chaudhury, Munoz-Barrutia and Unser, "Fast space-variant elliptical
 * filtering using box splines".
 *
 * What is computed (per channel, per pass):
 *
 *     out[n] = sum_k f[k] beta^4_{a(n)}(n - k)            (eq. (discrete) with
 *                                                          the Dirac-comb input)
 *
 * realised by Algorithm 1: the running sums RS1..RS4 with lattice scales
 * b = (1, sqrt2, 1, sqrt2) (Sec. 3.1 step (1)), then at every pixel the 16-tap
 * finite difference of eq. (final_eqn) with the taps of Table 1 and the shift
 * tau of Sec. 3.1 step (2), sampling the ZP-interpolated pre-integrated image
 * (App. F).  The per-pixel scale vector a(n) comes from the pixel's covariance
 * by the optimisation of Sec. 3.2.2; order m > 1 runs m passes with a/sqrt(m)
 * (Sec. 3.3).  N (directions) must be 4.
 *
 * Conventions (all entry points):
 *  - Images are row-major: sample (row r, column c, channel ch) sits at
 *    data[r * row_stride + c * channels + ch]; x = column, y = row; an
 *    orientation theta is measured from +x towards +y.  Outside the image the
 *    input is zero (zero extension).
 *  - Every pointer to image, field or output data is DEVICE memory owned by the
 *    caller; the library never frees it.  The library owns its workspace, which
 *    lives in the context (allocated on first use, reused, grown on demand).
 *  - Work is enqueued on the caller's stream and returns without waiting,
 *    except where a report is requested (svf_filter with rep != NULL, the
 *    batch and server calls documented below).
 *  - No exception crosses the ABI.  Argument errors are detected on the host
 *    before anything is enqueued and returned as a status; svf_last_error()
 *    gives a message.  A context must not be used from two threads at once.
 */
#ifndef SVF_H
#define SVF_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SVF_OK = 0,
    SVF_EINVAL = 1,        /* bad argument, or (with a report) invalid field content */
    SVF_EUNSUPPORTED = 2,  /* N != 4, unsupported dtype / variant combination */
    SVF_ENOMEM = 3,        /* workspace would exceed the context's HBM budget, or allocation failed */
    SVF_EHIP = 4,          /* a HIP runtime call failed */
    SVF_EBUSY = 5,         /* server queue full / request not admitted */
    SVF_ECANCELLED = 6,    /* request cancelled */
    SVF_ERANGE = 7         /* (with a report) a support exceeded max_reach_px; those outputs are not valid */
} svf_status;

typedef enum { SVF_F32 = 0, SVF_U16 = 1 } svf_dtype;

/* Per-pixel field describing the filter at each pixel (float32, H x W x K). */
typedef enum {
    SVF_FIELD_COV3 = 0,    /* K = 3: (C11, C12, C22) covariance of the whole filter, px^2 (descriptor D3) */
    SVF_FIELD_SRT3 = 1,    /* K = 3: (sigma, rho, theta): size s = 2 sigma^2 = lambda_max + lambda_min,
                              elongation rho = lambda_max / lambda_min >= 1, orientation theta (rad) of the
                              major axis (descriptor D1; isotropic covariance sigma^2 I) */
    SVF_FIELD_SCALES4 = 2  /* K = 4: box scales (a1, a2, a3, a4) of the whole filter, px (> 0);
                              pass scales are a / sqrt(order) */
} svf_field_kind;

/* Arithmetic of the running sums. */
typedef enum {
    SVF_PRE_F64 = 0,   /* binary64 sums */
    SVF_PRE_F32C = 1,  /* binary32 pairs (hi, lo) with error-free (two-sum / two-product) accumulation */
    SVF_PRE_I64 = 2    /* exact 64-bit integer sums without the sqrt2 factors (uint16 input, first pass);
                          later passes of an order > 1 filter use SVF_PRE_F64 */
} svf_preint;

typedef struct {
    void *data;          /* device pointer */
    int32_t dtype;       /* svf_dtype; outputs are always SVF_F32 */
    int32_t channels;    /* 1..4 */
    int64_t H, W;        /* rows, columns (>= 0) */
    int64_t row_stride;  /* elements between rows, >= W * channels */
} svf_image;

typedef struct {
    const float *data;   /* device pointer, H x W x K floats (K = 3 or 4) */
    int32_t kind;        /* svf_field_kind */
    int32_t reserved;
    int64_t row_stride;  /* floats between rows, >= W * K; for SCALES4 a multiple of 4 (16-byte rows) */
} svf_field;

/* Values of a pass input outside the image.  The running sums (Sec. 2.1) need a
 * boundary condition and the paper leaves it open.  Every pass of an order-m
 * filter extends its own input by the rule: output n is
 * sum_k f_ext[k] beta(n - k) over the whole lattice. */
typedef enum {
    SVF_BOUNDARY_ZERO = 0,       /* f = 0 outside the image (mass leaks at the borders) */
    SVF_BOUNDARY_REPLICATE = 1,  /* f[i] = f[clamp(i, 0, N - 1)] per axis */
    SVF_BOUNDARY_SYMMETRIC = 2   /* half-sample mirror per axis: f[-1 - i] = f[i], f[2N - 1 - i] = f[i]
                                    (period 2N; an image narrower than the support reflects again) */
} svf_boundary;

/* From the field to the scale vector (Sec. 3.2.2). */
typedef enum {
    SVF_SCALE_SOLVE = 0,  /* the optimisation solved at every pixel (floor eps_px2 * order on a_k^2) */
    SVF_SCALE_LUT = 1     /* the paper's table: unit-size solutions over u = 1/rho in [0, 1] and
                             phi in [0, pi/4] (lut_nodes^2 nodes, built once per (nodes, floor) on
                             the device and kept by the context); per pixel the octant k of theta,
                             bilinear interpolation at (1/rho, theta - k pi/4), the vector rotated
                             by k places ((a1,a2,a3,a4) -> (a4,a1,a2,a3) per octant) and scaled by
                             sqrt(s).  The floor is relative (lut_eps_rel * s); the covariance
                             error of the interpolation is ~1e-4 of s at 129 nodes. */
} svf_scale_method;

typedef struct {
    int32_t preint;       /* svf_preint, default SVF_PRE_F64 */
    int32_t fd_fp32;      /* 0: finite difference and interpolation in binary64 (default);
                             1: in binary32 (comparison variant; far less accurate) */
    double eps_px2;       /* floor on a_k^2 of every pass, px^2 (default 0.25, i.e. a_k >= 0.5 px);
                             the solve of the whole filter uses order * eps_px2 */
    int32_t tile;         /* output tile side for the segment-local pre-integration: 0 = automatic,
                             else 64, 128 or 256 */
    int32_t max_reach_px; /* largest support half-width of one pass the workspace is sized for
                             (default 128 px; <= 380) */
    int32_t bands;        /* svf_filter: 0 or 1 = whole-image launches in sequence on the caller's
                             stream (default); 2..8 = that many bands of tile rows (at least 4
                             tile rows each) on internal streams, pass p of a band starting once
                             pass p-1 of the bands its windows reach is done.  Results are the
                             same bit for bit. */
    int32_t boundary;     /* svf_boundary: what every pass reads outside the image (default
                             SVF_BOUNDARY_ZERO) */
    int32_t scale_map;    /* svf_scale_method: how the field becomes scales (default SVF_SCALE_SOLVE) */
    int32_t lut_nodes;    /* SVF_SCALE_LUT: nodes per table axis, 9..1025 (default 129) */
    double lut_eps_rel;   /* SVF_SCALE_LUT: floor on a_k^2 relative to the size s, in (0, 1]
                             (default 0.125); replaces eps_px2 */
} svf_opts;

typedef struct {
    int64_t clamped_px;    /* pixels whose elongation was lowered to the feasible maximum */
    int64_t eps_active_px; /* pixels with a component of a^2 at the floor */
    int64_t invalid_px;    /* pixels with a non-finite / non-positive-definite field entry: with
                              SVF_FIELD_COV3 / SVF_FIELD_SRT3 they are filtered with the smallest
                              isotropic scales instead; SVF_FIELD_SCALES4 entries that are not
                              finite and positive give NaN outputs */
    int64_t overflow_px;   /* pixels whose support exceeded max_reach_px; their outputs are NaN */
    double max_reach_px;   /* largest support half-width of one pass over the image */
} svf_report;

typedef struct svf_ctx svf_ctx;

/* Fill opts with the defaults listed above. */
void svf_default_opts(svf_opts *opts);

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the workspace
 * (0 = no cap).  Returns SVF_EHIP if the device cannot be selected. */
svf_status svf_create(svf_ctx **ctx, int device, size_t hbm_budget_bytes);

/* Release the workspace and the context.  Waits for the context's pending work. */
svf_status svf_destroy(svf_ctx *ctx);

/* Message of the last error on this context (never NULL). */
const char *svf_last_error(const svf_ctx *ctx);

/* Device workspace, in bytes, that svf_filter needs for these arguments
 * (Sec. 3.1: one pre-integrated window per output tile and channel, sized by
 * opts->max_reach_px; plus the scale field).  Host-only, no device access. */
svf_status svf_workspace_bytes(const svf_image *in, int N, int order, const svf_opts *opts, size_t *bytes);

/*
 * Scale-vector map (Sec. 3.2.2, Prop. 3.1): field -> scales of the whole
 * filter, float32 (a1, a2, a3, a4) per pixel into scales_out (device, H x W x 4,
 * contiguous).  An infeasible elongation is lowered to the largest feasible one
 * at the same size and orientation; eps is opts->eps_px2 * order.
 */
svf_status svf_scale_map(svf_ctx *ctx, const svf_field *field, int64_t H, int64_t W, int order,
                         const svf_opts *opts, float *scales_out, hipStream_t stream);

/*
 * Running sums RS1..RS4 (Sec. 3.1 step (1), Algorithm 1 step 2) of channel
 * `channel` of `in`, on the window rows [r0, r0+h) x cols [c0, c0+w) of the
 * lattice (may extend beyond the image: the input is zero there), with zero
 * initial conditions at the window's top, left and right edges.  g_out
 * (device, h x w contiguous) receives:
 *   SVF_PRE_F64  : double, g_b;
 *   SVF_PRE_F32C : float pairs (hi, lo) with hi + lo = g_b;
 *   SVF_PRE_I64  : int64, the integer sums G with g_b = 2 G (uint16 input only; exact).
 * Window side limited to 1024 columns.
 */
svf_status svf_preintegrate(svf_ctx *ctx, const svf_image *in, int channel, int64_t r0, int64_t c0, int64_t h,
                            int64_t w, int preint, void *g_out, hipStream_t stream);

/*
 * The filter: order-`order` (1..3) space-variant filtering of every channel of
 * `in` with the field, N = 4.  out must be SVF_F32 with in's H, W, channels; it
 * may be the same buffer as an SVF_F32 input (also with opts.bands > 1).  Pixels
 * whose pass support exceeds opts.max_reach_px, and pixels with invalid
 * SVF_FIELD_SCALES4 scales, are written as NaN whether or not a report is asked
 * for.  If rep != NULL the call waits for completion, fills *rep, and returns
 * SVF_EINVAL if invalid_px > 0 or SVF_ERANGE if overflow_px > 0.
 */
svf_status svf_filter(svf_ctx *ctx, const svf_image *in, const svf_field *field, int N, int order,
                      const svf_opts *opts, svf_image *out, hipStream_t stream, svf_report *rep);

/*
 * One pass with the iterated box spline beta^{4,m} (Sec. 2.3, eq. (iterated_spline);
 * Sec. 3.3, "Higher-order box splines"): per channel
 *
 *     out[n] = sum_k f[k] beta^{4,m}_{a(n)}(n - k),   a(n) = (scales of the field) / sqrt(m),
 *
 * the scales solved as for svf_filter of order m (floor m * opts.eps_px2), so that the
 * covariance is the field's.  beta^{4,m} is beta^4 convolved with itself m times
 * (Fourier transform prod_k sinc^m, eq. (conv2)); where svf_filter of order m applies
 * m passes of beta^4 with the scales of each pass's own pixels, this applies the exact
 * beta^{4,m} of each output pixel's scales.  m = 2.  Fast form: the running sums
 * RS1..RS4 applied twice on a window per 16 x 16 tile, the 81-tap difference
 * prod_k (1 - shift by a_k u_k)^2, interpolation with ZP*ZP.
 * Precision: the doubled sums grow like the window side^8, so the outputs of small
 * filters on busy images lose digits: a pixel whose rounding bound
 * 2^-46 max|g2| / prod_k a_k^2 (max over its tile's window) exceeds 1e-6 of the window's
 * largest input magnitude is written as NaN, as are pixels with invalid
 * SVF_FIELD_SCALES4 scales.  Windows up to the 157 KiB of LDS a work-group takes
 * (support half-width up to about 60 px) are summed in LDS; larger ones go to a
 * second launch that keeps each window in a global-memory slot of the context
 * (512 slots of the largest window: 0.5 GB at a half-width of 170 px; counted against
 * the context's budget).  With rep != NULL the call waits, fills *rep
 * (overflow_px = NaN outputs, max_reach_px = largest beta^{4,2} support half-width) and
 * returns SVF_ERANGE if some output is NaN, SVF_EINVAL for invalid field entries.  The
 * call waits for the scale map in any case (the window size follows from it).  A
 * support half-width above 2 opts.max_reach_px (two passes' worth) returns SVF_ERANGE
 * after the scale map, with the output not written (the report, if asked for, holds
 * the counts and max_reach_px).  SVF_EUNSUPPORTED: m != 2, opts.boundary other than zero, opts.preint other than
 * SVF_PRE_F64, opts.fd_fp32, opts.bands > 1.  out must not alias in.
 */
svf_status svf_filter_single(svf_ctx *ctx, const svf_image *in, const svf_field *field, int m,
                             const svf_opts *opts, svf_image *out, hipStream_t stream, svf_report *rep);

/*
 * svf_filter for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, checks and results as svf_filter (bit for bit: the same kernels),
 * without a report; it calls no allocating routine.  Its workspace is a fixed
 * array of the library in each device's memory, 64 MiB (enough for a one-channel
 * 512 x 512 image or a 3-channel 320 x 320 one at the default max_reach_px;
 * svf_workspace_bytes gives the need), held until the process ends; its address
 * on a device is looked up by svf_create.  Returns SVF_ENOMEM (nothing enqueued)
 * when the image needs more, SVF_EUNSUPPORTED for opts.scale_map = SVF_SCALE_LUT
 * or opts.bands > 1.  Every call on a device shares that device's array and
 * leaves its contents behind: calls that overlap on one device (on different
 * streams, or from different threads or contexts) race; enqueue them on one
 * stream.  Kernel timing (svf_set_timing) does not cover these calls.
 */
svf_status svf_filter_noalloc(svf_ctx *ctx, const svf_image *in, const svf_field *field, int N, int order,
                              const svf_opts *opts, svf_image *out, hipStream_t stream);

/*
 * Many images in one launch sequence: n images, each with its own field and
 * order (1..3).  All tiles of all images share one scale-map launch and, per
 * pass, one pre-integration and one finite-difference launch over a device
 * descriptor table (a work-group finds its image by a search over prefix
 * counts).  With use_graph != 0 the launch sequence is captured once per
 * distinct shape set into a HIP graph and replayed.  Results equal n
 * svf_filter calls with the same options bit for bit (opts.tile 0 means 256
 * here, so it is svf_filter with opts.tile = 256 that the batch reproduces).  Returns after enqueueing (the descriptor upload is
 * stream-ordered).
 */
svf_status svf_filter_batch(svf_ctx *ctx, int n, const svf_image *in, const svf_field *fields, const int *orders,
                            const svf_opts *opts, svf_image *out, hipStream_t stream, int use_graph);

/*
 * Reports of the last svf_filter_batch on this context (call it before any other
 * filter call on the context): waits for that batch's stream, fills reps[i] for
 * image i (n = the batch's image count), and returns SVF_EINVAL if some image has
 * invalid_px > 0, else SVF_ERANGE if some has overflow_px > 0 (those outputs are
 * NaN, as in svf_filter).
 */
svf_status svf_filter_batch_report(svf_ctx *ctx, int n, svf_report *reps);

/* ---- feature-preserving smoothing (Sec. 4.2) ----
 *
 * The filter at every pixel is estimated from the image: the structure tensor
 * J = w * (g g^T), g the gradient, w an isotropic averaging window; theta* is
 * the direction of the eigenvector of the smaller eigenvalue of J (least
 * intensity variation, along the image features); with lmax >= lmin the
 * eigenvalues of gain * J: rho* = lmax / lmin if both are non-zero, 1 if both
 * are zero, max(1, lmax) if only lmax is; s* = lmax + lmin (a zero one counting
 * as 0).  Flat pixels (both zero) get the isotropic box spline with all scales
 * a_flat.  Details the paper leaves open, fixed here: g by central differences
 * (g1 along columns, g2 along rows; the neighbours of border pixels follow
 * opts->boundary); channels add their g g^T; w is the isotropic box spline of
 * covariance sigma_w^2 I (scales sigma_w sqrt 6, Thm. 2.2) iterated order_w
 * times and applied by the filter itself with opts (its pre-integration is
 * never SVF_PRE_I64: SVF_PRE_F64 then); gain scales J before the rules.
 */
typedef struct {
    double sigma_w;      /* window standard deviation, px (> 0; default 2) */
    int32_t order_w;     /* window passes 1..3 (default 1) */
    int32_t reserved;
    double gain;         /* the rules act on gain * J (> 0; default 1: the image's own units) */
    double lambda_zero;  /* an eigenvalue <= lambda_zero counts as zero (>= 0; default 0) */
    double a_flat;       /* box scales of the flat-pixel filter, px (> 0; default 1) */
} svf_st_params;

/* Fill p with the defaults listed above. */
void svf_st_default_params(svf_st_params *p);

/*
 * Structure tensor and the field it implies, for an image `in` (SVF_F32 or
 * SVF_U16, 1..4 channels, values taken as they are).  tensor_out (device, may
 * be NULL): (J11, J12, J22) float32 per pixel, rows tensor_row_stride floats
 * apart (>= 3 W), J not scaled by gain.  field_out (device, may be NULL, not
 * both): the SVF_FIELD_SRT3 field (sigma = sqrt(s* / 2), rho*, theta* in
 * [0, pi)), rows field_row_stride floats apart (>= 3 W).  Needs a workspace of
 * 12 B per pixel (24 if tensor_out is NULL) plus the filter's own for a
 * 3-channel image (svf_workspace_bytes).  Returns after enqueueing.
 */
svf_status svf_structure_tensor(svf_ctx *ctx, const svf_image *in, const svf_st_params *params,
                                const svf_opts *opts, float *tensor_out, int64_t tensor_row_stride,
                                float *field_out, int64_t field_row_stride, hipStream_t stream);

/*
 * The smoothing itself: svf_structure_tensor's field drives svf_filter of `in`
 * (order 1..3, opts as for svf_filter, the same boundary rule throughout) into
 * out (SVF_F32, in's shape).  Workspace: 24 B per pixel plus the larger of the
 * two filters' own.  rep as for svf_filter (of the final filter).
 */
svf_status svf_smooth_adaptive(svf_ctx *ctx, const svf_image *in, const svf_st_params *params, int order,
                               const svf_opts *opts, svf_image *out, hipStream_t stream, svf_report *rep);

/* ---- serving loop ----
 * A scheduler thread owned by the context admits requests (images of any size,
 * each with its own field and order) in arrival order while they fit in a
 * device-memory budget and a slot limit, and runs them with continuous
 * batching: every scheduler step enqueues, on the server's own stream, one
 * pass (pre-integration + finite difference, preceded by the scale map for a
 * request's first pass) of the requests in flight, oldest first, up to a
 * per-step work budget, all through the batched persistent kernels.  Requests
 * join and leave between steps.  Each request computes what
 * svf_filter_batch computes for it (svf_filter's result bit for bit;
 * opts.tile 0 means 256 here), bit for bit whatever the mix it ran in.  Input, field and output stay in caller-owned device memory
 * that must remain valid until the request is done.  The integer
 * pre-integration is not offered by the server (opts.preint must be F64 or
 * F32C).
 */
typedef struct {
    int32_t max_inflight;       /* requests on the device at once (default 16) */
    int32_t queue_capacity;     /* waiting requests; submit returns SVF_EBUSY beyond (default 1024) */
    uint64_t hbm_budget_bytes;  /* device memory for the windows and scales of requests in flight */
    int32_t step_mpixels;       /* work per scheduler step: passes are taken in admission order until
                                   their pixels x channels reach this many million (the oldest always
                                   runs; later, smaller passes fill what is left); <= 0: 64 */
    int32_t use_graph;          /* != 0: each step's launch sequence (descriptor upload, scale map, block
                                   plan, pre-integration, difference, counter download) is captured once
                                   per kernel set and grid sizes as a HIP graph and replayed; the kernels
                                   read the step's sizes from device memory */
    svf_opts opts;              /* options of every request */
} svf_server_cfg;

typedef struct {
    svf_image in;
    svf_field field;
    int32_t order;
    int32_t reserved;
    svf_image out;
} svf_request;

typedef struct {
    int32_t status;             /* SVF_OK when done, SVF_EBUSY while queued or running, else the error:
                                   SVF_EINVAL / SVF_ERANGE when pixels had invalid field entries / supports
                                   beyond max_reach_px (as svf_filter's report; the output is written,
                                   NaN at those pixels where svf_filter writes NaN), SVF_ECANCELLED,
                                   SVF_EHIP if a launch failed */
    int32_t done;
    double t_submit_us;         /* host steady clock, microseconds */
    double t_admit_us;
    double t_done_us;           /* when the host observed the request's last step complete */
} svf_result;

typedef struct {
    int64_t submitted, completed, rejected, steps;
    int64_t pixels;             /* output pixels x channels of completed requests */
    double busy_us;             /* wall time with at least one request in flight */
    int64_t cancelled;          /* requests ended by svf_server_cancel */
} svf_server_stats_t;

/* Start the scheduler (allocates hbm_budget_bytes on the context's device). */
svf_status svf_server_start(svf_ctx *ctx, const svf_server_cfg *cfg);
/* Queue a request (arguments are checked here); *id identifies it. */
svf_status svf_server_submit(svf_ctx *ctx, const svf_request *req, uint64_t *id);
/* Non-blocking state of a request.  A finished request's state stays readable
 * until 4 * queue_capacity + 1024 later requests have finished; after that its id
 * is unknown (SVF_EINVAL). */
svf_status svf_server_poll(svf_ctx *ctx, uint64_t id, svf_result *res);
/* Wait up to timeout_s seconds (< 0: forever) for a request; SVF_EBUSY on timeout. */
svf_status svf_server_wait(svf_ctx *ctx, uint64_t id, svf_result *res, double timeout_s);
/* Cancel a request.  A queued request ends at once; one in flight runs no
 * further pass and ends when the passes already on the device complete (its
 * output then holds an unspecified mix of passes).  Either way the request
 * ends with status SVF_ECANCELLED and SVF_OK is returned.  SVF_EBUSY (nothing
 * changed) when the request is done or its last pass is already launched: it
 * completes normally; SVF_EINVAL for an unknown id. */
svf_status svf_server_cancel(svf_ctx *ctx, uint64_t id);
svf_status svf_server_stats(svf_ctx *ctx, svf_server_stats_t *stats);
/* Drain the queue, stop the thread, release the server's memory. */
svf_status svf_server_stop(svf_ctx *ctx);

/* ---- kernel timing (for benchmarks): HIP events around every launch of the
 * library's kernels on the caller's stream. ---- */
svf_status svf_set_timing(svf_ctx *ctx, int enable);
/* Sum of event-measured durations (ms) and launch count of one kernel class
 * ("scale_map", "preint", "fd", "batch": a whole batch launch sequence, "st": the structure-tensor
 * gradient and eigenvalue kernels) since the last reset; waits for the recorded events.  reset != 0 clears the accumulators afterwards. */
svf_status svf_kernel_time(svf_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* SVF_H */

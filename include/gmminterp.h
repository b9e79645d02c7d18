/*
 * gmminterp.h -- C ABI of libgmminterp.so: Gaussian-mixture interpolation of
 * scattered points onto a regular H x W grid on an AMD Instinct MI355X (gfx950).
 *
 * Method (Skorokhodov, "Interpolating Points on a Non-Uniform Grid using a
 * Mixture of Gaussians", Section 2, Eq. 1 and Eq. 2): every known point j is an
 * isotropic Gaussian at p_j = (x_j, y_j) carrying a value vector c_j; the value
 * of output pixel i is the posterior mean
 *
 *     out_i = sum_j w_ij c_j / Z_i,   Z_i = sum_j w_ij,
 *     w_ij  = exp(-|g_i - p_j|^2 / (2 sigma_j^2)),
 *
 * where the sums run only over points "close enough" to the pixel (the
 * sentence after Eq. 2), here |g_i - p_j| <= radius * sigma_j, and every
 * channel is interpolated on its own (end of Section 2).  The paper's single
 * shared sigma is the case sigma_per_point = 0; the per-point sigma_j
 * generalises it, with the unnormalised kernel above (identical to Eq. 1 when
 * sigma is shared, since the density's 1/(2 pi sigma^2) cancels).
 *
 * Conventions shared by every entry point:
 *   - Output pixel (row v, column u) sits at (x = u, y = v), pixel units.
 *   - The radius test is inclusive and is evaluated in float32 without fused
 *     multiply-add, exactly as
 *         dx = u - x; dy = v - y; d2 = dx*dx + dy*dy;   (each op rounded)
 *         rs = radius * sigma; R2 = rs*rs;  include iff d2 <= R2.
 *   - A pixel with no point inside the radius (Z = 0) outputs 0 and has no
 *     gradient.
 *   - All tensor pointers are DEVICE pointers to contiguous float32 (or int32)
 *     arrays on the current HIP device; the caller owns every buffer.  Work is
 *     enqueued on `stream` (a hipStream_t; NULL = the default stream) and the
 *     calls return without synchronising and without allocating device memory,
 *     so they may be captured into a HIP graph.
 *   - Errors are reported by return code only; interp_last_error() returns a
 *     thread-local message for the last failing call of the calling thread.
 *     Host-side validation covers shapes, NULL pointers, alignment, sizes and
 *     radius.  Input VALUES (sigma > 0, finite positions) are the caller's
 *     contract: with invalid values the results are undefined but every memory
 *     access stays inside the documented buffers.
 */
#ifndef GMMINTERP_H
#define GMMINTERP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
enum {
  INTERP_OK = 0,
  INTERP_EINVAL = -1,    /* invalid argument (shape, pointer, size, radius) */
  INTERP_ENOMEM = -2,    /* request can never fit the server's memory budget */
  INTERP_EAGAIN = -3,    /* server queue full, try again later */
  INTERP_EHIP = -4,      /* a HIP runtime call failed (message has the HIP error) */
  INTERP_ENOTFOUND = -5  /* unknown server ticket */
};

/* Kernel variants (interp_problem.kernel, flags; 0 is the default kernel).
 *   INTERP_KERNEL_NORMALIZED  each weight keeps the normal density's factor
 *       1/(2 pi sigma_j^2) (diagonal: 1/(2 pi sigma_xj sigma_yj)), as in Eq. 1
 *       with the density N(q | mu_j, Sigma_j); with one shared sigma the factor
 *       cancels and the output equals the default kernel's.
 *   INTERP_KERNEL_DIAGONAL  axis-aligned anisotropic covariance
 *       diag(sigma_x^2, sigma_y^2) in place of sigma^2 I:
 *       w = exp(-(dx^2/sigma_x^2 + dy^2/sigma_y^2) / 2), truncated at
 *       Mahalanobis radius `radius`, decided in float32 without FMA as
 *         ix = 1/sigma_x; iy = 1/sigma_y; qx = dx*ix; qy = dy*iy;
 *         include iff qx*qx + qy*qy <= radius*radius     (each op rounded).
 *       sigma holds (sigma_x, sigma_y) pairs: [B, N, 2] per point or [B, 2]
 *       shared; grad_sigma has the same layout. */
enum { INTERP_KERNEL_NORMALIZED = 1, INTERP_KERNEL_DIAGONAL = 2 };

/* Storage type of the value-carrying arrays (interp_problem.storage):
 * values, out, grad_out and grad_values (and the sorted value records kept
 * from forward to backward) are float32, bfloat16 or IEEE half.  Every sum is
 * taken in float32; out and grad_values are rounded to the storage type once,
 * to nearest even.  Positions, sigmas, Z and their gradients stay float32.
 * Non-float32 storage takes the default kernel (kernel = 0). */
enum { INTERP_STORAGE_F32 = 0, INTERP_STORAGE_BF16 = 1, INTERP_STORAGE_F16 = 2 };

/* Problem shape.
 *   B      images in the batch (>= 1)
 *   N      points per image (>= 0; N = 0 gives an all-zero output)
 *   C      channels per point (1..32)
 *   H, W   output grid (1..32768 each); B*H*W and B*N below 2^31
 *   radius truncation radius in units of sigma, 0 < radius <= 12
 *   tile   side in pixels of the square spatial bins used to find near
 *          points: 4, 8, 16, 32 or 64; 0 selects the default 8
 *   sigma_per_point  1: sigma is [B, N]; 0: one shared sigma per image, [B]
 *          (with INTERP_KERNEL_DIAGONAL: [B, N, 2] and [B, 2])
 *   kernel 0 or INTERP_KERNEL_* flags (above).  The serving path takes
 *          kernel 0 only.
 *   storage INTERP_STORAGE_* (above); the serving path takes float32 only.
 */
typedef struct interp_problem {
  int32_t B, N, C, H, W;
  float radius;
  int32_t tile;
  int32_t sigma_per_point;
  int32_t kernel;
  int32_t storage;
} interp_problem;

/* Bytes of device scratch memory needed by interp_forward / interp_backward
 * for this problem (the same buffer may serve both).  0 if the problem is
 * invalid (the reason is in interp_last_error()). */
size_t interp_workspace_bytes(const interp_problem* prob);

/* Bytes of the state interp_forward leaves for interp_backward: the
 * normaliser Z [B,H,W] (float), the per-image neighbour reach, the bin
 * offsets, the binning permutation and the bin-sorted point records.
 * 0 if the problem is invalid. */
size_t interp_saved_bytes(const interp_problem* prob);

/* Forward pass (Eq. 1 and Eq. 2).
 *   pos     [B, N, 2] float32 (x = column, y = row), 8-byte aligned
 *   sigma   [B, N] or [B] float32 (see sigma_per_point), sigma > 0
 *   values  [B, N, C] float32
 *   out     [B, C, H, W] float32, written in full
 *   saved   interp_saved_bytes() bytes, 256-byte aligned, written; must be
 *           kept unchanged for interp_backward.  Required (not NULL).
 *   workspace  interp_workspace_bytes() bytes, 256-byte aligned
 * The *_size arguments are the byte sizes of the given buffers; a buffer
 * smaller than required is EINVAL.  pos/sigma/values may be NULL when N = 0.
 * Work is done by HIP kernels on `stream`; results are deterministic (the
 * per-pixel summation order is fixed by the stable bin order). */
int interp_forward(const interp_problem* prob, const float* pos, const float* sigma,
                   const float* values, float* out, void* saved, size_t saved_size,
                   void* workspace, size_t workspace_size, void* stream);

/* Forward pass without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, results and errors as
 * interp_forward, but the workspace is the library's own static scratch: a
 * device array of INTERP_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, reserved
 * when the library's code is loaded onto that GPU and held until the process
 * ends.  No hipMalloc/hipFree and no other allocating call is made (the
 * interp_profile_* hooks do not record this call's kernels).
 *   out, saved   as for interp_forward (caller-allocated outputs; saved may
 *                then go to interp_backward with a caller workspace)
 * EINVAL if the problem's forward workspace exceeds the scratch (the message
 * gives both sizes); nothing is launched then.  The first call on a device
 * looks up that device's copy of the scratch (the stream must belong to the
 * current device).  Every call on one GPU shares that GPU's scratch: calls
 * that overlap in time on one GPU (different streams or threads) race and
 * give undefined results; calls ordered on one stream are safe.  The
 * scratch keeps the last call's contents; everything the forward needs
 * zeroed is cleared by its own kernels. */
#define INTERP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int interp_forward_noalloc(const interp_problem* prob, const float* pos, const float* sigma,
                           const float* values, float* out, void* saved, size_t saved_size,
                           void* stream);

/* Backward pass: gradients of a scalar loss L given grad_out = dL/d out.
 *   pos, sigma, values, out, saved   exactly as given to / produced by the
 *                                    matching interp_forward call
 *   grad_out     [B, C, H, W] float32
 *   grad_pos     [B, N, 2] float32 or NULL (not computed)
 *   grad_sigma   [B, N] (per point) or [B] (shared: the sum over the image's
 *                points) float32, or NULL
 *   grad_values  [B, N, C] float32 or NULL
 * Gradients are overwritten, not accumulated.  Formulas (quotient rule on
 * Eq. 1, alpha_i = 1/Z_i, beta_i = alpha_i sum_k G_ik out_ik):
 *   dL/dc_jk = sum_i w_ij alpha_i G_ik
 *   A_ij = alpha_i sum_k G_ik c_jk - beta_i
 *   dL/dx_j = sum_i A_ij w_ij (u_i - x_j) / sigma_j^2   (y likewise)
 *   dL/dsigma_j = sum_i A_ij w_ij d2_ij / sigma_j^3
 * over the pixels inside the radius (the indicator's jump is not
 * differentiated).  Deterministic. */
int interp_backward(const interp_problem* prob, const float* pos, const float* sigma,
                    const float* values, const float* out, const void* saved, size_t saved_size,
                    const float* grad_out, float* grad_pos, float* grad_sigma, float* grad_values,
                    void* workspace, size_t workspace_size, void* stream);

/* Binning state left by interp_forward, for bit-exact checks of the spatial
 * counting sort.  Copies into caller device buffers:
 *   bin_of  [B, N] int32  bin of each point: by * ceil(W/tile) + bx with
 *           bx = clamp(floor(x / tile), 0, ceil(W/tile) - 1), by likewise
 *   count   [B, nb] int32 points per bin, nb = ceil(H/tile) * ceil(W/tile)
 *   offset  [B, nb + 1] int32 exclusive prefix sum of count (offset[nb] = N)
 *   perm    [B, N] int32  stable sort order: by bin, ties by point index
 * Any output may be NULL.  workspace/saved must be the ones of the forward
 * call, unchanged since. */
int interp_debug_bins(const interp_problem* prob, const void* saved, size_t saved_size,
                      const void* workspace, size_t workspace_size, int32_t* bin_of,
                      int32_t* count, int32_t* offset, int32_t* perm, void* stream);

/* Thread-local message describing the last error of this thread ("" if none). */
const char* interp_last_error(void);

/* Measurement hooks for benchmarks.  While enabled, every kernel the library
 * launches outside HIP graph capture is bracketed by a pair of HIP events on
 * the stream it is launched on.  interp_profile_enable(1) also clears the
 * previous records; interp_profile_enable(0) stops recording.
 * interp_profile_read waits for the recorded kernels and returns, summed over
 * the kernels whose name starts with `prefix` ("" for all), the total
 * duration in milliseconds and the number of launches.  Kernel names:
 * bin_keys, radix_hist, radix_scan, radix_scatter, bin_finish, fwd_plan,
 * forward, bwd_pixel, bwd_point, bwd_sigma_sum. */
int interp_profile_enable(int on);
int interp_profile_read(const char* prefix, double* total_ms, int64_t* launches);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent interpolation requests.
 *
 * A server owns one device arena of hbm_budget_bytes (allocated once at
 * creation), a device job table and a scheduler thread.  Requests are
 * admitted in arrival order as job slots and arena memory free up; each
 * scheduling round packs every admitted job into one replay of a captured
 * HIP graph of job-table kernels (binning, forward, backward), so the work of
 * requests of different sizes and channel counts overlaps on the device.
 * Each request's result equals that of interp_forward / interp_backward on
 * the same inputs (the kernels and summation order are the same).
 * ---------------------------------------------------------------------- */

typedef struct interp_server interp_server;

typedef struct interp_server_config {
  int32_t device;             /* HIP device ordinal */
  int32_t max_slots;          /* jobs resident at once (1..1024) */
  int32_t max_queue;          /* pending requests beyond which submit is EAGAIN */
  int32_t reserved;
  uint64_t hbm_budget_bytes;  /* arena size for all per-job device state */
} interp_server_config;

/* One request: a problem with B = 1 and device pointers that must stay valid
 * until the request is DONE or FAILED.  grad_out == NULL: forward only;
 * otherwise the backward runs too and writes the non-NULL grad_* outputs.
 * ready: a hipEvent_t recorded by the caller after the work that produces
 * the inputs (and last used the output buffers), or NULL.  The batch that
 * runs the request waits for it on the device before it reads or writes any
 * of the request's buffers; the event must stay valid until the request is
 * DONE or FAILED.  With NULL the inputs must already be complete. */
typedef struct interp_request {
  interp_problem prob;
  const float* pos;
  const float* sigma;
  const float* values;
  float* out;
  const float* grad_out;
  float* grad_pos;
  float* grad_sigma;
  float* grad_values;
  void* ready;
} interp_request;

enum { INTERP_QUEUED = 0, INTERP_RUNNING = 1, INTERP_DONE = 2, INTERP_FAILED = 3 };

typedef struct interp_status {
  int32_t state;              /* INTERP_QUEUED / RUNNING / DONE / FAILED */
  int32_t err;                /* INTERP_* code when FAILED */
  int64_t t_submit_ns;        /* CLOCK_MONOTONIC times */
  int64_t t_admit_ns;
  int64_t t_done_ns;
} interp_status;

/* Create a server (allocates the arena, job table, streams and graph
 * resources, starts the scheduler thread). */
int interp_server_create(const interp_server_config* cfg, interp_server** out);

/* Non-blocking submit.  ENOMEM if the request can never fit the budget,
 * EAGAIN if max_queue requests are pending, EINVAL for a bad request (B must
 * be 1 and C at most 4 on the serving path).  The server's streams are
 * ordered after the caller's work only through req->ready (see above).  On
 * success *ticket identifies the request. */
int interp_submit(interp_server* s, const interp_request* req, uint64_t* ticket);

/* Non-blocking submit of n requests in one call, queued in array order.
 * Every request is checked first: EINVAL (naming the request's index) when
 * one is invalid, and then none is queued.  Otherwise the requests are queued
 * in order until one cannot be (ENOMEM: it can never fit the budget; EAGAIN:
 * the queue is full), whose code is returned; *n_queued counts the requests
 * queued (tickets[0 .. *n_queued) identify them; the rest are not queued and
 * may be submitted again).  reqs: n requests as for interp_submit; tickets:
 * room for n tickets (host memory, the caller's).  One call takes the
 * server's lock once, so a client with many requests at hand does not pay a
 * submit per request. */
int interp_submit_many(interp_server* s, const interp_request* reqs, int32_t n, uint64_t* tickets,
                       int32_t* n_queued);

/* Non-blocking status query.  ENOTFOUND for an unknown ticket.  A ticket is
 * forgotten after a poll that returns DONE or FAILED. */
int interp_poll(interp_server* s, uint64_t ticket, interp_status* status);

/* Block until every submitted request is DONE or FAILED (or timeout_ms passes,
 * then EAGAIN; timeout_ms < 0 waits forever). */
int interp_server_drain(interp_server* s, int64_t timeout_ms);

/* Stop the scheduler: requests still queued become FAILED (EAGAIN), running
 * ones are finished, then every device resource is released. */
int interp_server_destroy(interp_server* s);

#ifdef __cplusplus
}
#endif

#endif /* GMMINTERP_H */

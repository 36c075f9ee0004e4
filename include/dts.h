/*
 * dts.h -- C ABI of libdts, the gfx950 (MI355X) hot path of the Domain Transform Solver.
 *
 * Method: A. Bapat and J.-M. Frahm, "The Domain Transform Solver", ECCV 2018
 * (arXiv:1805.04590).  Equation numbers count the paper's displayed equations in order:
 * Eq. (2) objective without the application term, Eq. (3) its gradient (the descent
 * direction), Eq. (6) the bilateral solver's per-pixel solution, Eq. (7) the variance
 * confidence, Eq. (8)-(9) the domain transform, Eq. (10) the edge-aware mean, Eq. (11)
 * the stereo objective.
 *
 * Conventions shared by every entry point
 *   - Every array pointer is a DEVICE pointer (memory of the current HIP device), fp32,
 *     planar row-major: guide [batch][Cg][H][W]; target, output and gradients
 *     [batch][Ct][H][W]; confidence [batch][Cc][H][W] with Cc = 1 (shared by all target
 *     channels) or Cc = Ct.
 *   - The caller owns every buffer, including the workspace, whose size it obtains from
 *     the matching *_workspace_bytes call.  The library allocates nothing and keeps no
 *     state between calls; a workspace must not be used by two calls that may run at the
 *     same time.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only enqueues
 *     work on it and returns without synchronising, so calls may be captured into a HIP
 *     graph.  Inputs are never written; outputs must not alias inputs unless the entry
 *     point says so.
 *   - Return value: DTS_OK (0) or a negative error code; nothing is enqueued when an
 *     argument check fails.  Values are not range-checked: NaN and Inf propagate.
 *   - Device-side failures (a bounded wait inside a kernel that timed out) set a flag in
 *     the workspace; dts_workspace_status() reads it back.
 */
#ifndef DTS_H
#define DTS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DTS_OK 0
#define DTS_EINVAL (-1)     /* null pointer, bad size, channel count, sigma, N or T      */
#define DTS_EWORKSPACE (-2) /* workspace null or smaller than *_workspace_bytes          */
#define DTS_EHIP (-3)       /* a HIP runtime call or kernel launch failed                */
#define DTS_ENOTSUP (-4)    /* shape beyond the supported limits (see DTS_MAX_*)         */
#define DTS_EDEVICE (-5)    /* a kernel reported a device-side failure (status call)     */

#define DTS_MAX_CHANNELS 16 /* Cg, Ct <= 16: the paper motivates 16-band imagery (Sec. 1) */
#define DTS_MAX_WIDTH 16384  /* row pass: at most 16 waves x 64 lanes x 16 pixels per row */
#define DTS_MAX_HEIGHT 32768

/* Solver parameters (Sec. 3.1 and Sec. 4).  sigma_s is the spatial standard deviation
 * in pixels (sigma_x = sigma_y), sigma_r the range standard deviation in guide units;
 * filter_iters N >= 1 domain-transform iterations per edge-aware mean (each a row pass
 * then a column pass); solver_iters T >= 0 gradient-descent iterations; lambda weighs the
 * edge-aware regulariser and step scales the Eq. (3) direction (both 0.99 in the paper). */
typedef struct dts_params {
    float sigma_s;
    float sigma_r;
    int filter_iters;
    int solver_iters;
    float lambda;
    float step;
} dts_params;

/* Workspace sizes in bytes (always a multiple of 256). */
size_t dts_filter_workspace_bytes(int batch, int H, int W, int Cs);
size_t dts_solve_workspace_bytes(int batch, int H, int W, int Ct, const dts_params* p);
size_t dts_solve_backward_workspace_bytes(int batch, int H, int W, int Cg, int Ct,
                                          const dts_params* p);

/* dts_filter -- the 2-D domain-transform edge-aware filter DT(src) (Sec. 3.2, Eq. (8)-(10)
 * in its recursive-filter form).  Distances from the guide's channel differences
 *   dx = sqrt(1 + (sigma_s/sigma_r)^2 sum_k (I_k[y][x] - I_k[y][x-1])^2)   (dy likewise),
 * weights w = a_i^d with a_i = exp(-sqrt(2)/sigma_Hi), sigma_Hi = sigma_s sqrt(3)
 * 2^(N-i) / sqrt(4^N - 1); then for i = 1..N a causal+anticausal recursive pass along
 * every row, then along every column.  All Cs channels of src use the same weights.
 * guide [batch][Cg][H][W], src/dst [batch][Cs][H][W]; dst may equal src (in place). */
int dts_filter(const float* guide, int Cg, const float* src, float* dst, int Cs, int batch,
               int H, int W, float sigma_s, float sigma_r, int filter_iters, void* workspace,
               size_t workspace_bytes, void* stream);

/* dts_solve -- gradient descent along Eq. (3) on the objective of Eq. (2):
 *   z^0 = target,  z^{k+1} = z^k - step (lambda (z^k - DT(z^k)) + c (z^k - target)),
 * k = 0..T-1, writing z^T to `out` [batch][Ct][H][W].  `checkpoints` is NULL or an array
 * of T slots [T][batch][Ct][H][W]; slot k receives z^k (slot 0 a copy of the target),
 * which is what dts_solve_backward reads.  T = 0 copies the target to `out`. */
int dts_solve(const float* guide, int Cg, const float* target, const float* conf, int Cc,
              int Ct, int batch, int H, int W, const dts_params* p, float* out,
              float* checkpoints, void* workspace, size_t workspace_bytes, void* stream);

/* dts_solve_noalloc -- dts_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, hosts that forbid allocation): the same
 * arguments and results as dts_solve without a workspace.  The workspace dts_solve
 * would need (dts_solve_workspace_bytes) lives instead in a 64 MiB scratch array that
 * the library holds on every device it runs on until the process ends, so the call
 * allocates nothing.  Returns DTS_ENOTSUP when dts_solve_workspace_bytes exceeds
 * 64 MiB (67108864 bytes; e.g. a 1-channel 2048 x 2048 or 3-channel 1920 x 1080 solve fits,
 * a 1-channel 2400 x 2400 one does not).
 * All calls on one device share that array: calls that may overlap on one device (other
 * streams, other threads) race and must be serialised by the caller.  The array keeps
 * the last call's contents; each call clears what must start at zero.  A device-side
 * failure flag (see dts_workspace_status) lands in the shared array and is not reported:
 * callers that need it use dts_solve with their own workspace. */
int dts_solve_noalloc(const float* guide, int Cg, const float* target, const float* conf, int Cc,
                      int Ct, int batch, int H, int W, const dts_params* p, float* out,
                      float* checkpoints, void* stream);

/* dts_solve_backward -- reverse-mode gradient of a scalar loss through dts_solve (not in
 * the paper; derived from Eq. (3) and the filter by the chain rule).  Given
 * grad_out = dL/dz^T and the T checkpoints written by dts_solve with the same inputs, it
 * writes dL/dtarget [batch][Ct][H][W], dL/dconf [batch][Cc][H][W] (summed over the target
 * channels when Cc = 1) and dL/dguide [batch][Cg][H][W].  Each gradient pointer may be
 * NULL to skip it (the guide gradient costs one extra accumulation per filter pass).
 * Per iteration the filter's pass inputs are recomputed from the checkpoint. */
int dts_solve_backward(const float* guide, int Cg, const float* target, const float* conf,
                       int Cc, int Ct, int batch, int H, int W, const dts_params* p,
                       const float* checkpoints, const float* grad_out, float* grad_target,
                       float* grad_conf, float* grad_guide, void* workspace,
                       size_t workspace_bytes, void* stream);

/* dts_solve and dts_solve_backward trading memory for the backward's recomputation (the
 * store-or-recompute choice of reverse mode; not in the paper).  dts_solve_tape is
 * dts_solve that also keeps, for every iteration k < T, the outputs of the first 2N - 1
 * of its 2N filter passes (N = filter_iters) in tape [T][2N-1][batch][Ct][H][W]; they go
 * there instead of into the workspace, so the forward moves the same bytes.
 * checkpoints and tape are required when T > 0 (DTS_EINVAL otherwise).
 * dts_solve_backward_tape is dts_solve_backward reading those pass inputs from tape
 * instead of recomputing them from the checkpoints (2N - 1 passes per iteration fewer);
 * its gradients are bitwise those of dts_solve_backward.  Workspaces as for dts_solve and
 * dts_solve_backward. */
int dts_solve_tape(const float* guide, int Cg, const float* target, const float* conf, int Cc, int Ct,
                   int batch, int H, int W, const dts_params* p, float* out, float* checkpoints, float* tape,
                   void* workspace, size_t workspace_bytes, void* stream);
int dts_solve_backward_tape(const float* guide, int Cg, const float* target, const float* conf, int Cc,
                            int Ct, int batch, int H, int W, const dts_params* p, const float* checkpoints,
                            const float* tape, const float* grad_out, float* grad_target, float* grad_conf,
                            float* grad_guide, void* workspace, size_t workspace_bytes, void* stream);

/* ---- Stereo refinement (Eq. (11), Sec. 3.3) ---- */

/* Workspace for dts_solve_stereo (0 if the shape is invalid). */
size_t dts_solve_stereo_workspace_bytes(int batch, int H, int W);

/* Disparity refinement of Eq. (11): the edge-aware smoothness of Eq. (2) guided by the left
 * image, a Charbonnier target term c rho(z - t) with rho(r) = sqrt(r^2 + epsilon^2), and
 * the photometric term gamma/2 sum_k (I_L,k(x) - I_R,k(x - z))^2 of a rectified pair.
 * Gradient descent with the edge-aware mean held fixed, as for dts_solve:
 *   z^0 = init (the target t if init is NULL),
 *   z^{k+1} = z^k - step (lambda (z^k - DT(z^k)) + D(z^k)),
 *   D = c rho'(z - t) + gamma sum_k (I_L,k - I_R,k(x - z)) dI_R,k/dx (x - z).
 * Disparities are in pixels: left pixel (x, y) matches the right image at (x - z, y),
 * read linearly along the row, the position clamped to [0, W - 1] (slope 0 where
 * clamped).  left, right [batch][Cg][H][W]; target, conf, out [batch][1][H][W]; p gives
 * sigma_s, sigma_r, filter_iters, solver_iters (T = 0 copies z^0), lambda, step.
 * init is NULL or [batch][1][H][W] (restarting a descent from a given iterate: the data
 * term keeps using the target).  gamma >= 0, epsilon > 0 (Sec. 4 uses 0.001 for both).
 * out must not alias target, conf, init or the images.  Errors as dts_solve. */
int dts_solve_stereo(const float* left, const float* right, int Cg, const float* target, const float* conf,
                     const float* init, int batch, int H, int W, const dts_params* p, float gamma, float epsilon,
                     float* out, void* workspace, size_t workspace_bytes, void* stream);

/* ---- Variance-based confidence (Eq. (7), Sec. 3.1) ---- */

/* Workspace for dts_variance_confidence (0 if the arguments are invalid). */
size_t dts_variance_confidence_workspace_bytes(int batch, int H, int W, int C);

/* Confidence from the edge-aware variance of z (Eq. (7)): V = DT(z^2) - DT(z)^2 with DT the
 * same domain-transform mean dts_filter computes (guide, sigma_s, sigma_r, filter_iters),
 * and conf = exp(-V / (2 sigma_c^2)), per channel.  z [batch][C][H][W] (1 <= C <= 8),
 * conf the same shape; conf may alias z.  V is used as computed: rounding can make it
 * slightly negative and conf slightly above 1.  The pairs (z, z^2) are filtered
 * together: the squaring happens in the first row pass and the workspace holds the 2C
 * filtered planes.  Errors as dts_filter; sigma_c must be finite and positive. */
int dts_variance_confidence(const float* guide, int Cg, const float* z, float* conf, int C, int batch,
                            int H, int W, float sigma_s, float sigma_r, int filter_iters, float sigma_c,
                            void* workspace, size_t workspace_bytes, void* stream);

/* ---- Box form of the edge-aware mean (Sec. 3.2, Eq. (10) as written) ---- */

/* Workspace for dts_filter_box / dts_solve_box with C signal channels and filter_iters
 * iterations (0 if the arguments are invalid). */
size_t dts_box_workspace_bytes(int batch, int H, int W, int C, int filter_iters);

/* Integer codes of the arc-length increments that decide box membership:
 * q = rint(256 d) with d = sqrt(1 + s2 sum_k (I_k[n] - I_k[n-1])^2) evaluated in float32,
 * every operation rounded to nearest, bands summed in order, s2 = (sigma_s/sigma_r)^2
 * rounded to float32; capped at 65536.  qx, qy: device arrays of batch*H*W uint32;
 * qx[..][0] and qy[..][0][..] are 0 (no pixel before them).  Errors as dts_distances. */
int dts_box_codes(const float* guide, int Cg, int batch, int H, int W, float sigma_s, float sigma_r,
                  unsigned int* qx, unsigned int* qy, void* stream);

/* Edge-aware mean with the box kernel that Eq. (10) writes: along a line, the mean of the
 * samples j with |ct_i - ct_j| <= R_i, where ct is the running sum of the codes of
 * dts_box_codes and R_i = floor(256 sqrt(3) sigma_Hi) is the box with the variance of
 * the recursive filter's iteration i (sigma_Hi as for dts_filter).  filter_iters (<= 8)
 * iterations, each along rows then columns, on every channel of src with the same boxes.
 * Layouts and aliasing as dts_filter.  Returns DTS_ENOTSUP when R_1 / 256 exceeds 255 pixels
 * (sigma_s above about 169 for N = 3) or its column ring exceeds the device's LDS. */
int dts_filter_box(const float* guide, int Cg, const float* src, float* dst, int C, int batch, int H, int W,
                   float sigma_s, float sigma_r, int filter_iters, void* workspace, size_t workspace_bytes,
                   void* stream);

/* dts_solve with the box form of the edge-aware mean: z^0 = t,
 * z^{k+1} = z^k - step (lambda (z^k - BOX(z^k)) + c (z^k - t)).  Arguments as dts_solve
 * without checkpoints; filter_iters <= 8; limits as dts_filter_box. */
int dts_solve_box(const float* guide, int Cg, const float* target, const float* conf, int Cc, int Ct, int batch,
                  int H, int W, const dts_params* p, float* out, void* workspace, size_t workspace_bytes,
                  void* stream);

/* ---- Support-weighted confidence (Sec. 3.1, after Eq. (6)) ---- */

/* Workspace for dts_support (0 if the shape is invalid). */
size_t dts_support_workspace_bytes(int batch, int H, int W);

/* Support of the edge-aware kernel, s_i = sum_j W_ij relative to a flat region, and
 * optionally the confidence weighted by it, conf_out = conf / s.  Sec. 3.1 divides the
 * confidence of the descent update by this support, as in the bilateral solver's
 * per-pixel solution (Eq. (6)).  W is read as the unnormalised domain-transform kernel:
 * each 1-D pass sums products of the weights a_i^d over both sides of a pixel, the pixel
 * counted once, and passes alternate rows and columns over filter_iters iterations
 * (guide, sigma_s, sigma_r as for dts_filter).  Each pass is scaled by
 * (1 - a_i) / (1 + a_i), so s is 1 deep inside a flat region and lies in (0, 1].
 * support [batch][H][W].  conf [batch][Cc][H][W] (1 <= Cc <= 16) and conf_out (same shape)
 * may be NULL together; conf_out may alias conf but neither may alias support.  The
 * support depends on the guide only: compute it once per guide.  Errors as dts_filter;
 * its column passes use the filter's chunked carry exchange, so a bounded wait that
 * gives up flags the workspace status (dts_workspace_status). */
int dts_support(const float* guide, int Cg, int batch, int H, int W, float sigma_s, float sigma_r,
                int filter_iters, float* support, const float* conf, int Cc, float* conf_out, void* workspace,
                size_t workspace_bytes, void* stream);

/* ---- Many uneven solves in one persistent launch ---- */

/* One independent solve: device pointers, shape and parameters (1 <= T, 1 <= N <= 8,
 * W <= 4096; at most DTS_BATCH_MAX_PROBLEMS per batch).  Layouts as above with batch 1. */
#define DTS_BATCH_MAX_PROBLEMS 1024
typedef struct dts_problem {
    const float* guide;
    const float* target;
    const float* conf;
    float* out;
    int H, W, Cg, Ct, Cc;
    float sigma_s, sigma_r;
    int filter_iters, solver_iters;
} dts_problem;

/* Filled by dts_batched_prepare, read by dts_solve_batched (host memory, plain data). */
typedef struct dts_batched_plan {
    int n, variant, n_phases, total_tiles, grid;
    float lambda, step;
    size_t workspace_bytes;
    size_t off_inst, off_prefix, off_tickets;
} dts_batched_plan;

/* Launch shapes of the batched kernel: rows per wave of the column chunks, target
 * channels per column group, and the size of a row tile (pixels x channels it aims
 * for).  The autotuner of the Python package picks one. */
int dts_batched_variant_count(void);
int dts_batched_variant_info(int variant, int* rows_per_wave, int* group_channels,
                             int* row_tile_pixels);
size_t dts_batched_workspace_bytes(const dts_problem* probs, int n, int variant);

/* Writes the instance table and the tile schedule for `probs` (host array of n problems)
 * into the workspace and waits for the copy on `stream`: call it outside graph capture.
 * The problems' device buffers must stay valid while the plan is used. */
int dts_batched_prepare(const dts_problem* probs, int n, float lambda, float step, int variant,
                        void* workspace, size_t workspace_bytes, dts_batched_plan* plan, void* stream);

/* Runs every planned solve (not in the paper; each instance is exactly what dts_solve
 * computes): one small reset kernel and one persistent kernel with one workgroup per
 * resident slot of the device.  The workgroups run the passes of all instances in
 * lockstep (pass p of every instance, a grid barrier, pass p + 1, ...), taking the row
 * and column tiles of a pass from a device-side ticket counter.  The kernel needs the
 * whole device: work running concurrently on other streams can delay the barriers,
 * which give up after a bounded wait and then make dts_workspace_status return
 * DTS_EDEVICE.  Allocates and copies nothing, so it can be captured into a HIP
 * graph and replayed; calls sharing one workspace must not overlap. */
int dts_solve_batched(const dts_batched_plan* plan, void* workspace, void* stream);

/* ---- The individual steps of the filter (each also runs inside the calls above) ---- */

/* dts_distances -- transformed distances of the domain transform (Sec. 3.2, Eq. (8)-(9)):
 *   dx[b][y][x] = sqrt(1 + (sigma_s/sigma_r)^2 sum_k (I_k[y][x] - I_k[y][x-1])^2), x >= 1,
 *   dy[b][y][x] = sqrt(1 + (sigma_s/sigma_r)^2 sum_k (I_k[y][x] - I_k[y-1][x])^2), y >= 1,
 * and 1 at x = 0 (dx) and y = 0 (dy).  guide [batch][Cg][H][W]; dx, dy [batch][H][W]. */
int dts_distances(const float* guide, int Cg, int batch, int H, int W, float sigma_s,
                  float sigma_r, float* dx, float* dy, void* stream);

/* Workspace of one dts_col_pass call. */
size_t dts_pass_workspace_bytes(int batch, int H, int W, int C);

/* dts_row_pass / dts_col_pass -- one causal+anticausal recursive pass of filter iteration
 * `iter` (1..N) along every row (weights a_iter^dx) or every column (a_iter^dy):
 *   J[0] = f[0], J[n] = (1 - w[n]) f[n] + w[n] J[n-1];
 *   K[L-1] = J[L-1], K[n] = (1 - w[n+1]) J[n] + w[n+1] K[n+1];  dst = K.
 * src/dst [batch][C][H][W] (dst may equal src); dx or dy [batch][H][W] from dts_distances. */
int dts_row_pass(const float* src, float* dst, const float* dx, int C, int batch, int H, int W,
                 float sigma_s, int iter, int filter_iters, void* stream);
int dts_col_pass(const float* src, float* dst, const float* dy, int C, int batch, int H, int W,
                 float sigma_s, int iter, int filter_iters, void* workspace,
                 size_t workspace_bytes, void* stream);

/* ---- Launch-shape tuning (process-wide; set before enqueuing work) ---- */

/* The column pass runs in one of several workgroup shapes per channel-group size (a
 * group is up to 4 target channels processed together): rows per wave x waves per
 * workgroup, a chunk of rows per workgroup.  Variants differ only in speed; results agree
 * to fp32 rounding.  info() returns DTS_EINVAL for an unknown index. */
int dts_col_variant_count(void);
int dts_col_variant_info(int variant, int* group_channels, int* rows_per_wave, int* waves);
/* Pin `variant` for channel groups of `group_channels` (1..4); -1 restores the default. */
int dts_tune_col_variant(int group_channels, int variant);
/* on != 0 (the default): the persistent column passes keep all chunks of a strip on one
 * XCD (workgroups are dealt to the 8 XCDs in turn), so the carry words a chunk waits for
 * are written from its own XCD; 0: chunk p % G of strip group p / G.  Results agree to
 * fp32 rounding. */
int dts_tune_col_xcd(int on);
/* Bounded waits of the column passes' carry exchange (also inside dts_solve_batched).
 * polls > 0: a wait gives up after about this many polls (default 2^21, each followed by
 * a short sleep), flags DTS_EDEVICE in the workspace status and lets its kernel finish;
 * 0 restores the default.  polls < 0 exercises that failure path: the waits look for a
 * tag that no kernel writes and give up after -polls polls, so every call with carries to
 * exchange (a column pass over more than one chunk) completes and reports DTS_EDEVICE;
 * its results are not defined.  Process-wide; set it before enqueuing work. */
int dts_tune_spin_limit(int polls);
/* Pixels per lane of the row pass: 4, 8 or 16; 0 restores the default, which depends on
 * the row width.  Rows whose width needs more than 16 waves at this setting fall back to
 * the default. */
int dts_tune_row_segment(int pixels_per_lane);
/* Column passes of the box kernel (dts_filter_box, dts_solve_box): on != 0 (the default)
 * runs a pass whose half-width h is at most 64 pixels as one kernel over a window of rows
 * in LDS; 0 takes the kernels used for wider boxes (a block prefix in the workspace and a
 * gather, or a ring down each column with the solver update) for every h.  Results agree
 * to fp32 rounding. */
int dts_tune_box_window(int on);

/* ---- Kernel timing (HIP events around each launch, on the launch's own stream) ---- */

/* One row of the timing table: a kernel variant, how many launches were recorded, their
 * summed duration and the algorithmic bytes those launches must move (inputs read once,
 * outputs written once, fp32). */
typedef struct dts_kernel_stat {
    char name[48];
    int launches;
    double total_ms;
    double bytes;
} dts_kernel_stat;

/* on != 0 clears the table and starts recording every launch of this process; on == 0
 * stops.  Not for use while a stream is being captured into a graph. */
int dts_profile_enable(int on);

/* Waits for the recorded launches, fills up to `max_rows` rows and returns the number of
 * kernel variants recorded (or a negative error code). */
int dts_profile_read(dts_kernel_stat* rows, int max_rows);

/* Reads back (synchronously, on `stream`) the device-side status flag of a workspace,
 * which every call clears when it starts: DTS_OK, or DTS_EDEVICE if a kernel of the most
 * recent call on this workspace reported a failure (a bounded wait that timed out, a work
 * ticket out of range).  The flag is cleared after it is read. */
int dts_workspace_status(void* workspace, void* stream);

/* Human-readable text of an error code (static storage). */
const char* dts_strerror(int code);

/* Text of the last HIP error seen by this thread (static thread-local storage). */
const char* dts_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DTS_H */

/*
 * slr.h -- C ABI of the spherical LiDAR surfel rasterizer (MI355X / gfx950).
 *
 * Differentiable rasterization of 2D Gaussian surfels into a spherical
 * (azimuth / elevation) range image, as in Splat-LOAM (Giacomini et al.,
 * arXiv 2503.17491): forward gives range D, normal N and opacity O per pixel
 * (Sec. 3.2.1, Eqs. ab_depth / ab_normal / ab_opacity), backward gives the
 * gradients of a loss w.r.t. the raw surfel parameters and w.r.t. the sensor
 * pose in se(3) (Supp. D "Gradient Computation"; pose update of Sec. 3.3.3).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Sensor model (Sec. 3.1, Supp. A): azimuth az = atan2(y, x), elevation
 *   el = atan2(z, sqrt(x^2 + y^2)); image coordinates u = fu*az + cu,
 *   v = fv*el + cv.  Pixel (i, j) (row, column) looks along the ray of
 *   (u, v) = (j + 1/2, i + 1/2).  The azimuth wraps with period 2*pi*|fu|
 *   pixels.  Sensor axes: x forward, y left, z up.
 * - Surfel raw parameters (Sec. 3.2): mean mu [3], quaternion (w, x, y, z)
 *   [4] (normalised inside; rotation columns t_alpha, t_beta, t_n), log-scales
 *   [2] (s = exp), opacity logit [1] (o = sigmoid).  FP32, row-major, device.
 * - Pose: T_cw (world -> sensor) as a row-major 4x4 FP64 matrix in DEVICE
 *   memory.  The pose gradient is w.r.t. delta = (rho; phi) in se(3) for
 *   T_cw(delta) = exp(-delta^) T_cw, i.e. the sensor pose update
 *   T_wc <- T_wc exp(delta) of Sec. 3.3.3; rho first.
 * - Compositing (Sec. 3.2.1, following the 3DGS blending it cites): a pair
 *   contributes when the ray meets the 3-sigma square |s_alpha|, |s_beta| <= 3
 *   in front of the near range, alpha = min(0.99, o G(s_hat)) >= 1/255, and
 *   the running transmittance would not drop below 1e-4.  Per-tile lists are
 *   ordered by the FP32 rounding of the centre range |R_cw mu + t_cw| and then
 *   by surfel index.  Outputs are the raw Eq. 4-6 sums (D/O is the expected
 *   range of the hit surface).
 * - Ownership: the caller owns every buffer (inputs, outputs, workspace).  The
 *   library allocates no device memory and keeps no device state between
 *   calls other than what it writes into the caller's workspace.  All device
 *   work is enqueued on the caller's HIP stream (hipStream_t passed as void*;
 *   NULL = the default stream).
 * - Errors: every call validates its arguments on the host before enqueuing
 *   anything and returns a negative status; slr_last_error() gives a
 *   thread-local message.  Gradient outputs are overwritten unless the
 *   caller asks for accumulation.
 */
#ifndef SLR_H
#define SLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t slr_status;
#define SLR_OK 0
#define SLR_E_INVALID (-1)     /* bad argument; nothing was enqueued */
#define SLR_E_CAPACITY (-2)    /* more (tile, surfel) pairs than the workspace holds */
#define SLR_E_HIP (-3)         /* a HIP runtime call failed */
#define SLR_E_UNSUPPORTED (-4) /* a valid request this build does not implement */

/* Spherical sensor: image size and the camera matrix K of Supp. A. */
typedef struct slr_sensor {
    int32_t height, width; /* rows (elevation), columns (azimuth); each in [1, 32767]
                              and 3 * height * width < 2^31 */
    double fu, cu, fv, cv; /* u = fu*az + cu, v = fv*el + cv; fu, fv must be < 0 */
    double near_m;         /* pairs with ray range t <= near_m are rejected, and
                              surfels whose centre range <= near_m are culled */
} slr_sensor;

/* Tile shape of the binning (Sec. 3.2.1 uses 16x16).  tile_h * tile_w must be
 * 256; supported shapes: 16x16, 8x32, 32x8, 4x64; a frame may have at most
 * 65535 tiles.  variant selects how the
 * forward compositing kernel reads a tile's surfel records: 0 = library
 * default, 1 = staged through LDS in batches by the whole workgroup, 2 = each
 * wave reads them through the scalar cache (no LDS, no workgroup barrier),
 * 3 = one workgroup of one wave per 64-pixel strip of the tile, records read
 * one per lane and shared through LDS (no workgroup barrier).
 * schedule selects the order in which the compositing kernels take tiles:
 * 0 = library default, 1 = tile-id order, 2 = longest surfel list first
 * (computed on the device after binning), 3 = the same order taken from a
 * device work queue by the one-wave forward (variant 3) and the workgroup
 * backward (bwd_variant 1 or 4), which then run as persistent kernels: as many
 * workgroups as the device holds at once, each taking the next item (strip
 * or tile) until none is left (the other kernels behave as with 2; results
 * identical to 2).  bwd_variant selects the form of
 * the compositing backward: 0 = the same as variant (the library default if
 * that is 0), 1 = one workgroup per tile (records staged through LDS, one
 * flush per tile and record), 3 = one wave per 64-pixel strip, 4 = the
 * fixed-order (deterministic) form of 1: the four waves' sums of a record
 * added in wave order, each (tile, record) flush written with plain stores
 * to a slot of its own (no floating-point atomics) and the slots of every
 * surfel summed by a gather kernel, frames in batch order and a record's
 * tiles in binning order, so the surfel and pose gradients are bit-identical
 * from run to run and for every schedule and forward variant (it stages 96
 * records per batch, ignoring bwd_batch, and the workspace grows by 64 bytes
 * per pair of capacity and 4 bytes per record).  Every variant
 * and schedule produces bit-identical forward outputs.  box selects the
 * bounding box of a surfel (Sec. 3.2.3, Supp. B): 0 = the exact angular box
 * of its 3-sigma square; 1 = the same box of the smaller square that can
 * still hold a pixel reaching alpha >= 1/255 (half-side k/16, k the smallest
 * integer with 255 o exp(-(k/16)^2 / 2) <= 0.999; surfels with 255 o <= 0.999
 * are culled) -- fewer pairs, identical images; 2 = the paper's relaxed box,
 * the angular extent of the square's four vertices only, which can miss
 * pixels (for comparison).  bwd_batch is the number of surfel records the
 * workgroup backward (bwd_variant 1) stages in LDS per batch: 0 = library
 * default (192), or 128 or 192; results do not depend on it beyond the
 * order of the gradient atomics. */
typedef struct slr_tiling {
    int32_t tile_h, tile_w;
    int32_t variant;
    int32_t schedule;
    int32_t bwd_variant;
    int32_t box;
    int32_t bwd_batch;
} slr_tiling;
#define SLR_BOX_EXACT 0
#define SLR_BOX_OPACITY 1
#define SLR_BOX_VERTEX 2
#define SLR_VARIANT_DEFAULT 0
#define SLR_VARIANT_LDS 1
#define SLR_VARIANT_SCALAR 2
#define SLR_VARIANT_WAVE 3
#define SLR_VARIANT_DETERMINISTIC 4   /* bwd_variant only */
#define SLR_SCHEDULE_DEFAULT 0
#define SLR_SCHEDULE_TILE 1
#define SLR_SCHEDULE_LONGEST 2
#define SLR_SCHEDULE_QUEUE 3

/* Surfel set: raw parameters in device memory, FP32, row-major. */
typedef struct slr_surfels {
    int64_t n;
    const float *means;      /* [n,3] */
    const float *quats;      /* [n,4]  w, x, y, z */
    const float *log_scales; /* [n,2] */
    const float *logits;     /* [n]   */
} slr_surfels;

/* Device views into a workspace after slr_render (binning results). */
typedef struct slr_views {
    const uint32_t *keys;        /* [n]  FP32 bit pattern of the centre range */
    const int32_t *counts;       /* [n]  tiles per surfel, 0 = culled */
    const int16_t *pixbox;       /* [n,8] r0, r1, c0, c1, c2, c3 (c2 = c3 = -1 if one interval), 0, 0 */
    const int32_t *sorted_tile;  /* [K]  tile index ty*tiles_x + tx, ascending */
    const int32_t *sorted_id;    /* [K]  surfel index, by (range key, index) within a tile */
    const int32_t *ranges;       /* [tiles,2] [start, end) into the sorted arrays; (0,0) if empty */
    const float *T_final;        /* [H,W] transmittance after the last contributor */
    const int32_t *n_proc;       /* [H,W] list entries processed up to the last contributor */
    const int32_t *census;       /* [4,H,W] work counters: forward evaluated list entries,
                                    forward contributors, backward evaluated entries,
                                    backward contributors */
    int64_t tiles_x, tiles_y;
} slr_views;

/* Supp. A: camera matrix from an angular extent (radians) and an image size.
 * out[4] = (fu, cu, fv, cv), host memory.  fu = -(W-1)/(az_max-az_min),
 * cu = W/2 (1 + (az_max+az_min)/(az_max-az_min)), and likewise for rows. */
slr_status slr_camera_matrix(double az_min, double az_max, double el_min, double el_max,
                             int32_t height, int32_t width, double *out);

/* Workspace bytes for one image of this size, n surfels and at most
 * pair_capacity (tile, surfel) pairs (Sec. 3.2.1 per-tile lists). */
slr_status slr_workspace_size(const slr_sensor *sensor, const slr_tiling *tiling, int64_t n,
                              int64_t pair_capacity, size_t *bytes);

/* Forward render (Sec. 3.2.1-3.2.3, Supp. D forward process), plain form:
 * projection + bounding box, binning with the radix sort, then per-tile
 * compositing.  Reads back the pair count K once (one host synchronisation)
 * and returns SLR_E_CAPACITY, with *pairs_out = K, if K exceeds the capacity
 * the workspace was sized for.  Outputs (device, FP32): depth [H,W],
 * normal [H,W,3], alpha [H,W].  The workspace keeps the binning and the
 * per-pixel state that slr_backward reads.  pairs_out: host, nullable. */
slr_status slr_render(const slr_surfels *surfels, const double *pose_cw, const slr_sensor *sensor,
                      const slr_tiling *tiling, void *workspace, size_t workspace_bytes,
                      int64_t pair_capacity, float *depth, float *normal, float *alpha,
                      int64_t *pairs_out, void *stream);

/* Backward (Supp. D gradient computation; se(3) pose gradient).  Reads the
 * workspace left by slr_render with the same surfels, pose, sensor and tiling.
 * Upstream gradients (device, FP32): dL_ddepth [H,W], dL_dnormal [H,W,3],
 * dL_dalpha [H,W]; any may be NULL (= zero).  Outputs (device, overwritten):
 * d_means [n,3], d_quats [n,4], d_log_scales [n,2], d_logits [n] (all four
 * set; all four may be NULL when n == 0), d_pose [6] FP64 (nullable).  With SLR_POSE_ONLY in
 * flags the surfel gradients are skipped (they must be NULL); with
 * SLR_ACCUMULATE the surfel gradients are added to the outputs' current
 * contents (a map shared by several keyframes); d_pose is always overwritten. */
#define SLR_POSE_ONLY 1u
#define SLR_ACCUMULATE 2u /* add into the surfel gradients instead of overwriting */
slr_status slr_backward(const slr_surfels *surfels, const double *pose_cw, const slr_sensor *sensor,
                        const slr_tiling *tiling, void *workspace, size_t workspace_bytes,
                        int64_t pair_capacity, const float *dL_ddepth, const float *dL_dnormal,
                        const float *dL_dalpha, float *d_means, float *d_quats, float *d_log_scales,
                        float *d_logits, double *d_pose, uint32_t flags, void *stream);

/* Pose-only Gauss-Newton normal equations of the range image (Sec. 3.3.3:
 * the keyframe pose is updated as T_wc <- T_wc exp(delta), delta = (rho; phi)
 * in se(3), by Gauss-Newton on Huber-robust residuals).  Reads the workspace
 * left by a successful slr_render with the same surfels, pose, sensor and
 * tiling.  With r = D - D_t per pixel, J = dD/d delta at delta = 0 (computed
 * in the reverse traversal of the compositing lists), m the pixel weight and
 * w(r) the Huber IRLS weight (1 for |r| <= huber_k, huber_k / |r| beyond;
 * huber_k <= 0: plain least squares, w = 1):
 *   H = sum m w J J^T,  g = sum m w r J,  cost = sum m rho(r)
 * (rho: r^2/2, or huber_k (|r| - huber_k/2) beyond the threshold); g is the
 * gradient of the cost and the Gauss-Newton step solves H delta = -g.
 * Inputs (device, FP32, [H,W]): depth = the range image that slr_render wrote,
 * target = D_t, weight = m (nullable: all ones; 0 drops a pixel, e.g. where
 * the target has no return).  Output (device FP64, overwritten, 43 values):
 * H row-major [0..35], g [36..41], cost [42].  Sums are taken in a fixed
 * order (bit-reproducible).  tiling.bwd_variant picks the kernel form:
 * SLR_VARIANT_WAVE runs one wave per 64-pixel strip (no workgroup barrier;
 * the faster form for a single keyframe), otherwise one workgroup per tile;
 * both see the same records in the same order per pixel and agree to the
 * last bits of FP32.  Errors: NULL depth, target or normal_eq, NaN huber_k,
 * and the same checks as slr_backward. */
slr_status slr_pose_gn(const slr_surfels *surfels, const double *pose_cw, const slr_sensor *sensor,
                       const slr_tiling *tiling, void *workspace, size_t workspace_bytes, int64_t pair_capacity,
                       const float *depth, const float *target, const float *weight, double huber_k,
                       double *normal_eq, void *stream);

/* Photometric registration normal equations (Sec. 3.3.3): every pixel u of
 * the rendered range image `depth` is back-projected with its range along
 * its pixel-centre ray, p = D(u) v(u), moved by T into the query sensor's
 * frame, q = T p, and projected back, u' = phi(q); the query range image is
 * read at u' by bilinear interpolation of its pixel centres, and
 *   r = |q| - D_q(u')   (= D(u) - D_q(u') at T = I, the printed residual).
 * T (device FP64 [4,4], row-major) maps the render's sensor frame to the
 * query's; the query pose is updated as T_wq <- T_wq exp(delta), i.e.
 * T <- exp(-delta^) T, and with J = dr/d delta, m the weight (nullable: ones)
 * and w the Huber IRLS weight (huber_k as in slr_pose_gn):
 *   H = sum m w J J^T,  g = sum m w r J,  cost = sum m rho(r).
 * A pixel takes part when D(u) > 0, m != 0, u' lies inside the grid of query
 * pixel centres (column in [0, W-1), row in [0, H-1)) and the four query
 * pixels around u' are > 0 (have a return).  Both images share `sensor`
 * (device FP32 [H,W]).  Output (device FP64, overwritten, 44 values): H
 * row-major [0..35], g [36..41], cost [42], number of pixels taken [43].
 * Workspace: device, 256-byte aligned, slr_photo_workspace_size bytes, no
 * state kept between calls.  Errors: NULL depth, query, pose_qm, normal_eq or
 * workspace, a workspace too small, NaN huber_k, an invalid sensor. */
slr_status slr_photo_workspace_size(const slr_sensor *sensor, size_t *bytes);
slr_status slr_photo_gn(const slr_sensor *sensor, const float *depth, const float *query, const float *weight,
                        const double *pose_qm, double huber_k, void *workspace, size_t workspace_bytes,
                        double *normal_eq, void *stream);

/* slr_photo_gn without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight registration loops, harnesses
 * that forbid allocation): the workgroup rows live in a static device array
 * of the library (1 MiB per GPU, held until the process ends), so the call
 * allocates nothing and takes images of at most 1,048,576 pixels (H * W;
 * larger ones return SLR_E_INVALID and launch nothing).  Same arguments,
 * output and errors as slr_photo_gn otherwise, and the same result bit for
 * bit (the same kernels in the same order).  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams or threads)
 * race and must be serialised by the caller.  Nothing in the array needs to
 * start at zero (each call writes every row it reads). */
slr_status slr_photo_gn_noalloc(const slr_sensor *sensor, const float *depth, const float *query,
                                const float *weight, const double *pose_qm, double huber_k, double *normal_eq,
                                void *stream);

/* Device pointers into a workspace filled by slr_render (for inspection and
 * tests). */
slr_status slr_workspace_views(const slr_sensor *sensor, const slr_tiling *tiling, int64_t n,
                               int64_t pair_capacity, void *workspace, size_t workspace_bytes,
                               slr_views *views);

/* ------------------------------------------------------------------------
 * Batched form (Sec. 3.3.2: the local model is refined over keyframes sampled
 * from its keyframe set; this form renders and differentiates the keyframes
 * of one refinement iteration together): many frames (keyframes, each with
 * its own pose, sensor and image size) rendered by one set of launches with
 * no host synchronisation,
 * so that a whole optimisation iteration can be captured in a HIP graph and
 * replayed.  Frames reference surfel sets; several frames may share one set
 * (one map seen from several keyframes), in which case the set's gradients
 * are summed over those frames.  Each frame is binned and composited with its
 * own tile shape (slr_frame.tile_h, tile_w; by default the tiling's), so
 * wide and narrow range images can share one launch; the compositing forms,
 * schedule, box mode and backward batch size are the batch's.
 *
 * Usage: size the workspace, call slr_batch_prepare once (it uploads the
 * sensor tables and the per-frame descriptors, i.e. every pointer below, into
 * the workspace), then call slr_batch_render / slr_batch_backward any number
 * of times with the same sets, frames and workspace (these two only enqueue
 * kernels).  Call slr_batch_prepare again when any pointer or size changes.
 * The pair count is checked on the device: if it exceeds pair_capacity the
 * frames render empty and the overflow word (see slr_batch_counters) holds
 * the required capacity.
 * ------------------------------------------------------------------------ */
typedef struct slr_frame {
    int32_t set;                      /* index into the sets array */
    const double *pose_cw;            /* device [4,4] FP64 */
    slr_sensor sensor;
    float *depth, *normal, *alpha;    /* device outputs [H,W], [H,W,3], [H,W] */
    const float *dL_ddepth, *dL_dnormal, *dL_dalpha; /* device upstream gradients, nullable */
    double *d_pose;                   /* device [6] FP64 pose gradient, nullable */
    int32_t tile_h, tile_w;           /* this frame's tile shape (one of the shapes slr_tiling
                                         accepts), or 0, 0 for the batch tiling's shape */
} slr_frame;

typedef struct slr_surfel_grads {
    float *means, *quats, *log_scales, *logits; /* device [n,3], [n,4], [n,2], [n] */
} slr_surfel_grads;

slr_status slr_batch_workspace_size(int32_t n_sets, const slr_surfels *sets, int32_t n_frames,
                                    const slr_frame *frames, const slr_tiling *tiling,
                                    int64_t pair_capacity, size_t *bytes);
slr_status slr_batch_prepare(int32_t n_sets, const slr_surfels *sets, int32_t n_frames, const slr_frame *frames,
                             const slr_tiling *tiling, int64_t pair_capacity, void *workspace,
                             size_t workspace_bytes, void *stream);
/* Forward of every frame (Sec. 3.2.1-3.2.3 and Supp. D forward process, as
 * slr_render): projection, one range sort and one tile sort for the batch,
 * one compositing launch over all tiles of all frames. */
slr_status slr_batch_render(int32_t n_sets, const slr_surfels *sets, int32_t n_frames, const slr_frame *frames,
                            const slr_tiling *tiling, int64_t pair_capacity, void *workspace,
                            size_t workspace_bytes, void *stream);
/* Backward of every frame (Supp. D gradient computation and the se(3) pose
 * gradient of Sec. 3.3.3, as slr_backward).  grads: host array of n_sets entries (device
 * pointers; an entry of all-NULL pointers skips that set), or NULL with
 * SLR_POSE_ONLY.  Frame pose gradients go to frames[f].d_pose when set.
 * With SLR_ACCUMULATE the set gradients are added to the outputs. */
slr_status slr_batch_backward(int32_t n_sets, const slr_surfels *sets, const slr_surfel_grads *grads,
                              int32_t n_frames, const slr_frame *frames, const slr_tiling *tiling,
                              int64_t pair_capacity, void *workspace, size_t workspace_bytes, uint32_t flags,
                              void *stream);
/* Tile autotuner (Sec. 3.2.1 splits the image into 16x16 tiles; here the
 * tile shape, compositing form and schedule of a batch are chosen by timing):
 * for each of the n_candidates tilings, renders and back-propagates the batch
 * once untimed and reps times timed (HIP events on stream; the call
 * synchronises), and writes the median ms per candidate to ms (host,
 * [n_candidates]; -1 for a candidate whose pairs overflowed pair_capacity) and
 * the fastest candidate's index to *best (host).  The workspace must hold the
 * largest candidate (slr_batch_workspace_size of each); outputs, upstream
 * gradients and grads are used as in slr_batch_render / slr_batch_backward and
 * are left holding the last candidate's results.  Errors: any invalid
 * candidate (nothing is launched then), SLR_E_CAPACITY if every candidate
 * overflowed. */
slr_status slr_batch_autotune(int32_t n_sets, const slr_surfels *sets, const slr_surfel_grads *grads,
                              int32_t n_frames, const slr_frame *frames, const slr_tiling *candidates,
                              int32_t n_candidates, int64_t pair_capacity, void *workspace, size_t workspace_bytes,
                              int32_t reps, double *ms, int32_t *best, void *stream);

/* Device address of seven uint64 words in the workspace (the per-tile lists
 * of Sec. 3.2.1): [0] the pair count K of the last render, [1] the overflow
 * word (K when K > pair_capacity, else 0), [2] the pair count actually
 * binned, [3] the number of surfel records that bin into at least one tile,
 * [4], [5] internal scheduling words, [6] the number of (frame, surfel)
 * records culled for invalid parameters (a non-finite mean, quaternion,
 * log-scale or logit, or a zero quaternion); such a surfel takes no part in
 * the render and gets zero gradients. */
slr_status slr_batch_counters(int32_t n_sets, const slr_surfels *sets, int32_t n_frames, const slr_frame *frames,
                              const slr_tiling *tiling, int64_t pair_capacity, void *workspace,
                              size_t workspace_bytes, const uint64_t **counters);

/* Device views into a batch workspace after slr_batch_render, for inspection
 * and tests.  Indices are global to the batch: record r of frame f is
 * item_off(f) + surfel index, where item_off(f) sums the surfel counts of the
 * sets of frames 0..f-1; tile t of frame f is tile_off(f) + ty*tiles_x + tx
 * (tile_off(f) sums the tile counts of frames 0..f-1); pixel (i, j) of frame f
 * is pix_off(f) + i*W + j (pix_off sums H*W of frames 0..f-1).  keys, counts
 * and pixbox are per record; sorted_tile / sorted_id hold (global tile,
 * record) of the K pairs; ranges is per global tile; T_final, n_proc and
 * census are per global pixel (census rows are the total pixel count apart).
 * tiles_x holds the batch's total tile count and tiles_y is 1. */
slr_status slr_batch_views(int32_t n_sets, const slr_surfels *sets, int32_t n_frames, const slr_frame *frames,
                           const slr_tiling *tiling, int64_t pair_capacity, void *workspace, size_t workspace_bytes,
                           slr_views *views);

/* Adam over the raw surfel parameters (the map refinement of Sec. 3.3.2
 * optimises them with Adam), PyTorch's single-tensor form:
 *   m <- m + (1 - beta1) (g - m),  v <- beta2 v + (1 - beta2) g^2,
 *   p <- p - lr / (1 - beta1^step) * m / (sqrt(v) / sqrt(1 - beta2^step) + eps).
 * Parameters (device, FP32, updated in place) are the surfel arrays of an
 * slr_surfels set; grads the matching slr_surfel_grads; m and v (device, FP32,
 * caller-owned, zero before the first step) are [n, 10] per surfel in the
 * order means, quaternion, log-scales, logit.  step >= 1.  Errors: NULL or
 * misaligned arrays, step < 1, non-finite or negative hyper-parameters. */
typedef struct slr_adam_config {
    double lr_means, lr_quats, lr_log_scales, lr_logits;
    double beta1, beta2, eps;
    int32_t step;
} slr_adam_config;
slr_status slr_adam_step(int64_t n, float *means, float *quats, float *log_scales, float *logits,
                         const slr_surfel_grads *grads, float *m, float *v, const slr_adam_config *cfg, void *stream);

/* Range and normal losses of Sec. 3.3.2 (Eqs. loss_range and loss_normal,
 * with rho_d = 1 and N(D) replaced by a given target normal), fused with
 * their gradients:
 *   L = w_d * sum_valid |D - D_t| + w_n * sum_valid (1 - N . N_t),
 * valid = D_t > 0 (the mask M_v).  Writes dL/dD [H,W] and dL/dN [H,W,3]
 * (device, FP32, overwritten) and adds L to *loss (device FP64, nullable).
 * w_d, w_n are typically 1 / |M_v|. */
slr_status slr_loss_l1_normal(int64_t pixels, const float *depth, const float *normal, const float *target_depth,
                              const float *target_normal, float w_d, float w_n, float *dL_ddepth,
                              float *dL_dnormal, double *loss, void *stream);

/* The same loss over several images in one call (the keyframes of a batch):
 * image f has its own pixel count, buffers (layouts as in
 * slr_loss_l1_normal, device, FP32; outputs overwritten) and weights, and its
 * gradients are bit-identical to an slr_loss_l1_normal call on it alone.  The
 * sum of the images' L is added to *loss (device FP64, nullable; the
 * summation order differs from separate calls).  frames is a host array of
 * n_frames entries, read before the call returns.  Errors: n_frames < 0, a
 * NULL frames array, a negative pixel count, a NULL buffer of an image with
 * pixels, non-finite weights (nothing is launched then). */
typedef struct slr_loss_frame {
    int64_t pixels;
    const float *depth, *normal, *target_depth, *target_normal;
    float w_d, w_n;
    float *dL_ddepth, *dL_dnormal;
} slr_loss_frame;
slr_status slr_loss_l1_normal_frames(int32_t n_frames, const slr_loss_frame *frames, double *loss, void *stream);

/* Range image of a point cloud (Sec. 3.1, Eq. spherical-projection): each
 * point (device FP32 [n,3], sensor frame) goes to (u, v) = K psi(p) and lands
 * in the pixel whose cell contains it, (i, j) = (floor(v), floor(u)) (pixel
 * centres at (j + 1/2, i + 1/2)); the pixel keeps the nearest return, the
 * range rounded once to FP32 from sqrt((x^2 + y^2) + z^2) in FP64; pixels
 * without a point get 0 (the valid mask of Sec. 3.3.1 is range > 0).  Points
 * with a non-finite coordinate, zero range or outside the image are dropped.
 * range: device FP32 [H,W], overwritten.  The result does not depend on the
 * order of the points. */
slr_status slr_cloud_to_range(const slr_sensor *sensor, int64_t n, const float *points, float *range,
                              void *stream);

/* Surface normals from the gradients of a range image (the N(D) of L_n,
 * Sec. 3.3.2): pixels are back-projected along their centre rays, dx and dy
 * are the central differences of the left/right and upper/lower neighbours,
 * N = dx x dy / |dx x dy| turned to face the sensor.  Zero on the border rows
 * and columns and where any of the five pixels has no return (range <= 0).
 * range: device FP32 [H,W]; normals: device FP32 [H,W,3], overwritten. */
slr_status slr_range_normals(const slr_sensor *sensor, const float *range, float *normals, void *stream);

/* Refinement losses of Sec. 3.3.2 on the valid pixels M_v = D_t > 0, fused
 * with their gradients (rho_d = 1):
 *   L = w_d sum |D - D_t| + w_n sum_{N_t != 0} (1 - N . N_t)
 *       + w_o sum -log max(O, 1e-6)
 * N_t is taken as given (e.g. slr_range_normals of a range image); its pixels
 * without a normal (all zero) are left out of L_n.  Writes dL/dD, dL/dN,
 * dL/dO (device FP32 [P], [P,3], [P], overwritten; dL/dO = -w_o/O where
 * O > 1e-6, else 0) and adds L to *loss (device FP64, nullable). */
slr_status slr_loss_map(int64_t pixels, const float *depth, const float *normal, const float *alpha,
                        const float *target_depth, const float *target_normal, float w_d, float w_n, float w_o,
                        float *dL_ddepth, float *dL_dnormal, float *dL_dalpha, double *loss, void *stream);

/* Scale regulariser of Sec. 3.3.2 with its sign corrected (the printed
 * tau_s - max(s) would reward growth): L_s = w_s sum max(0, max(s_a, s_b) -
 * tau_s), s = exp(log-scales) (device FP32 [n,2]).  Adds dL/d(log-scales) to
 * d_log_scales (device FP32 [n,2]; only the larger scale's entry, s_a on a
 * tie) and L to *loss (device FP64, nullable). */
slr_status slr_scale_reg(int64_t n, const float *log_scales, double tau_s, double w_s, float *d_log_scales,
                         double *loss, void *stream);

/* Local model initialisation (Sec. 3.3.1): a weight map from the range
 * gradients over the valid pixels and a weighted draw of n pixels, each
 * back-projected into a splat whose normal faces the sensor.
 *   weight(u) = 0 where range(u) <= 0 or mask(u) == 0 (mask nullable: ones),
 *               else floor(256 (|gx| + |gy|)) + 1 capped at 2^24 + 1, with
 *               gx, gy the FP32 central differences of the range image (0 on
 *               the border and next to a pixel without a return);
 *   draw k: t = min(floor(uniforms[k] * total), total - 1) over the exact
 *           integer prefix sums of the weights; the first pixel whose running
 *           sum exceeds t (uniforms: device FP64 [n] in [0, 1), the caller's
 *           random numbers);
 *   splat: mean T_wc (D v) (pose_cw: device FP64 [4,4] T_cw), normal
 *          n = -R_wc v, tangents t_a = normalize(n x e) with e the world z axis
 *          (x when |n_z| > 0.9) and t_b = n x t_a, quaternion (w,x,y,z), w >= 0,
 *          of (t_a t_b n); both log-scales log(D pitch scale_factor) with
 *          pitch the larger angular pixel pitch; logit as given.
 * Outputs (device): means [n,3], quats [n,4], log_scales [n,2], logits [n]
 * FP32 and pixel [n] int32 (the drawn pixel, row-major; -1 and zeros for
 * every draw when no pixel has weight).  Workspace: device, 256-byte
 * aligned, slr_init_workspace_size bytes. */
slr_status slr_init_workspace_size(const slr_sensor *sensor, size_t *bytes);
slr_status slr_init_splats(const slr_sensor *sensor, const float *range, const float *mask, const double *pose_cw,
                           int64_t n, const double *uniforms, double scale_factor, float logit, void *workspace,
                           size_t workspace_bytes, float *means, float *quats, float *log_scales, float *logits,
                           int32_t *pixel, void *stream);

/* Stage timers: when enabled, the library records HIP events on the
 * caller's stream around each stage it launches; slr_stage_times()
 * synchronises them and returns the accumulated milliseconds and launch
 * counts per stage (then resets).  Stages: 0 projection, 1 range sort,
 * 2 count scan, 3 emit + tile sort + ranges, 4 forward compositing,
 * 5 backward compositing, 6 per-surfel gradients, 7 loss, 8 Gauss-Newton
 * compositing, 9 photometric registration.  ms and counts are host arrays
 * of SLR_NUM_STAGES entries. */
#define SLR_NUM_STAGES 10
slr_status slr_stage_timer_enable(int32_t on);
slr_status slr_stage_times(double *ms, int64_t *counts);

const char *slr_status_string(slr_status status);
const char *slr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SLR_H */

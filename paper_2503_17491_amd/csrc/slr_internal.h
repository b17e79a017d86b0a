// slr_internal.h -- data layouts and launcher declarations shared by the HIP
// translation units of the rasterizer library.  Not part of the public ABI.
//
// The engine renders a batch of frames (keyframes) in one set of launches:
// every kernel reads a per-frame descriptor from device memory, records are
// indexed by a global item index (frame offset + surfel index), tiles by a
// global tile index (frame tile offset + local tile), so one range sort, one
// tile sort and one launch per compositing pass serve the whole batch.  The
// plain per-image form is the batch of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/slr.h"

namespace slr {

// Per-surfel record read by the per-tile compositing kernels (96 bytes).
// The ray-splat intersection of Sec. 3.2.2 / Supp. D is evaluated in
// Cramer form: with b_alpha, b_beta, b_c the sensor-frame columns of
// T = T_cw H and v the unit pixel ray,
//   P = b_beta x b_c,  Q = b_c x b_alpha,  M = b_alpha x b_beta,
//   s_hat = (P.v, Q.v) / (M.v),  range t = tau / (M.v),  tau = b_c . M,
// which equals the plane-pair construction p_hat = h_alpha x h_beta
// (p_hat = -(P.v, Q.v, M.v)) and the range |nu| of the hit point.
struct __align__(16) RasterRec {
    double P[3], Q[3], M[3];
    float tau, opac;
    float n[3];          // sensor-frame normal R_cw t_n
    uint32_t rows;       // first row | last row << 16 of the pixel box
};
static_assert(sizeof(RasterRec) == 96, "RasterRec layout");

// Sensor-frame splat axes of a record (rebuilt from its P, Q, M when a
// record's sums are converted into splat gradients).
struct __align__(16) FrameRec {
    double ba[3], bb[3], bc[3];
    float n[3];
    float pad[3];
};
static_assert(sizeof(FrameRec) == 96, "FrameRec layout");

// Unit direction of b_c of a record (FP64), the reference the backward
// subtracts from pixel rays before accumulating, and tau = b_c . M in FP64
// (both derived from the record when it is staged).
struct ChatRec {
    double c[3];
    double tau;
};

// Pixel box: rows [r0, r1], columns [c0, c1] and optionally [c2, c3]; frame
// index of the record and its tile count (a frame has at most 65535 tiles).
struct __align__(16) PixBox {
    int16_t r0, r1, c0, c1, c2, c3, frame;
    uint16_t cnt;
};

// The tiles of a record's pixel box in the order its pairs are emitted: row
// by row, and in a row the tiles of the first column interval, then those of
// the second (a box that wraps past column W - 1 has two; intervals that
// touch or overlap in tile columns are merged into the first).  Tile rows and
// columns are frame-local.
struct TileSpan {
    int ty0, ax0, na, bx0, len;   // first row, first interval [ax0, ax0 + na), second from bx0, tiles per row
};
__host__ __device__ inline TileSpan tile_span(const PixBox &b, int th, int tw)
{
    int ax0 = b.c0 / tw, ax1 = b.c1 / tw;
    int bx0 = 0, bx1 = -1;
    if (b.c2 >= 0) {
        bx0 = b.c2 / tw; bx1 = b.c3 / tw;
        if (bx0 <= ax1) { ax1 = bx1 > ax1 ? bx1 : ax1; bx0 = 0; bx1 = -1; }
    }
    return TileSpan{b.r0 / th, ax0, ax1 - ax0 + 1, bx0, (ax1 - ax0 + 1) + (bx1 - bx0 + 1)};
}
// Position of tile (ty, tx) among the emitted pairs of a record with span sp
// (the tile must be in the record's box).
__host__ __device__ inline int span_index(const TileSpan &sp, int ty, int tx)
{
    const int cc = (tx >= sp.ax0 && tx < sp.ax0 + sp.na) ? tx - sp.ax0 : sp.na + (tx - sp.bx0);
    return (ty - sp.ty0) * sp.len + cc;
}

// Per-frame descriptor (device memory).
struct __align__(16) FrameDesc {
    const double *pose;                                  // [4,4] T_cw
    const float *means, *quats, *lsc, *logits;           // the frame's surfel set
    float *depth, *normal, *alpha;                       // outputs
    const float *gD, *gN, *gO;                           // upstream gradients (nullable)
    double *d_pose;                                      // [6] pose gradient (never NULL)
    float *acc;                                          // the set's gradient accumulator
    const float *gn_target, *gn_weight;                  // Gauss-Newton target range, weight (nullable)
    double *gn;                                          // [43] Gauss-Newton output: H (6x6), g, cost
    double huber_k;                                      // Huber threshold (<= 0: least squares)
    int64_t n;                                           // surfels in the set
    int64_t item_off;                                    // first record index
    int64_t pix_off;                                     // first pixel of the per-pixel state
    int64_t tab_off;                                     // first double2 of the direction tables
    double fu, cu, fv, cv, near_m;
    int32_t H, W, th, tw, tiles_x, tiles_y, tile_off, set;
};

// Gradient accumulator per surfel (world frame): dL/d(s_a t_a), dL/d(s_b t_b),
// dL/dmu, dL/dt_n and dL/do.
constexpr int kAccStride = 13;

// Radix sort geometry.
constexpr int kSortThreads = 256;
// Items per thread of the radix-sort, compaction and count-scan kernels,
// chosen per sort from the size its grid is launched for: blocks of 1024, 2048
// or 4096 items, so that the few hundred thousand records of a single frame
// still spread over the chip in enough blocks, while a batch's millions move
// in larger ones.
__host__ __device__ inline int sort_items(int64_t n_max)
{
    return n_max >= (int64_t(1) << 23) ? 16 : (n_max >= (int64_t(1) << 20) ? 8 : 4);
}
constexpr int kEmitSlots = 512;                      // (tile, surfel) pairs per emit block (a power of two)
constexpr int kMaxDigitBits = 8;

// Workgroups of the one-wave compositing forms: 4 strips per tile, tiles in
// runs of 8 (see strip_of_block).
inline int64_t wave_blocks(int64_t tiles) { return 32 * ((tiles + 7) / 8); }

// Quad mode of the one-wave forward and Gauss-Newton kernels: the longest
// tiles whose list has at least kQuadMinList entries (at most quad_tile_cap of
// them, a multiple of 8) are composited as 16 sub-strips of 16 pixels, four
// records per step.  It shortens the longest strips about twofold at about
// 1.6 times their work, which pays while the chip has room: the cap keeps the
// launch within kQuadBudget workgroups (twice the 4096 waves the chip holds at
// four waves per SIMD), so a single 128x1024 frame (512 tiles) may take every
// long tile in quad mode, a 128x2048 frame (1024 tiles) about a third of them
// and a batch of eight 128x1024 frames none.  The count is decided on the
// device after binning (a u32 at misc + kMiscQuadTiles).
constexpr int kQuadMinList = 768;    // a boundary of the half-octave length buckets of the tile order
constexpr int64_t kQuadBudget = 8192;
constexpr size_t kMiscQuadTiles = 32;
constexpr size_t kMiscQueue = 40;      // u32 work-queue head of the persistent workgroup backward
constexpr size_t kMiscQueueFwd = 44;   // u32 work-queue head of the persistent one-wave forward
constexpr size_t kMiscInvalid = 48;    // u64 records culled for invalid parameters (counter word 6)
__host__ __device__ inline int64_t quad_tile_cap(int64_t tiles)
{
    const int64_t by_budget = (kQuadBudget - 4 * tiles) / 12;
    const int64_t c = tiles < by_budget ? tiles : by_budget;
    return c > 0 ? (c & ~int64_t(7)) : 0;
}

// Compositing variant and tile schedule used when the caller asks for the default.
constexpr int kDefaultVariant = SLR_VARIANT_WAVE;
constexpr int kDefaultSchedule = SLR_SCHEDULE_LONGEST;

// Angular margin (radians) by which the bounding box is widened on every side.
constexpr double kBoxMargin = 2e-5;

// Workspace layout of a batch (offsets in bytes from the workspace base).
struct Layout {
    int32_t frames, sets, th, tw, variant, schedule, bwd_variant, box_mode, bwd_batch;
    int64_t items, cap, tiles, pixels, acc_floats, tab_entries;
    int tile_bits, depth_passes, tile_passes;
    bool depth_in_1, tile_in_1;
    size_t desc, tables, tile_frame, rec, box, skey, key0, val0, key1, val1, cnt, off, estart, blocksum;
    size_t pt0, pv0, pt1, pv1, rcnt, rbox, pose_part, gn_part, ranges, order, hist, stateT, stateN, census, acc, scratch_pose, misc, total;
    size_t cmask;          // contribution mask of the one-wave forward (cmask_words u64)
    int64_t cmask_words;
    // fixed-order backward (bwd_variant SLR_VARIANT_DETERMINISTIC; 0 otherwise): the range-order
    // index of each record, one 64-B slot per pair for a (tile, record) flush and a bit per
    // pair marking the slots written by the current backward
    size_t rank, slots, slot_bits;
    int64_t slot_words;
    // misc: [0] u64 K, [8] u64 overflow (required K, 0 = fits), [64..) u32 digit totals
};

// Both longest-first schedules (the plain grid and the work queue) order the
// tiles on the device after binning.
inline bool longest_order(const Layout &L)
{
    return L.schedule == SLR_SCHEDULE_LONGEST || L.schedule == SLR_SCHEDULE_QUEUE;
}

struct FrameGeom {
    int32_t H, W, set;
    int32_t th, tw;   // the frame's tile shape
};

Layout make_layout(int32_t nframes, const FrameGeom *frames, int32_t nsets, const int64_t *set_n, int64_t cap,
                   int32_t th, int32_t tw, bool fixed_order);

// Floats of a pair slot of the fixed-order backward (13 used).
constexpr int kSlotFloats = 16;

// ---- launchers (all enqueue on `stream`) ----
void launch_write_desc(const FrameDesc *host_descs, int32_t count, FrameDesc *dev, hipStream_t stream);
void launch_tile_frame(const Layout &L, char *ws, hipStream_t stream);
void launch_project(const Layout &L, char *ws, int64_t max_n, hipStream_t stream);
void launch_depth_sort(const Layout &L, char *ws, hipStream_t stream);
void launch_scan_counts(const Layout &L, char *ws, hipStream_t stream);
void launch_emit_and_tile_sort(const Layout &L, char *ws, hipStream_t stream);
void launch_raster_fwd(const Layout &L, char *ws, hipStream_t stream);
void launch_raster_bwd(const Layout &L, char *ws, bool pose_only, hipStream_t stream);
void launch_pose_reduce(const Layout &L, char *ws, hipStream_t stream);
// Fixed-order backward: the range-order index of every binned record (before
// the compositing backward), and each surfel's slots summed into its set's
// accumulator, frames in batch order and a record's pairs in emission order
// (after it; acc of set `set`, n surfels).
void launch_record_rank(const Layout &L, char *ws, hipStream_t stream);
void launch_slot_gather(const Layout &L, char *ws, int32_t set, int64_t n, float *acc, hipStream_t stream);
void launch_raster_gn(const Layout &L, char *ws, hipStream_t stream);
void launch_gn_reduce(const Layout &L, char *ws, hipStream_t stream);

// Gauss-Newton partial row of one compositing workgroup: the 21 upper-triangle
// entries of H (row-major), the 6 of g, the cost, and the keyframe index.
constexpr int kGnVals = 28;
constexpr int kGnRow = 32;
void launch_surfel_grad(const float *quats, const float *lsc, const float *logits, int64_t n, const float *acc,
                        float *d_means, float *d_quats, float *d_log_scales, float *d_logits,
                        bool accumulate, hipStream_t stream);
void launch_loss_l1_normal(int64_t pixels, const float *depth, const float *normal, const float *td,
                           const float *tn, float wd, float wn, float *gD, float *gN, double *loss,
                           hipStream_t stream);
constexpr int kLossFramesPerLaunch = 16;
struct LossPack {
    slr_loss_frame f[kLossFramesPerLaunch];
};
void launch_loss_frames(int32_t n_frames, const slr_loss_frame *frames, double *loss, hipStream_t stream);
void launch_fill_u32(void *p, uint32_t v, int64_t count, hipStream_t stream);
size_t photo_workspace_bytes(int32_t H, int32_t W);
// Largest image (pixels) of the allocation-free photometric entry point, and
// the calling device's address of its static scratch (looked up once per device).
int64_t photo_static_max_pixels();
hipError_t photo_static_scratch(double **ptr);
void launch_cloud_to_range(int32_t H, int32_t W, double fu, double cu, double fv, double cv, int64_t n,
                           const float *pts, float *range, hipStream_t stream);
void launch_range_normals(int32_t H, int32_t W, double fu, double cu, double fv, double cv, const float *range,
                          float *normals, hipStream_t stream);
void launch_loss_map(int64_t P, const float *D, const float *N, const float *O, const float *Dt, const float *Nt,
                     float wd, float wn, float wo, float *gD, float *gN, float *gO, double *loss, hipStream_t stream);
void launch_scale_reg(int64_t n, const float *ls, double tau, double ws, float *g, double *loss, hipStream_t stream);
size_t init_workspace_bytes(int32_t H, int32_t W);
void launch_init_splats(int32_t H, int32_t W, double fu, double cu, double fv, double cv, const float *range,
                        const float *mask, const double *Tcw, int64_t n, const double *U, double scale, float logit,
                        char *ws, float *means, float *quats, float *ls, float *logits, int32_t *pix,
                        hipStream_t stream);
void launch_photo_gn(int32_t H, int32_t W, double fu, double cu, double fv, double cv, double huber_k,
                     const float *depth, const float *query, const float *weight, const double *T, double *part,
                     double *out, hipStream_t stream);
void launch_adam(int64_t n, float *means, float *quats, float *ls, float *logits, const float *gm, const float *gq,
                 const float *gl, const float *go, float *m, float *v, const float s[4], float omb1, float b2,
                 float omb2, float c2, float eps, hipStream_t stream);

}  // namespace slr

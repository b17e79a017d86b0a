// slr_internal.h -- data layouts and launcher declarations shared by the HIP
// translation units of the rasterizer library.  Not part of the public ABI.
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

// Sensor-frame splat axes for the per-surfel gradient conversion.
struct __align__(16) FrameRec {
    double ba[3], bb[3], bc[3];
    float n[3];
    float pad[3];
};
static_assert(sizeof(FrameRec) == 96, "FrameRec layout");

// Pixel box: rows [r0, r1], columns [c0, c1] and optionally [c2, c3].
struct __align__(16) PixBox {
    int16_t r0, r1, c0, c1, c2, c3, pad0, pad1;
};

// Gradient accumulator per surfel (world frame): dL/d(s_a t_a), dL/d(s_b t_b),
// dL/dmu, dL/dt_n and dL/do.
constexpr int kAccStride = 13;

// Radix sort geometry.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;                       // per thread
constexpr int kSortTile = kSortThreads * kSortItems; // items per block
constexpr int kMaxDigitBits = 8;

// Workspace layout for one image (offsets in bytes from the workspace base).
struct Layout {
    int64_t n, cap, H, W, th, tw, tiles_x, tiles_y, ntiles;
    int tile_bits;
    size_t tables, rec, frame, box, skey, key0, val0, key1, val1, cnt, off, blocksum;
    size_t pt0, pv0, pt1, pv1, ranges, hist, stateT, stateN, census, acc, misc, total;
    int depth_passes, tile_passes;
    // which buffers hold the sorted results after the passes
    bool depth_in_1, tile_in_1;
};

Layout make_layout(int64_t n, int64_t cap, int32_t H, int32_t W, int32_t th, int32_t tw);

// ---- launchers (all enqueue on `stream`) ----
void launch_project(const slr_surfels &s, const double *pose, const slr_sensor &sen, const Layout &L,
                    char *ws, double cos_m, double sin_m, hipStream_t stream);
void launch_depth_sort(const Layout &L, char *ws, hipStream_t stream);
void launch_scan_counts(const Layout &L, char *ws, hipStream_t stream);
void launch_emit_and_tile_sort(const Layout &L, char *ws, int64_t K, hipStream_t stream);
void launch_raster_fwd(const Layout &L, const slr_sensor &sen, char *ws, int64_t K, float *depth,
                       float *normal, float *alpha, hipStream_t stream);
void launch_raster_bwd(const Layout &L, const slr_sensor &sen, char *ws, const double *pose,
                       const float *gD, const float *gN, const float *gO, double *d_pose, bool pose_only,
                       hipStream_t stream);
void launch_surfel_grad(const slr_surfels &s, const Layout &L, char *ws, float *d_means, float *d_quats,
                        float *d_log_scales, float *d_logits, bool accumulate, hipStream_t stream);
void launch_loss_l1_normal(int64_t pixels, const float *depth, const float *normal, const float *td,
                           const float *tn, float wd, float wn, float *gD, float *gN, double *loss,
                           hipStream_t stream);
void launch_fill_u32(void *p, uint32_t v, int64_t count, hipStream_t stream);

}  // namespace slr

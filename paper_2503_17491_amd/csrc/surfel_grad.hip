// surfel_grad.hip -- per-surfel parameter gradients (Supp. D, last block).
//
// The compositing backward leaves, per surfel, the world-frame gradients
//   w_a = dL/d(s_a t_a), w_b = dL/d(s_b t_b), w_c = dL/dmu, w_n = dL/dt_n,
//   g_o = dL/do
// summed over pixels (and over keyframes that share the surfel).  This kernel
// maps them to the raw parameters: mean, unnormalised quaternion (through
// R(q/|q|)), log-scales and opacity logit.
#include "slr_internal.h"

namespace slr {
namespace {

// Per keyframe: the sum of the compositing workgroups' pose partials (6 values
// and the keyframe index in a row of 8 doubles), in a fixed order, written to
// the keyframe's pose gradient.
__global__ void __launch_bounds__(256)
k_pose_reduce(const FrameDesc *__restrict__ descs, const double *__restrict__ part, int64_t nparts)
{
    __shared__ double red[6][256];
    const int f = blockIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < nparts; b += blockDim.x) {
        const double *pp = part + 8 * b;
        if ((int)pp[6] != f) continue;
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] += pp[c];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) descs[f].d_pose[threadIdx.x] = red[threadIdx.x][0];
}

// Per keyframe: the sum of the Gauss-Newton workgroups' rows (kGnVals values
// and the keyframe index) in a fixed order, written out as H (6x6, both
// triangles), g (6) and the cost.  Frames without an output pointer are skipped.
__global__ void __launch_bounds__(128)
k_gn_reduce(const FrameDesc *__restrict__ descs, const double *__restrict__ part, int64_t nparts, int strips,
            const uint32_t *__restrict__ nquad_dev)
{
    __shared__ double red[kGnVals][128];
    const int f = blockIdx.x;
    double *out = descs[f].gn;
    if (!out) return;
    double v[kGnVals];
#pragma unroll
    for (int c = 0; c < kGnVals; ++c) v[c] = 0.0;
    // one row per tile slot, or (strips = 4) four strip rows per tile slot,
    // added in strip order first; with strips = 4 the first nquad slots (the
    // tiles composited in quad mode) have 16 sub-strip rows each, added in
    // groups of four
    const int64_t nquad = (strips == 4 && nquad_dev) ? (int64_t)*nquad_dev : 0;
    for (int64_t b = threadIdx.x; b < nparts; b += blockDim.x) {
        if (strips == 1) {
            const double *pp = part + (size_t)kGnRow * b;
            if ((int)pp[kGnVals] != f) continue;
#pragma unroll
            for (int c = 0; c < kGnVals; ++c) v[c] += pp[c];
        } else if (b < nquad) {
            const double *pp = part + (size_t)kGnRow * 16 * b;
            if ((int)pp[kGnVals] != f) continue;
#pragma unroll
            for (int c = 0; c < kGnVals; ++c) {
                double s4 = 0.0;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const double *pg = pp + (size_t)kGnRow * 4 * g;
                    s4 += ((pg[c] + pg[kGnRow + c]) + pg[2 * kGnRow + c]) + pg[3 * kGnRow + c];
                }
                v[c] += s4;
            }
        } else {
            const double *pp = part + (size_t)kGnRow * (16 * nquad + 4 * (b - nquad));
            if ((int)pp[kGnVals] != f) continue;
#pragma unroll
            for (int c = 0; c < kGnVals; ++c)
                v[c] += ((pp[c] + pp[kGnRow + c]) + pp[2 * kGnRow + c]) + pp[3 * kGnRow + c];
        }
    }
#pragma unroll
    for (int c = 0; c < kGnVals; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = 64; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < kGnVals; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        }
        __syncthreads();
    }
    const int t = threadIdx.x;
    if (t < 36) {
        const int a = t / 6, b = t % 6;
        const int lo = a < b ? a : b, hi = a < b ? b : a;
        out[t] = red[6 * lo - (lo * (lo - 1)) / 2 + (hi - lo)][0];   // row-major upper triangle
    } else if (t < 42) {
        out[t] = red[21 + (t - 36)][0];
    } else if (t == 42) {
        out[42] = red[27][0];
    }
}

__global__ void __launch_bounds__(256)
k_surfel_grad(int64_t n, const float *__restrict__ quats, const float *__restrict__ lsc,
              const float *__restrict__ logits, const float *__restrict__ acc, float *__restrict__ d_means,
              float *__restrict__ d_quats, float *__restrict__ d_ls, float *__restrict__ d_logits, int accumulate)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    float4 gq4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const float *a = acc + (size_t)k * kAccStride;
    bool any = false;
#pragma unroll
    for (int c = 0; c < kAccStride; ++c) any |= a[c] != 0.0f;
    if (!any) {  // culled or never composited: zero gradient
        if (accumulate) return;
        d_means[3 * k] = 0.f; d_means[3 * k + 1] = 0.f; d_means[3 * k + 2] = 0.f;
        *reinterpret_cast<float4 *>(d_quats + 4 * k) = gq4;
        d_ls[2 * k] = 0.f; d_ls[2 * k + 1] = 0.f;
        d_logits[k] = 0.f;
        return;
    }
    double wa[3] = {a[0], a[1], a[2]}, wb[3] = {a[3], a[4], a[5]}, wn[3] = {a[9], a[10], a[11]};
    const float4 q4 = *reinterpret_cast<const float4 *>(quats + 4 * k);
    const double qn = sqrt((double)q4.x * q4.x + (double)q4.y * q4.y + (double)q4.z * q4.z + (double)q4.w * q4.w);
    const double w = q4.x / qn, x = q4.y / qn, y = q4.z / qn, z = q4.w / qn;
    // columns of R(q): t_a, t_b
    const double ta[3] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y)};
    const double tb[3] = {2.0 * (x * y - w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z + w * x)};
    const double sa = exp((double)lsc[2 * k]), sb = exp((double)lsc[2 * k + 1]);
    // dL/dR, column-wise: (s_a w_a, s_b w_b, w_n)
    double G0[3], G1[3], G2[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) { G0[r] = sa * wa[r]; G1[r] = sb * wb[r]; G2[r] = wn[r]; }
    // R entries as functions of (w, x, y, z); d/dw, d/dx, d/dy, d/dz of
    //   col0 = (1-2(yy+zz), 2(xy+wz), 2(xz-wy))
    //   col1 = (2(xy-wz), 1-2(xx+zz), 2(yz+wx))
    //   col2 = (2(xz+wy), 2(yz-wx), 1-2(xx+yy))
    const double gw = 2.0 * (z * G0[1] - y * G0[2] - z * G1[0] + x * G1[2] + y * G2[0] - x * G2[1]);
    const double gx = 2.0 * (y * G0[1] + z * G0[2] + y * G1[0] - 2.0 * x * G1[1] + w * G1[2] + z * G2[0] -
                             w * G2[1] - 2.0 * x * G2[2]);
    const double gy = 2.0 * (-2.0 * y * G0[0] + x * G0[1] - w * G0[2] + x * G1[0] + z * G1[2] + w * G2[0] +
                             z * G2[1] - 2.0 * y * G2[2]);
    const double gz = 2.0 * (-2.0 * z * G0[0] + w * G0[1] + x * G0[2] - w * G1[0] - 2.0 * z * G1[1] + y * G1[2] +
                             x * G2[0] + y * G2[1]);
    const double dotq = gw * w + gx * x + gy * y + gz * z;
    gq4.x = (float)((gw - dotq * w) / qn);
    gq4.y = (float)((gx - dotq * x) / qn);
    gq4.z = (float)((gy - dotq * y) / qn);
    gq4.w = (float)((gz - dotq * z) / qn);
    float gm[3] = {a[6], a[7], a[8]};
    float gl0 = (float)(sa * (ta[0] * wa[0] + ta[1] * wa[1] + ta[2] * wa[2]));
    float gl1 = (float)(sb * (tb[0] * wb[0] + tb[1] * wb[1] + tb[2] * wb[2]));
    const double o = 1.0 / (1.0 + exp(-(double)logits[k]));
    float go = (float)(o * (1.0 - o) * a[12]);
    if (accumulate) {
        const float4 p = *reinterpret_cast<const float4 *>(d_quats + 4 * k);
        gq4.x += p.x; gq4.y += p.y; gq4.z += p.z; gq4.w += p.w;
        gm[0] += d_means[3 * k]; gm[1] += d_means[3 * k + 1]; gm[2] += d_means[3 * k + 2];
        gl0 += d_ls[2 * k]; gl1 += d_ls[2 * k + 1];
        go += d_logits[k];
    }
    *reinterpret_cast<float4 *>(d_quats + 4 * k) = gq4;
    d_means[3 * k] = gm[0]; d_means[3 * k + 1] = gm[1]; d_means[3 * k + 2] = gm[2];
    d_ls[2 * k] = gl0; d_ls[2 * k + 1] = gl1;
    d_logits[k] = go;
}

// ---- fixed-order backward ----

// rank[order[r]] = r for the binned records r < nvis (range order); the
// entries of records that bin into no tile keep the ~0u the launcher fills
// the array with first.
__global__ void __launch_bounds__(256)
k_record_rank(const uint32_t *__restrict__ order, const uint64_t *__restrict__ nvis, uint32_t *__restrict__ rank)
{
    const uint64_t n = *nvis;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x)
        rank[order[r]] = (uint32_t)r;
}

// One thread per surfel of a set: the slots its records' flushes wrote, frames
// in batch order and a record's pairs in emission order, summed in FP64 and
// written (not added) to the set's accumulator.  The pairs of record r are
// the emission slots [off[r], off[r + 1]) (the last record's run to the
// emitted count keff), below keff; a slot counts if the backward set its bit.
// Frames are taken kGatherFrames at a time with every rank, offset pair and
// first mask word loaded before the sums, so the scattered loads of a group
// are in flight together instead of one dependent chain per frame.
constexpr int kGatherFrames = 8;

__global__ void __launch_bounds__(256)
k_slot_gather(const FrameDesc *__restrict__ descs, int32_t nframes, int32_t set, int64_t n,
              const uint64_t *__restrict__ misc, const uint32_t *__restrict__ rank,
              const uint32_t *__restrict__ off, const float *__restrict__ slots,
              const uint32_t *__restrict__ bits, float *__restrict__ acc)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint64_t keff = misc[2], nvis = misc[3];
    double a[kAccStride];
#pragma unroll
    for (int v = 0; v < kAccStride; ++v) a[v] = 0.0;
    for (int32_t f0 = 0; f0 < nframes; f0 += kGatherFrames) {
        uint32_t r[kGatherFrames];
#pragma unroll
        for (int g = 0; g < kGatherFrames; ++g) {
            const int32_t f = f0 + g;
            r[g] = ~0u;
            if (f < nframes && descs[f].set == set) r[g] = rank[(uint32_t)(descs[f].item_off + k)];
        }
        uint64_t e0[kGatherFrames], e1[kGatherFrames];
#pragma unroll
        for (int g = 0; g < kGatherFrames; ++g) {
            e0[g] = 0;
            e1[g] = 0;
            if (r[g] != ~0u) {   // else the record bins into no tile
                e0[g] = off[r[g]];
                const uint64_t end = (uint64_t)r[g] + 1 < nvis ? (uint64_t)off[r[g] + 1] : keff;
                e1[g] = end < keff ? end : keff;
            }
        }
        uint32_t w[kGatherFrames];
#pragma unroll
        for (int g = 0; g < kGatherFrames; ++g) w[g] = e0[g] < e1[g] ? bits[e0[g] >> 5] : 0u;
#pragma unroll
        for (int g = 0; g < kGatherFrames; ++g) {
            uint32_t word = w[g];
            for (uint64_t e = e0[g]; e < e1[g]; ++e) {
                if (e > e0[g] && (e & 31) == 0) word = bits[e >> 5];   // the run crosses into the next word
                if (!((word >> (e & 31)) & 1u)) continue;
                const float4 *q = reinterpret_cast<const float4 *>(slots + (size_t)kSlotFloats * e);
                const float4 x0 = q[0], x1 = q[1], x2 = q[2];
                const float x3 = slots[(size_t)kSlotFloats * e + 12];
                a[0] += x0.x; a[1] += x0.y; a[2] += x0.z; a[3] += x0.w;
                a[4] += x1.x; a[5] += x1.y; a[6] += x1.z; a[7] += x1.w;
                a[8] += x2.x; a[9] += x2.y; a[10] += x2.z; a[11] += x2.w;
                a[12] += x3;
            }
        }
    }
#pragma unroll
    for (int v = 0; v < kAccStride; ++v) acc[kAccStride * k + v] = (float)a[v];
}

}  // namespace

void launch_record_rank(const Layout &L, char *ws, hipStream_t stream)
{
    if (L.items == 0) return;
    launch_fill_u32(ws + L.rank, ~0u, L.items, stream);
    const int64_t blocks = (L.items + 255) / 256;
    hipLaunchKernelGGL(k_record_rank, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(256), 0, stream,
                       reinterpret_cast<const uint32_t *>(ws + (L.depth_in_1 ? L.val1 : L.val0)),
                       reinterpret_cast<const uint64_t *>(ws + L.misc) + 3, reinterpret_cast<uint32_t *>(ws + L.rank));
}

void launch_slot_gather(const Layout &L, char *ws, int32_t set, int64_t n, float *acc, hipStream_t stream)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_slot_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       reinterpret_cast<const FrameDesc *>(ws + L.desc), L.frames, set, n,
                       reinterpret_cast<const uint64_t *>(ws + L.misc), reinterpret_cast<const uint32_t *>(ws + L.rank),
                       reinterpret_cast<const uint32_t *>(ws + L.off), reinterpret_cast<const float *>(ws + L.slots), reinterpret_cast<const uint32_t *>(ws + L.slot_bits),
                       acc);
}

void launch_pose_reduce(const Layout &L, char *ws, hipStream_t stream)
{
    if (L.frames == 0) return;
    // one row per compositing workgroup (the one-wave backward's grid includes
    // its quad-mode workgroups)
    const int64_t nparts = L.bwd_variant == SLR_VARIANT_WAVE
                               ? wave_blocks(L.tiles) + (longest_order(L) ? 16 * quad_tile_cap(L.tiles) : 0)
                               : L.tiles;
    hipLaunchKernelGGL(k_pose_reduce, dim3((unsigned)L.frames), dim3(256), 0, stream,
                       reinterpret_cast<const FrameDesc *>(ws + L.desc), reinterpret_cast<const double *>(ws + L.pose_part),
                       nparts);
}

void launch_gn_reduce(const Layout &L, char *ws, hipStream_t stream)
{
    if (L.frames == 0) return;
    hipLaunchKernelGGL(k_gn_reduce, dim3((unsigned)L.frames), dim3(128), 0, stream,
                       reinterpret_cast<const FrameDesc *>(ws + L.desc), reinterpret_cast<const double *>(ws + L.gn_part),
                       L.tiles, L.bwd_variant == SLR_VARIANT_WAVE ? 4 : 1,
                       longest_order(L) ? reinterpret_cast<const uint32_t *>(ws + L.misc + kMiscQuadTiles)
                                                          : nullptr);
}

void launch_surfel_grad(const float *quats, const float *lsc, const float *logits, int64_t n, const float *acc,
                        float *d_means, float *d_quats, float *d_log_scales, float *d_logits,
                        bool accumulate, hipStream_t stream)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_surfel_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, quats, lsc, logits,
                       acc, d_means, d_quats, d_log_scales, d_logits, accumulate ? 1 : 0);
}

}  // namespace slr

// support.hip -- HBM-bound support kernels around the rasterizer.
//
// Adam (Kingma and Ba) over the raw surfel parameters, one thread per surfel,
// in the form of PyTorch's single-tensor Adam:
//   m <- m + (1 - b1) (g - m),  v <- b2 v + (1 - b2) g^2,
//   p <- p - s_g m / (sqrt(v) / c2 + eps),  s_g = lr_g / (1 - b1^t), c2 = sqrt(1 - b2^t),
// with one learning rate per parameter group (means, quaternions, log-scales,
// opacity logits).  Moments are [n, 10] per surfel in that group order.
// 280 bytes of HBM traffic per surfel.
//
// Fused range + normal loss of Sec. 3.3.2 (Eqs. loss_range, loss_normal) with
// rho_d = 1 and the normal target given per pixel:
//   L = w_d sum_valid |D - D_t| + w_n sum_valid (1 - N . N_t),  valid = D_t > 0,
// writing dL/dD and dL/dN in the same pass and reducing L per block into one
// FP64 atomic.
#include "slr_internal.h"

namespace slr {
namespace {

// One pixel of the loss: writes dL/dD and dL/dN, returns its share of L.
// All loads are issued before the mask test, so a pixel costs one round trip.
__device__ __forceinline__ double loss_pixel(int64_t p, const float *__restrict__ D, const float *__restrict__ N,
                                             const float *__restrict__ Dt, const float *__restrict__ Nt, float wd,
                                             float wn, float *__restrict__ gD, float *__restrict__ gN)
{
    const float dt = Dt[p], d = D[p];
    const float t0 = Nt[3 * p], t1 = Nt[3 * p + 1], t2 = Nt[3 * p + 2];
    const float m0 = N[3 * p], m1 = N[3 * p + 1], m2 = N[3 * p + 2];
    float g = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
    double part = 0.0;
    if (dt > 0.f) {
        const float r = d - dt;
        g = r > 0.f ? wd : (r < 0.f ? -wd : 0.f);
        const float dot = m0 * t0 + m1 * t1 + m2 * t2;
        n0 = -wn * t0; n1 = -wn * t1; n2 = -wn * t2;
        part = (double)wd * fabsf(r) + (double)wn * (1.0f - dot);
    }
    gD[p] = g;
    gN[3 * p] = n0; gN[3 * p + 1] = n1; gN[3 * p + 2] = n2;
    return part;
}

// Block sum of the loss shares into one FP64 atomic.  Same-address atomics
// serialize, so the launches keep the number of blocks per image small.
__device__ __forceinline__ void loss_block_add(double part, double *loss)
{
    __shared__ double s_part[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double v = s_part[0] + s_part[1] + s_part[2] + s_part[3];
        if (v != 0.0) atomicAdd(loss, v);
    }
}

__global__ void __launch_bounds__(256)
k_loss_l1_normal(int64_t P, const float *__restrict__ D, const float *__restrict__ N, const float *__restrict__ Dt,
                 const float *__restrict__ Nt, float wd, float wn, float *__restrict__ gD, float *__restrict__ gN,
                 double *__restrict__ loss)
{
    double part = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x)
        part += loss_pixel(p, D, N, Dt, Nt, wd, wn, gD, gN);
    if (loss) loss_block_add(part, loss);
}

// The same loss over up to kLossFramesPerLaunch images in one launch
// (blockIdx.y = image), each with its own buffers and weights; every image's
// per-pixel arithmetic is that of k_loss_l1_normal.
__global__ void __launch_bounds__(256)
k_loss_frames(LossPack pack, double *__restrict__ loss)
{
    const slr_loss_frame &f = pack.f[blockIdx.y];
    double part = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < f.pixels;
         p += (int64_t)gridDim.x * blockDim.x)
        part += loss_pixel(p, f.depth, f.normal, f.target_depth, f.target_normal, f.w_d, f.w_n, f.dL_ddepth,
                           f.dL_dnormal);
    if (loss) loss_block_add(part, loss);
}

// blocks per image of the loss launches (see loss_block_add)
constexpr int64_t kLossBlocks = 64;

// omb1 = 1 - b1, omb2 = 1 - b2, both formed in FP64 on the host
__device__ __forceinline__ void adam1(float &p, float g, float &m, float &v, float s, float omb1, float b2, float omb2,
                                      float c2, float eps)
{
    m = fmaf(omb1, g - m, m);
    v = b2 * v + omb2 * (g * g);
    p = p - s * (m / (sqrtf(v) / c2 + eps));
}

__global__ void __launch_bounds__(256)
k_adam(int64_t n, float *__restrict__ means, float *__restrict__ quats, float *__restrict__ ls,
       float *__restrict__ logits, const float *__restrict__ gm, const float *__restrict__ gq,
       const float *__restrict__ gl, const float *__restrict__ go, float *__restrict__ mom, float *__restrict__ vel,
       float s_mean, float s_quat, float s_ls, float s_logit, float omb1, float b2, float omb2, float c2, float eps)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    float *m = mom + 10 * k, *v = vel + 10 * k;
    float mm[10], vv[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) { mm[c] = m[c]; vv[c] = v[c]; }
#pragma unroll
    for (int c = 0; c < 3; ++c) adam1(means[3 * k + c], gm[3 * k + c], mm[c], vv[c], s_mean, omb1, b2, omb2, c2, eps);
    float4 q = *reinterpret_cast<float4 *>(quats + 4 * k);
    const float4 g4 = *reinterpret_cast<const float4 *>(gq + 4 * k);
    adam1(q.x, g4.x, mm[3], vv[3], s_quat, omb1, b2, omb2, c2, eps);
    adam1(q.y, g4.y, mm[4], vv[4], s_quat, omb1, b2, omb2, c2, eps);
    adam1(q.z, g4.z, mm[5], vv[5], s_quat, omb1, b2, omb2, c2, eps);
    adam1(q.w, g4.w, mm[6], vv[6], s_quat, omb1, b2, omb2, c2, eps);
    *reinterpret_cast<float4 *>(quats + 4 * k) = q;
    adam1(ls[2 * k], gl[2 * k], mm[7], vv[7], s_ls, omb1, b2, omb2, c2, eps);
    adam1(ls[2 * k + 1], gl[2 * k + 1], mm[8], vv[8], s_ls, omb1, b2, omb2, c2, eps);
    adam1(logits[k], go[k], mm[9], vv[9], s_logit, omb1, b2, omb2, c2, eps);
#pragma unroll
    for (int c = 0; c < 10; ++c) { m[c] = mm[c]; v[c] = vv[c]; }
}

}  // namespace

void launch_adam(int64_t n, float *means, float *quats, float *ls, float *logits, const float *gm, const float *gq,
                 const float *gl, const float *go, float *m, float *v, const float s[4], float omb1, float b2,
                 float omb2, float c2, float eps, hipStream_t stream)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, means, quats, ls, logits, gm,
                       gq, gl, go, m, v, s[0], s[1], s[2], s[3], omb1, b2, omb2, c2, eps);
}

void launch_loss_l1_normal(int64_t P, const float *D, const float *N, const float *Dt, const float *Nt, float wd,
                           float wn, float *gD, float *gN, double *loss, hipStream_t stream)
{
    if (P <= 0) return;
    int64_t blocks = (P + 255) / 256;
    if (blocks > kLossBlocks) blocks = kLossBlocks;
    hipLaunchKernelGGL(k_loss_l1_normal, dim3((unsigned)blocks), dim3(256), 0, stream, P, D, N, Dt, Nt, wd, wn, gD,
                       gN, loss);
}

void launch_loss_frames(int32_t n_frames, const slr_loss_frame *frames, double *loss, hipStream_t stream)
{
    for (int32_t b = 0; b < n_frames; b += kLossFramesPerLaunch) {
        LossPack pack;
        const int c = n_frames - b < kLossFramesPerLaunch ? n_frames - b : kLossFramesPerLaunch;
        int64_t pmax = 0;
        for (int i = 0; i < c; ++i) {
            pack.f[i] = frames[b + i];
            pmax = frames[b + i].pixels > pmax ? frames[b + i].pixels : pmax;
        }
        if (pmax <= 0) continue;
        int64_t blocks = (pmax + 255) / 256;
        if (blocks > kLossBlocks) blocks = kLossBlocks;
        hipLaunchKernelGGL(k_loss_frames, dim3((unsigned)blocks, c), dim3(256), 0, stream, pack, loss);
    }
}

}  // namespace slr

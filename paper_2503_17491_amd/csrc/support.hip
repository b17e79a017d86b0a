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

__global__ void __launch_bounds__(256)
k_loss_l1_normal(int64_t P, const float *__restrict__ D, const float *__restrict__ N, const float *__restrict__ Dt,
                 const float *__restrict__ Nt, float wd, float wn, float *__restrict__ gD, float *__restrict__ gN,
                 double *__restrict__ loss)
{
    __shared__ double s_part[4];
    double part = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const float dt = Dt[p];
        float g = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
        if (dt > 0.f) {
            const float r = D[p] - dt;
            g = r > 0.f ? wd : (r < 0.f ? -wd : 0.f);
            const float t0 = Nt[3 * p], t1 = Nt[3 * p + 1], t2 = Nt[3 * p + 2];
            const float dot = N[3 * p] * t0 + N[3 * p + 1] * t1 + N[3 * p + 2] * t2;
            n0 = -wn * t0; n1 = -wn * t1; n2 = -wn * t2;
            part += (double)wd * fabsf(r) + (double)wn * (1.0f - dot);
        }
        gD[p] = g;
        gN[3 * p] = n0; gN[3 * p + 1] = n1; gN[3 * p + 2] = n2;
    }
    if (loss) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
        if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = part;
        __syncthreads();
        if (threadIdx.x == 0) {
            const double v = s_part[0] + s_part[1] + s_part[2] + s_part[3];
            if (v != 0.0) atomicAdd(loss, v);
        }
    }
}

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
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_loss_l1_normal, dim3((unsigned)blocks), dim3(256), 0, stream, P, D, N, Dt, Nt, wd, wn, gD,
                       gN, loss);
}

}  // namespace slr

// support.hip -- HBM-bound support kernels around the rasterizer.
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

}  // namespace

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

// photo.hip -- photometric registration normal equations (gfx950).
//
// Sec. 3.3.3: every pixel u of the rendered range image is back-projected
// with its range (p = D(u) v(u), v the unit ray of the pixel centre under K
// of Supp. A), moved into the query sensor's frame (q = T p), projected back
// (u' = phi(q)) and compared with the query range image read there by
// bilinear interpolation: r = |q| - D_q(u').  With T(delta) = exp(-delta^) T
// (the query pose updated as T_wq <- T_wq exp(delta)) and G = dr/dq =
// q/|q| - (dB/dx f_u d az/dq + dB/dy f_v d el/dq), the pixel's Jacobian row is
// J = (-G, G x q).  A pixel takes part when D(u) > 0, its weight is non-zero,
// u' lies inside the grid of query pixel centres and the four query pixels
// around it have a return.  Huber in IRLS form as in the Gauss-Newton kernel.
//
// One thread per pixel, all in FP64 (a few hundred operations per pixel on
// an image of ~10^5 pixels: the kernel is bound by its launch and its one
// gather of four query pixels, not by arithmetic).  The 21 + 6 + 2 sums of a
// workgroup are formed by FP64 butterflies over each wave and added over the
// four waves in a fixed order into a row of their own; k_photo_reduce sums
// the rows in a fixed order.
#include "slr_internal.h"

#include <mutex>

namespace slr {
namespace {

constexpr int kPhotoVals = 29;   // H upper triangle (21), g (6), cost, count
constexpr int kPhotoRow = 32;

struct PhotoArgs {
    double fu, cu, fv, cv, huber_k;
    int32_t H, W;
};

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(256)
k_photo_gn(PhotoArgs a, const float *__restrict__ depth, const float *__restrict__ query,
           const float *__restrict__ weight, const double *__restrict__ T, double *__restrict__ part)
{
    __shared__ double s_red[4][kPhotoVals];
    const int64_t npix = (int64_t)a.H * a.W;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double J[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double wgt = 0.0, wr = 0.0, cost = 0.0, cnt = 0.0;
    if (p < npix) {
        const float d = depth[p];
        const float m = weight ? weight[p] : 1.0f;
        if (d > 0.0f && m != 0.0f) {
            const int i = (int)(p / a.W), j = (int)(p - (int64_t)i * a.W);
            const double az = ((double)j + 0.5 - a.cu) / a.fu, el = ((double)i + 0.5 - a.cv) / a.fv;
            double sa, ca, se, ce;
            sincos(az, &sa, &ca);
            sincos(el, &se, &ce);
            const double px = (double)d * ce * ca, py = (double)d * ce * sa, pz = (double)d * se;
            const double qx = T[0] * px + T[1] * py + T[2] * pz + T[3];
            const double qy = T[4] * px + T[5] * py + T[6] * pz + T[7];
            const double qz = T[8] * px + T[9] * py + T[10] * pz + T[11];
            const double r2 = qx * qx + qy * qy, q2 = r2 + qz * qz;
            const double rxy = sqrt(r2), rq = sqrt(q2);
            const double x = a.fu * atan2(qy, qx) + a.cu - 0.5;
            const double y = a.fv * atan2(qz, rxy) + a.cv - 0.5;
            if (rxy > 0.0 && x >= 0.0 && x < (double)(a.W - 1) && y >= 0.0 && y < (double)(a.H - 1)) {
                const int x0 = (int)x, y0 = (int)y;   // non-negative: truncation is the floor
                const double fx = x - x0, fy = y - y0;
                const float *r0 = query + (int64_t)y0 * a.W + x0;
                const float *r1 = r0 + a.W;
                const double qa = r0[0], qb = r0[1], qc = r1[0], qd = r1[1];
                if (qa > 0.0 && qb > 0.0 && qc > 0.0 && qd > 0.0) {
                    const double B = (1.0 - fy) * ((1.0 - fx) * qa + fx * qb) + fy * ((1.0 - fx) * qc + fx * qd);
                    const double Bx = (1.0 - fy) * (qb - qa) + fy * (qd - qc);
                    const double By = (1.0 - fx) * (qc - qa) + fx * (qd - qb);
                    const double r = rq - B;
                    // d az/dq = (-qy, qx, 0) / r2;  d el/dq = (-qx qz / rxy, -qy qz / rxy, rxy) / q2
                    const double ka = a.fu * Bx / r2, ke = a.fv * By / q2;
                    const double Gx = qx / rq + ka * qy + ke * qx * qz / rxy;
                    const double Gy = qy / rq - ka * qx + ke * qy * qz / rxy;
                    const double Gz = qz / rq - ke * rxy;
                    J[0] = -Gx; J[1] = -Gy; J[2] = -Gz;
                    J[3] = Gy * qz - Gz * qy;
                    J[4] = Gz * qx - Gx * qz;
                    J[5] = Gx * qy - Gy * qx;
                    const double k = a.huber_k, ar = fabs(r);
                    const bool lin = k > 0.0 && ar > k;
                    wgt = (double)m * (lin ? k / ar : 1.0);
                    wr = wgt * r;
                    cost = (double)m * (lin ? k * (ar - 0.5 * k) : 0.5 * r * r);
                    cnt = 1.0;
                }
            }
        }
    }
    int c = 0;
#pragma unroll
    for (int u = 0; u < 6; ++u) {
#pragma unroll
        for (int v = u; v < 6; ++v) {
            const double s = wave_sum_f64(wgt * J[u] * J[v]);
            if (lane == 0) s_red[wid][c] = s;
            ++c;
        }
    }
#pragma unroll
    for (int u = 0; u < 6; ++u) {
        const double s = wave_sum_f64(wr * J[u]);
        if (lane == 0) s_red[wid][21 + u] = s;
    }
    {
        const double s0 = wave_sum_f64(cost), s1 = wave_sum_f64(cnt);
        if (lane == 0) { s_red[wid][27] = s0; s_red[wid][28] = s1; }
    }
    __syncthreads();
    if (threadIdx.x < kPhotoVals) {
        const int t = threadIdx.x;
        part[(size_t)kPhotoRow * blockIdx.x + t] = ((s_red[0][t] + s_red[1][t]) + s_red[2][t]) + s_red[3][t];
    }
}

// Fixed-order sum of the workgroup rows; writes H (6x6, both triangles), g,
// the cost and the count of pixels that took part.
__global__ void __launch_bounds__(128)
k_photo_reduce(const double *__restrict__ part, int64_t nparts, double *__restrict__ out)
{
    __shared__ double red[kPhotoVals][128];
    double v[kPhotoVals];
#pragma unroll
    for (int c = 0; c < kPhotoVals; ++c) v[c] = 0.0;
    for (int64_t b = threadIdx.x; b < nparts; b += blockDim.x) {
        const double *pp = part + (size_t)kPhotoRow * b;
#pragma unroll
        for (int c = 0; c < kPhotoVals; ++c) v[c] += pp[c];
    }
#pragma unroll
    for (int c = 0; c < kPhotoVals; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    for (int w = 64; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < kPhotoVals; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        }
        __syncthreads();
    }
    const int t = threadIdx.x;
    if (t < 36) {
        const int u = t / 6, v2 = t % 6;
        const int lo = u < v2 ? u : v2, hi = u < v2 ? v2 : u;
        out[t] = red[6 * lo - (lo * (lo - 1)) / 2 + (hi - lo)][0];
    } else if (t < 44) {
        out[t] = red[21 + (t - 36)][0];   // g (6), cost, count
    }
}

// Scratch of the allocation-free entry point: the workgroup rows of
// k_photo_gn for images of up to kPhotoStaticBlocks * 256 pixels (1 MiB per
// GPU, held for the life of the process).  Host code never passes this name
// to a kernel: it is a host-side stand-in for the array; the device address
// comes from hipGetSymbolAddress, once per device.
constexpr int64_t kPhotoStaticBlocks = 4096;
static __device__ __align__(256) double scratch[kPhotoStaticBlocks * kPhotoRow];

}  // namespace

int64_t photo_blocks(int32_t H, int32_t W) { return ((int64_t)H * W + 255) / 256; }

int64_t photo_static_max_pixels() { return kPhotoStaticBlocks * 256; }

hipError_t photo_static_scratch(double **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *a = nullptr;
        // the current device is `dev`: its copy of the array is looked up
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double *>(a);
    }
    *ptr = addr[dev];
    return hipSuccess;
}

size_t photo_workspace_bytes(int32_t H, int32_t W)
{
    return sizeof(double) * kPhotoRow * (size_t)(photo_blocks(H, W) > 0 ? photo_blocks(H, W) : 1);
}

void launch_photo_gn(int32_t H, int32_t W, double fu, double cu, double fv, double cv, double huber_k,
                     const float *depth, const float *query, const float *weight, const double *T, double *part,
                     double *out, hipStream_t stream)
{
    const int64_t nb = photo_blocks(H, W);
    PhotoArgs a{fu, cu, fv, cv, huber_k, H, W};
    if (nb > 0)
        hipLaunchKernelGGL(k_photo_gn, dim3((unsigned)nb), dim3(256), 0, stream, a, depth, query, weight, T, part);
    hipLaunchKernelGGL(k_photo_reduce, dim3(1), dim3(128), 0, stream, part, nb, out);
}

}  // namespace slr

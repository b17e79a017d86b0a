// mapping.hip -- mapping-side image kernels (gfx950): the range image of a
// point cloud (Sec. 3.1), normals from the gradients of a range image and the
// refinement losses L_d, L_n, L_o, L_s (Sec. 3.3.2).
//
// All of them are elementwise or nearest-neighbour image work: one thread per
// point, pixel or surfel, HBM- or launch-bound.
#include "slr_internal.h"

namespace slr {
namespace {

constexpr uint32_t kInfBits = 0x7f800000u;   // +inf: no return yet
constexpr double kOMin = 1e-6;               // opacity clamp of -log O

struct MapSensor {
    double fu, cu, fv, cv;
    int32_t H, W;
};

__global__ void __launch_bounds__(256) k_range_fill(uint32_t *__restrict__ D, int64_t n)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        D[p] = kInfBits;
}

// Spherical projection (Eq. spherical-projection): the point lands in the
// pixel whose cell contains (u, v) = K psi(p) and keeps the smallest range.
// Positive FP32 ranges order like their bit patterns, so an unsigned atomic
// minimum keeps the nearest return whatever the order of the points.
__global__ void __launch_bounds__(256)
k_cloud_scatter(int64_t n, const float *__restrict__ pts, MapSensor s, uint32_t *__restrict__ D)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double x = pts[3 * k], y = pts[3 * k + 1], z = pts[3 * k + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) return;
    const double rxy2 = x * x + y * y;
    const double r = sqrt(rxy2 + z * z);
    if (!(r > 0.0)) return;
    const double u = s.fu * atan2(y, x) + s.cu;
    const double v = s.fv * atan2(z, sqrt(rxy2)) + s.cv;
    const double jf = floor(u), iff = floor(v);
    if (!(jf >= 0.0 && jf < (double)s.W && iff >= 0.0 && iff < (double)s.H)) return;
    const float rf = (float)r;
    atomicMin(D + (int64_t)iff * s.W + (int64_t)jf, __float_as_uint(rf));
}

__global__ void __launch_bounds__(256) k_range_finalize(uint32_t *__restrict__ D, int64_t n)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        if (D[p] == kInfBits) D[p] = 0u;
}

__device__ __forceinline__ void pixel_point(const MapSensor &s, double d, double az, double el, double *p)
{
    double sa, ca, se, ce;
    sincos(az, &sa, &ca);
    sincos(el, &se, &ce);
    p[0] = d * ce * ca; p[1] = d * ce * sa; p[2] = d * se;
}

// Normals from the gradients of a range image: central differences of the
// back-projected neighbours, N = dx x dy / |dx x dy| turned to face the
// sensor; zero on the border and next to a missing return.
__global__ void __launch_bounds__(256)
k_range_normals(MapSensor s, const float *__restrict__ D, float *__restrict__ N)
{
    const int64_t npix = (int64_t)s.H * s.W;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const int i = (int)(p / s.W), j = (int)(p - (int64_t)i * s.W);
    float o0 = 0.f, o1 = 0.f, o2 = 0.f;
    if (i > 0 && i < s.H - 1 && j > 0 && j < s.W - 1) {
        const float dc = D[p], dl = D[p - 1], dr = D[p + 1], du = D[p - s.W], dd = D[p + s.W];
        if (dc > 0.f && dl > 0.f && dr > 0.f && du > 0.f && dd > 0.f) {
            const double az = ((double)j + 0.5 - s.cu) / s.fu, el = ((double)i + 0.5 - s.cv) / s.fv;
            const double azl = ((double)j - 0.5 - s.cu) / s.fu, azr = ((double)j + 1.5 - s.cu) / s.fu;
            const double elu = ((double)i - 0.5 - s.cv) / s.fv, eld = ((double)i + 1.5 - s.cv) / s.fv;
            double pc[3], pl[3], pr[3], pu[3], pd[3];
            pixel_point(s, dc, az, el, pc);
            pixel_point(s, dl, azl, el, pl);
            pixel_point(s, dr, azr, el, pr);
            pixel_point(s, du, az, elu, pu);
            pixel_point(s, dd, az, eld, pd);
            const double dx[3] = {pr[0] - pl[0], pr[1] - pl[1], pr[2] - pl[2]};
            const double dy[3] = {pu[0] - pd[0], pu[1] - pd[1], pu[2] - pd[2]};
            double n0 = dx[1] * dy[2] - dx[2] * dy[1];
            double n1 = dx[2] * dy[0] - dx[0] * dy[2];
            double n2 = dx[0] * dy[1] - dx[1] * dy[0];
            const double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
            if (nn > 0.0) {
                double sg = 1.0 / nn;
                if (n0 * pc[0] + n1 * pc[1] + n2 * pc[2] > 0.0) sg = -sg;
                o0 = (float)(n0 * sg); o1 = (float)(n1 * sg); o2 = (float)(n2 * sg);
            }
        }
    }
    N[3 * p] = o0; N[3 * p + 1] = o1; N[3 * p + 2] = o2;
}

__device__ __forceinline__ void block_add(double part, double *loss)
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

// Refinement losses on M_v = D_t > 0: w_d |D - D_t| + w_n (1 - N . N_t) where
// N_t is a normal (non-zero) + w_o (-log max(O, O_min)), with their gradients.
__global__ void __launch_bounds__(256)
k_loss_map(int64_t P, const float *__restrict__ D, const float *__restrict__ N, const float *__restrict__ O,
           const float *__restrict__ Dt, const float *__restrict__ Nt, float wd, float wn, float wo,
           float *__restrict__ gD, float *__restrict__ gN, float *__restrict__ gO, double *__restrict__ loss)
{
    double part = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const float dt = Dt[p];
        float g = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f, go = 0.f;
        if (dt > 0.f) {
            const float r = D[p] - dt;
            g = r > 0.f ? wd : (r < 0.f ? -wd : 0.f);
            part += (double)wd * fabs((double)D[p] - (double)dt);
            const float t0 = Nt[3 * p], t1 = Nt[3 * p + 1], t2 = Nt[3 * p + 2];
            if (t0 != 0.f || t1 != 0.f || t2 != 0.f) {
                n0 = -wn * t0; n1 = -wn * t1; n2 = -wn * t2;
                const double dot = (double)N[3 * p] * t0 + (double)N[3 * p + 1] * t1 + (double)N[3 * p + 2] * t2;
                part += (double)wn * (1.0 - dot);
            }
            const double o = O[p];
            const bool above = o > kOMin;
            go = above ? (float)(-(double)wo / o) : 0.f;
            part += -(double)wo * log(above ? o : kOMin);
        }
        gD[p] = g;
        gN[3 * p] = n0; gN[3 * p + 1] = n1; gN[3 * p + 2] = n2;
        gO[p] = go;
    }
    if (loss) block_add(part, loss);
}

// Scale cap (sign corrected): w_s max(0, max(s_a, s_b) - tau_s); the gradient
// goes to the log-scale of the larger scale (s_a on a tie) and is added.
__global__ void __launch_bounds__(256)
k_scale_reg(int64_t n, const float *__restrict__ ls, double tau, double ws, float *__restrict__ g,
            double *__restrict__ loss)
{
    double part = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const double sa = exp((double)ls[2 * k]), sb = exp((double)ls[2 * k + 1]);
        const bool first = sa >= sb;
        const double sm = first ? sa : sb;
        if (sm > tau) {
            part += ws * (sm - tau);
            g[2 * k + (first ? 0 : 1)] += (float)(ws * sm);
        }
    }
    if (loss) block_add(part, loss);
}

int grid_for(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

void launch_cloud_to_range(int32_t H, int32_t W, double fu, double cu, double fv, double cv, int64_t n,
                           const float *pts, float *range, hipStream_t stream)
{
    const int64_t npix = (int64_t)H * W;
    MapSensor s{fu, cu, fv, cv, H, W};
    uint32_t *D = reinterpret_cast<uint32_t *>(range);
    hipLaunchKernelGGL(k_range_fill, dim3(grid_for(npix)), dim3(256), 0, stream, D, npix);
    if (n > 0)
        hipLaunchKernelGGL(k_cloud_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, pts, s, D);
    hipLaunchKernelGGL(k_range_finalize, dim3(grid_for(npix)), dim3(256), 0, stream, D, npix);
}

void launch_range_normals(int32_t H, int32_t W, double fu, double cu, double fv, double cv, const float *range,
                          float *normals, hipStream_t stream)
{
    const int64_t npix = (int64_t)H * W;
    if (npix == 0) return;
    MapSensor s{fu, cu, fv, cv, H, W};
    hipLaunchKernelGGL(k_range_normals, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, stream, s, range,
                       normals);
}

void launch_loss_map(int64_t P, const float *D, const float *N, const float *O, const float *Dt, const float *Nt,
                     float wd, float wn, float wo, float *gD, float *gN, float *gO, double *loss, hipStream_t stream)
{
    if (P == 0) return;
    hipLaunchKernelGGL(k_loss_map, dim3(grid_for(P)), dim3(256), 0, stream, P, D, N, O, Dt, Nt, wd, wn, wo, gD, gN,
                       gO, loss);
}

void launch_scale_reg(int64_t n, const float *ls, double tau, double ws, float *g, double *loss, hipStream_t stream)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_scale_reg, dim3(grid_for(n)), dim3(256), 0, stream, n, ls, tau, ws, g, loss);
}

}  // namespace slr

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

// ---- local model initialisation (Sec. 3.3.1) ----
// Integer weights from the range gradients (FP32 central differences, exact
// IEEE operations, no square root) over the valid pixels:
// floor(256 (|gx| + |gy|)) + 1, capped; 0 without a return or where the mask is 0.
__global__ void __launch_bounds__(256)
k_init_weights(MapSensor s, const float *__restrict__ D, const float *__restrict__ mask, uint32_t *__restrict__ w)
{
    const int64_t npix = (int64_t)s.H * s.W;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const int i = (int)(p / s.W), j = (int)(p - (int64_t)i * s.W);
    const float d = D[p];
    const bool valid = d > 0.f && (!mask || mask[p] != 0.f);
    uint32_t out = 0;
    if (valid) {
        float g = 0.f;
        if (i > 0 && i < s.H - 1 && j > 0 && j < s.W - 1) {
            const float dl = D[p - 1], dr = D[p + 1], du = D[p - s.W], dd = D[p + s.W];
            if (dl > 0.f && dr > 0.f && du > 0.f && dd > 0.f) {
                const float gx = (dr - dl) * 0.5f, gy = (dd - du) * 0.5f;
                g = fabsf(gx) + fabsf(gy);
            }
        }
        const float q = fminf(floorf(g * 256.0f), 16777216.0f);
        out = (uint32_t)q + 1u;
    }
    w[p] = out;
}

constexpr int kScanPer = 1024;   // items per scan block (256 threads x 4)

__device__ __forceinline__ uint64_t block_incl_scan(uint64_t v, uint64_t *sh)
{
    // inclusive scan over the 256 threads of a block (Hillis-Steele in LDS)
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint64_t add = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    return sh[threadIdx.x];
}

__global__ void __launch_bounds__(256)
k_scan_sums(const uint32_t *__restrict__ w, int64_t n, uint64_t *__restrict__ bsum)
{
    __shared__ uint64_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * kScanPer + 4 * threadIdx.x;
    uint64_t v = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (base + e < n) v += w[base + e];
    const uint64_t inc = block_incl_scan(v, sh);
    if (threadIdx.x == 255) bsum[blockIdx.x] = inc;
}

// exclusive prefix of the block sums, in place (one block, chunks of 256)
__global__ void __launch_bounds__(256) k_scan_bsums(uint64_t *__restrict__ bsum, int64_t nb)
{
    __shared__ uint64_t sh[256];
    uint64_t carry = 0;
    for (int64_t c = 0; c < nb; c += 256) {
        const int64_t k = c + threadIdx.x;
        const uint64_t v = k < nb ? bsum[k] : 0;
        const uint64_t inc = block_incl_scan(v, sh);
        if (k < nb) bsum[k] = carry + inc - v;
        carry += sh[255];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256)
k_scan_final(const uint32_t *__restrict__ w, int64_t n, const uint64_t *__restrict__ bexcl, uint64_t *__restrict__ cum)
{
    __shared__ uint64_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * kScanPer + 4 * threadIdx.x;
    uint64_t x[4];
    uint64_t v = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        x[e] = base + e < n ? w[base + e] : 0;
        v += x[e];
    }
    const uint64_t inc = block_incl_scan(v, sh);
    uint64_t run = bexcl[blockIdx.x] + inc - v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        run += x[e];
        if (base + e < n) cum[base + e] = run;
    }
}

__device__ void quat_from_rot(const double R[3][3], double q[4])
{
    const double t = R[0][0] + R[1][1] + R[2][2];
    if (t > 0.0) {
        const double s = 2.0 * sqrt(1.0 + t);
        q[0] = 0.25 * s; q[1] = (R[2][1] - R[1][2]) / s; q[2] = (R[0][2] - R[2][0]) / s; q[3] = (R[1][0] - R[0][1]) / s;
    } else if (R[0][0] > R[1][1] && R[0][0] > R[2][2]) {
        const double s = 2.0 * sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]);
        q[0] = (R[2][1] - R[1][2]) / s; q[1] = 0.25 * s; q[2] = (R[0][1] + R[1][0]) / s; q[3] = (R[0][2] + R[2][0]) / s;
    } else if (R[1][1] > R[2][2]) {
        const double s = 2.0 * sqrt(1.0 + R[1][1] - R[0][0] - R[2][2]);
        q[0] = (R[0][2] - R[2][0]) / s; q[1] = (R[0][1] + R[1][0]) / s; q[2] = 0.25 * s; q[3] = (R[1][2] + R[2][1]) / s;
    } else {
        const double s = 2.0 * sqrt(1.0 + R[2][2] - R[0][0] - R[1][1]);
        q[0] = (R[1][0] - R[0][1]) / s; q[1] = (R[0][2] + R[2][0]) / s; q[2] = (R[1][2] + R[2][1]) / s; q[3] = 0.25 * s;
    }
    if (q[0] < 0.0) { q[0] = -q[0]; q[1] = -q[1]; q[2] = -q[2]; q[3] = -q[3]; }
}

// One draw per thread: t = min(floor(U total), total - 1), the first pixel
// whose running weight exceeds t (binary search), and its splat: mean
// T_wc (D v), normal -R_wc v facing the sensor, tangents from the world z
// axis (x when the normal is within acos 0.9 of z), both scales
// D * pitch * scale_factor, the given logit.
__global__ void __launch_bounds__(256)
k_init_sample(int64_t n, const double *__restrict__ U, const uint64_t *__restrict__ cum, MapSensor s,
              const float *__restrict__ D, const double *__restrict__ Tcw, double scale, float logit,
              float *__restrict__ means, float *__restrict__ quats, float *__restrict__ ls,
              float *__restrict__ logits, int32_t *__restrict__ pix)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t npix = (int64_t)s.H * s.W;
    const uint64_t total = npix > 0 ? cum[npix - 1] : 0;
    if (total == 0) {
        pix[k] = -1;
        means[3 * k] = means[3 * k + 1] = means[3 * k + 2] = 0.f;
        quats[4 * k] = quats[4 * k + 1] = quats[4 * k + 2] = quats[4 * k + 3] = 0.f;
        ls[2 * k] = ls[2 * k + 1] = 0.f;
        logits[k] = 0.f;
        return;
    }
    uint64_t t = (uint64_t)floor(U[k] * (double)total);
    if (t > total - 1) t = total - 1;
    int64_t lo = 0, hi = npix - 1;     // first index with cum > t (exists: cum[npix-1] = total > t)
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cum[mid] > t) hi = mid; else lo = mid + 1;
    }
    const int i = (int)(lo / s.W), j = (int)(lo - (int64_t)i * s.W);
    const double az = ((double)j + 0.5 - s.cu) / s.fu, el = ((double)i + 0.5 - s.cv) / s.fv;
    double sa, ca, se, ce;
    sincos(az, &sa, &ca);
    sincos(el, &se, &ce);
    const double v[3] = {ce * ca, ce * sa, se};
    const double d = D[lo];
    double Rwc[3][3], twc[3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Rwc[r][c] = Tcw[4 * c + r];
    for (int r = 0; r < 3; ++r) twc[r] = -(Rwc[r][0] * Tcw[3] + Rwc[r][1] * Tcw[7] + Rwc[r][2] * Tcw[11]);
    double nrm[3], mu[3];
    for (int r = 0; r < 3; ++r) {
        mu[r] = (Rwc[r][0] * (d * v[0]) + Rwc[r][1] * (d * v[1]) + Rwc[r][2] * (d * v[2])) + twc[r];
        nrm[r] = -(Rwc[r][0] * v[0] + Rwc[r][1] * v[1] + Rwc[r][2] * v[2]);
    }
    const double e[3] = {fabs(nrm[2]) > 0.9 ? 1.0 : 0.0, 0.0, fabs(nrm[2]) > 0.9 ? 0.0 : 1.0};
    double ta[3] = {nrm[1] * e[2] - nrm[2] * e[1], nrm[2] * e[0] - nrm[0] * e[2], nrm[0] * e[1] - nrm[1] * e[0]};
    const double tn = sqrt(ta[0] * ta[0] + ta[1] * ta[1] + ta[2] * ta[2]);
    ta[0] /= tn; ta[1] /= tn; ta[2] /= tn;
    const double tb[3] = {nrm[1] * ta[2] - nrm[2] * ta[1], nrm[2] * ta[0] - nrm[0] * ta[2], nrm[0] * ta[1] - nrm[1] * ta[0]};
    const double R[3][3] = {{ta[0], tb[0], nrm[0]}, {ta[1], tb[1], nrm[1]}, {ta[2], tb[2], nrm[2]}};
    double q[4];
    quat_from_rot(R, q);
    const double pitch = fmax(fabs(1.0 / s.fu), fabs(1.0 / s.fv));
    const float lsc = (float)log(d * pitch * scale);
    pix[k] = (int32_t)lo;
    means[3 * k] = (float)mu[0]; means[3 * k + 1] = (float)mu[1]; means[3 * k + 2] = (float)mu[2];
    quats[4 * k] = (float)q[0]; quats[4 * k + 1] = (float)q[1]; quats[4 * k + 2] = (float)q[2]; quats[4 * k + 3] = (float)q[3];
    ls[2 * k] = lsc; ls[2 * k + 1] = lsc;
    logits[k] = logit;
}

int grid_for(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// Launches that end in one same-address FP64 atomic per block: those
// atomics serialize, so few blocks loop over the items.
int grid_reduce(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (int)(b < 128 ? (b > 0 ? b : 1) : 128);
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
    hipLaunchKernelGGL(k_loss_map, dim3(grid_reduce(P)), dim3(256), 0, stream, P, D, N, O, Dt, Nt, wd, wn, wo, gD, gN,
                       gO, loss);
}

size_t init_workspace_bytes(int32_t H, int32_t W)
{
    const int64_t n = (int64_t)H * W, nb = (n + kScanPer - 1) / kScanPer;
    const size_t a = ((4 * (size_t)n + 255) / 256) * 256, b = ((8 * (size_t)n + 255) / 256) * 256;
    return a + b + 8 * (size_t)(nb > 0 ? nb : 1);
}

void launch_init_splats(int32_t H, int32_t W, double fu, double cu, double fv, double cv, const float *range,
                        const float *mask, const double *Tcw, int64_t n, const double *U, double scale, float logit,
                        char *ws, float *means, float *quats, float *ls, float *logits, int32_t *pix,
                        hipStream_t stream)
{
    const int64_t npix = (int64_t)H * W, nb = (npix + kScanPer - 1) / kScanPer;
    MapSensor s{fu, cu, fv, cv, H, W};
    uint32_t *w = reinterpret_cast<uint32_t *>(ws);
    uint64_t *cum = reinterpret_cast<uint64_t *>(ws + ((4 * (size_t)npix + 255) / 256) * 256);
    uint64_t *bsum = reinterpret_cast<uint64_t *>(reinterpret_cast<char *>(cum) + ((8 * (size_t)npix + 255) / 256) * 256);
    if (npix > 0) {
        hipLaunchKernelGGL(k_init_weights, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, stream, s, range, mask, w);
        hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, stream, w, npix, bsum);
        hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(256), 0, stream, bsum, nb);
        hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(256), 0, stream, w, npix, bsum, cum);
    }
    if (n > 0)
        hipLaunchKernelGGL(k_init_sample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, U, cum, s, range,
                           Tcw, scale, logit, means, quats, ls, logits, pix);
}

void launch_scale_reg(int64_t n, const float *ls, double tau, double ws, float *g, double *loss, hipStream_t stream)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_scale_reg, dim3(grid_reduce(n)), dim3(256), 0, stream, n, ls, tau, ws, g, loss);
}

}  // namespace slr

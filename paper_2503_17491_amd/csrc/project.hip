// project.hip -- per-surfel spherical projection and bounding box (gfx950).
//
// One thread per surfel:
//   * the splat-to-sensor transform T = T_cw H of Supp. D (b_alpha, b_beta,
//     b_c, n) in FP64, packed into the compositing record (Cramer form, see
//     RasterRec; the backward rebuilds the axes from it);
//   * the range key: FP32 rounding of |b_c|;
//   * the bounding box of Sec. 3.2.3 / Supp. B, computed as the exact angular
//     box of the 3-sigma splat square, widened by an angular margin, with the
//     azimuth seam handled by ordering directions instead of angles (angles
//     only guess where the exact direction tests start);
//   * the tile count of the box.
// The key and the box use only IEEE-exact FP64 +,-,*,/,sqrt in a fixed order
// (this translation unit is compiled with contraction off) plus host-made
// direction tables, so the binning is reproducible bit for bit.
#include "slr_internal.h"

#pragma clang fp contract(off)

namespace slr {
namespace {

// exp for the box scales: reduction by ln 2 and the degree-13 Taylor
// polynomial of exp on [-ln2/2, ln2/2] (textbook method, a few ulp).
__device__ double box_exp(double x)
{
    const double LN2 = 0.6931471805599453;
    const double INV_LN2 = 1.4426950408889634;
    double k = floor(x * INV_LN2 + 0.5);
    double r = x - k * LN2;
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)k);
}

__device__ inline double xcross(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

// Direction order on (-pi, pi]: true when angle(a) <= angle(b).
__device__ inline bool angle_le(double ax, double ay, double bx, double by)
{
    bool ua = (ay > 0.0) || (ay == 0.0 && ax < 0.0);
    bool ub = (by > 0.0) || (by == 0.0 && bx < 0.0);
    if (ua != ub) return !ua && ub;
    return xcross(ax, ay, bx, by) >= 0.0;
}

// Elevation of (r, z) strictly below elevation of (r', z') (r, r' >= 0).
__device__ inline bool elev_below(double r, double z, double r2, double z2) { return z * r2 - r * z2 < 0.0; }

// First index in [0, n) where a monotone predicate holds (n if none), as a
// bisection finds it, but started from a guess: two independent probes at
// g - 1 and g settle it when the guess is right; otherwise the bisection runs
// on the side the probes leave open.  The guess changes only the cost.
template <class Pred>
__device__ int first_true(int g, int n, const Pred &pred)
{
    g = g < 0 ? 0 : (g > n ? n : g);
    const bool below = g > 0 ? pred(g - 1) : false;
    const bool at = g < n ? pred(g) : true;
    if (!below && at) return g;
    int lo = below ? 0 : g + 1, hi = below ? g - 1 : n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pred(mid)) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Guess of the first index i with a boundary position x <= i (ceil) or
// x < i (floor + 1), from an FP32 estimate; 0 when x is not a usable number.
__device__ inline int guess_ceil(float x, int n) { return (x > -1.0f && x < (float)n + 1.0f) ? (int)ceilf(x) : 0; }
__device__ inline int guess_above(float x, int n)
{
    return (x > -1.0f && x < (float)n + 1.0f) ? (int)floorf(x) + 1 : 0;
}

struct BoxOut {
    int nint;   // 0 = empty
    int r0, r1, c[4];
};

// Opacity-aware half-side of the support square (box mode 1): a pair only
// contributes where alpha = o G >= 1/255, inside |s_hat|^2 <= 2 ln(255 o); the
// square of half-side k/16 holds that disk for the smallest integer k with
// 255 o exp(-(k/16)^2 / 2) <= 0.999 (binary search with the reproducible exp,
// so the integer decision is reproducible).  0: no pixel can reach the
// threshold (255 o <= 0.999); 3: the disk is not inside the 3-sigma square.
__device__ double support_radius(double logit)
{
    const double o = 1.0 / (1.0 + box_exp(-logit));
    const double c = 255.0 * o;
    if (c <= 0.999) return 0.0;
    if (!(c * box_exp(-(48.0 * 48.0) / 512.0) <= 0.999)) return 3.0;
    int lo = 1, hi = 48;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (c * box_exp(-(double)(mid * mid) / 512.0) <= 0.999) hi = mid; else lo = mid + 1;
    }
    return (double)lo / 16.0;
}

// Exact angular box of the square {C + a A + b B : |a|, |b| <= 1}; range = |C|.
// vertex_only: the relaxed box of Supp. B (no pierce test, no stationary
// points on the edges), kept for comparison -- it can miss pixels.
__device__ BoxOut angular_box(const double A[3], const double B[3], const double C[3], double range, int H, int W,
                              const double2 *__restrict__ col, const double2 *__restrict__ rlo,
                              const double2 *__restrict__ rhi, double cm, double sm, bool vertex_only,
                              float fu, float cu, float fv, float cv)
{
    BoxOut o;
    o.nint = 0;
    bool full_az = false, to_top = false, to_bottom = false;
    // Does the z-axis meet the square?  With n = A x B (det = n_z) it meets the
    // plane at height (n.C)/det; all of the square lies within |C| + |A| + |B|
    // of the sensor.  E bounds the rounding of n.C and det; a case that the
    // rounding leaves open widens the box.
    double det = A[0] * B[1] - A[1] * B[0];
    double n0 = A[1] * B[2] - A[2] * B[1], n1 = A[2] * B[0] - A[0] * B[2];
    double sc = (n0 * C[0] + n1 * C[1]) + det * C[2];
    double an = sqrt((A[0] * A[0] + A[1] * A[1]) + A[2] * A[2]);
    double bn = sqrt((B[0] * B[0] + B[1] * B[1]) + B[2] * B[2]);
    double nn = sqrt((n0 * n0 + n1 * n1) + det * det);
    double Rb = (range + an) + bn;
    double E = 4e-15 * (an * bn);
    double as = fabs(sc);
    if (vertex_only) {
        // the relaxed box: no pierce test
    } else if (!(as > (1e-9 * Rb) * nn + E * range)) {
        full_az = to_top = to_bottom = true;      // sensor (nearly) in the square's plane
    } else if (as - E * range > Rb * (fabs(det) + E)) {
        // the axis meets the plane beyond the square, or never
    } else if (!(fabs(det) >= 1e-6 * nn)) {
        full_az = to_top = to_bottom = true;      // ill-conditioned solve
    } else {
        // where the z-axis crosses the square's plane, in splat units
        double a = (B[0] * C[1] - B[1] * C[0]) / det;
        double b = (A[1] * C[0] - A[0] * C[1]) / det;
        if (fabs(a) <= 1.0 + 1e-6 && fabs(b) <= 1.0 + 1e-6) {
            double zp = (C[2] + a * A[2]) + b * B[2];
            full_az = true;
            to_top = zp >= 0.0;
            to_bottom = zp <= 0.0;
        }
    }
    double V[4][3];
    const double sa[4] = {-1.0, 1.0, 1.0, -1.0};
    const double sb[4] = {-1.0, -1.0, 1.0, 1.0};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int r = 0; r < 3; ++r) V[k][r] = (C[r] + sa[k] * A[r]) + sb[k] * B[r];

    // elevation extremes over the boundary: vertices + one stationary point per edge
    double rmax = 0, zmax = 0, rmin = 0, zmin = 0;
    bool have = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double *P0 = V[k];
        const double *P1 = V[(k + 1) & 3];
        double dx = P1[0] - P0[0], dy = P1[1] - P0[1], dz = P1[2] - P0[2];
        double qd = P0[0] * dx + P0[1] * dy;
        double q2 = P0[0] * P0[0] + P0[1] * P0[1];
        double d2 = dx * dx + dy * dy;
        double den = dz * qd - P0[2] * d2;
        double cx[2], cy[2], cz[2];
        int nc = 1;
        cx[0] = P0[0]; cy[0] = P0[1]; cz[0] = P0[2];
        if (!vertex_only && den != 0.0) {
            double ts = (P0[2] * qd - dz * q2) / den;
            if (ts > 0.0 && ts < 1.0) {
                cx[1] = P0[0] + ts * dx; cy[1] = P0[1] + ts * dy; cz[1] = P0[2] + ts * dz;
                nc = 2;
            }
        }
        for (int c = 0; c < nc; ++c) {
            double r = sqrt(cx[c] * cx[c] + cy[c] * cy[c]), z = cz[c];
            if (!have) { rmax = rmin = r; zmax = zmin = z; have = true; continue; }
            if (elev_below(rmax, zmax, r, z)) { rmax = r; zmax = z; }
            if (elev_below(r, z, rmin, zmin)) { rmin = r; zmin = z; }
        }
    }
    // rows: elevation decreases with the row index
    // Row i has elevation (i + 1/2 - cv) / fv (fv < 0: decreasing with i); the
    // guesses invert that in FP32, the decisions are the exact FP64 tests.
    const float kMarginF = (float)kBoxMargin;
    int r0, r1;
    if (to_top) {
        r0 = 0;
    } else {  // first row with el_i - margin <= el_max
        const float el = atan2f((float)zmax, (float)rmax);
        r0 = first_true(guess_ceil(fv * (el + kMarginF) + cv - 0.5f, H), H, [&](int i) {
            const double2 e = rlo[i];
            return zmax * e.x - rmax * e.y >= 0.0;
        });
    }
    if (to_bottom) {
        r1 = H - 1;
    } else {  // last row with el_i + margin >= el_min
        const float el = atan2f((float)zmin, (float)rmin);
        r1 = first_true(guess_above(fv * (el - kMarginF) + cv - 0.5f, H), H, [&](int i) {
                 const double2 e = rhi[i];
                 return !(zmin * e.x - rmin * e.y <= 0.0);
             }) - 1;
    }
    if (r0 > r1) return o;
    o.r0 = r0; o.r1 = r1;

    if (!full_az) {
        int klo = 0, khi = 0;
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            if (xcross(V[klo][0], V[klo][1], V[k][0], V[k][1]) < 0.0) klo = k;
            if (xcross(V[khi][0], V[khi][1], V[k][0], V[k][1]) > 0.0) khi = k;
        }
        // widen the arc by the margin on both sides
        double lx = V[klo][0] * cm + V[klo][1] * sm, ly = V[klo][1] * cm - V[klo][0] * sm;
        double ux = V[khi][0] * cm - V[khi][1] * sm, uy = V[khi][0] * sm + V[khi][1] * cm;
        if (!(xcross(lx, ly, ux, uy) > 0.0)) {
            full_az = true;
        } else {
            // column j has azimuth (j + 1/2 - cu) / fu (fu < 0: decreasing with j)
            const float azu = atan2f((float)uy, (float)ux), azl = atan2f((float)ly, (float)lx);
            // first column with azimuth <= upper end
            const int jf = first_true(guess_ceil(fu * azu + cu - 0.5f, W), W, [&](int j) {
                const double2 d = col[j];
                return angle_le(d.x, d.y, ux, uy);
            });
            // last column with azimuth >= lower end
            const int jl = first_true(guess_above(fu * azl + cu - 0.5f, W), W, [&](int j) {
                               const double2 d = col[j];
                               return !angle_le(lx, ly, d.x, d.y);
                           }) - 1;
            if (angle_le(lx, ly, ux, uy)) {
                if (jf > jl) return o;
                o.c[0] = jf; o.c[1] = jl; o.c[2] = -1; o.c[3] = -1;
                o.nint = 1;
                return o;
            }
            int m = 0;  // the arc crosses the seam
            o.c[2] = -1; o.c[3] = -1;
            if (jl >= 0) { o.c[0] = 0; o.c[1] = jl; m = 1; }
            if (jf <= W - 1) { o.c[2 * m] = jf; o.c[2 * m + 1] = W - 1; ++m; }
            o.nint = m;
            return o;
        }
    }
    o.c[0] = 0; o.c[1] = W - 1; o.c[2] = -1; o.c[3] = -1;
    o.nint = 1;
    return o;
}

__device__ inline void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

__global__ void __launch_bounds__(256)
k_project(const FrameDesc *__restrict__ descs, const double2 *__restrict__ tables, double cm, double sm,
          RasterRec *__restrict__ rec, PixBox *__restrict__ box,
          uint32_t *__restrict__ keys, int32_t *__restrict__ counts, int box_mode,
          unsigned long long *__restrict__ n_invalid)
{
    const FrameDesc &fd = descs[blockIdx.y];
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= fd.n) return;
    const int64_t it = fd.item_off + k;
    const int H = fd.H, W = fd.W;
    const double2 *col = tables + fd.tab_off;
    const double2 *rlo = col + W + H;
    const double2 *rhi = rlo + H;
    float fm0 = fd.means[3 * k], fm1 = fd.means[3 * k + 1], fm2 = fd.means[3 * k + 2];
    float4 fq = *reinterpret_cast<const float4 *>(fd.quats + 4 * k);
    float fl0 = fd.lsc[2 * k], fl1 = fd.lsc[2 * k + 1], flg = fd.logits[k];
    bool fin = isfinite(fm0) && isfinite(fm1) && isfinite(fm2) && isfinite(fq.x) && isfinite(fq.y) &&
               isfinite(fq.z) && isfinite(fq.w) && isfinite(fl0) && isfinite(fl1) && isfinite(flg);
    double w = fq.x, x = fq.y, y = fq.z, z = fq.w;
    double qq = ((w * w + x * x) + y * y) + z * z;
    bool ok = fin && qq > 0.0;
    if (!ok) atomicAdd(n_invalid, 1ull);   // culled: a non-finite parameter or a zero quaternion (rare)
    double rad = 3.0;
    if (ok && box_mode == SLR_BOX_OPACITY) {
        rad = support_radius((double)flg);
        ok = rad > 0.0;
    }
    double R[9], t[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        R[3 * e] = fd.pose[4 * e]; R[3 * e + 1] = fd.pose[4 * e + 1]; R[3 * e + 2] = fd.pose[4 * e + 2];
        t[e] = fd.pose[4 * e + 3];
    }
    double A[3], B[3], C[3], N[3], ba[3], bb[3];
    double range = 0.0;
    if (ok) {
        double qn = sqrt(qq);
        w = w / qn; x = x / qn; y = y / qn; z = z / qn;
        double ta[3] = {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y)};
        double tb[3] = {2.0 * (x * y - w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z + w * x)};
        double tn[3] = {2.0 * (x * z + w * y), 2.0 * (y * z - w * x), 1.0 - 2.0 * (x * x + y * y)};
        double s3a = rad * box_exp((double)fl0), s3b = rad * box_exp((double)fl1);
        double Aw[3] = {s3a * ta[0], s3a * ta[1], s3a * ta[2]};
        double Bw[3] = {s3b * tb[0], s3b * tb[1], s3b * tb[2]};
        // the splat axes themselves (independent of the box's half-side, so that
        // every box mode composites identical records)
        double sa1 = box_exp((double)fl0), sb1 = box_exp((double)fl1);
        double Au[3] = {sa1 * ta[0], sa1 * ta[1], sa1 * ta[2]};
        double Bu[3] = {sb1 * tb[0], sb1 * tb[1], sb1 * tb[2]};
        double m0 = fm0, m1 = fm1, m2 = fm2;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double *Rr = R + 3 * r;
            A[r] = (Rr[0] * Aw[0] + Rr[1] * Aw[1]) + Rr[2] * Aw[2];
            B[r] = (Rr[0] * Bw[0] + Rr[1] * Bw[1]) + Rr[2] * Bw[2];
            C[r] = ((Rr[0] * m0 + Rr[1] * m1) + Rr[2] * m2) + t[r];
            N[r] = (Rr[0] * tn[0] + Rr[1] * tn[1]) + Rr[2] * tn[2];
            ba[r] = (Rr[0] * Au[0] + Rr[1] * Au[1]) + Rr[2] * Au[2];
            bb[r] = (Rr[0] * Bu[0] + Rr[1] * Bu[1]) + Rr[2] * Bu[2];
        }
        range = sqrt((C[0] * C[0] + C[1] * C[1]) + C[2] * C[2]);
        ok = range > fd.near_m;
    }
    BoxOut bx;
    bx.nint = 0;
    if (ok)
        bx = angular_box(A, B, C, range, H, W, col, rlo, rhi, cm, sm, box_mode == SLR_BOX_VERTEX, (float)fd.fu,
                         (float)fd.cu, (float)fd.fv, (float)fd.cv);
    int32_t cnt = 0;
    PixBox pb = {-1, -1, -1, -1, -1, -1, (int16_t)blockIdx.y, 0};
    if (bx.nint > 0) {
        const int th = fd.th, tw = fd.tw;
        int ty0 = bx.r0 / th, ty1 = bx.r1 / th;
        int ax0 = bx.c[0] / tw, ax1 = bx.c[1] / tw;
        int nr = 1, bx0 = 0, bx1 = -1;
        if (bx.nint == 2) {
            bx0 = bx.c[2] / tw; bx1 = bx.c[3] / tw;
            if (bx0 <= ax1) { ax1 = bx1 > ax1 ? bx1 : ax1; }
            else nr = 2;
        }
        cnt = (ax1 - ax0 + 1) * (ty1 - ty0 + 1);
        if (nr == 2) cnt += (bx1 - bx0 + 1) * (ty1 - ty0 + 1);
        pb.r0 = (int16_t)bx.r0; pb.r1 = (int16_t)bx.r1;
        pb.c0 = (int16_t)bx.c[0]; pb.c1 = (int16_t)bx.c[1];
        pb.c2 = (int16_t)(bx.nint == 2 ? bx.c[2] : -1); pb.c3 = (int16_t)(bx.nint == 2 ? bx.c[3] : -1);
    }
    counts[it] = cnt;
    pb.cnt = (uint16_t)cnt;
    box[it] = pb;
    if (cnt == 0) {
        keys[it] = 0xFFFFFFFFu;
        return;
    }
    float key = (float)range;
    keys[it] = __float_as_uint(key);

    // compositing record: b_alpha, b_beta, b_c = C
    RasterRec rr;
    cross3(bb, C, rr.P);
    cross3(C, ba, rr.Q);
    cross3(ba, bb, rr.M);
    rr.tau = (float)((C[0] * rr.M[0] + C[1] * rr.M[1]) + C[2] * rr.M[2]);
    rr.opac = 1.0f / (1.0f + expf(-flg));
    rr.n[0] = (float)N[0]; rr.n[1] = (float)N[1]; rr.n[2] = (float)N[2];
    rr.rows = (uint32_t)bx.r0 | ((uint32_t)bx.r1 << 16);
    rec[it] = rr;
}

// Descriptor upload through kernel arguments (no host buffer outlives the call).
constexpr int kDescPerLaunch = 8;
struct DescPack {
    FrameDesc d[kDescPerLaunch];
};
__global__ void k_write_desc(DescPack pack, int count, FrameDesc *__restrict__ dst)
{
    const int i = threadIdx.x;
    if (i < count) dst[i] = pack.d[i];
}

// Frame index of every global tile.
__global__ void __launch_bounds__(256)
k_tile_frame(const FrameDesc *__restrict__ descs, int32_t *__restrict__ tile_frame)
{
    const FrameDesc &fd = descs[blockIdx.y];
    const int nt = fd.tiles_x * fd.tiles_y;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x)
        tile_frame[fd.tile_off + t] = (int32_t)blockIdx.y;
}

}  // namespace

void launch_write_desc(const FrameDesc *host_descs, int32_t count, FrameDesc *dev, hipStream_t stream)
{
    for (int32_t b = 0; b < count; b += kDescPerLaunch) {
        DescPack pack;
        const int c = count - b < kDescPerLaunch ? count - b : kDescPerLaunch;
        for (int i = 0; i < c; ++i) pack.d[i] = host_descs[b + i];
        hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(kDescPerLaunch), 0, stream, pack, c, dev + b);
    }
}

void launch_tile_frame(const Layout &L, char *ws, hipStream_t stream)
{
    hipLaunchKernelGGL(k_tile_frame, dim3(8, L.frames), dim3(256), 0, stream,
                       reinterpret_cast<const FrameDesc *>(ws + L.desc), reinterpret_cast<int32_t *>(ws + L.tile_frame));
}

void launch_project(const Layout &L, char *ws, int64_t max_n, hipStream_t stream)
{
    launch_fill_u32(ws + L.misc + kMiscInvalid, 0u, 2, stream);
    if (max_n <= 0 || L.frames == 0) return;
    const int blocks = (int)((max_n + 255) / 256);
    hipLaunchKernelGGL(k_project, dim3(blocks, L.frames), dim3(256), 0, stream,
                       reinterpret_cast<const FrameDesc *>(ws + L.desc), reinterpret_cast<const double2 *>(ws + L.tables),
                       cos(kBoxMargin), sin(kBoxMargin), reinterpret_cast<RasterRec *>(ws + L.rec),
                       reinterpret_cast<PixBox *>(ws + L.box),
                       reinterpret_cast<uint32_t *>(ws + L.skey),
                       reinterpret_cast<int32_t *>(ws + L.cnt), (int)L.box_mode,
                       reinterpret_cast<unsigned long long *>(ws + L.misc + kMiscInvalid));
}

}  // namespace slr

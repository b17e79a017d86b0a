// raster.hip -- per-tile front-to-back compositing and its reverse-order
// backward (Sec. 3.2.1-3.2.2, Supp. D) on gfx950.
//
// One 256-thread workgroup per tile, one pixel per thread.  The tile's
// range-sorted list is staged through LDS in batches; every wave reads each
// staged record with broadcast LDS loads and skips, as a whole, records whose
// pixel-row interval misses the wave's rows.
//
// Intersection (Cramer form of the plane-pair solve): with the FP64 pixel ray
// v, a = P.v, b = Q.v, c = M.v give s_hat = (a, b) / c and the ray range
// t = tau / c.  The three dot products run in FP64 (CDNA4 issues FP64 FMA at
// the rate of unpacked FP32 FMA) because they cancel: far, small surfels
// would otherwise lose most FP32 digits of s_hat.  Everything after them runs
// in FP32.
//
// Backward: each pixel walks its list from the last contributor to the first,
// recovering the transmittance before each pair by division, keeping the
// suffix sums of the depth and normal channels.  With a = P.v, b = Q.v,
// c = M.v, the gradient w.r.t. the splat axes is, per pair,
//   g_alpha = db (v x b_c) + dc_s (b_beta x v) + (g_t/c) s_alpha M
//   g_beta  = da (b_c x v) + dc_s (v x b_alpha) + (g_t/c) s_beta M
//   g_c     = da (v x b_beta) + db (b_alpha x v) + (g_t/c) M
// (da, db, dc_s: dL/da, dL/db, dL/dc through s_hat; g_t = dL/d(range); the
// range path is folded in closed form, t v - b_c = s_alpha b_alpha +
// s_beta b_beta).  The sums over pixels are rebuilt from 18 per-pair partials:
// da (v - c_hat), db (v - c_hat), dc_s v, da, db, (g_t/c)(s_alpha, s_beta, 1),
// dL/do, dL/dn, where c_hat = b_c / |b_c|; subtracting c_hat in FP64 before
// rounding keeps the products with the long vector b_c free of cancellation.
// The partials are summed over the wave with DPP row shifts and broadcasts,
// then over the block's waves in LDS; one thread per record assembles the
// splat-axis gradients in FP64, adds the pose-gradient contribution, rotates
// to the world frame and issues the atomics.
#include "slr_internal.h"

#pragma clang fp contract(off)

namespace slr {
namespace {

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kNegHalfLog2e = -0.72134752044448170f;  // -1 / (2 ln 2)
// A wave with at most this many unfinished pixels walks the rest of its list
// one pixel at a time with 64 records per step (see k_raster_fwd).
constexpr int kStragglers = 16;

__device__ __forceinline__ float bcast(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int bcast(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double bcast(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

struct PairEval {
    float sa, sb, t, rc, G, alpha;
    bool clamped;
    double c;   // M.v in FP64 (the backward refines the range with it)
};

// Shared by forward and backward so both take identical decisions.
__device__ __forceinline__ bool eval_pair(const RasterRec &r, double vx, double vy, double vz, float near_m,
                                          PairEval &e)
{
    const double a = fma(r.P[2], vz, fma(r.P[1], vy, r.P[0] * vx));
    const double b = fma(r.Q[2], vz, fma(r.Q[1], vy, r.Q[0] * vx));
    const double c = fma(r.M[2], vz, fma(r.M[1], vy, r.M[0] * vx));
    const float af = (float)a, bf = (float)b, cf = (float)c;
    const float lim = 3.0f * fabsf(cf);
    if (!(fabsf(af) <= lim && fabsf(bf) <= lim && cf != 0.0f)) return false;
    const float rc = __builtin_amdgcn_rcpf(cf);
    const float t = r.tau * rc;
    if (!(t > near_m)) return false;
    const float sa = af * rc, sb = bf * rc;
    const float q = fmaf(sa, sa, sb * sb);
    const float G = __builtin_amdgcn_exp2f(kNegHalfLog2e * q);
    const float ag = r.opac * G;
    if (ag < kAlphaMin) return false;
    e.sa = sa; e.sb = sb; e.t = t; e.rc = rc; e.G = G; e.c = c;
    e.clamped = ag > kAlphaMax;
    e.alpha = e.clamped ? kAlphaMax : ag;
    return true;
}

// The same arithmetic as eval_pair without control flow: every quantity is
// computed and the returned flag says whether the pair contributes, so two
// pairs can be evaluated side by side; where it returns true, e holds exactly
// the values eval_pair gives.
__device__ __forceinline__ bool eval_pair_flat(const RasterRec &r, double vx, double vy, double vz, float near_m,
                                               PairEval &e)
{
    const double a = fma(r.P[2], vz, fma(r.P[1], vy, r.P[0] * vx));
    const double b = fma(r.Q[2], vz, fma(r.Q[1], vy, r.Q[0] * vx));
    const double c = fma(r.M[2], vz, fma(r.M[1], vy, r.M[0] * vx));
    const float af = (float)a, bf = (float)b, cf = (float)c;
    const float lim = 3.0f * fabsf(cf);
    const bool sup = fabsf(af) <= lim && fabsf(bf) <= lim && cf != 0.0f;
    const float rc = __builtin_amdgcn_rcpf(cf);
    const float t = r.tau * rc;
    const float sa = af * rc, sb = bf * rc;
    const float q = fmaf(sa, sa, sb * sb);
    const float G = __builtin_amdgcn_exp2f(kNegHalfLog2e * q);
    const float ag = r.opac * G;
    e.sa = sa; e.sb = sb; e.t = t; e.rc = rc; e.G = G; e.c = c;
    e.clamped = ag > kAlphaMax;
    e.alpha = e.clamped ? kAlphaMax : ag;
    return sup && (t > near_m) && !(ag < kAlphaMin);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v)
{
    int s = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false);
    return v + __int_as_float(s);
}

template <int CTRL>
__device__ __forceinline__ float dpp_perm(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// x + y after lanes 32..63 of x are exchanged with lanes 0..31 of y
// (v_permlane32_swap): lanes 0..31 hold x's half sums, lanes 32..63 y's.
__device__ __forceinline__ float fold32(float x, float y)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// x + y after the odd 16-lane rows of x are exchanged with the even rows of y
// (v_permlane16_swap): rows 0, 2 hold x's row-pair sums, rows 1, 3 y's.
__device__ __forceinline__ float fold16(float x, float y)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Within every group of 2*BIT lanes: the low half keeps x's pair sums, the high
// half y's; the partner lane comes from the DPP permutation CTRL (a mirror or
// quad permutation that maps each half onto the other).
template <int BIT, int CTRL>
__device__ __forceinline__ float fold_lanes(float x, float y, int lane)
{
    const bool hi = (lane & BIT) != 0;
    const float s = hi ? y : x, t = hi ? x : y;
    return s + dpp_perm<CTRL>(t);
}

// Wave sums of 18 per-lane values by a transposed butterfly: each stage halves
// the lanes a value spans and packs two values into one register, so the 18
// sums cost 43 VALU operations instead of six DPP steps per value.  On return
// lane l holds the sum of value bitrev6(l) for bitrev6(l) < 18 (all 64 lanes
// must be active).
__device__ __forceinline__ float wave_sum18(const float (&g)[18], int lane)
{
    float z[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) z[m] = fold32(g[2 * m], g[2 * m + 1]);
    float w[5];
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = fold16(z[2 * q], z[2 * q + 1]);
    w[4] = fold16(z[8], 0.0f);
    const float u0 = fold_lanes<8, 0x140>(w[0], w[1], lane);  // row_mirror
    const float u1 = fold_lanes<8, 0x140>(w[2], w[3], lane);
    const float u2 = w[4] + dpp_perm<0x140>(w[4]);
    const float v0 = fold_lanes<4, 0x141>(u0, u1, lane);      // row_half_mirror
    const float v1 = u2 + dpp_perm<0x141>(u2);
    const float r = fold_lanes<2, 0x4e>(v0, v1, lane);        // quad_perm [2,3,0,1]
    return r + dpp_perm<0xb1>(r);                             // quad_perm [1,0,3,2]
}

__device__ __forceinline__ int bitrev6(int l) { return (int)(__builtin_bitreverse32((uint32_t)l) >> 26); }

__global__ void __launch_bounds__(256)
k_raster_fwd(const FrameDesc *__restrict__ descs, const int32_t *__restrict__ tile_frame,
             const uint32_t *__restrict__ order,
             const RasterRec *__restrict__ rec, const uint32_t *__restrict__ pval, const int2 *__restrict__ ranges,
             const double2 *__restrict__ tables, float *__restrict__ stT_all, int32_t *__restrict__ stN_all,
             int32_t *__restrict__ census_all, int64_t total_pixels)
{
    __shared__ RasterRec srec[256];
    __shared__ __align__(4) uint8_t slist[4][256];
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const FrameDesc &fd = descs[tile_frame[tile]];
    // the frame's tile shape: TH x TW = 256 pixels, TW a power of two
    const int TW = fd.tw, TH = fd.th, tws = __builtin_ctz((unsigned)fd.tw);
    const int H = fd.H, W = fd.W, tiles_x = fd.tiles_x;
    const float near_m = (float)fd.near_m;
    const double2 *col = tables + fd.tab_off, *rowc = col + W;
    float *depth = fd.depth, *normal = fd.normal, *alpha = fd.alpha;
    float *stT = stT_all + fd.pix_off;
    int32_t *stN = stN_all + fd.pix_off;
    int32_t *census = census_all + fd.pix_off;
    const int ltile = tile - fd.tile_off;
    const int ty = ltile / tiles_x, tx = ltile - ty * tiles_x;
    const int lx = threadIdx.x & (TW - 1), ly = threadIdx.x >> tws;
    const int i = ty * TH + ly, j = tx * TW + lx;
    const bool inside = (i < H) && (j < W);
    const double2 cr = rowc[min(i, H - 1)], cc = col[min(j, W - 1)];
    const double vx = cr.x * cc.x, vy = cr.x * cc.y, vz = cr.y;
    const int2 rg = ranges[tile];
    const int wid = threadIdx.x >> 6;
    const int wr0 = ty * TH + ((wid * 64) >> tws), wr1 = ty * TH + ((wid * 64 + 63) >> tws);
    float T = 1.0f, D = 0.0f, N0 = 0.0f, N1 = 0.0f, N2 = 0.0f, O = 0.0f;
    int last = 0, n_eval = 0, n_con = 0;
    bool done = !inside;
    const int lane = threadIdx.x & 63;
    for (int b0 = rg.x; b0 < rg.y; b0 += 256) {
        if (__syncthreads_count(!done) == 0) break;
        const int idx = b0 + threadIdx.x;
        if (idx < rg.y) srec[threadIdx.x] = rec[pval[idx]];
        __syncthreads();
        const int cnt = min(256, rg.y - b0);
        // the batch's records whose pixel rows meet this wave's rows, in list order
        int nact = 0;
        for (int base = 0; base < cnt; base += 64) {
            const int k = base + lane;
            bool meets = false;
            if (k < cnt) {
                const uint32_t rows = srec[k].rows;
                meets = !((int)(rows >> 16) < wr0 || (int)(rows & 0xffffu) > wr1);
            }
            const uint64_t m = __ballot(meets);
            if (meets) slist[wid][nact + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = (uint8_t)k;
            nact += __popcll(m);
        }
        __syncthreads();
        // two records per step: both evaluations are independent, the blends
        // then follow in list order
        int q = 0;
        for (; q < nact; q += 2) {
            const uint64_t live = __ballot(!done);
            if (live == 0 || __popcll(live) <= kStragglers) break;
            // q is even: both slots come in one 16-bit read
            const uint32_t two = *reinterpret_cast<const uint16_t *>(&slist[wid][q]);
            const int k0 = (int)(two & 0xffu);
            const bool has1 = q + 1 < nact;
            const int k1 = has1 ? (int)(two >> 8) : k0;
            PairEval e0, e1;
            const bool ok0 = eval_pair_flat(srec[k0], vx, vy, vz, near_m, e0);
            const bool ok1 = eval_pair_flat(srec[k1], vx, vy, vz, near_m, e1) && has1;
            if (!done) {
                ++n_eval;
                if (ok0) {
                    const float tT = T * (1.0f - e0.alpha);
                    if (tT < kTMin) {
                        done = true;
                    } else {
                        const float w = e0.alpha * T;
                        D = fmaf(w, e0.t, D);
                        N0 = fmaf(w, srec[k0].n[0], N0);
                        N1 = fmaf(w, srec[k0].n[1], N1);
                        N2 = fmaf(w, srec[k0].n[2], N2);
                        O += w;
                        T = tT;
                        last = b0 + k0 + 1 - rg.x;
                        ++n_con;
                    }
                }
            }
            if (has1 && !done) {
                ++n_eval;
                if (ok1) {
                    const float tT = T * (1.0f - e1.alpha);
                    if (tT < kTMin) {
                        done = true;
                    } else {
                        const float w = e1.alpha * T;
                        D = fmaf(w, e1.t, D);
                        N0 = fmaf(w, srec[k1].n[0], N0);
                        N1 = fmaf(w, srec[k1].n[1], N1);
                        N2 = fmaf(w, srec[k1].n[2], N2);
                        O += w;
                        T = tT;
                        last = b0 + k1 + 1 - rg.x;
                        ++n_con;
                    }
                }
            }
        }
        // Few unfinished pixels left: each of them in turn takes the wave, whose
        // lanes evaluate 64 consecutive list entries for that pixel's ray; the
        // contributing entries are then blended in list order with the same
        // arithmetic as above, so the result does not depend on the mode.
        uint64_t live = q < nact ? __ballot(!done) : 0ull;
        while (live) {
            const int pl = (int)__builtin_ctzll(live);
            live &= live - 1;
            const double pvx = bcast(vx, pl), pvy = bcast(vy, pl), pvz = bcast(vz, pl);
            float sT = bcast(T, pl), sD = bcast(D, pl), sN0 = bcast(N0, pl), sN1 = bcast(N1, pl),
                  sN2 = bcast(N2, pl), sO = bcast(O, pl);
            int sLast = bcast(last, pl), sEval = 0, sCon = 0;
            bool sDone = false;
            for (int c = q; c < nact && !sDone; c += 64) {
                const int e = c + lane;
                const bool in = e < nact;
                const int k = slist[wid][in ? e : c];
                PairEval ev;
                const bool ok = eval_pair_flat(srec[k], pvx, pvy, pvz, near_m, ev) && in;
                uint64_t cm = __ballot(ok);
                int counted = min(64, nact - c);
                while (cm) {
                    const int jl = (int)__builtin_ctzll(cm);
                    cm &= cm - 1;
                    const float a = bcast(ev.alpha, jl), tj = bcast(ev.t, jl);
                    const int kj = bcast(k, jl);
                    const float tT = sT * (1.0f - a);
                    if (tT < kTMin) {
                        sDone = true;
                        counted = jl + 1;
                        break;
                    }
                    const float w = a * sT;
                    sD = fmaf(w, tj, sD);
                    sN0 = fmaf(w, srec[kj].n[0], sN0);
                    sN1 = fmaf(w, srec[kj].n[1], sN1);
                    sN2 = fmaf(w, srec[kj].n[2], sN2);
                    sO += w;
                    sT = tT;
                    sLast = b0 + kj + 1 - rg.x;
                    ++sCon;
                }
                sEval += counted;
            }
            if (lane == pl) {
                T = sT; D = sD; N0 = sN0; N1 = sN1; N2 = sN2; O = sO;
                last = sLast; n_eval += sEval; n_con += sCon; done = sDone;
            }
        }
    }
    if (inside) {
        const int p = i * W + j;
        census[p] = n_eval;
        census[total_pixels + p] = n_con;
        depth[p] = D;
        alpha[p] = O;
        normal[3 * p] = N0; normal[3 * p + 1] = N1; normal[3 * p + 2] = N2;
        stT[p] = T;
        stN[p] = last;
    }
}

// Strip and tile slot of a one-wave workgroup.  Each run of 32 workgroups
// covers 8 tile slots x 4 strips, arranged so that the 4 strips of a tile
// have the same workgroup index modulo 8: workgroups are handed to the 8 XCDs
// in turn, so a tile's strips share one XCD's L2 for the tile's records.
// Returns false for the padding workgroups past the last tile.
// Contribution mask: one bit per (strip, list entry), set by the one-wave
// forward when some pixel of the strip composited the entry.  Word w of the
// 64-entry chunks of tile t's list, strip s, sits at 4 (floor(start / 64) + t
// + w) + s (start = the tile's first pair): tiles never share a word.
__host__ __device__ inline int64_t cmask_word(int tile, int start, int strip, int chunk)
{
    return 4 * ((int64_t)(start >> 6) + tile + chunk) + strip;
}

// OR of a 64-bit value over the wave (every lane gets the result).
__device__ __forceinline__ uint64_t wave_or64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)v, o, 64), hi = __shfl_xor((uint32_t)(v >> 32), o, 64);
        v |= ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// Whether some strip of the tile composited list entry pos (true without a mask).
__device__ __forceinline__ bool any_strip_wants(const uint64_t *cmask, int tile, int start, int pos)
{
    if (!cmask) return true;
    const uint64_t *w = cmask + cmask_word(tile, start, 0, pos >> 6);
    return (((w[0] | w[1] | w[2] | w[3]) >> (pos & 63)) & 1ull) != 0;
}

// A mask word (wave-uniform) in scalar registers; all ones without a mask.
__device__ __forceinline__ uint64_t mask_word(const uint64_t *cm, int idx)
{
    if (!cm) return ~0ull;
    const uint64_t w = cm[idx];
    return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(w >> 32)) << 32) |
           (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)w);
}

__device__ __forceinline__ bool strip_of_block(int64_t ntiles, int &strip, int &tslot)
{
    const int j = (int)(blockIdx.x & 31u);
    strip = j >> 3;
    tslot = (int)(blockIdx.x >> 5) * 8 + (j & 7);
    return tslot < ntiles;
}

// Forward, one wave per 64-pixel strip of a tile (a tile's strips are
// independent workgroups: no workgroup barrier, and the strips of a long list
// run on different compute units).  The list is read in chunks of 64 records,
// one per lane, with the next chunk's loads in flight while the current one is
// composited.  While the wave has many unfinished pixels, the chunk's records
// that meet the strip's rows are compacted into LDS and every lane composites
// its own pixel against them, two at a time; with few unfinished pixels left,
// each of them in turn takes the wave and the lanes evaluate their own
// records for that pixel.  Same arithmetic and order as k_raster_fwd, hence
// bit-identical results.
// Quad mode of the one-wave forward, for the longest lists: the wave takes 16
// pixels of the tile (a sub-strip: pixels 16 sub .. 16 sub + 15 in row-major
// tile order), four lanes per pixel (lane = 4 pixel + slot).  The chunk's
// records that meet the sub-strip's rows are compacted as in the strip mode;
// each step the four lanes of a pixel evaluate four consecutive compacted
// records for that pixel's ray, and all four blend the four results in list
// order (the values travel by DPP quad broadcasts).  A strip of a long list is
// thus walked by four waves at a quarter of the records each, and each walks
// only the records that meet its fewer rows.  Same evaluation and blending
// arithmetic in the same order as the strip mode: identical images and state.
__device__ __forceinline__ void fwd_quad(const FrameDesc &fd, int tile, int sub, const RasterRec *__restrict__ rec,
                                         const uint32_t *__restrict__ pval, const int2 *__restrict__ ranges,
                                         const double2 *__restrict__ tables, float *__restrict__ stT_all,
                                         int32_t *__restrict__ stN_all, int32_t *__restrict__ census_all,
                                         int64_t total_pixels, uint64_t *__restrict__ cmask, RasterRec *sbuf,
                                         uint8_t *sidx)
{
    const int TW = fd.tw, TH = fd.th, tws = __builtin_ctz((unsigned)fd.tw);
    const int H = fd.H, W = fd.W, tiles_x = fd.tiles_x;
    const float near_m = (float)fd.near_m;
    const double2 *col = tables + fd.tab_off, *rowc = col + W;
    const int ltile = tile - fd.tile_off;
    const int ty = ltile / tiles_x, tx = ltile - ty * tiles_x;
    const int lane = threadIdx.x, px = lane >> 2, slot = lane & 3;
    const int q16 = 16 * sub + px;   // pixel index within the tile, row-major
    const int i = ty * TH + (q16 >> tws), j = tx * TW + (q16 & (TW - 1));
    const bool inside = (i < H) && (j < W);
    const double2 cr = rowc[min(i, H - 1)], cc = col[min(j, W - 1)];
    const double vx = cr.x * cc.x, vy = cr.x * cc.y, vz = cr.y;
    const int2 rg = ranges[tile];
    const int wr0 = ty * TH + ((16 * sub) >> tws), wr1 = ty * TH + ((16 * sub + 15) >> tws);
    float T = 1.0f, D = 0.0f, N0 = 0.0f, N1 = 0.0f, N2 = 0.0f, O = 0.0f;
    int last = 0, n_eval = 0, n_con = 0;
    bool done = !inside;
    // the words of the strip holding this sub-strip (its four sub-strips OR into them)
    uint64_t *cm = cmask ? cmask + cmask_word(tile, rg.x, sub >> 2, 0) : nullptr;
    // list entry c + lane travels as six 16-byte words in registers (a record
    // copied as a struct would be placed in scratch memory)
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    u32x4 nrec[6];
    if (rg.x + lane < rg.y) {
        const u32x4 *src = reinterpret_cast<const u32x4 *>(rec + pval[rg.x + lane]);
#pragma unroll
        for (int f = 0; f < 6; ++f) nrec[f] = src[f];
    }
    for (int c = rg.x; c < rg.y; c += 64) {
        if (__ballot(!done) == 0) break;
        const bool inchunk = c + lane < rg.y;
        bool meets = false;
        if (inchunk) {
            const uint32_t rows = nrec[5].w;
            meets = !((int)(rows >> 16) < wr0 || (int)(rows & 0xffffu) > wr1);
        }
        const uint64_t m = __ballot(meets);
        const int nact = __popcll(m);
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (meets) {
            u32x4 *dst = reinterpret_cast<u32x4 *>(&sbuf[rank]);
#pragma unroll
            for (int f = 0; f < 6; ++f) dst[f] = nrec[f];
            sidx[rank] = (uint8_t)lane;
        }
        // the next chunk's loads go out once this one is staged
        __builtin_amdgcn_sched_barrier(0);
        if (c + 64 + lane < rg.y) {
            const u32x4 *src = reinterpret_cast<const u32x4 *>(rec + pval[c + 64 + lane]);
#pragma unroll
            for (int f = 0; f < 6; ++f) nrec[f] = src[f];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint64_t contrib = 0;   // chunk entries this lane's pixel composited
        for (int q = 0; q < nact; q += 4) {
            if (__ballot(!done) == 0) break;
            const int k = q + slot;
            PairEval e;
            const bool ok = eval_pair_flat(sbuf[min(k, nact - 1)], vx, vy, vz, near_m, e) && k < nact;
            const uint32_t okq = (uint32_t)(__ballot(ok) >> (lane & ~3)) & 0xfu;
            const float a4[4] = {dpp_perm<0x00>(e.alpha), dpp_perm<0x55>(e.alpha), dpp_perm<0xAA>(e.alpha),
                                 dpp_perm<0xFF>(e.alpha)};
            const float t4[4] = {dpp_perm<0x00>(e.t), dpp_perm<0x55>(e.t), dpp_perm<0xAA>(e.t), dpp_perm<0xFF>(e.t)};
            const int nu = min(4, nact - q);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u < nu && !done) {
                    ++n_eval;
                    if ((okq >> u) & 1u) {
                        const float tT = T * (1.0f - a4[u]);
                        if (tT < kTMin) {
                            done = true;
                        } else {
                            const float w = a4[u] * T;
                            D = fmaf(w, t4[u], D);
                            N0 = fmaf(w, sbuf[q + u].n[0], N0);
                            N1 = fmaf(w, sbuf[q + u].n[1], N1);
                            N2 = fmaf(w, sbuf[q + u].n[2], N2);
                            O += w;
                            T = tT;
                            const int su = sidx[q + u];
                            last = c + su + 1 - rg.x;
                            ++n_con;
                            contrib |= 1ull << su;
                        }
                    }
                }
            }
        }
        if (cm) {
            contrib = wave_or64(contrib);
            if (lane == 0 && contrib)
                atomicOr(reinterpret_cast<unsigned long long *>(cm + 4 * ((c - rg.x) >> 6)), (unsigned long long)contrib);
        }
        __builtin_amdgcn_wave_barrier();   // sbuf is rewritten by the next chunk
    }
    if (inside && slot == 0) {
        const int p = i * W + j;
        census_all[fd.pix_off + p] = n_eval;
        census_all[total_pixels + fd.pix_off + p] = n_con;
        fd.depth[p] = D;
        fd.alpha[p] = O;
        fd.normal[3 * p] = N0; fd.normal[3 * p + 1] = N1; fd.normal[3 * p + 2] = N2;
        stT_all[fd.pix_off + p] = T;
        stN_all[fd.pix_off + p] = last;
    }
}

// Work of a one-wave forward workgroup.  The first 16 * nquad workgroups take
// the nquad longest tiles (the first slots of the longest-first order) in quad
// mode, 16 sub-strips each, in runs of 128 = 8 tiles x 16 sub-strips arranged
// so that a tile's sub-strips share one XCD (see strip_of_block); the rest take
// one 64-pixel strip of the remaining tiles each.  Returns 0 for padding
// workgroups, 1 for a strip (strip, tslot), 2 for a sub-strip (sub, tslot).
__device__ __forceinline__ int fwd_work_of_block(int64_t b, int64_t ntiles, int64_t nquad, int &part, int &tslot)
{
    if (b < 16 * nquad) {
        const int j = (int)(b & 127);
        part = j >> 3;
        tslot = (int)(b >> 7) * 8 + (j & 7);
        return 2;
    }
    const int64_t b2 = b - 16 * nquad;
    const int j = (int)(b2 & 31);
    part = j >> 3;
    tslot = (int)nquad + (int)(b2 >> 5) * 8 + (j & 7);
    return tslot < ntiles ? 1 : 0;
}

// One work item of the one-wave forward (a strip, a quad sub-strip or padding);
// item b is what workgroup b of the plain grid takes.
__device__ __forceinline__ void fwd_w_item(int64_t b, const FrameDesc *__restrict__ descs,
                                           const int32_t *__restrict__ tile_frame, const uint32_t *__restrict__ order,
                                           const RasterRec *__restrict__ rec, const uint32_t *__restrict__ pval,
                                           const int2 *__restrict__ ranges, const double2 *__restrict__ tables,
                                           float *__restrict__ stT_all, int32_t *__restrict__ stN_all,
                                           int32_t *__restrict__ census_all, int64_t total_pixels, int64_t ntiles,
                                           int64_t nquad, uint64_t *__restrict__ cmask, RasterRec *sbuf,
                                           uint8_t *sidx)
{
    int strip, tslot;
    const int kind = fwd_work_of_block(b, ntiles, nquad, strip, tslot);
    if (kind == 0) return;
    if (kind == 2) {
        const int qt = (int)order[tslot];
        fwd_quad(descs[tile_frame[qt]], qt, strip, rec, pval, ranges, tables, stT_all, stN_all, census_all,
                 total_pixels, cmask, sbuf, sidx);
        return;
    }
    const int tile = order ? (int)order[tslot] : tslot;
    const FrameDesc &fd = descs[tile_frame[tile]];
    // the frame's tile shape: TH x TW = 256 pixels, TW a power of two, strips of SR rows
    const int TW = fd.tw, TH = fd.th, tws = __builtin_ctz((unsigned)fd.tw), SR = 64 >> tws;
    const int H = fd.H, W = fd.W, tiles_x = fd.tiles_x;
    const float near_m = (float)fd.near_m;
    const double2 *col = tables + fd.tab_off, *rowc = col + W;
    float *depth = fd.depth, *normal = fd.normal, *alpha = fd.alpha;
    float *stT = stT_all + fd.pix_off;
    int32_t *stN = stN_all + fd.pix_off;
    int32_t *census = census_all + fd.pix_off;
    const int ltile = tile - fd.tile_off;
    const int ty = ltile / tiles_x, tx = ltile - ty * tiles_x;
    const int lane = threadIdx.x;
    const int i = ty * TH + strip * SR + (lane >> tws), j = tx * TW + (lane & (TW - 1));
    const bool inside = (i < H) && (j < W);
    const double2 cr = rowc[min(i, H - 1)], cc = col[min(j, W - 1)];
    const double vx = cr.x * cc.x, vy = cr.x * cc.y, vz = cr.y;
    const int2 rg = ranges[tile];
    const int wr0 = ty * TH + strip * SR, wr1 = wr0 + SR - 1;
    float T = 1.0f, D = 0.0f, N0 = 0.0f, N1 = 0.0f, N2 = 0.0f, O = 0.0f;
    int last = 0, n_eval = 0, n_con = 0;
    bool done = !inside;
    // this strip's words of the contribution mask (one bit per list entry)
    uint64_t *cm = cmask ? cmask + cmask_word(tile, rg.x, strip, 0) : nullptr;
    RasterRec nxt;
    if (rg.x + lane < rg.y) nxt = rec[pval[rg.x + lane]];
    for (int c = rg.x; c < rg.y; c += 64) {
        uint64_t live = __ballot(!done);
        if (live == 0) break;
        const RasterRec r = nxt;   // list entry c + lane
        const bool inchunk = c + lane < rg.y;
        if (c + 64 + lane < rg.y) nxt = rec[pval[c + 64 + lane]];
        bool meets = false;
        if (inchunk) {
            const uint32_t rows = r.rows;
            meets = !((int)(rows >> 16) < wr0 || (int)(rows & 0xffffu) > wr1);
        }
        const uint64_t m = __ballot(meets);
        const int nact = __popcll(m);
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        int q = 0;
        uint64_t contrib = 0;   // chunk entries composited by some pixel of the strip (few-pixels mode)
        uint64_t mine = 0;      // chunk entries this lane's pixel composited (many-pixels mode)
        if (__popcll(live) > kStragglers) {
            if (meets) { sbuf[rank] = r; sidx[rank] = (uint8_t)lane; }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (; q < nact; q += 2) {
                live = __ballot(!done);
                if (live == 0 || __popcll(live) <= kStragglers) break;
                const bool has1 = q + 1 < nact;
                const int k0 = q, k1 = has1 ? q + 1 : q;
                PairEval e0, e1;
                const bool ok0 = eval_pair_flat(sbuf[k0], vx, vy, vz, near_m, e0);
                const bool ok1 = eval_pair_flat(sbuf[k1], vx, vy, vz, near_m, e1) && has1;
                if (!done) {
                    ++n_eval;
                    if (ok0) {
                        const float tT = T * (1.0f - e0.alpha);
                        if (tT < kTMin) {
                            done = true;
                        } else {
                            const float w = e0.alpha * T;
                            D = fmaf(w, e0.t, D);
                            N0 = fmaf(w, sbuf[k0].n[0], N0);
                            N1 = fmaf(w, sbuf[k0].n[1], N1);
                            N2 = fmaf(w, sbuf[k0].n[2], N2);
                            O += w;
                            T = tT;
                            const int s0 = sidx[k0];
                            last = c + s0 + 1 - rg.x;
                            ++n_con;
                            mine |= 1ull << s0;
                        }
                    }
                }
                if (has1 && !done) {
                    ++n_eval;
                    if (ok1) {
                        const float tT = T * (1.0f - e1.alpha);
                        if (tT < kTMin) {
                            done = true;
                        } else {
                            const float w = e1.alpha * T;
                            D = fmaf(w, e1.t, D);
                            N0 = fmaf(w, sbuf[k1].n[0], N0);
                            N1 = fmaf(w, sbuf[k1].n[1], N1);
                            N2 = fmaf(w, sbuf[k1].n[2], N2);
                            O += w;
                            T = tT;
                            const int s1 = sidx[k1];
                            last = c + s1 + 1 - rg.x;
                            ++n_con;
                            mine |= 1ull << s1;
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();   // sbuf is rewritten by the next chunk
        }
        // few unfinished pixels: the chunk's remaining entries (compacted rank >= q)
        // are evaluated by their own lanes for one pixel at a time
        const bool rem = meets && rank >= q;
        live = q < nact ? __ballot(!done) : 0ull;
        while (live) {
            const int pl = (int)__builtin_ctzll(live);
            live &= live - 1;
            const double pvx = bcast(vx, pl), pvy = bcast(vy, pl), pvz = bcast(vz, pl);
            float sT = bcast(T, pl), sD = bcast(D, pl), sN0 = bcast(N0, pl), sN1 = bcast(N1, pl),
                  sN2 = bcast(N2, pl), sO = bcast(O, pl);
            int sLast = bcast(last, pl), sCon = 0;
            PairEval ev;
            const bool ok = eval_pair_flat(r, pvx, pvy, pvz, near_m, ev) && rem;
            uint64_t hits = __ballot(ok);
            int counted = nact - q;
            bool sDone = false;
            while (hits) {
                const int jl = (int)__builtin_ctzll(hits);
                hits &= hits - 1;
                const float a = bcast(ev.alpha, jl), tj = bcast(ev.t, jl);
                const float tT = sT * (1.0f - a);
                if (tT < kTMin) {
                    sDone = true;
                    // entries evaluated: those of rank q .. rank(jl)
                    counted = bcast(rank, jl) - q + 1;
                    break;
                }
                const float w = a * sT;
                sD = fmaf(w, tj, sD);
                sN0 = fmaf(w, bcast(r.n[0], jl), sN0);
                sN1 = fmaf(w, bcast(r.n[1], jl), sN1);
                sN2 = fmaf(w, bcast(r.n[2], jl), sN2);
                sO += w;
                sT = tT;
                sLast = c + jl + 1 - rg.x;
                ++sCon;
                contrib |= 1ull << jl;
            }
            if (lane == pl) {
                T = sT; D = sD; N0 = sN0; N1 = sN1; N2 = sN2; O = sO;
                last = sLast; n_eval += counted; n_con += sCon; done = sDone;
            }
        }
        if (cm) {
            contrib |= wave_or64(mine);
            if (lane == 0) cm[4 * ((c - rg.x) >> 6)] = contrib;   // this strip is the word's only writer
        }
    }
    if (inside) {
        const int p = i * W + j;
        census[p] = n_eval;
        census[total_pixels + p] = n_con;
        depth[p] = D;
        alpha[p] = O;
        normal[3 * p] = N0; normal[3 * p + 1] = N1; normal[3 * p + 2] = N2;
        stT[p] = T;
        stN[p] = last;
    }
}

// Forward, one wave per strip: workgroup b takes item b, or (QUEUE: the
// persistent form of the work-queue schedule) an occupancy-sized grid takes
// the items in order from a device counter zeroed before the launch.
template <bool QUEUE>
__global__ void __launch_bounds__(64)
k_raster_fwd_w(const FrameDesc *__restrict__ descs, const int32_t *__restrict__ tile_frame,
               const uint32_t *__restrict__ order,
               const RasterRec *__restrict__ rec, const uint32_t *__restrict__ pval, const int2 *__restrict__ ranges,
               const double2 *__restrict__ tables, float *__restrict__ stT_all, int32_t *__restrict__ stN_all,
               int32_t *__restrict__ census_all, int64_t total_pixels, int64_t ntiles,
               const uint32_t *__restrict__ nquad_dev, uint64_t *__restrict__ cmask, uint32_t *__restrict__ queue,
               int64_t nitems)
{
    __shared__ RasterRec sbuf[64];
    __shared__ uint8_t sidx[64];
    const int64_t nquad = (order && nquad_dev) ? (int64_t)*nquad_dev : 0;
    if (!QUEUE) {
        fwd_w_item((int64_t)blockIdx.x, descs, tile_frame, order, rec, pval, ranges, tables, stT_all, stN_all,
                   census_all, total_pixels, ntiles, nquad, cmask, sbuf, sidx);
        return;
    }
    for (;;) {
        uint32_t v = 0;
        if (threadIdx.x == 0) v = atomicAdd(queue, 1u);
        const int64_t item = (int64_t)__shfl(v, 0, 64);
        if (item >= nitems) break;
        fwd_w_item(item, descs, tile_frame, order, rec, pval, ranges, tables, stT_all, stN_all, census_all,
                   total_pixels, ntiles, nquad, cmask, sbuf, sidx);
        __builtin_amdgcn_wave_barrier();
    }
}

// Forward, scalar-cache variant: every wave walks the tile's list on its own.
// The record index and the record itself are wave-uniform, so they are read
// with scalar loads into SGPRs and feed the VALU as scalar operands; no LDS,
// no workgroup barrier, and a wave leaves as soon as its 64 pixels are done.
__global__ void __launch_bounds__(256)
k_raster_fwd_s(const FrameDesc *__restrict__ descs, const int32_t *__restrict__ tile_frame,
             const uint32_t *__restrict__ order,
               const RasterRec *__restrict__ rec, const uint32_t *__restrict__ pval, const int2 *__restrict__ ranges,
               const double2 *__restrict__ tables, float *__restrict__ stT_all, int32_t *__restrict__ stN_all,
               int32_t *__restrict__ census_all, int64_t total_pixels)
{
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const FrameDesc &fd = descs[tile_frame[tile]];
    // the frame's tile shape: TH x TW = 256 pixels, TW a power of two
    const int TW = fd.tw, TH = fd.th, tws = __builtin_ctz((unsigned)fd.tw);
    const int H = fd.H, W = fd.W, tiles_x = fd.tiles_x;
    const float near_m = (float)fd.near_m;
    const double2 *col = tables + fd.tab_off, *rowc = col + W;
    const int ltile = tile - fd.tile_off;
    const int ty = ltile / tiles_x, tx = ltile - ty * tiles_x;
    const int lx = threadIdx.x & (TW - 1), ly = threadIdx.x >> tws;
    const int i = ty * TH + ly, j = tx * TW + lx;
    const bool inside = (i < H) && (j < W);
    const double2 cr = rowc[min(i, H - 1)], cc = col[min(j, W - 1)];
    const double vx = cr.x * cc.x, vy = cr.x * cc.y, vz = cr.y;
    const int2 rg = ranges[tile];
    const int wid = threadIdx.x >> 6;
    const int wr0 = ty * TH + ((wid * 64) >> tws), wr1 = ty * TH + ((wid * 64 + 63) >> tws);
    float T = 1.0f, D = 0.0f, N0 = 0.0f, N1 = 0.0f, N2 = 0.0f, O = 0.0f;
    int last = 0, n_eval = 0, n_con = 0;
    bool done = !inside;
    // software pipeline: the next record's scalar loads are issued before the
    // current record is composited
    RasterRec nxt;
    if (rg.x < rg.y) nxt = rec[__builtin_amdgcn_readfirstlane(pval[rg.x])];
    for (int idx = rg.x; idx < rg.y; ++idx) {
        if (__all(done)) break;
        const RasterRec r = nxt;
        if (idx + 1 < rg.y) nxt = rec[__builtin_amdgcn_readfirstlane(pval[idx + 1])];
        const uint32_t rows = __builtin_amdgcn_readfirstlane(r.rows);
        if ((int)(rows >> 16) < wr0 || (int)(rows & 0xffffu) > wr1) continue;
        if (done) continue;
        ++n_eval;
        PairEval e;
        if (!eval_pair(r, vx, vy, vz, near_m, e)) continue;
        const float tT = T * (1.0f - e.alpha);
        if (tT < kTMin) { done = true; continue; }
        const float w = e.alpha * T;
        D = fmaf(w, e.t, D);
        N0 = fmaf(w, r.n[0], N0);
        N1 = fmaf(w, r.n[1], N1);
        N2 = fmaf(w, r.n[2], N2);
        O += w;
        T = tT;
        last = idx + 1 - rg.x;
        ++n_con;
    }
    if (inside) {
        const int p = i * W + j;
        fd.depth[p] = D;
        fd.alpha[p] = O;
        fd.normal[3 * p] = N0; fd.normal[3 * p + 1] = N1; fd.normal[3 * p + 2] = N2;
        stT_all[fd.pix_off + p] = T;
        stN_all[fd.pix_off + p] = last;
        census_all[fd.pix_off + p] = n_eval;
        census_all[total_pixels + fd.pix_off + p] = n_con;
    }
}

constexpr int kBwdBatch = 192;   // default records staged per backward batch (fits 4 workgroups per CU)
constexpr int kDetBatch = 96;    // the fixed-order form's batch (its four rows of sums take 4x the LDS;
                                 // 96 records still fit 4 workgroups per CU)
constexpr int kNg = 18;

__device__ __forceinline__ void dcross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Upstream gradients and final transmittance of one pixel.
struct BwdUpstream {
    float gd, go, gn0, gn1, gn2, Tfin;
};

// Reverse-order state of one pixel: T is the transmittance behind the next
// pair to visit (A_k once it is divided by 1 - alpha_k); Bs the suffix sum of
// c_i alpha_i A_i over the pairs already visited; the reference values are
// those of the pixel's last contributor (the first pair met in reverse).
struct BwdState {
    float T, Bs, Kref, tref, nr0, nr1, nr2;
    bool have_ref;
};

// One contributing pair of a pixel, met in reverse list order (Supp. D):
// advances the state and writes the pair's 18 partials.
//   dL/dalpha_k = c_k A_k + (K T_final - B_k) / (1 - alpha_k), with
//   c_k = gD (t_k - t_ref) + gN . (n_k - n_ref), B_k the suffix sum of c_i alpha_i A_i
//   and K = gD t_ref + gN . n_ref + gO: the reference removes the cancellation of
//   the unshifted form.  The partials are centred on the surfel centre's
//   direction ch: da (v - ch), db (v - ch), dc_s v, da, db, (dL/dt / c)(s_a, s_b, 1),
//   dL/do, dL/dn.
// The scalar part of one reverse step: advances the state and returns
// da = dL/da, db = dL/db (a = P.v, b = Q.v), dcs = the c = M.v part of the
// s_hat path, tt = (dL/dt) / c, dop = dL/do and the pair's weight w = alpha A.
struct BwdScalars {
    float da, db, dcs, tt, dop, w;
};

// The range of a pair to FP64 accuracy as t + t_lo: t = tau * rcp(c) carries
// the FP32 rounding of tau, which is the same for every pixel of a record, so
// coplanar surfels (whose exact ranges at a pixel coincide) would differ by a
// systematic 1e-7 relative error and the depth channel's dL/dalpha, which is a
// difference of such ranges, would be off by that much.  One correction step
// with the record's FP64 tau and the FP64 c removes it.
__device__ __forceinline__ float range_low(const PairEval &e, double tau)
{
    return (float)fma(-(double)e.t, e.c, tau) * e.rc;
}

__device__ __forceinline__ BwdScalars bwd_step(BwdState &st, const PairEval &e, float n0, float n1, float n2,
                                               const BwdUpstream &u, float tlo)
{
    const float r1 = __builtin_amdgcn_rcpf(1.0f - e.alpha);
    const float A = st.T * r1;  // transmittance in front of this pair
    if (!st.have_ref) {
        st.have_ref = true;
        st.tref = e.t; st.nr0 = n0; st.nr1 = n1; st.nr2 = n2;
        st.Kref = u.gd * st.tref + u.gn0 * st.nr0 + u.gn1 * st.nr1 + u.gn2 * st.nr2 + u.go;
    }
    // t_ref is the FP32 value of the reference's range (any fixed value is exact
    // algebra), t_k = t + t_lo to FP64 accuracy
    const float ck = u.gd * ((e.t - st.tref) + tlo) + u.gn0 * (n0 - st.nr0) + u.gn1 * (n1 - st.nr1) +
                     u.gn2 * (n2 - st.nr2);
    const float dA = ck * A + (st.Kref * u.Tfin - st.Bs) * r1;
    const float w = e.alpha * A;
    st.Bs = fmaf(ck, w, st.Bs);
    st.T = A;
    const float gt = u.gd * w;  // dL/d(range)
    float dsa = 0.0f, dsb = 0.0f, dop = 0.0f;
    if (!e.clamped) {
        const float f = -dA * e.alpha;
        dsa = f * e.sa; dsb = f * e.sb;
        dop = dA * e.G;
    }
    const float da = dsa * e.rc, db = dsb * e.rc;
    const float dcs = -(dsa * e.sa + dsb * e.sb) * e.rc;
    const float tt = gt * e.rc;
    return {da, db, dcs, tt, dop, w};
}

// The 18 partials of a pair from its reverse step's scalars.
__device__ __forceinline__ void bwd_partials(const BwdScalars &q, const PairEval &e, const double *ch,
                                             const BwdUpstream &u, double vx, double vy, double vz, float (&g)[18])
{
    const float da = q.da, db = q.db, dcs = q.dcs, tt = q.tt, dop = q.dop, w = q.w;
    const float ex = (float)(vx - ch[0]), ey = (float)(vy - ch[1]), ez = (float)(vz - ch[2]);
    const float fvx = (float)vx, fvy = (float)vy, fvz = (float)vz;
    g[0] = da * ex; g[1] = da * ey; g[2] = da * ez;
    g[3] = db * ex; g[4] = db * ey; g[5] = db * ez;
    g[6] = dcs * fvx; g[7] = dcs * fvy; g[8] = dcs * fvz;
    g[9] = da; g[10] = db;
    g[11] = tt * e.sa; g[12] = tt * e.sb; g[13] = tt;
    g[14] = dop;
    g[15] = u.gn0 * w; g[16] = u.gn1 * w; g[17] = u.gn2 * w;
}

__device__ __forceinline__ void bwd_pair(BwdState &st, const PairEval &e, float n0, float n1, float n2,
                                         const ChatRec &chr, const BwdUpstream &u, double vx, double vy, double vz,
                                         float (&g)[18])
{
    const BwdScalars q = bwd_step(st, e, n0, n1, n2, u, range_low(e, chr.tau));
    bwd_partials(q, e, chr.c, u, vx, vy, vz, g);
}

template <int CTRL>
__device__ __forceinline__ double dpp_perm_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// The evaluations of the four lanes of this lane's quad (every lane active).
__device__ __forceinline__ void quad_evals(const PairEval &e, int lane, PairEval (&eu)[4])
{
    eu[0].sa = dpp_perm<0x00>(e.sa); eu[1].sa = dpp_perm<0x55>(e.sa);
    eu[2].sa = dpp_perm<0xAA>(e.sa); eu[3].sa = dpp_perm<0xFF>(e.sa);
    eu[0].sb = dpp_perm<0x00>(e.sb); eu[1].sb = dpp_perm<0x55>(e.sb);
    eu[2].sb = dpp_perm<0xAA>(e.sb); eu[3].sb = dpp_perm<0xFF>(e.sb);
    eu[0].t = dpp_perm<0x00>(e.t); eu[1].t = dpp_perm<0x55>(e.t);
    eu[2].t = dpp_perm<0xAA>(e.t); eu[3].t = dpp_perm<0xFF>(e.t);
    eu[0].rc = dpp_perm<0x00>(e.rc); eu[1].rc = dpp_perm<0x55>(e.rc);
    eu[2].rc = dpp_perm<0xAA>(e.rc); eu[3].rc = dpp_perm<0xFF>(e.rc);
    eu[0].G = dpp_perm<0x00>(e.G); eu[1].G = dpp_perm<0x55>(e.G);
    eu[2].G = dpp_perm<0xAA>(e.G); eu[3].G = dpp_perm<0xFF>(e.G);
    eu[0].alpha = dpp_perm<0x00>(e.alpha); eu[1].alpha = dpp_perm<0x55>(e.alpha);
    eu[2].alpha = dpp_perm<0xAA>(e.alpha); eu[3].alpha = dpp_perm<0xFF>(e.alpha);
    eu[0].c = dpp_perm_d<0x00>(e.c); eu[1].c = dpp_perm_d<0x55>(e.c);
    eu[2].c = dpp_perm_d<0xAA>(e.c); eu[3].c = dpp_perm_d<0xFF>(e.c);
    const uint32_t clq = (uint32_t)(__ballot(e.clamped) >> (lane & ~3)) & 0xfu;
#pragma unroll
    for (int u = 0; u < 4; ++u) eu[u].clamped = (clq >> u) & 1u;
}

// The splat axes from a record: P, Q, M are the cofactors of (b_alpha b_beta
// b_c), so P x Q = tau b_c, Q x M = tau b_alpha, M x P = tau b_beta with
// tau^2 = M . (P x Q) and the sign of the stored tau (FP64, ~1e-12 relative).
__device__ __forceinline__ void record_axes(const RasterRec &r, double *ba, double *bb, double *bc)
{
    double pq[3], qm[3], mp[3];
    dcross(r.P, r.Q, pq); dcross(r.Q, r.M, qm); dcross(r.M, r.P, mp);
    const double t2 = (r.M[0] * pq[0] + r.M[1] * pq[1]) + r.M[2] * pq[2];
    const double it = (r.tau < 0.0f ? -1.0 : 1.0) / sqrt(t2);
#pragma unroll
    for (int c = 0; c < 3; ++c) { ba[c] = qm[c] * it; bb[c] = mp[c] * it; bc[c] = pq[c] * it; }
}

// Unit direction of b_c, the centring reference of the partials: the
// direction of P x Q with the sign of tau.  The accumulation and the flush
// read the same staged value.
__device__ __forceinline__ void centre_dir(const RasterRec &r, ChatRec &ch)
{
    double pq[3];
    dcross(r.P, r.Q, pq);
    const double sgn = r.tau < 0.0f ? -1.0 : 1.0;
    const double sg = sgn / sqrt((pq[0] * pq[0] + pq[1] * pq[1]) + pq[2] * pq[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) ch.c[c] = pq[c] * sg;
    ch.tau = sgn * sqrt((r.M[0] * pq[0] + r.M[1] * pq[1]) + r.M[2] * pq[2]);
}

// tau = b_c . M in FP64 from the cofactors (tau^2 = M . (P x Q)), with the sign
// of the record's FP32 tau.
__device__ __forceinline__ double record_tau(const RasterRec &r)
{
    double pq[3];
    dcross(r.P, r.Q, pq);
    return (r.tau < 0.0f ? -1.0 : 1.0) * sqrt((r.M[0] * pq[0] + r.M[1] * pq[1]) + r.M[2] * pq[2]);
}

// The axes of a staged record for its flush.
__device__ __forceinline__ FrameRec flush_axes(const RasterRec &r)
{
    FrameRec fr;
    record_axes(r, fr.ba, fr.bb, fr.bc);
    fr.n[0] = r.n[0]; fr.n[1] = r.n[1]; fr.n[2] = r.n[2];
    return fr;
}

// A record's pixel sums of the 18 partials -> dL/d(b_alpha, b_beta, b_c, n) in
// FP64 (dPv = E_a + A_a ch, dQv = E_b + A_b ch; g_alpha = E_b x b_c + b_beta x C_s
// + T_a M, g_beta = b_c x E_a + C_s x b_alpha + T_b M, g_c = dPv x b_beta +
// b_alpha x dQv + T_c M), their se(3) pose contribution into pacc, and (acc not
// NULL) the world-frame gradients added to the record's accumulator, or with
// STORE written with plain stores to a 64-B aligned slot of its own.
template <bool STORE = false>
__device__ __forceinline__ void flush_record(const float (&s)[18], const FrameRec &fr, const double *M,
                                             const double *ch, const double *pose, float *acc, double (&pacc)[6])
{
    const double Ea[3] = {s[0], s[1], s[2]}, Eb[3] = {s[3], s[4], s[5]}, Cs[3] = {s[6], s[7], s[8]};
    const double Aa = s[9], Ab = s[10], Ta = s[11], Tb = s[12], Tc = s[13];
    double dPv[3], dQv[3];  // sum da v, sum db v
#pragma unroll
    for (int c = 0; c < 3; ++c) { dPv[c] = Ea[c] + Aa * ch[c]; dQv[c] = Eb[c] + Ab * ch[c]; }
    double t1[3], t2[3];
    double ga[3], gb[3], gc[3];
    dcross(Eb, fr.bc, t1); dcross(fr.bb, Cs, t2);
#pragma unroll
    for (int c = 0; c < 3; ++c) ga[c] = t1[c] + t2[c] + Ta * M[c];
    dcross(fr.bc, Ea, t1); dcross(Cs, fr.ba, t2);
#pragma unroll
    for (int c = 0; c < 3; ++c) gb[c] = t1[c] + t2[c] + Tb * M[c];
    dcross(dPv, fr.bb, t1); dcross(fr.ba, dQv, t2);
#pragma unroll
    for (int c = 0; c < 3; ++c) gc[c] = t1[c] + t2[c] + Tc * M[c];
    const double gn[3] = {s[15], s[16], s[17]};
    const double nn[3] = {fr.n[0], fr.n[1], fr.n[2]};
    // pose: d b / d rho = -I, d b / d phi = [b]_x
    double c1[3], c2[3], c3[3], c4[3];
    dcross(gc, fr.bc, c1); dcross(ga, fr.ba, c2); dcross(gb, fr.bb, c3); dcross(gn, nn, c4);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        pacc[c] -= gc[c];
        pacc[3 + c] += c1[c] + c2[c] + c3[c] + c4[c];
    }
    if (acc) {
        double R[9];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            R[3 * e] = pose[4 * e]; R[3 * e + 1] = pose[4 * e + 1]; R[3 * e + 2] = pose[4 * e + 2];
        }
        float w[kAccStride];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            w[c] = (float)(R[c] * ga[0] + R[3 + c] * ga[1] + R[6 + c] * ga[2]);
            w[3 + c] = (float)(R[c] * gb[0] + R[3 + c] * gb[1] + R[6 + c] * gb[2]);
            w[6 + c] = (float)(R[c] * gc[0] + R[3 + c] * gc[1] + R[6 + c] * gc[2]);
            w[9 + c] = (float)(R[c] * gn[0] + R[3 + c] * gn[1] + R[6 + c] * gn[2]);
        }
        w[12] = s[14];
        if (STORE) {
            float4 *q = reinterpret_cast<float4 *>(acc);
            q[0] = make_float4(w[0], w[1], w[2], w[3]);
            q[1] = make_float4(w[4], w[5], w[6], w[7]);
            q[2] = make_float4(w[8], w[9], w[10], w[11]);
            acc[12] = w[12];
        } else {
#pragma unroll
            for (int c = 0; c < kAccStride; ++c) atomicAdd(acc + c, w[c]);
        }
    }
}


// QUEUE: the persistent form.  An occupancy-sized grid whose workgroups take
// the tiles' slots of the longest-first order from a device counter (zeroed
// before the launch) until the order is exhausted; otherwise workgroup b takes
// slot b.  Either way tile t writes pose row t, so the results are the same
// (and do not depend on the tile schedule either).
// DET: the fixed-order form.  Each wave keeps its own row of record sums, the
// flush adds the four rows in wave order, and a (tile, record) flush goes with
// plain stores to the slot of the pair (its index in the record's emission
// order: rank, off and rbox of the binning give it), whose bit it sets in
// slot_bits; the slots are summed per surfel afterwards in a fixed order.  The
// results then do not depend on the order in which workgroups run.
template <int BATCH, bool QUEUE, bool DET>
__global__ void __launch_bounds__(256, 4)  // 4 waves per SIMD: at most 128 VGPRs
k_raster_bwd(const FrameDesc *__restrict__ descs, const int32_t *__restrict__ tile_frame,
             const uint32_t *__restrict__ order,
             const RasterRec *__restrict__ rec,
             const uint32_t *__restrict__ pval, const int2 *__restrict__ ranges, const double2 *__restrict__ tables,
             const float *__restrict__ stT_all,
             const int32_t *__restrict__ stN_all, int32_t *__restrict__ census_all, int64_t total_pixels,
             double *__restrict__ pose_part, int pose_only, uint32_t *__restrict__ queue, int ntiles,
             const uint64_t *__restrict__ cmask, const uint32_t *__restrict__ rank,
             const uint32_t *__restrict__ off, const PixBox *__restrict__ rbox, float *__restrict__ slots,
             uint32_t *__restrict__ slot_bits)
{
    constexpr int NROW = DET ? 4 : 1;
    __shared__ RasterRec srec[BATCH];
    __shared__ ChatRec schat[BATCH];
    __shared__ float sred[NROW][kNg][BATCH];   // wave sums: added in LDS by the four waves, or one row per wave
    __shared__ int sflag[BATCH];
    __shared__ uint8_t slist[4][BATCH];
    __shared__ int s_last;
    __shared__ double s_pose[4][6];

    __shared__ int s_item;
    for (int pass = 0;; ++pass) {
        int item = (int)blockIdx.x;
        if (QUEUE) {
            __syncthreads();   // every thread has read the previous slot
            if (threadIdx.x == 0) s_item = (int)atomicAdd(queue, 1u);
            __syncthreads();
            item = s_item;
            if (item >= ntiles) break;
        } else if (pass > 0) {
            break;
        }
        const int tile = order ? (int)order[item] : item;
        const FrameDesc &fd = descs[tile_frame[tile]];
        // the frame's tile shape: TH x TW = 256 pixels, TW a power of two
        const int TW = fd.tw, TH = fd.th, tws = __builtin_ctz((unsigned)fd.tw);
        const int H = fd.H, W = fd.W, tiles_x = fd.tiles_x;
        const float near_m = (float)fd.near_m;
        const double2 *col = tables + fd.tab_off, *rowc = col + W;
        const float *stT = stT_all + fd.pix_off;
        const int32_t *stN = stN_all + fd.pix_off;
        int32_t *census = census_all + fd.pix_off;
        const float *gD = fd.gD, *gN = fd.gN, *gO = fd.gO;
        const double *pose = fd.pose;
        float *acc = fd.acc;
        const int ltile = tile - fd.tile_off;
        const int ty = ltile / tiles_x, tx = ltile - ty * tiles_x;
        const int lx = threadIdx.x & (TW - 1), ly = threadIdx.x >> tws;
        const int i = ty * TH + ly, j = tx * TW + lx;
        const bool inside = (i < H) && (j < W);
        const double2 cr = rowc[min(i, H - 1)], cc = col[min(j, W - 1)];
        const double vx = cr.x * cc.x, vy = cr.x * cc.y, vz = cr.y;
        const int2 rg = ranges[tile];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        const int red_val = bitrev6(lane);  // the wave sum this lane holds after wave_sum18
        const int wr0 = ty * TH + ((wid * 64) >> tws), wr1 = ty * TH + ((wid * 64 + 63) >> tws);
        const int p = inside ? i * W + j : 0;
        float T = inside ? stT[p] : 1.0f;
        const int last = inside ? stN[p] : 0;
        const float Tfin = T;
        const float gd = (inside && gD) ? gD[p] : 0.0f;
        const float go = (inside && gO) ? gO[p] : 0.0f;
        const float gn0 = (inside && gN) ? gN[3 * p] : 0.0f;
        const float gn1 = (inside && gN) ? gN[3 * p + 1] : 0.0f;
        const float gn2 = (inside && gN) ? gN[3 * p + 2] : 0.0f;
        if (threadIdx.x == 0) s_last = 0;
        for (int e = threadIdx.x; e < NROW * kNg * BATCH; e += blockDim.x) (&sred[0][0][0])[e] = 0.0f;
        for (int e = threadIdx.x; e < BATCH; e += blockDim.x) sflag[e] = 0;
        if (threadIdx.x < 24) (&s_pose[0][0])[threadIdx.x] = 0.0;
        __syncthreads();
        if (last > 0) atomicMax(&s_last, last);
        __syncthreads();
        const int end = rg.x + s_last;
        int wlast = last;  // the wave's largest contributor count
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) wlast = max(wlast, __shfl_xor(wlast, o, 64));

        // dL/dalpha_k = c_k A_k - B_k / (1 - alpha_k) + K T_final / (1 - alpha_k), with
        // c_k = gD (t_k - t_ref) + gN . (n_k - n_ref), B_k the suffix sum of c_i alpha_i A_i
        // and K = gD t_ref + gN . n_ref + gO: the reference (the last contributor, met
        // first in reverse) removes the cancellation of the unshifted form.
        BwdState st = {T, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, false};
        const BwdUpstream up = {gd, go, gn0, gn1, gn2, Tfin};
        int n_eval = 0, n_con = 0;

        for (int b_end = end; b_end > rg.x; b_end -= BATCH) {
            const int b0 = max(rg.x, b_end - BATCH);
            const int cnt = b_end - b0;
            __syncthreads();
            // records no strip walks are not staged (no wave's compaction takes them)
            if ((int)threadIdx.x < cnt && any_strip_wants(cmask, tile, rg.x, b0 + (int)threadIdx.x - rg.x)) {
                const uint32_t id = pval[b0 + threadIdx.x];
                srec[threadIdx.x] = rec[id];
                centre_dir(srec[threadIdx.x], schat[threadIdx.x]);
            }
            __syncthreads();
            // the batch's records that meet this wave's rows and lie before its last
            // contributor, in list order; they are walked in reverse
            int nact = 0;
            for (int base = 0; base < cnt; base += 64) {
                const int kk = base + lane;
                bool meets = false;
                if (kk < cnt) {
                    const uint32_t rows = srec[kk].rows;
                    const int pos = b0 + kk - rg.x;
                    meets = !((int)(rows >> 16) < wr0 || (int)(rows & 0xffffu) > wr1) && pos < wlast &&
                            (!cmask || ((cmask[cmask_word(tile, rg.x, wid, pos >> 6)] >> (pos & 63)) & 1ull));
                }
                const uint64_t m = __ballot(meets);
                if (meets) slist[wid][nact + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = (uint8_t)kk;
                nact += __popcll(m);
            }
            // a wave's walk reads only its own list and the records staged before the
            // barrier above, so only the wave's own slist writes need to be visible
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int q = nact - 1; q >= 0; q -= 2) {
                // two entries per step: both evaluations are independent of the
                // reverse chain, which then takes them in list order
                const bool has1 = q >= 1;
                const int ka = slist[wid][q], kb = slist[wid][has1 ? q - 1 : q];
                const int posa = b0 + ka - rg.x, posb = b0 + kb - rg.x;
                PairEval ea, eb;
                n_eval += (posa < last ? 1 : 0) + (has1 && posb < last ? 1 : 0);
                const bool acta = eval_pair_flat(srec[ka], vx, vy, vz, near_m, ea) && posa < last;
                const bool actb = eval_pair_flat(srec[kb], vx, vy, vz, near_m, eb) && posb < last && has1;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int k = h ? kb : ka;
                    const bool act = h ? actb : acta;
                    // about half of the walked entries meet no lane: they skip the partials
                    if (__any(act)) {
                        float g[kNg];
#pragma unroll
                        for (int v = 0; v < kNg; ++v) g[v] = 0.0f;
                        if (act) {
                            ++n_con;
                            bwd_pair(st, h ? eb : ea, srec[k].n[0], srec[k].n[1], srec[k].n[2], schat[k], up, vx, vy, vz, g);
                        }
                        static_assert(kNg == 18, "wave_sum18 reduces 18 values");
                        const float tot = wave_sum18(g, lane);
                        if (red_val < kNg) {
                            if (DET) sred[DET ? wid : 0][red_val][k] = tot;
                            else atomicAdd(&sred[0][red_val][k], tot);
                        }
                        if (lane == 0) sflag[k] = 1;
                    }
                }
            }
            __syncthreads();
            // the pose partials of this batch's flushes, summed over the wave into s_pose
            double pacc[6] = {0, 0, 0, 0, 0, 0};
            bool flushed = false;
            if ((int)threadIdx.x < cnt) {
                const int k = threadIdx.x;
                if (sflag[k]) {
                    flushed = true;
                    // take the record's sums and leave the slots zeroed for the next batch
                    float s[kNg];
#pragma unroll
                    for (int v = 0; v < kNg; ++v) {
                        if constexpr (DET) {
                            s[v] = ((sred[0][v][k] + sred[NROW - 3][v][k]) + sred[NROW - 2][v][k]) + sred[NROW - 1][v][k];
#pragma unroll
                            for (int w = 0; w < NROW; ++w) sred[w][v][k] = 0.0f;
                        } else {
                            s[v] = sred[0][v][k];
                            sred[0][v][k] = 0.0f;
                        }
                    }
                    sflag[k] = 0;
                    const uint32_t id = pval[b0 + k];
                    const FrameRec fr = flush_axes(srec[k]);
                    if constexpr (DET) {
                        float *slot = nullptr;
                        if (!pose_only) {
                            // the pair's index in its record's emission order
                            const uint32_t r = rank[id];
                            const uint32_t e = off[r] + (uint32_t)span_index(tile_span(rbox[r], TH, TW), ty, tx);
                            slot = slots + (size_t)kSlotFloats * e;
                            atomicOr(slot_bits + (e >> 5), 1u << (e & 31));
                        }
                        flush_record<true>(s, fr, srec[k].M, schat[k].c, pose, slot, pacc);
                    } else {
                        flush_record(s, fr, srec[k].M, schat[k].c, pose,
                                     pose_only ? nullptr : acc + (size_t)(id - fd.item_off) * kAccStride, pacc);
                    }
                }
            }
            if (__any(flushed)) {
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    double v = pacc[c];
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
                    if (lane == 0) s_pose[wid][c] += v;
                }
            }
        }
        if (inside) {
            census[2 * total_pixels + p] = n_eval;
            census[3 * total_pixels + p] = n_con;
        }
        // the four waves' pose sums into the tile's own row (summed per keyframe in
        // a fixed order by k_pose_reduce; no atomics)
        __syncthreads();
        if (threadIdx.x < 6) {
            pose_part[8 * (size_t)tile + threadIdx.x] =
                s_pose[0][threadIdx.x] + s_pose[1][threadIdx.x] + s_pose[2][threadIdx.x] + s_pose[3][threadIdx.x];
        }
        if (threadIdx.x == 6) {
            pose_part[8 * (size_t)tile + 6] = (double)tile_frame[tile];
        }

    }
}

// Sum over the 16 lanes of the wave that share lane & 3 (the four rows'
// lanes of one slot): rotations by 4 and 8 inside each 16-lane row keep the
// slot, then the rows are folded.  Every lane ends with its slot's total.
__device__ __forceinline__ float slot_sum16(float x)
{
    x = dpp_add<0x124, 0xf>(x);   // row_ror:4
    x = dpp_add<0x128, 0xf>(x);   // row_ror:8
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}

// Quad mode of the one-wave backward (the counterpart of fwd_quad and gn_quad):
// 16 pixels of the tile, four lanes per pixel.  Each step the four lanes of a
// pixel evaluate four consecutive compacted records (slot 0 the latest in list
// order); every lane advances its pixel's reverse state through the four in
// reverse list order with the broadcast evaluations, keeping its own record's
// step, and forms its own pair's 18 partials; the partials of each slot's
// record are summed over its 16 pixels and stored for the record, which
// flushes at the end of the chunk as in the strip form.  A pixel's reverse
// chain sees the same pairs in the same order as in the strip form.
__device__ __forceinline__ void bwd_quad(const FrameDesc &fd, int tile, int sub, const RasterRec *__restrict__ rec,
                                         const uint32_t *__restrict__ pval, const int2 *__restrict__ ranges,
                                         const double2 *__restrict__ tables, const float *__restrict__ stT_all,
                                         const int32_t *__restrict__ stN_all, int32_t *__restrict__ census_all,
                                         int64_t total_pixels, double *prow, int frame, int pose_only,
                                         const uint64_t *__restrict__ cmask, RasterRec *sbuf, ChatRec *schat,
                                         float (*sred)[64], uint8_t *slist)
{
    const int TW = fd.tw, TH = fd.th, tws = __builtin_ctz((unsigned)fd.tw);
    const int H = fd.H, W = fd.W, tiles_x = fd.tiles_x;
    const float near_m = (float)fd.near_m;
    const double2 *col = tables + fd.tab_off, *rowc = col + W;
    const float *stT = stT_all + fd.pix_off;
    const int32_t *stN = stN_all + fd.pix_off;
    int32_t *census = census_all + fd.pix_off;
    const int ltile = tile - fd.tile_off;
    const int ty = ltile / tiles_x, tx = ltile - ty * tiles_x;
    const int lane = threadIdx.x, slot = lane & 3;
    const int q16 = 16 * sub + (lane >> 2);   // pixel index within the tile, row-major
    const int i = ty * TH + (q16 >> tws), j = tx * TW + (q16 & (TW - 1));
    const bool inside = (i < H) && (j < W);
    const double2 cr = rowc[min(i, H - 1)], cc = col[min(j, W - 1)];
    const double vx = cr.x * cc.x, vy = cr.x * cc.y, vz = cr.y;
    const int2 rg = ranges[tile];
    const int wr0 = ty * TH + ((16 * sub) >> tws), wr1 = ty * TH + ((16 * sub + 15) >> tws);
    const int p = inside ? i * W + j : 0;
    const int last = inside ? stN[p] : 0;
    const float T0 = inside ? stT[p] : 1.0f;
    BwdUpstream up;
    up.gd = (inside && fd.gD) ? fd.gD[p] : 0.0f;
    up.go = (inside && fd.gO) ? fd.gO[p] : 0.0f;
    up.gn0 = (inside && fd.gN) ? fd.gN[3 * p] : 0.0f;
    up.gn1 = (inside && fd.gN) ? fd.gN[3 * p + 1] : 0.0f;
    up.gn2 = (inside && fd.gN) ? fd.gN[3 * p + 2] : 0.0f;
    up.Tfin = T0;
    BwdState st = {T0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, false};
    int wlast = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wlast = max(wlast, __shfl_xor(wlast, o, 64));
    for (int v = 0; v < kNg; ++v) sred[v][lane] = 0.0f;
    double pacc[6] = {0, 0, 0, 0, 0, 0};
    int n_eval = 0, n_con = 0;
    float *acc_base = pose_only ? nullptr : fd.acc;
    const int end = rg.x + wlast;   // entries at or beyond end precede no contributor of the sub-strip
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    // the words of the strip holding this sub-strip: entries no pixel of the strip
    // composited are not walked
    const uint64_t *cm = cmask ? cmask + cmask_word(tile, rg.x, sub >> 2, 0) : nullptr;
    for (int c = wlast > 0 ? rg.x + ((wlast - 1) & ~63) : rg.x - 64; c >= rg.x; c -= 64) {
        bool meets = false;
        uint32_t id = 0;
        const uint64_t cw = mask_word(cm, 4 * ((c - rg.x) >> 6));
        if (c + lane < end && ((cw >> lane) & 1ull)) {
            id = pval[c + lane];
            const u32x4 *src = reinterpret_cast<const u32x4 *>(rec + id);
            u32x4 w[6];
#pragma unroll
            for (int f = 0; f < 6; ++f) w[f] = src[f];
            const uint32_t rows = w[5].w;
            meets = !((int)(rows >> 16) < wr0 || (int)(rows & 0xffffu) > wr1);
            if (meets) {
                u32x4 *dst = reinterpret_cast<u32x4 *>(&sbuf[lane]);
#pragma unroll
                for (int f = 0; f < 6; ++f) dst[f] = w[f];
                centre_dir(sbuf[lane], schat[lane]);
            }
        }
        const uint64_t m = __ballot(meets);
        const int nact = __popcll(m);
        if (meets)
            slist[__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                (uint8_t)lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint64_t fmask = 0;   // chunk records with sums in sred
        for (int q = nact - 1; q >= 0; q -= 4) {
            const int kq = q - slot;   // this lane's compacted index: slot 0 the latest in list order
            const int k = slist[kq >= 0 ? kq : 0];
            const bool cand = kq >= 0 && c + k - rg.x < last;
            n_eval += cand ? 1 : 0;
            PairEval e;
            const bool act = eval_pair_flat(sbuf[k], vx, vy, vz, near_m, e) && cand;
            const uint64_t am = __ballot(act);
            if (am == 0) continue;
            const uint32_t actq = (uint32_t)(am >> (lane & ~3)) & 0xfu;
            PairEval eu[4];
            quad_evals(e, lane, eu);
            BwdScalars mine = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if ((actq >> u) & 1u) {
                    const int ku = slist[q - u];
                    const RasterRec &r = sbuf[ku];
                    const BwdScalars sc = bwd_step(st, eu[u], r.n[0], r.n[1], r.n[2], up, range_low(eu[u], schat[ku].tau));
                    if (u == slot) mine = sc;
                }
            }
            float g[kNg];
#pragma unroll
            for (int v = 0; v < kNg; ++v) g[v] = 0.0f;
            if (act) {
                ++n_con;
                bwd_partials(mine, e, schat[k].c, up, vx, vy, vz, g);
            }
#pragma unroll
            for (int v = 0; v < kNg; ++v) g[v] = slot_sum16(g[v]);
            // lanes 0..3 store the totals of slots 0..3 (records with a contributing pixel)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if ((am & (0x1111111111111111ull << u)) != 0) {
                    const int ku = slist[q - u];
                    if (lane == u) {
#pragma unroll
                        for (int v = 0; v < kNg; ++v) sred[v][ku] = g[v];
                    }
                    fmask |= 1ull << ku;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if ((fmask >> lane) & 1ull) {
            float s[kNg];
#pragma unroll
            for (int v = 0; v < kNg; ++v) { s[v] = sred[v][lane]; sred[v][lane] = 0.0f; }
            const FrameRec fr = flush_axes(sbuf[lane]);
            flush_record(s, fr, sbuf[lane].M, schat[lane].c, fd.pose,
                         acc_base ? acc_base + (size_t)(id - fd.item_off) * kAccStride : nullptr, pacc);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // a pixel's counts are the sums over its four lanes
    n_eval += __shfl_xor(n_eval, 1, 64);
    n_eval += __shfl_xor(n_eval, 2, 64);
    n_con += __shfl_xor(n_con, 1, 64);
    n_con += __shfl_xor(n_con, 2, 64);
    if (inside && slot == 0) {
        census[2 * total_pixels + p] = n_eval;
        census[3 * total_pixels + p] = n_con;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double v = pacc[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        pacc[k] = v;
    }
    if (lane < 6) {
        double v = pacc[0];
#pragma unroll
        for (int k = 1; k < 6; ++k) v = lane == k ? pacc[k] : v;
        prow[lane] = v;
    }
    if (lane == 6) prow[6] = (double)frame;
}

// Backward, one wave per 64-pixel strip (the counterpart of k_raster_fwd_w).
// The strip's list is walked in reverse, 64 records per chunk (one per lane,
// the previous chunk's loads in flight), from its last contributor down.
// Many active pixels: every lane runs its pixel's reverse update against the
// compacted records and each record's 18 partials are summed over the wave;
// few active pixels (those whose last contributor lies further along the
// list): each of them in turn takes the wave, the lanes evaluate their own
// records for it and the contributing ones are visited in reverse order.  At
// the end of a chunk every lane flushes its own record's sums.
__global__ void __launch_bounds__(64, 3)   // 3 waves per SIMD: at most 168 VGPRs
k_raster_bwd_w(const FrameDesc *__restrict__ descs, const int32_t *__restrict__ tile_frame,
               const uint32_t *__restrict__ order,
               const RasterRec *__restrict__ rec, const uint32_t *__restrict__ pval, const int2 *__restrict__ ranges,
               const double2 *__restrict__ tables, const float *__restrict__ stT_all,
               const int32_t *__restrict__ stN_all, int32_t *__restrict__ census_all, int64_t total_pixels,
               double *__restrict__ pose_part, int pose_only, int64_t ntiles,
               const uint32_t *__restrict__ nquad_dev, const uint64_t *__restrict__ cmask)
{
    __shared__ RasterRec sbuf[64];
    __shared__ ChatRec schat[64];
    __shared__ float sred[kNg][64];
    __shared__ uint8_t slist[64];
    int strip, tslot;
    const int64_t nquad = (order && nquad_dev) ? (int64_t)*nquad_dev : 0;
    const int kind = fwd_work_of_block((int64_t)blockIdx.x, ntiles, nquad, strip, tslot);
    if (kind == 0) {
        if (threadIdx.x == 6) pose_part[8 * (size_t)blockIdx.x + 6] = -1.0;   // no keyframe
        return;
    }
    if (kind == 2) {
        const int qt = (int)order[tslot];
        bwd_quad(descs[tile_frame[qt]], qt, strip, rec, pval, ranges, tables, stT_all, stN_all, census_all,
                 total_pixels, pose_part + 8 * (size_t)blockIdx.x, tile_frame[qt], pose_only, cmask, sbuf, schat, sred,
                 slist);
        return;
    }
    const int tile = order ? (int)order[tslot] : tslot;
    const FrameDesc &fd = descs[tile_frame[tile]];
    // the frame's tile shape: TH x TW = 256 pixels, TW a power of two, strips of SR rows
    const int TW = fd.tw, TH = fd.th, tws = __builtin_ctz((unsigned)fd.tw), SR = 64 >> tws;
    const int H = fd.H, W = fd.W, tiles_x = fd.tiles_x;
    const float near_m = (float)fd.near_m;
    const double2 *col = tables + fd.tab_off, *rowc = col + W;
    const float *stT = stT_all + fd.pix_off;
    const int32_t *stN = stN_all + fd.pix_off;
    int32_t *census = census_all + fd.pix_off;
    const int ltile = tile - fd.tile_off;
    const int ty = ltile / tiles_x, tx = ltile - ty * tiles_x;
    const int lane = threadIdx.x;
    const int i = ty * TH + strip * SR + (lane >> tws), j = tx * TW + (lane & (TW - 1));
    const bool inside = (i < H) && (j < W);
    const double2 cr = rowc[min(i, H - 1)], cc = col[min(j, W - 1)];
    const double vx = cr.x * cc.x, vy = cr.x * cc.y, vz = cr.y;
    const int2 rg = ranges[tile];
    const int wr0 = ty * TH + strip * SR, wr1 = wr0 + SR - 1;
    const int red_val = bitrev6(lane);
    const int p = inside ? i * W + j : 0;
    const int last = inside ? stN[p] : 0;
    const float T0 = inside ? stT[p] : 1.0f;
    BwdUpstream up;
    up.gd = (inside && fd.gD) ? fd.gD[p] : 0.0f;
    up.go = (inside && fd.gO) ? fd.gO[p] : 0.0f;
    up.gn0 = (inside && fd.gN) ? fd.gN[3 * p] : 0.0f;
    up.gn1 = (inside && fd.gN) ? fd.gN[3 * p + 1] : 0.0f;
    up.gn2 = (inside && fd.gN) ? fd.gN[3 * p + 2] : 0.0f;
    up.Tfin = T0;
    BwdState st = {T0, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, false};
    int wlast = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wlast = max(wlast, __shfl_xor(wlast, o, 64));
    for (int v = 0; v < kNg; ++v) sred[v][lane] = 0.0f;
    double pacc[6] = {0, 0, 0, 0, 0, 0};
    int n_eval = 0, n_con = 0;
    float *acc_base = pose_only ? nullptr : fd.acc;
    const int end = rg.x + wlast;   // entries at or beyond end precede no contributor of the strip
    int c = wlast > 0 ? rg.x + ((wlast - 1) & ~63) : rg.x - 64;
    // a record travels as six 16-byte words (the last one ends with the rows word)
    static_assert(sizeof(RasterRec) == 96 && offsetof(RasterRec, rows) == 92, "record layout");
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    u32x4 nrec[6];
    uint32_t nid = 0;
    // this strip's words of the contribution mask: entries no pixel of the strip
    // composited are neither read nor walked
    const uint64_t *cm = cmask ? cmask + cmask_word(tile, rg.x, strip, 0) : nullptr;
    uint64_t cw = c >= rg.x ? mask_word(cm, 4 * ((c - rg.x) >> 6)) : ~0ull;
    if (c >= rg.x && c + lane < end && ((cw >> lane) & 1ull)) {
        nid = pval[c + lane];
        const u32x4 *src = reinterpret_cast<const u32x4 *>(rec + nid);
#pragma unroll
        for (int f = 0; f < 6; ++f) nrec[f] = src[f];
    }
    for (; c >= rg.x; c -= 64) {
        const bool inr = c + lane < end && ((cw >> lane) & 1ull);
        const uint32_t id = nid;
        bool meets = false;
        if (inr) {
            const uint32_t rows = nrec[5].w;
            meets = !((int)(rows >> 16) < wr0 || (int)(rows & 0xffffu) > wr1);
        }
        if (meets) {
            u32x4 *dst = reinterpret_cast<u32x4 *>(&sbuf[lane]);
#pragma unroll
            for (int f = 0; f < 6; ++f) dst[f] = nrec[f];
            centre_dir(sbuf[lane], schat[lane]);
        }
        // keep the next chunk's loads below the staging arithmetic (their
        // registers would otherwise be live across it)
        __builtin_amdgcn_sched_barrier(0);
        cw = c - 64 >= rg.x ? mask_word(cm, 4 * ((c - 64 - rg.x) >> 6)) : ~0ull;
        if (c - 64 >= rg.x && ((cw >> lane) & 1ull)) {   // the previous chunk's records, read while this one is processed
            nid = pval[c - 64 + lane];
            const u32x4 *src = reinterpret_cast<const u32x4 *>(rec + nid);
#pragma unroll
            for (int f = 0; f < 6; ++f) nrec[f] = src[f];
        }
        const uint64_t m = __ballot(meets);
        const int nact = __popcll(m);
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (meets) slist[rank] = (uint8_t)lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint64_t fmask = 0;   // records of this chunk with partials in sred
        uint64_t live = __ballot(last > c - rg.x);
        if (__popcll(live) > kStragglers) {
            for (int q = nact - 1; q >= 0; q -= 2) {
                const bool has1 = q >= 1;
                const int ka = slist[q], kb = slist[has1 ? q - 1 : q];
                const int posa = c + ka - rg.x, posb = c + kb - rg.x;
                PairEval ea, eb;
                n_eval += (posa < last ? 1 : 0) + (has1 && posb < last ? 1 : 0);
                const bool acta = eval_pair_flat(sbuf[ka], vx, vy, vz, near_m, ea) && posa < last;
                const bool actb = eval_pair_flat(sbuf[kb], vx, vy, vz, near_m, eb) && posb < last && has1;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int k = h ? kb : ka;
                    const bool act = h ? actb : acta;
                    if (__any(act)) {
                        float g[kNg];
#pragma unroll
                        for (int v = 0; v < kNg; ++v) g[v] = 0.0f;
                        if (act) {
                            ++n_con;
                            bwd_pair(st, h ? eb : ea, sbuf[k].n[0], sbuf[k].n[1], sbuf[k].n[2], schat[k], up, vx, vy, vz, g);
                        }
                        static_assert(kNg == 18, "wave_sum18 reduces 18 values");
                        const float tot = wave_sum18(g, lane);
                        if (red_val < kNg) sred[red_val][k] = tot;
                        fmask |= 1ull << k;
                    }
                }
            }
        } else {
            const int pos_l = c + lane - rg.x;
            while (live) {
                const int pl = (int)__builtin_ctzll(live);
                live &= live - 1;
                const double pvx = bcast(vx, pl), pvy = bcast(vy, pl), pvz = bcast(vz, pl);
                const int plast = bcast(last, pl);
                BwdUpstream pu;
                pu.gd = bcast(up.gd, pl); pu.go = bcast(up.go, pl); pu.gn0 = bcast(up.gn0, pl);
                pu.gn1 = bcast(up.gn1, pl); pu.gn2 = bcast(up.gn2, pl); pu.Tfin = bcast(up.Tfin, pl);
                BwdState ps;
                ps.T = bcast(st.T, pl); ps.Bs = bcast(st.Bs, pl); ps.Kref = bcast(st.Kref, pl);
                ps.tref = bcast(st.tref, pl); ps.nr0 = bcast(st.nr0, pl); ps.nr1 = bcast(st.nr1, pl);
                ps.nr2 = bcast(st.nr2, pl); ps.have_ref = bcast(st.have_ref ? 1 : 0, pl) != 0;
                const bool cand = meets && pos_l < plast;
                PairEval ev;
                const bool ok = eval_pair_flat(sbuf[lane], pvx, pvy, pvz, near_m, ev) && cand;
                const int pe = __popcll(__ballot(cand));
                uint64_t hits = __ballot(ok);
                const int pc = __popcll(hits);
                while (hits) {
                    const int jl = 63 - (int)__builtin_clzll(hits);   // reverse list order
                    hits &= ~(1ull << jl);
                    PairEval ej;
                    ej.sa = bcast(ev.sa, jl); ej.sb = bcast(ev.sb, jl); ej.t = bcast(ev.t, jl);
                    ej.rc = bcast(ev.rc, jl); ej.G = bcast(ev.G, jl); ej.alpha = bcast(ev.alpha, jl);
                    ej.clamped = bcast(ev.clamped ? 1 : 0, jl) != 0;
                    ej.c = bcast(ev.c, jl);
                    float g[kNg];
                    bwd_pair(ps, ej, sbuf[jl].n[0], sbuf[jl].n[1], sbuf[jl].n[2], schat[jl], pu, pvx, pvy, pvz, g);
                    if (lane == jl) {
#pragma unroll
                        for (int v = 0; v < kNg; ++v) sred[v][jl] += g[v];
                    }
                    fmask |= 1ull << jl;
                }
                if (lane == pl) {
                    st = ps;
                    n_eval += pe;
                    n_con += pc;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if ((fmask >> lane) & 1ull) {
            float s[kNg];
#pragma unroll
            for (int v = 0; v < kNg; ++v) { s[v] = sred[v][lane]; sred[v][lane] = 0.0f; }
            const FrameRec fr = flush_axes(sbuf[lane]);
            flush_record(s, fr, sbuf[lane].M, schat[lane].c, fd.pose,
                         acc_base ? acc_base + (size_t)(id - fd.item_off) * kAccStride : nullptr, pacc);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (inside) {
        census[2 * total_pixels + p] = n_eval;
        census[3 * total_pixels + p] = n_con;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double v = pacc[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        pacc[k] = v;
    }
    if (lane < 6) {
        double v = pacc[0];
#pragma unroll
        for (int k = 1; k < 6; ++k) v = lane == k ? pacc[k] : v;
        pose_part[8 * (size_t)blockIdx.x + lane] = v;
    }
    if (lane == 6) pose_part[8 * (size_t)blockIdx.x + 6] = (double)tile_frame[tile];
}

// Pose-only Gauss-Newton normal equations (Sec. 3.3.3, T_wc <- T_wc exp(delta)).
// The reverse traversal of the backward with a unit upstream range gradient
// gives every contributing pair's dD/d(s_hat, t) (bwd_step).  Moving the
// sensor by rho moves the ray origin to rho, turning it by phi turns the ray
// to v + phi x v; with a = P.v, b = Q.v, c = M.v and the origin o, s_hat =
// (v.((o - b_c) x b_beta), v.(b_alpha x (o - b_c))) / c and t = (tau - M.o) / c,
// so per pair
//   dD/drho += da (b_beta x v) + db (v x b_alpha) - tt M
//   dD/dphi += v x (da P + db Q + (dcs - tt t) M)
// summed in registers per pixel (FP32).  Each pixel then adds m w J J^T,
// m w r J and m rho(r) (r = D - D_target, w the Huber IRLS weight, m the
// caller's weight) in FP64; the workgroup's sums go to a row of their own,
// summed per keyframe in a fixed order by k_gn_reduce.
__global__ void __launch_bounds__(256)
k_raster_gn(const FrameDesc *__restrict__ descs, const int32_t *__restrict__ tile_frame,
            const uint32_t *__restrict__ order, const RasterRec *__restrict__ rec,
            const uint32_t *__restrict__ pval, const int2 *__restrict__ ranges,
            const double2 *__restrict__ tables, const float *__restrict__ stT_all,
            const int32_t *__restrict__ stN_all, double *__restrict__ gn_part, const uint64_t *__restrict__ cmask)
{
    __shared__ RasterRec srec[kBwdBatch];
    __shared__ float sab[kBwdBatch][6];   // b_alpha, b_beta in FP32
    __shared__ double stau[kBwdBatch];    // tau in FP64
    __shared__ uint8_t slist[4][kBwdBatch];
    __shared__ int s_last;
    __shared__ double s_red[4][kGnVals];

    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const FrameDesc &fd = descs[tile_frame[tile]];
    // the frame's tile shape: TH x TW = 256 pixels, TW a power of two
    const int TW = fd.tw, TH = fd.th, tws = __builtin_ctz((unsigned)fd.tw);
    const int H = fd.H, W = fd.W, tiles_x = fd.tiles_x;
    const float near_m = (float)fd.near_m;
    const double2 *col = tables + fd.tab_off, *rowc = col + W;
    const float *stT = stT_all + fd.pix_off;
    const int32_t *stN = stN_all + fd.pix_off;
    const int ltile = tile - fd.tile_off;
    const int ty = ltile / tiles_x, tx = ltile - ty * tiles_x;
    const int lx = threadIdx.x & (TW - 1), ly = threadIdx.x >> tws;
    const int i = ty * TH + ly, j = tx * TW + lx;
    const bool inside = (i < H) && (j < W);
    const double2 cr = rowc[min(i, H - 1)], cc = col[min(j, W - 1)];
    const double vx = cr.x * cc.x, vy = cr.x * cc.y, vz = cr.y;
    const float fvx = (float)vx, fvy = (float)vy, fvz = (float)vz;
    const int2 rg = ranges[tile];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int wr0 = ty * TH + ((wid * 64) >> tws), wr1 = ty * TH + ((wid * 64 + 63) >> tws);
    const int p = inside ? i * W + j : 0;
    const float Tfin = inside ? stT[p] : 1.0f;
    const int last = inside ? stN[p] : 0;
    if (threadIdx.x == 0) s_last = 0;
    __syncthreads();
    if (last > 0) atomicMax(&s_last, last);
    __syncthreads();
    const int end = rg.x + s_last;
    int wlast = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wlast = max(wlast, __shfl_xor(wlast, o, 64));

    BwdState st = {Tfin, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, false};
    const BwdUpstream up = {1.0f, 0.0f, 0.0f, 0.0f, 0.0f, Tfin};   // dL/dD = 1
    float J[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};

    for (int b_end = end; b_end > rg.x; b_end -= kBwdBatch) {
        const int b0 = max(rg.x, b_end - kBwdBatch);
        const int cnt = b_end - b0;
        __syncthreads();
        // records no strip walks are not staged (no wave's compaction takes them)
        if ((int)threadIdx.x < cnt && any_strip_wants(cmask, tile, rg.x, b0 + (int)threadIdx.x - rg.x)) {
            const uint32_t id = pval[b0 + threadIdx.x];
            srec[threadIdx.x] = rec[id];
            double ba[3], bb[3], bc[3];
            record_axes(srec[threadIdx.x], ba, bb, bc);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sab[threadIdx.x][c] = (float)ba[c];
                sab[threadIdx.x][3 + c] = (float)bb[c];
            }
            stau[threadIdx.x] = record_tau(srec[threadIdx.x]);
        }
        __syncthreads();
        int nact = 0;
        for (int base = 0; base < cnt; base += 64) {
            const int kk = base + lane;
            bool meets = false;
            if (kk < cnt) {
                const uint32_t rows = srec[kk].rows;
                const int pos = b0 + kk - rg.x;
                meets = !((int)(rows >> 16) < wr0 || (int)(rows & 0xffffu) > wr1) && pos < wlast &&
                        (!cmask || ((cmask[cmask_word(tile, rg.x, wid, pos >> 6)] >> (pos & 63)) & 1ull));
            }
            const uint64_t m = __ballot(meets);
            if (meets) slist[wid][nact + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = (uint8_t)kk;
            nact += __popcll(m);
        }
        __syncthreads();
        for (int q = nact - 1; q >= 0; --q) {
            const int k = slist[wid][q];
            const int pos = b0 + k - rg.x;
            PairEval e;
            const bool act = eval_pair_flat(srec[k], vx, vy, vz, near_m, e) && pos < last;
            if (act) {
                const RasterRec &r = srec[k];
                const BwdScalars s = bwd_step(st, e, r.n[0], r.n[1], r.n[2], up, range_low(e, stau[k]));
                const float ax = sab[k][0], ay = sab[k][1], az = sab[k][2];
                const float bx = sab[k][3], by = sab[k][4], bz = sab[k][5];
                const float Mx = (float)r.M[0], My = (float)r.M[1], Mz = (float)r.M[2];
                J[0] += s.da * (by * fvz - bz * fvy) + s.db * (fvy * az - fvz * ay) - s.tt * Mx;
                J[1] += s.da * (bz * fvx - bx * fvz) + s.db * (fvz * ax - fvx * az) - s.tt * My;
                J[2] += s.da * (bx * fvy - by * fvx) + s.db * (fvx * ay - fvy * ax) - s.tt * Mz;
                const float km = s.dcs - s.tt * e.t;
                const float gx = s.da * (float)r.P[0] + s.db * (float)r.Q[0] + km * Mx;
                const float gy = s.da * (float)r.P[1] + s.db * (float)r.Q[1] + km * My;
                const float gz = s.da * (float)r.P[2] + s.db * (float)r.Q[2] + km * Mz;
                J[3] += fvy * gz - fvz * gy;
                J[4] += fvz * gx - fvx * gz;
                J[5] += fvx * gy - fvy * gx;
            }
        }
    }

    // this pixel's terms, then wave sums (FP64 butterflies) and the four waves in order
    double Jd[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) Jd[c] = J[c];
    double wgt = 0.0, wr = 0.0, cost = 0.0;
    if (inside) {
        const float m = fd.gn_weight ? fd.gn_weight[p] : 1.0f;
        if (m != 0.0f) {
            const double r = (double)fd.depth[p] - (double)fd.gn_target[p];
            const double k = fd.huber_k, a = fabs(r);
            const bool lin = k > 0.0 && a > k;
            wgt = (double)m * (lin ? k / a : 1.0);
            wr = wgt * r;
            cost = (double)m * (lin ? k * (a - 0.5 * k) : 0.5 * r * r);
        }
    }
    int c = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
#pragma unroll
        for (int b = a; b < 6; ++b) {
            double v = wgt * Jd[a] * Jd[b];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) s_red[wid][c] = v;
            ++c;
        }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        double v = wr * Jd[a];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) s_red[wid][21 + a] = v;
    }
    {
        double v = cost;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) s_red[wid][27] = v;
    }
    __syncthreads();
    double *row = gn_part + (size_t)kGnRow * blockIdx.x;
    if (threadIdx.x < kGnVals) {
        const int t = threadIdx.x;
        row[t] = ((s_red[0][t] + s_red[1][t]) + s_red[2][t]) + s_red[3][t];
    }
    if (threadIdx.x == kGnVals) row[kGnVals] = (double)tile_frame[tile];
}

// The pixel's Gauss-Newton terms (m w J J^T, m w r J, m rho(r); Huber in IRLS
// form) summed over the wave by FP64 butterflies into one partial row.
__device__ __forceinline__ void gn_row(const FrameDesc &fd, bool take, int p, const float (&J)[6], double *row,
                                       int lane, int frame)
{
    double Jd[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) Jd[q] = J[q];
    double wgt = 0.0, wr = 0.0, cost = 0.0;
    if (take) {
        const float mw = fd.gn_weight ? fd.gn_weight[p] : 1.0f;
        if (mw != 0.0f) {
            const double r = (double)fd.depth[p] - (double)fd.gn_target[p];
            const double k = fd.huber_k, a = fabs(r);
            const bool lin = k > 0.0 && a > k;
            wgt = (double)mw * (lin ? k / a : 1.0);
            wr = wgt * r;
            cost = (double)mw * (lin ? k * (a - 0.5 * k) : 0.5 * r * r);
        }
    }
    int cidx = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
#pragma unroll
        for (int b = a; b < 6; ++b) {
            double v = wgt * Jd[a] * Jd[b];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) row[cidx] = v;
            ++cidx;
        }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        double v = wr * Jd[a];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) row[21 + a] = v;
    }
    {
        double v = cost;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) row[27] = v;
    }
    if (lane == 0) row[kGnVals] = (double)frame;
}

// The Jacobian row dD/d(rho, phi) of one contributing pair (see k_raster_gn).
__device__ __forceinline__ void gn_pair_row(const BwdScalars &sc, const RasterRec &r, const float *ab, float t,
                                            float fvx, float fvy, float fvz, float (&jc)[6])
{
    const float ax = ab[0], ay = ab[1], az = ab[2];
    const float bx = ab[3], by = ab[4], bz = ab[5];
    const float Mx = (float)r.M[0], My = (float)r.M[1], Mz = (float)r.M[2];
    jc[0] = sc.da * (by * fvz - bz * fvy) + sc.db * (fvy * az - fvz * ay) - sc.tt * Mx;
    jc[1] = sc.da * (bz * fvx - bx * fvz) + sc.db * (fvz * ax - fvx * az) - sc.tt * My;
    jc[2] = sc.da * (bx * fvy - by * fvx) + sc.db * (fvx * ay - fvy * ax) - sc.tt * Mz;
    const float km = sc.dcs - sc.tt * t;
    const float gx = sc.da * (float)r.P[0] + sc.db * (float)r.Q[0] + km * Mx;
    const float gy = sc.da * (float)r.P[1] + sc.db * (float)r.Q[1] + km * My;
    const float gz = sc.da * (float)r.P[2] + sc.db * (float)r.Q[2] + km * Mz;
    jc[3] = fvy * gz - fvz * gy;
    jc[4] = fvz * gx - fvx * gz;
    jc[5] = fvx * gy - fvy * gx;
}


// Quad mode of the one-wave Gauss-Newton kernel (the counterpart of fwd_quad):
// 16 pixels of the tile, four lanes per pixel.  Each step the four lanes of a
// pixel evaluate four consecutive compacted records (slot 0 the latest in list
// order); every lane then advances the pixel's reverse state through the four
// in reverse list order with the broadcast evaluations, keeping its own
// record's step, forms its own record's Jacobian row, and all four add the
// four rows in reverse list order.  The same steps and sums in the same order
// as the strip mode: each pixel's J is identical.
__device__ __forceinline__ void gn_quad(const FrameDesc &fd, int tile, int sub, const RasterRec *__restrict__ rec,
                                        const uint32_t *__restrict__ pval, const int2 *__restrict__ ranges,
                                        const double2 *__restrict__ tables, const float *__restrict__ stT_all,
                                        const int32_t *__restrict__ stN_all, double *row, int frame,
                                        const uint64_t *__restrict__ cmask, RasterRec *sbuf, float (*sab)[6],
                                        double *stau, uint8_t *slist)
{
    const int TW = fd.tw, TH = fd.th, tws = __builtin_ctz((unsigned)fd.tw);
    const int H = fd.H, W = fd.W, tiles_x = fd.tiles_x;
    const float near_m = (float)fd.near_m;
    const double2 *col = tables + fd.tab_off, *rowc = col + W;
    const float *stT = stT_all + fd.pix_off;
    const int32_t *stN = stN_all + fd.pix_off;
    const int ltile = tile - fd.tile_off;
    const int ty = ltile / tiles_x, tx = ltile - ty * tiles_x;
    const int lane = threadIdx.x, slot = lane & 3;
    const int q16 = 16 * sub + (lane >> 2);
    const int i = ty * TH + (q16 >> tws), j = tx * TW + (q16 & (TW - 1));
    const bool inside = (i < H) && (j < W);
    const double2 cr = rowc[min(i, H - 1)], cc = col[min(j, W - 1)];
    const double vx = cr.x * cc.x, vy = cr.x * cc.y, vz = cr.y;
    const float fvx = (float)vx, fvy = (float)vy, fvz = (float)vz;
    const int2 rg = ranges[tile];
    const int wr0 = ty * TH + ((16 * sub) >> tws), wr1 = ty * TH + ((16 * sub + 15) >> tws);
    const int p = inside ? i * W + j : 0;
    const float Tfin = inside ? stT[p] : 1.0f;
    const int last = inside ? stN[p] : 0;
    int wlast = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wlast = max(wlast, __shfl_xor(wlast, o, 64));
    BwdState st = {Tfin, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, false};
    const BwdUpstream up = {1.0f, 0.0f, 0.0f, 0.0f, 0.0f, Tfin};   // dL/dD = 1
    float J[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    const int end = rg.x + wlast;
    // the words of the strip holding this sub-strip: entries no pixel of the strip composited are skipped
    const uint64_t *cm = cmask ? cmask + cmask_word(tile, rg.x, sub >> 2, 0) : nullptr;
    for (int c = wlast > 0 ? rg.x + ((wlast - 1) & ~63) : rg.x - 64; c >= rg.x; c -= 64) {
        bool meets = false;
        const uint64_t cw = mask_word(cm, 4 * ((c - rg.x) >> 6));
        if (c + lane < end && ((cw >> lane) & 1ull)) {
            sbuf[lane] = rec[pval[c + lane]];
            const uint32_t rows = sbuf[lane].rows;
            meets = !((int)(rows >> 16) < wr0 || (int)(rows & 0xffffu) > wr1);
        }
        if (meets) {
            double ba[3], bb[3], bc[3];
            record_axes(sbuf[lane], ba, bb, bc);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                sab[lane][q] = (float)ba[q];
                sab[lane][3 + q] = (float)bb[q];
            }
            stau[lane] = record_tau(sbuf[lane]);
        }
        const uint64_t m = __ballot(meets);
        const int nact = __popcll(m);
        if (meets)
            slist[__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                (uint8_t)lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int q = nact - 1; q >= 0; q -= 4) {
            const int kq = q - slot;   // this lane's compacted index: slot 0 the latest in list order
            const int k = slist[kq >= 0 ? kq : 0];
            PairEval e;
            const bool act = eval_pair_flat(sbuf[k], vx, vy, vz, near_m, e) && kq >= 0 && c + k - rg.x < last;
            const uint32_t actq = (uint32_t)(__ballot(act) >> (lane & ~3)) & 0xfu;
            PairEval eu[4];
            quad_evals(e, lane, eu);
            BwdScalars mine = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if ((actq >> u) & 1u) {
                    const int ku = slist[q - u];
                    const RasterRec &r = sbuf[ku];
                    const BwdScalars sc = bwd_step(st, eu[u], r.n[0], r.n[1], r.n[2], up, range_low(eu[u], stau[ku]));
                    if (u == slot) mine = sc;
                }
            }
            float jc[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            if (act) gn_pair_row(mine, sbuf[k], sab[k], e.t, fvx, fvy, fvz, jc);
            float j4[4][6];
#pragma unroll
            for (int a = 0; a < 6; ++a) {
                j4[0][a] = dpp_perm<0x00>(jc[a]); j4[1][a] = dpp_perm<0x55>(jc[a]);
                j4[2][a] = dpp_perm<0xAA>(jc[a]); j4[3][a] = dpp_perm<0xFF>(jc[a]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if ((actq >> u) & 1u) {
#pragma unroll
                    for (int a = 0; a < 6; ++a) J[a] += j4[u][a];
                }
            }
        }
        // every lane is done with this chunk's records before they are replaced
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    gn_row(fd, inside && slot == 0, p, J, row, lane, frame);
}

// Gauss-Newton terms, one wave per 64-pixel strip (the counterpart of
// k_raster_gn without its workgroup barrier).  The strip's list is read from
// its wave's last contributor backwards in chunks of 64 records, one per lane;
// the records that meet the strip's rows are compacted and every lane runs the
// reverse step for its pixel over them in reverse order.  A pixel sees the
// same records in the same order with the same arithmetic as in k_raster_gn;
// the wave's sums go to a row of their own.  The tiles the forward took in
// quad mode are taken in quad mode here too (gn_quad), 16 rows each; rows
// 16 nquad + 4 (slot - nquad) + strip hold the other tiles' strips, and
// k_gn_reduce adds a tile's rows in a fixed order.
__global__ void __launch_bounds__(64)
k_raster_gn_w(const FrameDesc *__restrict__ descs, const int32_t *__restrict__ tile_frame,
              const uint32_t *__restrict__ order, const RasterRec *__restrict__ rec,
              const uint32_t *__restrict__ pval, const int2 *__restrict__ ranges,
              const double2 *__restrict__ tables, const float *__restrict__ stT_all,
              const int32_t *__restrict__ stN_all, double *__restrict__ gn_part, int64_t ntiles,
              const uint32_t *__restrict__ nquad_dev, const uint64_t *__restrict__ cmask)
{
    __shared__ RasterRec sbuf[64];
    __shared__ float sab[64][6];   // b_alpha, b_beta in FP32
    __shared__ double stau[64];    // tau in FP64
    __shared__ uint8_t slist[64];
    int strip, tslot;
    const int64_t nquad = (order && nquad_dev) ? (int64_t)*nquad_dev : 0;
    const int kind = fwd_work_of_block((int64_t)blockIdx.x, ntiles, nquad, strip, tslot);
    if (kind == 0) return;
    if (kind == 2) {   // 16 rows per quad tile, in sub-strip order
        const int qt = (int)order[tslot];
        gn_quad(descs[tile_frame[qt]], qt, strip, rec, pval, ranges, tables, stT_all, stN_all,
                gn_part + (size_t)kGnRow * (16 * (size_t)tslot + strip), tile_frame[qt], cmask, sbuf, sab, stau,
                slist);
        return;
    }
    const int tile = order ? (int)order[tslot] : tslot;
    const FrameDesc &fd = descs[tile_frame[tile]];
    // the frame's tile shape: TH x TW = 256 pixels, TW a power of two, strips of SR rows
    const int TW = fd.tw, TH = fd.th, tws = __builtin_ctz((unsigned)fd.tw), SR = 64 >> tws;
    const int H = fd.H, W = fd.W, tiles_x = fd.tiles_x;
    const float near_m = (float)fd.near_m;
    const double2 *col = tables + fd.tab_off, *rowc = col + W;
    const float *stT = stT_all + fd.pix_off;
    const int32_t *stN = stN_all + fd.pix_off;
    const int ltile = tile - fd.tile_off;
    const int ty = ltile / tiles_x, tx = ltile - ty * tiles_x;
    const int lane = threadIdx.x;
    const int i = ty * TH + strip * SR + (lane >> tws), j = tx * TW + (lane & (TW - 1));
    const bool inside = (i < H) && (j < W);
    const double2 cr = rowc[min(i, H - 1)], cc = col[min(j, W - 1)];
    const double vx = cr.x * cc.x, vy = cr.x * cc.y, vz = cr.y;
    const float fvx = (float)vx, fvy = (float)vy, fvz = (float)vz;
    const int2 rg = ranges[tile];
    const int wr0 = ty * TH + strip * SR, wr1 = wr0 + SR - 1;
    const int p = inside ? i * W + j : 0;
    const float Tfin = inside ? stT[p] : 1.0f;
    const int last = inside ? stN[p] : 0;
    int wlast = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wlast = max(wlast, __shfl_xor(wlast, o, 64));

    BwdState st = {Tfin, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, false};
    const BwdUpstream up = {1.0f, 0.0f, 0.0f, 0.0f, 0.0f, Tfin};   // dL/dD = 1
    float J[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    const int end = rg.x + wlast;   // entries at or beyond end precede no contributor of the strip
    // this strip's words of the contribution mask: entries no pixel of the strip composited are skipped
    const uint64_t *cm = cmask ? cmask + cmask_word(tile, rg.x, strip, 0) : nullptr;
    for (int c = wlast > 0 ? rg.x + ((wlast - 1) & ~63) : rg.x - 64; c >= rg.x; c -= 64) {
        bool meets = false;
        const uint64_t cw = mask_word(cm, 4 * ((c - rg.x) >> 6));
        if (c + lane < end && ((cw >> lane) & 1ull)) {
            sbuf[lane] = rec[pval[c + lane]];
            const uint32_t rows = sbuf[lane].rows;
            meets = !((int)(rows >> 16) < wr0 || (int)(rows & 0xffffu) > wr1);
        }
        if (meets) {
            double ba[3], bb[3], bc[3];
            record_axes(sbuf[lane], ba, bb, bc);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                sab[lane][q] = (float)ba[q];
                sab[lane][3 + q] = (float)bb[q];
            }
            stau[lane] = record_tau(sbuf[lane]);
        }
        const uint64_t m = __ballot(meets);
        const int nact = __popcll(m);
        if (meets)
            slist[__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                (uint8_t)lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int q = nact - 1; q >= 0; q -= 2) {
            // two entries per step: both evaluations ahead of the reverse chain
            const bool has1 = q >= 1;
            const int ka = slist[q], kb = slist[has1 ? q - 1 : q];
            PairEval ea, eb;
            const bool acta = eval_pair_flat(sbuf[ka], vx, vy, vz, near_m, ea) && c + ka - rg.x < last;
            const bool actb = eval_pair_flat(sbuf[kb], vx, vy, vz, near_m, eb) && c + kb - rg.x < last && has1;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h ? actb : acta) {
                    const int k = h ? kb : ka;
                    const PairEval &e = h ? eb : ea;
                    const RasterRec &r = sbuf[k];
                    const BwdScalars sc = bwd_step(st, e, r.n[0], r.n[1], r.n[2], up, range_low(e, stau[k]));
                    float jc[6];
                    gn_pair_row(sc, r, sab[k], e.t, fvx, fvy, fvz, jc);
#pragma unroll
                    for (int a = 0; a < 6; ++a) J[a] += jc[a];
                }
            }
        }
        // every lane is done with this chunk's records before they are replaced
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // this pixel's terms and the wave's sums (FP64 butterflies), as in k_raster_gn;
    // the strip rows follow the quad tiles' 16 rows each
    gn_row(fd, inside, p, J, gn_part + (size_t)kGnRow * (16 * (size_t)nquad + 4 * (size_t)(tslot - nquad) + strip), lane,
           tile_frame[tile]);
}


// Grid of a persistent kernel: as many workgroups of `threads` as the device
// holds at once (CU count x occupancy), at most `items`.
template <class K>
int64_t resident_grid(K kern, int threads, int64_t items)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) == hipSuccess && cus > 0 && per_cu > 0)
        return std::min<int64_t>(items, (int64_t)cus * per_cu);
    return items;
}

void fwd_launch(const Layout &L, char *ws, hipStream_t stream)
{
    const uint32_t *pval = reinterpret_cast<const uint32_t *>(ws + (L.tile_in_1 ? L.pv1 : L.pv0));
    const bool wave = L.variant == SLR_VARIANT_WAVE;
    if (wave) {
        const bool longest = longest_order(L);
        const int64_t items = wave_blocks(L.tiles) + (longest ? 16 * quad_tile_cap(L.tiles) : 0);
        const bool queue = L.schedule == SLR_SCHEDULE_QUEUE;
        auto kern = queue ? k_raster_fwd_w<true> : k_raster_fwd_w<false>;
        uint32_t *counter = reinterpret_cast<uint32_t *>(ws + L.misc + kMiscQueueFwd);
        const int64_t grid = queue ? resident_grid(kern, 64, items) : items;
        if (queue) launch_fill_u32(counter, 0u, 1, stream);
        uint64_t *cmask = reinterpret_cast<uint64_t *>(ws + L.cmask);
        // a strip stores the word of every chunk it walks (and the backward reads no
        // other); only quad sub-strips OR into their strip's words, which must start clear
        if (longest && quad_tile_cap(L.tiles) > 0) launch_fill_u32(cmask, 0u, 2 * L.cmask_words, stream);
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64), 0, stream,
                           reinterpret_cast<const FrameDesc *>(ws + L.desc),
                           reinterpret_cast<const int32_t *>(ws + L.tile_frame),
                           longest ? reinterpret_cast<const uint32_t *>(ws + L.order) : nullptr,
                           reinterpret_cast<const RasterRec *>(ws + L.rec), pval,
                           reinterpret_cast<const int2 *>(ws + L.ranges), reinterpret_cast<const double2 *>(ws + L.tables),
                           reinterpret_cast<float *>(ws + L.stateT), reinterpret_cast<int32_t *>(ws + L.stateN),
                           reinterpret_cast<int32_t *>(ws + L.census), L.pixels, L.tiles,
                           longest ? reinterpret_cast<const uint32_t *>(ws + L.misc + kMiscQuadTiles) : nullptr,
                           cmask, counter, items);
        return;
    }
    hipLaunchKernelGGL(L.variant == SLR_VARIANT_SCALAR ? k_raster_fwd_s : k_raster_fwd,
                       dim3((unsigned)L.tiles), dim3(256), 0, stream,
                       reinterpret_cast<const FrameDesc *>(ws + L.desc), reinterpret_cast<const int32_t *>(ws + L.tile_frame),
                       longest_order(L) ? reinterpret_cast<const uint32_t *>(ws + L.order) : nullptr,
                       reinterpret_cast<const RasterRec *>(ws + L.rec), pval, reinterpret_cast<const int2 *>(ws + L.ranges),
                       reinterpret_cast<const double2 *>(ws + L.tables), reinterpret_cast<float *>(ws + L.stateT),
                       reinterpret_cast<int32_t *>(ws + L.stateN), reinterpret_cast<int32_t *>(ws + L.census), L.pixels);
}

// The contribution mask, when the forward that preceded (same layout) wrote one.
inline const uint64_t *contribution_mask(const Layout &L, const char *ws)
{
    return L.variant == SLR_VARIANT_WAVE ? reinterpret_cast<const uint64_t *>(ws + L.cmask) : nullptr;
}

void bwd_launch(const Layout &L, char *ws, bool pose_only, hipStream_t stream)
{
    const uint32_t *pval = reinterpret_cast<const uint32_t *>(ws + (L.tile_in_1 ? L.pv1 : L.pv0));
    const uint64_t *cmask = contribution_mask(L, ws);
    const bool wave = L.bwd_variant == SLR_VARIANT_WAVE;
    const uint32_t *ord = longest_order(L) ? reinterpret_cast<const uint32_t *>(ws + L.order) : nullptr;
    if (wave) {
        const int64_t grid = wave_blocks(L.tiles) + (ord ? 16 * quad_tile_cap(L.tiles) : 0);
        hipLaunchKernelGGL(k_raster_bwd_w, dim3((unsigned)grid), dim3(64), 0, stream,
                           reinterpret_cast<const FrameDesc *>(ws + L.desc),
                           reinterpret_cast<const int32_t *>(ws + L.tile_frame), ord,
                           reinterpret_cast<const RasterRec *>(ws + L.rec), pval,
                           reinterpret_cast<const int2 *>(ws + L.ranges), reinterpret_cast<const double2 *>(ws + L.tables),
                           reinterpret_cast<const float *>(ws + L.stateT), reinterpret_cast<const int32_t *>(ws + L.stateN),
                           reinterpret_cast<int32_t *>(ws + L.census), L.pixels,
                           reinterpret_cast<double *>(ws + L.pose_part), pose_only ? 1 : 0, L.tiles,
                           ord ? reinterpret_cast<const uint32_t *>(ws + L.misc + kMiscQuadTiles) : nullptr, cmask);
        return;
    }
    const bool queue = L.schedule == SLR_SCHEDULE_QUEUE;
    const bool det = L.bwd_variant == SLR_VARIANT_DETERMINISTIC;
    auto kern = det ? (queue ? k_raster_bwd<kDetBatch, true, true> : k_raster_bwd<kDetBatch, false, true>)
                : L.bwd_batch == 128 ? (queue ? k_raster_bwd<128, true, false> : k_raster_bwd<128, false, false>)
                                     : (queue ? k_raster_bwd<kBwdBatch, true, false> : k_raster_bwd<kBwdBatch, false, false>);
    uint32_t *counter = reinterpret_cast<uint32_t *>(ws + L.misc + kMiscQueue);
    const int64_t grid = queue ? resident_grid(kern, 256, L.tiles) : L.tiles;
    if (queue) launch_fill_u32(counter, 0u, 1, stream);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), 0, stream,
                       reinterpret_cast<const FrameDesc *>(ws + L.desc), reinterpret_cast<const int32_t *>(ws + L.tile_frame),
                       ord, reinterpret_cast<const RasterRec *>(ws + L.rec), pval,
                       reinterpret_cast<const int2 *>(ws + L.ranges), reinterpret_cast<const double2 *>(ws + L.tables),
                       reinterpret_cast<const float *>(ws + L.stateT), reinterpret_cast<const int32_t *>(ws + L.stateN),
                       reinterpret_cast<int32_t *>(ws + L.census), L.pixels, reinterpret_cast<double *>(ws + L.pose_part),
                       pose_only ? 1 : 0, counter, (int)L.tiles, cmask,
                       det ? reinterpret_cast<const uint32_t *>(ws + L.rank) : nullptr,
                       reinterpret_cast<const uint32_t *>(ws + L.off), reinterpret_cast<const PixBox *>(ws + L.rbox),
                       det ? reinterpret_cast<float *>(ws + L.slots) : nullptr,
                       det ? reinterpret_cast<uint32_t *>(ws + L.slot_bits) : nullptr);
}

void gn_launch(const Layout &L, char *ws, hipStream_t stream)
{
    const uint32_t *pval = reinterpret_cast<const uint32_t *>(ws + (L.tile_in_1 ? L.pv1 : L.pv0));
    const uint64_t *cmask = contribution_mask(L, ws);
    const uint32_t *ord = longest_order(L) ? reinterpret_cast<const uint32_t *>(ws + L.order) : nullptr;
    if (L.bwd_variant == SLR_VARIANT_WAVE) {
        const int64_t grid = wave_blocks(L.tiles) + (ord ? 16 * quad_tile_cap(L.tiles) : 0);
        hipLaunchKernelGGL(k_raster_gn_w, dim3((unsigned)grid), dim3(64), 0, stream,
                           reinterpret_cast<const FrameDesc *>(ws + L.desc),
                           reinterpret_cast<const int32_t *>(ws + L.tile_frame), ord,
                           reinterpret_cast<const RasterRec *>(ws + L.rec), pval,
                           reinterpret_cast<const int2 *>(ws + L.ranges), reinterpret_cast<const double2 *>(ws + L.tables),
                           reinterpret_cast<const float *>(ws + L.stateT), reinterpret_cast<const int32_t *>(ws + L.stateN),
                           reinterpret_cast<double *>(ws + L.gn_part), L.tiles,
                           ord ? reinterpret_cast<const uint32_t *>(ws + L.misc + kMiscQuadTiles) : nullptr, cmask);
        return;
    }
    hipLaunchKernelGGL(k_raster_gn, dim3((unsigned)L.tiles), dim3(256), 0, stream,
                       reinterpret_cast<const FrameDesc *>(ws + L.desc), reinterpret_cast<const int32_t *>(ws + L.tile_frame),
                       ord, reinterpret_cast<const RasterRec *>(ws + L.rec), pval, reinterpret_cast<const int2 *>(ws + L.ranges), reinterpret_cast<const double2 *>(ws + L.tables),
                       reinterpret_cast<const float *>(ws + L.stateT), reinterpret_cast<const int32_t *>(ws + L.stateN),
                       reinterpret_cast<double *>(ws + L.gn_part), cmask);
}

}  // namespace

void launch_raster_fwd(const Layout &L, char *ws, hipStream_t stream)
{
    if (L.tiles == 0) return;
    fwd_launch(L, ws, stream);
}

void launch_raster_bwd(const Layout &L, char *ws, bool pose_only, hipStream_t stream)
{
    if (L.tiles == 0) return;
    bwd_launch(L, ws, pose_only, stream);
}

void launch_raster_gn(const Layout &L, char *ws, hipStream_t stream)
{
    if (L.tiles == 0) return;
    gn_launch(L, ws, stream);
}

}  // namespace slr

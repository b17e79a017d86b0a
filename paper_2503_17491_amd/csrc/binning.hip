// binning.hip -- per-tile, range-sorted surfel lists (Sec. 3.2.1) on gfx950.
//
// The lists are the pairs (tile, surfel) ordered by (tile, range key, surfel
// index).  They are produced by a least-significant-digit radix sort on the
// composite (tile, range) key, split in two stages because all pairs of one
// surfel share its range digits:
//   0. the surfels that bin into at least one tile are compacted, in index
//      order, into (range key, index) pairs: on a LiDAR frame a third or more
//      of the map is behind the sensor, culled or outside the image;
//   1. the range digits are sorted at surfel granularity: a stable LSD radix
//      sort of those pairs (8-bit digits, 4 passes);
//   2. the pairs are emitted in that order (exclusive scan of the per-surfel
//      tile counts, then blocks of a fixed number of output slots expand the
//      surfels that cover them);
//   3. the tile digits are sorted with the same stable LSD radix passes over
//      the K pairs (ceil(log2 tiles / 8) passes);
//   4. tile ranges [start, end) from key boundaries.
// Every step is integer-only and deterministic.
//
// The radix pass is the classic three-kernel form: per-block digit histograms,
// a per-digit scan over blocks, and a scatter whose in-block ranks are stable.
// Ranks come from 64-lane ballots: for each row of 64 consecutive items a wave
// forms, per lane, the mask of lanes holding the same digit (one ballot per
// digit bit), so the rank in the row is a popcount and a per-wave running
// counter in LDS carries the rank across rows.
#include "slr_internal.h"

namespace slr {
namespace {

constexpr int kWaves = kSortThreads / 64;
constexpr int kEmitThreads = 256;
constexpr int kScanItems = 16;                         // per thread in the per-digit scan over blocks
constexpr int kScanChunk = kSortThreads * kScanItems;

__device__ inline uint64_t lanemask_lt() { return (1ull << (threadIdx.x & 63)) - 1ull; }

// Exclusive scan across a 256-thread block; returns the prefix, *total = sum.
__device__ uint32_t block_exscan(uint32_t v, uint32_t *s_wave, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        uint32_t s = s_wave[w];
        pre += (w < wid) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
k_radix_hist(const uint32_t *__restrict__ keys, int64_t n_max, const uint64_t *__restrict__ n_dev, int shift,
             int bits, uint32_t *__restrict__ hist, int nblocks)
{
    __shared__ uint32_t h[256];
    const int64_t n = n_dev ? (int64_t)min((uint64_t)n_max, *n_dev) : n_max;
    const int nb = 1 << bits;
    for (int d = threadIdx.x; d < nb; d += kSortThreads) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (kSortThreads * ITEMS);
    const uint32_t mask = (uint32_t)nb - 1u;
#pragma unroll 4
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < nb; d += kSortThreads) hist[(int64_t)d * nblocks + blockIdx.x] = h[d];
}

// One block per digit: exclusive scan of that digit's counts over blocks.
__global__ void __launch_bounds__(kSortThreads)
k_radix_rowscan(uint32_t *__restrict__ hist, int nblocks, uint32_t *__restrict__ totals)
{
    __shared__ uint32_t s_wave[kWaves];
    __shared__ uint32_t s_items[kScanChunk];
    uint32_t *row = hist + (int64_t)blockIdx.x * nblocks;
    uint32_t carry = 0;
    // chunks of kScanChunk counts: coalesced loads into LDS, kScanItems
    // consecutive counts per thread, one block scan per chunk
    for (int c0 = 0; c0 < nblocks; c0 += kScanChunk) {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const int b = c0 + i * kSortThreads + threadIdx.x;
            s_items[i * kSortThreads + threadIdx.x] = b < nblocks ? row[b] : 0u;
        }
        __syncthreads();
        uint32_t local[kScanItems], sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            local[i] = sum;
            sum += s_items[threadIdx.x * kScanItems + i];
        }
        uint32_t tot;
        const uint32_t pre = carry + block_exscan(sum, s_wave, &tot);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) s_items[threadIdx.x * kScanItems + i] = pre + local[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const int b = c0 + i * kSortThreads + threadIdx.x;
            if (b < nblocks) row[b] = s_items[i * kSortThreads + threadIdx.x];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
k_radix_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
                uint32_t *__restrict__ vout, int64_t n_max, const uint64_t *__restrict__ n_dev, int shift, int bits,
                const uint32_t *__restrict__ hist, const uint32_t *__restrict__ totals, int nblocks,
                const PixBox *__restrict__ box_in, uint32_t *__restrict__ cnt_out, PixBox *__restrict__ box_out)
{
    const int64_t n = n_dev ? (int64_t)min((uint64_t)n_max, *n_dev) : n_max;
    // the grid is sized for the capacity: blocks past the items have nothing to move
    if ((int64_t)blockIdx.x * (kSortThreads * ITEMS) >= n) return;
    __shared__ uint32_t s_base[256], s_start[256], s_gbase[256];
    __shared__ uint32_t s_cnt[kWaves][256];
    __shared__ uint32_t s_wave[kWaves];
    __shared__ uint32_t s_key[(kSortThreads * ITEMS)], s_val[(kSortThreads * ITEMS)];
    const int nb = 1 << bits;
    const uint32_t mask = (uint32_t)nb - 1u;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    // digit bases: exclusive scan of the global digit totals
    {
        uint32_t v = threadIdx.x < nb ? totals[threadIdx.x] : 0u;
        uint32_t tot;
        uint32_t ex = block_exscan(v, s_wave, &tot);
        s_base[threadIdx.x] = ex;
    }
    for (int d = lane; d < 256; d += 64) s_cnt[wid][d] = 0;
    __syncthreads();

    const int64_t base = (int64_t)blockIdx.x * (kSortThreads * ITEMS) + (int64_t)wid * ((kSortThreads * ITEMS) / kWaves);
    uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * 64 + lane;
        bool valid = idx < n;
        key[i] = valid ? kin[idx] : 0u;
        val[i] = valid ? vin[idx] : 0u;
        uint32_t d = (key[i] >> shift) & mask;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            uint64_t bb = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bb : ~bb;
        }
        uint32_t before = (uint32_t)__popcll(m & lt);
        uint32_t prev = valid ? s_cnt[wid][d] : 0u;
        rank[i] = prev + before;
        // the highest lane of each digit group publishes the new running count
        if (valid && (m >> lane) == 1ull) s_cnt[wid][d] = prev + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit (one per thread): the waves' offsets within the block's group of
    // that digit, the group's size, then the groups' starts in the block
    uint32_t dcount = 0;
    if ((int)threadIdx.x < nb) {
        uint32_t off = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t c = s_cnt[w][threadIdx.x];
            s_cnt[w][threadIdx.x] = off;
            off += c;
        }
        dcount = off;
    }
    uint32_t tot;
    const uint32_t dstart = block_exscan(dcount, s_wave, &tot);
    if ((int)threadIdx.x < nb) {
        s_start[threadIdx.x] = dstart;
        s_gbase[threadIdx.x] = s_base[threadIdx.x] + hist[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    }
    __syncthreads();
    // the block's items in LDS in digit order (stable: wave, then item order)
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = base + (int64_t)i * 64 + lane;
        if (idx < n) {
            const uint32_t d = (key[i] >> shift) & mask;
            const uint32_t lp = s_start[d] + s_cnt[wid][d] + rank[i];
            s_key[lp] = key[i];
            s_val[lp] = val[i];
        }
    }
    __syncthreads();
    // each digit's run goes out to consecutive addresses from consecutive threads
    const int64_t b0 = (int64_t)blockIdx.x * (kSortThreads * ITEMS);
    const int nvalid = (int)min((int64_t)(kSortThreads * ITEMS), n - b0);
    for (int j = threadIdx.x; j < nvalid; j += kSortThreads) {
        const uint32_t k = s_key[j], v = s_val[j];
        const uint32_t d = (k >> shift) & mask;
        const uint32_t pos = s_gbase[d] + ((uint32_t)j - s_start[d]);
        kout[pos] = k;
        vout[pos] = v;
        // optionally the record's box (with its tile count) follows it into sorted order
        if (box_out) {
            const PixBox bx = box_in[v];
            box_out[pos] = bx;
            cnt_out[pos] = bx.cnt;
        }
    }
}

// ---- scan of tile counts in range order ----
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
k_scan_reduce(const uint32_t *__restrict__ rcounts, int64_t n_max, const uint64_t *__restrict__ n_dev,
              uint32_t *__restrict__ blocksum)
{
    __shared__ uint32_t s_wave[kWaves];
    const int64_t n = (int64_t)min((uint64_t)n_max, *n_dev);
    const int64_t base = (int64_t)blockIdx.x * (kSortThreads * ITEMS);
    uint32_t acc = 0;
#pragma unroll 4
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        if (idx < n) acc += rcounts[idx];
    }
    uint32_t tot;
    block_exscan(acc, s_wave, &tot);
    if (threadIdx.x == 0) blocksum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kSortThreads)
k_scan_blocks(uint32_t *__restrict__ blocksum, int nblocks, uint64_t *__restrict__ total_out, int64_t cap)
{
    __shared__ uint32_t s_wave[kWaves];
    uint64_t carry = 0;
    for (int b0 = 0; b0 < nblocks; b0 += kSortThreads) {
        int b = b0 + threadIdx.x;
        uint32_t v = b < nblocks ? blocksum[b] : 0u;
        uint32_t tot;
        uint32_t ex = block_exscan(v, s_wave, &tot);
        if (b < nblocks) blocksum[b] = (uint32_t)carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        total_out[0] = carry;
        // pair-capacity check (cap >= 0): the effective pair count is K, or 0
        // with the overflow word set to K when K exceeds the capacity
        if (cap >= 0) {
            total_out[1] = carry > (uint64_t)cap ? carry : 0;
            total_out[2] = carry > (uint64_t)cap ? 0 : carry;
        }
    }
}

template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
k_scan_apply(const uint32_t *__restrict__ rcounts, int64_t n_max, const uint64_t *__restrict__ n_dev,
             const uint32_t *__restrict__ blocksum, uint32_t *__restrict__ offsets, uint32_t *__restrict__ estart,
             uint64_t cap)
{
    __shared__ uint32_t s_wave[kWaves];
    __shared__ uint32_t s_items[(kSortThreads * ITEMS)];
    const int64_t n = (int64_t)min((uint64_t)n_max, *n_dev);
    const int64_t base = (int64_t)blockIdx.x * (kSortThreads * ITEMS);
#pragma unroll 4
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        s_items[i * kSortThreads + threadIdx.x] = idx < n ? rcounts[idx] : 0u;
    }
    __syncthreads();
    // each thread scans a contiguous run of ITEMS
    uint32_t local[ITEMS], sum = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        local[i] = sum;
        sum += s_items[threadIdx.x * ITEMS + i];
    }
    uint32_t tot;
    uint32_t pre = block_exscan(sum, s_wave, &tot) + blocksum[blockIdx.x];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) s_items[threadIdx.x * ITEMS + i] = pre + local[i];
    __syncthreads();
#pragma unroll 4
    for (int i = 0; i < ITEMS; ++i) {
        int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        if (idx < n) {
            const uint32_t o = s_items[i * kSortThreads + threadIdx.x];
            offsets[idx] = o;
            // the record holding the first slot of emit block m: exactly one
            // record covers each slot m kEmitSlots < K (blocks past the pair
            // capacity are never emitted)
            const uint64_t e = min((uint64_t)o + rcounts[idx], cap);
            for (uint64_t m = ((uint64_t)o + kEmitSlots - 1) / kEmitSlots; m * kEmitSlots < e; ++m)
                estart[m] = (uint32_t)idx;
        }
    }
}

// ---- compaction of the records that bin into some tile ----
// Records without a tile (culled, behind, outside the image: count 0) do not
// enter the range sort.  The visible ones keep their index order, so the
// stable sort still breaks range ties by index.
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
k_vis_count(const int32_t *__restrict__ cnt, int64_t n, uint32_t *__restrict__ blocksum)
{
    __shared__ uint32_t s_wave[kWaves];
    const int64_t base = (int64_t)blockIdx.x * (kSortThreads * ITEMS);
    uint32_t acc = 0;
#pragma unroll 4
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        if (idx < n) acc += cnt[idx] > 0 ? 1u : 0u;
    }
    uint32_t tot;
    block_exscan(acc, s_wave, &tot);
    if (threadIdx.x == 0) blocksum[blockIdx.x] = tot;
}

// Ranks are row-major like the radix scatter's: items base + i kSortThreads +
// t, so every wave's surviving lanes of one row write consecutive slots.
template <int ITEMS>
__global__ void __launch_bounds__(kSortThreads)
k_vis_write(const uint32_t *__restrict__ keys, const int32_t *__restrict__ cnt, int64_t n,
            const uint32_t *__restrict__ blocksum, uint32_t *__restrict__ kout, uint32_t *__restrict__ vout)
{
    constexpr int kSlots = ITEMS * kWaves;
    __shared__ uint32_t s_pre[kSlots];   // (row, wave) -> rank of its first survivor in the block
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * (kSortThreads * ITEMS);
    uint64_t mask[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
        mask[i] = __ballot(idx < n && cnt[idx] > 0);
        if (lane == 0) s_pre[i * kWaves + wid] = (uint32_t)__popcll(mask[i]);
    }
    __syncthreads();
    if (wid == 0) {
        uint32_t carry = 0;
        for (int c0 = 0; c0 < kSlots; c0 += 64) {
            const int c = c0 + lane;
            const uint32_t v = c < kSlots ? s_pre[c] : 0u;
            uint32_t x = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (c < kSlots) s_pre[c] = carry + x - v;
            carry += __shfl(x, 63, 64);
        }
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    const uint32_t b0 = blocksum[blockIdx.x];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if ((mask[i] >> lane) & 1ull) {
            const int64_t idx = base + (int64_t)i * kSortThreads + threadIdx.x;
            const uint32_t pos = b0 + s_pre[i * kWaves + wid] + (uint32_t)__popcll(mask[i] & lt);
            kout[pos] = keys[idx];
            vout[pos] = (uint32_t)idx;
        }
    }
}

// Pairs of the records in range order, kEmitSlots output slots per block.
// The pair counts are skewed (the nearest surfels come first in range order
// and span the most tiles), so the work is split by slots, not by records:
// block m fills slots [m S, m S + S) and decodes into LDS the records that
// cover them, from the one the scan marked as holding slot m S on.  Every
// record has at least one pair, so a block sees at most S + 1 records.  A
// slot's record is the last one whose offset is <= the slot; within a record
// the slots go row by row, and in a row the first column interval, then the
// second.  Consecutive threads write consecutive pairs of slots.
__global__ void __launch_bounds__(kEmitThreads)
k_emit(const FrameDesc *__restrict__ descs, const uint32_t *__restrict__ order, const uint32_t *__restrict__ offsets,
       const PixBox *__restrict__ rbox, const uint32_t *__restrict__ estart, const uint64_t *__restrict__ n_dev,
       const uint64_t *__restrict__ keff, uint32_t *__restrict__ ptile, uint32_t *__restrict__ pval)
{
    constexpr int kRecs = kEmitSlots + 1;
    __shared__ uint32_t s_off[kRecs], s_id[kRecs], s_row0[kRecs];
    __shared__ int32_t s_ty0[kRecs], s_ax0[kRecs], s_na[kRecs], s_bx0[kRecs], s_len[kRecs], s_tx[kRecs];
    const uint64_t K = *keff, n = *n_dev;
    const uint64_t q0 = (uint64_t)blockIdx.x * kEmitSlots;
    if (q0 >= K || n == 0) return;
    const uint64_t qend = q0 + kEmitSlots < K ? q0 + kEmitSlots : K;
    const uint32_t k0 = estart[blockIdx.x];
    uint64_t klast = qend < K ? (uint64_t)estart[blockIdx.x + 1] : n - 1;
    klast = klast < n - 1 ? klast : n - 1;
    const int nrec = klast < k0 ? 1 : (int)min(klast - k0 + 1, (uint64_t)kRecs);
    for (int i = threadIdx.x; i < nrec; i += kEmitThreads) {
        const uint32_t r = k0 + (uint32_t)i;
        const PixBox b = rbox[r];
        const FrameDesc &fd = descs[b.frame];
        const TileSpan sp = tile_span(b, fd.th, fd.tw);
        s_off[i] = offsets[r];
        s_id[i] = order[r];
        s_ty0[i] = sp.ty0;
        s_ax0[i] = sp.ax0;
        s_na[i] = sp.na;
        s_bx0[i] = sp.bx0;
        s_len[i] = sp.len;
        s_tx[i] = fd.tiles_x;
        s_row0[i] = (uint32_t)fd.tile_off;
    }
    __syncthreads();
    // two consecutive slots per thread: a search for the first, and the second
    // is in the same record or the next one
    static_assert(kEmitSlots == 2 * kEmitThreads, "two slots per thread");
    const uint64_t q = q0 + 2 * (uint64_t)threadIdx.x;
    if (q >= qend) return;
    const uint32_t qq = (uint32_t)q;
    int lo = 0;
#pragma unroll
    for (int step = kEmitSlots; step > 0; step >>= 1)
        if (lo + step < nrec && s_off[lo + step] <= qq) lo += step;
    uint32_t tile[2], val[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (h == 1 && lo + 1 < nrec && s_off[lo + 1] <= qq + 1) ++lo;
        const int j = (int)(qq + h - s_off[lo]);
        const int len = s_len[lo], na = s_na[lo];
        const int dy = j / len, cc = j - dy * len;
        const int tx = cc < na ? s_ax0[lo] + cc : s_bx0[lo] + (cc - na);
        tile[h] = s_row0[lo] + (uint32_t)((s_ty0[lo] + dy) * s_tx[lo] + tx);
        val[h] = s_id[lo];
    }
    if (q + 1 < qend) {   // q is even: an aligned pair of slots
        *reinterpret_cast<uint2 *>(ptile + q) = make_uint2(tile[0], tile[1]);
        *reinterpret_cast<uint2 *>(pval + q) = make_uint2(val[0], val[1]);
    } else {
        ptile[q] = tile[0];
        pval[q] = val[0];
    }
}

__global__ void __launch_bounds__(256)
k_ranges(const uint32_t *__restrict__ ptile, const uint64_t *__restrict__ keff, int2 *__restrict__ ranges)
{
    const int64_t K = (int64_t)*keff;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < K; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t t = ptile[p];
        if (p == 0 || ptile[p - 1] != t) ranges[t].x = (int)p;
        if (p == K - 1 || ptile[p + 1] != t) ranges[t].y = (int)(p + 1);
    }
}

// Longest-first tile schedule: tiles are bucketed by their list length on a
// half-octave scale (bucket 0 = empty) and written out in descending bucket
// order, so the compositing kernels, which take tile order[blockIdx.x], start
// the long lists first and fill the end of the launch with short ones.  One
// workgroup.  Within a bucket the tiles keep their index order (a stable
// counting sort), so the order depends only on the list lengths: the partial
// rows the compositing kernels write per tile slot, which fixed-order
// reductions add up slot by slot, then come out the same on every render.
constexpr int kOrderBuckets = 65;
constexpr int kOrderThreads = 1024;

__device__ __forceinline__ int order_bucket(int len)
{
    if (len <= 0) return 0;
    const int e = 31 - __clz(len);
    const int half = e > 0 ? (len >> (e - 1)) & 1 : 0;
    return 1 + 2 * e + half;
}

__global__ void __launch_bounds__(kOrderThreads)
k_tile_order(const int2 *__restrict__ ranges, int64_t tiles, uint32_t *__restrict__ order,
             uint32_t *__restrict__ nquad)
{
    constexpr int kW = kOrderThreads / 64;
    __shared__ uint32_t hist[kOrderBuckets];
    __shared__ uint32_t wcnt[kW][kOrderBuckets];   // per wave of a chunk: its tiles per bucket, then their first slot
    for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    for (int64_t t = threadIdx.x; t < tiles; t += blockDim.x) {
        const int2 r = ranges[t];
        atomicAdd(&hist[order_bucket(r.y - r.x)], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the tiles whose list reaches kQuadMinList entries fill the first slots of
        // the order (their buckets come first); the forward's quad mode takes them,
        // rounded up to whole runs of 8 slots, at most quad_tile_cap
        uint32_t acc = 0, nl = 0;
        const int qb = order_bucket(kQuadMinList);
        for (int b = kOrderBuckets - 1; b >= 0; --b) {
            const uint32_t c = hist[b];
            hist[b] = acc;
            acc += c;
            if (b == qb) nl = acc;
        }
        const uint64_t cap = (uint64_t)quad_tile_cap(tiles);
        const uint64_t n8 = ((uint64_t)nl + 7) & ~uint64_t(7);
        *nquad = (uint32_t)(n8 < cap ? n8 : cap);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    // chunks of kOrderThreads tiles in index order; in a chunk, waves in order
    // and lanes in order: a tile's slot is its bucket's next free slot plus the
    // tiles of its bucket before it in the chunk
    for (int64_t base = 0; base < tiles; base += kOrderThreads) {
        for (int e = threadIdx.x; e < kW * kOrderBuckets; e += blockDim.x) (&wcnt[0][0])[e] = 0u;
        __syncthreads();
        const int64_t t = base + threadIdx.x;
        int b = -1;
        if (t < tiles) {
            const int2 r = ranges[t];
            b = order_bucket(r.y - r.x);
        }
        // the lanes of this wave with the same bucket (one ballot per distinct bucket)
        uint64_t peers = 0;
        uint64_t todo = __ballot(b >= 0);
        while (todo) {
            const int lb = __shfl(b, __ffsll((unsigned long long)todo) - 1, 64);
            const uint64_t m = __ballot(b == lb);
            if (b == lb) peers = m;
            todo &= ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (b >= 0 && rank == 0) wcnt[wid][b] = (uint32_t)__popcll(peers);
        __syncthreads();
        if ((int)threadIdx.x < kOrderBuckets) {
            const int bb = threadIdx.x;
            uint32_t acc = hist[bb];
            for (int w = 0; w < kW; ++w) {
                const uint32_t c = wcnt[w][bb];
                wcnt[w][bb] = acc;
                acc += c;
            }
            hist[bb] = acc;
        }
        __syncthreads();
        if (b >= 0) order[wcnt[wid][b] + rank] = (uint32_t)t;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// One LSD pass; swaps the roles of (k0,v0) and (k1,v1).
// n_max sizes the grid; n_dev (nullable) holds the actual count on the device.
template <int ITEMS>
void radix_pass_t(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, int64_t n_max,
                  const uint64_t *n_dev, int shift, int bits, uint32_t *hist, uint32_t *totals, hipStream_t stream,
                  const PixBox *box_in, uint32_t *cnt_out, PixBox *box_out)
{
    const int nblocks = (int)((n_max + kSortThreads * ITEMS - 1) / (kSortThreads * ITEMS));
    hipLaunchKernelGGL(k_radix_hist<ITEMS>, dim3(nblocks), dim3(kSortThreads), 0, stream, kin, n_max, n_dev, shift, bits,
                       hist, nblocks);
    hipLaunchKernelGGL(k_radix_rowscan, dim3(1 << bits), dim3(kSortThreads), 0, stream, hist, nblocks, totals);
    hipLaunchKernelGGL(k_radix_scatter<ITEMS>, dim3(nblocks), dim3(kSortThreads), 0, stream, kin, vin, kout, vout, n_max,
                       n_dev, shift, bits, hist, totals, nblocks, box_in, cnt_out, box_out);
}

void radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, int64_t n_max,
                const uint64_t *n_dev, int shift, int bits, uint32_t *hist, uint32_t *totals, hipStream_t stream,
                const PixBox *box_in = nullptr, uint32_t *cnt_out = nullptr, PixBox *box_out = nullptr)
{
    switch (sort_items(n_max)) {
    case 4: radix_pass_t<4>(kin, vin, kout, vout, n_max, n_dev, shift, bits, hist, totals, stream, box_in, cnt_out, box_out); break;
    case 8: radix_pass_t<8>(kin, vin, kout, vout, n_max, n_dev, shift, bits, hist, totals, stream, box_in, cnt_out, box_out); break;
    default: radix_pass_t<16>(kin, vin, kout, vout, n_max, n_dev, shift, bits, hist, totals, stream, box_in, cnt_out, box_out);
    }
}

template <int ITEMS>
void compact_visible_t(const uint32_t *ks, const int32_t *cnt, int64_t items, uint32_t *bs, uint64_t *nvis, uint32_t *k0,
                       uint32_t *v0, hipStream_t stream)
{
    const int nblocks = (int)((items + kSortThreads * ITEMS - 1) / (kSortThreads * ITEMS));
    hipLaunchKernelGGL(k_vis_count<ITEMS>, dim3(nblocks), dim3(kSortThreads), 0, stream, cnt, items, bs);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kSortThreads), 0, stream, bs, nblocks, nvis, (int64_t)-1);
    hipLaunchKernelGGL(k_vis_write<ITEMS>, dim3(nblocks), dim3(kSortThreads), 0, stream, ks, cnt, items, bs, k0, v0);
}

template <int ITEMS>
void scan_counts_t(const uint32_t *rcounts, int64_t items, const uint64_t *nvis, uint32_t *bs, uint64_t *misc,
                   int64_t cap, uint32_t *off, uint32_t *estart, hipStream_t stream)
{
    const int nblocks = (int)((items + kSortThreads * ITEMS - 1) / (kSortThreads * ITEMS));
    hipLaunchKernelGGL(k_scan_reduce<ITEMS>, dim3(nblocks), dim3(kSortThreads), 0, stream, rcounts, items, nvis, bs);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kSortThreads), 0, stream, bs, nblocks, misc, cap);
    hipLaunchKernelGGL(k_scan_apply<ITEMS>, dim3(nblocks), dim3(kSortThreads), 0, stream, rcounts, items, nvis, bs, off,
                       estart, (uint64_t)cap);
}

}  // namespace

void launch_fill_u32(void *p, uint32_t v, int64_t count, hipStream_t stream)
{
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                       reinterpret_cast<uint32_t *>(p), v, count);
}

void launch_depth_sort(const Layout &L, char *ws, hipStream_t stream)
{
    if (L.items == 0) return;
    const uint32_t *ks = reinterpret_cast<const uint32_t *>(ws + L.skey);
    uint32_t *k0 = reinterpret_cast<uint32_t *>(ws + L.key0), *v0 = reinterpret_cast<uint32_t *>(ws + L.val0);
    uint32_t *k1 = reinterpret_cast<uint32_t *>(ws + L.key1), *v1 = reinterpret_cast<uint32_t *>(ws + L.val1);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    uint32_t *totals = reinterpret_cast<uint32_t *>(ws + L.misc + 64);
    uint64_t *nvis = reinterpret_cast<uint64_t *>(ws + L.misc) + 3;
    // the records that bin into some tile, in index order, into (key0, val0)
    const int32_t *cnt = reinterpret_cast<const int32_t *>(ws + L.cnt);
    uint32_t *bs = reinterpret_cast<uint32_t *>(ws + L.blocksum);
    switch (sort_items(L.items)) {
    case 4: compact_visible_t<4>(ks, cnt, L.items, bs, nvis, k0, v0, stream); break;
    case 8: compact_visible_t<8>(ks, cnt, L.items, bs, nvis, k0, v0, stream); break;
    default: compact_visible_t<16>(ks, cnt, L.items, bs, nvis, k0, v0, stream);
    }
    for (int p = 0; p < L.depth_passes; ++p) {
        const bool even = (p % 2) == 0;
        const bool last = p == L.depth_passes - 1;
        radix_pass(even ? k0 : k1, even ? v0 : v1, even ? k1 : k0, even ? v1 : v0, L.items, nvis, 8 * p, 8, hist, totals,
                   stream, last ? reinterpret_cast<const PixBox *>(ws + L.box) : nullptr,
                   last ? reinterpret_cast<uint32_t *>(ws + L.rcnt) : nullptr,
                   last ? reinterpret_cast<PixBox *>(ws + L.rbox) : nullptr);
    }
}

void launch_scan_counts(const Layout &L, char *ws, hipStream_t stream)
{
    uint64_t *misc = reinterpret_cast<uint64_t *>(ws + L.misc);
    if (L.items == 0) {
        launch_fill_u32(misc, 0u, 8, stream);
        return;
    }
    const uint64_t *nvis = misc + 3;
    const uint32_t *rcounts = reinterpret_cast<const uint32_t *>(ws + L.rcnt);   // in range order
    uint32_t *bs = reinterpret_cast<uint32_t *>(ws + L.blocksum);
    uint32_t *off = reinterpret_cast<uint32_t *>(ws + L.off), *est = reinterpret_cast<uint32_t *>(ws + L.estart);
    switch (sort_items(L.items)) {
    case 4: scan_counts_t<4>(rcounts, L.items, nvis, bs, misc, L.cap, off, est, stream); break;
    case 8: scan_counts_t<8>(rcounts, L.items, nvis, bs, misc, L.cap, off, est, stream); break;
    default: scan_counts_t<16>(rcounts, L.items, nvis, bs, misc, L.cap, off, est, stream);
    }
}

static void launch_tile_order(const Layout &L, char *ws, hipStream_t stream)
{
    if (!longest_order(L) || L.tiles == 0) return;
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, stream, reinterpret_cast<const int2 *>(ws + L.ranges),
                       L.tiles, reinterpret_cast<uint32_t *>(ws + L.order),
                       reinterpret_cast<uint32_t *>(ws + L.misc + kMiscQuadTiles));
}

void launch_emit_and_tile_sort(const Layout &L, char *ws, hipStream_t stream)
{
    int2 *ranges = reinterpret_cast<int2 *>(ws + L.ranges);
    launch_fill_u32(ranges, 0u, 2 * L.tiles, stream);
    if (L.items == 0 || L.cap == 0) {
        launch_tile_order(L, ws, stream);
        return;
    }
    const uint64_t *keff = reinterpret_cast<const uint64_t *>(ws + L.misc) + 2;
    const uint32_t *order = reinterpret_cast<const uint32_t *>(ws + (L.depth_in_1 ? L.val1 : L.val0));
    uint32_t *t0 = reinterpret_cast<uint32_t *>(ws + L.pt0), *v0 = reinterpret_cast<uint32_t *>(ws + L.pv0);
    uint32_t *t1 = reinterpret_cast<uint32_t *>(ws + L.pt1), *v1 = reinterpret_cast<uint32_t *>(ws + L.pv1);
    hipLaunchKernelGGL(k_emit, dim3((unsigned)((L.cap + kEmitSlots - 1) / kEmitSlots)), dim3(kEmitThreads), 0, stream,
                       reinterpret_cast<const FrameDesc *>(ws + L.desc), order,
                       reinterpret_cast<const uint32_t *>(ws + L.off), reinterpret_cast<const PixBox *>(ws + L.rbox),
                       reinterpret_cast<const uint32_t *>(ws + L.estart),
                       reinterpret_cast<const uint64_t *>(ws + L.misc) + 3, keff, t0, v0);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    uint32_t *totals = reinterpret_cast<uint32_t *>(ws + L.misc + 64);
    // split the tile bits evenly over the passes (each <= 8 bits)
    int done = 0;
    for (int p = 0; p < L.tile_passes; ++p) {
        int bits = (L.tile_bits - done + (L.tile_passes - p) - 1) / (L.tile_passes - p);
        const bool even = (p % 2) == 0;
        radix_pass(even ? t0 : t1, even ? v0 : v1, even ? t1 : t0, even ? v1 : v0, L.cap, keff, done, bits, hist,
                   totals, stream);
        done += bits;
    }
    const uint32_t *ts = L.tile_in_1 ? t1 : t0;
    const int64_t rblocks = (L.cap + 255) / 256;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)(rblocks < 8192 ? rblocks : 8192)), dim3(256), 0, stream, ts, keff,
                       ranges);
    launch_tile_order(L, ws, stream);
}

}  // namespace slr

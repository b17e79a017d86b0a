// capi.cpp -- C ABI of the spherical surfel rasterizer: argument validation,
// workspace layout, host-made sensor tables, frame descriptors and launch
// orchestration.  The plain calls (slr_render / slr_backward) are the batch
// of one frame plus a host read-back of the pair count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "slr_internal.h"

using slr::FrameDesc;
using slr::FrameGeom;
using slr::Layout;

namespace {

thread_local std::string g_last_error;

slr_status fail(slr_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(SLR_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int ceil_log2(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b < 1 ? 1 : b;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

slr_status check_sensor(const slr_sensor *s)
{
    if (!s) return fail(SLR_E_INVALID, "sensor is NULL");
    if (s->height <= 0 || s->width <= 0 || s->height > 32767 || s->width > 32767)
        return fail(SLR_E_INVALID, "image size %d x %d out of range [1, 32767]", s->height, s->width);
    // the kernels index pixels and the three normal channels with 32-bit integers
    if (3 * (int64_t)s->height * s->width >= (int64_t(1) << 31))
        return fail(SLR_E_INVALID, "image size %d x %d: 3 H W must stay below 2^31", s->height, s->width);
    if (!(s->fu < 0.0) || !(s->fv < 0.0) || !std::isfinite(s->fu) || !std::isfinite(s->fv) ||
        !std::isfinite(s->cu) || !std::isfinite(s->cv))
        return fail(SLR_E_INVALID, "camera matrix must be finite with fu < 0 and fv < 0");
    if (!(s->near_m >= 0.0) || !std::isfinite(s->near_m)) return fail(SLR_E_INVALID, "near_m must be >= 0");
    // the planes h_x, h_y of a pixel ray are undefined at the poles
    const double el_top = (0.5 - s->cv) / s->fv, el_bot = ((double)s->height - 0.5 - s->cv) / s->fv;
    const double lim = 89.0 * M_PI / 180.0;
    if (std::fabs(el_top) >= lim || std::fabs(el_bot) >= lim)
        return fail(SLR_E_INVALID, "vertical field of view reaches +-89 degrees");
    const double az0 = (0.5 - s->cu) / s->fu, az1 = ((double)s->width - 0.5 - s->cu) / s->fu;
    if (std::fabs(az0) > M_PI + 1e-9 || std::fabs(az1) > M_PI + 1e-9)
        return fail(SLR_E_INVALID, "column azimuths must lie within [-pi, pi]");
    return SLR_OK;
}

bool tile_shape_ok(int32_t th, int32_t tw)
{
    return (th == 16 && tw == 16) || (th == 8 && tw == 32) || (th == 32 && tw == 8) || (th == 4 && tw == 64);
}

slr_status check_tiling(const slr_tiling *t)
{
    if (!t) return fail(SLR_E_INVALID, "tiling is NULL");
    if (!tile_shape_ok(t->tile_h, t->tile_w)) return fail(SLR_E_INVALID, "unsupported tile shape %dx%d", t->tile_h, t->tile_w);
    if (t->variant < SLR_VARIANT_DEFAULT || t->variant > SLR_VARIANT_WAVE)
        return fail(SLR_E_INVALID, "unknown compositing variant %d", t->variant);
    if (t->bwd_variant != SLR_VARIANT_DEFAULT && t->bwd_variant != SLR_VARIANT_LDS && t->bwd_variant != SLR_VARIANT_WAVE &&
        t->bwd_variant != SLR_VARIANT_DETERMINISTIC)
        return fail(SLR_E_INVALID, "unknown backward variant %d (0, 1, 3 or 4)", t->bwd_variant);
    if (t->bwd_batch != 0 && t->bwd_batch != 128 && t->bwd_batch != 192)
        return fail(SLR_E_INVALID, "unsupported backward batch %d (0, 128 or 192)", t->bwd_batch);
    if (t->schedule < SLR_SCHEDULE_DEFAULT || t->schedule > SLR_SCHEDULE_QUEUE)
        return fail(SLR_E_INVALID, "unknown tile schedule %d", t->schedule);
    if (t->box < SLR_BOX_EXACT || t->box > SLR_BOX_VERTEX) return fail(SLR_E_INVALID, "unknown box mode %d", t->box);
    return SLR_OK;
}

slr_status check_surfels(const slr_surfels *s)
{
    if (!s) return fail(SLR_E_INVALID, "surfels is NULL");
    if (s->n < 0 || s->n > (int64_t(1) << 30))
        return fail(SLR_E_INVALID, "surfel count %lld out of range", (long long)s->n);
    if (s->n > 0 && (!s->means || !s->quats || !s->log_scales || !s->logits))
        return fail(SLR_E_INVALID, "surfel parameter pointer is NULL");
    if (!aligned(s->means, 4) || !aligned(s->quats, 16) || !aligned(s->log_scales, 8) || !aligned(s->logits, 4))
        return fail(SLR_E_INVALID, "surfel arrays misaligned (quats need 16 bytes, log_scales 8)");
    return SLR_OK;
}

// Host-made direction tables (column centres, row centres, rows -/+ margin),
// cached for the life of the process so that asynchronous uploads never
// outlive their source.
std::mutex g_tab_mu;
std::map<std::tuple<int, int, double, double, double, double>, std::unique_ptr<std::vector<double>>> g_tables;

const std::vector<double> &tables_for(const slr_sensor &s)
{
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto key = std::make_tuple(s.height, s.width, s.fu, s.cu, s.fv, s.cv);
    auto it = g_tables.find(key);
    if (it != g_tables.end()) return *it->second;
    const int H = s.height, W = s.width;
    auto t = std::make_unique<std::vector<double>>(2 * (size_t)(W + 3 * H));
    double *col = t->data(), *row = col + 2 * W, *rlo = row + 2 * H, *rhi = rlo + 2 * H;
    for (int j = 0; j < W; ++j) {
        const double az = (((double)j + 0.5) - s.cu) / s.fu;
        col[2 * j] = std::cos(az);
        col[2 * j + 1] = std::sin(az);
    }
    for (int i = 0; i < H; ++i) {
        const double el = (((double)i + 0.5) - s.cv) / s.fv;
        row[2 * i] = std::cos(el);
        row[2 * i + 1] = std::sin(el);
        rlo[2 * i] = std::cos(el - slr::kBoxMargin);
        rlo[2 * i + 1] = std::sin(el - slr::kBoxMargin);
        rhi[2 * i] = std::cos(el + slr::kBoxMargin);
        rhi[2 * i + 1] = std::sin(el + slr::kBoxMargin);
    }
    auto &ref = *t;
    g_tables.emplace(key, std::move(t));
    return ref;
}

// ---- stage timers (HIP events on the caller's stream) ----
struct StageEvent {
    int stage;
    hipEvent_t a, b;
};
std::mutex g_timer_mu;
bool g_timer_on = false;
std::vector<StageEvent> g_pending;
double g_stage_ms[SLR_NUM_STAGES];
int64_t g_stage_n[SLR_NUM_STAGES];

struct StageScope {
    hipEvent_t a = nullptr, b = nullptr;
    int stage;
    hipStream_t s;
    StageScope(int st, hipStream_t stream) : stage(st), s(stream)
    {
        if (!g_timer_on) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
        if (hipEventRecord(a, s) != hipSuccess) { (void)hipEventDestroy(a); (void)hipEventDestroy(b); a = b = nullptr; }
    }
    ~StageScope()
    {
        if (!a) return;
        if (hipEventRecord(b, s) != hipSuccess) { (void)hipEventDestroy(a); (void)hipEventDestroy(b); return; }
        std::lock_guard<std::mutex> lk(g_timer_mu);
        g_pending.push_back({stage, a, b});
    }
};

// ---- batch description on the host ----
struct Batch {
    std::vector<FrameGeom> geom;
    std::vector<int64_t> set_n;
    Layout L;
    int64_t max_n = 0;
};

slr_status check_batch(int32_t n_sets, const slr_surfels *sets, int32_t n_frames, const slr_frame *frames,
                       const slr_tiling *tiling, int64_t cap, Batch *b)
{
    slr_status st;
    if (n_sets < 0 || n_frames < 0 || n_frames > 32767) return fail(SLR_E_INVALID, "bad set or frame count");
    if ((n_sets > 0 && !sets) || (n_frames > 0 && !frames)) return fail(SLR_E_INVALID, "sets or frames is NULL");
    if ((st = check_tiling(tiling)) != SLR_OK) return st;
    if (cap < 0 || cap > 0x7fffffffLL) return fail(SLR_E_INVALID, "pair_capacity must be in [0, 2^31)");
    b->set_n.resize(n_sets);
    for (int32_t s = 0; s < n_sets; ++s) {
        if ((st = check_surfels(&sets[s])) != SLR_OK) return st;
        b->set_n[s] = sets[s].n;
    }
    b->geom.resize(n_frames);
    int64_t items = 0;
    for (int32_t f = 0; f < n_frames; ++f) {
        const slr_frame &fr = frames[f];
        if (fr.set < 0 || fr.set >= n_sets)
            return fail(SLR_E_INVALID, "frame %d: set index %d out of range", f, fr.set);
        if ((st = check_sensor(&fr.sensor)) != SLR_OK) return st;
        if (!fr.pose_cw || !aligned(fr.pose_cw, 8))
            return fail(SLR_E_INVALID, "frame %d: pose must be a non-NULL, 8-byte aligned device pointer", f);
        // the frame's own tile shape, or the batch's
        const int32_t th = (fr.tile_h || fr.tile_w) ? fr.tile_h : tiling->tile_h;
        const int32_t tw = (fr.tile_h || fr.tile_w) ? fr.tile_w : tiling->tile_w;
        if (!tile_shape_ok(th, tw)) return fail(SLR_E_INVALID, "frame %d: unsupported tile shape %dx%d", f, th, tw);
        const int64_t ftiles = (int64_t)((fr.sensor.height + th - 1) / th) * ((fr.sensor.width + tw - 1) / tw);
        if (ftiles > 65535) return fail(SLR_E_INVALID, "frame %d has %lld tiles, limit 65535", f, (long long)ftiles);
        b->geom[f] = FrameGeom{fr.sensor.height, fr.sensor.width, fr.set, th, tw};
        items += sets[fr.set].n;
        if (sets[fr.set].n > b->max_n) b->max_n = sets[fr.set].n;
    }
    if (items >= (int64_t(1) << 31)) return fail(SLR_E_INVALID, "batch has %lld records, limit 2^31", (long long)items);
    b->L = slr::make_layout(n_frames, b->geom.data(), n_sets, b->set_n.data(), cap, tiling->tile_h, tiling->tile_w,
                            tiling->bwd_variant == SLR_VARIANT_DETERMINISTIC);
    b->L.variant = tiling->variant == SLR_VARIANT_DEFAULT ? slr::kDefaultVariant : tiling->variant;
    // the backward form: as asked, else the forward's (the scalar-cache forward pairs with the workgroup backward)
    b->L.bwd_variant = tiling->bwd_variant != SLR_VARIANT_DEFAULT ? tiling->bwd_variant
                       : (b->L.variant == SLR_VARIANT_WAVE ? SLR_VARIANT_WAVE : SLR_VARIANT_LDS);
    b->L.bwd_batch = tiling->bwd_batch != 0 ? tiling->bwd_batch : 192;
    b->L.schedule = tiling->schedule == SLR_SCHEDULE_DEFAULT ? slr::kDefaultSchedule : tiling->schedule;
    b->L.box_mode = tiling->box;
    if (b->L.tiles >= (int64_t(1) << 24)) return fail(SLR_E_INVALID, "batch has too many tiles");
    return SLR_OK;
}

// Host descriptors of every frame (device pointers into the workspace).
std::vector<FrameDesc> make_descs(const Batch &B, const slr_surfels *sets, const slr_frame *frames,
                                  const slr_tiling *tiling, char *ws)
{
    const Layout &L = B.L;
    std::vector<int64_t> acc_off(B.set_n.size() + 1, 0);
    for (size_t s = 0; s < B.set_n.size(); ++s) acc_off[s + 1] = acc_off[s] + B.set_n[s] * slr::kAccStride;
    std::vector<FrameDesc> d(L.frames);
    int64_t item = 0, pix = 0, tab = 0, tile = 0;
    for (int32_t f = 0; f < L.frames; ++f) {
        const slr_frame &fr = frames[f];
        const slr_surfels &sf = sets[fr.set];
        FrameDesc &x = d[f];
        memset(&x, 0, sizeof(x));
        x.pose = fr.pose_cw;
        x.means = sf.means; x.quats = sf.quats; x.lsc = sf.log_scales; x.logits = sf.logits;
        x.depth = fr.depth; x.normal = fr.normal; x.alpha = fr.alpha;
        x.gD = fr.dL_ddepth; x.gN = fr.dL_dnormal; x.gO = fr.dL_dalpha;
        x.d_pose = fr.d_pose ? fr.d_pose : reinterpret_cast<double *>(ws + L.scratch_pose) + 6 * f;
        x.acc = reinterpret_cast<float *>(ws + L.acc) + acc_off[fr.set];
        x.n = sf.n;
        x.item_off = item;
        x.pix_off = pix;
        x.tab_off = tab;
        x.fu = fr.sensor.fu; x.cu = fr.sensor.cu; x.fv = fr.sensor.fv; x.cv = fr.sensor.cv;
        x.near_m = fr.sensor.near_m;
        x.H = fr.sensor.height; x.W = fr.sensor.width;
        x.th = B.geom[f].th; x.tw = B.geom[f].tw;
        x.tiles_x = (x.W + x.tw - 1) / x.tw;
        x.tiles_y = (x.H + x.th - 1) / x.th;
        x.tile_off = (int32_t)tile;
        x.set = fr.set;
        item += sf.n;
        pix += (int64_t)x.H * x.W;
        tab += x.W + 3 * x.H;
        tile += (int64_t)x.tiles_x * x.tiles_y;
    }
    return d;
}

slr_status upload_tables(const Batch &B, const slr_frame *frames, char *ws, hipStream_t s)
{
    int64_t tab = 0;
    for (int32_t f = 0; f < B.L.frames; ++f) {
        const std::vector<double> &t = tables_for(frames[f].sensor);
        HIP_TRY(hipMemcpyAsync(ws + B.L.tables + tab * 16, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice,
                               s));
        tab += frames[f].sensor.width + 3 * frames[f].sensor.height;
    }
    return SLR_OK;
}

slr_status check_ws(const Layout &L, void *ws, size_t bytes)
{
    if (!ws || !aligned(ws, 256)) return fail(SLR_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
    if (bytes < L.total) return fail(SLR_E_INVALID, "workspace has %zu bytes, needs %zu", bytes, L.total);
    return SLR_OK;
}

void enqueue_render_front(const Batch &B, char *ws, hipStream_t s)
{
    {
        StageScope t(0, s);
        slr::launch_project(B.L, ws, B.max_n, s);
    }
    {
        StageScope t(1, s);
        slr::launch_depth_sort(B.L, ws, s);
    }
    {
        StageScope t(2, s);
        slr::launch_scan_counts(B.L, ws, s);
    }
}

void enqueue_render_back(const Batch &B, char *ws, hipStream_t s)
{
    {
        StageScope t(3, s);
        slr::launch_emit_and_tile_sort(B.L, ws, s);
    }
    {
        StageScope t(4, s);
        slr::launch_raster_fwd(B.L, ws, s);
    }
}

void enqueue_backward(const Batch &B, const slr_surfels *sets, const slr_surfel_grads *grads, char *ws,
                      bool pose_only, bool accumulate, hipStream_t s)
{
    const Layout &L = B.L;
    // the fixed-order form writes every accumulator entry it uses in its gather
    const bool fixed = L.bwd_variant == SLR_VARIANT_DETERMINISTIC;
    if (!pose_only) {
        if (fixed) {
            slr::launch_fill_u32(ws + L.slot_bits, 0u, L.slot_words, s);
            slr::launch_record_rank(L, ws, s);
        } else {
            slr::launch_fill_u32(ws + L.acc, 0u, L.acc_floats, s);
        }
    }
    {
        StageScope t(5, s);
        slr::launch_raster_bwd(L, ws, pose_only, s);
    }
    slr::launch_pose_reduce(L, ws, s);
    if (pose_only) return;
    StageScope t(6, s);
    int64_t off = 0;
    for (int32_t k = 0; k < L.sets; ++k) {
        const slr_surfel_grads &g = grads[k];
        if (g.means && fixed)
            slr::launch_slot_gather(L, ws, k, sets[k].n, reinterpret_cast<float *>(ws + L.acc) + off, s);
        if (g.means)
            slr::launch_surfel_grad(sets[k].quats, sets[k].log_scales, sets[k].logits, sets[k].n,
                                    reinterpret_cast<const float *>(ws + L.acc) + off, g.means, g.quats, g.log_scales,
                                    g.logits, accumulate, s);
        off += sets[k].n * slr::kAccStride;
    }
}

slr_status check_grads(int32_t n_sets, const slr_surfel_grads *grads, bool pose_only)
{
    if (pose_only) {
        if (!grads) return SLR_OK;
        for (int32_t k = 0; k < n_sets; ++k)
            if (grads[k].means || grads[k].quats || grads[k].log_scales || grads[k].logits)
                return fail(SLR_E_INVALID, "SLR_POSE_ONLY takes NULL surfel gradients");
        return SLR_OK;
    }
    if (!grads) return fail(SLR_E_INVALID, "grads is NULL without SLR_POSE_ONLY");
    for (int32_t k = 0; k < n_sets; ++k) {
        const slr_surfel_grads &g = grads[k];
        const int nset = (g.means != nullptr) + (g.quats != nullptr) + (g.log_scales != nullptr) + (g.logits != nullptr);
        if (nset != 0 && nset != 4) return fail(SLR_E_INVALID, "set %d: surfel gradient pointers must all be set", k);
        if (nset == 4 && !aligned(g.quats, 16)) return fail(SLR_E_INVALID, "set %d: d_quats must be 16-byte aligned", k);
    }
    return SLR_OK;
}

}  // namespace

namespace slr {

Layout make_layout(int32_t nframes, const FrameGeom *frames, int32_t nsets, const int64_t *set_n, int64_t cap,
                   int32_t th, int32_t tw, bool fixed_order)
{
    Layout L{};
    L.frames = nframes; L.sets = nsets; L.th = th; L.tw = tw; L.cap = cap;
    for (int32_t f = 0; f < nframes; ++f) {
        const int64_t tx = (frames[f].W + frames[f].tw - 1) / frames[f].tw, ty = (frames[f].H + frames[f].th - 1) / frames[f].th;
        L.tiles += tx * ty;
        L.pixels += (int64_t)frames[f].H * frames[f].W;
        L.tab_entries += frames[f].W + 3 * frames[f].H;
        L.items += set_n[frames[f].set];
    }
    for (int32_t s = 0; s < nsets; ++s) L.acc_floats += set_n[s] * kAccStride;
    L.tile_bits = ceil_log2(L.tiles > 0 ? L.tiles : 1);
    L.depth_passes = 4;
    L.tile_passes = (L.tile_bits + kMaxDigitBits - 1) / kMaxDigitBits;
    L.depth_in_1 = (L.depth_passes % 2) == 1;
    L.tile_in_1 = (L.tile_passes % 2) == 1;
    const int64_t nn = L.items > 0 ? L.items : 1, cc = cap > 0 ? cap : 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + (bytes ? bytes : 1), 256); return at; };
    L.desc = take(sizeof(FrameDesc) * (size_t)(nframes > 0 ? nframes : 1));
    L.tables = take(16 * (size_t)L.tab_entries);
    L.tile_frame = take(4 * (size_t)L.tiles);
    L.rec = take(sizeof(RasterRec) * nn);
    L.box = take(sizeof(PixBox) * nn);
    L.skey = take(4 * nn);
    L.key0 = take(4 * nn); L.val0 = take(4 * nn); L.key1 = take(4 * nn); L.val1 = take(4 * nn);
    L.cnt = take(4 * nn);
    L.off = take(4 * nn);
    // per emit block: the record holding its first pair slot
    L.estart = take(4 * (size_t)(cc / kEmitSlots + 2));
    const int64_t tn = kSortThreads * sort_items(nn), tk = kSortThreads * sort_items(cc);
    const int64_t nb_n = (nn + tn - 1) / tn, nb_k = (cc + tk - 1) / tk;
    L.blocksum = take(4 * nb_n);
    L.pt0 = take(4 * cc); L.pv0 = take(4 * cc); L.pt1 = take(4 * cc); L.pv1 = take(4 * cc);
    // tile counts and boxes of the records in range order (written by the range sort's last pass)
    L.rcnt = take(4 * nn);
    L.rbox = take(sizeof(PixBox) * nn);
    // per compositing workgroup: its pose partial (6 doubles) and keyframe index
    // (the one-wave backward's grid adds 16 quad-mode workgroups per quad tile)
    L.pose_part = take(sizeof(double) * 8 *
                       (size_t)((wave_blocks(L.tiles) > L.tiles ? wave_blocks(L.tiles) : L.tiles) + 16 * quad_tile_cap(L.tiles)));
    // per Gauss-Newton workgroup (one per tile) or strip wave (four per tile): its partial normal equations
    // four strip rows per tile, sixteen for the tiles composited in quad mode
    L.gn_part = take(sizeof(double) * kGnRow * (4 * (size_t)L.tiles + 12 * (size_t)quad_tile_cap(L.tiles)));
    L.ranges = take(8 * (size_t)L.tiles);
    L.order = take(4 * (size_t)L.tiles);
    L.hist = take(4 * 256 * (size_t)(nb_n > nb_k ? nb_n : nb_k));
    L.stateT = take(4 * (size_t)L.pixels);
    L.stateN = take(4 * (size_t)L.pixels);
    L.census = take(16 * (size_t)L.pixels);
    // one bit per (strip, list entry): four strips' 64-entry chunk words per chunk of the
    // pair list, plus one spare chunk per tile (a tile's words start at its first chunk)
    L.cmask_words = 4 * (L.cap / 64 + L.tiles + 2);
    L.cmask = take(8 * (size_t)L.cmask_words);
    L.acc = take(4 * (size_t)L.acc_floats);
    if (fixed_order) {
        L.rank = take(4 * (size_t)nn);
        L.slots = take(4 * (size_t)kSlotFloats * (size_t)cc);
        L.slot_words = (cc + 31) / 32;
        L.slot_bits = take(4 * (size_t)L.slot_words);
    }
    L.scratch_pose = take(48 * (size_t)(nframes > 0 ? nframes : 1));
    L.misc = take(4096);
    L.total = o;
    return L;
}

}  // namespace slr

extern "C" {

const char *slr_status_string(slr_status st)
{
    switch (st) {
    case SLR_OK: return "ok";
    case SLR_E_INVALID: return "invalid argument";
    case SLR_E_CAPACITY: return "pair capacity exceeded";
    case SLR_E_HIP: return "HIP runtime error";
    case SLR_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *slr_last_error(void) { return g_last_error.c_str(); }

slr_status slr_camera_matrix(double az_min, double az_max, double el_min, double el_max, int32_t height,
                             int32_t width, double *out)
{
    if (!out) return fail(SLR_E_INVALID, "out is NULL");
    if (height <= 0 || width <= 0) return fail(SLR_E_INVALID, "image size must be positive");
    const double fh = az_max - az_min, fv = el_max - el_min;
    if (!(fh > 0.0) || !(fv > 0.0)) return fail(SLR_E_INVALID, "field of view must be positive");
    out[0] = -((double)width - 1.0) / fh;
    out[1] = (double)width / 2.0 * (1.0 + (az_max + az_min) / fh);
    out[2] = -((double)height - 1.0) / fv;
    out[3] = (double)height / 2.0 * (1.0 + (el_max + el_min) / fv);
    return SLR_OK;
}

// ---------------------------------------------------------------- plain form
static slr_status plain_batch(const slr_surfels *surfels, const double *pose_cw, const slr_sensor *sensor,
                              const slr_tiling *tiling, int64_t cap, slr_frame *frame, Batch *B)
{
    slr_status st;
    if ((st = check_surfels(surfels)) != SLR_OK) return st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    memset(frame, 0, sizeof(*frame));
    frame->set = 0;
    frame->pose_cw = pose_cw;
    frame->sensor = *sensor;
    return check_batch(1, surfels, 1, frame, tiling, cap, B);
}

slr_status slr_workspace_size(const slr_sensor *sensor, const slr_tiling *tiling, int64_t n, int64_t pair_capacity,
                              size_t *bytes)
{
    slr_status st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if ((st = check_tiling(tiling)) != SLR_OK) return st;
    if (!bytes) return fail(SLR_E_INVALID, "bytes is NULL");
    if (n < 0 || pair_capacity < 0 || pair_capacity > 0x7fffffffLL || n > (int64_t(1) << 30))
        return fail(SLR_E_INVALID, "n and pair_capacity out of range");
    FrameGeom g{sensor->height, sensor->width, 0, tiling->tile_h, tiling->tile_w};
    *bytes = slr::make_layout(1, &g, 1, &n, pair_capacity, tiling->tile_h, tiling->tile_w,
                              tiling->bwd_variant == SLR_VARIANT_DETERMINISTIC).total;
    return SLR_OK;
}

slr_status slr_render(const slr_surfels *surfels, const double *pose_cw, const slr_sensor *sensor,
                      const slr_tiling *tiling, void *workspace, size_t workspace_bytes, int64_t pair_capacity,
                      float *depth, float *normal, float *alpha, int64_t *pairs_out, void *stream)
{
    slr_frame fr;
    Batch B;
    slr_status st = plain_batch(surfels, pose_cw, sensor, tiling, pair_capacity, &fr, &B);
    if (st != SLR_OK) return st;
    if ((st = check_ws(B.L, workspace, workspace_bytes)) != SLR_OK) return st;
    if (!depth || !normal || !alpha) return fail(SLR_E_INVALID, "output pointer is NULL");
    fr.depth = depth; fr.normal = normal; fr.alpha = alpha;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    if ((st = upload_tables(B, &fr, ws, s)) != SLR_OK) return st;
    std::vector<FrameDesc> d = make_descs(B, surfels, &fr, tiling, ws);
    slr::launch_write_desc(d.data(), 1, reinterpret_cast<FrameDesc *>(ws + B.L.desc), s);
    slr::launch_tile_frame(B.L, ws, s);
    enqueue_render_front(B, ws, s);
    uint64_t K = 0;
    HIP_TRY(hipMemcpyAsync(&K, ws + B.L.misc, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipGetLastError());
    if (pairs_out) *pairs_out = (int64_t)K;
    if ((int64_t)K > pair_capacity)
        return fail(SLR_E_CAPACITY, "%llu (tile, surfel) pairs exceed the capacity %lld", (unsigned long long)K,
                    (long long)pair_capacity);
    enqueue_render_back(B, ws, s);
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_backward(const slr_surfels *surfels, const double *pose_cw, const slr_sensor *sensor,
                        const slr_tiling *tiling, void *workspace, size_t workspace_bytes, int64_t pair_capacity,
                        const float *dL_ddepth, const float *dL_dnormal, const float *dL_dalpha, float *d_means,
                        float *d_quats, float *d_log_scales, float *d_logits, double *d_pose, uint32_t flags,
                        void *stream)
{
    slr_frame fr;
    Batch B;
    slr_status st = plain_batch(surfels, pose_cw, sensor, tiling, pair_capacity, &fr, &B);
    if (st != SLR_OK) return st;
    if ((st = check_ws(B.L, workspace, workspace_bytes)) != SLR_OK) return st;
    const bool pose_only = (flags & SLR_POSE_ONLY) != 0;
    const bool accumulate = (flags & SLR_ACCUMULATE) != 0;
    const int nset = (d_means != nullptr) + (d_quats != nullptr) + (d_log_scales != nullptr) + (d_logits != nullptr);
    if (pose_only && nset != 0) return fail(SLR_E_INVALID, "SLR_POSE_ONLY takes NULL surfel gradients");
    // an empty set may pass NULL gradient arrays (there is nothing to write)
    if (!pose_only && nset != 4 && !(surfels->n == 0 && nset == 0))
        return fail(SLR_E_INVALID, "surfel gradient pointers must all be set");
    if (!pose_only && !aligned(d_quats, 16)) return fail(SLR_E_INVALID, "d_quats must be 16-byte aligned");
    if (pose_only && !d_pose) return fail(SLR_E_INVALID, "SLR_POSE_ONLY needs d_pose");
    if (flags & ~(SLR_POSE_ONLY | SLR_ACCUMULATE)) return fail(SLR_E_INVALID, "unknown flags 0x%x", flags);
    fr.dL_ddepth = dL_ddepth; fr.dL_dnormal = dL_dnormal; fr.dL_dalpha = dL_dalpha;
    fr.d_pose = d_pose;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    // rewrite the descriptor with the backward's pointers (outputs are not read)
    std::vector<FrameDesc> d = make_descs(B, surfels, &fr, tiling, ws);
    slr::launch_write_desc(d.data(), 1, reinterpret_cast<FrameDesc *>(ws + B.L.desc), s);
    slr_surfel_grads g{d_means, d_quats, d_log_scales, d_logits};
    enqueue_backward(B, surfels, &g, ws, pose_only, accumulate, s);
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_pose_gn(const slr_surfels *surfels, const double *pose_cw, const slr_sensor *sensor,
                       const slr_tiling *tiling, void *workspace, size_t workspace_bytes, int64_t pair_capacity,
                       const float *depth, const float *target, const float *weight, double huber_k,
                       double *normal_eq, void *stream)
{
    slr_frame fr;
    Batch B;
    slr_status st = plain_batch(surfels, pose_cw, sensor, tiling, pair_capacity, &fr, &B);
    if (st != SLR_OK) return st;
    if ((st = check_ws(B.L, workspace, workspace_bytes)) != SLR_OK) return st;
    if (!depth || !target || !normal_eq) return fail(SLR_E_INVALID, "depth, target and normal_eq must be set");
    if (std::isnan(huber_k)) return fail(SLR_E_INVALID, "huber_k is NaN");
    fr.depth = const_cast<float *>(depth);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    std::vector<FrameDesc> d = make_descs(B, surfels, &fr, tiling, ws);
    d[0].gn_target = target;
    d[0].gn_weight = weight;
    d[0].gn = normal_eq;
    d[0].huber_k = huber_k;
    slr::launch_write_desc(d.data(), 1, reinterpret_cast<FrameDesc *>(ws + B.L.desc), s);
    {
        StageScope t(8, s);
        slr::launch_raster_gn(B.L, ws, s);
    }
    slr::launch_gn_reduce(B.L, ws, s);
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_photo_workspace_size(const slr_sensor *sensor, size_t *bytes)
{
    slr_status st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if (!bytes) return fail(SLR_E_INVALID, "bytes is NULL");
    *bytes = slr::photo_workspace_bytes(sensor->height, sensor->width);
    return SLR_OK;
}

slr_status slr_photo_gn(const slr_sensor *sensor, const float *depth, const float *query, const float *weight,
                        const double *pose_qm, double huber_k, void *workspace, size_t workspace_bytes,
                        double *normal_eq, void *stream)
{
    slr_status st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if (!depth || !query || !pose_qm || !normal_eq)
        return fail(SLR_E_INVALID, "depth, query, pose_qm and normal_eq must be set");
    if (std::isnan(huber_k)) return fail(SLR_E_INVALID, "huber_k is NaN");
    const size_t need = slr::photo_workspace_bytes(sensor->height, sensor->width);
    if (!workspace || !aligned(workspace, 256)) return fail(SLR_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
    if (workspace_bytes < need) return fail(SLR_E_INVALID, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    {
        StageScope t(9, s);
        slr::launch_photo_gn(sensor->height, sensor->width, sensor->fu, sensor->cu, sensor->fv, sensor->cv, huber_k,
                             depth, query, weight, pose_qm, reinterpret_cast<double *>(workspace), normal_eq, s);
    }
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_photo_gn_noalloc(const slr_sensor *sensor, const float *depth, const float *query,
                                const float *weight, const double *pose_qm, double huber_k, double *normal_eq,
                                void *stream)
{
    slr_status st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if (!depth || !query || !pose_qm || !normal_eq)
        return fail(SLR_E_INVALID, "depth, query, pose_qm and normal_eq must be set");
    if (std::isnan(huber_k)) return fail(SLR_E_INVALID, "huber_k is NaN");
    const int64_t npix = (int64_t)sensor->height * sensor->width;
    if (npix > slr::photo_static_max_pixels())
        return fail(SLR_E_INVALID, "image of %lld pixels exceeds the %lld pixels of the static scratch; use "
                                   "slr_photo_gn with a workspace", (long long)npix,
                    (long long)slr::photo_static_max_pixels());
    double *part = nullptr;
    HIP_TRY(slr::photo_static_scratch(&part));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    {
        StageScope t(9, s);
        slr::launch_photo_gn(sensor->height, sensor->width, sensor->fu, sensor->cu, sensor->fv, sensor->cv, huber_k,
                             depth, query, weight, pose_qm, part, normal_eq, s);
    }
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_cloud_to_range(const slr_sensor *sensor, int64_t n, const float *points, float *range, void *stream)
{
    slr_status st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if (n < 0) return fail(SLR_E_INVALID, "negative point count");
    if ((n > 0 && !points) || !range) return fail(SLR_E_INVALID, "points and range must be set");
    slr::launch_cloud_to_range(sensor->height, sensor->width, sensor->fu, sensor->cu, sensor->fv, sensor->cv, n,
                               points, range, reinterpret_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_range_normals(const slr_sensor *sensor, const float *range, float *normals, void *stream)
{
    slr_status st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if (!range || !normals) return fail(SLR_E_INVALID, "range and normals must be set");
    slr::launch_range_normals(sensor->height, sensor->width, sensor->fu, sensor->cu, sensor->fv, sensor->cv, range,
                              normals, reinterpret_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_loss_map(int64_t pixels, const float *depth, const float *normal, const float *alpha,
                        const float *target_depth, const float *target_normal, float w_d, float w_n, float w_o,
                        float *dL_ddepth, float *dL_dnormal, float *dL_dalpha, double *loss, void *stream)
{
    if (pixels < 0) return fail(SLR_E_INVALID, "negative pixel count");
    if (pixels > 0 && (!depth || !normal || !alpha || !target_depth || !target_normal || !dL_ddepth || !dL_dnormal ||
                       !dL_dalpha))
        return fail(SLR_E_INVALID, "loss buffer is NULL");
    if (!std::isfinite(w_d) || !std::isfinite(w_n) || !std::isfinite(w_o))
        return fail(SLR_E_INVALID, "loss weights must be finite");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    {
        StageScope t(7, s);
        slr::launch_loss_map(pixels, depth, normal, alpha, target_depth, target_normal, w_d, w_n, w_o, dL_ddepth,
                             dL_dnormal, dL_dalpha, loss, s);
    }
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_scale_reg(int64_t n, const float *log_scales, double tau_s, double w_s, float *d_log_scales,
                         double *loss, void *stream)
{
    if (n < 0) return fail(SLR_E_INVALID, "negative surfel count");
    if (n > 0 && (!log_scales || !d_log_scales)) return fail(SLR_E_INVALID, "log_scales and d_log_scales must be set");
    if (!std::isfinite(tau_s) || !std::isfinite(w_s)) return fail(SLR_E_INVALID, "tau_s and w_s must be finite");
    slr::launch_scale_reg(n, log_scales, tau_s, w_s, d_log_scales, loss, reinterpret_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_init_workspace_size(const slr_sensor *sensor, size_t *bytes)
{
    slr_status st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if (!bytes) return fail(SLR_E_INVALID, "bytes is NULL");
    *bytes = slr::init_workspace_bytes(sensor->height, sensor->width);
    return SLR_OK;
}

slr_status slr_init_splats(const slr_sensor *sensor, const float *range, const float *mask, const double *pose_cw,
                           int64_t n, const double *uniforms, double scale_factor, float logit, void *workspace,
                           size_t workspace_bytes, float *means, float *quats, float *log_scales, float *logits,
                           int32_t *pixel, void *stream)
{
    slr_status st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if (n < 0) return fail(SLR_E_INVALID, "negative draw count");
    if (!range || !pose_cw) return fail(SLR_E_INVALID, "range and pose_cw must be set");
    if (n > 0 && (!uniforms || !means || !quats || !log_scales || !logits || !pixel))
        return fail(SLR_E_INVALID, "uniforms and every output must be set");
    if (!(scale_factor > 0.0) || !std::isfinite(scale_factor)) return fail(SLR_E_INVALID, "scale_factor must be > 0");
    if (!std::isfinite(logit)) return fail(SLR_E_INVALID, "logit must be finite");
    const size_t need = slr::init_workspace_bytes(sensor->height, sensor->width);
    if (!workspace || !aligned(workspace, 256)) return fail(SLR_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
    if (workspace_bytes < need) return fail(SLR_E_INVALID, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
    slr::launch_init_splats(sensor->height, sensor->width, sensor->fu, sensor->cu, sensor->fv, sensor->cv, range, mask,
                            pose_cw, n, uniforms, scale_factor, logit, reinterpret_cast<char *>(workspace), means, quats,
                            log_scales, logits, pixel, reinterpret_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

// ---------------------------------------------------------------- batched form
slr_status slr_batch_workspace_size(int32_t n_sets, const slr_surfels *sets, int32_t n_frames,
                                    const slr_frame *frames, const slr_tiling *tiling, int64_t pair_capacity,
                                    size_t *bytes)
{
    if (!bytes) return fail(SLR_E_INVALID, "bytes is NULL");
    Batch B;
    slr_status st = check_batch(n_sets, sets, n_frames, frames, tiling, pair_capacity, &B);
    if (st != SLR_OK) return st;
    *bytes = B.L.total;
    return SLR_OK;
}

slr_status slr_batch_prepare(int32_t n_sets, const slr_surfels *sets, int32_t n_frames, const slr_frame *frames,
                             const slr_tiling *tiling, int64_t pair_capacity, void *workspace, size_t workspace_bytes,
                             void *stream)
{
    Batch B;
    slr_status st = check_batch(n_sets, sets, n_frames, frames, tiling, pair_capacity, &B);
    if (st != SLR_OK) return st;
    if ((st = check_ws(B.L, workspace, workspace_bytes)) != SLR_OK) return st;
    for (int32_t f = 0; f < n_frames; ++f)
        if (!frames[f].depth || !frames[f].normal || !frames[f].alpha)
            return fail(SLR_E_INVALID, "frame %d: output pointer is NULL", f);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    if ((st = upload_tables(B, frames, ws, s)) != SLR_OK) return st;
    std::vector<FrameDesc> d = make_descs(B, sets, frames, tiling, ws);
    slr::launch_write_desc(d.data(), n_frames, reinterpret_cast<FrameDesc *>(ws + B.L.desc), s);
    slr::launch_tile_frame(B.L, ws, s);
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_batch_render(int32_t n_sets, const slr_surfels *sets, int32_t n_frames, const slr_frame *frames,
                            const slr_tiling *tiling, int64_t pair_capacity, void *workspace, size_t workspace_bytes,
                            void *stream)
{
    Batch B;
    slr_status st = check_batch(n_sets, sets, n_frames, frames, tiling, pair_capacity, &B);
    if (st != SLR_OK) return st;
    if ((st = check_ws(B.L, workspace, workspace_bytes)) != SLR_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    enqueue_render_front(B, ws, s);
    enqueue_render_back(B, ws, s);
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_batch_backward(int32_t n_sets, const slr_surfels *sets, const slr_surfel_grads *grads, int32_t n_frames,
                              const slr_frame *frames, const slr_tiling *tiling, int64_t pair_capacity,
                              void *workspace, size_t workspace_bytes, uint32_t flags, void *stream)
{
    Batch B;
    slr_status st = check_batch(n_sets, sets, n_frames, frames, tiling, pair_capacity, &B);
    if (st != SLR_OK) return st;
    if ((st = check_ws(B.L, workspace, workspace_bytes)) != SLR_OK) return st;
    if (flags & ~(SLR_POSE_ONLY | SLR_ACCUMULATE)) return fail(SLR_E_INVALID, "unknown flags 0x%x", flags);
    const bool pose_only = (flags & SLR_POSE_ONLY) != 0;
    if ((st = check_grads(n_sets, grads, pose_only)) != SLR_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    enqueue_backward(B, sets, grads, ws, pose_only, (flags & SLR_ACCUMULATE) != 0, s);
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_batch_autotune(int32_t n_sets, const slr_surfels *sets, const slr_surfel_grads *grads,
                              int32_t n_frames, const slr_frame *frames, const slr_tiling *candidates,
                              int32_t n_candidates, int64_t pair_capacity, void *workspace, size_t workspace_bytes,
                              int32_t reps, double *ms, int32_t *best, void *stream)
{
    if (!candidates || n_candidates < 1) return fail(SLR_E_INVALID, "no candidate tilings");
    if (!ms || !best) return fail(SLR_E_INVALID, "ms and best must be host pointers");
    if (reps < 1) return fail(SLR_E_INVALID, "reps must be >= 1");
    // validate every candidate first: nothing is launched for an invalid set
    std::vector<Batch> bs(n_candidates);
    for (int32_t c = 0; c < n_candidates; ++c) {
        slr_status st = check_batch(n_sets, sets, n_frames, frames, &candidates[c], pair_capacity, &bs[c]);
        if (st != SLR_OK) return st;
        if ((st = check_ws(bs[c].L, workspace, workspace_bytes)) != SLR_OK) return st;
        if ((st = check_grads(n_sets, grads, false)) != SLR_OK) return st;
        for (int32_t f = 0; f < n_frames; ++f)
            if (!frames[f].depth || !frames[f].normal || !frames[f].alpha)
                return fail(SLR_E_INVALID, "frame %d: output pointer is NULL", f);
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SLR_E_HIP, "hipEventCreate failed");
    }
    slr_status res = SLR_OK;
    double best_ms = 0.0;
    *best = -1;
    for (int32_t c = 0; c < n_candidates && res == SLR_OK; ++c) {
        const Batch &B = bs[c];
        if ((res = upload_tables(B, frames, ws, s)) != SLR_OK) break;
        std::vector<FrameDesc> d = make_descs(B, sets, frames, &candidates[c], ws);
        slr::launch_write_desc(d.data(), n_frames, reinterpret_cast<FrameDesc *>(ws + B.L.desc), s);
        slr::launch_tile_frame(B.L, ws, s);
        // one untimed step, then the median of reps timed steps (render + backward)
        std::vector<float> t;
        for (int32_t r = -1; r < reps; ++r) {
            if (r >= 0 && hipEventRecord(e0, s) != hipSuccess) { res = fail(SLR_E_HIP, "hipEventRecord failed"); break; }
            enqueue_render_front(B, ws, s);
            enqueue_render_back(B, ws, s);
            enqueue_backward(B, sets, grads, ws, false, false, s);
            if (r < 0) continue;
            float x = 0.0f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&x, e0, e1) != hipSuccess) {
                res = fail(SLR_E_HIP, "timing failed");
                break;
            }
            t.push_back(x);
        }
        if (res != SLR_OK) break;
        // a candidate whose pairs overflowed the capacity did not render: not eligible
        uint64_t over = 0;
        if (hipMemcpy(&over, ws + B.L.misc + 8, sizeof(over), hipMemcpyDeviceToHost) != hipSuccess) {
            res = fail(SLR_E_HIP, "hipMemcpy failed");
            break;
        }
        std::sort(t.begin(), t.end());
        ms[c] = over ? -1.0 : (double)t[t.size() / 2];
        if (!over && (*best < 0 || ms[c] < best_ms)) { *best = c; best_ms = ms[c]; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (res != SLR_OK) return res;
    if (*best < 0) return fail(SLR_E_CAPACITY, "every candidate overflowed the pair capacity");
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_batch_counters(int32_t n_sets, const slr_surfels *sets, int32_t n_frames, const slr_frame *frames,
                              const slr_tiling *tiling, int64_t pair_capacity, void *workspace, size_t workspace_bytes,
                              const uint64_t **counters)
{
    if (!counters) return fail(SLR_E_INVALID, "counters is NULL");
    Batch B;
    slr_status st = check_batch(n_sets, sets, n_frames, frames, tiling, pair_capacity, &B);
    if (st != SLR_OK) return st;
    if ((st = check_ws(B.L, workspace, workspace_bytes)) != SLR_OK) return st;
    *counters = reinterpret_cast<const uint64_t *>(reinterpret_cast<char *>(workspace) + B.L.misc);
    return SLR_OK;
}

// ---------------------------------------------------------------- support
slr_status slr_loss_l1_normal(int64_t pixels, const float *depth, const float *normal, const float *target_depth,
                              const float *target_normal, float w_d, float w_n, float *dL_ddepth, float *dL_dnormal,
                              double *loss, void *stream)
{
    if (pixels < 0) return fail(SLR_E_INVALID, "negative pixel count");
    if (pixels > 0 && (!depth || !normal || !target_depth || !target_normal || !dL_ddepth || !dL_dnormal))
        return fail(SLR_E_INVALID, "loss buffer is NULL");
    if (!std::isfinite(w_d) || !std::isfinite(w_n)) return fail(SLR_E_INVALID, "loss weights must be finite");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    {
        StageScope t(7, s);
        slr::launch_loss_l1_normal(pixels, depth, normal, target_depth, target_normal, w_d, w_n, dL_ddepth,
                                   dL_dnormal, loss, s);
    }
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_loss_l1_normal_frames(int32_t n_frames, const slr_loss_frame *frames, double *loss, void *stream)
{
    if (n_frames < 0) return fail(SLR_E_INVALID, "negative frame count");
    if (n_frames > 0 && !frames) return fail(SLR_E_INVALID, "frames is NULL");
    for (int32_t f = 0; f < n_frames; ++f) {
        const slr_loss_frame &x = frames[f];
        if (x.pixels < 0) return fail(SLR_E_INVALID, "frame %d: negative pixel count", f);
        if (x.pixels > 0 && (!x.depth || !x.normal || !x.target_depth || !x.target_normal || !x.dL_ddepth ||
                             !x.dL_dnormal))
            return fail(SLR_E_INVALID, "frame %d: loss buffer is NULL", f);
        if (!std::isfinite(x.w_d) || !std::isfinite(x.w_n))
            return fail(SLR_E_INVALID, "frame %d: loss weights must be finite", f);
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    {
        StageScope t(7, s);
        slr::launch_loss_frames(n_frames, frames, loss, s);
    }
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_adam_step(int64_t n, float *means, float *quats, float *log_scales, float *logits,
                         const slr_surfel_grads *grads, float *m, float *v, const slr_adam_config *cfg, void *stream)
{
    if (n < 0) return fail(SLR_E_INVALID, "negative surfel count");
    if (!cfg || !grads) return fail(SLR_E_INVALID, "config or gradients are NULL");
    if (cfg->step < 1) return fail(SLR_E_INVALID, "Adam step must be >= 1");
    const double hp[7] = {cfg->lr_means, cfg->lr_quats, cfg->lr_log_scales, cfg->lr_logits, cfg->beta1, cfg->beta2, cfg->eps};
    for (double x : hp)
        if (!std::isfinite(x) || x < 0.0) return fail(SLR_E_INVALID, "Adam hyper-parameters must be finite and >= 0");
    if (cfg->beta1 >= 1.0 || cfg->beta2 >= 1.0) return fail(SLR_E_INVALID, "Adam betas must be < 1");
    if (n > 0) {
        if (!means || !quats || !log_scales || !logits || !m || !v || !grads->means || !grads->quats ||
            !grads->log_scales || !grads->logits)
            return fail(SLR_E_INVALID, "Adam array is NULL");
        if (!aligned(quats, 16) || !aligned(grads->quats, 16))
            return fail(SLR_E_INVALID, "quaternion arrays must be 16-byte aligned");
    }
    const double bc1 = 1.0 - std::pow(cfg->beta1, cfg->step);
    const double bc2 = 1.0 - std::pow(cfg->beta2, cfg->step);
    const float s[4] = {(float)(cfg->lr_means / bc1), (float)(cfg->lr_quats / bc1), (float)(cfg->lr_log_scales / bc1),
                        (float)(cfg->lr_logits / bc1)};
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    slr::launch_adam(n, means, quats, log_scales, logits, grads->means, grads->quats, grads->log_scales, grads->logits,
                     m, v, s, (float)(1.0 - cfg->beta1), (float)cfg->beta2, (float)(1.0 - cfg->beta2),
                     (float)std::sqrt(bc2), (float)cfg->eps, st);
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_stage_timer_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_timer_mu);
    g_timer_on = on != 0;
    return SLR_OK;
}

slr_status slr_stage_times(double *ms, int64_t *counts)
{
    if (!ms || !counts) return fail(SLR_E_INVALID, "ms and counts must be non-NULL");
    std::vector<StageEvent> ev;
    {
        std::lock_guard<std::mutex> lk(g_timer_mu);
        ev.swap(g_pending);
    }
    slr_status st = SLR_OK;
    for (auto &e : ev) {
        float t = 0.f;
        if (hipEventSynchronize(e.b) != hipSuccess || hipEventElapsedTime(&t, e.a, e.b) != hipSuccess) st = SLR_E_HIP;
        g_stage_ms[e.stage] += t;
        g_stage_n[e.stage] += 1;
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (int k = 0; k < SLR_NUM_STAGES; ++k) {
        ms[k] = g_stage_ms[k];
        counts[k] = g_stage_n[k];
        g_stage_ms[k] = 0.0;
        g_stage_n[k] = 0;
    }
    if (st != SLR_OK) return fail(st, "stage event query failed");
    return SLR_OK;
}

slr_status slr_workspace_views(const slr_sensor *sensor, const slr_tiling *tiling, int64_t n, int64_t pair_capacity,
                               void *workspace, size_t workspace_bytes, slr_views *v)
{
    slr_status st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if ((st = check_tiling(tiling)) != SLR_OK) return st;
    if (!workspace || !v) return fail(SLR_E_INVALID, "workspace and views must be non-NULL");
    if (n < 0 || pair_capacity < 0) return fail(SLR_E_INVALID, "negative size");
    FrameGeom g{sensor->height, sensor->width, 0, tiling->tile_h, tiling->tile_w};
    Layout L = slr::make_layout(1, &g, 1, &n, pair_capacity, tiling->tile_h, tiling->tile_w,
                                tiling->bwd_variant == SLR_VARIANT_DETERMINISTIC);
    if (workspace_bytes < L.total) return fail(SLR_E_INVALID, "workspace too small");
    char *ws = reinterpret_cast<char *>(workspace);
    v->keys = reinterpret_cast<const uint32_t *>(ws + L.skey);
    v->counts = reinterpret_cast<const int32_t *>(ws + L.cnt);
    v->pixbox = reinterpret_cast<const int16_t *>(ws + L.box);
    v->sorted_tile = reinterpret_cast<const int32_t *>(ws + (L.tile_in_1 ? L.pt1 : L.pt0));
    v->sorted_id = reinterpret_cast<const int32_t *>(ws + (L.tile_in_1 ? L.pv1 : L.pv0));
    v->ranges = reinterpret_cast<const int32_t *>(ws + L.ranges);
    v->T_final = reinterpret_cast<const float *>(ws + L.stateT);
    v->n_proc = reinterpret_cast<const int32_t *>(ws + L.stateN);
    v->census = reinterpret_cast<const int32_t *>(ws + L.census);
    v->tiles_x = (sensor->width + tiling->tile_w - 1) / tiling->tile_w;
    v->tiles_y = (sensor->height + tiling->tile_h - 1) / tiling->tile_h;
    return SLR_OK;
}

slr_status slr_batch_views(int32_t n_sets, const slr_surfels *sets, int32_t n_frames, const slr_frame *frames,
                           const slr_tiling *tiling, int64_t pair_capacity, void *workspace, size_t workspace_bytes,
                           slr_views *v)
{
    if (!v) return fail(SLR_E_INVALID, "views is NULL");
    Batch B;
    slr_status st = check_batch(n_sets, sets, n_frames, frames, tiling, pair_capacity, &B);
    if (st != SLR_OK) return st;
    if ((st = check_ws(B.L, workspace, workspace_bytes)) != SLR_OK) return st;
    const Layout &L = B.L;
    char *ws = reinterpret_cast<char *>(workspace);
    v->keys = reinterpret_cast<const uint32_t *>(ws + L.skey);
    v->counts = reinterpret_cast<const int32_t *>(ws + L.cnt);
    v->pixbox = reinterpret_cast<const int16_t *>(ws + L.box);
    v->sorted_tile = reinterpret_cast<const int32_t *>(ws + (L.tile_in_1 ? L.pt1 : L.pt0));
    v->sorted_id = reinterpret_cast<const int32_t *>(ws + (L.tile_in_1 ? L.pv1 : L.pv0));
    v->ranges = reinterpret_cast<const int32_t *>(ws + L.ranges);
    v->T_final = reinterpret_cast<const float *>(ws + L.stateT);
    v->n_proc = reinterpret_cast<const int32_t *>(ws + L.stateN);
    v->census = reinterpret_cast<const int32_t *>(ws + L.census);
    v->tiles_x = L.tiles;
    v->tiles_y = 1;
    return SLR_OK;
}

}  // extern "C"

// capi.cpp -- C ABI of the spherical surfel rasterizer: argument validation,
// workspace layout, host-made sensor tables and launch orchestration.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "slr_internal.h"

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

// Angular margin (radians) by which the bounding box is widened on every side.
constexpr double kBoxMargin = 2e-5;

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

slr_status check_tiling(const slr_tiling *t)
{
    if (!t) return fail(SLR_E_INVALID, "tiling is NULL");
    const bool ok = (t->tile_h == 16 && t->tile_w == 16) || (t->tile_h == 8 && t->tile_w == 32) ||
                    (t->tile_h == 32 && t->tile_w == 8) || (t->tile_h == 4 && t->tile_w == 64);
    if (!ok) return fail(SLR_E_INVALID, "unsupported tile shape %dx%d", t->tile_h, t->tile_w);
    return SLR_OK;
}

slr_status check_surfels(const slr_surfels *s)
{
    if (!s) return fail(SLR_E_INVALID, "surfels is NULL");
    if (s->n < 0 || s->n > (int64_t(1) << 30)) return fail(SLR_E_INVALID, "surfel count %lld out of range", (long long)s->n);
    if (s->n > 0 && (!s->means || !s->quats || !s->log_scales || !s->logits))
        return fail(SLR_E_INVALID, "surfel parameter pointer is NULL");
    if (!aligned(s->means, 4) || !aligned(s->quats, 16) || !aligned(s->log_scales, 8) || !aligned(s->logits, 4))
        return fail(SLR_E_INVALID, "surfel arrays misaligned (quats need 16 bytes, log_scales 8)");
    return SLR_OK;
}

// Host-made direction tables: column centres, row centres, rows -/+ margin.
std::vector<double> make_tables(const slr_sensor &s)
{
    const int H = s.height, W = s.width;
    std::vector<double> t(2 * (size_t)(W + 3 * H));
    double *col = t.data(), *row = col + 2 * W, *rlo = row + 2 * H, *rhi = rlo + 2 * H;
    for (int j = 0; j < W; ++j) {
        const double az = (((double)j + 0.5) - s.cu) / s.fu;
        col[2 * j] = std::cos(az);
        col[2 * j + 1] = std::sin(az);
    }
    for (int i = 0; i < H; ++i) {
        const double el = (((double)i + 0.5) - s.cv) / s.fv;
        row[2 * i] = std::cos(el);
        row[2 * i + 1] = std::sin(el);
        rlo[2 * i] = std::cos(el - kBoxMargin);
        rlo[2 * i + 1] = std::sin(el - kBoxMargin);
        rhi[2 * i] = std::cos(el + kBoxMargin);
        rhi[2 * i + 1] = std::sin(el + kBoxMargin);
    }
    return t;
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
        hipEventRecord(a, s);
    }
    ~StageScope()
    {
        if (!a) return;
        hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_timer_mu);
        g_pending.push_back({stage, a, b});
    }
};

}  // namespace

namespace slr {

Layout make_layout(int64_t n, int64_t cap, int32_t H, int32_t W, int32_t th, int32_t tw)
{
    Layout L{};
    L.n = n; L.cap = cap; L.H = H; L.W = W; L.th = th; L.tw = tw;
    L.tiles_x = (W + tw - 1) / tw;
    L.tiles_y = (H + th - 1) / th;
    L.ntiles = L.tiles_x * L.tiles_y;
    L.tile_bits = ceil_log2(L.ntiles);
    L.depth_passes = 4;
    L.tile_passes = (L.tile_bits + kMaxDigitBits - 1) / kMaxDigitBits;
    L.depth_in_1 = (L.depth_passes % 2) == 1;
    L.tile_in_1 = (L.tile_passes % 2) == 1;
    const int64_t nn = n > 0 ? n : 1, cc = cap > 0 ? cap : 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
    L.tables = take(sizeof(double) * 2 * (size_t)(W + 3 * H));
    L.rec = take(sizeof(RasterRec) * nn);
    L.frame = take(sizeof(FrameRec) * nn);
    L.box = take(sizeof(PixBox) * nn);
    L.skey = take(4 * nn);
    L.key0 = take(4 * nn); L.val0 = take(4 * nn); L.key1 = take(4 * nn); L.val1 = take(4 * nn);
    L.cnt = take(4 * nn);
    L.off = take(4 * nn);
    const int64_t nb_n = (nn + kSortTile - 1) / kSortTile, nb_k = (cc + kSortTile - 1) / kSortTile;
    L.blocksum = take(4 * nb_n);
    L.pt0 = take(4 * cc); L.pv0 = take(4 * cc); L.pt1 = take(4 * cc); L.pv1 = take(4 * cc);
    L.ranges = take(8 * (size_t)L.ntiles);
    L.hist = take(4 * 256 * (size_t)(nb_n > nb_k ? nb_n : nb_k));
    L.stateT = take(4 * (size_t)H * W);
    L.stateN = take(4 * (size_t)H * W);
    L.census = take(16 * (size_t)H * W);
    L.acc = take(4 * (size_t)kAccStride * nn);
    L.misc = take(4096);
    L.total = o;
    return L;
}

}  // namespace slr

using slr::Layout;

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

slr_status slr_workspace_size(const slr_sensor *sensor, const slr_tiling *tiling, int64_t n, int64_t pair_capacity,
                              size_t *bytes)
{
    slr_status st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if ((st = check_tiling(tiling)) != SLR_OK) return st;
    if (!bytes) return fail(SLR_E_INVALID, "bytes is NULL");
    if (n < 0 || pair_capacity < 0 || pair_capacity > 0x7fffffffLL)
        return fail(SLR_E_INVALID, "n and pair_capacity must be in [0, 2^31)");
    *bytes = slr::make_layout(n, pair_capacity, sensor->height, sensor->width, tiling->tile_h, tiling->tile_w).total;
    return SLR_OK;
}

static slr_status common_checks(const slr_surfels *surfels, const double *pose, const slr_sensor *sensor,
                                const slr_tiling *tiling, void *ws, size_t ws_bytes, int64_t cap, Layout *L)
{
    slr_status st;
    if ((st = check_surfels(surfels)) != SLR_OK) return st;
    if ((st = check_sensor(sensor)) != SLR_OK) return st;
    if ((st = check_tiling(tiling)) != SLR_OK) return st;
    if (!pose || !aligned(pose, 8)) return fail(SLR_E_INVALID, "pose must be a non-NULL, 8-byte aligned device pointer");
    if (cap < 0 || cap > 0x7fffffffLL) return fail(SLR_E_INVALID, "pair_capacity must be in [0, 2^31)");
    if (!ws || !aligned(ws, 256)) return fail(SLR_E_INVALID, "workspace must be non-NULL and 256-byte aligned");
    *L = slr::make_layout(surfels->n, cap, sensor->height, sensor->width, tiling->tile_h, tiling->tile_w);
    if (ws_bytes < L->total)
        return fail(SLR_E_INVALID, "workspace has %zu bytes, needs %zu", ws_bytes, L->total);
    return SLR_OK;
}

slr_status slr_render(const slr_surfels *surfels, const double *pose_cw, const slr_sensor *sensor,
                      const slr_tiling *tiling, void *workspace, size_t workspace_bytes, int64_t pair_capacity,
                      float *depth, float *normal, float *alpha, int64_t *pairs_out, void *stream)
{
    Layout L;
    slr_status st = common_checks(surfels, pose_cw, sensor, tiling, workspace, workspace_bytes, pair_capacity, &L);
    if (st != SLR_OK) return st;
    if (!depth || !normal || !alpha) return fail(SLR_E_INVALID, "output pointer is NULL");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    std::vector<double> tab = make_tables(*sensor);
    HIP_TRY(hipMemcpyAsync(ws + L.tables, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
    {
        StageScope t(0, s);
        slr::launch_project(*surfels, pose_cw, *sensor, L, ws, std::cos(kBoxMargin), std::sin(kBoxMargin), s);
    }
    {
        StageScope t(1, s);
        slr::launch_depth_sort(L, ws, s);
    }
    uint64_t K = 0;
    if (L.n > 0) {
        {
            StageScope t(2, s);
            slr::launch_scan_counts(L, ws, s);
        }
        HIP_TRY(hipMemcpyAsync(&K, ws + L.misc, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));  // K, and the table upload's host buffer
    HIP_TRY(hipGetLastError());
    if (pairs_out) *pairs_out = (int64_t)K;
    if ((int64_t)K > pair_capacity)
        return fail(SLR_E_CAPACITY, "%llu (tile, surfel) pairs exceed the capacity %lld", (unsigned long long)K,
                    (long long)pair_capacity);
    {
        StageScope t(3, s);
        slr::launch_emit_and_tile_sort(L, ws, (int64_t)K, s);
    }
    {
        StageScope t(4, s);
        slr::launch_raster_fwd(L, *sensor, ws, (int64_t)K, depth, normal, alpha, s);
    }
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

slr_status slr_backward(const slr_surfels *surfels, const double *pose_cw, const slr_sensor *sensor,
                        const slr_tiling *tiling, void *workspace, size_t workspace_bytes, int64_t pair_capacity,
                        const float *dL_ddepth, const float *dL_dnormal, const float *dL_dalpha, float *d_means,
                        float *d_quats, float *d_log_scales, float *d_logits, double *d_pose, uint32_t flags,
                        void *stream)
{
    Layout L;
    slr_status st = common_checks(surfels, pose_cw, sensor, tiling, workspace, workspace_bytes, pair_capacity, &L);
    if (st != SLR_OK) return st;
    const bool pose_only = (flags & SLR_POSE_ONLY) != 0;
    const bool accumulate = (flags & SLR_ACCUMULATE) != 0;
    const int nset = (d_means != nullptr) + (d_quats != nullptr) + (d_log_scales != nullptr) + (d_logits != nullptr);
    if (pose_only && nset != 0) return fail(SLR_E_INVALID, "SLR_POSE_ONLY takes NULL surfel gradients");
    if (!pose_only && nset != 4) return fail(SLR_E_INVALID, "surfel gradient pointers must all be set");
    if (!pose_only && !aligned(d_quats, 16)) return fail(SLR_E_INVALID, "d_quats must be 16-byte aligned");
    if (pose_only && !d_pose) return fail(SLR_E_INVALID, "SLR_POSE_ONLY needs d_pose");
    if (flags & ~(SLR_POSE_ONLY | SLR_ACCUMULATE)) return fail(SLR_E_INVALID, "unknown flags 0x%x", flags);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    double *dpose = d_pose ? d_pose : reinterpret_cast<double *>(ws + L.misc + 2048);
    slr::launch_fill_u32(dpose, 0u, 12, s);
    if (!pose_only) slr::launch_fill_u32(ws + L.acc, 0u, (int64_t)slr::kAccStride * L.n, s);
    if (L.ntiles > 0) {
        StageScope t(5, s);
        slr::launch_raster_bwd(L, *sensor, ws, pose_cw, dL_ddepth, dL_dnormal, dL_dalpha, dpose, pose_only, s);
    }
    if (!pose_only) {
        StageScope t(6, s);
        slr::launch_surfel_grad(*surfels, L, ws, d_means, d_quats, d_log_scales, d_logits, accumulate, s);
    }
    HIP_TRY(hipGetLastError());
    return SLR_OK;
}

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
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
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
    Layout L = slr::make_layout(n, pair_capacity, sensor->height, sensor->width, tiling->tile_h, tiling->tile_w);
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
    v->tiles_x = L.tiles_x;
    v->tiles_y = L.tiles_y;
    return SLR_OK;
}

}  // extern "C"

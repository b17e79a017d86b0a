"""Python binding of libslr.so (argument marshalling only).

Every step of the render and its backward runs in the HIP library; PyTorch
provides device memory and the current stream.  If the library is missing the
import fails loudly: there is no fallback path.
"""
import ctypes as C
import json
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslr.so")

SLR_OK, SLR_E_INVALID, SLR_E_CAPACITY, SLR_E_HIP, SLR_E_UNSUPPORTED = 0, -1, -2, -3, -4
SLR_POSE_ONLY = 1
SLR_ACCUMULATE = 2
NUM_STAGES = 10
STAGES = ["project", "range_sort", "count_scan", "emit_tile_sort", "raster_fwd", "raster_bwd", "surfel_grad", "loss",
          "pose_gn", "photo_gn"]


class Sensor(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("fu", C.c_double), ("cu", C.c_double),
                ("fv", C.c_double), ("cv", C.c_double), ("near_m", C.c_double)]


class Tiling(C.Structure):
    _fields_ = [("tile_h", C.c_int32), ("tile_w", C.c_int32), ("variant", C.c_int32), ("schedule", C.c_int32),
                ("bwd_variant", C.c_int32), ("box", C.c_int32), ("bwd_batch", C.c_int32)]


VARIANT_DEFAULT, VARIANT_LDS, VARIANT_SCALAR, VARIANT_WAVE = 0, 1, 2, 3
VARIANT_DETERMINISTIC = 4   # backward form only: fixed-order sums, bit-reproducible gradients
SCHEDULE_DEFAULT, SCHEDULE_TILE, SCHEDULE_LONGEST, SCHEDULE_QUEUE = 0, 1, 2, 3


class Surfels(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("quats", C.c_void_p), ("log_scales", C.c_void_p),
                ("logits", C.c_void_p)]


class Views(C.Structure):
    _fields_ = [("keys", C.c_void_p), ("counts", C.c_void_p), ("pixbox", C.c_void_p), ("sorted_tile", C.c_void_p),
                ("sorted_id", C.c_void_p), ("ranges", C.c_void_p), ("T_final", C.c_void_p), ("n_proc", C.c_void_p),
                ("census", C.c_void_p), ("tiles_x", C.c_int64), ("tiles_y", C.c_int64)]


class Frame(C.Structure):
    _fields_ = [("set", C.c_int32), ("pose_cw", C.c_void_p), ("sensor", Sensor), ("depth", C.c_void_p),
                ("normal", C.c_void_p), ("alpha", C.c_void_p), ("dL_ddepth", C.c_void_p), ("dL_dnormal", C.c_void_p),
                ("dL_dalpha", C.c_void_p), ("d_pose", C.c_void_p), ("tile_h", C.c_int32), ("tile_w", C.c_int32)]


class SurfelGrads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("quats", C.c_void_p), ("log_scales", C.c_void_p), ("logits", C.c_void_p)]


class LossFrame(C.Structure):
    _fields_ = [("pixels", C.c_int64), ("depth", C.c_void_p), ("normal", C.c_void_p), ("target_depth", C.c_void_p),
                ("target_normal", C.c_void_p), ("w_d", C.c_float), ("w_n", C.c_float), ("dL_ddepth", C.c_void_p),
                ("dL_dnormal", C.c_void_p)]


EXPORTS = ["slr_camera_matrix", "slr_workspace_size", "slr_render", "slr_backward", "slr_workspace_views",
           "slr_batch_workspace_size", "slr_batch_prepare", "slr_batch_render", "slr_batch_backward",
           "slr_batch_counters", "slr_batch_views", "slr_batch_autotune", "slr_loss_l1_normal", "slr_loss_l1_normal_frames", "slr_adam_step",
           "slr_stage_timer_enable", "slr_stage_times",
           "slr_pose_gn", "slr_photo_workspace_size", "slr_photo_gn", "slr_photo_gn_noalloc", "slr_cloud_to_range", "slr_range_normals", "slr_loss_map",
           "slr_scale_reg", "slr_init_workspace_size", "slr_init_splats", "slr_status_string", "slr_last_error"]

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.slr_camera_matrix.argtypes = [D, D, D, D, I32, I32, P]
        L.slr_workspace_size.argtypes = [P, P, I64, I64, P]
        L.slr_render.argtypes = [P, P, P, P, P, C.c_size_t, I64, P, P, P, P, P]
        L.slr_backward.argtypes = [P, P, P, P, P, C.c_size_t, I64, P, P, P, P, P, P, P, P, C.c_uint32, P]
        L.slr_workspace_views.argtypes = [P, P, I64, I64, P, C.c_size_t, P]
        L.slr_pose_gn.argtypes = [P, P, P, P, P, C.c_size_t, I64, P, P, P, D, P, P]
        L.slr_photo_workspace_size.argtypes = [P, P]
        L.slr_photo_gn.argtypes = [P, P, P, P, P, D, P, C.c_size_t, P, P]
        L.slr_photo_gn_noalloc.argtypes = [P, P, P, P, P, D, P, P]
        L.slr_cloud_to_range.argtypes = [P, I64, P, P, P]
        L.slr_range_normals.argtypes = [P, P, P, P]
        L.slr_loss_map.argtypes = [I64, P, P, P, P, P, C.c_float, C.c_float, C.c_float, P, P, P, P, P]
        L.slr_scale_reg.argtypes = [I64, P, D, D, P, P, P]
        L.slr_init_workspace_size.argtypes = [P, P]
        L.slr_init_splats.argtypes = [P, P, P, P, I64, P, D, C.c_float, P, C.c_size_t, P, P, P, P, P, P]
        BATCH = [I32, P, I32, P, P, I64, P, C.c_size_t]
        L.slr_batch_workspace_size.argtypes = [I32, P, I32, P, P, I64, P]
        L.slr_batch_prepare.argtypes = BATCH + [P]
        L.slr_batch_render.argtypes = BATCH + [P]
        L.slr_batch_backward.argtypes = [I32, P, P, I32, P, P, I64, P, C.c_size_t, C.c_uint32, P]
        L.slr_batch_counters.argtypes = BATCH + [P]
        L.slr_batch_views.argtypes = BATCH + [P]
        L.slr_batch_autotune.argtypes = [I32, P, P, I32, P, P, I32, I64, P, C.c_size_t, I32, P, P, P]
        L.slr_loss_l1_normal.argtypes = [I64, P, P, P, P, C.c_float, C.c_float, P, P, P, P]
        L.slr_loss_l1_normal_frames.argtypes = [I32, P, P, P]
        L.slr_adam_step.argtypes = [I64, P, P, P, P, P, P, P, P, P]
        L.slr_stage_timer_enable.argtypes = [I32]
        L.slr_stage_times.argtypes = [P, P]
        L.slr_status_string.argtypes = [I32]
        L.slr_status_string.restype = C.c_char_p
        L.slr_last_error.restype = C.c_char_p
        for f in ("slr_camera_matrix", "slr_workspace_size", "slr_render", "slr_backward", "slr_workspace_views",
                  "slr_batch_workspace_size", "slr_batch_prepare", "slr_batch_render", "slr_batch_backward",
                  "slr_batch_counters", "slr_batch_views", "slr_batch_autotune", "slr_loss_l1_normal",
                  "slr_loss_l1_normal_frames",
                  "slr_adam_step", "slr_stage_timer_enable", "slr_stage_times", "slr_pose_gn", "slr_photo_workspace_size",
                  "slr_photo_gn", "slr_photo_gn_noalloc", "slr_cloud_to_range", "slr_range_normals", "slr_loss_map", "slr_scale_reg",
                  "slr_init_workspace_size", "slr_init_splats"):
            getattr(L, f).restype = I32
        _lib = L
    return _lib


class SlrError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        msg = lib().slr_last_error().decode()
        super().__init__(f"{what}: {lib().slr_status_string(status).decode()}: {msg}")


def _check(st, what):
    if st != SLR_OK:
        raise SlrError(st, what)


def camera_matrix(az_min, az_max, el_min, el_max, H, W):
    """(fu, cu, fv, cv) of the camera matrix K (Supp. A)."""
    out = (C.c_double * 4)()
    _check(lib().slr_camera_matrix(az_min, az_max, el_min, el_max, H, W, out), "slr_camera_matrix")
    return tuple(out)


def make_sensor(H, W, az=(-math.pi, math.pi), el=(math.radians(-25.0), math.radians(15.0)), near=0.2):
    fu, cu, fv, cv = camera_matrix(az[0], az[1], el[0], el[1], H, W)
    return dict(height=H, width=W, fu=fu, cu=cu, fv=fv, cv=cv, near=near)


def _sensor(s):
    return Sensor(int(s["height"]), int(s["width"]), float(s["fu"]), float(s["cu"]), float(s["fv"]),
                  float(s["cv"]), float(s["near"]))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def workspace_size(sensor, tiling, n, capacity):
    b = C.c_size_t(0)
    s, t = _sensor(sensor), Tiling(*tiling)
    _check(lib().slr_workspace_size(C.byref(s), C.byref(t), int(n), int(capacity), C.byref(b)), "slr_workspace_size")
    return int(b.value)


def _surfels(means, quats, log_scales, logits):
    for name, t in (("means", means), ("quats", quats), ("log_scales", log_scales), ("logits", logits)):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return Surfels(means.shape[0], means.data_ptr(), quats.data_ptr(), log_scales.data_ptr(), logits.data_ptr())


def _pose(T_cw):
    if T_cw.dtype != torch.float64 or not T_cw.is_cuda or T_cw.shape != (4, 4) or not T_cw.is_contiguous():
        raise ValueError("T_cw must be a contiguous float64 CUDA tensor of shape (4, 4)")
    return T_cw


class Renderer:
    """One image's workspace; grows its pair capacity on demand (plain form)."""

    def __init__(self, sensor, tiling=(16, 16), capacity=1 << 20, device="cuda"):
        self.sensor = dict(sensor)
        self.tiling = tuple(tiling)
        self.capacity = int(capacity)
        self.device = device
        self.n = -1
        self.ws = None
        self.K = 0
        # bumped by every forward: the workspace holds the binning and per-pixel
        # state of the last render only, which a pending backward must match
        self.generation = 0

    def _ensure(self, n):
        need = workspace_size(self.sensor, self.tiling, n, self.capacity)
        if self.ws is None or self.ws.numel() < need or self.n != n:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            self.n = n

    def forward(self, means, quats, log_scales, logits, T_cw):
        sf = _surfels(means, quats, log_scales, logits)
        _pose(T_cw)
        H, W = int(self.sensor["height"]), int(self.sensor["width"])
        dev = means.device
        depth = torch.empty((H, W), dtype=torch.float32, device=dev)
        normal = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
        alpha = torch.empty((H, W), dtype=torch.float32, device=dev)
        s, t = _sensor(self.sensor), Tiling(*self.tiling)
        for _ in range(3):
            self._ensure(sf.n)
            K = C.c_int64(0)
            st = lib().slr_render(C.byref(sf), _ptr(T_cw), C.byref(s), C.byref(t), _ptr(self.ws), self.ws.numel(),
                                  self.capacity, _ptr(depth), _ptr(normal), _ptr(alpha), C.byref(K), _stream())
            if st == SLR_E_CAPACITY:
                self.capacity = int(K.value * 1.25) + 1024
                self.ws = None
                continue
            _check(st, "slr_render")
            self.K = int(K.value)
            self.generation += 1
            return depth, normal, alpha
        raise SlrError(SLR_E_CAPACITY, "slr_render")

    def backward(self, means, quats, log_scales, logits, T_cw, dL_dD, dL_dN, dL_dO, pose_only=False,
                 want_pose=True, out=None):
        """Gradients of the last render.  out=(grads dict, dpose) adds into
        existing buffers (SLR_ACCUMULATE) instead of allocating new ones."""
        sf = _surfels(means, quats, log_scales, logits)
        _pose(T_cw)
        for name, g in (("dL_ddepth", dL_dD), ("dL_dnormal", dL_dN), ("dL_dalpha", dL_dO)):
            if g is not None and (g.dtype != torch.float32 or not g.is_contiguous()):
                raise ValueError(f"{name} must be contiguous float32")
        n = sf.n
        dev = means.device
        g = None
        flags = SLR_POSE_ONLY if pose_only else 0
        if out is not None:
            g, dpose = out
            flags |= SLR_ACCUMULATE
        else:
            if not pose_only:
                g = dict(means=torch.empty((n, 3), dtype=torch.float32, device=dev),
                         quats=torch.empty((n, 4), dtype=torch.float32, device=dev),
                         log_scales=torch.empty((n, 2), dtype=torch.float32, device=dev),
                         logits=torch.empty((n,), dtype=torch.float32, device=dev))
            dpose = torch.empty(6, dtype=torch.float64, device=dev) if (want_pose or pose_only) else None
        s, t = _sensor(self.sensor), Tiling(*self.tiling)
        st = lib().slr_backward(C.byref(sf), _ptr(T_cw), C.byref(s), C.byref(t), _ptr(self.ws), self.ws.numel(),
                                self.capacity, _ptr(dL_dD), _ptr(dL_dN), _ptr(dL_dO),
                                _ptr(g["means"]) if g else None, _ptr(g["quats"]) if g else None,
                                _ptr(g["log_scales"]) if g else None, _ptr(g["logits"]) if g else None,
                                _ptr(dpose), flags, _stream())
        _check(st, "slr_backward")
        return g, dpose

    def pose_gn(self, means, quats, log_scales, logits, T_cw, depth, target, weight=None, huber_k=0.0, out=None):
        """Pose-only Gauss-Newton normal equations of the last render
        (slr_pose_gn): returns (H [6,6], g [6], cost []) as FP64 CUDA tensors
        (views of one 43-value buffer; `out` reuses a given buffer)."""
        sf = _surfels(means, quats, log_scales, logits)
        _pose(T_cw)
        for name, a in (("depth", depth), ("target", target), ("weight", weight)):
            if a is not None and (a.dtype != torch.float32 or not a.is_contiguous()):
                raise ValueError(f"{name} must be contiguous float32")
        buf = out if out is not None else torch.empty(43, dtype=torch.float64, device=means.device)
        s, t = _sensor(self.sensor), Tiling(*self.tiling)
        _check(lib().slr_pose_gn(C.byref(sf), _ptr(T_cw), C.byref(s), C.byref(t), _ptr(self.ws), self.ws.numel(),
                                 self.capacity, _ptr(depth), _ptr(target), _ptr(weight), float(huber_k), _ptr(buf),
                                 _stream()), "slr_pose_gn")
        return buf[:36].view(6, 6), buf[36:42], buf[42]

    def views(self):
        """Copies of the binning results and per-pixel state of the last render."""
        v = Views()
        s, t = _sensor(self.sensor), Tiling(*self.tiling)
        _check(lib().slr_workspace_views(C.byref(s), C.byref(t), self.n, self.capacity, _ptr(self.ws),
                                         self.ws.numel(), C.byref(v)), "slr_workspace_views")
        base = self.ws.data_ptr()
        H, W = int(self.sensor["height"]), int(self.sensor["width"])

        def take(ptr, count, dtype):
            off = ptr - base
            nbytes = count * torch.tensor([], dtype=dtype).element_size()
            return self.ws[off:off + nbytes].view(dtype).clone()

        n, K = self.n, self.K
        nt = int(v.tiles_x * v.tiles_y)
        return dict(keys=take(v.keys, n, torch.int32), counts=take(v.counts, n, torch.int32),
                    pixbox=take(v.pixbox, 8 * n, torch.int16).view(n, 8),
                    sorted_tile=take(v.sorted_tile, K, torch.int32), sorted_id=take(v.sorted_id, K, torch.int32),
                    ranges=take(v.ranges, 2 * nt, torch.int32).view(nt, 2),
                    T_final=take(v.T_final, H * W, torch.float32).view(H, W),
                    n_proc=take(v.n_proc, H * W, torch.int32).view(H, W),
                    census=take(v.census, 4 * H * W, torch.int32).view(4, H, W), tiles_x=int(v.tiles_x),
                    tiles_y=int(v.tiles_y), K=K)


# Candidate tilings of the autotuner: (tile_h, tile_w, forward variant,
# schedule, backward variant[, backward batch]); the renderer's box mode is
# inserted as the sixth entry.
BOX_EXACT, BOX_OPACITY, BOX_VERTEX = 0, 1, 2
TUNE_CANDIDATES = [(th, tw, VARIANT_WAVE, SCHEDULE_LONGEST, bv) for th, tw in ((16, 16), (8, 32), (32, 8))
                   for bv in (VARIANT_WAVE, VARIANT_LDS)] + [(32, 8, VARIANT_LDS, SCHEDULE_LONGEST, VARIANT_LDS),
                                                             (32, 8, VARIANT_WAVE, SCHEDULE_LONGEST, VARIANT_LDS, 128),
                                                             (16, 16, VARIANT_WAVE, SCHEDULE_LONGEST, VARIANT_LDS, 128),
                                                             (32, 8, VARIANT_WAVE, SCHEDULE_QUEUE, VARIANT_LDS)]
_tuned = {}   # image-size class -> tiling chosen by the autotuner

# The autotuner's choices persist across processes in a JSON file when
# SLR_AUTOTUNE_CACHE names one: one entry per (device name, frame image sizes,
# set sizes), the chosen tiling as a list.  A missing or unreadable file is an
# empty cache; entries are written by replacing the file.
AUTOTUNE_CACHE_ENV = "SLR_AUTOTUNE_CACHE"


def _cache_key(key, device_name):
    frames, sets = key
    return json.dumps({"device": device_name, "frames": [list(f) for f in frames], "sets": list(sets)},
                      sort_keys=True)


def _cache_read(path):
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def autotune_cache_lookup(key, device_name, path=None):
    """The cached tiling of an image-size class on a device, or None."""
    path = path or os.environ.get(AUTOTUNE_CACHE_ENV)
    if not path:
        return None
    t = _cache_read(path).get(_cache_key(key, device_name))
    return tuple(int(x) for x in t) if isinstance(t, list) and len(t) >= 5 else None


def autotune_cache_store(key, device_name, tiling, path=None):
    """Record the tiling of an image-size class on a device (no-op without a path)."""
    path = path or os.environ.get(AUTOTUNE_CACHE_ENV)
    if not path:
        return
    data = _cache_read(path)
    data[_cache_key(key, device_name)] = [int(x) for x in tiling]
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class BatchRenderer:
    """Batched form: many frames (each its own pose, sensor and image size;
    frames may share a surfel set) rendered and differentiated by one set of
    launches with no host synchronisation, so a whole iteration can be
    captured in a HIP graph.  Buffers (outputs, upstream gradients, pose and
    surfel gradients) are owned here and stay at fixed addresses.

    sets:   list of dicts with means, quats, log_scales, logits (CUDA tensors)
    frames: list of dicts with set (index), T_cw (float64 [4,4] CUDA), sensor,
            optionally tile = (tile_h, tile_w): the frame's own tile shape
    """

    def __init__(self, sets, frames, tiling=(16, 16), capacity=1 << 22, device="cuda"):
        """tiling: (tile_h, tile_w[, variant[, schedule]]) or "auto" (the
        autotuner's choice for this image-size class, tuned on first use)."""
        self.sets = sets
        self.frames = frames
        self._key = (tuple((int(f["sensor"]["height"]), int(f["sensor"]["width"])) for f in frames),
                     tuple(int(st["means"].shape[0]) for st in sets))
        auto = isinstance(tiling, str) and tiling == "auto"
        if auto and self._key not in _tuned:
            cached = autotune_cache_lookup(self._key, torch.cuda.get_device_name(device))
            if cached is not None:
                _tuned[self._key] = cached
        self.tiling = _tuned.get(self._key, TUNE_CANDIDATES[0]) if auto else tuple(tiling)
        self.capacity = int(capacity)
        self.device = device
        self.out, self.up, self.dpose = [], [], []
        for f in frames:
            H, W = int(f["sensor"]["height"]), int(f["sensor"]["width"])
            _pose(f["T_cw"])
            self.out.append((torch.zeros((H, W), device=device), torch.zeros((H, W, 3), device=device),
                             torch.zeros((H, W), device=device)))
            self.up.append((torch.zeros((H, W), device=device), torch.zeros((H, W, 3), device=device),
                            torch.zeros((H, W), device=device)))
            self.dpose.append(torch.zeros(6, dtype=torch.float64, device=device))
        self.grads = [dict(means=torch.zeros_like(st["means"]), quats=torch.zeros_like(st["quats"]),
                           log_scales=torch.zeros_like(st["log_scales"]), logits=torch.zeros_like(st["logits"]))
                      for st in sets]
        self._c_sets = (Surfels * max(len(sets), 1))(*[_surfels(st["means"], st["quats"], st["log_scales"],
                                                                 st["logits"]) for st in sets])
        self._c_grads = (SurfelGrads * max(len(sets), 1))(*[SurfelGrads(g["means"].data_ptr(), g["quats"].data_ptr(),
                                                                         g["log_scales"].data_ptr(),
                                                                         g["logits"].data_ptr()) for g in self.grads])
        self._make_frames()
        self.ws = None
        self.prepare()
        if auto and self._key not in _tuned:
            self.autotune()

    def _make_frames(self):
        self._c_frames = (Frame * max(len(self.frames), 1))(*[
            Frame(int(f["set"]), f["T_cw"].data_ptr(), _sensor(f["sensor"]), o[0].data_ptr(), o[1].data_ptr(),
                  o[2].data_ptr(), u[0].data_ptr(), u[1].data_ptr(), u[2].data_ptr(), dp.data_ptr(),
                  *(tuple(f.get("tile") or (0, 0))))
            for f, o, u, dp in zip(self.frames, self.out, self.up, self.dpose)])

    def frame_tile(self, f):
        """(tile_h, tile_w) of frame f: its own shape or the batch tiling's."""
        t = self.frames[f].get("tile")
        return (int(t[0]), int(t[1])) if t else (int(self.tiling[0]), int(self.tiling[1]))

    def set_frame_tiles(self, tiles):
        """Give frame f the tile shape tiles[f] ((tile_h, tile_w), or None for the
        batch tiling's) and re-prepare the workspace."""
        for f, t in zip(self.frames, tiles):
            f["tile"] = None if t is None else (int(t[0]), int(t[1]))
        self._make_frames()
        self.prepare()

    def tune_frame_tiles(self, shapes=((16, 16), (8, 32), (32, 8), (4, 64)), reps=3):
        """Tile shape per image-size class: for each class of frames with the same
        (H, W), in turn, every shape is timed on the whole batch (render +
        backward, the batch's other settings fixed) and the fastest kept.
        Returns {(H, W): (tile_h, tile_w)}."""
        classes = {}
        for k, f in enumerate(self.frames):
            classes.setdefault((int(f["sensor"]["height"]), int(f["sensor"]["width"])), []).append(k)
        cur = [self.frame_tile(k) for k in range(len(self.frames))]
        arr = (Tiling * 1)(Tiling(*self.tiling))
        ms = (C.c_double * 1)()
        best_i = C.c_int32(-1)
        for cls, members in classes.items():
            timed = {}
            for sh in shapes:
                trial = list(cur)
                for k in members:
                    trial[k] = sh
                self.set_frame_tiles(trial)
                _check(lib().slr_batch_autotune(len(self.sets), self._c_sets, self._c_grads, len(self.frames),
                                                self._c_frames, arr, 1, self.capacity, _ptr(self.ws), self.ws.numel(),
                                                int(reps), ms, C.byref(best_i), _stream()), "slr_batch_autotune")
                if ms[0] > 0:
                    timed[sh] = ms[0]
            best = min(timed, key=timed.get)
            for k in members:
                cur[k] = best
        self.set_frame_tiles(cur)
        return {cls: cur[members[0]] for cls, members in classes.items()}

    def autotune(self, candidates=None, reps=3):
        """Time render + backward of this batch for each candidate tiling (median
        of reps, after one untimed step) and keep the fastest.  Returns
        {tiling: ms} (-1 where the pairs overflowed the capacity)."""
        box = tuple(self.tiling)[5] if len(self.tiling) > 5 else 0   # the binning's box mode is kept
        cands = []
        for c in (candidates or TUNE_CANDIDATES):
            c = tuple(c) + (0,) * max(0, 5 - len(c))
            cands.append(c[:5] + (box,) + c[5:])
        arr = (Tiling * len(cands))(*[Tiling(*c) for c in cands])
        need = 0
        for c in cands:
            b = C.c_size_t(0)
            t = Tiling(*c)
            _check(lib().slr_batch_workspace_size(len(self.sets), self._c_sets, len(self.frames), self._c_frames,
                                                  C.byref(t), self.capacity, C.byref(b)), "slr_batch_workspace_size")
            need = max(need, b.value)
        if self.ws.numel() < need:
            self.ws = torch.empty(int(need), dtype=torch.uint8, device=self.device)
        ms = (C.c_double * len(cands))()
        best = C.c_int32(-1)
        _check(lib().slr_batch_autotune(len(self.sets), self._c_sets, self._c_grads, len(self.frames), self._c_frames,
                                        arr, len(cands), self.capacity, _ptr(self.ws), self.ws.numel(), int(reps), ms,
                                        C.byref(best), _stream()), "slr_batch_autotune")
        self.tiling = cands[best.value]
        _tuned[self._key] = self.tiling
        autotune_cache_store(self._key, torch.cuda.get_device_name(self.device), self.tiling)
        self.prepare()
        return {c: ms[k] for k, c in enumerate(cands)}

    def _args(self):
        t = Tiling(*self.tiling)
        return [len(self.sets), self._c_sets, len(self.frames), self._c_frames, C.byref(t), self.capacity]

    def prepare(self):
        b = C.c_size_t(0)
        _check(lib().slr_batch_workspace_size(*self._args(), C.byref(b)), "slr_batch_workspace_size")
        if self.ws is None or self.ws.numel() < b.value:
            self.ws = torch.empty(int(b.value), dtype=torch.uint8, device=self.device)
        _check(lib().slr_batch_prepare(*self._args(), _ptr(self.ws), self.ws.numel(), _stream()), "slr_batch_prepare")
        ptr = C.c_void_p(0)
        _check(lib().slr_batch_counters(*self._args(), _ptr(self.ws), self.ws.numel(), C.byref(ptr)),
               "slr_batch_counters")
        off = ptr.value - self.ws.data_ptr()
        self.counters = self.ws[off:off + 56].view(torch.int64)

    def render(self):
        _check(lib().slr_batch_render(*self._args(), _ptr(self.ws), self.ws.numel(), _stream()), "slr_batch_render")

    def backward(self, pose_only=False, accumulate=False):
        flags = (SLR_POSE_ONLY if pose_only else 0) | (SLR_ACCUMULATE if accumulate else 0)
        a = self._args()
        _check(lib().slr_batch_backward(a[0], a[1], None if pose_only else self._c_grads, a[2], a[3], a[4], a[5],
                                        _ptr(self.ws), self.ws.numel(), flags, _stream()), "slr_batch_backward")

    def views(self):
        """Copies of the batch's binning results and per-pixel state (global
        record, tile and pixel indices; see slr_batch_views) plus the
        per-frame offsets item_off, tile_off, pix_off (host lists)."""
        v = Views()
        _check(lib().slr_batch_views(*self._args(), _ptr(self.ws), self.ws.numel(), C.byref(v)), "slr_batch_views")
        base = self.ws.data_ptr()

        def take(ptr, count, dtype):
            off = ptr - base
            nbytes = count * torch.tensor([], dtype=dtype).element_size()
            return self.ws[off:off + nbytes].view(dtype).clone()

        item_off, tile_off, pix_off = [], [], []
        it = tl = px = 0
        for k, f in enumerate(self.frames):
            th, tw = self.frame_tile(k)
            H, W = int(f["sensor"]["height"]), int(f["sensor"]["width"])
            item_off.append(it); tile_off.append(tl); pix_off.append(px)
            it += int(self.sets[int(f["set"])]["means"].shape[0])
            tl += ((H + th - 1) // th) * ((W + tw - 1) // tw)
            px += H * W
        K, _ = self.pairs()
        return dict(keys=take(v.keys, it, torch.int32), counts=take(v.counts, it, torch.int32),
                    pixbox=take(v.pixbox, 8 * it, torch.int16).view(it, 8),
                    sorted_tile=take(v.sorted_tile, K, torch.int32), sorted_id=take(v.sorted_id, K, torch.int32),
                    ranges=take(v.ranges, 2 * tl, torch.int32).view(tl, 2),
                    T_final=take(v.T_final, px, torch.float32), n_proc=take(v.n_proc, px, torch.int32),
                    census=take(v.census, 4 * px, torch.int32).view(4, px), item_off=item_off, tile_off=tile_off,
                    pix_off=pix_off, K=K)

    def pairs(self):
        """(K, overflow) of the last render (synchronises)."""
        c = self.counters.cpu().tolist()
        return int(c[0]), int(c[1])

    def binned_records(self):
        """Number of surfel records of the last render that bin into some tile (synchronises)."""
        return int(self.counters[3].cpu())

    def invalid_records(self):
        """Number of (frame, surfel) records of the last render culled for a non-finite
        parameter or a zero quaternion (synchronises)."""
        return int(self.counters[6].cpu())

    def ensure_capacity(self, margin=1.25):
        """Grow the pair capacity if the last render overflowed; True if it did."""
        K, over = self.pairs()
        if over:
            self.capacity = int(over * margin) + 4096
            self.prepare()
            return True
        return False


def loss_l1_normal(D, N, Dt, Nt, w_d, w_n, gD, gN, loss=None):
    """Fused range + normal loss and its gradients (writes gD, gN; adds to loss)."""
    P = D.numel()
    _check(lib().slr_loss_l1_normal(P, _ptr(D), _ptr(N), _ptr(Dt), _ptr(Nt), float(w_d), float(w_n), _ptr(gD),
                                    _ptr(gN), _ptr(loss), _stream()), "slr_loss_l1_normal")


def loss_l1_normal_frames(items, loss=None):
    """The fused loss over several images in one launch.  items: sequence of
    (D, N, Dt, Nt, w_d, w_n, gD, gN) per image (writes gD, gN; adds the sum of
    the images' losses to loss)."""
    arr = (LossFrame * max(len(items), 1))()
    for i, (D, N, Dt, Nt, w_d, w_n, gD, gN) in enumerate(items):
        P = D.numel()
        for t, k in ((Dt, 1), (N, 3), (Nt, 3), (gD, 1), (gN, 3)):
            if t.numel() != k * P:
                raise ValueError(f"image {i}: buffer sizes do not match {P} pixels")
        arr[i] = LossFrame(P, D.data_ptr(), N.data_ptr(), Dt.data_ptr(), Nt.data_ptr(), float(w_d), float(w_n),
                           gD.data_ptr(), gN.data_ptr())
    _check(lib().slr_loss_l1_normal_frames(len(items), arr, _ptr(loss), _stream()), "slr_loss_l1_normal_frames")


class AdamConfig(C.Structure):
    _fields_ = [("lr_means", C.c_double), ("lr_quats", C.c_double), ("lr_log_scales", C.c_double),
                ("lr_logits", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("step", C.c_int32)]


def cloud_to_range(sensor, points, out=None):
    """Range image [H,W] (FP32 CUDA) of a sensor-frame point cloud [n,3] (slr_cloud_to_range)."""
    if points.dtype != torch.float32 or not points.is_contiguous() or points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be a contiguous float32 [n, 3] tensor")
    H, W = int(sensor["height"]), int(sensor["width"])
    out = out if out is not None else torch.empty((H, W), dtype=torch.float32, device=points.device)
    s = _sensor(sensor)
    _check(lib().slr_cloud_to_range(C.byref(s), points.shape[0], _ptr(points), _ptr(out), _stream()),
           "slr_cloud_to_range")
    return out


def range_normals(sensor, range_image, out=None):
    """Normals [H,W,3] (FP32 CUDA) from the gradients of a range image (slr_range_normals)."""
    if range_image.dtype != torch.float32 or not range_image.is_contiguous():
        raise ValueError("range_image must be contiguous float32")
    H, W = int(sensor["height"]), int(sensor["width"])
    out = out if out is not None else torch.empty((H, W, 3), dtype=torch.float32, device=range_image.device)
    s = _sensor(sensor)
    _check(lib().slr_range_normals(C.byref(s), _ptr(range_image), _ptr(out), _stream()), "slr_range_normals")
    return out


def loss_map(D, N, O, Dt, Nt, w_d, w_n, w_o, gD, gN, gO, loss=None):
    """Fused L_d + L_n + L_o and their gradients (slr_loss_map; writes gD, gN, gO, adds to loss)."""
    _check(lib().slr_loss_map(D.numel(), _ptr(D), _ptr(N), _ptr(O), _ptr(Dt), _ptr(Nt), float(w_d), float(w_n),
                              float(w_o), _ptr(gD), _ptr(gN), _ptr(gO), _ptr(loss), _stream()), "slr_loss_map")


def scale_reg(log_scales, tau_s, w_s, d_log_scales, loss=None):
    """Scale cap L_s (slr_scale_reg): adds its gradient to d_log_scales and its value to loss."""
    _check(lib().slr_scale_reg(log_scales.shape[0], _ptr(log_scales), float(tau_s), float(w_s), _ptr(d_log_scales),
                               _ptr(loss), _stream()), "slr_scale_reg")


def init_splats(sensor, range_image, pose_cw, uniforms, mask=None, scale_factor=1.0, logit=0.0):
    """Local model initialisation (slr_init_splats): splats drawn from a range
    image by the range-gradient weight map; returns dict of CUDA tensors
    means [n,3], quats [n,4], log_scales [n,2], logits [n], pixel [n] int32."""
    for name, a in (("range_image", range_image), ("mask", mask)):
        if a is not None and (a.dtype != torch.float32 or not a.is_contiguous()):
            raise ValueError(f"{name} must be contiguous float32")
    if uniforms.dtype != torch.float64 or not uniforms.is_contiguous():
        raise ValueError("uniforms must be contiguous float64")
    _pose(pose_cw)
    n = uniforms.numel()
    dev = range_image.device
    s = _sensor(sensor)
    nb = C.c_size_t(0)
    _check(lib().slr_init_workspace_size(C.byref(s), C.byref(nb)), "slr_init_workspace_size")
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    out = dict(means=torch.empty((n, 3), dtype=torch.float32, device=dev),
               quats=torch.empty((n, 4), dtype=torch.float32, device=dev),
               log_scales=torch.empty((n, 2), dtype=torch.float32, device=dev),
               logits=torch.empty((n,), dtype=torch.float32, device=dev),
               pixel=torch.empty((n,), dtype=torch.int32, device=dev))
    _check(lib().slr_init_splats(C.byref(s), _ptr(range_image), _ptr(mask), _ptr(pose_cw), n, _ptr(uniforms),
                                 float(scale_factor), float(logit), _ptr(ws), ws.numel(), _ptr(out["means"]),
                                 _ptr(out["quats"]), _ptr(out["log_scales"]), _ptr(out["logits"]), _ptr(out["pixel"]),
                                 _stream()), "slr_init_splats")
    return out


def photo_workspace_size(sensor):
    s = _sensor(sensor)
    n = C.c_size_t(0)
    _check(lib().slr_photo_workspace_size(C.byref(s), C.byref(n)), "slr_photo_workspace_size")
    return int(n.value)


def photo_gn(sensor, depth, query, pose_qm, weight=None, huber_k=0.0, ws=None, out=None):
    """Photometric registration normal equations (slr_photo_gn): returns
    (H [6,6], g [6], cost [], count []) as FP64 CUDA tensors (views of one
    44-value buffer).  depth, query, weight: contiguous FP32 [H,W] CUDA
    tensors; pose_qm: FP64 [4,4] CUDA tensor (render frame -> query frame)."""
    for name, a in (("depth", depth), ("query", query), ("weight", weight)):
        if a is not None and (a.dtype != torch.float32 or not a.is_contiguous()):
            raise ValueError(f"{name} must be contiguous float32")
    _pose(pose_qm)
    if ws is None:
        ws = torch.empty(photo_workspace_size(sensor), dtype=torch.uint8, device=depth.device)
    buf = out if out is not None else torch.empty(44, dtype=torch.float64, device=depth.device)
    s = _sensor(sensor)
    _check(lib().slr_photo_gn(C.byref(s), _ptr(depth), _ptr(query), _ptr(weight), _ptr(pose_qm), float(huber_k),
                              _ptr(ws), ws.numel(), _ptr(buf), _stream()), "slr_photo_gn")
    return buf[:36].view(6, 6), buf[36:42], buf[42], buf[43]


def photo_gn_noalloc(sensor, depth, query, pose_qm, out, weight=None, huber_k=0.0):
    """slr_photo_gn_noalloc: photo_gn without a workspace (the library's static
    scratch; images of at most 2^20 pixels; calls that overlap on one GPU race).
    out: FP64 CUDA tensor of 44 values, overwritten (H [0..35], g, cost, count)."""
    for name, a in (("depth", depth), ("query", query), ("weight", weight)):
        if a is not None and (a.dtype != torch.float32 or not a.is_contiguous()):
            raise ValueError(f"{name} must be contiguous float32")
    if out.dtype != torch.float64 or out.numel() < 44 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor of at least 44 values")
    _pose(pose_qm)
    s = _sensor(sensor)
    _check(lib().slr_photo_gn_noalloc(C.byref(s), _ptr(depth), _ptr(query), _ptr(weight), _ptr(pose_qm),
                                      float(huber_k), _ptr(out), _stream()), "slr_photo_gn_noalloc")
    return out[:36].view(6, 6), out[36:42], out[42], out[43]


def adam_step(params, grads, m, v, lr, step, betas=(0.9, 0.999), eps=1e-15):
    """One fused Adam step on a surfel set in place.  params / grads: dicts of
    means [n,3], quats [n,4], log_scales [n,2], logits [n]; m, v: [n,10] FP32
    moments (zero before step 1); lr: dict with one rate per group."""
    n = params["means"].shape[0]
    g = SurfelGrads(_ptr(grads["means"]), _ptr(grads["quats"]), _ptr(grads["log_scales"]), _ptr(grads["logits"]))
    cfg = AdamConfig(float(lr["means"]), float(lr["quats"]), float(lr["log_scales"]), float(lr["logits"]),
                     float(betas[0]), float(betas[1]), float(eps), int(step))
    _check(lib().slr_adam_step(n, _ptr(params["means"]), _ptr(params["quats"]),
                               _ptr(params["log_scales"]), _ptr(params["logits"]), C.byref(g), _ptr(m), _ptr(v),
                               C.byref(cfg), _stream()), "slr_adam_step")


def stage_timer(on):
    _check(lib().slr_stage_timer_enable(1 if on else 0), "slr_stage_timer_enable")


def stage_times():
    """{stage: (ms, launches)} accumulated since the last call (synchronises)."""
    ms = (C.c_double * NUM_STAGES)()
    n = (C.c_int64 * NUM_STAGES)()
    _check(lib().slr_stage_times(ms, n), "slr_stage_times")
    return {STAGES[k]: (ms[k], n[k]) for k in range(NUM_STAGES)}


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, quats, log_scales, logits, xi, T_cw, renderer):
        D, N, O = renderer.forward(means, quats, log_scales, logits, T_cw)
        ctx.save_for_backward(means, quats, log_scales, logits, T_cw)
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.surfel_grad = any(ctx.needs_input_grad[:4])
        return D, N, O

    @staticmethod
    def backward(ctx, gD, gN, gO):
        means, quats, log_scales, logits, T_cw = ctx.saved_tensors
        r = ctx.renderer
        if r.generation != ctx.generation:
            raise RuntimeError("the Renderer rendered again after this render and before its backward: its "
                               "workspace no longer holds this render's binning and per-pixel state (use one "
                               "Renderer per differentiable render in a graph)")
        gD = None if gD is None else gD.contiguous().float()
        gN = None if gN is None else gN.contiguous().float()
        gO = None if gO is None else gO.contiguous().float()
        want_pose = ctx.needs_input_grad[4]
        g, dpose = r.backward(means, quats, log_scales, logits, T_cw, gD, gN, gO,
                              pose_only=not ctx.surfel_grad, want_pose=want_pose)
        if g is None:
            return None, None, None, None, dpose, None, None
        return g["means"], g["quats"], g["log_scales"], g["logits"], (dpose if want_pose else None), None, None


def render(means, quats, log_scales, logits, T_cw, renderer, xi=None):
    """Differentiable render -> (depth [H,W], normal [H,W,3], alpha [H,W]).

    T_cw: float64 [4,4] CUDA tensor (world -> sensor).  xi: optional float64
    [6] CUDA leaf standing for the local pose perturbation delta = (rho; phi)
    of T_wc <- T_wc exp(delta), taken at delta = 0; its .grad is dL/ddelta.
    Raises if xi is not zero.  One Renderer holds the state of its last render
    only: a backward through an earlier render of the same Renderer raises.
    """
    if xi is None:
        xi = torch.zeros(6, dtype=torch.float64, device=means.device)
    elif xi.shape != (6,) or bool((xi != 0).any()):
        # the render is taken at delta = 0: a stepped xi would be silently ignored
        raise ValueError("xi must be a zero [6] tensor (fold a pose step into T_cw and reset xi)")
    return _RenderFn.apply(means, quats, log_scales, logits, xi, T_cw, renderer)

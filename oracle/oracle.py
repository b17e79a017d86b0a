"""ctypes front end of oracle/oracle.c (test infrastructure only).

Every function takes and returns numpy arrays.  Surfel parameters are FP32
(the library's input precision); the oracle promotes them to FP64.  The pose
is T_cw as a 4x4 FP64 matrix.  A sensor is a dict with keys
height, width, fu, cu, fv, cv, near.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB lets the planted-mistake test point the pins at a mutated build.
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

# guard-band flag bits (oracle.c)
FLAG_SUPPORT, FLAG_NEAR, FLAG_AMIN, FLAG_TSTOP, FLAG_CLAMP, FLAG_KEYTIE = 1, 2, 4, 8, 16, 32
# default guard-band widths: support (splat units), near (m), alpha (relative), T-stop (relative).
# Each is >= 20x the FP32 error of the GPU path for that decision: s_hat from
# FP64 dot products rounded to FP32 (~4e-7), the ray range (~1e-7 relative),
# alpha = o G (~2e-6 relative), and transmittance accumulated over up to
# hundreds of contributors (~2e-5 relative).
DEFAULT_GUARD = (1e-5, 1e-5, 5e-5, 1e-3)


class _Sensor(C.Structure):
    _fields_ = [("height", C.c_int32), ("width", C.c_int32), ("fu", C.c_double), ("cu", C.c_double),
                ("fv", C.c_double), ("cv", C.c_double), ("near_m", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.or_camera_matrix.argtypes = [C.c_double] * 4 + [C.c_int32, C.c_int32, P]
        L.or_pixel_basis.argtypes = [P, C.c_int32, C.c_int32, P, P, P]
        L.or_render_pixels.argtypes = [C.c_int64, P, P, P, P, P, P, C.c_int64, P, P, P, P, P, P, P, P]
        L.or_backward_pixels.argtypes = [C.c_int64, P, P, P, P, P, P, C.c_int64, P, P, P, P, P, P, P, P, P, P]
        L.or_render_pixels_mode.argtypes = L.or_render_pixels.argtypes + [C.c_int32]
        L.or_render_variants.argtypes = [C.c_int64, P, P, P, P, P, P, C.c_int64, P, P, C.c_int32, P, P, P, P, P,
                                         C.c_int32]
        L.or_backward_pixels_mode.argtypes = L.or_backward_pixels.argtypes + [C.c_int32]
        L.or_bin.argtypes = [C.c_int64, P, P, P, P, P, P, C.c_int32, C.c_int32, C.c_double, C.c_int32,
                             P, P, P, P, C.c_int64, P, P, P, P]
        L.or_pair_support.argtypes = [P, P, P, C.c_double, P, P, C.c_int32, C.c_int32, P]
        L.or_frames.argtypes = [C.c_int64, P, P, P, P, P, C.c_double, P, P, P]
        L.or_box_exp.argtypes = [C.c_double]
        L.or_box_exp.restype = C.c_double
        L.or_support_radius.argtypes = [C.c_double]
        L.or_support_radius.restype = C.c_double
        for f in ("or_render_pixels", "or_backward_pixels", "or_render_pixels_mode", "or_backward_pixels_mode",
                  "or_render_variants",
                  "or_bin", "or_pair_support", "or_frames"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a, shape, exact=False):
    """Surfel parameters as the oracle's FP64 arrays.  By default they are first
    rounded to FP32, the library's input precision; exact=True keeps FP64."""
    a = np.asarray(a)
    if not exact:
        a = a.astype(np.float32)
    return np.ascontiguousarray(a, dtype=np.float64).reshape(shape)


def _sensor(s):
    return _Sensor(int(s["height"]), int(s["width"]), float(s["fu"]), float(s["cu"]),
                   float(s["fv"]), float(s["cv"]), float(s["near"]))


def _pose12(T):
    T = np.asarray(T, dtype=np.float64)
    return np.ascontiguousarray(np.concatenate([T[:3, :3].reshape(9), T[:3, 3]]))


def _surfels(means, quats, log_scales, logits, exact=False):
    n = int(np.asarray(means).shape[0])
    return (n, _f32(means, (n, 3), exact), _f32(quats, (n, 4), exact), _f32(log_scales, (n, 2), exact),
            _f32(logits, (n,), exact))


def camera_matrix(az_min, az_max, el_min, el_max, H, W):
    """K of Supp. A as (fu, cu, fv, cv)."""
    out = np.zeros(4, np.float64)
    lib().or_camera_matrix(az_min, az_max, el_min, el_max, H, W, _p(out))
    return tuple(float(x) for x in out)


def make_sensor(H, W, az=(-np.pi, np.pi), el=(np.deg2rad(-25.0), np.deg2rad(15.0)), near=0.2):
    fu, cu, fv, cv = camera_matrix(az[0], az[1], el[0], el[1], H, W)
    return dict(height=H, width=W, fu=fu, cu=cu, fv=fv, cv=cv, near=near)


def pixel_basis(sensor, i, j):
    v, hx, hy = (np.zeros(3) for _ in range(3))
    s = _sensor(sensor)
    lib().or_pixel_basis(C.byref(s), int(i), int(j), _p(v), _p(hx), _p(hy))
    return v, hx, hy


def all_pixels(sensor):
    H, W = int(sensor["height"]), int(sensor["width"])
    ii, jj = np.meshgrid(np.arange(H, dtype=np.int32), np.arange(W, dtype=np.int32), indexing="ij")
    return np.ascontiguousarray(np.stack([ii.ravel(), jj.ravel()], 1))


def render_pixels(means, quats, log_scales, logits, T_cw, sensor, pix=None, guard=DEFAULT_GUARD, exact=False,
                  cull=False):
    """Brute-force FP64 render of the listed pixels ([P,2] int32 (row, col); default: all).
    cull=True: the angular-cull mode (identical results, faster on large maps).

    Returns dict of depth [P], normal [P,3], alpha [P], T_final [P], n_contrib [P], flags [P].
    """
    n, m, q, ls, lo = _surfels(means, quats, log_scales, logits, exact)
    if pix is None:
        pix = all_pixels(sensor)
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 2)
    P = pix.shape[0]
    out = dict(depth=np.zeros(P), normal=np.zeros((P, 3)), alpha=np.zeros(P), T_final=np.zeros(P),
               n_contrib=np.zeros(P, np.int32), flags=np.zeros(P, np.int32))
    g = None if guard is None else np.ascontiguousarray(guard, dtype=np.float64)
    s = _sensor(sensor)
    pose = _pose12(T_cw)
    rc = lib().or_render_pixels_mode(n, _p(m), _p(q), _p(ls), _p(lo), _p(pose), C.byref(s), P, _p(pix), _p(g),
                                     _p(out["depth"]), _p(out["normal"]), _p(out["alpha"]), _p(out["T_final"]),
                                     _p(out["n_contrib"]), _p(out["flags"]), 1 if cull else 0)
    if rc != 0:
        raise RuntimeError("or_render_pixels failed")
    return out


def render_variants(means, quats, log_scales, logits, T_cw, sensor, pix, guard=DEFAULT_GUARD, max_flips=4,
                    cull=False, exact=False):
    """Every admissible result of the listed pixels: the decisions whose FP64
    value lies in the guard band of its threshold are taken both ways.

    Returns dict of depth [P,V], normal [P,V,3], alpha [P,V] (V = 2**max_flips;
    slot 0 is the plain render), nvar [P] (filled slots), overflow [P] (the
    pixel needs more than max_flips branches: not all results are listed)."""
    n, m, q, ls, lo = _surfels(means, quats, log_scales, logits, exact)
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 2)
    P = pix.shape[0]
    V = 1 << int(max_flips)
    out = dict(depth=np.zeros((P, V)), normal=np.zeros((P, V, 3)), alpha=np.zeros((P, V)),
               nvar=np.zeros(P, np.int32), overflow=np.zeros(P, np.int32))
    g = np.ascontiguousarray(guard, dtype=np.float64)
    s = _sensor(sensor)
    pose = _pose12(T_cw)
    rc = lib().or_render_variants(n, _p(m), _p(q), _p(ls), _p(lo), _p(pose), C.byref(s), P, _p(pix), _p(g),
                                  int(max_flips), _p(out["depth"]), _p(out["normal"]), _p(out["alpha"]),
                                  _p(out["nvar"]), _p(out["overflow"]), 1 if cull else 0)
    if rc != 0:
        raise RuntimeError("or_render_variants failed")
    return out


def render_image(means, quats, log_scales, logits, T_cw, sensor, guard=DEFAULT_GUARD, exact=False, cull=False):
    H, W = int(sensor["height"]), int(sensor["width"])
    o = render_pixels(means, quats, log_scales, logits, T_cw, sensor, None, guard, exact, cull)
    return dict(depth=o["depth"].reshape(H, W), normal=o["normal"].reshape(H, W, 3),
                alpha=o["alpha"].reshape(H, W), T_final=o["T_final"].reshape(H, W),
                n_contrib=o["n_contrib"].reshape(H, W), flags=o["flags"].reshape(H, W))


def backward_pixels(means, quats, log_scales, logits, T_cw, sensor, pix, dL_dD, dL_dN, dL_dO, exact=False,
                    with_abs=False, cull=False):
    """Analytic FP64 gradients of sum_p (dL_dD D + dL_dN . N + dL_dO O) over the listed pixels.

    Returns dict of means [n,3], quats [n,4], log_scales [n,2], logits [n], pose [6] (rho; phi);
    with_abs adds abs [n,10]: per surfel, sum over pixels of |per-pixel contribution| to each
    raw-parameter gradient (mean 3, quaternion 4, log-scales 2, logit 1).
    """
    n, m, q, ls, lo = _surfels(means, quats, log_scales, logits, exact)
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 2)
    P = pix.shape[0]
    gD = None if dL_dD is None else np.ascontiguousarray(dL_dD, np.float64).reshape(P)
    gN = None if dL_dN is None else np.ascontiguousarray(dL_dN, np.float64).reshape(P, 3)
    gO = None if dL_dO is None else np.ascontiguousarray(dL_dO, np.float64).reshape(P)
    out = dict(means=np.zeros((n, 3)), quats=np.zeros((n, 4)), log_scales=np.zeros((n, 2)),
               logits=np.zeros(n), pose=np.zeros(6))
    if with_abs:
        out["abs"] = np.zeros((n, 10))
    s = _sensor(sensor)
    pose = _pose12(T_cw)
    rc = lib().or_backward_pixels_mode(n, _p(m), _p(q), _p(ls), _p(lo), _p(pose), C.byref(s), P, _p(pix),
                                       _p(gD), _p(gN), _p(gO), _p(out["means"]), _p(out["quats"]),
                                       _p(out["log_scales"]), _p(out["logits"]), _p(out["pose"]),
                                       _p(out.get("abs")), 1 if cull else 0)
    if rc != 0:
        raise RuntimeError("or_backward_pixels failed")
    return out


def bin_surfels(means, quats, log_scales, logits, T_cw, sensor, tile_h=16, tile_w=16, margin=2e-5,
                capacity=None, box_mode=0):
    """Bit-mirror binning: keys, counts, pixel boxes, rects, sorted (tile, id) and tile ranges.
    box_mode 0: the 3-sigma square; 1: the opacity-aware support radius."""
    n, m, q, ls, lo = _surfels(means, quats, log_scales, logits)
    H, W = int(sensor["height"]), int(sensor["width"])
    ntiles = ((H + tile_h - 1) // tile_h) * ((W + tile_w - 1) // tile_w)
    keys = np.zeros(n, np.uint32)
    counts = np.zeros(n, np.int32)
    pixbox = np.zeros((n, 6), np.int32)
    rects = np.zeros((n, 8), np.int32)
    ranges = np.zeros((ntiles, 2), np.int32)
    K = np.zeros(1, np.int64)
    s = _sensor(sensor)
    pose = _pose12(T_cw)
    cap = capacity
    if cap is None:
        rc = lib().or_bin(n, _p(m), _p(q), _p(ls), _p(lo), _p(pose), C.byref(s), tile_h, tile_w, margin, box_mode,
                          _p(keys), _p(counts), _p(pixbox), _p(rects), 0, _p(K), None, None, _p(ranges))
        cap = int(K[0])
    st = np.zeros(max(cap, 1), np.int32)
    sid = np.zeros(max(cap, 1), np.int32)
    rc = lib().or_bin(n, _p(m), _p(q), _p(ls), _p(lo), _p(pose), C.byref(s), tile_h, tile_w, margin, box_mode,
                      _p(keys), _p(counts), _p(pixbox), _p(rects), cap, _p(K), _p(st), _p(sid), _p(ranges))
    if rc < 0:
        raise RuntimeError("or_bin failed")
    k = int(K[0])
    return dict(keys=keys, counts=counts, pixbox=pixbox, rects=rects, K=k, overflow=(rc == 1),
                sorted_tile=st[:k] if rc == 0 else None, sorted_id=sid[:k] if rc == 0 else None,
                ranges=ranges, tiles_x=(W + tile_w - 1) // tile_w, tiles_y=(H + tile_h - 1) // tile_h)


def pair_support(mean, quat, log_scale, logit, T_cw, sensor, i, j):
    """Geometric support test of one (pixel, surfel) pair; returns (bool, s_hat)."""
    mu = _f32(mean, (3,)); q = _f32(quat, (4,)); ls = _f32(log_scale, (2,))
    lg = float(np.float32(logit))
    sh = np.zeros(2)
    s = _sensor(sensor)
    pose = _pose12(T_cw)
    r = lib().or_pair_support(_p(mu), _p(q), _p(ls), C.c_double(lg), _p(pose), C.byref(s),
                              int(i), int(j), _p(sh))
    return bool(r), sh


def frames(means, quats, log_scales, logits, T_cw, near=0.2):
    """Per-surfel (b_alpha, b_beta, b_c, n, o, s_a, s_b) [n,15], key bits [n], valid [n]."""
    n, m, q, ls, lo = _surfels(means, quats, log_scales, logits)
    out = np.zeros((n, 15))
    keys = np.zeros(n, np.uint32)
    valid = np.zeros(n, np.int32)
    pose = _pose12(T_cw)
    lib().or_frames(n, _p(m), _p(q), _p(ls), _p(lo), _p(pose), near, _p(out), _p(keys), _p(valid))
    return out, keys, valid


def box_exp(x):
    return lib().or_box_exp(float(x))


def support_radius(logit):
    """Opacity-aware half-side of the support square (box mode 1), in sigma units."""
    return lib().or_support_radius(float(logit))

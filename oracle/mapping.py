"""Mapping-side image operations of Sec. 3.1 and Sec. 3.3.1-3.3.2, by
definition (FP64 numpy oracle; test infrastructure only -- the product path
never imports it).

cloud_to_range -- the spherical projection of a point cloud (Sec. 3.1, Eq.
    spherical-projection): each point p (sensor frame) goes to
    (u, v) = K psi(p) and lands in the pixel whose cell contains it,
    (i, j) = (floor(v), floor(u)) (pixel centres at (j + 1/2, i + 1/2)); the
    pixel keeps the nearest return (smallest range |p|), 0 where no point
    lands.  The range is |p| = sqrt((x^2 + y^2) + z^2) in FP64 from the FP32
    coordinates, rounded once to FP32.  Points with a non-finite coordinate,
    zero range or outside the image are dropped.

range_normals -- the surface normals N(D) estimated from the gradients of a
    range image (Sec. 3.3.2, L_n): back-project the pixels p = D v, take the
    central differences dx = p(i, j+1) - p(i, j-1), dy = p(i-1, j) - p(i+1, j),
    N = dx x dy / |dx x dy|, turned to face the sensor (N . p(i, j) <= 0).
    Zero on the border rows and columns and where any of the five pixels has
    no return (D <= 0) or the cross product vanishes.

loss_map -- the per-pixel refinement losses of Sec. 3.3.2 on M_v = D_t > 0:
    L = w_d sum |D - D_t| + w_n sum_{N_t != 0} (1 - N . N_t)
        + w_o sum -log(max(O, O_min))
    with rho_d = 1, the estimated normal N_t = N(D) taken as given (its
    pixels without a normal are left out of L_n) and O_min = 1e-6.  Gradients
    w_d sign(D - D_t) (sign decided in FP32), -w_n N_t, and -w_o / O where
    O > O_min (0 below, where the clamp is active).

scale_reg -- the scale cap of Sec. 3.3.2, sign corrected (the printed
    tau_s - max(s) would reward growth): L_s = w_s sum_i max(0, max(s_a, s_b)
    - tau_s), s = exp(log-scales); the gradient w.r.t. the log-scale of the
    larger scale (s_a on a tie) is w_s s_max where s_max > tau_s.
"""
import numpy as np

O_MIN = 1e-6
EDGE_GUARD = 1e-9   # pixels: a point this close to a cell edge may land on either side


def cloud_to_range(points, sensor):
    """Returns (range image [H,W] FP32, ambiguous [H,W] bool: pixels a point
    within EDGE_GUARD of a cell edge could have landed in)."""
    H, W = int(sensor["height"]), int(sensor["width"])
    P = np.asarray(points, np.float32).astype(np.float64).reshape(-1, 3)
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    with np.errstate(invalid="ignore", over="ignore"):
        r64 = np.sqrt((x * x + y * y) + z * z)
        u = sensor["fu"] * np.arctan2(y, x) + sensor["cu"]
        v = sensor["fv"] * np.arctan2(z, np.sqrt(x * x + y * y)) + sensor["cv"]
    ok = np.isfinite(P).all(1) & (r64 > 0) & np.isfinite(u) & np.isfinite(v)
    u, v, r64 = u[ok], v[ok], r64[ok]
    j, i = np.floor(u), np.floor(v)
    inside = (j >= 0) & (j < W) & (i >= 0) & (i < H)
    ji, ii = j[inside].astype(np.int64), i[inside].astype(np.int64)
    D = np.full((H, W), np.inf, np.float32)
    np.minimum.at(D, (ii, ji), r64[inside].astype(np.float32))
    D[np.isinf(D)] = 0.0
    # pixels that a point near a cell edge could reach
    amb = np.zeros((H, W), bool)
    fu_, fv_ = u - np.floor(u), v - np.floor(v)
    near = (np.minimum(fu_, 1 - fu_) < EDGE_GUARD) | (np.minimum(fv_, 1 - fv_) < EDGE_GUARD)
    for uu, vv in zip(u[near], v[near]):
        for a in (np.floor(uu - EDGE_GUARD), np.floor(uu + EDGE_GUARD)):
            for b in (np.floor(vv - EDGE_GUARD), np.floor(vv + EDGE_GUARD)):
                if 0 <= a < W and 0 <= b < H:
                    amb[int(b), int(a)] = True
    return D, amb


def pixel_points(sensor, D):
    H, W = int(sensor["height"]), int(sensor["width"])
    i, j = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    az = (j + 0.5 - sensor["cu"]) / sensor["fu"]
    el = (i + 0.5 - sensor["cv"]) / sensor["fv"]
    v = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], -1)
    return np.asarray(D, np.float64)[..., None] * v


def range_normals(sensor, D):
    """[H, W, 3] unit normals (FP64), zero where undefined."""
    D = np.asarray(D, np.float64)
    H, W = D.shape
    p = pixel_points(sensor, D)
    N = np.zeros((H, W, 3))
    if H < 3 or W < 3:
        return N
    dx = p[1:-1, 2:] - p[1:-1, :-2]
    dy = p[:-2, 1:-1] - p[2:, 1:-1]
    n = np.cross(dx, dy)
    nn = np.linalg.norm(n, axis=-1)
    ok = (D[1:-1, 1:-1] > 0) & (D[1:-1, 2:] > 0) & (D[1:-1, :-2] > 0) & (D[:-2, 1:-1] > 0) & (D[2:, 1:-1] > 0)
    ok &= nn > 0
    n = n / np.where(ok, nn, 1.0)[..., None]
    flip = (n * p[1:-1, 1:-1]).sum(-1) > 0
    n = np.where(flip[..., None], -n, n)
    N[1:-1, 1:-1] = np.where(ok[..., None], n, 0.0)
    return N


def loss_map(D, N, O, Dt, Nt, w_d, w_n, w_o):
    """Returns (L, dL/dD [P], dL/dN [P,3], dL/dO [P]) for flattened images."""
    D = np.asarray(D, np.float32).reshape(-1)
    Dt = np.asarray(Dt, np.float32).reshape(-1)
    O = np.asarray(O, np.float32).reshape(-1)
    N = np.asarray(N, np.float32).reshape(-1, 3)
    Nt = np.asarray(Nt, np.float32).reshape(-1, 3)
    valid = Dt > 0
    has_n = valid & (Nt != 0).any(1)
    r32 = D - Dt
    gD = np.where(valid, np.float32(w_d) * np.sign(r32), np.float32(0)).astype(np.float32)
    gN = np.where(has_n[:, None], -np.float32(w_n) * Nt, np.float32(0)).astype(np.float32)
    O64 = O.astype(np.float64)
    above = O64 > O_MIN
    gO = np.where(valid & above, -w_o / np.where(above, O64, 1.0), 0.0)
    r = D.astype(np.float64) - Dt.astype(np.float64)
    dot = (N.astype(np.float64) * Nt.astype(np.float64)).sum(1)
    L = float((w_d * np.abs(r))[valid].sum() + (w_n * (1.0 - dot))[has_n].sum()
              + (-w_o * np.log(np.maximum(O64, O_MIN)))[valid].sum())
    return L, gD, gN, gO


def scale_reg(log_scales, tau_s, w_s):
    """Returns (L_s, dL/d log_scales [n,2])."""
    ls = np.asarray(log_scales, np.float32).astype(np.float64).reshape(-1, 2)
    s = np.exp(ls)
    first = s[:, 0] >= s[:, 1]
    smax = np.where(first, s[:, 0], s[:, 1])
    over = smax > tau_s
    L = float(w_s * (smax - tau_s)[over].sum())
    g = np.zeros_like(ls)
    g[over & first, 0] = w_s * smax[over & first]
    g[over & ~first, 1] = w_s * smax[over & ~first]
    return L, g


# ---------------------------------------------------------------------------
# Local model initialisation (Sec. 3.3.1): a weight map from the range
# gradients over the valid pixels, weighted sampling of n_d pixels, splats
# back-projected from them with their normals facing the sensor.
#
#   gx = (D(i, j+1) - D(i, j-1)) / 2,  gy = (D(i+1, j) - D(i-1, j)) / 2  (FP32,
#        zero on the border or next to a pixel without a return)
#   weight(u) = 0 where D(u) <= 0 or the caller's mask is 0, else
#               floor(256 (|gx| + |gy|)) + 1 (an integer: 1 on flat ground,
#               more across edges), capped at 2^24
#   cum = inclusive prefix sum of the weights (exact integers)
#   sample k: t = min(floor(U_k total) (FP64), total - 1), the first pixel with cum > t
#   splat: mean = T_wc (D v), normal n = -R_wc v, tangents t_a = normalize(n x
#          e), e = world z unless |n_z| > 0.9 (then world x), t_b = n x t_a,
#          quaternion (w >= 0) of R = (t_a t_b n), both scales D theta_px k
#          (theta_px the larger angular pixel pitch), the given logit.
# ---------------------------------------------------------------------------
WEIGHT_CAP = 1 << 24


def init_weights(D, mask=None):
    D = np.asarray(D, np.float32)
    H, W = D.shape
    m = np.ones((H, W), np.float32) if mask is None else np.asarray(mask, np.float32)
    w = np.zeros((H, W), np.int64)
    valid = (D > 0) & (m != 0)
    gx = np.zeros((H, W), np.float32)
    gy = np.zeros((H, W), np.float32)
    inner = np.zeros((H, W), bool)
    inner[1:-1, 1:-1] = ((D[1:-1, 2:] > 0) & (D[1:-1, :-2] > 0) & (D[2:, 1:-1] > 0) & (D[:-2, 1:-1] > 0))
    half = np.float32(0.5)
    gx[1:-1, 1:-1] = (D[1:-1, 2:] - D[1:-1, :-2]) * half
    gy[1:-1, 1:-1] = (D[2:, 1:-1] - D[:-2, 1:-1]) * half
    g = np.where(inner, np.abs(gx) + np.abs(gy), np.float32(0)).astype(np.float32)
    q = np.floor(g * np.float32(256.0)).astype(np.float64)
    w[valid] = np.minimum(q[valid], WEIGHT_CAP).astype(np.int64) + 1
    return w


def quat_from_rot(R):
    """(w, x, y, z), w >= 0, of a rotation matrix (Shepperd's method)."""
    t = R[0, 0] + R[1, 1] + R[2, 2]
    if t > 0:
        s = 2.0 * np.sqrt(1.0 + t)
        q = np.array([0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s])
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = 2.0 * np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2])
        q = np.array([(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s])
    elif R[1, 1] > R[2, 2]:
        s = 2.0 * np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2])
        q = np.array([(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s])
    else:
        s = 2.0 * np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1])
        q = np.array([(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s])
    return q if q[0] >= 0 else -q


def init_splats(sensor, D, T_cw, uniforms, mask=None, scale_factor=1.0, logit=0.0):
    """Returns dict pixel [n] (-1 when no pixel has weight), means [n,3],
    quats [n,4], log_scales [n,2], logits [n] (FP32) and the weights."""
    D = np.asarray(D, np.float32)
    H, W = D.shape
    w = init_weights(D, mask).reshape(-1)
    cum = np.cumsum(w)
    total = int(cum[-1]) if cum.size else 0
    U = np.asarray(uniforms, np.float64).reshape(-1)
    n = U.size
    out = dict(pixel=np.full(n, -1, np.int32), means=np.zeros((n, 3), np.float32),
               quats=np.zeros((n, 4), np.float32), log_scales=np.zeros((n, 2), np.float32),
               logits=np.zeros(n, np.float32), weights=w.reshape(H, W))
    if total == 0:
        return out
    # U total can round up to total for U within an ulp of 1: the draw stays on the last pixel
    t = np.minimum(np.floor(U * float(total)).astype(np.int64), total - 1)
    idx = np.searchsorted(cum, t, side="right")
    T_cw = np.asarray(T_cw, np.float64)
    Rwc = T_cw[:3, :3].T
    twc = -Rwc @ T_cw[:3, 3]
    pitch = max(abs(1.0 / sensor["fu"]), abs(1.0 / sensor["fv"]))
    for k in range(n):
        p = int(idx[k])
        i, j = divmod(p, W)
        az = (j + 0.5 - sensor["cu"]) / sensor["fu"]
        el = (i + 0.5 - sensor["cv"]) / sensor["fv"]
        v = np.array([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])
        d = float(D[i, j])
        nrm = -(Rwc @ v)
        e = np.array([1.0, 0.0, 0.0]) if abs(nrm[2]) > 0.9 else np.array([0.0, 0.0, 1.0])
        ta = np.cross(nrm, e)
        ta /= np.linalg.norm(ta)
        tb = np.cross(nrm, ta)
        R = np.stack([ta, tb, nrm], 1)
        out["pixel"][k] = p
        out["means"][k] = Rwc @ (d * v) + twc
        out["quats"][k] = quat_from_rot(R)
        out["log_scales"][k] = np.log(d * pitch * scale_factor)
        out["logits"][k] = logit
    return out

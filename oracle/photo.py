"""Photometric registration normal equations between a rendered range image
and a query range image (FP64 oracle; test infrastructure only -- the
product path never imports it).

Sec. 3.3.3 (photometric registration): every pixel u of the rendered range
image D is back-projected with its range, p = phi^-1(u, D(u)) = D(u) v(u)
(Sec. 3.1: v the unit ray of the pixel centre under K of Supp. A), moved into
the query sensor's frame, q = T p, and projected back, u' = phi(q); the
query range image D_q is read there by bilinear interpolation of its pixel
centres.  The residual compares the range of the moved point with the query:

    r_u = |q| - D_q(u')        (= D(u) - D_q(u') at T = I, the printed form)

Pose convention: T maps the render's sensor frame to the query's; the query
frame's pose is updated as T_wq <- T_wq exp(delta), so T(delta) = exp(-delta^) T
and dq/drho = -I, dq/dphi = [q]_x.  With G = dr/dq,

    J_u = (-G, G x q),   G = q/|q| - (dB/dx dx/dq + dB/dy dy/dq)

where B is the bilinear interpolant and (x, y) = (u' - 1/2, v' - 1/2) the
continuous column and row.  A pixel takes part when D(u) > 0, its weight is
non-zero, 0 <= x < W-1, 0 <= y < H-1 and the four query pixels around u' have
a return (> 0).  With the Huber loss (threshold k; k <= 0: least squares) in
IRLS form, w = rho'(r)/r:

    H = sum m w J J^T,  g = sum m w r J,  cost = sum m rho(r),  count.
"""
import numpy as np

from .gn import huber


def pixel_rays(sensor):
    """[H, W, 3] unit rays of the pixel centres (u, v) = (j + 1/2, i + 1/2)."""
    H, W = int(sensor["height"]), int(sensor["width"])
    i, j = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    az = (j + 0.5 - sensor["cu"]) / sensor["fu"]
    el = (i + 0.5 - sensor["cv"]) / sensor["fv"]
    return np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], -1)


def warp(sensor, depth, T):
    """Moved points q [H,W,3] and continuous query coordinates (x, y) of every pixel."""
    p = np.asarray(depth, np.float64)[..., None] * pixel_rays(sensor)
    T = np.asarray(T, np.float64)
    q = p @ T[:3, :3].T + T[:3, 3]
    az = np.arctan2(q[..., 1], q[..., 0])
    el = np.arctan2(q[..., 2], np.hypot(q[..., 0], q[..., 1]))
    x = sensor["fu"] * az + sensor["cu"] - 0.5
    y = sensor["fv"] * el + sensor["cv"] - 0.5
    return q, x, y


def bilinear(img, x, y):
    """Value, d/dx, d/dy of the bilinear interpolant of img at (x, y) (inside
    the grid), and whether all four neighbours are > 0."""
    img = np.asarray(img, np.float64)
    x0 = np.floor(x).astype(np.int64)
    y0 = np.floor(y).astype(np.int64)
    fx, fy = x - x0, y - y0
    a = img[y0, x0]
    b = img[y0, x0 + 1]
    c = img[y0 + 1, x0]
    d = img[y0 + 1, x0 + 1]
    val = (1 - fy) * ((1 - fx) * a + fx * b) + fy * ((1 - fx) * c + fx * d)
    dx = (1 - fy) * (b - a) + fy * (d - c)
    dy = (1 - fx) * (c - a) + fx * (d - b)
    ok = (a > 0) & (b > 0) & (c > 0) & (d > 0)
    return val, dx, dy, ok


def photo_gn(sensor, depth, query, T, weight=None, huber_k=0.0):
    """Normal equations (see the module text).  depth, query, weight: [H, W]
    (weight None = ones); T: 4x4 render-to-query transform.  Returns dict with
    H [6,6], g [6], cost, count and the per-pixel residual, J and validity."""
    Hh, Ww = int(sensor["height"]), int(sensor["width"])
    D = np.asarray(depth, np.float64)
    m = np.ones((Hh, Ww)) if weight is None else np.asarray(weight, np.float64)
    q, x, y = warp(sensor, D, T)
    rq = np.linalg.norm(q, axis=-1)
    inside = (D > 0) & (m != 0) & (rq > 0) & (x >= 0) & (x < Ww - 1) & (y >= 0) & (y < Hh - 1)
    xs, ys = np.where(inside, x, 0.0), np.where(inside, y, 0.0)
    B, Bx, By, ok = bilinear(query, xs, ys)
    valid = inside & ok
    rho2 = q[..., 0] ** 2 + q[..., 1] ** 2
    rhoxy = np.sqrt(rho2)
    safe = np.where(valid, 1.0, 0.0)
    inv_r2 = np.where(valid, 1.0 / np.where(valid, rho2, 1.0), 0.0)
    inv_q2 = np.where(valid, 1.0 / np.where(valid, rq * rq, 1.0), 0.0)
    daz = np.stack([-q[..., 1] * inv_r2, q[..., 0] * inv_r2, np.zeros_like(rq)], -1)
    rx = np.where(valid, rhoxy, 1.0)
    dell = np.stack([-q[..., 0] * q[..., 2] / rx * inv_q2, -q[..., 1] * q[..., 2] / rx * inv_q2, rhoxy * inv_q2], -1)
    qhat = q / np.where(valid, rq, 1.0)[..., None]
    G = qhat - (Bx * sensor["fu"])[..., None] * daz - (By * sensor["fv"])[..., None] * dell
    G = G * safe[..., None]
    J = np.concatenate([-G, np.cross(G, q)], -1).reshape(-1, 6)
    r = np.where(valid, rq - B, 0.0).reshape(-1)
    rho, w = huber(r, huber_k)
    mv = (m * valid).reshape(-1)
    Hm = (J * (mv * w)[:, None]).T @ J
    g = J.T @ (mv * w * r)
    cost = float((mv * rho).sum())
    return dict(H=Hm, g=g, cost=cost, count=int(valid.sum()), residual=r.reshape(Hh, Ww), J=J,
                valid=valid, x=x, y=y)

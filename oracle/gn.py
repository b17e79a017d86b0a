"""Pose-only Gauss-Newton normal equations of a rendered range image (FP64
oracle; test infrastructure only -- the product path never imports it).

Sec. 3.3.3 (frame-to-model registration): the keyframe pose is updated as
T_k^w <- T_k^w exp(delta), delta = (rho; phi) in se(3), by a second-order
Gauss-Newton method on Huber-robust range residuals.  For the rendered range
image D(u) of the map at the pose and a target range image D_t(u), with a
per-pixel weight m_u >= 0:

    r_u   = D(u) - D_t(u)
    J_u   = dD(u)/d delta at delta = 0            (a 6-vector per pixel)
    cost  = sum_u m_u rho(r_u)
    H     = sum_u m_u w(r_u) J_u J_u^T            (6x6, symmetric)
    g     = sum_u m_u w(r_u) r_u J_u = d cost / d delta

where rho is the Huber loss with threshold k (r^2/2 for |r| <= k, k(|r| - k/2)
beyond; k <= 0 means plain least squares, rho = r^2/2) and w(r) = rho'(r)/r
its iteratively-reweighted least-squares weight (1 inside, k/|r| outside).
The Gauss-Newton step solves H delta = -g.

J_u is the oracle's analytic se(3) gradient (Supp. D chain rule, pose part) of
the scalar D(u) alone: backward_pixels on that one pixel with a unit upstream
range gradient.  Parity unpinned beyond what the tests state: J against
finite differences of the forward, g against finite differences of the cost.
"""
import numpy as np

from .oracle import all_pixels, backward_pixels, render_image


def huber(r, k):
    """(rho(r), w(r)) of the Huber loss with threshold k (k <= 0: least squares)."""
    r = np.asarray(r, np.float64)
    if k is None or k <= 0:
        return 0.5 * r * r, np.ones_like(r)
    a = np.abs(r)
    inside = a <= k
    rho = np.where(inside, 0.5 * r * r, k * (a - 0.5 * k))
    w = np.where(inside, 1.0, k / np.where(inside, 1.0, a))
    return rho, w


def pose_jacobian(means, quats, log_scales, logits, T_cw, sensor, pix, exact=False, cull=False):
    """[P, 6] rows dD(u)/d delta (rho; phi) of the listed pixels ([P, 2] (row, col)).
    cull: the oracle's result-identical angular-cull mode (faster on large maps)."""
    pix = np.ascontiguousarray(pix, dtype=np.int32).reshape(-1, 2)
    J = np.zeros((pix.shape[0], 6))
    one = np.ones(1)
    for p in range(pix.shape[0]):
        J[p] = backward_pixels(means, quats, log_scales, logits, T_cw, sensor, pix[p:p + 1], one, None, None,
                               exact=exact, cull=cull)["pose"]
    return J


def pose_gn(means, quats, log_scales, logits, T_cw, sensor, target, weight=None, huber_k=0.0, exact=False,
            cull=False):
    """Normal equations of the pose-only Gauss-Newton step (see the module text).

    target, weight: [H, W] (weight None = all ones).  Returns dict with H [6,6],
    g [6], cost, and the per-pixel depth [H,W], residual [H,W] and J [H*W, 6]
    (rows of zero-weight pixels are left zero).
    """
    Hh, Ww = int(sensor["height"]), int(sensor["width"])
    img = render_image(means, quats, log_scales, logits, T_cw, sensor, exact=exact, cull=cull)
    D = img["depth"].reshape(-1)
    t = np.asarray(target, np.float64).reshape(-1)
    m = np.ones(Hh * Ww) if weight is None else np.asarray(weight, np.float64).reshape(-1)
    r = D - t
    rho, w = huber(r, huber_k)
    sel = np.nonzero(m != 0)[0]
    J = np.zeros((Hh * Ww, 6))
    if sel.size:
        J[sel] = pose_jacobian(means, quats, log_scales, logits, T_cw, sensor, all_pixels(sensor)[sel], exact, cull)
    mw = m * w
    H = (J * mw[:, None]).T @ J
    g = J.T @ (mw * r)
    cost = float((m * rho).sum())
    return dict(H=H, g=g, cost=cost, depth=D.reshape(Hh, Ww), residual=r.reshape(Hh, Ww), J=J,
                flags=img["flags"])

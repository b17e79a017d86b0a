"""Pins of the oracle's pose-only Gauss-Newton normal equations (Sec. 3.3.3).

* The Huber weight against the loss's closed form (value continuity at the
  threshold, w(r) r = rho'(r) by finite differences, least squares for k <= 0).
* Per-pixel Jacobian rows dD(u)/d delta against FP64 central differences of
  the oracle's forward under T_wc <- T_wc exp(delta).
* g against central differences of the cost itself (least squares and Huber).
* The per-pixel rows, weighted and summed, against the oracle's batch pose
  gradient.
* Convergence: Gauss-Newton steps on a registration problem (a room of
  overlapping surfels, target rendered at a known pose) shrink the pose error.
"""
import math

import numpy as np
import pytest

import oracle as O
from tests import helpers as h
from tests import test_oracle_backward as tb


def test_huber_closed_form():
    k = 0.3
    r = np.array([-2.0, -0.31, -0.3, -0.1, 0.0, 0.05, 0.3, 0.29, 1.7])
    rho, w = O.huber(r, k)
    # continuity at |r| = k and the two branches
    lo, _ = O.huber(np.array([k - 1e-12, -k + 1e-12]), k)
    hi, _ = O.huber(np.array([k + 1e-12, -k - 1e-12]), k)
    np.testing.assert_allclose(lo, hi, atol=1e-11)
    np.testing.assert_allclose(rho[np.abs(r) <= k], 0.5 * r[np.abs(r) <= k] ** 2)
    # the IRLS weight times r is the derivative of rho
    e = 1e-7
    d = (O.huber(r + e, k)[0] - O.huber(r - e, k)[0]) / (2 * e)
    np.testing.assert_allclose(w * r, d, rtol=1e-6, atol=1e-9)
    # k <= 0: plain least squares
    rho0, w0 = O.huber(r, 0.0)
    np.testing.assert_allclose(rho0, 0.5 * r * r)
    assert (w0 == 1).all()


def _scene(seed0):
    s, mu, q, ls, lg, T, keep = tb.clean_scene(seed0)
    return s, mu, q, ls, lg, T, keep


@pytest.mark.parametrize("seed0", [100, 300])
def test_jacobian_rows_match_fd(seed0):
    s, mu, q, ls, lg, T, keep = _scene(seed0)
    r0 = O.render_pixels(mu, q, ls, lg, T, s, guard=tb.GUARD_FD, exact=True)
    pix_all = O.all_pixels(s)
    sel = np.nonzero(keep & (r0["n_contrib"] >= 2))[0][:12]
    assert sel.size >= 6
    pix = pix_all[sel]
    J = O.pose_jacobian(mu, q, ls, lg, T, s, pix, exact=True)
    eps = 1e-7
    fd = np.zeros_like(J)
    for e in range(6):
        vals = []
        for sgn in (1, -1):
            d = np.zeros(6)
            d[e] = sgn * eps
            r = O.render_pixels(mu, q, ls, lg, h.perturb_cw(T, d), s, pix=pix, guard=tb.GUARD_FD, exact=True)
            assert (r["flags"] == 0).all()
            vals.append(r["depth"])
        fd[:, e] = (vals[0] - vals[1]) / (2 * eps)
    scale = np.maximum(np.linalg.norm(fd, axis=1), 1e-3)
    err = np.linalg.norm(J - fd, axis=1) / scale
    assert err.max() < 1e-6, (J, fd)
    # the translation rows are not trivially zero and rotation enters too
    assert np.abs(J[:, :3]).max() > 1e-2 and np.abs(J[:, 3:]).max() > 1e-2


@pytest.mark.parametrize("huber_k", [0.0, 0.05])
def test_g_is_the_cost_gradient(huber_k):
    s, mu, q, ls, lg, T, keep = _scene(100)
    g = np.random.default_rng(7)
    r0 = O.render_pixels(mu, q, ls, lg, T, s, guard=tb.GUARD_FD, exact=True)
    target = (r0["depth"] + g.normal(0.0, 0.1, r0["depth"].shape)).reshape(s["height"], s["width"])
    weight = (keep * g.uniform(0.5, 2.0, keep.shape)).reshape(s["height"], s["width"])
    out = O.pose_gn(mu, q, ls, lg, T, s, target, weight, huber_k, exact=True)
    if huber_k > 0:  # both branches of the loss are exercised
        rr = np.abs(out["residual"].reshape(-1)[keep])
        assert (rr > huber_k).sum() >= 3 and (rr <= huber_k).sum() >= 3

    def cost(Tp):
        r = O.render_pixels(mu, q, ls, lg, Tp, s, guard=tb.GUARD_FD, exact=True)
        assert (r["flags"][keep] == 0).all()
        rho, _ = O.huber(r["depth"] - target.reshape(-1), huber_k)
        return (weight.reshape(-1) * rho).sum()

    eps = 1e-7
    fd = np.zeros(6)
    for e in range(6):
        d = np.zeros(6)
        d[e] = eps
        fd[e] = (cost(h.perturb_cw(T, d)) - cost(h.perturb_cw(T, -d))) / (2 * eps)
    assert np.linalg.norm(out["g"] - fd) / max(np.linalg.norm(fd), 1e-6) < 1e-6, (out["g"], fd)
    # H is symmetric positive semidefinite
    Hm = out["H"]
    np.testing.assert_allclose(Hm, Hm.T, rtol=0, atol=1e-12 * np.abs(Hm).max())
    assert np.linalg.eigvalsh(Hm).min() >= -1e-9 * np.abs(Hm).max()


def test_rows_sum_to_batch_pose_gradient():
    s, mu, q, ls, lg, T, keep = _scene(300)
    pix = O.all_pixels(s)
    gD = np.random.default_rng(3).normal(size=pix.shape[0]) * keep
    J = O.pose_jacobian(mu, q, ls, lg, T, s, pix, exact=True)
    whole = O.backward_pixels(mu, q, ls, lg, T, s, pix, gD, None, None, exact=True)["pose"]
    np.testing.assert_allclose(gD @ J, whole, rtol=1e-10, atol=1e-12 * np.abs(whole).max())


def room_scene(spacing=0.5, scale=0.3, size=(10.0, 8.0, 4.0), z0=-1.6, seed=0):
    """Overlapping, nearly opaque surfels on the six faces of a box room around
    the sensor, normals pointing in."""
    g = np.random.default_rng(seed)
    X, Y, Z = size
    mus, qs = [], []

    def face(c0, u, v, n, lu, lv):
        nu, nv = int(round(lu / spacing)), int(round(lv / spacing))
        for a in range(nu + 1):
            for b in range(nv + 1):
                p = c0 + (a * spacing) * u + (b * spacing) * v
                mus.append(p + g.normal(0, 0.01, 3))
                qs.append(h.facing_surfel(p, n, g.uniform(0, 2 * math.pi)))

    x0, y0 = -0.45 * X, -0.4 * Y
    ex, ey, ez = np.eye(3)
    face(np.array([x0, y0, z0]), ex, ey, ez, X, Y)              # floor
    face(np.array([x0, y0, z0 + Z]), ex, ey, -ez, X, Y)         # ceiling
    face(np.array([x0, y0, z0]), ex, ez, ey, X, Z)              # wall y = y0
    face(np.array([x0, y0 + Y, z0]), ex, ez, -ey, X, Z)         # wall y = y0 + Y
    face(np.array([x0, y0, z0]), ey, ez, ex, Y, Z)              # wall x = x0
    face(np.array([x0 + X, y0, z0]), ey, ez, -ex, Y, Z)         # wall x = x0 + X
    n = len(mus)
    return (np.array(mus), np.array(qs), np.full((n, 2), math.log(scale)), np.full(n, 3.0))


def pose_error(T_a, T_b):
    E = T_a @ np.linalg.inv(T_b)
    ang = math.acos(max(-1.0, min(1.0, (np.trace(E[:3, :3]) - 1.0) / 2.0)))
    return np.linalg.norm(E[:3, 3]), ang


def test_gauss_newton_steps_converge():
    s = O.make_sensor(16, 96)
    mu, q, ls, lg = room_scene()
    T_true = np.eye(4)
    target = O.render_image(mu, q, ls, lg, T_true, s, exact=True)
    hit = target["alpha"] > 0.5
    T = h.perturb_cw(T_true, np.array([0.04, -0.03, 0.02, 0.004, -0.006, 0.008]))
    errs = [pose_error(T, T_true)]
    for it in range(3):
        out = O.pose_gn(mu, q, ls, lg, T, s, target["depth"], hit & (target["flags"] == 0), 0.0, exact=True)
        delta = -np.linalg.solve(out["H"], out["g"])
        T = h.perturb_cw(T, delta)
        errs.append(pose_error(T, T_true))
    t_err = [e[0] for e in errs]
    a_err = [e[1] for e in errs]
    assert t_err[1] < 0.3 * t_err[0] and a_err[1] < 0.3 * a_err[0], errs
    assert t_err[-1] < 2e-3 and a_err[-1] < 2e-4, errs

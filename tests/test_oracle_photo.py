"""Pins of the oracle's photometric registration normal equations (Sec. 3.3.3).

* Round trip: with T = I every pixel projects back onto its own centre, so
  the interpolated query is the query pixel and r = D - D_q.
* The bilinear interpolant reproduces an affine image exactly, with its
  slopes as derivatives.
* The projection against numpy's arctan2 form of phi (Sec. 3.1).
* g against central differences of the cost (least squares and Huber) under
  T <- exp(-delta^) T; H symmetric positive semidefinite.
* Gauss-Newton steps from the identity recover the query sensor's pose on a
  room of overlapping surfels rendered from two poses.
"""
import numpy as np
import pytest

import oracle as O
from tests import helpers as h
from tests.test_oracle_gn import pose_error, room_scene


def sensor_small():
    return O.make_sensor(24, 128)


def test_identity_round_trip():
    s = sensor_small()
    g = np.random.default_rng(1)
    D = g.uniform(1.0, 20.0, (24, 128))
    Q = g.uniform(1.0, 20.0, (24, 128))
    q, x, y = O.photo.warp(s, D, np.eye(4))
    ii, jj = np.meshgrid(np.arange(24), np.arange(128), indexing="ij")
    np.testing.assert_allclose(x, jj, atol=1e-9)
    np.testing.assert_allclose(y, ii, atol=1e-9)
    np.testing.assert_allclose(np.linalg.norm(q, axis=-1), D, rtol=1e-14)
    out = O.photo_gn(s, D, Q, np.eye(4))
    inner = (ii < 23) & (jj < 127)
    # pixels whose centre lands a rounding error below the cell start fall in the
    # cell before; everything else reads its own query pixel
    assert out["valid"][inner].mean() > 0.95
    v = out["valid"]
    np.testing.assert_allclose(out["residual"][v], (D - Q)[v], atol=1e-8)


def test_bilinear_reproduces_affine_image():
    g = np.random.default_rng(2)
    a, b, c = 7.0, 0.31, -0.17
    ii, jj = np.meshgrid(np.arange(20), np.arange(50), indexing="ij")
    img = a + b * jj + c * ii
    x = g.uniform(0, 48.999, 200)
    y = g.uniform(0, 18.999, 200)
    val, dx, dy, ok = O.photo.bilinear(img, x, y)
    np.testing.assert_allclose(val, a + b * x + c * y, rtol=1e-13)
    np.testing.assert_allclose(dx, b, rtol=1e-12)
    np.testing.assert_allclose(dy, c, rtol=1e-12)
    assert ok.all()


def test_projection_matches_arctan2_form():
    s = sensor_small()
    g = np.random.default_rng(3)
    T = h.perturb_cw(np.eye(4), g.normal(0, 0.05, 6))
    D = g.uniform(2.0, 30.0, (24, 128))
    q, x, y = O.photo.warp(s, D, T)
    u, v = h.project(s, q)
    np.testing.assert_allclose(x, u - 0.5, atol=1e-9)
    np.testing.assert_allclose(y, v - 0.5, atol=1e-9)


def two_views(sensor, delta_q):
    mu, q, ls, lg = room_scene()
    D = O.render_image(mu, q, ls, lg, np.eye(4), sensor, exact=True)["depth"]
    Tq = h.perturb_cw(np.eye(4), np.asarray(delta_q, np.float64))   # T_cw of the query sensor
    Dq = O.render_image(mu, q, ls, lg, Tq, sensor, exact=True)["depth"]
    return D, Dq, Tq


@pytest.mark.parametrize("huber_k", [0.0, 0.02])
def test_g_is_the_cost_gradient(huber_k):
    s = sensor_small()
    D, Dq, Tq = two_views(s, [0.05, -0.04, 0.02, 0.01, -0.01, 0.02])
    T = h.perturb_cw(np.eye(4), np.array([0.02, 0.01, -0.01, 0.004, 0.003, -0.005]))
    wgt = np.random.default_rng(4).uniform(0.5, 1.5, D.shape)
    out = O.photo_gn(s, D, Dq, T, wgt, huber_k)
    assert out["count"] > 0.5 * D.size
    if huber_k > 0:
        rr = np.abs(out["residual"][out["valid"]])
        assert (rr > huber_k).sum() > 20 and (rr <= huber_k).sum() > 20

    def cost(Tp):
        o = O.photo_gn(s, D, Dq, Tp, wgt, huber_k)
        assert o["count"] == out["count"]
        return o["cost"]

    eps = 1e-7
    fd = np.zeros(6)
    for e in range(6):
        d = np.zeros(6)
        d[e] = eps
        fd[e] = (cost(h.perturb_cw(T, d)) - cost(h.perturb_cw(T, -d))) / (2 * eps)
    assert np.linalg.norm(out["g"] - fd) <= 1e-5 * np.linalg.norm(fd), (out["g"], fd)
    Hm = out["H"]
    np.testing.assert_allclose(Hm, Hm.T, rtol=0, atol=1e-12 * np.abs(Hm).max())
    assert np.linalg.eigvalsh(Hm).min() >= -1e-9 * np.abs(Hm).max()


def test_gauss_newton_recovers_query_pose():
    s = O.make_sensor(32, 192)
    D, Dq, Tq = two_views(s, [0.06, -0.05, 0.03, 0.01, -0.015, 0.02])
    T = np.eye(4)
    errs = [pose_error(T, Tq)]
    for it in range(6):
        out = O.photo_gn(s, D, Dq, T, None, 0.0)
        delta = -np.linalg.solve(out["H"], out["g"])
        T = h.perturb_cw(T, delta)
        errs.append(pose_error(T, Tq))
    assert errs[1][0] < 0.5 * errs[0][0] and errs[1][1] < 0.5 * errs[0][1], errs
    assert errs[-1][0] < 5e-3 and errs[-1][1] < 1e-3, errs

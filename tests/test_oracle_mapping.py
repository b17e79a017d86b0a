"""Pins of the oracle's mapping-side image operations (Sec. 3.1, 3.3.1-3.3.2).

* cloud_to_range: points back-projected from pixel centres at known ranges
  (textbook rays of tests/helpers) come back as that range image; the nearest
  of several returns is kept; invalid and out-of-view points are dropped; the
  seam azimuths land in the first and last columns.
* range_normals: a sphere around the sensor gives N = -v exactly (central
  differences are symmetric), a plane gives its own normal facing the sensor;
  borders and pixels next to a missing return are zero.
* loss_map: finite differences in D, N, O; a two-pixel case worked by hand.
* scale_reg: closed form and finite differences.
"""
import math

import numpy as np

import oracle as O
from tests import helpers as h


def sensor():
    return O.make_sensor(16, 64)


def test_cloud_round_trip_and_nearest_return():
    s = sensor()
    g = np.random.default_rng(1)
    ii, jj = np.meshgrid(np.arange(16), np.arange(64), indexing="ij")
    Dt = g.uniform(1.0, 50.0, (16, 64)).astype(np.float32)
    keep = g.uniform(size=(16, 64)) < 0.8
    P = (Dt[..., None].astype(np.float64) * h.ray_dir(s, ii, jj))[keep]
    # farther duplicates of some pixels: the nearest return stays
    far = P[:100] * 1.5
    # invalid points: non-finite, the origin, below the field of view
    bad = np.array([[np.nan, 1, 1], [0, 0, 0], [1.0, 0.0, -5.0], [np.inf, 0, 0]])
    D, amb = O.mapping.cloud_to_range(np.concatenate([far, P, bad]).astype(np.float32), s)
    assert not amb.any()
    want = np.where(keep, Dt, 0.0).astype(np.float32)
    # the FP32 point coordinates move the range by an ulp or so
    np.testing.assert_allclose(D, want, rtol=3e-7)
    assert ((D > 0) == keep).all()


def test_cloud_seam_columns():
    s = O.make_sensor(16, 64)
    el = ((7 + 0.5) - s["cv"]) / s["fv"]
    pts = np.array([[-math.cos(el), 0.0, math.sin(el)],            # az = +pi
                    [-math.cos(el), -1e-9, math.sin(el)]]) * 10.0  # az just above -pi
    D, amb = O.mapping.cloud_to_range(pts.astype(np.float32), s)
    assert D[7, 0] > 0 and D[7, 63] > 0 and (D > 0).sum() == 2


def test_normals_sphere_and_plane():
    s = sensor()
    N = O.mapping.range_normals(s, np.full((16, 64), 7.0))
    ii, jj = np.meshgrid(np.arange(16), np.arange(64), indexing="ij")
    v = h.ray_dir(s, ii, jj)
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(N[inner], -v[inner], atol=1e-12)
    assert not N[0].any() and not N[-1].any() and not N[:, 0].any() and not N[:, -1].any()
    # the ground plane z = -1.8: D = -1.8 / v_z where the ray points down
    Dp = np.where(v[..., 2] < -1e-3, -1.8 / np.where(v[..., 2] < -1e-3, v[..., 2], -1.0), 0.0)
    Np = O.mapping.range_normals(s, Dp)
    ok = (Np != 0).any(-1)
    assert ok.sum() > 100
    np.testing.assert_allclose(Np[ok], np.tile([0.0, 0.0, 1.0], (ok.sum(), 1)), atol=1e-9)
    # a missing return clears its four neighbours' normals
    Dh = np.full((16, 64), 7.0)
    Dh[8, 30] = 0.0
    Nh = O.mapping.range_normals(s, Dh)
    for (a, b) in ((8, 30), (7, 30), (9, 30), (8, 29), (8, 31)):
        assert not Nh[a, b].any()
    assert Nh[8, 28].any() and Nh[6, 30].any()


def test_loss_map_fd_and_hand_case():
    g = np.random.default_rng(2)
    P = 40
    D = g.uniform(1, 10, P).astype(np.float32)
    Dt = (D + g.normal(0, 0.3, P)).astype(np.float32)
    Dt[:5] = 0.0
    N = g.normal(size=(P, 3)).astype(np.float32)
    Nt = g.normal(size=(P, 3)).astype(np.float32)
    Nt[5:8] = 0.0
    Oo = g.uniform(0.05, 0.99, P).astype(np.float32)
    w = (0.7, 0.4, 0.2)
    L, gD, gN, gO = O.mapping.loss_map(D, N, Oo, Dt, Nt, *w)

    def f(D_, N_, O_):
        return O.mapping.loss_map(D_, N_, O_, Dt, Nt, *w)[0]

    e = 2.0 ** -10   # exact when added to these FP32 values, the images' precision
    for k in range(8, 14):
        d = np.zeros(P, np.float64)
        d[k] = e
        fd = (f(D + d, N, Oo) - f(D - d, N, Oo)) / (2 * e)
        assert abs(fd - gD[k]) < 1e-6
        fo = (f(D, N, Oo + d) - f(D, N, Oo - d)) / (2 * e)
        assert abs(fo - gO[k]) < 1e-3 * abs(gO[k])
        for c in range(3):
            dn = np.zeros((P, 3))
            dn[k, c] = e
            fn = (f(D, N + dn, Oo) - f(D, N - dn, Oo)) / (2 * e)
            assert abs(fn - gN[k, c]) < 1e-6
    assert not gD[:5].any() and not gO[:5].any() and not gN[5:8].any()
    # two pixels by hand
    L2, d2, n2, o2 = O.mapping.loss_map([2.0, 3.0], [[0, 0, 1], [1, 0, 0]], [0.5, 1e-8], [1.5, 3.5],
                                        [[0, 0, 1], [0, 0, 0]], 1.0, 2.0, 3.0)
    want = 0.5 + 0.5 + 2.0 * (1 - 1) + 3.0 * (-math.log(0.5) - math.log(1e-6))
    assert abs(L2 - want) < 1e-9
    assert list(d2) == [1.0, -1.0] and abs(o2[0] + 6.0) < 1e-12 and o2[1] == 0.0
    assert list(n2[0]) == [0, 0, -2.0] and not n2[1].any()


def test_scale_reg_closed_form_and_fd():
    ls = np.log(np.array([[0.2, 0.1], [0.3, 0.6], [0.05, 0.05], [1.0, 1.0]], np.float32))
    L, g = O.mapping.scale_reg(ls, 0.25, 2.0)
    assert abs(L - 2.0 * ((0.6 - 0.25) + (1.0 - 0.25))) < 1e-6
    assert g[0].tolist() == [0, 0] and g[2].tolist() == [0, 0]
    assert abs(g[1, 1] - 1.2) < 1e-6 and g[1, 0] == 0 and abs(g[3, 0] - 2.0) < 1e-6 and g[3, 1] == 0
    e = 2.0 ** -12   # exact when added to the FP32 log-scales
    for k, c in ((1, 1), (3, 0), (0, 0)):
        d = np.zeros_like(ls, dtype=np.float64)
        d[k, c] = e
        fd = (O.mapping.scale_reg(ls + d, 0.25, 2.0)[0] - O.mapping.scale_reg(ls - d, 0.25, 2.0)[0]) / (2 * e)
        if k != 3:  # the tie at [3] has a kink
            assert abs(fd - g[k, c]) < 1e-5, (k, c, fd, g[k, c])


def test_init_weights_on_a_ramp():
    ii, jj = np.meshgrid(np.arange(10), np.arange(20), indexing="ij")
    D = (5.0 + 0.125 * jj).astype(np.float32)          # gx = 0.125 exactly, gy = 0
    D[4, 7] = 0.0
    w = O.mapping.init_weights(D)
    assert w[4, 7] == 0
    # interior pixels away from the hole: floor(256 * 0.125) + 1 = 33; border and next to the hole: 1
    assert w[2, 2] == 33 and w[0, 5] == 1 and w[9, 5] == 1 and w[5, 0] == 1 and w[5, 19] == 1
    assert w[4, 6] == 1 and w[4, 8] == 1 and w[3, 7] == 1 and w[5, 7] == 1
    mask = np.ones_like(D)
    mask[:, :10] = 0
    wm = O.mapping.init_weights(D, mask)
    assert not wm[:, :10].any() and (wm[:, 11:19][1:-1] == 33).all()


def test_init_sampling_by_brute_force_and_frequency():
    s = O.make_sensor(12, 40)
    g = np.random.default_rng(5)
    D = g.uniform(2.0, 10.0, (12, 40)).astype(np.float32)
    D[g.uniform(size=D.shape) < 0.2] = 0.0
    U = g.uniform(size=4000)
    out = O.mapping.init_splats(s, D, np.eye(4), U)
    w = out["weights"].reshape(-1)
    total = int(w.sum())
    for k in range(200):   # brute force: the pixel whose interval holds floor(U total)
        t = int(np.floor(U[k] * total))
        acc = 0
        for p, wp in enumerate(w):
            if acc <= t < acc + wp:
                break
            acc += wp
        assert out["pixel"][k] == p
    freq = np.bincount(out["pixel"], minlength=w.size)
    expect = U.size * w / total
    big = expect > 20
    assert np.abs(freq[big] - expect[big]).max() < 5 * np.sqrt(expect[big]).max()
    assert (freq[w == 0] == 0).all()


def test_init_splats_geometry():
    s = O.make_sensor(12, 40)
    g = np.random.default_rng(6)
    D = g.uniform(2.0, 10.0, (12, 40)).astype(np.float32)
    T_cw = h.perturb_cw(np.eye(4), np.array([0.5, -0.2, 0.1, 0.1, -0.2, 0.3]))
    out = O.mapping.init_splats(s, D, T_cw, g.uniform(size=300), scale_factor=1.5, logit=-0.5)
    Twc = np.linalg.inv(T_cw)
    pitch = max(abs(1 / s["fu"]), abs(1 / s["fv"]))
    for k in range(300):
        p = out["pixel"][k]
        i, j = divmod(int(p), 40)
        mu = out["means"][k].astype(np.float64)
        ps = T_cw[:3, :3] @ mu + T_cw[:3, 3]                 # back in the sensor frame
        u, v = h.project(s, ps)
        assert abs(u - (j + 0.5)) < 1e-4 and abs(v - (i + 0.5)) < 1e-4
        assert abs(np.linalg.norm(ps) - D[i, j]) < 1e-5 * D[i, j]
        q = out["quats"][k].astype(np.float64)
        assert abs(np.linalg.norm(q) - 1) < 1e-6 and q[0] >= 0
        R = h.rot_from_quat_wxyz(q)
        n = R[:, 2]
        assert np.dot(n, mu - Twc[:3, 3]) < 0                  # faces the sensor
        np.testing.assert_allclose(n, -(Twc[:3, :3] @ h.ray_dir(s, i, j)), atol=1e-6)
        np.testing.assert_allclose(out["log_scales"][k], math.log(float(D[i, j]) * pitch * 1.5), rtol=1e-6,
                                   atol=1e-7)
        assert out["logits"][k] == np.float32(-0.5)
    last = O.mapping.init_splats(s, D, T_cw, [np.nextafter(1.0, 0.0)])
    assert last["pixel"][0] == 12 * 40 - 1
    empty = O.mapping.init_splats(s, np.zeros((12, 40), np.float32), T_cw, [0.3, 0.7])
    assert (empty["pixel"] == -1).all() and not empty["means"].any()

"""Pins of the oracle's guard-band variants (or_render_variants).

A decision whose FP64 value lies within rounding distance of its threshold
may be taken either way by an FP32 evaluation; the variants are the results
with each such decision taken both ways.  Pinned by: slot 0 equal to the
plain render bit for bit with a single result wherever the plain render
flags nothing; and closed forms of one-decision cases built on the
fronto-parallel surfel (Sec. 3.2.1 blending, Eqs. ab_depth / ab_opacity):
a pixel ray meeting the 3-sigma square exactly on its edge (the textbook
ray-plane solve gives s_hat), a surfel of opacity 1/255 (1 + 1e-7), and a
list whose stop test lands 1e-6 above T = 1e-4."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2503_17491_amd import synth
from tests import helpers as h
from tests.test_oracle_bin import adversarial_scene

EXCL = O.FLAG_SUPPORT | O.FLAG_NEAR | O.FLAG_AMIN | O.FLAG_TSTOP


@pytest.mark.parametrize("mk,mkT,hw", [
    (lambda: synth.shell_scene(3000, 1), lambda: np.eye(4), (64, 512)),
    (lambda: synth.structured_scene(30000, 3)[0], lambda: synth.circle_poses(8, 1)[2], (64, 512)),
    (adversarial_scene, lambda: np.eye(4), (32, 256)),
])
def test_variant_zero_is_the_plain_render(mk, mkT, hw):
    sc, T = mk(), mkT()
    s = O.make_sensor(*hw)
    pix = O.all_pixels(s)
    a = O.render_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, s, pix)
    v = O.render_variants(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, s, pix, max_flips=3)
    np.testing.assert_array_equal(v["depth"][:, 0], a["depth"])
    np.testing.assert_array_equal(v["alpha"][:, 0], a["alpha"])
    np.testing.assert_array_equal(v["normal"][:, 0], a["normal"])
    clean = (a["flags"] & EXCL) == 0
    assert (v["nvar"][clean] == 1).all() and (v["overflow"][clean] == 0).all()
    assert (v["nvar"] >= 1).all()
    # the culled form lists the same variants
    c = O.render_variants(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, s, pix, max_flips=3, cull=True)
    for k in ("depth", "alpha", "normal", "nvar", "overflow"):
        np.testing.assert_array_equal(c[k], v[k])


def _sets(v, q):
    n = int(v["nvar"][q])
    return sorted((float(v["depth"][q, k]), float(v["alpha"][q, k])) for k in range(n))


def test_support_edge_both_ways():
    """A fronto-parallel surfel centred on pixel (30, 200) at 10 m, scaled so
    that the ray of pixel (30, 205) meets its plane exactly on the edge of the
    3-sigma square: that pixel has two admissible results, nothing, or the
    pair with alpha = o exp(-|s_hat|^2 / 2) at the ray-plane range."""
    s = O.make_sensor(64, 512)
    i, j, jj, d, o = 30, 200, 205, 10.0, 0.9
    v = h.ray_dir(s, i, j)
    q = h.facing_surfel(d * v, -v, 0.2)
    w = h.ray_dir(s, i, jj)
    sh1, _ = h.ray_plane_shat(*h.sensor_frame_vectors(d * v, q, np.log([1.0, 1.0]), 0.0, np.eye(4))[:4], w)
    scale = max(abs(sh1[0]), abs(sh1[1])) / 3.0          # |s_hat| = 3 on the edge
    ls = np.log([scale, scale])
    ba, bb, bc, n, _, _ = h.sensor_frame_vectors(d * v, q, ls, 0.0, np.eye(4))
    sh, t = h.ray_plane_shat(ba, bb, bc, n, w)
    assert abs(max(abs(sh[0]), abs(sh[1])) - 3.0) < 1e-9
    alpha = o * math.exp(-0.5 * (sh[0] ** 2 + sh[1] ** 2))
    assert alpha > 1.0 / 255.0
    lg = math.log(o / (1 - o))
    r = O.render_variants((d * v)[None], q[None], ls[None], [lg], np.eye(4), s, [[i, jj]], exact=True)
    assert r["nvar"][0] == 2 and r["overflow"][0] == 0
    got = _sets(r, 0)
    assert got[0] == (0.0, 0.0)
    assert got[1][1] == pytest.approx(alpha, rel=1e-9)
    assert got[1][0] == pytest.approx(alpha * t, rel=1e-9)       # the range |nu| = t along the unit ray


def test_alpha_floor_both_ways():
    """A surfel of opacity (1/255)(1 + 1e-7) at its centre pixel: alpha sits on
    the 1/255 floor, so it contributes (D = o d, O = o) or not."""
    s = O.make_sensor(64, 512)
    i, j, d = 20, 100, 7.0
    o = (1.0 / 255.0) * (1.0 + 1e-7)
    v = h.ray_dir(s, i, j)
    q = h.facing_surfel(d * v, -v, 0.3)
    r = O.render_variants((d * v)[None], q[None], np.log([[0.3, 0.2]]), [math.log(o / (1 - o))], np.eye(4), s,
                          [[i, j]], exact=True)
    assert r["nvar"][0] == 2 and r["overflow"][0] == 0
    got = _sets(r, 0)
    assert got[0] == (0.0, 0.0)
    assert got[1][1] == pytest.approx(o, rel=1e-12)
    assert got[1][0] == pytest.approx(o * d, rel=1e-12)


def test_stop_rule_both_ways():
    """Four fronto-parallel surfels on one ray, opacities 0.95, 0.95, o3, 0.5 with
    0.0025 (1 - o3) = 1e-4 (1 + 1e-6): the stop test before the third lands in
    the guard band.  Either the list stops after two (D = 0.95*4 + 0.05*0.95*6)
    or the third is blended as well (+ 0.0025 o3 8); the fourth always stops."""
    s = O.make_sensor(64, 512)
    i, j = 30, 200
    o3 = 1.0 - 0.04 * (1.0 + 1e-6)
    ops, ds = [0.95, 0.95, o3, 0.5], [4.0, 6.0, 8.0, 10.0]
    v = h.ray_dir(s, i, j)
    mus = np.stack([d * v for d in ds])
    qs = np.stack([h.facing_surfel(d * v, -v, d) for d in ds])
    lss = np.log(np.full((4, 2), 0.3))
    lg = [math.log(o / (1 - o)) for o in ops]
    r = O.render_variants(mus, qs, lss, lg, np.eye(4), s, [[i, j]], exact=True)
    assert r["nvar"][0] == 2 and r["overflow"][0] == 0
    two = (0.95 * 4 + 0.05 * 0.95 * 6, 0.95 + 0.05 * 0.95)
    three = (two[0] + 0.0025 * o3 * 8, two[1] + 0.0025 * o3)
    got = _sets(r, 0)
    assert got[0][0] == pytest.approx(two[0], rel=1e-12) and got[0][1] == pytest.approx(two[1], rel=1e-12)
    assert got[1][0] == pytest.approx(three[0], rel=1e-12) and got[1][1] == pytest.approx(three[1], rel=1e-12)
    # slot 0 is the plain render: the stop test passes (T stays above 1e-4), so the third is blended
    assert r["depth"][0, 0] == pytest.approx(three[0], rel=1e-12)


def test_branch_limit_reports_overflow():
    """With no branch allowed a flagged pixel reports overflow and lists only
    the plain render."""
    s = O.make_sensor(64, 512)
    i, j, d = 20, 100, 7.0
    o = (1.0 / 255.0) * (1.0 + 1e-7)
    v = h.ray_dir(s, i, j)
    q = h.facing_surfel(d * v, -v, 0.3)
    r = O.render_variants((d * v)[None], q[None], np.log([[0.3, 0.2]]), [math.log(o / (1 - o))], np.eye(4), s,
                          [[i, j]], max_flips=0, exact=True)
    assert r["nvar"][0] == 1 and r["overflow"][0] == 1

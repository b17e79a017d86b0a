"""The oracle's angular-cull mode against its own brute force.

The cull skips a (pixel, surfel) pair only when the line of the pixel ray
misses the bounding sphere of the surfel's 3-sigma square (a pair whose
support test must fail), found through azimuth x elevation bins of the
spheres' cones.  It must give the brute-force result bit for bit: every
output, the per-pixel state and the guard-band flags; the backward agrees to
the rounding of its order-dependent FP64 sums.  Scenes: a shell, a posed
structured scene, the adversarial scene of the box pins (seam, pierced z-axis,
near-sensor, grazing, huge surfels), surfels straddling the sensor's vertical
axis at both poles of the direction sphere, and a sensor with a zero near
range (intersections behind the sensor are tested as well)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2503_17491_amd import synth
from tests import helpers as h
from tests.test_oracle_bin import adversarial_scene


def polar_scene():
    """Surfels straight above and below the sensor and some whose bounding
    sphere holds the sensor: their cones reach the poles or cover every
    direction."""
    g = np.random.default_rng(31)
    mus, qs, lss = [], [], []
    for k in range(60):
        z = g.choice([-1.0, 1.0]) * g.uniform(0.5, 12.0)
        mu = np.array([g.normal(scale=0.3), g.normal(scale=0.3), z])
        mus.append(mu)
        qs.append(h.facing_surfel(mu, g.normal(size=3), g.uniform(0, 6.3)))
        lss.append(np.log(g.uniform(0.1, 3.0, 2)))
    for k in range(20):
        d = g.normal(size=3)
        d /= np.linalg.norm(d)
        mu = d * g.uniform(0.3, 2.0)
        mus.append(mu)
        qs.append(h.facing_surfel(mu, g.normal(size=3), g.uniform(0, 6.3)))
        lss.append(np.log(g.uniform(1.0, 4.0, 2)))
    n = len(mus)
    return dict(means=np.array(mus, np.float32), quats=np.array(qs, np.float32),
                log_scales=np.array(lss, np.float32), logits=g.normal(size=n).astype(np.float32))


CASES = [
    ("shell-3k-64x512", lambda: synth.shell_scene(3000, 1), lambda: np.eye(4), (64, 512), 0.2),
    ("structured-20k-posed-64x512", lambda: synth.structured_scene(20000, 5)[0], lambda: synth.circle_poses(8, 1)[2],
     (64, 512), 0.2),
    ("adversarial-32x256", adversarial_scene, lambda: np.eye(4), (32, 256), 0.2),
    ("polar-32x256-near0", polar_scene, lambda: synth.perturbed_pose(5, 0.2, 20.0), (32, 256), 0.0),
]


@pytest.mark.parametrize("name,mk,mkT,hw,near", CASES, ids=[c[0] for c in CASES])
def test_cull_forward_identical(name, mk, mkT, hw, near):
    sc, T = mk(), mkT()
    s = O.make_sensor(*hw, near=near)
    a = O.render_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, s)
    b = O.render_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, s, cull=True)
    assert (a["n_contrib"] > 0).sum() > 100
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("name,mk,mkT,hw,near", CASES[1:], ids=[c[0] for c in CASES[1:]])
def test_cull_backward_identical(name, mk, mkT, hw, near):
    sc, T = mk(), mkT()
    s = O.make_sensor(*hw, near=near)
    pix = O.all_pixels(s)
    g = np.random.default_rng(4)
    P = len(pix)
    gD, gN, gO = g.normal(size=P), g.normal(size=(P, 3)), g.normal(size=P)
    a = O.backward_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, s, pix, gD, gN, gO)
    b = O.backward_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, s, pix, gD, gN, gO, cull=True)
    for k in a:
        scale = float(np.abs(a[k]).max())
        assert scale > 0, k
        np.testing.assert_allclose(b[k], a[k], rtol=1e-10, atol=1e-12 * scale, err_msg=k)

"""GPU parity of the photometric registration normal equations (slr_photo_gn,
Sec. 3.3.3) through the C ABI.

Both sides compute in FP64 from the same FP32 images, so H, g and the cost
agree to 1e-6 of their size on the room case (40x136, ragged) and to 1e-4 at
the benchmark's image size (128x1024 ray-cast images of the structured
scene), where a pixel landing within rounding distance of a cell edge may
read a different cell; the number of pixels taken must agree to 2.
Properties: zero residual at the identity against itself, zero output for an
empty image, repeatability, and Gauss-Newton recovery of the query pose.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2503_17491_amd import synth, targets
from tests import helpers as h
from tests.test_oracle_gn import pose_error, room_scene

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print("[gpu-photo]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def slr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_17491_amd import slr as S
    S.lib()
    return S


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(DEV)


def gpu_photo(S, sensor, D, Q, T, W=None, k=0.0):
    Hm, g, c, n = S.photo_gn(sensor, dev32(D), dev32(Q), dev64(T), None if W is None else dev32(W), k)
    torch.cuda.synchronize()
    return Hm.cpu().numpy(), g.cpu().numpy(), float(c.cpu()), int(n.cpu())


def room_views(sensor, delta_q):
    mu, q, ls, lg = room_scene()
    D = O.render_image(mu, q, ls, lg, np.eye(4), sensor, exact=True)["depth"].astype(np.float32)
    Tq = h.perturb_cw(np.eye(4), np.asarray(delta_q, np.float64))
    Dq = O.render_image(mu, q, ls, lg, Tq, sensor, exact=True)["depth"].astype(np.float32)
    return D, Dq, Tq


def check(S, sensor, D, Q, T, W, k, tol, count_slack):
    Hm, g, c, n = gpu_photo(S, sensor, D, Q, T, W, k)
    ref = O.photo_gn(sensor, D.astype(np.float64), Q.astype(np.float64), T,
                     None if W is None else np.asarray(W, np.float32).astype(np.float64), k)
    np.testing.assert_array_equal(Hm, Hm.T)
    assert abs(n - ref["count"]) <= count_slack, (n, ref["count"])
    assert np.abs(Hm - ref["H"]).max() <= tol * np.abs(ref["H"]).max(), (Hm, ref["H"])
    assert np.linalg.norm(g - ref["g"]) <= tol * np.linalg.norm(ref["g"]), (g, ref["g"])
    assert abs(c - ref["cost"]) <= tol * ref["cost"], (c, ref["cost"])
    return ref


@pytest.mark.parametrize("k", [0.0, 0.02])
@pytest.mark.parametrize("weighted", [False, True])
def test_photo_matches_oracle_room(slr, k, weighted):
    sensor = O.make_sensor(40, 136)
    D, Dq, Tq = room_views(sensor, [0.05, -0.04, 0.02, 0.01, -0.01, 0.02])
    T = h.perturb_cw(np.eye(4), np.array([0.02, 0.01, -0.01, 0.004, 0.003, -0.005]))
    W = np.random.default_rng(9).uniform(0.0, 2.0, D.shape) if weighted else None
    say("room 40x136 huber", k, "weighted", weighted)
    ref = check(slr, sensor, D, Dq, T, W, k, 1e-6, 0)
    assert ref["count"] > 0.5 * D.size


@pytest.mark.parametrize("k", [0.0, 0.1])
def test_photo_matches_oracle_fullsize(slr, k):
    sc, prims = synth.structured_scene(1000, 0)
    sensor = slr.make_sensor(128, 1024)
    TA = synth.circle_poses(8, 0)[0]
    TB = h.perturb_cw(TA, np.array([0.05, -0.04, 0.02, 0.004, -0.006, 0.008]))
    DA, _ = targets.raycast(prims, sensor, TA, seed=1)
    DB, _ = targets.raycast(prims, sensor, TB, seed=2)
    T = h.perturb_cw(np.eye(4), np.array([0.01, 0.02, -0.01, 0.002, -0.001, 0.003]))
    say("fullsize 128x1024 huber", k)
    ref = check(slr, sensor, DA, DB, T, None, k, 1e-4, 2)
    assert ref["count"] > 0.5 * DA.size


def test_photo_identity_and_degenerate(slr):
    sensor = slr.make_sensor(64, 512)
    sc, prims = synth.structured_scene(1000, 0)
    D, _ = targets.raycast(prims, sensor, synth.circle_poses(8, 0)[1], seed=3)
    say("identity, empty, repeat")
    Hm, g, c, n = gpu_photo(slr, sensor, D, D, np.eye(4))
    assert n > 0.5 * D.size
    assert np.linalg.norm(g) <= 1e-9 * np.abs(Hm).max() and c <= 1e-12 * n
    z = np.zeros_like(D)
    Hz, gz, cz, nz = gpu_photo(slr, sensor, z, D, np.eye(4))
    assert nz == 0 and cz == 0.0 and not Hz.any() and not gz.any()
    T = h.perturb_cw(np.eye(4), np.array([0.03, 0.0, 0.01, 0.0, 0.002, 0.0]))
    a = gpu_photo(slr, sensor, D, D, T, None, 0.1)
    b = gpu_photo(slr, sensor, D, D, T, None, 0.1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2] and a[3] == b[3]


def test_photo_gauss_newton_recovers_query_pose(slr):
    sensor = O.make_sensor(32, 192)
    D, Dq, Tq = room_views(sensor, [0.06, -0.05, 0.03, 0.01, -0.015, 0.02])
    T = np.eye(4)
    errs = [pose_error(T, Tq)]
    for it in range(6):
        Hm, g, c, n = gpu_photo(slr, sensor, D, Dq, T)
        T = h.perturb_cw(T, -np.linalg.solve(Hm, g))
        errs.append(pose_error(T, Tq))
        say("photometric GN", it, "cost", c, "pixels", n, "error", errs[-1])
    assert errs[1][0] < 0.5 * errs[0][0] and errs[1][1] < 0.5 * errs[0][1], errs
    assert errs[-1][0] < 5e-3 and errs[-1][1] < 1e-3, errs

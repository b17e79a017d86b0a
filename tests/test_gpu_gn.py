"""GPU parity of the pose-only Gauss-Newton normal equations (slr_pose_gn,
Sec. 3.3.3) through the C ABI.

* Against the FP64 oracle (H, g, cost) on a room of overlapping surfels seen
  from a perturbed pose, ragged image (40x136), every tile shape, least
  squares and Huber, random per-pixel weights; pixels inside the oracle's
  guard band get weight 0 on both sides.  Every entry of H and g at 1e-3
  relative, with a floor of 1e-2 of the entry's Cauchy-Schwarz scale
  (sqrt(H_ii H_jj) for H_ij, sqrt(H_ii S) for g_i with S = sum m w r^2, the
  largest either can be); the cost at 1e-4.
* On the benchmark's map (1M surfels, 128x1024, keyframe 0 moved by a small
  step, the oracle's image at the keyframe pose as the target): every entry
  of H and g against the oracle as above on 48 pixels, half of them in the
  longest tiles that the one-wave form composites in quad mode, for both
  forms; the cost within the bound the forward's range tolerance implies.
* At the benchmark's size (1M surfels, 128x1024, the analytic target): H is
  symmetric positive semidefinite, the cost equals the plain sum over pixels,
  and g equals the pose gradient that slr_backward computes for the upstream
  range gradient m r (the same quantity by another route) to 1e-3.
* Gauss-Newton iterations through the GPU converge to the target's pose.
* Repeatability (bit-identical calls), an empty map, zero weights.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2503_17491_amd import synth
from tests import helpers as h
from tests.test_oracle_gn import pose_error, room_scene

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"
EXCL = O.FLAG_SUPPORT | O.FLAG_NEAR | O.FLAG_AMIN | O.FLAG_TSTOP


def say(*a):
    print("[gpu-gn]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def slr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_17491_amd import slr as S
    S.lib()
    return S


def room_dict():
    mu, q, ls, lg = room_scene()
    return dict(means=mu.astype(np.float32), quats=q.astype(np.float32), log_scales=ls.astype(np.float32),
                logits=lg.astype(np.float32))


def to_dev(sc):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(DEV) for k, v in sc.items()}


def pose_dev(T):
    return torch.from_numpy(np.ascontiguousarray(T, dtype=np.float64)).to(DEV)


def gpu_gn(S, sc, T, sensor, target, weight, huber_k, tiling):
    r = S.Renderer(sensor, tiling, 1 << 18)
    d = to_dev(sc)
    Td = pose_dev(T)
    D, N, A = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], Td)
    tg = torch.from_numpy(np.ascontiguousarray(target, np.float32)).to(DEV)
    wt = None if weight is None else torch.from_numpy(np.ascontiguousarray(weight, np.float32)).to(DEV)
    Hm, g, c = r.pose_gn(d["means"], d["quats"], d["log_scales"], d["logits"], Td, D, tg, wt, huber_k)
    torch.cuda.synchronize()
    return Hm.cpu().numpy(), g.cpu().numpy(), float(c.cpu()), D


_ORACLE = {}


def room_case(huber_k):
    """Scene, sensor, poses, target and weights of the parity case, and the
    oracle's normal equations (computed once per Huber threshold)."""
    if huber_k in _ORACLE:
        return _ORACLE[huber_k]
    sc = room_dict()
    sensor = O.make_sensor(40, 136)
    T_true = np.eye(4)
    T = h.perturb_cw(T_true, np.array([0.08, -0.06, 0.03, 0.01, -0.012, 0.015]))
    tgt = O.render_image(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T_true, sensor)
    cur = O.render_image(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor)
    g = np.random.default_rng(5)
    weight = (tgt["alpha"] > 0.5) & ((cur["flags"] & EXCL) == 0)
    weight = weight * g.uniform(0.5, 1.5, weight.shape)
    target = tgt["depth"].astype(np.float32).astype(np.float64)
    ref = O.pose_gn(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor, target,
                    weight.astype(np.float32).astype(np.float64), huber_k)
    _ORACLE[huber_k] = (sc, sensor, T, target, weight, ref)
    return _ORACLE[huber_k]


def assert_gn_close(Hm, g, ref, weight, huber_k, tol=1e-3, floor=1e-2):
    """Per-entry check of the normal equations against the oracle's: |dH_ij| <=
    tol max(|H_ij|, floor sqrt(H_ii H_jj)) and |dg_i| <= tol max(|g_i|, floor
    sqrt(H_ii S)), S = sum m w r^2 (Cauchy-Schwarz bounds |H_ij| and |g_i| by
    these scales).  Prints the largest error of each kind."""
    Hr, gr = ref["H"], ref["g"]
    r = ref["residual"].reshape(-1)
    _, w = O.huber(r, huber_k)
    S = float((np.asarray(weight, np.float64).reshape(-1) * w * r * r).sum())
    dg = np.sqrt(np.diag(Hr))
    scaleH = np.maximum(np.abs(Hr), floor * np.outer(dg, dg))
    scaleg = np.maximum(np.abs(gr), floor * dg * np.sqrt(S))
    eH = np.abs(Hm - Hr) / scaleH
    eg = np.abs(g - gr) / scaleg
    floored = int((np.abs(Hr) < floor * np.outer(dg, dg)).sum() + (np.abs(gr) < floor * dg * np.sqrt(S)).sum())
    say(f"   H entry err max {eH.max():.2e}, g entry err max {eg.max():.2e} "
        f"({floored} of 42 entries below the floor)")
    assert eH.max() <= tol, (eH, Hm, Hr)
    assert eg.max() <= tol, (eg, g, gr)


@pytest.mark.parametrize("huber_k", [0.0, 0.03])
@pytest.mark.parametrize("tiling", [(16, 16), (32, 8, 3, 2, 1), (8, 32), (4, 64)])
def test_pose_gn_matches_oracle(slr, huber_k, tiling):
    sc, sensor, T, target, weight, ref = room_case(huber_k)
    say("room 40x136", "huber", huber_k, "tiling", tiling)
    Hm, g, c, _ = gpu_gn(slr, sc, T, sensor, target, weight, huber_k, tiling)
    if huber_k > 0:
        rr = np.abs(ref["residual"])[weight > 0]
        assert (rr > huber_k).sum() > 20 and (rr <= huber_k).sum() > 20
    np.testing.assert_array_equal(Hm, Hm.T)
    assert_gn_close(Hm, g, ref, weight, huber_k)
    assert abs(c - ref["cost"]) <= 1e-4 * ref["cost"], (c, ref["cost"])


def test_pose_gn_repeatable_and_degenerate(slr):
    sc, sensor, T, target, weight, ref = room_case(0.0)
    say("repeatable, zero weight, empty map")
    r = slr.Renderer(sensor, (16, 16), 1 << 18)
    d = to_dev(sc)
    Td = pose_dev(T)
    D, N, A = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], Td)
    tg = torch.from_numpy(target.astype(np.float32)).to(DEV)
    wt = torch.from_numpy(weight.astype(np.float32)).to(DEV)
    a = [t.clone() for t in r.pose_gn(d["means"], d["quats"], d["log_scales"], d["logits"], Td, D, tg, wt)]
    b = [t.clone() for t in r.pose_gn(d["means"], d["quats"], d["log_scales"], d["logits"], Td, D, tg, wt)]
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    # also after a fresh render (binning and tile order recomputed), for both forms
    for tl in ((16, 16), (16, 16, 3, 2, 1)):
        rr = slr.Renderer(sensor, tl, 1 << 18)
        outs = []
        for _ in range(2):
            Dr, _, _ = rr.forward(d["means"], d["quats"], d["log_scales"], d["logits"], Td)
            outs.append([t.clone() for t in rr.pose_gn(d["means"], d["quats"], d["log_scales"], d["logits"], Td, Dr,
                                                       tg, wt)])
        for x, y in zip(*outs):
            assert torch.equal(x, y), tl
    z = r.pose_gn(d["means"], d["quats"], d["log_scales"], d["logits"], Td, D, tg, torch.zeros_like(wt))
    for x in z:
        assert not x.cpu().numpy().any()
    # an empty map renders nothing: J = 0, the cost is the weighted sum over the targets
    empty = {k: v[:0] for k, v in sc.items()}
    e = slr.Renderer(sensor, (16, 16), 1 << 10)
    de = to_dev(empty)
    De, _, _ = e.forward(de["means"], de["quats"], de["log_scales"], de["logits"], Td)
    He, ge, ce = e.pose_gn(de["means"], de["quats"], de["log_scales"], de["logits"], Td, De, tg, wt, 0.0)
    assert not He.cpu().numpy().any() and not ge.cpu().numpy().any()
    want = float((0.5 * weight * target ** 2).sum())
    assert abs(float(ce.cpu()) - want) <= 1e-6 * want


def same_gn(a, b):
    np.testing.assert_array_equal(b[0], b[0].T)
    assert np.abs(a[0] - b[0]).max() <= 1e-12 * np.abs(a[0]).max()
    assert np.abs(a[1] - b[1]).max() <= 1e-12 * np.abs(a[1]).max()
    assert abs(a[2] - b[2]) <= 1e-12 * abs(a[2])


def test_pose_gn_wave_form_matches_workgroup_form(slr):
    """One wave per strip (backward form 3) and one workgroup per tile
    (backward form 1) give the same normal equations: each pixel sees the same
    records in the same order, and a tile's four strip sums are added in the
    workgroup's order.  The two kernels may contract different multiply-adds
    (FP32 last-bit differences in a pixel's terms), so the comparison allows
    1e-12 relative.  The room case at all tile shapes, and the benchmark's map
    at 128x1024."""
    from paper_2503_17491_amd import targets
    sc, sensor, T, target, weight, ref = room_case(0.03)
    for th, tw in ((16, 16), (32, 8), (8, 32), (4, 64)):
        say("wave vs workgroup form, room", th, tw)
        a = gpu_gn(slr, sc, T, sensor, target, weight, 0.03, (th, tw, 3, 2, 1))
        b = gpu_gn(slr, sc, T, sensor, target, weight, 0.03, (th, tw, 3, 2, 3))
        same_gn(a[:3], b[:3])
        assert_gn_close(b[0], b[1], ref, weight, 0.03)
    big, prims = synth.structured_scene(1_000_000, 0)
    Tb = synth.circle_poses(8, 0)[0]
    sb = slr.make_sensor(128, 1024)
    Dt, _ = targets.raycast(prims, sb, Tb, seed=100)
    m = (Dt > 0).astype(np.float32)
    out = []
    for bv in (1, 3):
        say("wave vs workgroup form, 1M 128x1024, backward form", bv)
        r = slr.Renderer(sb, (32, 8, 3, 2, bv), 4 << 20)
        d = to_dev(big)
        Td = pose_dev(Tb)
        D, N, A = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], Td)
        Hm, g, c = r.pose_gn(d["means"], d["quats"], d["log_scales"], d["logits"], Td, D,
                             torch.from_numpy(Dt).to(DEV), torch.from_numpy(m).to(DEV), 0.05)
        out.append((Hm.cpu().numpy(), g.cpu().numpy(), float(c.cpu())))
        del r
        torch.cuda.empty_cache()
    same_gn(out[0], out[1])


def test_pose_gn_fullsize_properties(slr):
    """The benchmark's map and image size: 1M structured-scene surfels, 128x1024."""
    from paper_2503_17491_amd import targets
    sc, prims = synth.structured_scene(1_000_000, 0)
    T = synth.circle_poses(8, 0)[0]
    sensor = slr.make_sensor(128, 1024)
    Dt, _ = targets.raycast(prims, sensor, T, seed=100)
    for tiling, k in (((32, 8, 3, 2, 1), 0.0), ((16, 16, 3, 2, 3), 0.05)):
        say("fullsize 1M 128x1024", tiling, "huber", k)
        r = slr.Renderer(sensor, tiling, 4 << 20)
        d = to_dev(sc)
        Td = pose_dev(T)
        D, N, A = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], Td)
        tg = torch.from_numpy(Dt).to(DEV)
        m = (tg > 0).float()
        Hm, g, c = r.pose_gn(d["means"], d["quats"], d["log_scales"], d["logits"], Td, D, tg, m, k)
        Hn, gn, cn = Hm.cpu().numpy(), g.cpu().numpy(), float(c.cpu())
        np.testing.assert_array_equal(Hn, Hn.T)
        assert np.linalg.eigvalsh(Hn).min() >= -1e-9 * np.abs(Hn).max()
        res = (D.double() - tg.double())
        a = res.abs()
        if k > 0:
            rho = torch.where(a <= k, 0.5 * res * res, k * (a - 0.5 * k))
            w = torch.where(a <= k, torch.ones_like(a), k / a)
        else:
            rho, w = 0.5 * res * res, torch.ones_like(a)
        want = float((m.double() * rho).sum().cpu())
        assert abs(cn - want) <= 1e-9 * abs(want), (cn, want)
        # g is the pose gradient of the cost: the backward with dL/dD = m w r gives it too
        up = (m.double() * w * res).float().contiguous()
        _, dpose = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], Td, up, None, None,
                              pose_only=True)
        dp = dpose.cpu().numpy()
        assert np.linalg.norm(gn - dp) <= 1e-3 * np.linalg.norm(dp), (gn, dp)
        del r
        torch.cuda.empty_cache()


_HEADLINE = {}


def headline_case():
    """The benchmark's map (1M structured-scene surfels, seed 0) and keyframe 0
    moved by a small pose step; the target is the oracle's range image at the
    keyframe's own pose; weight 1 on 32 pixels of the 4 longest-list tiles at
    32x8 (composited in quad mode by the one-wave form) and 16 random pixels,
    all with the oracle's decisions at the moved pose away from every
    threshold and a return in the target.  (The oracle forms each pixel's
    Jacobian row with a backward call of its own, about a second each on this
    map, which bounds the pixel count.)"""
    if _HEADLINE:
        return _HEADLINE["case"]
    sc, _ = synth.structured_scene(1_000_000, 0)
    T_true = synth.circle_poses(8, 0)[0]
    T = h.perturb_cw(T_true, np.array([0.02, -0.015, 0.01, 0.002, -0.003, 0.0025]))
    sensor = O.make_sensor(128, 1024)
    say("oracle renders of the 1M map at the keyframe pose and the moved pose")
    args = (sc["means"], sc["quats"], sc["log_scales"], sc["logits"])
    tgt = O.render_image(*args, T_true, sensor, cull=True)
    cur = O.render_image(*args, T, sensor, cull=True)
    bins = O.bin_surfels(*args, T, sensor, 32, 8)
    L = bins["ranges"][:, 1] - bins["ranges"][:, 0]
    ok = (tgt["alpha"] > 0.5) & ((cur["flags"] & (EXCL | O.FLAG_CLAMP)) == 0)
    g = np.random.default_rng(71)
    weight = np.zeros((128, 1024))
    for t in np.argsort(-L, kind="stable")[:4]:
        ty, tx = divmod(int(t), bins["tiles_x"])
        ii, jj = np.nonzero(ok[ty * 32:(ty + 1) * 32, tx * 8:(tx + 1) * 8])
        pick = g.permutation(ii.size)[:8]
        weight[ty * 32 + ii[pick], tx * 8 + jj[pick]] = 1.0
    ii, jj = np.nonzero(ok & (weight == 0))
    pick = g.permutation(ii.size)[:16]
    weight[ii[pick], jj[pick]] = 1.0
    target = tgt["depth"].astype(np.float32).astype(np.float64)
    say(f"oracle normal equations over {int(weight.sum())} pixels (longest list {int(L.max())})")
    ref = O.pose_gn(*args, T, sensor, target, weight, 0.05, cull=True)
    _HEADLINE["case"] = (sc, sensor, T, target, weight, ref)
    return _HEADLINE["case"]


@pytest.mark.parametrize("tiling", [(32, 8, 3, 2, 3), (32, 8, 3, 2, 1)])
def test_pose_gn_headline_map_matches_oracle(slr, tiling):
    """Gauss-Newton normal equations on the benchmark's map against the
    oracle, entry by entry: the one-wave form (its longest tiles in quad mode)
    and the workgroup form."""
    sc, sensor, T, target, weight, ref = headline_case()
    say("1M map, keyframe 0 moved, tiling", tiling)
    Hm, g, c, _ = gpu_gn(slr, sc, T, sensor, target, weight, 0.05, tiling)
    assert_gn_close(Hm, g, ref, weight, 0.05)
    # the cost moves with the range by |d rho / d r| <= |r|: a range within the
    # forward's 1e-4 relative bound keeps it within sum m |r| 1e-4 D
    bound = 1e-4 * float((weight * np.abs(ref["residual"]) * np.abs(ref["depth"])).sum())
    say(f"   cost {c:.6e} against {ref['cost']:.6e} (bound {bound:.1e})")
    assert abs(c - ref["cost"]) <= bound, (c, ref["cost"], bound)


def test_gauss_newton_iterations_converge(slr):
    sc = room_dict()
    sensor = slr.make_sensor(32, 256)
    T_true = np.eye(4)
    tgt = O.render_image(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T_true, sensor)
    target = torch.from_numpy(tgt["depth"].astype(np.float32)).to(DEV)
    weight = torch.from_numpy((tgt["alpha"] > 0.5).astype(np.float32)).to(DEV)
    T = h.perturb_cw(T_true, np.array([0.1, -0.08, 0.05, 0.02, -0.015, 0.025]))
    r = slr.Renderer(sensor, (16, 16), 1 << 18)
    d = to_dev(sc)
    errs = [pose_error(T, T_true)]
    for it in range(5):
        Td = pose_dev(T)
        D, _, _ = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], Td)
        Hm, g, c = r.pose_gn(d["means"], d["quats"], d["log_scales"], d["logits"], Td, D, target, weight, 0.0)
        delta = -np.linalg.solve(Hm.cpu().numpy(), g.cpu().numpy())
        T = h.perturb_cw(T, delta)
        errs.append(pose_error(T, T_true))
        say("GN iteration", it, "cost", float(c.cpu()), "error", errs[-1])
    for a, b in zip(errs[:3], errs[1:4]):  # every early step at least halves both errors
        assert b[0] < 0.5 * a[0] and b[1] < 0.5 * a[1], errs
    assert errs[-1][0] < 1e-4 and errs[-1][1] < 1e-5, errs

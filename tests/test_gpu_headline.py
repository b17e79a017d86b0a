"""Oracle parity at the benchmark's own workload, through the C ABI.

The map is the 1M-surfel structured scene (seed 0), the keyframes are the
eight 128x1024 poses on the 5 m circle (seed 0), and the tiling is the one
the benchmark's autotuner picks on it: 32x8 tiles, the one-wave forward, the
workgroup backward staging 128 or 192 records per LDS batch.  Per keyframe
this is about 1.8M (tile, surfel) pairs with lists of up to 15k records at
the horizon.

* Binning of keyframe 0 (plain form): keys, tile counts, pixel boxes, the
  sorted (tile, surfel) lists and the tile ranges bit-exact against the
  oracle's mirror (Sec. 3.2.1, Supp. B).
* Forward of keyframe 0 on every pixel of the image against the FP64 oracle
  (Sec. 3.2.1 Eqs. ab_depth, ab_normal, ab_opacity); see tests/gpu_checks.py
  for the admissible-result rule.
* Backward of keyframe 0 with random upstream gradients on every pixel whose
  decisions lie away from all thresholds, for both LDS batch sizes, the
  one-wave backward (whose longest tiles take the quad mode) and the
  fixed-order backward, against the oracle's analytic gradients (Supp. D; the
  se(3) pose gradient).
* The eight-keyframe batch: each keyframe's sorted lists and tile ranges are
  the oracle's binning of that keyframe; keyframe 0's images equal the plain
  form's bit for bit; the other keyframes' images match the oracle on 2048
  random pixels plus every pixel of their longest-list tile.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2503_17491_amd import synth
from tests import gpu_checks as GC

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"
H, W = 128, 1024
TH, TW = 32, 8


def say(*a):
    print("[gpu-headline]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def slr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_17491_amd import slr as S
    S.lib()
    return S


@pytest.fixture(scope="module")
def case(slr):
    say("building the 1M-surfel map and the eight keyframe poses")
    sc, _ = synth.structured_scene(1_000_000, 0)
    poses = synth.circle_poses(8, 0)
    sensor = slr.make_sensor(H, W)
    assert sensor == O.make_sensor(H, W)
    d = GC.to_dev(torch, sc)
    say("oracle binning of keyframe 0")
    ref_bin = O.bin_surfels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], poses[0], sensor, TH, TW)
    return dict(sc=sc, poses=poses, sensor=sensor, d=d, ref_bin=ref_bin)


def tiling(slr, batch, bwd=None):
    bwd = slr.VARIANT_LDS if bwd is None else bwd
    return (TH, TW, slr.VARIANT_WAVE, slr.SCHEDULE_LONGEST, bwd, slr.BOX_EXACT, batch)


def longest_tiles(ranges, tiles_x, k):
    L = ranges[:, 1] - ranges[:, 0]
    top = np.argsort(-L, kind="stable")[:k]
    pix = []
    for t in top:
        ty, tx = divmod(int(t), tiles_x)
        ii, jj = np.meshgrid(np.arange(ty * TH, min((ty + 1) * TH, H)), np.arange(tx * TW, min((tx + 1) * TW, W)),
                             indexing="ij")
        pix.append(np.stack([ii.ravel(), jj.ravel()], 1))
    return np.concatenate(pix).astype(np.int32), L[top]


def test_headline_binning_bit_exact(slr, case):
    r = slr.Renderer(case["sensor"], tiling(slr, 192), 4 << 20)
    d = case["d"]
    say("plain render of keyframe 0")
    r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], GC.pose_dev(torch, case["poses"][0]))
    torch.cuda.synchronize()
    v = r.views()
    ref = case["ref_bin"]
    cnt = v["counts"].cpu().numpy()
    np.testing.assert_array_equal(cnt, ref["counts"])
    vis = cnt > 0
    np.testing.assert_array_equal(v["keys"].cpu().numpy().view(np.uint32)[vis], ref["keys"][vis])
    np.testing.assert_array_equal(v["pixbox"].cpu().numpy()[vis, :6].astype(np.int32), ref["pixbox"][vis])
    assert v["K"] == ref["K"]
    np.testing.assert_array_equal(v["sorted_tile"].cpu().numpy(), ref["sorted_tile"])
    np.testing.assert_array_equal(v["sorted_id"].cpu().numpy(), ref["sorted_id"])
    np.testing.assert_array_equal(v["ranges"].cpu().numpy(), ref["ranges"])
    L = ref["ranges"][:, 1] - ref["ranges"][:, 0]
    say(f"keyframe 0: K {ref['K']} pairs, {int(vis.sum())} binned surfels, longest list {int(L.max())}")


def test_headline_forward_full_image(slr, case):
    r = slr.Renderer(case["sensor"], tiling(slr, 192), 4 << 20)
    d = case["d"]
    T = case["poses"][0]
    D, N, A = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], GC.pose_dev(torch, T))
    torch.cuda.synchronize()
    say("forward keyframe 0, all 131072 pixels")
    GC.forward_verdict(D.cpu().numpy(), N.cpu().numpy(), A.cpu().numpy(), case["sc"], T, case["sensor"],
                       label="1M surfels, keyframe 0, 128x1024")
    pix, L = longest_tiles(case["ref_bin"]["ranges"], case["ref_bin"]["tiles_x"], 4)
    say(f"   (the 4 longest-list tiles, {L.tolist()} records, are among them)")


@pytest.fixture(scope="module")
def dense_upstream(case):
    """Random upstream gradients on every clean pixel of keyframe 0 and the
    oracle's gradients for them (computed once for both batch sizes)."""
    sc, T, sensor = case["sc"], case["poses"][0], case["sensor"]
    say("clean pixels of keyframe 0")
    pix = GC.clean_pixels(sc, T, sensor)
    g = np.random.default_rng(31)
    P = pix.shape[0]
    gD = g.normal(size=P).astype(np.float32)
    gN = g.normal(size=(P, 3)).astype(np.float32)
    gO = g.normal(size=P).astype(np.float32)
    say(f"oracle backward over {P} pixels")
    ref = GC.oracle_backward(sc, T, sensor, pix, gD, gN, gO)
    return pix, gD, gN, gO, ref


@pytest.mark.parametrize("batch", [128, 192, "wave", "fixed"])
def test_headline_backward_dense(slr, case, dense_upstream, batch):
    """The workgroup backward at both LDS batch sizes, the one-wave
    backward, whose longest tiles (lists of 768 entries or more) a single
    keyframe takes in quad mode, and the fixed-order backward."""
    pix, gD, gN, gO, ref = dense_upstream
    tl = (tiling(slr, 0, slr.VARIANT_WAVE) if batch == "wave"
          else tiling(slr, 0, slr.VARIANT_DETERMINISTIC) if batch == "fixed" else tiling(slr, batch))
    r = slr.Renderer(case["sensor"], tl, 4 << 20)
    d = case["d"]
    Td = GC.pose_dev(torch, case["poses"][0])
    r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], Td)
    GDi = np.zeros((H, W), np.float32); GNi = np.zeros((H, W, 3), np.float32); GOi = np.zeros((H, W), np.float32)
    GDi[pix[:, 0], pix[:, 1]] = gD; GNi[pix[:, 0], pix[:, 1]] = gN; GOi[pix[:, 0], pix[:, 1]] = gO
    g, dp = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], Td, torch.from_numpy(GDi).to(DEV),
                       torch.from_numpy(GNi).to(DEV), torch.from_numpy(GOi).to(DEV))
    torch.cuda.synchronize()
    GC.backward_verdict({k: v.cpu().numpy() for k, v in g.items()}, dp.cpu().numpy(), ref,
                        label=f"1M surfels, keyframe 0, {pix.shape[0]} pixels, "
                              + ("one-wave backward (quad mode)" if batch == "wave"
                                 else "fixed-order backward" if batch == "fixed" else f"LDS batch {batch}"))


def test_headline_batch_lists_and_images(slr, case):
    sc, poses, sensor, d = case["sc"], case["poses"], case["sensor"], case["d"]
    frames = [dict(set=0, T_cw=GC.pose_dev(torch, T), sensor=sensor) for T in poses]
    br = slr.BatchRenderer([d], frames, tiling(slr, 192), capacity=24 << 20)
    br.render()
    torch.cuda.synchronize()
    K, over = br.pairs()
    assert over == 0
    v = br.views()
    st, sid, rg = v["sorted_tile"].cpu().numpy(), v["sorted_id"].cpu().numpy(), v["ranges"].cpu().numpy()
    p0 = 0
    rng = np.random.default_rng(41)
    for f, T in enumerate(poses):
        ref = case["ref_bin"] if f == 0 else O.bin_surfels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"],
                                                         T, sensor, TH, TW)
        k, t0, i0 = ref["K"], v["tile_off"][f], v["item_off"][f]
        nt = ref["ranges"].shape[0]
        np.testing.assert_array_equal(st[p0:p0 + k] - t0, ref["sorted_tile"])
        np.testing.assert_array_equal(sid[p0:p0 + k] - i0, ref["sorted_id"])
        mine = rg[t0:t0 + nt].copy()
        full = mine[:, 1] > mine[:, 0]
        mine[full] -= p0
        np.testing.assert_array_equal(mine, ref["ranges"])
        say(f"keyframe {f}: {k} pairs, lists and ranges equal the oracle's")
        Dg, Ng, Ag = (t.cpu().numpy() for t in br.out[f])
        if f == 0:
            r = slr.Renderer(sensor, tiling(slr, 192), 4 << 20)
            D0, N0, A0 = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], frames[0]["T_cw"])
            for a, b in zip((Dg, Ng, Ag), (D0, N0, A0)):
                np.testing.assert_array_equal(a, b.cpu().numpy())
        else:
            pix = np.stack([rng.integers(0, H, 2048), rng.integers(0, W, 2048)], 1).astype(np.int32)
            lp, _ = longest_tiles(ref["ranges"], ref["tiles_x"], 1)
            GC.forward_verdict(Dg, Ng, Ag, sc, T, sensor, np.concatenate([pix, lp]),
                               label=f"batched keyframe {f}")
        p0 += k
    assert p0 == K


def test_batch_of_nine_matches_plain(slr, case):
    """Nine keyframes of the 1M-surfel map in one batch (9 M records: the range
    sort, compaction and count scan take their 4096-item blocks, which the
    eight-keyframe batch does not reach) against the plain form of each
    keyframe (2048-item blocks): identical sorted lists, tile ranges and
    images, bit for bit."""
    sensor, d = case["sensor"], case["d"]
    poses = synth.circle_poses(9, 3)
    frames = [dict(set=0, T_cw=GC.pose_dev(torch, T), sensor=sensor) for T in poses]
    br = slr.BatchRenderer([d], frames, tiling(slr, 192), capacity=28 << 20)
    br.render()
    torch.cuda.synchronize()
    K, over = br.pairs()
    assert over == 0
    v = br.views()
    st, sid, rg = v["sorted_tile"].cpu().numpy(), v["sorted_id"].cpu().numpy(), v["ranges"].cpu().numpy()
    r = slr.Renderer(sensor, tiling(slr, 192), 4 << 20)
    p0 = 0
    for f, fr in enumerate(frames):
        D, N, A = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], fr["T_cw"])
        torch.cuda.synchronize()
        pv = r.views()
        k, t0, i0 = pv["K"], v["tile_off"][f], v["item_off"][f]
        np.testing.assert_array_equal(st[p0:p0 + k] - t0, pv["sorted_tile"].cpu().numpy())
        np.testing.assert_array_equal(sid[p0:p0 + k] - i0, pv["sorted_id"].cpu().numpy())
        nt = pv["ranges"].shape[0]
        mine = rg[t0:t0 + nt].copy()
        full = mine[:, 1] > mine[:, 0]
        mine[full] -= p0
        np.testing.assert_array_equal(mine, pv["ranges"].cpu().numpy())
        for a, b in zip(br.out[f], (D, N, A)):
            assert torch.equal(a, b), f"keyframe {f}"
        p0 += k
    assert p0 == K
    say(f"nine keyframes: {K} pairs, lists, ranges and images equal the plain form's")


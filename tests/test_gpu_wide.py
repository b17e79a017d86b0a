"""Oracle parity on the wide-frame workload of the 2M-surfel mapping loop,
through the C ABI: 2 000 000 urban-scene surfels (seed 5) in one 128x2048
frame at the identity pose.  The frame has 1024 tiles, so the quad mode of
the one-wave forward and backward takes only its longest tiles (the cap of
the launch budget) and the rest of the long tiles run as 64-pixel strips --
a split a single 128x1024 frame never reaches.

* Forward on 4096 random pixels plus every pixel of the 4 longest-list tiles
  against the FP64 oracle (Sec. 3.2.1; see tests/gpu_checks.py for the
  admissible-result rule).
* Backward with random upstream gradients on the clean pixels of that
  sample, for the one-wave backward (quad mode) and the workgroup backward,
  against the oracle's analytic gradients (Supp. D; the se(3) pose gradient).
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
H, W = 128, 2048
TH, TW = 16, 16


def say(*a):
    print("[gpu-wide]", *a, flush=True)
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
    say("building the 2M-surfel urban map")
    sc, _ = synth.structured_scene(2_000_000, 5, kind="urban")
    sensor = slr.make_sensor(H, W)
    assert sensor == O.make_sensor(H, W)
    T = np.eye(4)
    d = GC.to_dev(torch, sc)
    r = slr.Renderer(sensor, (TH, TW, slr.VARIANT_WAVE, slr.SCHEDULE_LONGEST, slr.VARIANT_WAVE), 8 << 20)
    r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], GC.pose_dev(torch, T))
    torch.cuda.synchronize()
    rg = r.views()["ranges"].cpu().numpy()
    L = rg[:, 1] - rg[:, 0]
    tiles_x = W // TW
    top = np.argsort(-L, kind="stable")[:4]
    pix = []
    for t in top:
        ty, tx = divmod(int(t), tiles_x)
        ii, jj = np.meshgrid(np.arange(ty * TH, (ty + 1) * TH), np.arange(tx * TW, (tx + 1) * TW), indexing="ij")
        pix.append(np.stack([ii.ravel(), jj.ravel()], 1))
    g = np.random.default_rng(51)
    pix.append(np.stack([g.integers(0, H, 4096), g.integers(0, W, 4096)], 1))
    pix = np.unique(np.concatenate(pix).astype(np.int32), axis=0)
    say(f"{int((L >= 768).sum())} tiles with lists of 768 entries or more (longest {int(L.max())}); "
        f"{pix.shape[0]} sampled pixels")
    return dict(sc=sc, sensor=sensor, T=T, d=d, pix=pix, nlong=int((L >= 768).sum()))


def test_wide_forward_sampled(slr, case):
    sc, sensor, T, d, pix = case["sc"], case["sensor"], case["T"], case["d"], case["pix"]
    r = slr.Renderer(sensor, (TH, TW, slr.VARIANT_WAVE, slr.SCHEDULE_LONGEST, slr.VARIANT_WAVE), 8 << 20)
    D, N, A = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], GC.pose_dev(torch, T))
    torch.cuda.synchronize()
    GC.forward_verdict(D.cpu().numpy(), N.cpu().numpy(), A.cpu().numpy(), sc, T, sensor, pix,
                       label="2M urban surfels, 128x2048")


@pytest.fixture(scope="module")
def upstream(case):
    sc, T, sensor = case["sc"], case["T"], case["sensor"]
    pix = GC.clean_pixels(sc, T, sensor, case["pix"])
    g = np.random.default_rng(52)
    P = pix.shape[0]
    gD = g.normal(size=P).astype(np.float32)
    gN = g.normal(size=(P, 3)).astype(np.float32)
    gO = g.normal(size=P).astype(np.float32)
    say(f"oracle backward over {P} clean pixels")
    return pix, gD, gN, gO, GC.oracle_backward(sc, T, sensor, pix, gD, gN, gO)


@pytest.mark.parametrize("bwd", ["wave", "lds"])
def test_wide_backward_sampled(slr, case, upstream, bwd):
    pix, gD, gN, gO, ref = upstream
    bv = slr.VARIANT_WAVE if bwd == "wave" else slr.VARIANT_LDS
    r = slr.Renderer(case["sensor"], (TH, TW, slr.VARIANT_WAVE, slr.SCHEDULE_LONGEST, bv), 8 << 20)
    d = case["d"]
    Td = GC.pose_dev(torch, case["T"])
    r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], Td)
    GDi = np.zeros((H, W), np.float32); GNi = np.zeros((H, W, 3), np.float32); GOi = np.zeros((H, W), np.float32)
    GDi[pix[:, 0], pix[:, 1]] = gD; GNi[pix[:, 0], pix[:, 1]] = gN; GOi[pix[:, 0], pix[:, 1]] = gO
    g, dp = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], Td, torch.from_numpy(GDi).to(DEV),
                       torch.from_numpy(GNi).to(DEV), torch.from_numpy(GOi).to(DEV))
    torch.cuda.synchronize()
    GC.backward_verdict({k: v.cpu().numpy() for k, v in g.items()}, dp.cpu().numpy(), ref,
                        label=f"2M urban surfels, 128x2048, {pix.shape[0]} pixels, "
                              + ("one-wave backward (quad mode on the longest tiles)" if bwd == "wave"
                                 else "workgroup backward"))

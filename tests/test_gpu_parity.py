"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

* Binning (keys, tile counts, pixel boxes, sorted (tile, surfel) lists, tile
  ranges): bit-exact.
* Forward: relative 1e-4 on depth / alpha / normal against one of the
  oracle's admissible results of each pixel (the plain render, or, where a
  decision lies within rounding distance of its threshold, that decision
  taken the other way); see tests/gpu_checks.py.
* Backward: relative 1e-3 on per-surfel gradient blocks and on the pose
  6-vector, against the oracle's analytic FP64 gradients.  A block's error is
  divided by max(|g_ref|, 1e-3 RMS, 1e-2 sum_pixels |contribution|): a
  gradient that is a near-cancelling sum of per-pixel contributions is held to
  1e-5 of the magnitude summed, the precision an FP32 sum can promise; the
  blocks that need that term are counted and printed.
Large configurations compare sampled pixels (forward) or use upstream
gradients that are non-zero only on sampled pixels (backward).
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
EXCL = O.FLAG_SUPPORT | O.FLAG_NEAR | O.FLAG_AMIN | O.FLAG_TSTOP


def say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def slr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_17491_amd import slr as S
    S.lib()
    return S


def to_dev(sc):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(DEV) for k, v in sc.items()}


def pose_dev(T):
    return torch.from_numpy(np.ascontiguousarray(T, dtype=np.float64)).to(DEV)


def gpu_render(S, sc, T, sensor, tiling=(16, 16), capacity=1 << 16):
    r = S.Renderer(sensor, tiling, capacity)
    d = to_dev(sc)
    Td = pose_dev(T)
    D, N, A = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], Td)
    torch.cuda.synchronize()
    return r, d, Td, D.cpu().numpy().astype(np.float64), N.cpu().numpy().astype(np.float64), \
        A.cpu().numpy().astype(np.float64)


def assert_forward_close(D, N, A, sc, T, sensor, pix=None):
    return GC.forward_verdict(D, N, A, sc, T, sensor, pix)


# ---------------------------------------------------------------- binning
def giant_scene():
    """A shell scene plus a few surfels far larger than the sensor's
    surroundings: a horizontal one above the sensor (pierced by the z-axis:
    full azimuth, every row up to the top), one below, and a vertical wall,
    so single records span more pair slots than one emit block holds."""
    sc = synth.shell_scene(3000, 12)
    sc["means"][:3] = np.array([[0.4, 0.3, 3.0], [-0.2, 0.5, -2.5], [6.0, 0.5, 0.2]], np.float32)
    sc["quats"][:3] = np.array([[1, 0, 0, 0], [1, 0, 0, 0], [0.7071068, 0, 0.7071068, 0]], np.float32)
    sc["log_scales"][:3] = np.log(np.array([[30.0, 25.0], [20.0, 30.0], [15.0, 12.0]], np.float32))
    sc["logits"][:3] = 2.0
    return sc


BIN_CASES = [
    ("giant-surfels-128x2048-8x32", giant_scene, lambda: np.eye(4), (128, 2048), (8, 32)),
    ("shell-2k-64x512", lambda: synth.shell_scene(2000, 1), lambda: np.eye(4), (64, 512), (16, 16)),
    ("shell-2k-64x512-8x32", lambda: synth.shell_scene(2000, 1), lambda: np.eye(4), (64, 512), (8, 32)),
    ("shell-5k-posed-4x64", lambda: synth.shell_scene(5000, 4), lambda: synth.perturbed_pose(4, 1.0, 30.0),
     (32, 1800), (4, 64)),
    ("structured-20k-posed-32x8", lambda: synth.structured_scene(20000, 8)[0], lambda: synth.circle_poses(8, 3)[5],
     (128, 1024), (32, 8)),
    ("ragged-37x300", lambda: synth.shell_scene(3000, 9), lambda: np.eye(4), (37, 300), (16, 16)),
]


@pytest.mark.parametrize("name,mk,mkT,hw,tiling", BIN_CASES, ids=[c[0] for c in BIN_CASES])
def test_binning_bit_exact(slr, name, mk, mkT, hw, tiling):
    say("binning", name)
    sc, T = mk(), mkT()
    sensor = O.make_sensor(*hw)
    ssensor = slr.make_sensor(*hw)
    assert ssensor == sensor
    r, d, Td, D, N, A = gpu_render(slr, sc, T, ssensor, tiling)
    v = r.views()
    ref = O.bin_surfels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor, tiling[0], tiling[1])
    cnt = v["counts"].cpu().numpy()
    np.testing.assert_array_equal(cnt, ref["counts"])
    vis = cnt > 0
    np.testing.assert_array_equal(v["keys"].cpu().numpy().view(np.uint32)[vis], ref["keys"][vis])
    np.testing.assert_array_equal(v["pixbox"].cpu().numpy()[vis, :6].astype(np.int32), ref["pixbox"][vis])
    assert v["K"] == ref["K"]
    np.testing.assert_array_equal(v["sorted_tile"].cpu().numpy(), ref["sorted_tile"])
    np.testing.assert_array_equal(v["sorted_id"].cpu().numpy(), ref["sorted_id"])
    np.testing.assert_array_equal(v["ranges"].cpu().numpy(), ref["ranges"])
    say("binning", name, "K", ref["K"], "visible", int(vis.sum()))


# ---------------------------------------------------------------- forward
def test_forward_parity_shell_full_image(slr):
    say("forward shell-2k-64x512 full image")
    sc = synth.shell_scene(2000, 1)
    sensor = slr.make_sensor(64, 512)
    r, d, Td, D, N, A = gpu_render(slr, sc, np.eye(4), sensor)
    ref = O.render_image(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], np.eye(4), sensor)
    assert_forward_close(D, N, A, sc, np.eye(4), sensor)
    v = r.views()
    ok = (ref["flags"] & EXCL) == 0
    np.testing.assert_allclose(v["T_final"].cpu().numpy()[ok], ref["T_final"][ok], rtol=1e-4, atol=1e-6)


def test_forward_parity_posed_structured(slr):
    say("forward structured-30k-posed-128x1024 full image")
    sc, _ = synth.structured_scene(30000, 12)
    T = synth.circle_poses(8, 0)[3]
    sensor = slr.make_sensor(128, 1024)
    r, d, Td, D, N, A = gpu_render(slr, sc, T, sensor, (8, 32))
    assert_forward_close(D, N, A, sc, T, sensor)


def test_forward_identical_across_tilings_and_runs(slr):
    say("forward tiling invariance")
    sc = synth.shell_scene(4000, 2)
    sensor = slr.make_sensor(64, 512)
    outs = []
    # (h, w, 2): the forward that reads records through the scalar cache;
    # (h, w, v, 2): tiles taken longest list first
    for tiling in [(16, 16), (8, 32), (32, 8), (4, 64), (16, 16), (16, 16, 2), (8, 32, 2), (4, 64, 2),
                   (16, 16, 1, 2), (32, 8, 2, 2), (16, 16, 3), (32, 8, 3), (4, 64, 3, 1)]:
        _, _, _, D, N, A = gpu_render(slr, sc, np.eye(4), sensor, tiling)
        outs.append((D, N, A))
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            np.testing.assert_array_equal(a, b)


def test_forward_state_identical_across_variants(slr):
    """Same tiling, the compositing kernels (records staged in LDS by the
    workgroup, with the few-pixels-left mode; through the scalar cache; one
    wave per strip, whose longest tiles take the quad mode): identical
    per-pixel state and contribution counts, not only identical images.  The
    evaluated-entry count is the same where both walk the same rows; the quad
    mode walks only the records that meet its sub-strip's rows, never more."""
    say("forward variants: per-pixel state and census")
    cases = [(synth.shell_scene(4000, 2), (64, 512), np.eye(4)),
             (synth.structured_scene(30000, 3)[0], (64, 512), np.eye(4)),
             # lists of several thousand entries: the quad mode takes the longest tiles
             (synth.structured_scene(300000, 3)[0], (128, 1024), synth.circle_poses(8, 0)[1])]
    for sc, hw, T in cases:
        sensor = slr.make_sensor(*hw)
        for group in ([(16, 16, 1), (16, 16, 2), (16, 16, 3)], [(8, 32, 1), (8, 32, 3)], [(32, 8, 1), (32, 8, 3)]):
            views = []
            for tiling in group:
                r, _, _, D, N, A = gpu_render(slr, sc, T, sensor, tiling, 1 << 22)
                v = r.views()
                views.append((D, N, A, v["T_final"].cpu().numpy(), v["n_proc"].cpu().numpy(),
                              v["census"][1].cpu().numpy(), v["census"][0].cpu().numpy()))
            for other in views[1:]:
                for a, b in zip(views[0][:6], other[:6]):
                    np.testing.assert_array_equal(a, b)
                assert (other[6] <= views[0][6]).all()
            say(f"   {hw} {group[0][:2]}: evaluated entries {int(views[0][6].sum())} (workgroup form), "
                f"{int(views[-1][6].sum())} (one wave per strip)")


def test_forward_parity_fullsize_sampled(slr):
    """200k surfels on the structured scene at 128x1024 (the fwd+bwd workload)."""
    say("forward structured-200k-128x1024 sampled")
    sc, _ = synth.structured_scene(200000, 2)
    sensor = slr.make_sensor(128, 1024)
    r, d, Td, D, N, A = gpu_render(slr, sc, np.eye(4), sensor, (16, 16), 1 << 20)
    g = np.random.default_rng(0)
    pix = np.stack([g.integers(0, 128, 600), g.integers(0, 1024, 600)], 1).astype(np.int32)
    # plus every pixel of one tile at the horizon and one at the seam
    ii, jj = np.meshgrid(np.arange(48, 64), np.arange(0, 16), indexing="ij")
    pix = np.concatenate([pix, np.stack([ii.ravel(), jj.ravel()], 1).astype(np.int32)])
    assert_forward_close(D, N, A, sc, np.eye(4), sensor, pix)


# ---------------------------------------------------------------- backward
def check_backward(slr, sc, T, sensor, pix, gD, gN, gO, tiling=(16, 16), capacity=1 << 16):
    r, d, Td, D, N, A = gpu_render(slr, sc, T, sensor, tiling, capacity)
    H, W = sensor["height"], sensor["width"]
    GD = np.zeros((H, W), np.float32); GN = np.zeros((H, W, 3), np.float32); GO = np.zeros((H, W), np.float32)
    GD[pix[:, 0], pix[:, 1]] = gD; GN[pix[:, 0], pix[:, 1]] = gN; GO[pix[:, 0], pix[:, 1]] = gO
    g, dpose = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], Td,
                          torch.from_numpy(GD).to(DEV), torch.from_numpy(GN).to(DEV), torch.from_numpy(GO).to(DEV))
    torch.cuda.synchronize()
    ref = GC.oracle_backward(sc, T, sensor, pix, gD, gN, gO)
    GC.backward_verdict({k: v.cpu().numpy() for k, v in g.items()}, dpose.cpu().numpy(), ref)
    return r, d, Td, g, dpose


def clean_pixels(sc, T, sensor, pix=None):
    return GC.clean_pixels(sc, T, sensor, pix)


def test_backward_parity_shell_full_image(slr):
    say("backward shell-2k-64x512 all pixels")
    sc = synth.shell_scene(2000, 1)
    sensor = slr.make_sensor(64, 512)
    T = synth.perturbed_pose(1, 0.3, 5.0)
    pix = clean_pixels(sc, T, sensor)
    g = np.random.default_rng(1)
    P = pix.shape[0]
    check_backward(slr, sc, T, sensor, pix, g.normal(size=P).astype(np.float32),
                   g.normal(size=(P, 3)).astype(np.float32), g.normal(size=P).astype(np.float32))


def test_backward_parity_structured_posed(slr):
    say("backward structured-20k-posed-64x512 all pixels, 8x32 tiles, scalar forward, longest-first")
    sc, _ = synth.structured_scene(20000, 5)
    sensor = slr.make_sensor(64, 512)
    T = synth.circle_poses(8, 1)[2]
    pix = clean_pixels(sc, T, sensor)
    g = np.random.default_rng(2)
    P = pix.shape[0]
    check_backward(slr, sc, T, sensor, pix, g.normal(size=P).astype(np.float32),
                   g.normal(size=(P, 3)).astype(np.float32), g.normal(size=P).astype(np.float32), (8, 32, 2, 2))


def test_backward_parity_fullsize_dense(slr):
    """200k structured-scene surfels on the full 128x1024 image, random upstream
    gradients on every pixel whose decisions lie away from all thresholds."""
    say("backward structured-200k-128x1024 dense upstream")
    sc, _ = synth.structured_scene(200000, 2)
    sensor = slr.make_sensor(128, 1024)
    g = np.random.default_rng(3)
    pix = clean_pixels(sc, np.eye(4), sensor)
    P = pix.shape[0]
    assert P > 0.95 * 128 * 1024
    # one-wave forward with the workgroup backward, 32x8 tiles
    check_backward(slr, sc, np.eye(4), sensor, pix, g.normal(size=P).astype(np.float32),
                   g.normal(size=(P, 3)).astype(np.float32), g.normal(size=P).astype(np.float32), (32, 8, 3, 2, 1),
                   1 << 20)


@pytest.mark.parametrize("tiling", [(16, 16, 3, 2, 4), (4, 64, 1, 1, 4), (8, 32, 2, 3, 4)])
def test_backward_parity_fixed_order(slr, tiling):
    """The fixed-order backward (flushes written to per-pair slots, summed
    per surfel in binning order) against the oracle's analytic gradients on
    every clean pixel of the shell scene, whose surfels at the seam have
    pixel boxes of two column intervals; three tile shapes, every schedule."""
    say("backward shell-2k-64x512 fixed order", tiling)
    sc = synth.shell_scene(2000, 1)
    sensor = slr.make_sensor(64, 512)
    T = synth.perturbed_pose(1, 0.3, 5.0)
    pix = clean_pixels(sc, T, sensor)
    g = np.random.default_rng(1)
    P = pix.shape[0]
    r, *_ = check_backward(slr, sc, T, sensor, pix, g.normal(size=P).astype(np.float32),
                           g.normal(size=(P, 3)).astype(np.float32), g.normal(size=P).astype(np.float32), tiling)
    v = r.views()
    box = v["pixbox"].cpu().numpy()
    wraps = int(((v["counts"].cpu().numpy() > 0) & (box[:, 4] >= 0)).sum())
    say(f"   {wraps} binned surfels with a box wrapping past the seam")
    assert wraps > 0


def test_backward_batch_sizes_agree(slr):
    """The workgroup backward stages 128 or 192 records per LDS batch
    (slr_tiling.bwd_batch): the same pairs in the same per-pixel order, so the
    gradients agree up to the order of the float atomics and the per-tile
    pose partials; the forward is untouched."""
    sc, _ = synth.structured_scene(20000, 5)
    sensor = slr.make_sensor(64, 512)
    T = synth.circle_poses(8, 1)[2]
    g = np.random.default_rng(19)
    GD = torch.from_numpy(g.normal(size=(64, 512)).astype(np.float32)).to(DEV)
    GN = torch.from_numpy(g.normal(size=(64, 512, 3)).astype(np.float32)).to(DEV)
    GO = torch.from_numpy(g.normal(size=(64, 512)).astype(np.float32)).to(DEV)
    outs = []
    for batch in (192, 128):
        say("backward batch", batch)
        r, d, Td, D, N, A = gpu_render(slr, sc, T, sensor, (32, 8, 3, 2, 1, 0, batch), 1 << 20)
        gr, dp = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], Td, GD, GN, GO)
        torch.cuda.synchronize()
        outs.append((D, [gr[k].cpu().numpy().copy() for k in ("means", "quats", "log_scales", "logits")],
                     dp.cpu().numpy().copy()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])
    for a, b in zip(outs[0][1], outs[1][1]):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * float(np.abs(a).max()))
    np.testing.assert_allclose(outs[0][2], outs[1][2], rtol=1e-6, atol=1e-9 * float(np.abs(outs[0][2]).max()))


def test_backward_repeatable(slr):
    """The pose gradient is reduced from per-workgroup partials in a fixed
    order: with the one-wave form (whose record sums are deterministic) two
    backward calls give bit-identical pose gradients; the surfel gradients are
    added with float atomics and agree to rounding."""
    say("backward repeatability")
    sc, _ = synth.structured_scene(20000, 5)
    sensor = slr.make_sensor(64, 512)
    T = synth.circle_poses(8, 1)[2]
    g = np.random.default_rng(9)
    GD = torch.from_numpy(g.normal(size=(64, 512)).astype(np.float32)).to(DEV)
    GN = torch.from_numpy(g.normal(size=(64, 512, 3)).astype(np.float32)).to(DEV)
    GO = torch.from_numpy(g.normal(size=(64, 512)).astype(np.float32)).to(DEV)
    r, d, Td, D, N, A = gpu_render(slr, sc, T, sensor, (16, 16, 3), 1 << 20)
    outs = []
    for _ in range(2):
        gr, dp = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], Td, GD, GN, GO)
        torch.cuda.synchronize()
        outs.append(([gr[k].cpu().numpy().copy() for k in ("means", "quats", "log_scales", "logits")],
                     dp.cpu().numpy().copy()))
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    for a, b in zip(outs[0][0], outs[1][0]):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6 * float(np.abs(a).max()))


def test_pose_only_matches_full_backward(slr):
    say("backward pose-only vs full")
    sc = synth.shell_scene(3000, 6)
    sensor = slr.make_sensor(64, 512)
    T = synth.perturbed_pose(2, 0.5, 3.0)
    r, d, Td, D, N, A = gpu_render(slr, sc, T, sensor)
    gD = torch.randn(64, 512, device=DEV)
    _, p_full = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], Td, gD, None, None)
    g_none, p_only = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], Td, gD, None, None,
                                pose_only=True)
    assert g_none is None
    np.testing.assert_allclose(p_only.cpu().numpy(), p_full.cpu().numpy(), rtol=1e-6)


def test_autograd_function(slr):
    say("autograd wrapper")
    sc = synth.shell_scene(1500, 7)
    sensor = slr.make_sensor(64, 512)
    d = to_dev(sc)
    for k in d:
        d[k].requires_grad_(True)
    Td = pose_dev(synth.perturbed_pose(3))
    xi = torch.zeros(6, dtype=torch.float64, device=DEV, requires_grad=True)
    r = slr.Renderer(sensor)
    D, N, A = slr.render(d["means"], d["quats"], d["log_scales"], d["logits"], Td, r, xi)
    w = torch.randn_like(D)
    loss = (D * w).sum() + N.sum() + A.sum()
    loss.backward()
    g, dp = r.backward(d["means"].detach(), d["quats"].detach(), d["log_scales"].detach(), d["logits"].detach(), Td,
                       w, torch.ones_like(N), torch.ones_like(A))
    for k in ("means", "quats", "log_scales", "logits"):
        np.testing.assert_allclose(d[k].grad.cpu().numpy(), g[k].cpu().numpy(), rtol=1e-4, atol=1e-5)
    np.testing.assert_allclose(xi.grad.cpu().numpy(), dp.cpu().numpy(), rtol=1e-6)


def test_autograd_stale_render_raises(slr):
    """Two differentiable renders through one Renderer before backward: the
    workspace holds the second render's state, so the first one's backward
    must raise instead of returning gradients of the wrong binning; the second
    one's backward still works.  A non-zero xi is rejected."""
    say("autograd: stale render, non-zero xi")
    sc = synth.shell_scene(1500, 7)
    sensor = slr.make_sensor(64, 512)
    d = to_dev(sc)
    for k in d:
        d[k].requires_grad_(True)
    r = slr.Renderer(sensor)
    D1, _, _ = slr.render(d["means"], d["quats"], d["log_scales"], d["logits"], pose_dev(synth.perturbed_pose(3)), r)
    D2, _, _ = slr.render(d["means"], d["quats"], d["log_scales"], d["logits"], pose_dev(synth.perturbed_pose(4)), r)
    with pytest.raises(RuntimeError, match="rendered again"):
        D1.sum().backward(retain_graph=True)
    for k in d:
        d[k].grad = None
    D2.sum().backward()
    assert torch.isfinite(d["means"].grad).all() and d["means"].grad.abs().sum() > 0
    xi = torch.full((6,), 1e-3, dtype=torch.float64, device=DEV, requires_grad=True)
    with pytest.raises(ValueError, match="xi"):
        slr.render(d["means"], d["quats"], d["log_scales"], d["logits"], pose_dev(np.eye(4)), r, xi)


# ---------------------------------------------------------------- edge cases
def test_edge_cases(slr):
    say("edge: empty, all culled, capacity overflow")
    sensor = slr.make_sensor(64, 512)
    empty = {k: v[:0] for k, v in synth.shell_scene(1, 0).items()}
    r, d, Td, D, N, A = gpu_render(slr, empty, np.eye(4), sensor)
    assert not D.any() and not A.any() and not N.any()
    g, dp = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], Td, torch.ones(64, 512, device=DEV),
                       None, None)
    assert g["means"].numel() == 0 and not dp.cpu().numpy().any()
    # every surfel culled: inside the near range or non-finite
    sc = synth.shell_scene(50, 3)
    sc["means"][:] = 0.05
    sc["logits"][0] = np.nan
    r, d, Td, D, N, A = gpu_render(slr, sc, np.eye(4), sensor)
    assert not D.any() and r.K == 0
    g, dp = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], Td, torch.ones(64, 512, device=DEV),
                       None, None)
    assert not g["means"].cpu().numpy().any()
    # capacity overflow: explicit status with the needed K, then the renderer grows and succeeds
    sc = synth.shell_scene(2000, 1)
    ref = O.bin_surfels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], np.eye(4), sensor)
    r = slr.Renderer(sensor, (16, 16), capacity=16)
    dd = to_dev(sc)
    D, N, A = r.forward(dd["means"], dd["quats"], dd["log_scales"], dd["logits"], pose_dev(np.eye(4)))
    assert r.K == ref["K"] and r.capacity >= ref["K"]
    import ctypes as C
    s, t = slr._sensor(sensor), slr.Tiling(16, 16)
    sf = slr._surfels(dd["means"], dd["quats"], dd["log_scales"], dd["logits"])
    ws = torch.empty(slr.workspace_size(sensor, (16, 16), 2000, 10), dtype=torch.uint8, device=DEV)
    K = C.c_int64(0)
    Tp = pose_dev(np.eye(4))
    st = slr.lib().slr_render(C.byref(sf), C.c_void_p(Tp.data_ptr()), C.byref(s), C.byref(t),
                              C.c_void_p(ws.data_ptr()), ws.numel(), 10, C.c_void_p(D.data_ptr()),
                              C.c_void_p(N.data_ptr()), C.c_void_p(A.data_ptr()), C.byref(K), slr._stream())
    assert st == slr.SLR_E_CAPACITY and K.value == ref["K"]

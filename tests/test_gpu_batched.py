"""Batched form (many keyframes, one set of launches, HIP-graph capturable)
against the plain per-image form and the oracle, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2503_17491_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print("[gpu-batched]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def slr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_17491_amd import slr as S
    S.lib()
    return S


def dev_set(sc):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(DEV) for k, v in sc.items()}


def make_batch(slr, tiling=(16, 16), capacity=4 << 20, tiles=None):
    """tiles: per-frame tile shapes (None: the batch tiling's for every frame)."""
    shared, _ = synth.structured_scene(40000, 21)
    own = synth.shell_scene(5000, 22)
    sets = [dev_set(shared), dev_set(own)]
    poses = synth.circle_poses(3, 4)
    sizes = [(64, 512), (32, 1800), (128, 1024), (37, 300)]
    frames = []
    for k, (H, W) in enumerate(sizes):
        T = poses[k % 3] if k < 3 else synth.perturbed_pose(5)
        frames.append(dict(set=0 if k < 3 else 1, T_cw=torch.from_numpy(T).to(DEV), T_np=T,
                           sensor=slr.make_sensor(H, W), tile=None if tiles is None else tiles[k]))
    return sets, frames, [shared, own], slr.BatchRenderer(sets, frames, tiling, capacity)


def upstream(br, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    for u in br.up:
        for t in u:
            t.copy_(torch.randn(t.shape, generator=g))


def plain_frame(slr, st, f, tiling, up):
    r = slr.Renderer(f["sensor"], tiling, 1 << 20)
    D, N, A = r.forward(st["means"], st["quats"], st["log_scales"], st["logits"], f["T_cw"])
    g, dp = r.backward(st["means"], st["quats"], st["log_scales"], st["logits"], f["T_cw"], up[0], up[1], up[2])
    return (D, N, A), g, dp, r


@pytest.mark.parametrize("tiling", [(16, 16), (8, 32)])
def test_batched_matches_plain(slr, tiling):
    say("batched vs plain", tiling)
    sets, frames, _, br = make_batch(slr, tiling)
    upstream(br, 1)
    br.render()
    br.backward()
    torch.cuda.synchronize()
    K, over = br.pairs()
    assert over == 0 and K > 0
    sum_g = {k: torch.zeros_like(v) for k, v in br.grads[0].items()}
    Ksum = vis = 0
    for k, f in enumerate(frames):
        (D, N, A), g, dp, r = plain_frame(slr, sets[f["set"]], f, tiling, br.up[k])
        Ksum += r.K
        vis += int((r.views()["counts"] > 0).sum())
        # forward: bit-identical (same per-pixel contributor order and arithmetic)
        for a, b in zip((D, N, A), br.out[k]):
            assert torch.equal(a, b), f"frame {k}"
        np.testing.assert_allclose(br.dpose[k].cpu().numpy(), dp.cpu().numpy(), rtol=1e-6, atol=1e-9)
        if f["set"] == 0:
            for key in sum_g:
                sum_g[key] += g[key]
        else:
            for key in g:
                np.testing.assert_allclose(br.grads[1][key].cpu().numpy(), g[key].cpu().numpy(), rtol=1e-4,
                                           atol=1e-6)
    assert K == Ksum
    assert br.binned_records() == vis
    for key in sum_g:
        a, b = br.grads[0][key].cpu().numpy(), sum_g[key].cpu().numpy()
        scale = np.abs(b).max()
        assert np.abs(a - b).max() <= 1e-4 * scale, key


@pytest.mark.parametrize("batch", [128, 192, "wave"])
def test_queue_schedule_matches_longest(slr, batch):
    """The persistent workgroup backward (tiles taken from a device work queue
    by an occupancy-sized grid) against the same kernel launched one
    workgroup per tile: identical images, gradients equal up to the order of
    the float atomics, every tile visited once (pose rows and census)."""
    say("work-queue backward vs one workgroup per tile, batch", batch)
    res = []
    for sched in (slr.SCHEDULE_LONGEST, slr.SCHEDULE_QUEUE):
        # "wave": the one-wave backward (not persistent) after the persistent forward
        tiling = ((32, 8, slr.VARIANT_WAVE, sched, slr.VARIANT_WAVE, 0, 0) if batch == "wave"
                  else (32, 8, slr.VARIANT_WAVE, sched, slr.VARIANT_LDS, 0, batch))
        sets, frames, _, br = make_batch(slr, tiling)
        upstream(br, 3)
        for _ in range(2):   # a second step: the queue head is reset before every launch
            for g in br.grads:
                for t in g.values():
                    t.zero_()
            br.render()
            br.backward()
        torch.cuda.synchronize()
        res.append(([tuple(t.clone() for t in o) for o in br.out], [{k: v.clone() for k, v in g.items()} for g in br.grads],
                    [d.clone() for d in br.dpose], br.views()["census"].clone()))
    (o0, g0, d0, c0), (o1, g1, d1, c1) = res
    for a, b in zip(o0, o1):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    assert torch.equal(c0, c1)
    for ga, gb in zip(g0, g1):
        for key in ga:
            a, b = gb[key].cpu().numpy(), ga[key].cpu().numpy()
            assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max(), key
    for a, b in zip(d0, d1):
        np.testing.assert_allclose(b.cpu().numpy(), a.cpu().numpy(), rtol=1e-6, atol=1e-12)


def test_fixed_order_backward_is_deterministic(slr):
    """The fixed-order backward (bwd_variant 4): surfel and pose gradients bit
    for bit the same over repeated steps, every tile schedule (tile order,
    longest first, the persistent work queue) and every forward variant, with
    outputs overwritten whatever they held; equal to the float-atomic
    workgroup backward up to the order of its sums.  Also for a batch whose
    frames have their own tile shapes.  The one-wave backward's pose gradients
    (per-slot partial rows over a tile order that depends only on the list
    lengths) are also equal over re-renders."""
    det = slr.VARIANT_DETERMINISTIC

    def run(tiling, tiles=None, fill=0.0):
        sets, frames, _, br = make_batch(slr, tiling, tiles=tiles)
        upstream(br, 3)
        out = []
        for _ in range(2):
            for g in br.grads:
                for t in g.values():
                    t.fill_(fill)
            br.render()
            br.backward()
            torch.cuda.synchronize()
            out.append(([{k: v.clone() for k, v in g.items()} for g in br.grads], [d.clone() for d in br.dpose]))
        return out

    def same(a, b, what):
        for ga, gb in zip(a[0], b[0]):
            for key in ga:
                assert torch.equal(ga[key], gb[key]), (what, key)
        for da, db in zip(a[1], b[1]):
            assert torch.equal(da, db), (what, "pose")

    ref = None
    for fv, sched in ((3, 2), (3, 1), (3, 3), (1, 2), (2, 1)):
        say(f"fixed-order backward, forward variant {fv}, schedule {sched}")
        for got in run((16, 16, fv, sched, det), fill=7.0 if sched == 1 else 0.0):
            if ref is None:
                ref = got
            same(ref, got, (fv, sched))
    say("float-atomic workgroup backward on the same batch")
    atom = run((16, 16, 3, 2, slr.VARIANT_LDS, 0, 192))[0]
    for ga, gb in zip(ref[0], atom[0]):
        for key in ga:
            a, b = ga[key].cpu().numpy(), gb[key].cpu().numpy()
            assert np.isfinite(a).all()
            assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max(), key
    for da, db in zip(ref[1], atom[1]):
        np.testing.assert_allclose(da.cpu().numpy(), db.cpu().numpy(), rtol=1e-6, atol=1e-12)
    say("fixed-order backward with SLR_ACCUMULATE: a second backward adds exactly the same gradients")
    sets, frames, _, br = make_batch(slr, (16, 16, 3, 2, det))
    upstream(br, 3)
    br.render()
    br.backward()
    torch.cuda.synchronize()
    once = [{k: v.clone() for k, v in g.items()} for g in br.grads]
    br.backward(accumulate=True)
    torch.cuda.synchronize()
    for ga, gb in zip(once, br.grads):
        for key in ga:
            assert torch.equal(gb[key], ga[key] * 2), key
            assert torch.equal(ga[key], ref[0][0][key] if ga is once[0] else ref[0][1][key]), key
    say("fixed-order backward over ten keyframes of one set (the gather takes frames eight at a time)")
    shared, _ = synth.structured_scene(30000, 23)
    dset = dev_set(shared)
    poses10 = synth.circle_poses(10, 6)
    fr10 = [dict(set=0, T_cw=torch.from_numpy(T).to(DEV), sensor=slr.make_sensor(64, 512)) for T in poses10]
    outs = []
    for tl in ((16, 16, 3, 2, det), (16, 16, 3, 3, det), (16, 16, 3, 2, slr.VARIANT_LDS, 0, 192)):
        b10 = slr.BatchRenderer([dset], fr10, tl, 1 << 22)
        upstream(b10, 9)
        b10.render()
        b10.backward()
        torch.cuda.synchronize()
        outs.append({k: v.clone() for k, v in b10.grads[0].items()})
        del b10
    for key in outs[0]:
        assert torch.equal(outs[0][key], outs[1][key]), key
        a, b = outs[0][key].cpu().numpy(), outs[2][key].cpu().numpy()
        assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max(), key
    say("one-wave backward: pose gradients (fixed-order sums over tile slots) equal over re-renders")
    wave = run((16, 16, 3, 2, slr.VARIANT_WAVE))
    for da, db in zip(wave[0][1], wave[1][1]):
        assert torch.equal(da, db)
    say("fixed-order backward, mixed tile shapes")
    mixed = run((16, 16, 3, 3, det), tiles=MIXED_TILES)
    same(mixed[0], mixed[1], "mixed tiles")
    mixed2 = run((16, 16, 3, 1, det), tiles=MIXED_TILES)
    same(mixed[0], mixed2[0], "mixed tiles, tile order")


def test_invalid_surfels_counted_and_inert(slr):
    """Surfels with a non-finite parameter or a zero quaternion are culled in
    every frame that renders their set, counted in the batch's counter word,
    and take no part: finite images and gradients, zero gradients for them."""
    say("invalid surfels: counted, culled, zero gradients")
    sc = synth.shell_scene(5000, 41)
    bad = {3: ("means", 0, np.nan), 10: ("quats", None, 0.0), 17: ("log_scales", 1, np.inf),
           25: ("logits", None, np.nan), 31: ("quats", 2, -np.inf), 44: ("means", 2, np.inf)}
    for i, (key, col, val) in bad.items():
        if col is None:
            sc[key][i] = val
        else:
            sc[key][i, col] = val
    other = synth.shell_scene(3000, 42)
    sets = [dev_set(sc), dev_set(other)]
    poses = synth.circle_poses(3, 5)
    frames = [dict(set=0, T_cw=torch.from_numpy(poses[0]).to(DEV), sensor=slr.make_sensor(64, 512)),
              dict(set=1, T_cw=torch.from_numpy(poses[1]).to(DEV), sensor=slr.make_sensor(32, 1024)),
              dict(set=0, T_cw=torch.from_numpy(poses[2]).to(DEV), sensor=slr.make_sensor(64, 1024))]
    br = slr.BatchRenderer(sets, frames, (16, 16), 1 << 20)
    upstream(br, 5)
    br.render()
    br.backward()
    torch.cuda.synchronize()
    assert br.invalid_records() == 2 * len(bad)   # two frames render the set with the invalid surfels
    for o in br.out:
        for t in o:
            assert torch.isfinite(t).all()
    idx = torch.tensor(sorted(bad), device=DEV)
    for key, g in br.grads[0].items():
        assert torch.isfinite(g).all(), key
        assert (g[idx] == 0).all(), key
    for d in br.dpose:
        assert torch.isfinite(d).all()
    # a clean render counts none
    sets[0] = dev_set(synth.shell_scene(5000, 41))
    br2 = slr.BatchRenderer(sets, frames, (16, 16), 1 << 20)
    br2.render()
    torch.cuda.synchronize()
    assert br2.invalid_records() == 0


MIXED_TILES = [(8, 32), (4, 64), (32, 8), (16, 16)]


@pytest.mark.parametrize("bwd", [1, 3, 4])
def test_batched_mixed_tiles(slr, bwd):
    """Every frame with its own tile shape in one batch (one compositing launch
    over tiles of four shapes): each frame's sorted (tile, surfel) lists and
    tile ranges equal the oracle's binning at that shape, its images equal the
    plain form's at that shape bit for bit, its pose gradient and the set
    gradients match the plain form's; the images also match the oracle.  With
    the fixed-order backward (4) the gradients of the set only one frame
    renders equal the plain form's bit for bit."""
    from tests import gpu_checks as GC
    say("mixed tile shapes, backward form", bwd)
    sets, frames, host_sets, br = make_batch(slr, (16, 16, 3, 2, bwd), tiles=MIXED_TILES)
    upstream(br, 3)
    br.render()
    br.backward()
    torch.cuda.synchronize()
    K, over = br.pairs()
    assert over == 0 and K > 0
    v = br.views()
    st, sid, rg = v["sorted_tile"].cpu().numpy(), v["sorted_id"].cpu().numpy(), v["ranges"].cpu().numpy()
    sum_g = {k: torch.zeros_like(x) for k, x in br.grads[0].items()}
    p0 = 0
    for k, f in enumerate(frames):
        th, tw = MIXED_TILES[k]
        assert br.frame_tile(k) == (th, tw)
        sc = host_sets[f["set"]]
        ref = O.bin_surfels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], f["T_np"], f["sensor"], th, tw)
        n, t0, i0 = ref["K"], v["tile_off"][k], v["item_off"][k]
        nt = ref["ranges"].shape[0]
        np.testing.assert_array_equal(st[p0:p0 + n] - t0, ref["sorted_tile"])
        np.testing.assert_array_equal(sid[p0:p0 + n] - i0, ref["sorted_id"])
        mine = rg[t0:t0 + nt].copy()
        full = mine[:, 1] > mine[:, 0]
        mine[full] -= p0
        np.testing.assert_array_equal(mine, ref["ranges"])
        p0 += n
        (D, N, A), g, dp, r = plain_frame(slr, sets[f["set"]], f, (th, tw, 3, 2, bwd), br.up[k])
        for a, b in zip((D, N, A), br.out[k]):
            assert torch.equal(a, b), f"frame {k}"
        np.testing.assert_allclose(br.dpose[k].cpu().numpy(), dp.cpu().numpy(), rtol=1e-6, atol=1e-9)
        if f["set"] == 0:
            for key in sum_g:
                sum_g[key] += g[key]
        elif bwd == slr.VARIANT_DETERMINISTIC:   # the same flushes, summed in the same order
            for key in g:
                assert torch.equal(br.grads[1][key], g[key]), key
        else:   # the same sums up to the order of the float atomics
            for key in g:
                a, b = br.grads[1][key].cpu().numpy(), g[key].cpu().numpy()
                assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max(), key
        GC.forward_verdict(br.out[k][0].cpu().numpy(), br.out[k][1].cpu().numpy(), br.out[k][2].cpu().numpy(),
                           sc, f["T_np"], f["sensor"], label=f"mixed-tile frame {k} ({th}x{tw})")
    assert p0 == K
    for key in sum_g:
        a, b = br.grads[0][key].cpu().numpy(), sum_g[key].cpu().numpy()
        assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max(), key


def test_tune_frame_tiles(slr):
    """The per-class tile tuner gives every frame a supported shape, frames of
    one image size the same one, and the batch still renders what the plain
    form renders at those shapes."""
    say("per-class tile tuning")
    sets, frames, _, br = make_batch(slr, (16, 16, 3, 2, 1))
    upstream(br, 4)
    chosen = br.tune_frame_tiles(reps=1)
    shapes = {(16, 16), (8, 32), (32, 8), (4, 64)}
    for k, f in enumerate(frames):
        hw = (f["sensor"]["height"], f["sensor"]["width"])
        assert chosen[hw] in shapes and br.frame_tile(k) == chosen[hw]
    br.render()
    torch.cuda.synchronize()
    for k, f in enumerate(frames):
        (D, N, A), _, _, _ = plain_frame(slr, sets[f["set"]], f, br.frame_tile(k) + (3, 2, 1), br.up[k])
        for a, b in zip((D, N, A), br.out[k]):
            assert torch.equal(a, b), f"frame {k}"


def test_batched_forward_matches_oracle(slr):
    say("batched vs oracle")
    sets, frames, host_sets, br = make_batch(slr)
    br.render()
    torch.cuda.synchronize()
    EX = O.FLAG_SUPPORT | O.FLAG_NEAR | O.FLAG_AMIN | O.FLAG_TSTOP
    for k, f in enumerate(frames):
        sc = host_sets[f["set"]]
        if f["sensor"]["height"] * f["sensor"]["width"] > 70000:
            g = np.random.default_rng(k)
            pix = np.stack([g.integers(0, f["sensor"]["height"], 3000), g.integers(0, f["sensor"]["width"], 3000)],
                           1).astype(np.int32)
        else:
            pix = O.all_pixels(f["sensor"])
        ref = O.render_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], f["T_np"], f["sensor"], pix)
        D = br.out[k][0].cpu().numpy()[pix[:, 0], pix[:, 1]].astype(np.float64)
        A = br.out[k][2].cpu().numpy()[pix[:, 0], pix[:, 1]].astype(np.float64)
        ok = (ref["flags"] & EX) == 0
        assert ok.mean() > 0.99
        eD = np.abs(D - ref["depth"]) / np.maximum(np.abs(ref["depth"]), 1.0)
        eA = np.abs(A - ref["alpha"]) / np.maximum(ref["alpha"], 1e-2)
        say(f"frame {k}: depth {eD[ok].max():.2e} alpha {eA[ok].max():.2e}")
        assert eD[ok].max() <= 1e-4 and eA[ok].max() <= 1e-4


def test_batched_overflow_flag_then_grow(slr):
    say("batched overflow")
    sets, frames, _, br = make_batch(slr, capacity=1000)
    br.render()
    K, over = br.pairs()
    assert over == K and K > 1000
    assert not any(o[0].any().item() for o in br.out)  # nothing was binned
    assert br.ensure_capacity()
    br.render()
    K2, over2 = br.pairs()
    assert over2 == 0 and K2 == K
    assert any(o[0].any().item() for o in br.out)


@pytest.mark.parametrize("bwd", [0, 4])
def test_graph_capture_replays_match_eager(slr, bwd):
    """Render + backward captured in one HIP graph and replayed with eager work
    in between: images equal the eager ones bit for bit, gradients to the
    order of the float atomics, or bit for bit with the fixed-order backward
    (4), whose mask and rank buffers are cleared by fill kernels inside the
    graph."""
    say("graph capture, backward form", bwd)
    sets, frames, _, br = make_batch(slr, (16, 16, 3, 2, bwd))
    upstream(br, 2)
    br.render()
    br.backward()
    torch.cuda.synchronize()
    ref_out = [tuple(t.clone() for t in o) for o in br.out]
    ref_g = {k: v.clone() for k, v in br.grads[0].items()}
    ref_p = [p.clone() for p in br.dpose]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        br.render()
        br.backward()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s):
        br.render()
        br.backward()
    for rep in range(3):
        for o in br.out:  # eager work between replays
            for t in o:
                t.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for o, r in zip(br.out, ref_out):
            for a, b in zip(o, r):
                assert torch.equal(a, b), f"replay {rep}"
        for k in ref_g:
            if bwd == 4:
                assert torch.equal(br.grads[0][k], ref_g[k]), (rep, k)
                continue
            d = (br.grads[0][k] - ref_g[k]).abs().max().item()
            assert d <= 1e-4 * ref_g[k].abs().max().item(), (rep, k)
        for p, r in zip(br.dpose, ref_p):
            if bwd == 4:
                assert torch.equal(p, r), rep
                continue
            np.testing.assert_allclose(p.cpu().numpy(), r.cpu().numpy(), rtol=1e-6, atol=1e-9)


def test_graph_step_with_loss_replays_match_eager(slr):
    """The benchmark's step (render, loss over all keyframes in one launch,
    backward) captured once and replayed: every replay matches the eager step
    (images and loss gradients bit for bit, surfel and pose gradients to the
    atomics' order, the loss to its summation order)."""
    say("graph capture with the multi-image loss")
    sets, frames, _, br = make_batch(slr)
    g = torch.Generator(device="cpu").manual_seed(3)
    tg = []
    for f in frames:
        H, W = int(f["sensor"]["height"]), int(f["sensor"]["width"])
        Dt = (torch.rand(H, W, generator=g) * 30.0) * (torch.rand(H, W, generator=g) > 0.2)
        Nt = torch.nn.functional.normalize(torch.randn(H, W, 3, generator=g), dim=-1)
        tg.append((Dt.to(DEV), Nt.to(DEV), 1.0 / max(int((Dt > 0).sum()), 1)))
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)

    def step():
        br.render()
        slr.loss_l1_normal_frames([(br.out[k][0], br.out[k][1], Dt, Nt, w, w, br.up[k][0], br.up[k][1])
                                   for k, (Dt, Nt, w) in enumerate(tg)], loss)
        br.backward()

    step()
    torch.cuda.synchronize()
    ref_out = [tuple(t.clone() for t in o) for o in br.out]
    ref_up = [(u[0].clone(), u[1].clone()) for u in br.up]
    ref_g = {k: v.clone() for k, v in br.grads[0].items()}
    ref_p = [p.clone() for p in br.dpose]
    ref_loss = loss.item()
    assert ref_loss > 0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=s):
        step()
    for rep in range(3):
        loss.zero_()   # eager work between replays
        for o in br.out:
            for t in o:
                t.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for o, r in zip(br.out, ref_out):
            for a, b in zip(o, r):
                assert torch.equal(a, b), f"replay {rep}"
        for u, r in zip(br.up, ref_up):
            assert torch.equal(u[0], r[0]) and torch.equal(u[1], r[1]), f"replay {rep}"
        assert abs(loss.item() - ref_loss) <= 1e-9 * ref_loss, rep
        for k in ref_g:
            d = (br.grads[0][k] - ref_g[k]).abs().max().item()
            assert d <= 1e-4 * ref_g[k].abs().max().item(), (rep, k)
        for p, r in zip(br.dpose, ref_p):
            np.testing.assert_allclose(p.cpu().numpy(), r.cpu().numpy(), rtol=1e-6, atol=1e-9)


def test_autotune_picks_a_candidate(slr):
    say("autotune")
    sets, frames, _, br = make_batch(slr, (16, 16))
    upstream(br, 3)
    cands = [(16, 16, 3, 2, 3), (8, 32, 3, 2, 1), (16, 16, 1, 2, 1)]
    ms = br.autotune(cands, reps=2)
    # each candidate keeps the renderer's box mode (0 here) as its sixth entry
    assert set(ms) == {c + (0,) for c in cands} and all(v > 0 for v in ms.values())
    assert br.tiling == min(ms, key=ms.get)
    br.render()
    torch.cuda.synchronize()
    ref = slr.BatchRenderer(sets, frames, br.tiling, 4 << 20)
    ref.render()
    torch.cuda.synchronize()
    for a, b in zip(br.out, ref.out):
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    # an invalid candidate is refused before anything runs
    with pytest.raises(slr.SlrError):
        br.autotune([(16, 16, 3, 2, 3), (12, 12, 3, 2, 3)])

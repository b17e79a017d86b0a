"""The benchmark's other workloads (``python bench.py --config NAME``), one JSON
line each.  The default ``bench.py`` run is the headline workload; these are
the remaining configurations of the measurement plan:

  fwd-2k          2,000 shell surfels (seed 1), 64x512, identity pose: forward
                  only, latency of one render (plain form, and the batched form
                  of one frame replayed from a HIP graph).
  map-200k        200,000 structured-scene surfels (seed 2), 128x1024: forward
                  + fused L1 range / normal loss against the analytic ray-cast
                  target + backward, plain and batched (one frame, graph) iter/s.
  odometry-300k   300,000 shell surfels (seed 3), 128x1024, target rendered at
                  the identity, start 0.5 m / 3 deg away (Sec. 3.3.3); 20
                  pose-only iterations of Adam on the se(3) increment, and 20
                  damped Gauss-Newton (Levenberg-Marquardt, Huber 0.1 m)
                  iterations from the rasterizer's normal equations; iter/s and
                  the final pose error of each (FP64 pose accumulation on the
                  host).
  batch-uneven    eight keyframes of uneven sizes (64x1024 ... 32x1024), each
                  with its own structured scene of 50k-500k surfels (seeds
                  40-47) and its own ray-cast target: batched (one launch per
                  pass, HIP graph, autotuned forms, a tile shape per image-size
                  class) against the plain per-keyframe loop.
  map-2m-adam     2,000,000 urban-scene surfels (seed 5), 128x2048: 100
                  iterations of forward + loss + backward + fused Adam on the
                  raw parameters.
  n-sweep         the map-200k generator (seed 6) at N = 50k ... 2M, 128x1024:
                  fwd + bwd iter/s (plain and batched) and workspace bytes.

Every line also carries the FP64 oracle timed on the host cores on a stated
pixel sample (one thread and all threads), scaled to the workload.
"""
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _omp_threads(n):
    """Set the OpenMP thread count of the oracle's parallel regions (libgomp)."""
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except OSError:
        pass


def oracle_baseline(sc, T, sensor, pixels_per_iter, budget_s=6.0, backward=True):
    """FP64 oracle (angular-cull mode) on a random pixel sample of one frame,
    forward (+ backward with a unit range gradient), one thread and all
    threads; scaled to `pixels_per_iter` pixels per iteration."""
    import oracle as O
    H, W = int(sensor["height"]), int(sensor["width"])
    all_threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    g = np.random.default_rng(7)
    out = {}
    for label, threads in (("one_thread", 1), ("all_threads", all_threads)):
        _omp_threads(threads)
        P, t1 = 64, 0.0
        for _ in range(4):
            pix = np.stack([g.integers(0, H, P), g.integers(0, W, P)], 1).astype(np.int32)
            t = time.perf_counter()
            O.render_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor, pix, cull=True)
            if backward:
                O.backward_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor, pix,
                                  np.ones(P), None, None, cull=True)
            t1 = time.perf_counter() - t
            if t1 >= 0.5 * budget_s or P >= H * W:
                break
            P = min(H * W, max(P + 1, int(P * budget_s / max(t1, 1e-3))))
        s_iter = t1 / P * pixels_per_iter
        out[label] = {"value": round(1.0 / s_iter, 6), "unit": "iter/s", "cores": threads,
                      "sample": f"{P} random pixels in {t1:.2f}s (includes the cull index over {len(sc['logits'])} "
                                f"surfels), scaled to {pixels_per_iter} pixels"}
    _omp_threads(all_threads)
    return {"kind": "oracle", "fwd_and_bwd": bool(backward), **out}


def _time(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / steps


def _graph(torch, fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fn()
    return g


def _dev(torch, sc):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in sc.items()}


def _zero_upstream(br):
    """The autotuner runs with upstream gradients of one; a step's range and
    normal gradients come from the loss, and the opacity channel has none."""
    for u in br.up:
        for x in u:
            x.zero_()


def _batch_step(slr, br, tgts, loss):
    br.render()
    slr.loss_l1_normal_frames([(br.out[k][0], br.out[k][1], t["Dt"], t["Nt"], t["w"], t["w"], br.up[k][0],
                                br.up[k][1]) for k, t in enumerate(tgts)], loss)
    br.backward()


def _target(torch, targets, prims, sensor, T, seed):
    Dt, Nt = targets.raycast(prims, sensor, T, seed=seed)
    return dict(Dt=torch.from_numpy(Dt).cuda(), Nt=torch.from_numpy(Nt).cuda(),
                w=1.0 / max(int((Dt > 0).sum()), 1))


def _plain_fwd_bwd(slr, r, d, T, t, scratch, loss):
    D, N, _ = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], T)
    gD, gN = scratch
    slr.loss_l1_normal(D, N, t["Dt"], t["Nt"], t["w"], t["w"], gD, gN, loss)
    return r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], T, gD, gN, None)


def config_fwd_2k(torch, slr, synth, targets, args):
    sc = synth.shell_scene(2000, 1)
    sensor = slr.make_sensor(64, 512)
    d = _dev(torch, sc)
    T = torch.eye(4, dtype=torch.float64, device="cuda")
    r = slr.Renderer(sensor, (16, 16), 1 << 16)
    plain = _time(torch, lambda: r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], T), args.steps,
                  args.warmup)
    br = slr.BatchRenderer([d], [dict(set=0, T_cw=T, sensor=sensor)], (16, 16), capacity=1 << 16)
    g = _graph(torch, br.render)
    batched = _time(torch, g.replay, args.steps, args.warmup)
    K, over = br.pairs()
    cpu = oracle_baseline(sc, np.eye(4), sensor, 64 * 512, backward=False)
    return {"metric": "forward latency, 2k surfels, 64x512", "value": round(plain * 1e3, 4), "unit": "ms",
            "higher_is_better": False, "n_gpus": 1, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "2000 shell surfels (seed 1), 64x512, identity pose, forward only",
                       "plain_ms": round(plain * 1e3, 4), "plain_iter_s": round(1 / plain, 1),
                       "batched_graph_ms": round(batched * 1e3, 4), "batched_iter_s": round(1 / batched, 1),
                       "pairs": K},
            "cpu_baseline": cpu}


def config_map_200k(torch, slr, synth, targets, args, n=200_000, seed=2):
    sc, prims = synth.structured_scene(n, seed)
    sensor = slr.make_sensor(128, 1024)
    d = _dev(torch, sc)
    T = torch.eye(4, dtype=torch.float64, device="cuda")
    t = _target(torch, targets, prims, sensor, np.eye(4), seed=200 + seed)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    scratch = (torch.empty(128, 1024, device="cuda"), torch.empty(128, 1024, 3, device="cuda"))
    frames = [dict(set=0, T_cw=T, sensor=sensor)]
    br = slr.BatchRenderer([d], frames, slr.TUNE_CANDIDATES[0], capacity=max(4 << 20, 16 * n))
    for u in br.up:
        for x in u:
            x.fill_(1.0)
    br.autotune(reps=3)
    _zero_upstream(br)
    tiling = tuple(br.tiling)
    _batch_step(slr, br, [t], loss)
    if br.ensure_capacity():
        _batch_step(slr, br, [t], loss)
    K, _ = br.pairs()
    best_plain = None
    for bv in (slr.VARIANT_LDS, slr.VARIANT_WAVE):   # the plain form's backward form by timing (untimed)
        cand = tiling[:4] + (bv,) + tiling[5:]
        r = slr.Renderer(sensor, cand, capacity=max(1 << 20, int(1.3 * K)))
        dt = _time(torch, lambda: _plain_fwd_bwd(slr, r, d, T, t, scratch, loss), 3, 1)
        if best_plain is None or dt < best_plain[0]:
            best_plain = (dt, cand, r)
    r = best_plain[2]
    plain = _time(torch, lambda: _plain_fwd_bwd(slr, r, d, T, t, scratch, loss), args.steps, args.warmup)
    g = _graph(torch, lambda: _batch_step(slr, br, [t], loss))
    batched = _time(torch, g.replay, args.steps, args.warmup)
    ws = int(br.ws.numel())
    return dict(plain_iter_s=1 / plain, batched_iter_s=1 / batched, pairs=K, tiling=list(tiling),
                plain_tiling=list(best_plain[1]), workspace_bytes=ws, sc=sc, sensor=sensor)


def _pose_err(T, Tt):
    D = np.linalg.inv(Tt) @ T
    ang = math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(D[:3, :3]) - 1) / 2))))
    return float(np.linalg.norm(D[:3, 3])), ang


def _hat(x):
    M = np.zeros((4, 4))
    r, p = x[:3], x[3:]
    M[:3, :3] = [[0, -p[2], p[1]], [p[2], 0, -p[0]], [-p[1], p[0], 0]]
    M[:3, 3] = r
    return M


def _expm(M):
    """Matrix exponential of a 4x4 se(3) element (scaling and squaring of the series)."""
    k = max(0, int(math.ceil(math.log2(max(np.abs(M).max(), 1e-300)))) + 4)
    A = M / (2 ** k)
    E, term = np.eye(4), np.eye(4)
    for i in range(1, 20):
        term = term @ A / i
        E = E + term
    for _ in range(k):
        E = E @ E
    return E


def config_odometry(torch, slr, synth, targets, args):
    sc = synth.shell_scene(300_000, 3)
    sensor = slr.make_sensor(128, 1024)
    d = _dev(torch, sc)
    a4 = (d["means"], d["quats"], d["log_scales"], d["logits"])
    T_true = np.eye(4)
    tiling = (16, 16, slr.VARIANT_WAVE, slr.SCHEDULE_LONGEST, slr.VARIANT_WAVE)
    r = slr.Renderer(sensor, tiling, capacity=4 << 20)
    Dt, _, Ot = r.forward(*a4, torch.from_numpy(T_true).cuda())
    Dt, Ot = Dt.clone(), Ot.clone()
    m = (Ot > 0.5).float()
    cnt = float(m.sum())
    Nz = torch.zeros(128, 1024, 3, device="cuda")
    T0 = synth.perturbed_pose(3, 0.5, 3.0)
    e0 = _pose_err(T0, T_true)
    # the tile shape of the single-frame loop by timing render + normal equations at the start pose
    # (untimed; the images do not depend on it)
    best = None
    Td0 = torch.from_numpy(T0).cuda()
    for th, tw in ((16, 16), (32, 8), (8, 32)):
        cand = (th, tw, slr.VARIANT_WAVE, slr.SCHEDULE_LONGEST, slr.VARIANT_WAVE)
        rr = slr.Renderer(sensor, cand, capacity=4 << 20)

        def probe(rr=rr):
            D0, _, _ = rr.forward(*a4, Td0)
            rr.pose_gn(*a4, Td0, D0, Dt, m, 0.1)

        dt = _time(torch, probe, 5, 2)
        if best is None or dt < best[0]:
            best = (dt, cand, rr)
    tiling, r = best[1], best[2]
    res = {"tile": f"{tiling[0]}x{tiling[1]}"}
    # Adam on the se(3) increment: gradient of mean |D - D_t| over O_t > 0.5
    T = T0.copy()
    mom, vel = np.zeros(6), np.zeros(6)
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-12
    Dtm = torch.where(m > 0, Dt, torch.zeros_like(Dt)).contiguous()
    gD, gN = torch.empty_like(Dt), torch.empty_like(Nz)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(1, 21):
        Td = torch.from_numpy(T).cuda()
        D, N, _ = r.forward(*a4, Td)
        slr.loss_l1_normal(D, N, Dtm, Nz, 1.0 / cnt, 0.0, gD, gN, loss)
        _, dp = r.backward(*a4, Td, gD, None, None, pose_only=True)
        g = dp.cpu().numpy()
        mom = b1 * mom + (1 - b1) * g
        vel = b2 * vel + (1 - b2) * g * g
        step = lr * (mom / (1 - b1 ** it)) / (np.sqrt(vel / (1 - b2 ** it)) + eps)
        T = _expm(-_hat(-step)) @ T   # T_wc <- T_wc exp(-step): a descent step on delta
    torch.cuda.synchronize()
    res["adam"] = {"iter_s": round(20 / (time.perf_counter() - t0), 2), "lr": lr,
                   "final_error_m_deg": [round(x, 5) for x in _pose_err(T, T_true)]}
    # Gauss-Newton from the rasterizer's normal equations, Huber-robust (Sec. 3.3.3),
    # with Levenberg-Marquardt damping: a step that raises the cost is not taken
    # and the damping grows (each iteration = one render + normal equations)
    T = T0.copy()
    lam, huber_k = 1e-4, 0.1
    taken = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Td = torch.from_numpy(T).cuda()
    D, _, _ = r.forward(*a4, Td)
    Hm, gv, c = r.pose_gn(*a4, Td, D, Dt, m, huber_k)
    Hn, gn, cost = Hm.cpu().numpy(), gv.cpu().numpy(), float(c.cpu())
    for it in range(20):
        delta = -np.linalg.solve(Hn + lam * np.diag(np.diag(Hn)), gn)
        Tn = _expm(-_hat(delta)) @ T
        Td = torch.from_numpy(Tn).cuda()
        D, _, _ = r.forward(*a4, Td)
        Hm, gv, c = r.pose_gn(*a4, Td, D, Dt, m, huber_k)
        cn = float(c.cpu())
        if cn < cost:
            T, cost, Hn, gn = Tn, cn, Hm.cpu().numpy(), gv.cpu().numpy()
            lam = max(lam / 3.0, 1e-7)
            taken += 1
        else:
            lam *= 10.0
    torch.cuda.synchronize()
    res["gauss_newton"] = {"iter_s": round(21 / (time.perf_counter() - t0), 2), "huber_k": huber_k,
                           "steps_taken": taken,
                           "final_error_m_deg": [round(x, 6) for x in _pose_err(T, T_true)]}
    cpu = oracle_baseline(sc, T0, sensor, 128 * 1024, backward=True)
    return {"metric": "pose-only iter/s, 300k surfels, 128x1024, 20 iterations from 0.5 m / 3 deg",
            "value": res["gauss_newton"]["iter_s"], "unit": "iter/s", "higher_is_better": True, "n_gpus": 1,
            "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "300000 shell surfels (seed 3), 128x1024, target rendered at the identity, "
                                   "start 0.5 m / 3 deg (seed 3)", "start_error_m_deg": [round(x, 4) for x in e0],
                       **res},
            "cpu_baseline": cpu}


def config_batch_uneven(torch, slr, synth, targets, args):
    kfs = synth.uneven_batch(40)
    sets, frames, tgts, sensors = [], [], [], []
    for i, k in enumerate(kfs):
        sensor = slr.make_sensor(k["H"], k["W"])
        sensors.append(sensor)
        sets.append(_dev(torch, k["surfels"]))
        T = torch.eye(4, dtype=torch.float64, device="cuda")
        frames.append(dict(set=i, T_cw=T, sensor=sensor))
        tgts.append(_target(torch, targets, k["prims"], sensor, np.eye(4), seed=400 + i))
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    br = slr.BatchRenderer(sets, frames, slr.TUNE_CANDIDATES[0], capacity=24 << 20)
    for u in br.up:
        for x in u:
            x.fill_(1.0)
    tune = br.autotune(reps=3)
    _zero_upstream(br)
    uniform = tuple(br.tiling)
    per_class = br.tune_frame_tiles(reps=3)
    _zero_upstream(br)
    log("uneven batch tiling", uniform, "per class", per_class)
    _batch_step(slr, br, tgts, loss)
    if br.ensure_capacity():
        _batch_step(slr, br, tgts, loss)
    K, _ = br.pairs()
    g = _graph(torch, lambda: _batch_step(slr, br, tgts, loss))
    batched = _time(torch, g.replay, args.steps, args.warmup)
    # the same batch with one tile shape for every frame
    br.set_frame_tiles([None] * len(frames))
    _batch_step(slr, br, tgts, loss)
    g2 = _graph(torch, lambda: _batch_step(slr, br, tgts, loss))
    batched_uniform = _time(torch, g2.replay, args.steps, args.warmup)
    # plain loop: each keyframe with its class's tile shape and the faster backward form
    scratch = [(torch.empty(s["height"], s["width"], device="cuda"),
                torch.empty(s["height"], s["width"], 3, device="cuda")) for s in sensors]
    best = None
    for bv in (slr.VARIANT_LDS, slr.VARIANT_WAVE):
        rs = [slr.Renderer(s, per_class[(s["height"], s["width"])] + uniform[2:4] + (bv,) + uniform[5:],
                           capacity=4 << 20) for s in sensors]

        def plain_step():
            for i, r in enumerate(rs):
                _plain_fwd_bwd(slr, r, sets[i], frames[i]["T_cw"], tgts[i], scratch[i], loss)
        dt = _time(torch, plain_step, 3, 1)
        if best is None or dt < best[0]:
            best = (dt, bv, plain_step)
    plain = _time(torch, best[2], args.steps, args.warmup)
    n = [int(k["surfels"]["logits"].shape[0]) for k in kfs]
    return {"metric": "fwd+bwd iter/s, 8 uneven keyframes (50k-500k surfels each); batched vs plain",
            "value": round(1 / batched, 3), "unit": "iter/s", "higher_is_better": True, "n_gpus": 1,
            "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "keyframes " + ", ".join(f"{k['H']}x{k['W']}" for k in kfs)
                                   + f"; structured scenes of {n} surfels (seeds 40-47); ray-cast targets",
                       "batched_iter_s": round(1 / batched, 3), "batched_uniform_tile_iter_s":
                           round(1 / batched_uniform, 3), "plain_iter_s": round(1 / plain, 3),
                       "tiling": list(uniform),
                       "tile_per_class": {f"{h}x{w}": f"{a}x{b}" for (h, w), (a, b) in per_class.items()},
                       "plain_bwd_variant": best[1], "pairs_per_step": K,
                       "autotune_ms": {f"{c[0]}x{c[1]}/f{c[2]}/b{c[4]}": round(v, 3) for c, v in tune.items()}}}


def config_map_2m(torch, slr, synth, targets, args):
    sc, prims = synth.structured_scene(2_000_000, 5, kind="urban")
    sensor = slr.make_sensor(128, 2048)
    d = _dev(torch, sc)
    T = torch.eye(4, dtype=torch.float64, device="cuda")
    t = _target(torch, targets, prims, sensor, np.eye(4), seed=500)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    br = slr.BatchRenderer([d], [dict(set=0, T_cw=T, sensor=sensor)], slr.TUNE_CANDIDATES[0], capacity=16 << 20)
    for u in br.up:
        for x in u:
            x.fill_(1.0)
    br.autotune(reps=3)
    _zero_upstream(br)
    _batch_step(slr, br, [t], loss)
    if br.ensure_capacity():
        _batch_step(slr, br, [t], loss)
    n = d["logits"].shape[0]
    mom = torch.zeros(n, 10, device="cuda")
    vel = torch.zeros(n, 10, device="cuda")
    lr = dict(means=1e-3, quats=1e-3, log_scales=5e-3, logits=5e-2)
    iters = 100
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(1, iters + 1):
        loss.zero_()
        _batch_step(slr, br, [t], loss)
        slr.adam_step(d, br.grads[0], mom, vel, lr, it)
        if it in (1, iters):
            losses.append(float(loss.item()))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    K, over = br.pairs()
    cpu = oracle_baseline(sc, np.eye(4), sensor, 128 * 2048, budget_s=6.0, backward=True)
    return {"metric": "fwd+bwd+Adam iter/s, 2M urban surfels, 128x2048, 100 iterations", "value": round(iters / dt, 3),
            "unit": "iter/s", "higher_is_better": True, "n_gpus": 1, "dtype": "f32+f64", "data": "synthetic",
            "config": {"workload": "2000000 urban-scene surfels (seed 5), 128x2048, ray-cast target, fused "
                                   "L1 range + normal loss, Adam (lr 1e-3/1e-3/5e-3/5e-2) on the raw parameters",
                       "tiling": list(br.tiling), "pairs_last_iter": K, "overflowed": int(over),
                       "loss_first_last": [round(x, 5) for x in losses],
                       "note": "eager launches (the Adam step count changes every iteration), no host sync"},
            "cpu_baseline": cpu}


def config_n_sweep(torch, slr, synth, targets, args):
    rows = []
    for n in (50_000, 100_000, 200_000, 300_000, 500_000, 1_000_000, 2_000_000):
        r = config_map_200k(torch, slr, synth, targets, args, n=n, seed=6)
        rows.append({"n": n, "plain_iter_s": round(r["plain_iter_s"], 2), "batched_iter_s": round(r["batched_iter_s"], 2),
                     "pairs": r["pairs"], "workspace_bytes": r["workspace_bytes"], "tiling": r["tiling"]})
        log("n-sweep", rows[-1])
        torch.cuda.empty_cache()
    return {"metric": "fwd+bwd iter/s vs surfel count, 128x1024 (structured scene, seed 6)",
            "value": rows[-1]["batched_iter_s"], "unit": "iter/s", "higher_is_better": True, "n_gpus": 1,
            "dtype": "f32+f64", "data": "synthetic", "config": {"workload": "200k-generator scenes at N = 50k ... 2M, 128x1024", "rows": rows}}


def run(name, args):
    import torch

    from paper_2503_17491_amd import slr, synth, targets
    slr.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if name == "map-200k":
        r = config_map_200k(torch, slr, synth, targets, args)
        cpu = oracle_baseline(r["sc"], np.eye(4), r["sensor"], 128 * 1024, backward=True)
        out = {"metric": "fwd+bwd iter/s, 200k surfels, 128x1024", "value": round(r["batched_iter_s"], 3),
               "unit": "iter/s", "higher_is_better": True, "n_gpus": 1, "dtype": "f32+f64", "data": "synthetic",
               "config": {"workload": "200000 structured-scene surfels (seed 2), 128x1024, fused L1 range + "
                                      "normal loss against the ray-cast target",
                          "batched_iter_s": round(r["batched_iter_s"], 3), "plain_iter_s": round(r["plain_iter_s"], 3),
                          "pairs": r["pairs"], "tiling": r["tiling"], "plain_tiling": r["plain_tiling"],
                          "workspace_bytes": r["workspace_bytes"]},
               "cpu_baseline": cpu}
    else:
        fn = {"fwd-2k": config_fwd_2k, "odometry-300k": config_odometry, "batch-uneven": config_batch_uneven, "map-2m-adam": config_map_2m,
              "n-sweep": config_n_sweep}[name]
        out = fn(torch, slr, synth, targets, args)
    out["steps"], out["warmup"] = args.steps, args.warmup
    print(json.dumps(out), flush=True)

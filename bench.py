#!/usr/bin/env python
"""Throughput of the spherical surfel rasterizer's fwd+bwd on one MI355X.

Workload: 1,000,000 surfels on the structured synthetic scene (ground, 30
boxes, 20 cylinders; seed 0), eight 128x1024 keyframes on a 5 m circle at
sensor height (random yaw, seed 0) sharing that map, range + normal L1 loss
against analytic ray-cast targets.  One step = for every keyframe: render
(projection, bounding box, binning with the radix sort, compositing), fused
loss and gradients, backward (compositing backward, per-surfel gradients
summed over the keyframes, pose gradient per keyframe).  Inputs are resident
in HBM before the timed region.

Prints one JSON line: the metric, per-stage times, the roofline of the dominant
compositing kernel and the FP64 oracle's CPU baseline.
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd iter/s, 128x1024 range image, 1M surfels; batched vs plain"
N_SURFELS = 1_000_000
N_KF = 8
H, W = 128, 1024

# Algorithmic FLOPs (FMA = 2) per unit of compositing work.
FWD_EVAL_FLOPS = 18      # 3 three-term FP64 dot products + support bound, reciprocal, range
FWD_CONTRIB_FLOPS = 20   # Gaussian, alpha, blending of range, normal and opacity
BWD_EVAL_FLOPS = 18
BWD_CONTRIB_FLOPS = 70   # recompute alpha, transmittance recovery, dL/dalpha, 14 partials
GN_CONTRIB_FLOPS = 96    # recompute alpha, reverse step with a unit range gradient, 6-vector Jacobian update
PEAK_TFLOPS = 78.6       # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA), unpacked FP32 / FP64
PEAK_HBM_GBS = 8000.0
TUNE_MARGIN = 0.01       # autotune times closer than this are a tie (run-to-run spread is about 1 %)
SINGLE_FRAME_SHAPES = ((16, 16), (32, 8), (8, 32))   # tile shapes the single-frame forms are timed on
# Algorithmic HBM bytes of the compositing launches: per (tile, surfel) pair the
# 4-B id and the 64-B compositing record are gathered (+52 B of gradient
# accumulation in the backward); per pixel the forward writes 20 B of outputs
# and 8 B of state, the backward reads 20 B of upstream gradients and 8 B of state.
FWD_PAIR_BYTES, FWD_PIXEL_BYTES = 68, 28
BWD_PAIR_BYTES, BWD_PIXEL_BYTES = 120, 28


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_workload(torch, slr, synth, targets):
    t0 = time.time()
    sc, prims = synth.structured_scene(N_SURFELS, 0)
    poses = synth.circle_poses(N_KF, 0)
    sensor = slr.make_sensor(H, W)
    dev = "cuda"
    d = {k: torch.from_numpy(v).to(dev) for k, v in sc.items()}
    kfs = []
    for k, T in enumerate(poses):
        Dt, Nt = targets.raycast(prims, sensor, T, seed=100 + k)
        nvalid = int((Dt > 0).sum())
        kfs.append(dict(T=torch.from_numpy(T).to(dev), Dt=torch.from_numpy(Dt).to(dev),
                        Nt=torch.from_numpy(Nt).to(dev), w=1.0 / max(nvalid, 1), T_np=T))
    log(f"workload built in {time.time() - t0:.1f}s")
    return sc, d, sensor, kfs


def plain_step(torch, slr, d, kfs, rend, grads, dposes, scratch, loss):
    for k, kf in enumerate(kfs):
        r = rend[k]
        D, N, O = r.forward(d["means"], d["quats"], d["log_scales"], d["logits"], kf["T"])
        gD, gN = scratch
        slr.loss_l1_normal(D, N, kf["Dt"], kf["Nt"], kf["w"], kf["w"], gD, gN, loss)
        if k == 0:
            g, dp = r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], kf["T"], gD, gN, None)
            for key in grads:
                grads[key] = g[key]
            dposes[0] = dp
        else:
            r.backward(d["means"], d["quats"], d["log_scales"], d["logits"], kf["T"], gD, gN, None,
                       out=(grads, dposes[k]))


def make_batch(torch, slr, d, sensor, kfs, tiling):
    frames = [dict(set=0, T_cw=kf["T"], sensor=sensor) for kf in kfs]
    br = slr.BatchRenderer([d], frames, tiling, capacity=24 << 20)
    return br


def batched_step(slr, br, kfs, loss):
    br.render()
    slr.loss_l1_normal_frames([(br.out[k][0], br.out[k][1], kf["Dt"], kf["Nt"], kf["w"], kf["w"], br.up[k][0],
                                br.up[k][1]) for k, kf in enumerate(kfs)], loss)
    br.backward()


def _traffic_summaries(kernel):
    """{tiling label: fields} of the committed counter summaries of `kernel`
    (profiles/<kernel>_traffic_8x128x1024_1M*.txt) taken on the current
    compositing source."""
    import glob
    import hashlib
    with open(os.path.join(ROOT, "paper_2503_17491_amd", "csrc", "raster.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    out = {}
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{kernel}_traffic_8x128x1024_1M*.txt"))):
        fields = {}
        with open(path) as f:
            for line in f:
                if ":" in line:
                    k, v = line.split(":", 1)
                    fields[k.strip()] = v.strip()
        if fields.get("raster.hip sha256") == sha and "traffic bytes per launch" in fields and "tiling" in fields:
            out[fields["tiling"]] = fields
    return out


def counted_traffic(kernel, tiling):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE runs, copy-calibrated) of this tiling
    (tile, forward and backward form, batch), or None when none was taken on
    the current compositing source with it."""
    fields = _traffic_summaries(kernel).get(tiling)
    return None if fields is None else int(float(fields["traffic bytes per launch"]))


def profiled_tilings(kernel):
    """Tiling labels with a committed counter summary of `kernel` taken on the
    current compositing source."""
    return set(_traffic_summaries(kernel))


def tiling_label(th, tw, var, bvar, bbatch, sch=0):
    vnames = {0: "default", 1: "lds", 2: "scalar", 3: "wave", 4: "fixed"}
    return f"{th}x{tw} fwd {vnames[var]} bwd {vnames[bvar]}" + (
        f" batch {bbatch}" if bvar == 1 and bbatch not in (0, 192) else "") + (" queue" if sch == 3 else "")


def roofline(kernel, flops, nbytes, ms, traffic):
    """Roofline of one compositing launch from its algorithmic work: the bound
    is the one the arithmetic intensity (FLOP per algorithmic byte) puts it
    under, against the ridge PEAK_TFLOPS / PEAK_HBM_GBS = 9.8 FLOP/B; both
    fractions are reported.  traffic: counted HBM bytes per launch or None."""
    gbs = nbytes / (ms * 1e-3) / 1e9
    tfs = flops / (ms * 1e-3) / 1e12
    intensity = flops / max(nbytes, 1)
    ridge = PEAK_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    if intensity < ridge:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(tfs, 3), "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tfs / PEAK_TFLOPS, 4)}
    roof.update({"traffic": traffic, "kernel": kernel, "avg_launch_ms": round(ms, 4),
                 "algorithmic_bytes_per_launch": int(nbytes), "flops_per_launch": int(flops),
                 "intensity_flop_per_byte": round(intensity, 2), "ridge_flop_per_byte": round(ridge, 2),
                 "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
                 "alu_tflops": round(tfs, 3), "alu_frac": round(tfs / PEAK_TFLOPS, 4)})
    if traffic is not None:   # the counted bytes over the same launch time
        roof["counted_gbs"] = round(traffic / (ms * 1e-3) / 1e9, 1)
        roof["counted_frac"] = round(traffic / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
    return roof


def measure_gn(torch, slr, d, sensor, kf, tiling, steps):
    """Pose-only Gauss-Newton iterations on keyframe 0 (plain form): render at
    the pose, then the normal equations against the keyframe's target (least
    squares, weight 1 where the target has a return).  The 6x6 solve is the
    caller's and is not timed.  The normal equations take their
    one-wave-per-strip form (backward form 3): on one keyframe's 512 tiles the
    workgroup form waits at its barrier; the tile shape is picked by timing
    (untimed).  The kernel walks the pairs the backward walks, so its
    algorithmic FLOP come from the backward census of the same tiling."""
    m = (kf["Dt"] > 0).float()
    buf = torch.empty(43, dtype=torch.float64, device="cuda")
    a5 = (d["means"], d["quats"], d["log_scales"], d["logits"], kf["T"])

    def one(rr):
        D, _, _ = rr.forward(*a5)
        rr.pose_gn(*a5, D, kf["Dt"], m, 0.0, out=buf)

    best = None
    for th, tw in SINGLE_FRAME_SHAPES:
        cand = (th, tw) + tuple(tiling[2:4]) + (slr.VARIANT_WAVE,) + tuple(tiling[5:])
        rr = slr.Renderer(sensor, cand, capacity=4 << 20)
        for _ in range(3):
            one(rr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            one(rr)
        torch.cuda.synchronize()
        dt_c = time.perf_counter() - t0
        if best is None or dt_c < best[0]:
            best = (dt_c, cand)
        del rr
    tiling = best[1]
    r = slr.Renderer(sensor, tiling, capacity=4 << 20)
    zero = torch.zeros_like(kf["Dt"])
    D, _, _ = r.forward(*a5)
    r.backward(*a5, zero, None, None, pose_only=True)   # fills the backward census of this tiling
    census0 = r.views()["census"].to(torch.int64).sum(dim=(1, 2)).tolist()

    def one_r():
        one(r)

    for _ in range(3):
        one_r()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_r()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    slr.stage_timer(True)
    slr.stage_times()
    n = max(3, steps // 2)
    for _ in range(n):
        one_r()
    st = slr.stage_times()
    slr.stage_timer(False)
    ms = st["pose_gn"][0] / max(st["pose_gn"][1], 1)
    flops = BWD_EVAL_FLOPS * census0[2] + GN_CONTRIB_FLOPS * census0[3]
    ach = flops / (ms * 1e-3) / 1e12
    return {"workload": "keyframe 0 of the map, 128x1024: render + Gauss-Newton normal equations per iteration",
            "iter_s": round(steps / dt, 3), "kernel": "raster_gn_w", "form": "one wave per 64-pixel strip",
            "tile": f"{tiling[0]}x{tiling[1]}",
            "kernel_ms": round(ms, 4),
            "render_ms": round(sum(st[k][0] for k in ("project", "range_sort", "count_scan", "emit_tile_sort",
                                                       "raster_fwd")) / n, 4),
            "bound": "alu", "achieved": round(ach, 3), "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / PEAK_TFLOPS, 4), "flops_per_launch": int(flops)}


def measure_photo(torch, slr, sensor, kf, depth, steps):
    """Photometric registration normal equations on one 128x1024 frame: the
    rendered range of keyframe 0 against the keyframe's ray-cast scan, the
    identity as the render-to-query transform."""
    T = torch.eye(4, dtype=torch.float64, device="cuda")
    ws = torch.empty(slr.photo_workspace_size(sensor), dtype=torch.uint8, device="cuda")
    buf = torch.empty(44, dtype=torch.float64, device="cuda")
    for _ in range(3):
        slr.photo_gn(sensor, depth, kf["Dt"], T, None, 0.1, ws=ws, out=buf)
    torch.cuda.synchronize()
    slr.stage_timer(True)
    slr.stage_times()
    for _ in range(steps):
        slr.photo_gn(sensor, depth, kf["Dt"], T, None, 0.1, ws=ws, out=buf)
    st = slr.stage_times()
    slr.stage_timer(False)
    ms = st["photo_gn"][0] / max(st["photo_gn"][1], 1)
    px = depth.numel()
    return {"workload": "rendered range of keyframe 0 against its ray-cast scan, 128x1024, Huber 0.1 m",
            "kernel_ms": round(ms, 4), "pixels_per_s": round(px / (ms * 1e-3), 1),
            "pixels_taken": int(buf[43].item()),
            "bound": "latency: 8 B of images per pixel, ~1 MB per launch"}


def measure_mapping(torch, slr, sensor, kf, d, steps):
    """Mapping-side image kernels on keyframe 0's scan (its ray-cast target
    back-projected into a sensor-frame point cloud): cloud to range image,
    normals from range gradients, the fused refinement losses, the scale cap
    over the map, and 100k initialisation draws.  HIP events on the launch
    stream, mean over `steps` calls each."""
    Dt = kf["Dt"]
    Hh, Ww = Dt.shape
    ii, jj = torch.meshgrid(torch.arange(Hh, device="cuda", dtype=torch.float64),
                            torch.arange(Ww, device="cuda", dtype=torch.float64), indexing="ij")
    az = (jj + 0.5 - sensor["cu"]) / sensor["fu"]
    el = (ii + 0.5 - sensor["cv"]) / sensor["fv"]
    ray = torch.stack([torch.cos(el) * torch.cos(az), torch.cos(el) * torch.sin(az), torch.sin(el)], -1)
    pts = (Dt.double()[..., None] * ray)[Dt > 0].float().contiguous()
    rng = torch.empty_like(Dt)
    nrm = torch.empty(Hh, Ww, 3, device="cuda")
    gD, gN, gO = torch.empty_like(Dt), torch.empty_like(nrm), torch.empty_like(Dt)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    O = torch.full_like(Dt, 0.9)
    gls = torch.zeros_like(d["log_scales"])
    U = torch.rand(100_000, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    calls = {
        "cloud_to_range": lambda: slr.cloud_to_range(sensor, pts, out=rng),
        "range_normals": lambda: slr.range_normals(sensor, Dt, out=nrm),
        "loss_map": lambda: slr.loss_map(Dt, nrm, O, Dt, nrm, 1.0, 1.0, 1.0, gD, gN, gO, loss),
        "scale_reg": lambda: slr.scale_reg(d["log_scales"], 0.5, 1.0, gls, loss),
        "init_splats": lambda: slr.init_splats(sensor, Dt, kf["T"], U),
    }
    out = {"scan_points": int(pts.shape[0]), "image": f"{Hh}x{Ww}", "surfels": int(d["log_scales"].shape[0]),
           "init_draws": int(U.numel())}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[name + "_ms"] = round(a.elapsed_time(b) / steps, 4)
    return out


def cpu_baseline(sc, sensor, kfs, budget_s):
    """The FP64 oracle on a bounded sample: fwd+bwd of random pixels of keyframe 0,
    in the angular-cull mode (identical results to the brute force, faster)."""
    import numpy as np

    import oracle as O
    T = kfs[0]["T_np"]
    Dt = kfs[0]["Dt"].cpu().numpy()
    g = np.random.default_rng(7)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def run(P):
        pix = np.stack([g.integers(0, H, P), g.integers(0, W, P)], 1).astype(np.int32)
        t = time.perf_counter()
        r = O.render_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor, pix, cull=True)
        valid = Dt[pix[:, 0], pix[:, 1]] > 0
        gD = np.where(valid, np.sign(r["depth"] - Dt[pix[:, 0], pix[:, 1]]), 0.0)
        O.backward_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor, pix, gD, None, None,
                          cull=True)
        return time.perf_counter() - t

    def omp_threads(n):   # the oracle's OpenMP regions (libgomp)
        try:
            ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        except OSError:
            pass

    def measure(nthreads, budget):
        # grow the sample until it takes about `budget` (at most six tries; every try
        # pays the cull index once, so the early ones understate the per-pixel rate)
        omp_threads(nthreads)
        P, t1 = 4 * nthreads, 0.0
        for k in range(6):
            t1 = run(P)
            if t1 >= 0.6 * budget or P >= H * W * N_KF or k == 5:
                break
            P = min(H * W * N_KF, max(P + 1, int(P * min(10.0, budget / max(t1, 1e-3)))))
        return P, t1

    def sample(P, t1):
        return (f"FP64 oracle fwd+bwd of {P} random pixels of keyframe 0 (every pixel ray against the "
                f"{N_SURFELS} surfels, in its result-identical angular-cull mode; each call builds its cull "
                f"index) in {t1:.1f}s, scaled to {N_KF}x{H}x{W} pixels per iteration")

    P, t1 = measure(threads, budget_s)
    out = {"value": 1.0 / (t1 / P * H * W * N_KF), "unit": "iter/s", "cores": threads, "kind": "oracle",
           "sample": sample(P, t1)}
    P1, t11 = measure(1, budget_s / 2)
    out["one_thread"] = {"value": 1.0 / (t11 / P1 * H * W * N_KF), "unit": "iter/s", "cores": 1,
                         "sample": sample(P1, t11)}
    omp_threads(threads)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", choices=["batched", "plain"], default="batched",
                    help="form whose iter/s is reported as value (both are always timed)")
    ap.add_argument("--no-graph", action="store_true", help="batched form without HIP-graph capture")
    ap.add_argument("--tile", default="auto",
                    help="HxW tile shape, or auto: the autotuner picks shape, form and schedule (untimed)")
    ap.add_argument("--variant", choices=["default", "lds", "scalar", "wave"], default="default",
                    help="forward compositing kernel: records staged in LDS, or read through the scalar cache")
    ap.add_argument("--bwd-variant", choices=["default", "lds", "wave", "fixed"], default="default",
                    help="backward compositing kernel: one workgroup per tile, one wave per strip, or the "
                         "fixed-order (deterministic) workgroup form")
    ap.add_argument("--schedule", choices=["default", "tile", "longest", "queue"], default="default",
                    help="order in which the compositing kernels take tiles")
    ap.add_argument("--only", choices=["both", "batched"], default="both",
                    help="batched: skip the plain form (short profiling runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one 256 MiB device-to-device copy first (calibrates HBM counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gn", action="store_true", help="skip the pose-only Gauss-Newton measurement")
    ap.add_argument("--box", choices=["exact", "opacity", "vertex"], default="exact",
                    help="bounding box: exact 3-sigma square, opacity-aware square (same images, fewer pairs), "
                         "or the relaxed vertex-only box (can miss pixels)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--bwd-batch", type=int, choices=[0, 128, 192], default=0,
                    help="records per LDS batch of the workgroup backward (0: library default)")
    ap.add_argument("--config", choices=["headline", "fwd-2k", "map-200k", "odometry-300k", "batch-uneven", "map-2m-adam", "n-sweep"], default="headline",
                    help="workload: the headline (default) or one of the other configurations (bench_configs.py)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: sharding keyframes over several GPUs (with an all-reduce of the "
              "surfel gradients) is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.config != "headline":
        import bench_configs
        bench_configs.run(args.config, args)
        return

    import torch

    from paper_2503_17491_amd import slr, synth, targets
    slr.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    var = {"default": slr.VARIANT_DEFAULT, "lds": slr.VARIANT_LDS, "scalar": slr.VARIANT_SCALAR,
           "wave": slr.VARIANT_WAVE}[args.variant]
    sch = {"default": slr.SCHEDULE_DEFAULT, "tile": slr.SCHEDULE_TILE, "longest": slr.SCHEDULE_LONGEST,
           "queue": slr.SCHEDULE_QUEUE}[args.schedule]
    th = tw = None
    bvar = {"default": 0, "lds": slr.VARIANT_LDS, "wave": slr.VARIANT_WAVE,
            "fixed": slr.VARIANT_DETERMINISTIC}[args.bwd_variant]
    box = {"exact": slr.BOX_EXACT, "opacity": slr.BOX_OPACITY, "vertex": slr.BOX_VERTEX}[args.box]
    bbatch = args.bwd_batch
    if args.tile != "auto":
        th, tw = (int(x) for x in args.tile.split("x"))
    if args.copy_calib:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 268435456 bytes read, 268435456 bytes written")
        del src, dst
    sc, d, sensor, kfs = build_workload(torch, slr, synth, targets)
    br = None
    tune_ms = None
    if th is None:
        # the autotuner times every candidate tiling on this batch (outside the timed region)
        br = make_batch(torch, slr, d, sensor, kfs, tuple(slr.TUNE_CANDIDATES[0]) + (box,))
        for u in br.up:
            for t in u:
                t.fill_(1.0)
        tune_ms = br.autotune(reps=5)
        for u in br.up:   # the step's upstream gradients come from the loss; the opacity channel has none
            for t in u:
                t.zero_()
        # candidates within TUNE_MARGIN of the fastest are a tie within timing
        # noise: among them the one whose HBM counters are committed is taken,
        # so that the line can carry the counted traffic of the launch it times
        prof = profiled_tilings("raster_bwd")
        best_ms = min(v for v in tune_ms.values() if v > 0)
        near = [(v, tuple(c)) for c, v in tune_ms.items()
                if 0 < v <= best_ms * (1 + TUNE_MARGIN) and
                tiling_label(c[0], c[1], c[2], c[4], c[6] if len(c) > 6 else 0, c[3]) in prof]
        if near:
            c = min(near)[1]   # the fastest of them
            if c != tuple(br.tiling):
                log(f"autotune: {c} is within {TUNE_MARGIN:.0%} of the fastest and has committed counters")
                br.tiling = c
                br.prepare()
        th, tw, var, sch, bvar, box = br.tiling[:6]
        bbatch = br.tiling[6] if len(br.tiling) > 6 else 0
        log("autotuned tiling:", br.tiling, {f"{c[0]}x{c[1]}/f{c[2]}/b{c[4]}" + (f"/{c[6]}" if len(c) > 6 else "") +
                                             ("/queue" if c[3] == slr.SCHEDULE_QUEUE else ""): round(v, 3)
                                             for c, v in tune_ms.items()})
    tiling = (th, tw, var, sch, bvar, box, bbatch)
    grads = {k: None for k in ("means", "quats", "log_scales", "logits")}
    dposes = [torch.zeros(6, dtype=torch.float64, device="cuda") for _ in kfs]
    scratch = (torch.empty(H, W, device="cuda"), torch.empty(H, W, 3, device="cuda"))
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    plain_tiling = tiling
    if tune_ms is not None and args.only == "both":
        # the plain loop renders one keyframe per launch, where the backward's
        # workgroup barrier weighs more and a single frame's 512 tiles fill the
        # chip differently: its tile shape and backward form are picked by
        # timing them on the plain loop (untimed)
        best = None
        for ph, pw, bv in [(a, b, v) for a, b in SINGLE_FRAME_SHAPES for v in (slr.VARIANT_LDS, slr.VARIANT_WAVE)]:
            cand = (ph, pw, var, sch, bv, box, bbatch)
            rr = [slr.Renderer(sensor, cand, capacity=4 << 20) for _ in kfs]
            plain_step(torch, slr, d, kfs, rr, grads, dposes, scratch, loss)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                plain_step(torch, slr, d, kfs, rr, grads, dposes, scratch, loss)
            torch.cuda.synchronize()
            dt_c = time.perf_counter() - t0
            if best is None or dt_c < best[0]:
                best = (dt_c, cand)
            del rr
        plain_tiling = best[1]
        log("plain form tiling:", plain_tiling)
    rend = [slr.Renderer(sensor, plain_tiling, capacity=4 << 20) for _ in kfs]

    plain_iters = None
    if args.only == "both":
        # ---- plain form: per-keyframe launches, one host sync per keyframe for the pair count
        for _ in range(args.warmup):
            plain_step(torch, slr, d, kfs, rend, grads, dposes, scratch, loss)
        torch.cuda.synchronize()
        log("plain warmup done; pairs per keyframe:", [r.K for r in rend])
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plain_step(torch, slr, d, kfs, rend, grads, dposes, scratch, loss)
        torch.cuda.synchronize()
        plain_dt = time.perf_counter() - t0
        plain_iters = args.steps / plain_dt
        log(f"plain: {args.steps} steps in {plain_dt:.3f}s -> {plain_iters:.2f} iter/s")
    else:
        plain_step(torch, slr, d, kfs, rend, grads, dposes, scratch, loss)
        torch.cuda.synchronize()
    ef = cf = eb = cb = 0
    if plain_tiling != tiling:   # the census of the batched form's tiling
        del rend
        rend = [slr.Renderer(sensor, tiling, capacity=4 << 20) for _ in kfs]
        plain_step(torch, slr, d, kfs, rend, grads, dposes, scratch, loss)
        torch.cuda.synchronize()
    for r in rend:  # per-keyframe work census (the backward's equals the batched form's)
        c = r.views()["census"].to(torch.int64).sum(dim=(1, 2)).tolist()
        ef += c[0]; cf += c[1]; eb += c[2]; cb += c[3]
    pairs = int(sum(r.K for r in rend))
    del rend
    torch.cuda.empty_cache()

    # ---- batched form: all keyframes per launch, no host sync, one graph launch per iteration
    if br is None:
        br = make_batch(torch, slr, d, sensor, kfs, tiling)
    batched_step(slr, br, kfs, loss)
    if br.ensure_capacity():
        batched_step(slr, br, kfs, loss)
    K, over = br.pairs()
    assert over == 0 and K == pairs, (K, over, pairs)
    graph = None
    if not args.no_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            batched_step(slr, br, kfs, loss)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            batched_step(slr, br, kfs, loss)
    run = (lambda: graph.replay()) if graph is not None else (lambda: batched_step(slr, br, kfs, loss))
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    batched_dt = time.perf_counter() - t0
    batched_iters = args.steps / batched_dt
    K, over = br.pairs()
    assert over == 0
    # the batched launches' own census (a single keyframe may take the forward's
    # quad mode, which walks fewer entries; the batch does not)
    ef, cf, eb, cb = br.views()["census"].to(torch.int64).sum(dim=1).tolist()
    # per-kernel durations: HIP events on the launch stream around each stage of
    # the same batched step, run eagerly right after the timed loop (warm GPU)
    nst = max(3, args.steps // 2)
    slr.stage_timer(True)
    slr.stage_times()
    for _ in range(nst):
        batched_step(slr, br, kfs, loss)
    torch.cuda.synchronize()
    stages = slr.stage_times()
    slr.stage_timer(False)
    log(f"batched{'+graph' if graph is not None else ''}: {args.steps} steps in {batched_dt:.3f}s -> "
        f"{batched_iters:.2f} iter/s")

    fwd_ms = stages["raster_fwd"][0] / max(stages["raster_fwd"][1], 1)
    bwd_ms = stages["raster_bwd"][0] / max(stages["raster_bwd"][1], 1)
    fwd_flops = FWD_EVAL_FLOPS * ef + FWD_CONTRIB_FLOPS * cf   # one batched launch covers all keyframes
    bwd_flops = BWD_EVAL_FLOPS * eb + BWD_CONTRIB_FLOPS * cb
    px = N_KF * H * W
    fwd_bytes = FWD_PAIR_BYTES * pairs + FWD_PIXEL_BYTES * px
    bwd_bytes = BWD_PAIR_BYTES * pairs + BWD_PIXEL_BYTES * px
    if bwd_ms >= fwd_ms:
        dom, flops, nbytes, ms = "raster_bwd", bwd_flops, bwd_bytes, bwd_ms
    else:
        dom, flops, nbytes, ms = "raster_fwd", fwd_flops, fwd_bytes, fwd_ms
    tiling_name = tiling_label(th, tw, var, bvar, bbatch, sch)
    traffic = counted_traffic(dom, tiling_name)
    roof = roofline(dom, flops, nbytes, ms, traffic)
    stage_ms = {k: round(v[0] / nst, 4) for k, v in stages.items()}
    if args.form == "plain" and plain_iters is None:
        raise SystemExit("--form plain needs --only both")
    value = batched_iters if args.form == "batched" else plain_iters
    dt = batched_dt if args.form == "batched" else plain_dt

    gn = photo = mapping = None
    if not args.no_gn:
        gn = measure_gn(torch, slr, d, sensor, kfs[0], tiling, args.steps)
        log("pose-only Gauss-Newton:", gn)
        photo = measure_photo(torch, slr, sensor, kfs[0], br.out[0][0], args.steps)
        log("photometric registration:", photo)
        mapping = measure_mapping(torch, slr, sensor, kfs[0], d, args.steps)
        log("mapping kernels:", mapping)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(sc, sensor, kfs, args.cpu_seconds)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{N_SURFELS} surfels (structured scene), {N_KF} keyframes {H}x{W} sharing the "
                               f"map, fwd + L1 range/normal loss + bwd per keyframe",
                   "form": args.form, "graph": graph is not None, "tile": f"{th}x{tw}", "variant": {0: "default", 1: "lds", 2: "scalar", 3: "wave"}[var],
                   "schedule": {0: "default", 1: "tile", 2: "longest", 3: "queue"}[sch],
                   "bwd_variant": {0: "default", 1: "lds", 3: "wave", 4: "fixed"}[bvar],
                   "bwd_batch": bbatch if bbatch else 192, "autotuned": tune_ms is not None,
                   "box": args.box,
                   "keyframes": N_KF,
                   "surfels": N_SURFELS, "batched_iter_s": round(batched_iters, 3),
                   "plain_iter_s": None if plain_iters is None else round(plain_iters, 3),
                   "plain_tile": f"{plain_tiling[0]}x{plain_tiling[1]}",
                   "plain_bwd_variant": {0: "default", 1: "lds", 3: "wave", 4: "fixed"}[plain_tiling[4]],
                   "pairs_per_step": pairs,
                   "census": {"fwd_eval": ef, "fwd_contrib": cf, "bwd_eval": eb, "bwd_contrib": cb}},
        "roofline": roof, "cpu_baseline": cpu, "stage_ms_per_step": stage_ms, "pose_gn": gn, "photo_gn": photo, "mapping": mapping,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Comparisons of the HIP path's outputs with the FP64 oracle, shared by the
GPU parity tests (no test is collected from this module).

Forward: every compared pixel must equal one of the oracle's admissible
results within 1e-4 relative (depth against max(|D|, 1 m), alpha against
max(O, 1e-2), normal against max(|N|, 1e-2)).  A pixel has one admissible
result, the plain FP64 render, unless one of its decisions (3-sigma support,
near range, the 1/255 alpha floor, the 1e-4 stop; the 3DGS blending
conventions of Sec. 3.2.1) lies within rounding distance of its threshold;
then the oracle takes each such decision both ways and lists every outcome.
A pixel that matches none of its listed results fails the test; only a pixel
whose list was cut short (more than 2^max_flips outcomes) may stay
unverified, and their fraction is bounded.

Backward: per-surfel parameter blocks within 1e-3 of the oracle's analytic
FP64 gradient, relative to max(|g_ref|, 1e-3 RMS, 1e-2 sum_pixels
|contribution|), the pose 6-vector within 1e-3 of its norm.  How many blocks
pass only because of the summed-magnitude term is printed with their error
under the plain bound max(|g_ref|, 1e-3 RMS).
"""
import math
import sys

import numpy as np

import oracle as O

DEV = "cuda"
EXCL = O.FLAG_SUPPORT | O.FLAG_NEAR | O.FLAG_AMIN | O.FLAG_TSTOP
TOL_FWD = 1e-4
TOL_GRAD = 1e-3


def say(*a):
    print("[gpu-check]", *a, flush=True)
    sys.stdout.flush()


def to_dev(torch, sc):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(DEV) for k, v in sc.items()}


def pose_dev(torch, T):
    return torch.from_numpy(np.ascontiguousarray(T, dtype=np.float64)).to(DEV)


def _errors(D, N, A, rD, rN, rA):
    eD = np.abs(D - rD) / np.maximum(np.abs(rD), 1.0)
    eA = np.abs(A - rA) / np.maximum(rA, 1e-2)
    eN = np.linalg.norm(N - rN, axis=-1) / np.maximum(np.linalg.norm(rN, axis=-1), 1e-2)
    return np.maximum(np.maximum(eD, eA), eN), eD, eA, eN


def forward_verdict(D, N, A, sc, T, sensor, pix=None, cull=True, max_unverified=1e-3, max_flips=4, label=""):
    """D [H,W], N [H,W,3], A [H,W]: the GPU's images (numpy); pix [P,2]
    (row, col) pixels to compare, None for the whole image.  Asserts the
    verdict described in the module docstring and returns its counts."""
    if pix is None:
        pix = O.all_pixels(sensor)
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
    gD = np.asarray(D, np.float64)[pix[:, 0], pix[:, 1]]
    gA = np.asarray(A, np.float64)[pix[:, 0], pix[:, 1]]
    gN = np.asarray(N, np.float64)[pix[:, 0], pix[:, 1]]
    ref = O.render_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor, pix, cull=cull)
    e, eD, eA, eN = _errors(gD, gN, gA, ref["depth"], ref["normal"], ref["alpha"])
    flagged = (ref["flags"] & EXCL) != 0
    clean = ~flagged
    bad_clean = clean & (e > TOL_FWD)
    # flagged pixels that differ from the plain render: compare with every admissible result
    off = np.nonzero(flagged & (e > TOL_FWD))[0]
    matched_other = unverified = 0
    mismatch = []
    if off.size:
        rv = O.render_variants(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor, pix[off],
                               max_flips=max_flips, cull=cull)
        for q, p in enumerate(off):
            nv = int(rv["nvar"][q])
            ev, _, _, _ = _errors(gD[p], gN[p][None, :], gA[p], rv["depth"][q, :nv], rv["normal"][q, :nv],
                                  rv["alpha"][q, :nv])
            if (ev <= TOL_FWD).any():
                matched_other += 1
            elif rv["overflow"][q]:
                unverified += 1
            else:
                mismatch.append((tuple(pix[p]), float(e[p]), nv))
    P = pix.shape[0]
    stats = dict(pixels=P, flagged=int(flagged.sum()), matched_other_outcome=matched_other, unverified=unverified,
                 max_err_clean=float(e[clean].max()) if clean.any() else 0.0,
                 max_err_depth=float(eD[clean].max()) if clean.any() else 0.0,
                 max_err_alpha=float(eA[clean].max()) if clean.any() else 0.0,
                 max_err_normal=float(eN[clean].max()) if clean.any() else 0.0)
    say(f"forward {label}: {P} pixels, {stats['flagged']} with a decision in the guard band "
        f"({stats['flagged'] / max(P, 1):.2%}), {matched_other} of them match another admissible outcome, "
        f"{unverified} unverified ({unverified / max(P, 1):.4%}); max err on the others: depth "
        f"{stats['max_err_depth']:.2e} alpha {stats['max_err_alpha']:.2e} normal {stats['max_err_normal']:.2e}")
    assert not bad_clean.any(), f"{int(bad_clean.sum())} pixels off by more than {TOL_FWD}: " \
                                f"{[(tuple(pix[p]), float(e[p])) for p in np.nonzero(bad_clean)[0][:8]]}"
    assert not mismatch, f"{len(mismatch)} flagged pixels match no admissible result: {mismatch[:8]}"
    assert unverified <= max_unverified * P, stats
    # every pixel is a valid compositing result
    assert (gA >= -1e-6).all() and (gA <= 1 + 1e-6).all()
    assert (np.linalg.norm(gN, axis=1) <= gA + 1e-5).all()
    return stats


def block_err(g, ref, absum, name=""):
    """max over surfels of |g - ref| / max(|ref|, 1e-3 RMS, 1e-2 |absum|) per parameter block;
    the RMS is taken over the surfels whose reference block is non-zero, absum is the
    oracle's per-surfel sum over pixels of |per-pixel contribution|."""
    g, ref = g.reshape(g.shape[0], -1), ref.reshape(ref.shape[0], -1)
    nrm = np.linalg.norm(ref, axis=1)
    touched = nrm > 0
    rms = math.sqrt(float((nrm[touched] ** 2).mean())) if touched.any() else 1.0
    den_plain = np.maximum(nrm, 1e-3 * rms)
    den = np.maximum(den_plain, 1e-2 * np.linalg.norm(absum.reshape(absum.shape[0], -1), axis=1))
    d = np.linalg.norm(g - ref, axis=1)
    e, e_plain = d / den, d / den_plain
    wide = touched & (e_plain > TOL_GRAD) & (e <= TOL_GRAD)
    nt = int(touched.sum())
    say(f"   {name:10s} blocks {nt}: err p50 {np.median(e[touched]) if nt else 0:.1e} p99.9 "
        f"{np.quantile(e[touched], 0.999) if nt else 0:.1e} max {e.max() if e.size else 0:.1e}; "
        f"pass only through the summed-magnitude term: {int(wide.sum())} ({wide.sum() / max(nt, 1):.3%}), "
        f"their plain-bound err max {e_plain[wide].max() if wide.any() else 0:.1e}")
    return float(e.max()) if e.size else 0.0, int(wide.sum()), nt


def oracle_backward(sc, T, sensor, pix, gD, gN, gO, cull=True):
    return O.backward_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor, pix,
                             None if gD is None else np.asarray(gD, np.float64),
                             None if gN is None else np.asarray(gN, np.float64),
                             None if gO is None else np.asarray(gO, np.float64), with_abs=True, cull=cull)


def backward_verdict(g, dpose, ref, label=""):
    """g: dict of GPU gradients (numpy), dpose [6]; ref: oracle_backward's dict."""
    cols = dict(means=slice(0, 3), quats=slice(3, 7), log_scales=slice(7, 9), logits=slice(9, 10))
    say(f"backward {label}")
    errs, wide, tot = {}, 0, 0
    for k in ("means", "quats", "log_scales", "logits"):
        errs[k], w, t = block_err(np.asarray(g[k], np.float64), ref[k], ref["abs"][:, cols[k]], k)
        wide += w
        tot += t
    dp = np.asarray(dpose, np.float64)
    errs["pose"] = float(np.linalg.norm(dp - ref["pose"]) / max(np.linalg.norm(ref["pose"]), 1e-12))
    say("   errors", {k: f"{v:.2e}" for k, v in errs.items()},
        f"; blocks passing only through the summed-magnitude term: {wide} of {tot}")
    for k, v in errs.items():
        assert v <= TOL_GRAD, (k, v)
    return errs, wide, tot


def clean_pixels(sc, T, sensor, pix=None, cull=True):
    """Pixels whose oracle decisions are away from every threshold (incl. the alpha
    clamp, where the gradient jumps): the backward is compared on these."""
    ref = O.render_pixels(sc["means"], sc["quats"], sc["log_scales"], sc["logits"], T, sensor, pix, cull=cull)
    keep = (ref["flags"] & (EXCL | O.FLAG_CLAMP)) == 0
    p = O.all_pixels(sensor) if pix is None else np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
    return p[keep]

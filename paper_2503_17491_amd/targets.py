"""Synthetic LiDAR targets: analytic ray casting of the structured scenes.

The structured scenes of ``synth`` are built from primitives (ground plane,
axis-aligned boxes, vertical cylinders).  Casting the sensor's pixel rays
against those primitives gives the range image D_t and normal image N_t that
stand in for a LiDAR scan projected onto the sensor's image (Sec. 3.1); the
valid mask M_v of Sec. 3.3.1 is D_t > 0.  Gaussian range noise (sigma 2 cm)
is added to hit pixels.  Input data only: no rasterizer arithmetic.
"""
import numpy as np

from . import synth


def pixel_rays(sensor):
    """World-independent unit directions [H, W, 3] of the pixel centres."""
    H, W = int(sensor["height"]), int(sensor["width"])
    az = ((np.arange(W) + 0.5) - sensor["cu"]) / sensor["fu"]
    el = ((np.arange(H) + 0.5) - sensor["cv"]) / sensor["fv"]
    ce, se = np.cos(el)[:, None], np.sin(el)[:, None]
    return np.stack([ce * np.cos(az)[None], ce * np.sin(az)[None], np.broadcast_to(se, (H, W))], -1)


def raycast(prims, sensor, T_cw, noise=0.02, seed=0):
    """(D_t [H,W] float32, N_t [H,W,3] float32 in the sensor frame)."""
    Twc = synth.pose_inverse(np.asarray(T_cw, np.float64))
    Rwc, o = Twc[:3, :3], Twc[:3, 3]
    d = pixel_rays(sensor) @ Rwc.T  # world directions
    H, W = d.shape[:2]
    best = np.full((H, W), np.inf)
    nrm = np.zeros((H, W, 3))
    dx, dy, dz = d[..., 0], d[..., 1], d[..., 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        for p in prims:
            if p["kind"] == "ground":
                t = (p["z"] - o[2]) / dz
                x, y = o[0] + t * dx, o[1] + t * dy
                ok = (t > 1e-6) & (x >= p["x0"]) & (x <= p["x1"]) & (y >= p["y0"]) & (y <= p["y1"])
                upd = ok & (t < best)
                best[upd] = t[upd]
                nrm[upd] = [0.0, 0.0, 1.0]
            elif p["kind"] == "box":
                lo, hi = p["lo"], p["hi"]
                t0 = np.full((H, W), -np.inf)
                t1 = np.full((H, W), np.inf)
                axis = np.zeros((H, W), np.int64)
                sign = np.zeros((H, W))
                for a, da in enumerate((dx, dy, dz)):
                    ta = (lo[a] - o[a]) / da
                    tb = (hi[a] - o[a]) / da
                    tn = np.minimum(ta, tb)
                    tf = np.maximum(ta, tb)
                    par = da == 0
                    inside = (o[a] >= lo[a]) & (o[a] <= hi[a])
                    tn = np.where(par, np.where(inside, -np.inf, np.inf), tn)
                    tf = np.where(par, np.where(inside, np.inf, -np.inf), tf)
                    enter = tn > t0
                    axis = np.where(enter, a, axis)
                    sign = np.where(enter, -np.sign(da), sign)
                    t0 = np.maximum(t0, tn)
                    t1 = np.minimum(t1, tf)
                ok = (t0 <= t1) & (t0 > 1e-6)
                upd = ok & (t0 < best)
                best[upd] = t0[upd]
                n = np.zeros((H, W, 3))
                for a in range(3):
                    n[..., a] = np.where(axis == a, sign, 0.0)
                nrm[upd] = n[upd]
            else:
                ox, oy = o[0] - p["cx"], o[1] - p["cy"]
                A = dx * dx + dy * dy
                B = 2 * (ox * dx + oy * dy)
                Cc = ox * ox + oy * oy - p["r"] ** 2
                disc = B * B - 4 * A * Cc
                sq = np.sqrt(np.maximum(disc, 0))
                t = (-B - sq) / (2 * A)
                z = o[2] + t * dz
                ok = (disc >= 0) & (A > 0) & (t > 1e-6) & (z >= p["z0"]) & (z <= p["z1"])
                upd = ok & (t < best)
                best[upd] = t[upd]
                hx, hy = ox + t * dx, oy + t * dy
                rr = np.sqrt(hx * hx + hy * hy)
                n = np.stack([hx / rr, hy / rr, np.zeros_like(hx)], -1)
                nrm[upd] = n[upd]
    hit = np.isfinite(best)
    g = synth.rng(seed)
    D = np.where(hit, best + noise * g.normal(size=best.shape), 0.0)
    D = np.where(hit & (D > 0), D, 0.0)
    Ns = nrm @ np.asarray(T_cw)[:3, :3].T  # world -> sensor
    Ns[~hit] = 0.0
    return D.astype(np.float32), Ns.astype(np.float32)

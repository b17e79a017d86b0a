"""Seeded synthetic inputs: surfel scenes and sensor poses.

This module holds no rasterizer arithmetic.  It draws raw surfel parameters
(means, unnormalised quaternions (w, x, y, z), log-scales, opacity logits) and
poses with ``numpy.random.Generator(PCG64(seed))`` in FP64, then casts the
surfels to FP32.  The same arrays feed both the HIP library and the CPU oracle.

Scene recipes (the paper's datasets are not available; these stand in for the
LiDAR sequences of its Sec. 4 at the same image sizes):
  shell       centres uniform in the volume of a 2-40 m spherical shell,
              quaternions uniform on S^3, log-scales U(ln 0.05, ln 1.0),
              opacity logits N(0, 1).
  structured  ground plane z = -1.8 m over [-40, 40]^2, 30 axis-aligned boxes
              on the ground (centre in the 4-35 m annulus, sides U(1, 6) m,
              height U(1.5, 8) m; 4 sides + top), 20 vertical cylinders (axis
              in the 3-35 m annulus, radius U(0.15, 0.8) m, height U(2, 8) m).
              Surfels are placed uniformly by area with the normal along the
              outward surface normal, the first tangent at a uniform in-plane
              angle, log-scales U(ln 0.05, ln 0.5), logits N(0, 1).
  urban       the structured recipe on a 200 x 200 m ground with 400 boxes on
              a jittered 10 m grid (footprint U(4, 20) m, height U(3, 25) m)
              and 200 cylinders (radius U(0.1, 0.6) m, height U(3, 10) m).
"""
import math

import numpy as np

GROUND_Z = -1.8


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _quat_from_frame(ta, tb, tn):
    """Unit quaternion (w, x, y, z) of the rotation with columns (ta, tb, tn)."""
    R = np.stack([ta, tb, tn], axis=-1)  # [..., 3, 3]
    m00, m11, m22 = R[..., 0, 0], R[..., 1, 1], R[..., 2, 2]
    tr = m00 + m11 + m22
    q = np.zeros(R.shape[:-2] + (4,))
    c0 = tr > 0
    s = np.sqrt(np.maximum(tr + 1.0, 1e-300)) * 2
    q0 = np.stack([0.25 * s, (R[..., 2, 1] - R[..., 1, 2]) / s, (R[..., 0, 2] - R[..., 2, 0]) / s,
                   (R[..., 1, 0] - R[..., 0, 1]) / s], -1)
    c1 = (~c0) & (m00 > m11) & (m00 > m22)
    s1 = np.sqrt(np.maximum(1.0 + m00 - m11 - m22, 1e-300)) * 2
    q1 = np.stack([(R[..., 2, 1] - R[..., 1, 2]) / s1, 0.25 * s1, (R[..., 0, 1] + R[..., 1, 0]) / s1,
                   (R[..., 0, 2] + R[..., 2, 0]) / s1], -1)
    c2 = (~c0) & (~c1) & (m11 > m22)
    s2 = np.sqrt(np.maximum(1.0 + m11 - m00 - m22, 1e-300)) * 2
    q2 = np.stack([(R[..., 0, 2] - R[..., 2, 0]) / s2, (R[..., 0, 1] + R[..., 1, 0]) / s2, 0.25 * s2,
                   (R[..., 1, 2] + R[..., 2, 1]) / s2], -1)
    c3 = (~c0) & (~c1) & (~c2)
    s3 = np.sqrt(np.maximum(1.0 + m22 - m00 - m11, 1e-300)) * 2
    q3 = np.stack([(R[..., 1, 0] - R[..., 0, 1]) / s3, (R[..., 0, 2] + R[..., 2, 0]) / s3,
                   (R[..., 1, 2] + R[..., 2, 1]) / s3, 0.25 * s3], -1)
    q = np.where(c0[..., None], q0, q)
    q = np.where(c1[..., None], q1, q)
    q = np.where(c2[..., None], q2, q)
    q = np.where(c3[..., None], q3, q)
    return q / np.linalg.norm(q, axis=-1, keepdims=True)


def _pack(means, quats, log_scales, logits):
    return dict(means=np.ascontiguousarray(means, np.float32),
                quats=np.ascontiguousarray(quats, np.float32),
                log_scales=np.ascontiguousarray(log_scales, np.float32),
                logits=np.ascontiguousarray(logits, np.float32))


def shell_scene(n, seed, r_min=2.0, r_max=40.0, ls_range=(math.log(0.05), math.log(1.0))):
    g = rng(seed)
    r = np.cbrt(g.uniform(r_min ** 3, r_max ** 3, n))
    d = g.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    q = g.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    ls = g.uniform(ls_range[0], ls_range[1], (n, 2))
    lo = g.normal(size=n)
    return _pack(d * r[:, None], q, ls, lo)


# ---------------------------------------------------------------------------
# structured scenes: primitives, then area-weighted surfel placement
# ---------------------------------------------------------------------------
def _annulus(g, k, r0, r1):
    rr = np.sqrt(g.uniform(r0 * r0, r1 * r1, k))
    ph = g.uniform(0, 2 * math.pi, k)
    return np.stack([rr * np.cos(ph), rr * np.sin(ph)], 1)


def _scene_primitives(g, kind):
    prims = []  # dicts: ground / box / cyl
    if kind == "structured":
        prims.append(dict(kind="ground", x0=-40.0, x1=40.0, y0=-40.0, y1=40.0, z=GROUND_Z))
        c = _annulus(g, 30, 4.0, 35.0)
        for k in range(30):
            sx, sy = g.uniform(1, 6, 2)
            h = g.uniform(1.5, 8.0)
            prims.append(dict(kind="box", lo=np.array([c[k, 0] - sx / 2, c[k, 1] - sy / 2, GROUND_Z]),
                              hi=np.array([c[k, 0] + sx / 2, c[k, 1] + sy / 2, GROUND_Z + h])))
        a = _annulus(g, 20, 3.0, 35.0)
        for k in range(20):
            prims.append(dict(kind="cyl", cx=a[k, 0], cy=a[k, 1], r=g.uniform(0.15, 0.8),
                              z0=GROUND_Z, z1=GROUND_Z + g.uniform(2.0, 8.0)))
    elif kind == "urban":
        prims.append(dict(kind="ground", x0=-100.0, x1=100.0, y0=-100.0, y1=100.0, z=GROUND_Z))
        for gx in range(20):
            for gy in range(20):
                cx = -95.0 + 10.0 * gx + g.uniform(-2.0, 2.0)
                cy = -95.0 + 10.0 * gy + g.uniform(-2.0, 2.0)
                sx, sy = g.uniform(4.0, 20.0, 2)
                h = g.uniform(3.0, 25.0)
                lo = np.array([cx - sx / 2, cy - sy / 2, GROUND_Z])
                hi = np.array([cx + sx / 2, cy + sy / 2, GROUND_Z + h])
                if lo[0] < 3.0 and hi[0] > -3.0 and lo[1] < 3.0 and hi[1] > -3.0:
                    continue  # keep the sensor neighbourhood free
                prims.append(dict(kind="box", lo=lo, hi=hi))
        a = _annulus(g, 200, 3.0, 95.0)
        for k in range(200):
            prims.append(dict(kind="cyl", cx=a[k, 0], cy=a[k, 1], r=g.uniform(0.1, 0.6),
                              z0=GROUND_Z, z1=GROUND_Z + g.uniform(3.0, 10.0)))
    else:
        raise ValueError(kind)
    return prims


def _faces(prims):
    """Planar rectangles (origin, e1, e2, outward normal) and cylinder sides with areas."""
    items = []
    for p in prims:
        if p["kind"] == "ground":
            o = np.array([p["x0"], p["y0"], p["z"]])
            items.append(("rect", o, np.array([p["x1"] - p["x0"], 0, 0]), np.array([0, p["y1"] - p["y0"], 0]),
                          np.array([0, 0, 1.0])))
        elif p["kind"] == "box":
            lo, hi = p["lo"], p["hi"]
            dx, dy, dz = hi - lo
            items.append(("rect", np.array([lo[0], lo[1], hi[2]]), np.array([dx, 0, 0]), np.array([0, dy, 0]),
                          np.array([0, 0, 1.0])))
            items.append(("rect", np.array([lo[0], lo[1], lo[2]]), np.array([dx, 0, 0]), np.array([0, 0, dz]),
                          np.array([0, -1.0, 0])))
            items.append(("rect", np.array([lo[0], hi[1], lo[2]]), np.array([dx, 0, 0]), np.array([0, 0, dz]),
                          np.array([0, 1.0, 0])))
            items.append(("rect", np.array([lo[0], lo[1], lo[2]]), np.array([0, dy, 0]), np.array([0, 0, dz]),
                          np.array([-1.0, 0, 0])))
            items.append(("rect", np.array([hi[0], lo[1], lo[2]]), np.array([0, dy, 0]), np.array([0, 0, dz]),
                          np.array([1.0, 0, 0])))
        else:
            items.append(("cyl", p))
    areas = []
    for it in items:
        if it[0] == "rect":
            areas.append(np.linalg.norm(np.cross(it[2], it[3])))
        else:
            p = it[1]
            areas.append(2 * math.pi * p["r"] * (p["z1"] - p["z0"]))
    return items, np.asarray(areas)


def structured_scene(n, seed, kind="structured", ls_range=(math.log(0.05), math.log(0.5))):
    """Surfels on ground/boxes/cylinders; returns (surfels dict, primitive list)."""
    g = rng(seed)
    prims = _scene_primitives(g, kind)
    items, areas = _faces(prims)
    counts = g.multinomial(n, areas / areas.sum())
    means, normals = [], []
    for it, c in zip(items, counts):
        if c == 0:
            continue
        if it[0] == "rect":
            _, o, e1, e2, nrm = it
            u = g.uniform(0, 1, (c, 2))
            means.append(o + u[:, :1] * e1 + u[:, 1:] * e2)
            normals.append(np.repeat(nrm[None], c, 0))
        else:
            p = it[1]
            ph = g.uniform(0, 2 * math.pi, c)
            z = g.uniform(p["z0"], p["z1"], c)
            nrm = np.stack([np.cos(ph), np.sin(ph), np.zeros(c)], 1)
            means.append(np.stack([p["cx"] + p["r"] * nrm[:, 0], p["cy"] + p["r"] * nrm[:, 1], z], 1))
            normals.append(nrm)
    means = np.concatenate(means)
    normals = np.concatenate(normals)
    perm = g.permutation(n)
    means, normals = means[perm], normals[perm]
    # tangent frame: a fixed helper axis, then a uniform in-plane rotation
    helper = np.where(np.abs(normals[:, 2:3]) < 0.9, np.array([[0, 0, 1.0]]), np.array([[1.0, 0, 0]]))
    e1 = np.cross(helper, normals)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(normals, e1)
    th = g.uniform(0, 2 * math.pi, n)
    ta = np.cos(th)[:, None] * e1 + np.sin(th)[:, None] * e2
    tb = np.cross(normals, ta)
    q = _quat_from_frame(ta, tb, normals)
    ls = g.uniform(ls_range[0], ls_range[1], (n, 2))
    lo = g.normal(size=n)
    return _pack(means, q, ls, lo), prims


# ---------------------------------------------------------------------------
# poses (4x4 FP64, T_cw = world -> sensor)
# ---------------------------------------------------------------------------
def rot_axis_angle(axis, angle):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def pose_inverse(T):
    Ti = np.eye(4)
    Ti[:3, :3] = T[:3, :3].T
    Ti[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return Ti


def circle_poses(k, seed, radius=5.0):
    """T_cw of k sensors on a circle of the given radius at sensor height, random yaw."""
    g = rng(seed)
    out = []
    for i in range(k):
        ph = 2 * math.pi * i / k
        yaw = g.uniform(-math.pi, math.pi)
        Twc = np.eye(4)
        Twc[:3, :3] = rot_axis_angle([0, 0, 1], yaw)
        Twc[:3, 3] = [radius * math.cos(ph), radius * math.sin(ph), 0.0]
        out.append(pose_inverse(Twc))
    return out


def perturbed_pose(seed, trans=0.5, rot_deg=3.0):
    """T_wc = exp of a 0.5 m translation along a uniform direction and a 3 deg
    rotation about a uniform axis; returns T_cw of that sensor."""
    g = rng(seed)
    d = g.normal(size=3)
    d /= np.linalg.norm(d)
    ax = g.normal(size=3)
    Twc = np.eye(4)
    Twc[:3, :3] = rot_axis_angle(ax, math.radians(rot_deg))
    Twc[:3, 3] = trans * d
    return pose_inverse(Twc)


BATCH_SIZES = [(64, 1024), (128, 1024), (32, 1800), (128, 2048), (64, 512), (128, 1024), (64, 2048), (32, 1024)]


def uneven_batch(seed_base=40):
    """Eight keyframes of uneven sizes, each with its own structured scene of
    N_i = floor(exp(U(ln 5e4, ln 5e5))) surfels."""
    out = []
    for i, (H, W) in enumerate(BATCH_SIZES):
        g = rng(seed_base + i)
        n = int(math.floor(math.exp(g.uniform(math.log(5e4), math.log(5e5)))))
        sc, prims = structured_scene(n, seed_base + i)
        out.append(dict(H=H, W=W, surfels=sc, prims=prims, T_cw=np.eye(4)))
    return out

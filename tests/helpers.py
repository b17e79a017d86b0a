"""Independent math used by the tests to pin the oracle (no oracle code here).

Rotations come from scipy, the pose exponential from scipy.linalg.expm, the
projection from numpy's arctan2 (Sec. 3.1, Eq. spherical-projection), and the
intersection from the textbook ray-plane solve.
"""
import math

import numpy as np
from scipy.linalg import expm
from scipy.spatial.transform import Rotation


def rot_from_quat_wxyz(q):
    q = np.asarray(q, np.float64)
    return Rotation.from_quat(np.concatenate([q[..., 1:], q[..., :1]], -1)).as_matrix()


def quat_wxyz_from_rot(R):
    x, y, z, w = Rotation.from_matrix(R).as_quat()
    return np.array([w, x, y, z])


def project(sensor, p):
    """phi(p) = K psi(p): (u, v) image coordinates of a sensor-frame point."""
    p = np.asarray(p, np.float64)
    az = np.arctan2(p[..., 1], p[..., 0])
    el = np.arctan2(p[..., 2], np.hypot(p[..., 0], p[..., 1]))
    return sensor["fu"] * az + sensor["cu"], sensor["fv"] * el + sensor["cv"]


def ray_dir(sensor, i, j):
    """Unit direction of pixel centre (i + 1/2, j + 1/2) by inverting K and psi."""
    az = ((j + 0.5) - sensor["cu"]) / sensor["fu"]
    el = ((i + 0.5) - sensor["cv"]) / sensor["fv"]
    return np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], -1)


def facing_surfel(center, normal, spin=0.0):
    """Quaternion (w,x,y,z) of a frame whose third column is `normal`."""
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    helper = np.array([0.0, 0.0, 1.0]) if abs(n[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    a = np.cross(helper, n)
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    ta = math.cos(spin) * a + math.sin(spin) * b
    tb = np.cross(n, ta)
    return quat_wxyz_from_rot(np.stack([ta, tb, n], 1))


def hat(d):
    rho, phi = d[:3], d[3:]
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]]
    M[:3, 3] = rho
    return M


def perturb_cw(T_cw, delta):
    """T_cw(delta) = exp(-delta^) T_cw, i.e. T_wc <- T_wc exp(delta)."""
    return expm(-hat(np.asarray(delta, np.float64))) @ T_cw


def sensor_frame_vectors(mu, q, ls, logit, T_cw):
    """b_alpha, b_beta, b_c, n (sensor frame), opacity and scales, from scipy."""
    R = rot_from_quat_wxyz(q / np.linalg.norm(q))
    s = np.exp(ls)
    Rc, tc = T_cw[:3, :3], T_cw[:3, 3]
    return (Rc @ (s[0] * R[:, 0]), Rc @ (s[1] * R[:, 1]), Rc @ mu + tc, Rc @ R[:, 2],
            1.0 / (1.0 + math.exp(-logit)), s)


def ray_plane_shat(ba, bb, bc, n, v):
    """Textbook ray-plane intersection: t* = (n.b_c)/(n.v), x = t* v, then the
    splat coordinates of x in the (b_alpha, b_beta) basis."""
    t = np.dot(n, bc) / np.dot(n, v)
    x = t * v
    return np.array([np.dot(x - bc, ba) / np.dot(ba, ba), np.dot(x - bc, bb) / np.dot(bb, bb)]), t

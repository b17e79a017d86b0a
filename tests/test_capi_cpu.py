"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol declared in include/slr.h, and rejects bad arguments on the host
before enqueuing anything."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2503_17491_amd import slr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "slr.h")).read()
    return sorted(set(re.findall(r"\b(slr_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = slr.lib()
    names = declared_symbols()
    assert "slr_render" in names and "slr_backward" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(slr.EXPORTS) == set(names)


def test_camera_matrix_matches_oracle():
    for (H, W, az, el) in [(64, 512, (-math.pi, math.pi), (-25, 15)), (32, 1800, (-1.2, 1.7), (-10, 30))]:
        a = slr.camera_matrix(az[0], az[1], math.radians(el[0]), math.radians(el[1]), H, W)
        b = O.camera_matrix(az[0], az[1], math.radians(el[0]), math.radians(el[1]), H, W)
        assert a == b


def test_workspace_size_and_validation():
    s = slr.make_sensor(128, 1024)
    n = slr.workspace_size(s, (16, 16), 1000, 5000)
    assert n > 1000 * 96
    assert slr.workspace_size(s, (16, 16), 0, 0) > 0
    with pytest.raises(slr.SlrError) as e:
        slr.workspace_size(s, (16, 8), 10, 10)
    assert e.value.status == slr.SLR_E_INVALID
    bad = dict(s, fu=-s["fu"])
    with pytest.raises(slr.SlrError):
        slr.workspace_size(bad, (16, 16), 10, 10)
    # the workgroup backward stages 128 or 192 records per batch (0: default)
    for batch in (0, 128, 192):
        assert slr.workspace_size(s, (32, 8, 3, 2, 1, 0, batch), 10, 10) > 0
    with pytest.raises(slr.SlrError) as e:
        slr.workspace_size(s, (32, 8, 3, 2, 1, 0, 100), 10, 10)
    assert e.value.status == slr.SLR_E_INVALID and "batch" in str(e.value)
    # schedules 0..3 (3: the work queue of the persistent workgroup backward)
    for sched in (0, 1, 2, 3):
        assert slr.workspace_size(s, (32, 8, 3, sched, 1, 0, 0), 10, 10) > 0
    with pytest.raises(slr.SlrError) as e:
        slr.workspace_size(s, (32, 8, 3, 4, 1, 0, 0), 10, 10)
    assert e.value.status == slr.SLR_E_INVALID and "schedule" in str(e.value)
    # backward forms 0, 1, 3 and 4 (4: the fixed-order form, whose workspace adds a
    # 64-B slot and a bit per pair of capacity and a rank per record)
    for bv in (0, 1, 3, 4):
        assert slr.workspace_size(s, (32, 8, 3, 2, bv, 0, 0), 10, 10) > 0
    for bv in (2, 5, -1):
        with pytest.raises(slr.SlrError) as e:
            slr.workspace_size(s, (32, 8, 3, 2, bv, 0, 0), 10, 10)
        assert e.value.status == slr.SLR_E_INVALID and "backward variant" in str(e.value)
    base = slr.workspace_size(s, (32, 8, 3, 2, 1, 0, 0), 100000, 1 << 20)
    det = slr.workspace_size(s, (32, 8, 3, 2, 4, 0, 0), 100000, 1 << 20)
    assert 64 * (1 << 20) + 4 * 100000 + (1 << 20) // 8 <= det - base <= 64 * (1 << 20) + 4 * 100000 + (1 << 20) // 8 + 768
    pole = slr.make_sensor(64, 512, el=(math.radians(-89.5), math.radians(10)))
    with pytest.raises(slr.SlrError) as e:
        slr.workspace_size(pole, (16, 16), 10, 10)
    assert "89" in str(e.value)


def _args(n=4):
    s = slr._sensor(slr.make_sensor(64, 512))
    t = slr.Tiling(16, 16)
    buf = np.zeros(1 << 16, np.uint8)
    return s, t, buf


def test_render_rejects_bad_arguments_without_gpu():
    L = slr.lib()
    s, t, buf = _args()
    arr = np.zeros(64, np.float32)
    p = C.c_void_p(arr.ctypes.data)
    sf = slr.Surfels(4, p, p, p, p)
    pose = np.zeros(16)
    out = np.zeros(64 * 512 * 3, np.float32)
    o = C.c_void_p(out.ctypes.data)
    # NULL pose
    st = L.slr_render(C.byref(sf), None, C.byref(s), C.byref(t), C.c_void_p(buf.ctypes.data), buf.size, 100,
                      o, o, o, None, None)
    assert st == slr.SLR_E_INVALID
    # negative count
    sf_bad = slr.Surfels(-1, p, p, p, p)
    st = L.slr_render(C.byref(sf_bad), C.c_void_p(pose.ctypes.data), C.byref(s), C.byref(t),
                      C.c_void_p(buf.ctypes.data), buf.size, 100, o, o, o, None, None)
    assert st == slr.SLR_E_INVALID
    # workspace too small
    ws = np.zeros(1024 + 256, np.uint8)
    wp = ws.ctypes.data + (-ws.ctypes.data) % 256
    st = L.slr_render(C.byref(sf), C.c_void_p(pose.ctypes.data), C.byref(s), C.byref(t), C.c_void_p(wp), 1024,
                      100, o, o, o, None, None)
    assert st == slr.SLR_E_INVALID
    assert b"needs" in L.slr_last_error()
    # unsupported tile shape
    t_bad = slr.Tiling(8, 8)
    st = L.slr_render(C.byref(sf), C.c_void_p(pose.ctypes.data), C.byref(s), C.byref(t_bad), C.c_void_p(wp), 1024,
                      100, o, o, o, None, None)
    assert st == slr.SLR_E_INVALID


def test_sensor_rejects_images_beyond_32bit_pixel_indices():
    """The compositing kernels index the three normal channels of a pixel with
    32-bit integers: images with 3 H W >= 2^31 are rejected up front."""
    L = slr.lib()
    t = slr.Tiling(16, 16)
    b = C.c_size_t(0)
    ok = slr._sensor(slr.make_sensor(26000, 27000))    # 3 H W = 2.106e9 < 2^31
    assert L.slr_workspace_size(C.byref(ok), C.byref(t), 10, 100, C.byref(b)) == slr.SLR_OK
    big = slr._sensor(slr.make_sensor(27000, 27000))   # 3 H W = 2.187e9 >= 2^31
    assert L.slr_workspace_size(C.byref(big), C.byref(t), 10, 100, C.byref(b)) == slr.SLR_E_INVALID
    assert b"2^31" in L.slr_last_error()


def test_backward_rejects_inconsistent_gradient_outputs():
    L = slr.lib()
    s, t, buf = _args()
    arr = np.zeros(64, np.float32)
    p = C.c_void_p(arr.ctypes.data)
    sf = slr.Surfels(4, p, p, p, p)
    pose = np.zeros(16)
    g = np.zeros(64, np.float32)
    gp = C.c_void_p(g.ctypes.data)
    big = np.zeros(1 << 24, np.uint8)
    wp = big.ctypes.data + (-big.ctypes.data) % 256
    # only some surfel gradients set
    st = L.slr_backward(C.byref(sf), C.c_void_p(pose.ctypes.data), C.byref(s), C.byref(t), C.c_void_p(wp),
                        big.size - 256, 100, None, None, None, gp, None, None, None, None, 0, None)
    assert st == slr.SLR_E_INVALID
    # pose-only with surfel gradients
    st = L.slr_backward(C.byref(sf), C.c_void_p(pose.ctypes.data), C.byref(s), C.byref(t), C.c_void_p(wp),
                        big.size - 256, 100, None, None, None, gp, gp, gp, gp, gp, slr.SLR_POSE_ONLY, None)
    assert st == slr.SLR_E_INVALID
    # unknown flag
    st = L.slr_backward(C.byref(sf), C.c_void_p(pose.ctypes.data), C.byref(s), C.byref(t), C.c_void_p(wp),
                        big.size - 256, 100, None, None, None, None, None, None, None, gp, 8, None)
    assert st == slr.SLR_E_INVALID


def test_pose_gn_rejects_bad_arguments_without_gpu():
    L = slr.lib()
    s, t, buf = _args()
    arr = np.zeros(64, np.float32)
    p = C.c_void_p(arr.ctypes.data)
    sf = slr.Surfels(4, p, p, p, p)
    pose = np.zeros(16)
    pp = C.c_void_p(pose.ctypes.data)
    img = np.zeros(64 * 512, np.float32)
    ip = C.c_void_p(img.ctypes.data)
    out = np.zeros(43)
    op = C.c_void_p(out.ctypes.data)
    big = np.zeros(1 << 24, np.uint8)
    wp = C.c_void_p(big.ctypes.data + (-big.ctypes.data) % 256)
    n = big.size - 256
    for depth, target, o, k in ((None, ip, op, 0.0), (ip, None, op, 0.0), (ip, ip, None, 0.0),
                                (ip, ip, op, float("nan"))):
        st = L.slr_pose_gn(C.byref(sf), pp, C.byref(s), C.byref(t), wp, n, 100, depth, target, None, k, o, None)
        assert st == slr.SLR_E_INVALID
    # a workspace too small for the plain form is refused too
    st = L.slr_pose_gn(C.byref(sf), pp, C.byref(s), C.byref(t), wp, 1024, 100, ip, ip, None, 0.0, op, None)
    assert st == slr.SLR_E_INVALID


def test_photo_gn_rejects_bad_arguments_without_gpu():
    L = slr.lib()
    s = slr._sensor(slr.make_sensor(64, 512))
    img = np.zeros(64 * 512, np.float32)
    ip = C.c_void_p(img.ctypes.data)
    T = np.eye(4)
    tp = C.c_void_p(T.ctypes.data)
    out = np.zeros(44)
    op = C.c_void_p(out.ctypes.data)
    need = slr.photo_workspace_size(slr.make_sensor(64, 512))
    assert need >= 8 * 29 * (64 * 512 // 256)
    big = np.zeros(need + 512, np.uint8)
    wp = C.c_void_p(big.ctypes.data + (-big.ctypes.data) % 256)
    for d, q, t, o, k in ((None, ip, tp, op, 0.0), (ip, None, tp, op, 0.0), (ip, ip, None, op, 0.0),
                          (ip, ip, tp, None, 0.0), (ip, ip, tp, op, float("nan"))):
        st = L.slr_photo_gn(C.byref(s), d, q, None, t, k, wp, need, o, None)
        assert st == slr.SLR_E_INVALID
    st = L.slr_photo_gn(C.byref(s), ip, ip, None, tp, 0.0, wp, need - 8, op, None)
    assert st == slr.SLR_E_INVALID and b"needs" in L.slr_last_error()
    st = L.slr_photo_gn(C.byref(s), ip, ip, None, tp, 0.0, None, need, op, None)
    assert st == slr.SLR_E_INVALID


def test_photo_gn_noalloc_rejects_bad_arguments_without_gpu():
    """Argument checks of the allocation-free form run before any device call."""
    L = slr.lib()
    s = slr._sensor(slr.make_sensor(64, 512))
    img = np.zeros(64 * 512, np.float32)
    ip = C.c_void_p(img.ctypes.data)
    T = np.eye(4)
    tp = C.c_void_p(T.ctypes.data)
    out = np.zeros(44)
    op = C.c_void_p(out.ctypes.data)
    for d, q, t, o, k in ((None, ip, tp, op, 0.0), (ip, None, tp, op, 0.0), (ip, ip, None, op, 0.0),
                          (ip, ip, tp, None, 0.0), (ip, ip, tp, op, float("nan"))):
        assert L.slr_photo_gn_noalloc(C.byref(s), d, q, None, t, k, o, None) == slr.SLR_E_INVALID
    big = slr._sensor(slr.make_sensor(1024, 1025))   # 1,049,600 pixels: more than the static scratch holds
    assert L.slr_photo_gn_noalloc(C.byref(big), ip, ip, None, tp, 0.0, op, None) == slr.SLR_E_INVALID
    assert b"static scratch" in L.slr_last_error()


def test_loss_frames_rejects_bad_arguments_without_gpu():
    L = slr.lib()
    buf = np.zeros(3 * 64, np.float32)
    p = buf.ctypes.data
    good = slr.LossFrame(64, p, p, p, p, 1.0, 1.0, p, p)
    assert L.slr_loss_l1_normal_frames(-1, None, None, None) == slr.SLR_E_INVALID
    assert L.slr_loss_l1_normal_frames(2, None, None, None) == slr.SLR_E_INVALID
    # valid calls pass validation (without a GPU the launch step then reports the runtime's error)
    assert L.slr_loss_l1_normal_frames(0, None, None, None) != slr.SLR_E_INVALID
    bad = [slr.LossFrame(-1, p, p, p, p, 1.0, 1.0, p, p), slr.LossFrame(64, p, None, p, p, 1.0, 1.0, p, p),
           slr.LossFrame(64, p, p, p, p, float("nan"), 1.0, p, p), slr.LossFrame(64, p, p, p, p, 1.0, float("inf"), p, p),
           slr.LossFrame(64, p, p, p, p, 1.0, 1.0, p, None)]
    for b in bad:
        arr = (slr.LossFrame * 2)(good, b)
        assert L.slr_loss_l1_normal_frames(2, arr, None, None) == slr.SLR_E_INVALID
        assert b"frame 1" in L.slr_last_error()
    # an image without pixels needs no buffers
    arr = (slr.LossFrame * 1)(slr.LossFrame(0, None, None, None, None, 1.0, 1.0, None, None))
    assert L.slr_loss_l1_normal_frames(1, arr, None, None) != slr.SLR_E_INVALID


def test_autotune_cache_roundtrip(tmp_path, monkeypatch):
    """The persistent autotune cache: a tiling stored for an image-size class
    and device is found again (also through the environment variable), other
    classes and devices miss, and an unreadable file is an empty cache."""
    path = str(tmp_path / "tune.json")
    key = (((128, 1024), (64, 512)), (1000000,))
    assert slr.autotune_cache_lookup(key, "gpu-a", path) is None
    slr.autotune_cache_store(key, "gpu-a", (32, 8, 3, 2, 1, 0, 192), path)
    assert slr.autotune_cache_lookup(key, "gpu-a", path) == (32, 8, 3, 2, 1, 0, 192)
    assert slr.autotune_cache_lookup(key, "gpu-b", path) is None
    assert slr.autotune_cache_lookup((((128, 1024),), (1000000,)), "gpu-a", path) is None
    slr.autotune_cache_store(key, "gpu-b", (16, 16, 3, 2, 3, 0), path)
    assert slr.autotune_cache_lookup(key, "gpu-a", path) == (32, 8, 3, 2, 1, 0, 192)
    monkeypatch.setenv(slr.AUTOTUNE_CACHE_ENV, path)
    assert slr.autotune_cache_lookup(key, "gpu-b") == (16, 16, 3, 2, 3, 0)
    with open(path, "w") as f:
        f.write("{ not json")
    assert slr.autotune_cache_lookup(key, "gpu-a") is None
    slr.autotune_cache_store(key, "gpu-a", (8, 32, 3, 2, 1, 0), path)
    assert slr.autotune_cache_lookup(key, "gpu-a") == (8, 32, 3, 2, 1, 0)
    monkeypatch.delenv(slr.AUTOTUNE_CACHE_ENV)
    assert slr.autotune_cache_lookup(key, "gpu-a") is None   # no path: process-local only

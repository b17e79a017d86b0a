"""Support kernels through the C ABI against the oracle: the fused range +
normal loss and the fused Adam step."""
import sys

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda"
LR = {"means": 1e-3, "quats": 1e-3, "log_scales": 5e-3, "logits": 5e-2}


def say(*a):
    print("[gpu-support]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def slr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_17491_amd import slr as S
    S.lib()
    return S


@pytest.mark.parametrize("H,W", [(64, 512), (37, 300), (1, 1)])
def test_loss_matches_oracle(slr, H, W):
    say("loss", H, W)
    g = np.random.default_rng(H * W)
    P = H * W
    D = g.uniform(0, 30, P).astype(np.float32)
    Dt = (D + g.normal(0, 0.5, P)).astype(np.float32)
    Dt[g.uniform(size=P) < 0.2] = 0.0
    N = g.normal(size=(P, 3)).astype(np.float32)
    Nt = g.normal(size=(P, 3)).astype(np.float32)
    Dt[:3] = D[:3]    # exact ties: zero range gradient
    wd, wn = 1.0 / max(P, 1), 0.5 / max(P, 1)
    t = {k: torch.from_numpy(np.ascontiguousarray(v)).to(DEV) for k, v in dict(D=D, N=N, Dt=Dt, Nt=Nt).items()}
    gD = torch.empty(P, device=DEV); gN = torch.empty(P, 3, device=DEV)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    slr.loss_l1_normal(t["D"], t["N"], t["Dt"], t["Nt"], wd, wn, gD, gN, loss)
    torch.cuda.synchronize()
    L, rD, rN = O.loss_l1_normal(D, N, Dt, Nt, wd, wn)
    np.testing.assert_array_equal(gD.cpu().numpy(), rD)
    np.testing.assert_array_equal(gN.cpu().numpy(), rN)
    assert abs(loss.item() - L) <= 1e-6 * max(abs(L), 1e-30) + 1e-12


def test_loss_frames_matches_single_image_calls(slr):
    """18 images (two launches of at most 16), ragged sizes and an empty one:
    gradients bit-identical to one call per image and to the oracle; the
    summed loss to the oracle's sum."""
    g = np.random.default_rng(7)
    sizes = [(64, 512), (37, 300), (1, 1), (0, 0)] + [(16, 64)] * 14
    items, ref, Lsum = [], [], 0.0
    for k, (H, W) in enumerate(sizes):
        P = H * W
        D = g.uniform(0, 30, P).astype(np.float32)
        Dt = (D + g.normal(0, 0.5, P)).astype(np.float32)
        Dt[g.uniform(size=P) < 0.2] = 0.0
        N = g.normal(size=(P, 3)).astype(np.float32)
        Nt = g.normal(size=(P, 3)).astype(np.float32)
        wd, wn = 1.0 / max(P, 1), (0.5 + 0.1 * k) / max(P, 1)
        t = [torch.from_numpy(np.ascontiguousarray(v)).to(DEV) for v in (D, N, Dt, Nt)]
        gD = torch.full((P,), 7.0, device=DEV)
        gN = torch.full((P, 3), 7.0, device=DEV)
        items.append((t[0], t[1], t[2], t[3], wd, wn, gD, gN))
        L, rD, rN = O.loss_l1_normal(D, N, Dt, Nt, wd, wn)
        ref.append((rD, rN))
        Lsum += L
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    say("loss over", len(items), "images")
    slr.loss_l1_normal_frames(items, loss)
    torch.cuda.synchronize()
    for k, it in enumerate(items):
        gD1, gN1 = torch.empty_like(it[6]), torch.empty_like(it[7])
        slr.loss_l1_normal(it[0], it[1], it[2], it[3], it[4], it[5], gD1, gN1, None)
        torch.cuda.synchronize()
        assert torch.equal(it[6], gD1) and torch.equal(it[7], gN1), k
        np.testing.assert_array_equal(it[6].cpu().numpy(), ref[k][0])
        np.testing.assert_array_equal(it[7].cpu().numpy(), ref[k][1])
    assert abs(loss.item() - Lsum) <= 1e-6 * abs(Lsum)


@pytest.mark.parametrize("n", [1, 1000, 70001])
def test_adam_matches_oracle(slr, n):
    say("adam", n)
    g = np.random.default_rng(n)
    p = {"means": g.normal(size=(n, 3)), "quats": g.normal(size=(n, 4)), "log_scales": g.normal(size=(n, 2)),
         "logits": g.normal(size=n)}
    p = {k: v.astype(np.float32) for k, v in p.items()}
    dp = {k: torch.from_numpy(v.copy()).to(DEV) for k, v in p.items()}
    m = torch.zeros(n, 10, device=DEV); v = torch.zeros(n, 10, device=DEV)
    rm = np.zeros((n, 10)); rv = np.zeros((n, 10))
    cur = {k: x.astype(np.float64) for k, x in p.items()}
    gsum = np.zeros((n, 10))   # sum over steps of |g|: scale of the FP32 error of m
    for step in range(1, 4):
        gr = {k: (g.normal(size=x.shape) * 10.0 ** g.uniform(-3, 1, size=x.shape)).astype(np.float32)
              for k, x in p.items()}
        gsum += np.abs(np.concatenate([gr[k].reshape(n, -1) for k in ("means", "quats", "log_scales", "logits")], 1))
        slr.adam_step(dp, {k: torch.from_numpy(x).to(DEV) for k, x in gr.items()}, m, v, LR, step, eps=1e-15)
        cur, rm, rv = O.adam_step(cur, gr, rm, rv, LR, step, eps=1e-15)
    torch.cuda.synchronize()
    for k in p:
        got = dp[k].cpu().numpy().astype(np.float64)
        # each step moves a parameter by at most ~lr: FP32 rounding of the
        # parameter plus a relative 1e-5 of the accumulated steps
        tol = 4 * np.finfo(np.float32).eps * np.abs(cur[k]) + 1e-5 * 3 * LR[k]
        assert (np.abs(got - cur[k]) <= tol).all(), (k, float(np.abs(got - cur[k]).max()))
    # m = m + (1 - b1)(g - m) may cancel: bound its error by FP32 rounding of the gradients it summed
    dm = np.abs(m.cpu().numpy() - rm)
    assert (dm <= 1e-5 * np.abs(rm) + 8 * np.finfo(np.float32).eps * gsum).all(), float(dm.max())
    # v sums squares: no cancellation
    np.testing.assert_allclose(v.cpu().numpy(), rv, rtol=1e-5, atol=1e-30)

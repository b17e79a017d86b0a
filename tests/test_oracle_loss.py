"""Pins of the oracle's range + normal loss (Sec. 3.3.2): its gradients
against central finite differences of its own value (away from the kinks),
the valid mask, and a hand-computed two-pixel case."""
import numpy as np

import oracle as O


def test_loss_gradients_finite_differences():
    g = np.random.default_rng(0)
    P = 40
    D = g.uniform(1, 10, P); Dt = D + g.choice([-1, 1], P) * g.uniform(0.1, 1, P)
    Dt[::7] = 0.0   # invalid pixels
    N = g.normal(size=(P, 3)); Nt = g.normal(size=(P, 3))
    wd, wn = 0.3, 0.7
    L, gD, gN = O.loss_l1_normal(D, N, Dt, Nt, wd, wn)
    h = 1e-2   # inputs are rounded to FP32; every |D - D_t| is at least 0.1 here
    for p in range(P):
        Dp, Dm = D.copy(), D.copy(); Dp[p] += h; Dm[p] -= h
        fd = (O.loss_l1_normal(Dp, N, Dt, Nt, wd, wn)[0] - O.loss_l1_normal(Dm, N, Dt, Nt, wd, wn)[0]) / (2 * h)
        assert abs(fd - gD[p]) < 1e-3, (p, fd, gD[p])
        for c in range(3):
            Np, Nm = N.copy(), N.copy(); Np[p, c] += h; Nm[p, c] -= h
            fd = (O.loss_l1_normal(D, Np, Dt, Nt, wd, wn)[0] - O.loss_l1_normal(D, Nm, Dt, Nt, wd, wn)[0]) / (2 * h)
            assert abs(fd - gN[p, c]) < 1e-3, (p, c, fd, gN[p, c])
    assert not gD[::7].any() and not gN[::7].any()


def test_loss_two_pixels_by_hand():
    D = np.array([2.0, 5.0]); Dt = np.array([3.0, 4.5])
    N = np.array([[0, 0, 1.0], [1.0, 0, 0]]); Nt = np.array([[0, 0, 1.0], [0, 1.0, 0]])
    L, gD, gN = O.loss_l1_normal(D, N, Dt, Nt, 2.0, 3.0)
    # |2-3| * 2 + |5-4.5| * 2 + 3 * (1 - 1) + 3 * (1 - 0)
    assert abs(L - (2.0 + 1.0 + 0.0 + 3.0)) < 1e-12
    np.testing.assert_array_equal(gD, [-2.0, 2.0])
    np.testing.assert_array_equal(gN, [[0, 0, -3.0], [0, -3.0, 0]])

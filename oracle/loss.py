"""Range and normal losses of Sec. 3.3.2 and their gradients, by definition
(test infrastructure only).

  L = w_d * sum_valid |D - D_t| + w_n * sum_valid (1 - N . N_t),   valid = D_t > 0

with rho_d = 1 (the plain L1 range residual) and a given target normal N_t per
pixel.  dL/dD = w_d * sign(D - D_t) on valid pixels (0 at D = D_t), dL/dN =
-w_n * N_t.  The sign is decided in FP32, the precision of the range image.
"""
import numpy as np


def loss_l1_normal(D, N, Dt, Nt, w_d, w_n):
    D = np.asarray(D, np.float32).reshape(-1)
    Dt = np.asarray(Dt, np.float32).reshape(-1)
    N = np.asarray(N, np.float32).reshape(-1, 3)
    Nt = np.asarray(Nt, np.float32).reshape(-1, 3)
    valid = Dt > 0
    r32 = D - Dt                      # FP32 residual: decides the sign
    gD = np.where(valid, np.float32(w_d) * np.sign(r32), np.float32(0)).astype(np.float32)
    gN = np.where(valid[:, None], -np.float32(w_n) * Nt, np.float32(0)).astype(np.float32)
    r = D.astype(np.float64) - Dt.astype(np.float64)
    dot = (N.astype(np.float64) * Nt.astype(np.float64)).sum(1)
    L = float((w_d * np.abs(r) + w_n * (1.0 - dot))[valid].sum())
    return L, gD, gN

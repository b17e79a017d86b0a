"""Pins of the oracle's Adam (Kingma and Ba, Algorithm 1, bias-corrected).

* Three steps equal torch.optim.Adam (float64, CPU) on the same tensors.
* First step closed form: with m0 = v0 = 0 the update is -lr * g / (|g| + eps'),
  i.e. -lr * sign(g) up to eps.
"""
import numpy as np
import torch

import oracle as O

LR = {"means": 1e-3, "quats": 1e-3, "log_scales": 5e-3, "logits": 5e-2}


def random_set(n, seed):
    g = np.random.default_rng(seed)
    p = {"means": g.normal(size=(n, 3)), "quats": g.normal(size=(n, 4)), "log_scales": g.normal(size=(n, 2)),
         "logits": g.normal(size=n)}
    return p


def test_adam_matches_torch():
    n = 50
    p = random_set(n, 0)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam([{"params": [tp[k]], "lr": LR[k]} for k, _ in O.adam.GROUPS], betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros((n, 10)); v = np.zeros((n, 10))
    cur = {k: val.copy() for k, val in p.items()}
    for step in range(1, 4):
        grads = random_set(n, 10 + step)
        for k in tp:
            tp[k].grad = torch.tensor(grads[k], dtype=torch.float64)
        opt.step()
        cur, m, v = O.adam_step(cur, grads, m, v, LR, step, eps=1e-8)
        for k in tp:
            np.testing.assert_allclose(cur[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adam_first_step_closed_form():
    n = 20
    p = random_set(n, 1)
    g = random_set(n, 2)
    out, m, v = O.adam_step(p, g, np.zeros((n, 10)), np.zeros((n, 10)), LR, 1, eps=1e-15)
    for k in p:
        np.testing.assert_allclose(out[k] - p[k], -LR[k] * np.sign(g[k]), rtol=1e-9)

"""Adam on the raw surfel parameters, in FP64 (test infrastructure only).

Follows Algorithm 1 of Kingma and Ba, "Adam: A Method for Stochastic
Optimization" (ICLR 2015), in the bias-corrected form where the correction is
applied to the step size and the denominator, and eps is added after the
correction of the second moment (the form PyTorch implements).  The map
refinement of Sec. 3.3.2 optimises the surfel parameters with Adam; one
learning rate per parameter group.
"""
import numpy as np

GROUPS = (("means", 3), ("quats", 4), ("log_scales", 2), ("logits", 1))


def adam_step(params, grads, m, v, lr, step, betas=(0.9, 0.999), eps=1e-15):
    """params, grads: dicts of arrays [n, k] (logits [n]); m, v: [n, 10] moments
    in group order.  Returns (new params, new m, new v), all float64."""
    b1, b2 = betas
    m = np.asarray(m, np.float64).copy()
    v = np.asarray(v, np.float64).copy()
    out = {}
    c = 0
    for name, k in GROUPS:
        p = np.asarray(params[name], np.float64).reshape(-1, k).copy()
        g = np.asarray(grads[name], np.float64).reshape(-1, k)
        mm, vv = m[:, c:c + k], v[:, c:c + k]
        mm[:] = b1 * mm + (1.0 - b1) * g
        vv[:] = b2 * vv + (1.0 - b2) * g * g
        m_hat = mm / (1.0 - b1 ** step)
        v_hat_sqrt = np.sqrt(vv) / np.sqrt(1.0 - b2 ** step)
        p -= lr[name] * m_hat / (v_hat_sqrt + eps)
        out[name] = p.reshape(np.shape(params[name]))
        c += k
    return out, m, v

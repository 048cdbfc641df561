"""Adam with the AMSGrad variant, Eqs. (8)-(13) of the paper, in FP64 numpy.

TEST INFRASTRUCTURE ONLY (part of the oracle).

State per parameter: first moment m, second moment v, and the running maximum
``vmax``. Step t is 1-based; the initial state is all zeros.

Modes:
  "paper": the running maximum is taken over the bias-corrected second moment
           v_hat_t = v_t / (1 - beta2^t), and theta -= lr * m_hat / (sqrt(vmax) + eps)
           (Eqs. 12-13 as printed);
  "torch": the running maximum is taken over the raw v_t and divided by the bias
           correction afterwards (the formulation of torch.optim.Adam with amsgrad);
  "off":   plain Adam, no running maximum.
"""

from __future__ import annotations

import numpy as np


def adam_step(theta, grad, m, v, vmax, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, mode="paper"):
    """Return the new (theta, m, v, vmax) after step ``t`` (1-based)."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    bc1 = 1.0 - beta1 ** t
    bc2 = 1.0 - beta2 ** t
    m_hat = m / bc1
    vmax = np.asarray(vmax, dtype=np.float64)
    if mode == "paper":
        vmax = np.maximum(vmax, v / bc2)
        denom = np.sqrt(vmax) + eps
    elif mode == "torch":
        vmax = np.maximum(vmax, v)
        denom = np.sqrt(vmax) / np.sqrt(bc2) + eps
    elif mode == "off":
        denom = np.sqrt(v / bc2) + eps
    else:
        raise ValueError(mode)
    theta = theta - lr * m_hat / denom
    return theta, m, v, vmax

"""Adam update, FP64 (test infrastructure only).

Adam as the paper uses it for the object, probe and position corrections
(Sec. S1.F "Optimizer", the AdamOptimizer class; step sizes from the user
interface listing): first and second moment estimates with bias correction.
The moment decay rates and epsilon are not given in the paper; the published
defaults of the Adam method (beta1 0.9, beta2 0.999, eps 1e-8) are used
unless a caller passes others.
"""
from __future__ import annotations

import numpy as np


def adam_step(x, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at iteration t (1-based).  Returns new (x, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return x - lr * m_hat / (np.sqrt(v_hat) + eps), m, v

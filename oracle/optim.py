"""First-order baseline of the optimiser comparison (plain FP64 numpy).

Test infrastructure: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may use this module.

The paper compares IRL with standard Lanczos and with Adam (Results,
"Efficiency and Numerical Stability of IRL Optimization", Fig. 2; Methods,
"Practical Matrix-Free Implementation", costs one Adam step as one gradient
evaluation).  Adam is the published algorithm of Kingma and Ba: exponential
moving averages of the gradient and of its elementwise square, each divided by
its bias (1 - beta^t), and a step of lr * m_hat / (sqrt(v_hat) + eps) against the
gradient.
"""
from __future__ import annotations

import numpy as np


def adam_step(theta: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int,
              lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step with step count t >= 1.  Returns (theta', m', v')."""
    if t < 1:
        raise ValueError("the step count starts at 1")
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v

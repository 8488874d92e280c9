"""FP64 oracle of the refinement optimizer step (test infrastructure only).

Adam as defined by Kingma & Ba (2015, Algorithm 1) -- the paper's map
refinement (Sec. 3.3) names no optimizer -- taken in the parameterisation
each surfel tensor names: theta = p (linear), theta = log p (tangent
scales), theta = log(p / (1 - p)) (opacity).  Written from the definition
with numpy; shares nothing with the HIP path.
"""
from __future__ import annotations

import numpy as np

LINEAR, LOG, LOGIT = 0, 1, 2
LOGIT_CLAMP = 1e-6   # logit parameters are first clamped into [1e-6, 1 - 1e-6]
LOG_FLOOR = 1e-30    # log parameters are first raised to >= 1e-30


def to_theta(p, g, kind):
    """(theta, dL/dtheta) from the activated value p and dL/dp."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    if kind == LOG:
        p = np.maximum(p, LOG_FLOOR)
        return np.log(p), g * p
    if kind == LOGIT:
        p = np.clip(p, LOGIT_CLAMP, 1.0 - LOGIT_CLAMP)
        return np.log(p) - np.log1p(-p), g * p * (1.0 - p)
    return p.copy(), g.copy()


def from_theta(theta, kind):
    if kind == LOG:
        return np.exp(theta)
    if kind == LOGIT:
        return 1.0 / (1.0 + np.exp(-theta))
    return theta


def adam_step(p, g, m, v, t, lr, kind=LINEAR, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step at step number t (>= 1).  Returns (p, m, v) as new arrays."""
    theta, gt = to_theta(p, g, kind)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * gt
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * gt * gt
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    theta = theta - lr * m_hat / (np.sqrt(v_hat) + eps)
    return from_theta(theta, kind), m, v

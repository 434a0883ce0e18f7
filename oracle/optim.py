"""Optimizer of the paper's training (Sec. V.D), in float64: Adam with the
gradient clipped at a global L2 norm, and a cosine-annealed learning rate.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this package.

Adam (Kingma and Ba, 2015, Algorithm 1), step t = 1, 2, ...:
  m_t = b1 m_{t-1} + (1 - b1) g_t          first moment
  v_t = b2 v_{t-1} + (1 - b2) g_t^2        second moment
  p_t = p_{t-1} - lr (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps)
Clipping by the global norm: g <- g min(1, c / (||g||_2 + 1e-6)).
Cosine annealing (Loshchilov and Hutter, 2017, without restarts):
  lr(t) = lr_min + (lr_max - lr_min) (1 + cos(pi t / T)) / 2.
"""
from __future__ import annotations

import numpy as np


def clip_by_global_norm(grad, max_norm: float):
    """(scaled gradient, norm before scaling); max_norm <= 0 leaves it as is."""
    g = np.asarray(grad, dtype=np.float64)
    norm = float(np.sqrt((g * g).sum()))
    if max_norm <= 0:
        return g, norm
    return g * min(1.0, max_norm / (norm + 1e-6)), norm


def adam_step(params, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8,
              clip: float = 0.0):
    """One step; returns (params, m, v, norm) as new float64 arrays."""
    g, norm = clip_by_global_norm(grad, clip)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    p = np.asarray(params, np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v, norm


def cosine_lr(t: int, total: int, lr_max: float, lr_min: float) -> float:
    if total <= 0:
        return lr_min
    x = min(max(t, 0), total) / total
    return lr_min + 0.5 * (lr_max - lr_min) * (1.0 + np.cos(np.pi * x))

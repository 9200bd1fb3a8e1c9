"""Oracle of the fitting loop's own arithmetic (test infrastructure only).

Plain float64 numpy, written from the definitions; only the test suite
imports it.

* ``light_reg``: the light term of the objective (Eq. 1), w2 E_light with
  E_light = sum_j |l_j - m_j|^2 and m_j the mean intensity of light j, read
  here as the mean of its three channels (the paper gives no formula for
  m_j).  The gradient 2 w2 (l_j - m_j) is the same whether m_j is held fixed
  or differentiated, because the deviations of one light sum to zero.
* ``adam``: one Adam step (Kingma and Ba 2015, Algorithm 1): biased first
  and second moment estimates, their bias corrections 1 - beta^t, and the
  update lr * m_hat / (sqrt(v_hat) + eps).  The paper does not name its
  optimiser; Adam is the reading taken for the fitting loop.
"""
from __future__ import annotations

import numpy as np


def light_reg(lights, w2: float):
    """Return (w2 * E_light, its gradient) for lights [n][3]."""
    L = np.asarray(lights, np.float64)
    m = L.mean(axis=1, keepdims=True)
    d = L - m
    return w2 * float((d * d).sum()), 2.0 * w2 * d


def adam(p, g, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns the new (p, m, v)."""
    p, g, m, v = (np.asarray(x, np.float64) for x in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v

"""Partial-fraction expansion of the inverse square root.

Test infrastructure only (see ``oracle/__init__.py``).

Eq. (1.2) replaces f(A) b = A^{-1/2} b by sum_s w_s (A + sigma_s)^{-1} b.  The
paper uses Neuberger's expansion (Fig. 1 and Fig. 3 captions), whose poles and
weights are

  theta_s = pi (s - 1/2) / (2 N),  sigma_s = tan^2 theta_s,
  w_s     = 1 / (N cos^2 theta_s),                  s = 1..N.

For x > 0 it equals x^{-1/2} times the rational function
  [(1 + sqrt x)^{2N} - (1 - sqrt x)^{2N}] / [(1 + sqrt x)^{2N} + (1 - sqrt x)^{2N}],
which the pinning tests use as an independent closed form.
"""
from __future__ import annotations

import numpy as np


def neuberger(n: int):
    """(sigma, w) of the N-pole Neuberger expansion, each shape (n,) float64."""
    s = np.arange(1, n + 1, dtype=np.float64)
    theta = np.pi * (s - 0.5) / (2.0 * n)
    sigma = np.tan(theta) ** 2
    w = 1.0 / (n * np.cos(theta) ** 2)
    return sigma, w


def pfe_scalar(x, sigma, w):
    """sum_s w_s / (x + sigma_s) for scalar or array x (real or complex)."""
    x = np.asarray(x)[..., None]
    return np.sum(w / (x + sigma), axis=-1)

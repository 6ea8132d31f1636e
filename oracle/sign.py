"""sign(H) b and the overlap operator from the PFE solve.

Test infrastructure only (see ``oracle/__init__.py``).

Section 1: D_ov(mu) = 1 + gamma5 sign(gamma5 D_w(mu)) (Eq. (1.1)), and
sign z = z / sqrt(z^2), so with H = gamma5 D_w and A = a H^2,
  sign(H) b = H (H^2)^{-1/2} b = sqrt(a) H f(A) b,   f(A) = A^{-1/2},
where f(A) b is the partial-fraction sum of Eq. (1.2).
"""
from __future__ import annotations

import numpy as np

from . import dirac, krylov


def pfe_sign_apply(op: dirac.Dirac, a_scale, b, sigmas, weights, l, tol,
                   max_outer, pass_=1, overlap=False):
    """sign(H) b (or D_ov b = b + gamma5 sign(H) b) through multi-shift BiCGstab(l)."""
    res = krylov.mshift_bicgstabl(lambda v: op.a_op(v, a_scale), b, sigmas,
                                  weights, l, tol, max_outer, pass_)
    y, info = res[0], res[1]
    out = np.sqrt(a_scale) * op.h(y)
    if overlap:
        out = b + dirac.g5(out)
    return out, info

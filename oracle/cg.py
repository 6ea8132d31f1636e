"""Multi-shift conjugate gradients for a Hermitian positive semi-definite A:
the single pass, Neuberger's double pass and the pseudo-double pass.

Test infrastructure only (see ``oracle/__init__.py``).

What is computed
----------------
y = sum_s w_s (A + sigma_s)^{-1} b (Eq. (1.2)) when A is Hermitian -- the
overlap kernel at mu = 0, where gamma5 D_w is Hermitian and A = a (gamma5
D_w)^2 is positive semi-definite.  This is the setting of Neuberger's
double-pass multi-shift CG, which Section 2 of the paper takes as the model
for its BiCGstab(l) variants, and of the pseudo-double pass that the
concluding section proposes for CG as well.

Seed: CG on S = A + sigma_0, sigma_0 = min_s sigma_s, x0 = 0, r_0 = p_0 = b:
    alpha_k = (r_k, r_k) / (p_k, S p_k),   r_{k+1} = r_k - alpha_k S p_k,
    beta_k = (r_{k+1}, r_{k+1}) / (r_k, r_k),   p_{k+1} = r_{k+1} + beta_k p_k.
Its residual polynomial (r_k = R_k(S) b) obeys
    R_{k+1}(t) = (1 + d_k - alpha_k t) R_k(t) - d_k R_{k-1}(t),
    d_k = alpha_k beta_{k-1} / alpha_{k-1}  (d_0 = 0).
Shift s, sigma' = sigma_s - sigma_0 >= 0: the CG iterate of (S + sigma') x = b
in the same Krylov space has the collinear residual r_k / zeta_k with
zeta_k = R_k(-sigma'), so
    zeta_{k+1} = (1 + d_k + alpha_k sigma') zeta_k - d_k zeta_{k-1},
and matching the shifted CG's own recurrences gives
    alpha^s_k = alpha_k zeta_k / zeta_{k+1},
    beta^s_k = beta_k (zeta_k / zeta_{k+1})^2,
    x^s += alpha^s_k p^s_k,   p^s_{k+1} = r_{k+1} / zeta_{k+1} + beta^s_k p^s_k,
    p^s_0 = b.
Freezing: shift s stops at the first k with ||r_k|| / |zeta_k| <= 0.9 tol ||b||
(its M_s = k; x^s then holds the terms k' < M_s); the seed stops when no
shift is active.  The fraction 0.9 leaves room for the rounding drift between
the recursive and the true residual, as in the BiCGstab(l) oracle.

Double pass (Neuberger).  Expanding p^s_k over the seed residuals,
    x^s = sum_{i < M_s} (e^s_i / zeta^s_i) r_i,
    e^s_{M_s - 1} = alpha^s_{M_s - 1},  e^s_i = alpha^s_i + beta^s_i e^s_{i+1},
so y = sum_i c_i r_i with c_i = sum_{s: i < M_s} w_s e^s_i / zeta^s_i.  Pass 1
runs the seed and the shift scalars only (recording alpha_k, beta_k, M_s);
the coefficients follow from the recorded scalars; pass 2 regenerates r_i from
b with the recorded alpha_k, beta_k (no inner products) and sums c_i r_i.
Pseudo-double pass: pass 1 keeps r_0 .. r_{N-1} and sums them directly.

Inner product (a, b) = sum conj(a_i) b_i; for Hermitian S the CG scalars are
real and their real parts are used.  All arithmetic complex128/float64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from .krylov import FREEZE_FRAC

OK, NOT_CONVERGED, BREAKDOWN = 0, 4, 5


def _dot_re(a, b) -> float:
    return float(np.vdot(a, b).real)


@dataclass
class CGInfo:
    iters: int = 0                       # seed iterations run (N)
    status: int = OK
    mv: int = 0
    dots: int = 0
    shift_iters: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=int))
    shift_resid: np.ndarray = field(default_factory=lambda: np.zeros(0))
    alphas: List[float] = field(default_factory=list)
    betas: List[float] = field(default_factory=list)


def _shift_scalars(alphas, betas, sp, M):
    """zeta_0..zeta_M, alpha^s_0..alpha^s_{M-1}, beta^s_0..beta^s_{M-1} of one
    shift from the seed's recorded alpha_k, beta_k (the same recurrences as
    the single pass)."""
    z = [1.0]
    zprev = 1.0
    a_s, b_s = [], []
    for k in range(M):
        d = alphas[k] * betas[k - 1] / alphas[k - 1] if k > 0 else 0.0
        zn = (1.0 + d + alphas[k] * sp) * z[k] - d * zprev
        a_s.append(alphas[k] * z[k] / zn)
        b_s.append(betas[k] * (z[k] / zn) ** 2)
        zprev = z[k]
        z.append(zn)
    return z, a_s, b_s


def double_pass_coefficients(alphas, betas, sps, weights, M):
    """c_i, i = 0..max(M)-1, such that sum_s w_s x^s = sum_i c_i r_i."""
    N = int(max(M)) if len(M) else 0
    c = np.zeros(N)
    for s in range(len(sps)):
        Ms = int(M[s])
        if Ms == 0:
            continue
        z, a_s, b_s = _shift_scalars(alphas, betas, sps[s], Ms)
        e = a_s[Ms - 1]
        c[Ms - 1] += weights[s] * e / z[Ms - 1]
        for i in range(Ms - 2, -1, -1):
            e = a_s[i] + b_s[i] * e
            c[i] += weights[s] * e / z[i]
    return c


def mshift_cg(a_mv: Callable, b: np.ndarray, sigmas, weights, tol: float, max_iter: int, pass_: int = 1,
              force_iters=None, want_shifts: bool = False):
    """y = sum_s w_s (A + sigma_s)^{-1} b by multi-shift CG.

    a_mv(v) = A v (Hermitian).  pass_ 1: single pass; 2: double pass;
    3: pseudo-double pass.  force_iters: per-shift freeze iterations M_s
    (replaces the residual test).  Returns (y, info) or, with want_shifts and
    pass_ 1, (y, info, x_shifts)."""
    sig = np.asarray(sigmas, dtype=float)
    w = np.asarray(weights, dtype=float)
    ns = len(sig)
    s0 = float(sig.min())
    sps = sig - s0
    info = CGInfo(shift_iters=np.zeros(ns, dtype=int), shift_resid=np.zeros(ns))
    bn = float(np.linalg.norm(b))
    y = np.zeros_like(b, dtype=complex)
    xs = np.zeros((ns,) + b.shape, dtype=complex) if pass_ == 1 else None
    if bn == 0.0:
        return (y, info, xs) if (want_shifts and pass_ == 1) else (y, info)
    force = None if force_iters is None else np.asarray(force_iters, dtype=int)

    def S(v):
        return a_mv(v) + s0 * v

    r = b.astype(complex).copy()
    p = r.copy()
    rr = _dot_re(r, r)
    zeta = np.ones(ns)
    zprev = np.ones(ns)
    active = np.ones(ns, dtype=bool)
    ps = [r.copy() for _ in range(ns)] if pass_ == 1 else None
    stored = [r.copy()] if pass_ == 3 else None
    alpha_prev, beta_prev = 1.0, 0.0
    k = 0
    while active.any() and k < max_iter:
        wv = S(p)
        info.mv += 1
        pw = _dot_re(p, wv)
        info.dots += 1
        if not (pw > 0.0) or not np.isfinite(pw):
            info.status = BREAKDOWN
            break
        alpha = rr / pw
        d = alpha * beta_prev / alpha_prev if k > 0 else 0.0
        znext = np.where(active, (1.0 + d + alpha * sps) * zeta - d * zprev, zeta)
        for s in range(ns):
            if active[s] and pass_ == 1:
                xs[s] += (alpha * zeta[s] / znext[s]) * ps[s]
        r = r - alpha * wv
        rr_new = _dot_re(r, r)
        info.dots += 1
        beta = rr_new / rr
        info.alphas.append(alpha)
        info.betas.append(beta)
        for s in range(ns):
            if not active[s]:
                continue
            if pass_ == 1:
                ps[s] = r / znext[s] + (beta * (zeta[s] / znext[s]) ** 2) * ps[s]
            zprev[s] = zeta[s]
            zeta[s] = znext[s]
            res = np.sqrt(rr_new) / abs(zeta[s]) / bn
            info.shift_resid[s] = res
            done = (k + 1 >= force[s]) if force is not None else (res <= FREEZE_FRAC * tol)
            if done:
                active[s] = False
                info.shift_iters[s] = k + 1
        p = r + beta * p
        if pass_ == 3 and active.any():
            stored.append(r.copy())
        rr = rr_new
        alpha_prev, beta_prev = alpha, beta
        k += 1
    info.iters = k
    for s in range(ns):
        if active[s]:
            info.shift_iters[s] = k
            if info.status == OK:
                info.status = NOT_CONVERGED
    if pass_ == 1:
        for s in range(ns):
            y += w[s] * xs[s]
        return (y, info, xs) if want_shifts else (y, info)
    c = double_pass_coefficients(info.alphas, info.betas, sps, w, info.shift_iters)
    if pass_ == 3:
        for i in range(len(c)):
            y += c[i] * stored[i]
        return y, info
    # pass 2: regenerate r_0 .. r_{N-1} from b with the recorded scalars
    r = b.astype(complex).copy()
    p = r.copy()
    if len(c):
        y += c[0] * r
    for kk in range(len(c) - 1):
        wv = S(p)
        info.mv += 1
        r = r - info.alphas[kk] * wv
        y += c[kk + 1] * r
        p = r + info.betas[kk] * p
    return y, info

"""Gradients of L = Re <eta, y>, y = f(A) b (or y = sign(H) b).

Test infrastructure only (see ``oracle/__init__.py``).  Not in the paper:
the backward of the partial-fraction sum of Eq. (1.2), with the adjoint
solves done by the same multi-shift method.

Definitions: F = sum_s w_s (A + sigma_s)^{-1}, A = a H^2, H = gamma5 D_w(mu),
x_s = (A + sigma_s)^{-1} b, z_s = (A^+ + sigma_s)^{-1} eta.  Because
D(mu)^+ = gamma5 D(-mu) gamma5, H(mu)^+ = H(-mu) and A^+ = A(-mu): the adjoint
solves are forward solves at -mu.  Gradients of a real L are reported as
dL/dRe + i dL/dIm (the convention of PyTorch):

  grad_b       = F^+ eta = sum_s w_s z_s
  grad_w_s     = Re <eta, x_s>
  grad_sigma_s = -w_s Re <z_s, x_s>
  links        dL = -sum_s w_s Re <z_s, dA x_s>,  dA = a (dH H + H dH),
               dH = gamma5 dD, so dL = sum over pairs c Re <p, dD q> with
               c = -a w_s and (p, q) = (gamma5 z_s, H x_s), (gamma5 H(-mu) z_s, x_s).
  For sign(H) b = sqrt(a) H y the chain rule adds the pair (gamma5 eta, y)
  with c = sqrt(a) and replaces eta by sqrt(a) H(-mu) eta in the rest.

The link derivative of <p, dD q>: U_nu(x) enters (D q)(x) through the forward
hop and (D q)(x+nu) through the backward hop, so with
  M1_ab = sum_alpha conj(p(x)_{alpha a}) [(1 - gamma_nu) q(x+nu)]_{alpha b}
  M2_ab = sum_alpha conj(p(x+nu)_{alpha a}) [(1 + gamma_nu) q(x)]_{alpha b}
the gradient is  G_nu(x) += -c b_nu(x)/2 [e^{mu d_nu4} conj(M1) + e^{-mu d_nu4} M2^T].
"""
from __future__ import annotations

import numpy as np

from . import dirac, krylov


def link_force(op: dirac.Dirac, pairs, mu: float | None = None) -> np.ndarray:
    """sum over (c, p, q) of the gradient of c Re <p, D(mu) q> w.r.t. the links.

    p, q in [12][V] layout; returns [4][3][3][V] complex128."""
    mu = op.mu if mu is None else mu
    G = np.zeros((4,) + op.U.shape[1:], dtype=np.complex128)   # (4, t, z, y, x, 3, 3)
    for c, p, q in pairs:
        pg = dirac.spinor_to_grid(p, op.dims)
        qg = dirac.spinor_to_grid(q, op.dims)
        for nu in range(4):
            ax = 3 - nu
            qf = np.roll(qg, -1, axis=ax)                        # q(x + nu)
            pf = np.roll(pg, -1, axis=ax)                        # p(x + nu)
            proj1 = qf - dirac._spin_mul(dirac.GAMMA[nu], qf)   # (1 - gamma) q(x+nu)
            proj2 = qg + dirac._spin_mul(dirac.GAMMA[nu], qg)   # (1 + gamma) q(x)
            M1 = np.einsum("...sa,...sb->...ab", pg.conj(), proj1)
            M2 = np.einsum("...sa,...sb->...ab", pf.conj(), proj2)
            ef, eb = (np.exp(mu), np.exp(-mu)) if nu == 3 else (1.0, 1.0)
            bnu = op.bt if nu == 3 else 1.0                       # b_nu(x), shape (Lt,1,1,1,1,1)
            G[nu] += (-0.5 * c) * bnu * (ef * M1.conj() + eb * np.swapaxes(M2, -1, -2))
    return dirac.links_from_grid(G)


def shift_solutions(op, a, rhs, sigmas, weights, l, tol, max_outer, mu):
    res = krylov.mshift_bicgstabl(lambda v: op.a_op(v, a, mu), rhs, sigmas, weights, l, tol,
                                  max_outer, 1)
    return res[0], res[1], res[2]


def fab_backward(op: dirac.Dirac, a, b, eta, sigmas, weights, l, tol, max_outer, mode=0):
    """(grad_b, grad_w, grad_sigma, grad_links) of Re <eta, y>.

    mode 0: y = f(A) b; mode 1: y = sign(H) b = sqrt(a) H f(A) b."""
    sigmas = np.asarray(sigmas, dtype=np.float64)
    weights = np.asarray(weights, dtype=np.float64)
    mu = op.mu
    y, _, X = shift_solutions(op, a, b, sigmas, weights, l, tol, max_outer, mu)
    pairs = []
    if mode == 1:
        # L = Re <eta, sqrt(a) H y>: direct link term and eta' = sqrt(a) H^+ eta
        pairs.append((np.sqrt(a), dirac.g5(eta), y))
        eta = np.sqrt(a) * op.h(eta, -mu)
    gb, _, Z = shift_solutions(op, a, eta, sigmas, weights, l, tol, max_outer, -mu)
    gw = np.array([np.vdot(eta, X[s]).real for s in range(len(sigmas))])
    gs = np.array([-weights[s] * np.vdot(Z[s], X[s]).real for s in range(len(sigmas))])
    for s in range(len(sigmas)):
        c = -a * weights[s]
        pairs.append((c, dirac.g5(Z[s]), op.h(X[s], mu)))
        pairs.append((c, dirac.g5(op.h(Z[s], -mu)), X[s]))
    GU = link_force(op, pairs, mu)
    return gb, gw, gs, GU


def loss(op_factory, a, b, eta, sigmas, weights, l, tol, max_outer, mode=0):
    """L = Re <eta, y> for finite differences (op_factory() builds the operator)."""
    op = op_factory()
    y, _, _ = shift_solutions(op, a, b, sigmas, weights, l, tol, max_outer, op.mu)
    if mode == 1:
        y = np.sqrt(a) * op.h(y)
    return float(np.vdot(eta, y).real)

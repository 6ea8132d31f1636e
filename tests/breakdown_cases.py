"""Inputs that drive multi-shift BiCGstab(l) into each of its breakdown
branches, built with the oracle's operator only (shared by the oracle pins and
the GPU parity tests).

* gamma breakdown after S u_j (step j = 0 or 1 of the first outer
  iteration): a shadow residual r~ = b + t z with <r~, u_{j+1}> = 0.  In the
  first outer iteration every BiCG scalar is a function of the moments
  m_k = <r~, S^k b>: rho = m_0, gamma_0 = m_1, and (writing out steps 0 and
  1) gamma_1 = (m_0 / m_1^2)(m_2^2 - m_1 m_3), so gamma_0 = 0 is linear and
  gamma_1 = 0 (the 2 x 2 Hankel determinant of the moments, the classical
  Lanczos breakdown condition) quadratic in conj(t).
* Cholesky truncation of the MR normal equations: on the free field A is a
  scalar A(p) on each plane wave (a normal operator with orthogonal plane-wave
  eigenvectors).  With b the sum of 7 waves of distinct A(p) and r~ the sum
  of 4 of them, the BiCG polynomial R_4 after the l = 4 steps of the first
  outer iteration satisfies <r~, S^i R_4(S) b> = 0 for i < 4, a Vandermonde
  system on the 4 eigenvalues r~ sees, so R_4 vanishes there: r_0 keeps 3
  eigencomponents, the MR vectors S r_0 .. S^4 r_0 span 3 dimensions and the
  4th Cholesky pivot is rounding noise.  The 3-term MR step then solves the
  system exactly: every x_s equals the plane-wave solution.
* a shift breakdown, zeta_1 = R_1(-sigma') = 1 + alpha_0 sigma' = 0 for one
  shift sigma'_k: alpha_0 = m_0 / m_1, so a shadow residual with
  <r~, (S + sigma'_k) b> = 0 (linear in conj(t)) makes the shifted BiCG
  recurrence of that shift end at its first step.
* a shift whose |zeta psi| outgrows 1e300: sigma' = 1e60 with forced
  iterations (an unforced run freezes it at once, its residual estimate being
  ~1e-60).  It stops there as converged; its solution is (A + sigma_s)^{-1} b
  to rounding.
"""
from __future__ import annotations

import numpy as np

import workloads as wl
from oracle import dirac as od
from oracle import pfe


def _dot(x, y):
    return complex(np.vdot(x, y))


def gamma_breakdown_shadow(op, a, sigma0, b, z, step):
    """r~ = b + t z with gamma_step = <r~, S u_{step+1}> = 0 in the first
    outer iteration of BiCGstab(l) on S = a H^2 + sigma0 (step 0 or 1)."""
    S = lambda v: op.a_op(v, a) + sigma0 * v
    K = [b]
    for _ in range(3):
        K.append(S(K[-1]))
    A = [_dot(b, v) for v in K]      # moments of b
    B = [_dot(z, v) for v in K]      # moments of z; m_k = A_k + conj(t) B_k
    if step == 0:
        tau = -A[1] / B[1]
    else:
        qa = B[2] ** 2 - B[1] * B[3]
        qb = 2 * A[2] * B[2] - A[1] * B[3] - A[3] * B[1]
        qc = A[2] ** 2 - A[1] * A[3]
        tau = (-qb + np.sqrt(qb * qb - 4 * qa * qc)) / (2 * qa)
    return b + np.conj(tau) * z


def zeta_breakdown_shadow(op, a, sigma0, sigma_k, b, z):
    """r~ = b + t z with <r~, (A + sigma_k) b> = 0: zeta_1 of the shift
    sigma_k vanishes in the first BiCG step on S = a H^2 + sigma0."""
    Ab = op.a_op(b, a) + sigma_k * b
    tau = -_dot(b, Ab) / _dot(z, Ab)
    return b + np.conj(tau) * z


def zeta_case():
    """(workload, links, operator, a, sigma, w, b, r~, k) on the 4^3x8
    lattice: the shadow residual breaks the shifted recurrence of shift k."""
    wk = wl.WORKLOADS["4x4x4x8"]
    U = wk.links()
    op = od.Dirac(U, wk.dims, wk.mass, wk.mu, wk.bc_t)
    a = 1.0 / (1.01 * 36.5)
    sig, w = pfe.neuberger(wk.n_shift)
    b = wk.sources()[0]
    z = wl.gaussian_source(wk.dims, 7302)[0]
    k = 4
    return wk, U, op, a, sig, w, b, zeta_breakdown_shadow(op, a, sig.min(), sig[k], b, z), k


def gamma_case(step):
    """(workload, links, operator, a, sigma, w, b, r~) on the 4^3x8 lattice."""
    wk = wl.WORKLOADS["4x4x4x8"]
    U = wk.links()
    op = od.Dirac(U, wk.dims, wk.mass, wk.mu, wk.bc_t)
    a = 1.0 / (1.01 * 36.5)
    sig, w = pfe.neuberger(wk.n_shift)
    b = wk.sources()[0]
    z = wl.gaussian_source(wk.dims, 7301)[0]
    return wk, U, op, a, sig, w, b, gamma_breakdown_shadow(op, a, sig.min(), b, z, step)


def plane_wave(dims, n, chi):
    """e^{i p x} chi with p_k = 2 pi n_k / L_k (space), pi (2 n_4 + 1) / L_t (time)."""
    Lx, Ly, Lz, Lt = dims
    t, zz, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    p = [2 * np.pi * n[0] / Lx, 2 * np.pi * n[1] / Ly, 2 * np.pi * n[2] / Lz, np.pi * (2 * n[3] + 1) / Lt]
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * zz + p[3] * t)).reshape(-1)
    return chi[:, None] * ph[None, :], p


def free_eigenvalue(p, mass, mu, a):
    """A(p) = a [(4 + m - sum cos q)^2 + sum sin^2 q], q_4 = p_4 - i mu."""
    q = np.array(p, dtype=complex)
    q[3] -= 1j * mu
    return a * ((4 + mass - np.sum(np.cos(q))) ** 2 + np.sum(np.sin(q) ** 2))


CHOL_MOMENTA = [(0, 0, 0, 0), (1, 0, 0, 1), (1, 1, 0, 2), (2, 1, 1, 3), (1, 2, 2, 0), (2, 2, 2, 1), (0, 1, 2, 3)]
CHOL_SEEN = [0, 2, 4, 6]


def cholesky_case():
    """(dims, mass, mu, links, a, sigma, w, b, r~, waves, eigenvalues) on the
    free 4^3x8 lattice at mu = 0.05."""
    dims, mass, mu = (4, 4, 4, 8), -2.0, 0.05
    a = 1.0 / 36.5
    waves, lams = [], []
    for k, n in enumerate(CHOL_MOMENTA):
        chi = np.zeros(12, dtype=complex)
        chi[k % 12] = 1.0
        v, p = plane_wave(dims, n, chi)
        waves.append(v)
        lams.append(free_eigenvalue(p, mass, mu, a))
    b = sum(waves)
    rt = sum(waves[k] for k in CHOL_SEEN)
    sig, w = pfe.neuberger(10)
    return dims, mass, mu, wl.free_links(dims), a, sig, w, b, rt, waves, np.array(lams)


BIG_SHIFT = 1e60


def big_shift_case():
    """(workload, links, operator, a, sigma, w, b): three ordinary shifts and
    one of 1e60 on the 4^3x8 lattice."""
    wk = wl.WORKLOADS["4x4x4x8"]
    U = wk.links()
    op = od.Dirac(U, wk.dims, wk.mass, wk.mu, wk.bc_t)
    a = 1.0 / (1.01 * 36.5)
    sig = np.array([0.01, 0.1, 1.0, BIG_SHIFT])
    w = np.array([1.0, 0.5, 0.25, 1.0])
    return wk, U, op, a, sig, w, wk.sources()[0]

"""Low-mode deflation of the sign function at mu = 0 (H = gamma5 D_w Hermitian).

Test infrastructure only (see ``oracle/__init__.py``).

What is computed
----------------
The paper's overlap benchmarks deflate the eigenvalues of H = gamma5 D_w of
smallest modulus (Figs. 1, 3 and 4 state the number deflated): with the
eigenpairs (lambda_k, v_k), k < K, computed exactly,

    sign(H) b = sum_{k<K} sign(lambda_k) v_k <v_k, b> + sign(H) P b,
    P b = b - sum_{k<K} v_k <v_k, b>,

and only the second term is approximated, by sign(H) = sqrt(a) H f(a H^2)
with the partial-fraction expansion f(A) = sum_s w_s (A + sigma_s)^{-1}
(Eq. (1.2)).  The spectrum of H^2 seen by P b starts at lambda_K^2 instead of
lambda_0^2, so the same poles reach a smaller error.  At mu = 0 H is
Hermitian and the v_k are orthonormal (one set of vectors; at mu != 0 the
paper's deflation needs left and right eigenvectors, which this module does
not treat).

Here the eigenpairs come from a dense Hermitian eigensolver of the dense H
(small lattices only) -- the plain definition.  All arithmetic complex128.
"""
from __future__ import annotations

import numpy as np

from oracle import dirac as od
from oracle import krylov as ok


def dense_h(op: od.Dirac) -> np.ndarray:
    """Dense H = gamma5 D_w (row/col = k * V + s)."""
    D = od.dense_dw(od.links_from_grid(op.U), op.dims, op.mass, op.mu, op.bc_t)
    return od.dense_g5(op.V) @ D


def low_modes(op: od.Dirac, K: int):
    """The K eigenpairs of H of smallest |lambda| (mu = 0), sorted by |lambda|.
    Returns (lam [K], vecs [K][12][V])."""
    if op.mu != 0.0:
        raise ValueError("low_modes: H is Hermitian only at mu = 0")
    H = dense_h(op)
    lam, Q = np.linalg.eigh(H)
    order = np.argsort(np.abs(lam), kind="stable")[:K]
    vecs = np.stack([Q[:, i].reshape(12, op.V) for i in order])
    return lam[order], vecs


def exact_sign(op: od.Dirac, b: np.ndarray) -> np.ndarray:
    """sign(H) b from the full dense eigendecomposition (the definition)."""
    H = dense_h(op)
    lam, Q = np.linalg.eigh(H)
    return (Q @ (np.sign(lam) * (Q.conj().T @ b.reshape(-1)))).reshape(b.shape)


def project(vecs: np.ndarray, b: np.ndarray):
    """(c, P b): c_k = <v_k, b>, P b = b - sum_k v_k c_k."""
    c = np.array([np.vdot(v, b) for v in vecs])
    pb = b.astype(complex).copy()
    for k, v in enumerate(vecs):
        pb -= c[k] * v
    return c, pb


def sign_apply_deflated(op: od.Dirac, a_scale, b, lam, vecs, sigmas, weights, l, tol, max_outer, pass_=1):
    """sign(H) b with the given low modes deflated (exact part plus the PFE
    of the projected source; BiCGstab(l) multi-shift solve)."""
    c, pb = project(vecs, b)
    y = ok.mshift_bicgstabl(lambda v: op.a_op(v, a_scale), pb, sigmas, weights, l, tol, max_outer, pass_)[0]
    out = np.sqrt(a_scale) * op.h(y)
    for k, v in enumerate(vecs):
        out += np.sign(lam[k]) * c[k] * v
    return out

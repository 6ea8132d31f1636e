"""Pins of the low-mode deflation oracle (mu = 0).

  * the dense H = gamma5 D_w is Hermitian at mu = 0 and the returned low modes
    are orthonormal eigenvectors with the smallest |lambda|, in order;
  * the dense H equals the matrix-free operator column by column (two
    independent statements of D_w);
  * deflating every mode leaves no PFE part: the result is the exact sign(H) b;
  * with K modes deflated the error against the exact sign(H) b obeys the
    PFE error bound over the deflated interval [a lambda_K^2, a lambda_max^2]
    and is smaller than without deflation.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import deflation as odf
from oracle import dirac as od
from oracle import pfe
from oracle import sign as osg


def mu0_op(dims, seed):
    U = wl.gauge_links(dims, 0.6, seed)
    return od.Dirac(U, dims, -2.0, 0.0, -1)


def test_low_modes_are_the_smallest_eigenpairs():
    op = mu0_op((2, 2, 2, 4), 91)
    H = odf.dense_h(op)
    assert np.abs(H - H.conj().T).max() <= 1e-13
    lam, vecs = odf.low_modes(op, 12)
    assert np.all(np.diff(np.abs(lam)) >= 0)
    allv = np.linalg.eigvalsh(H)
    assert np.allclose(np.sort(np.abs(allv))[:12], np.abs(lam), rtol=0, atol=1e-12)
    M = vecs.reshape(12, -1)
    assert np.abs(M.conj() @ M.T - np.eye(12)).max() <= 1e-12
    for k in range(12):
        r = op.h(vecs[k]) - lam[k] * vecs[k]
        assert np.linalg.norm(r) <= 1e-12


def test_dense_h_matches_operator():
    op = mu0_op((2, 2, 2, 4), 92)
    H = odf.dense_h(op)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((12, op.V)) + 1j * rng.standard_normal((12, op.V))
    assert np.linalg.norm(H @ v.reshape(-1) - op.h(v).reshape(-1)) <= 1e-12 * np.linalg.norm(v)


def test_full_deflation_is_exact():
    op = mu0_op((2, 2, 2, 4), 93)
    n = 12 * op.V
    lam, vecs = odf.low_modes(op, n)
    b = wl.gaussian_source(op.dims, 94)[0]
    sig, w = pfe.neuberger(6)
    out = odf.sign_apply_deflated(op, 0.05, b, lam, vecs, sig, w, 2, 1e-10, 100)
    ref = odf.exact_sign(op, b)
    assert np.linalg.norm(out - ref) <= 1e-11 * np.linalg.norm(ref)


def test_partial_deflation_within_pfe_bound():
    dims = (4, 4, 4, 4)
    op = mu0_op(dims, 95)
    H = odf.dense_h(op)
    ev = np.linalg.eigvalsh(H)
    lmax = np.abs(ev).max()
    a = 1.0 / (1.01 * lmax ** 2)
    b = wl.gaussian_source(dims, 96)[0]
    sig, w = pfe.neuberger(10)
    K = 16
    lam, vecs = odf.low_modes(op, K)
    ref = odf.exact_sign(op, b)
    # PFE error of sign over the spectrum the projected source sees
    x = np.linspace(a * lam[-1] ** 2, a * lmax ** 2, 20001)
    eps_k = np.max(np.abs(np.sqrt(x) * pfe.pfe_scalar(x, sig, w) - 1.0))
    x0 = np.linspace(a * np.abs(ev).min() ** 2, a * lmax ** 2, 20001)
    eps_0 = np.max(np.abs(np.sqrt(x0) * pfe.pfe_scalar(x0, sig, w) - 1.0))
    tol = 1e-11
    out = odf.sign_apply_deflated(op, a, b, lam, vecs, sig, w, 2, tol, 3000)
    _, pb = odf.project(vecs, b)
    err = np.linalg.norm(out - ref)
    assert err <= 1.01 * eps_k * np.linalg.norm(pb) + 1e-8 * np.linalg.norm(b)
    plain = osg.pfe_sign_apply(op, a, b, sig, w, 2, tol, 3000)[0]
    err0 = np.linalg.norm(plain - ref)
    assert err0 <= 1.01 * eps_0 * np.linalg.norm(b) + 1e-8 * np.linalg.norm(b)
    assert err < err0 and eps_k < eps_0
    # the error itself, from the dense eigendecomposition: the PFE sign
    # sqrt(a) lambda f(a lambda^2) replaces sign(lambda) on every mode of the
    # source the PFE sees (P b deflated, b plain); the low modes are exact
    lam_all, Q = np.linalg.eigh(H)
    pfe_sign = np.sqrt(a) * lam_all * pfe.pfe_scalar(a * lam_all ** 2, sig, w)
    dsign = pfe_sign - np.sign(lam_all)
    e_defl = Q @ (dsign * (Q.conj().T @ pb.reshape(-1)))
    e_plain = Q @ (dsign * (Q.conj().T @ b.reshape(-1)))
    assert np.linalg.norm((out - ref).reshape(-1) - e_defl) <= 1e-8 * np.linalg.norm(b)
    assert np.linalg.norm((plain - ref).reshape(-1) - e_plain) <= 1e-8 * np.linalg.norm(b)

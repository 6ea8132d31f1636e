"""Pins of the oracle's BiCGstab(l), multi-shift single-pass and double-pass.

What pins what:
  * BiCGstab(1) == van der Vorst's textbook BiCGstab, iterate by iterate;
  * the BiCG coefficients alpha_n, beta_n of BiCGstab(l) do not depend on l
    and equal those of plain dense BiCG (catches the rho0 <- -omega rho0
    bookkeeping, the sign of beta, the step order);
  * MR by normal equations == MR by modified Gram-Schmidt;
  * converged solutions == dense solves;
  * multi-shift collinearity b - (S + sigma') x^s == r_0 / (zeta psi) at every
    outer iteration (pins zeta, pi, psi, alpha^s, beta^s, c_k, kappa);
  * the sigma' = 0 shift reproduces the seed; each shift == a separate solve;
  * free-field plane waves give x_s = b / (A(p) + sigma_s) exactly;
  * double-pass y == single-pass y, with 2x the Mv and the same dot count
    (Section 3 cost table);
  * f(A) b against the dense inverse square root within the PFE error.
"""
import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle import dirac as od
from oracle import krylov as ok
from oracle import pfe
from oracle import sign as osg


def problem(dims, eps, mu, seed, bc=-1):
    U = wl.gauge_links(dims, eps, seed)
    op = od.Dirac(U, dims, -2.0, mu, bc)
    rho = od.spectral_radius(op, wl.start_vector(dims, seed + 1), 100)
    return U, op, od.a_scale_from_radius(rho)


def dense_A(U, dims, mu, a, bc=-1):
    V = wl.volume(dims)
    D = od.dense_dw(U, dims, -2.0, mu, bc)
    H = od.dense_g5(V) @ D
    return a * H @ H, H


# --------------------------------------------------------------------------
# seed BiCGstab(l)
# --------------------------------------------------------------------------

def test_bicgstab1_equals_textbook_bicgstab():
    dims = (2, 2, 2, 4)
    U, op, a = problem(dims, 0.6, 0.05, 31)
    S = op.seed_op(a, 0.02)
    b = wl.gaussian_source(dims, 32)[0]
    x1, info = ok.bicgstabl(S, b, 1, 1e-10, 200, keep_x=True)
    xs = ok.bicgstab_textbook(S, b, 1e-10, 200)
    n = min(len(xs), len(info.xs), 25)
    for k in range(n):
        assert np.linalg.norm(info.xs[k] - xs[k]) <= 1e-9 * np.linalg.norm(xs[k])


def test_bicg_coefficients_independent_of_l_and_equal_dense_bicg():
    dims = (2, 2, 2, 2)
    U, op, a = problem(dims, 0.6, 0.1, 41)
    sig0 = 0.05
    S = op.seed_op(a, sig0)
    b = wl.gaussian_source(dims, 42)[0]
    A, _ = dense_A(U, dims, 0.1, a)
    Sd = A + sig0 * np.eye(A.shape[0])
    al_ref, be_ref = ok.bicg_textbook(Sd, b.reshape(-1), 12)
    for l in (1, 2, 3, 4):
        _, info = ok.bicgstabl(S, b, l, 1e-30, 12 // l)
        al = np.array(info.alphas[:12])
        be = np.array(info.betas[:12])
        assert np.allclose(al, al_ref[:len(al)], rtol=1e-7)
        # BiCGstab direction update u = r - beta u  <->  BiCG p = r + beta p
        assert be[0] == 0
        assert np.allclose(be[1:], -be_ref[:len(be) - 1], rtol=1e-7)


@pytest.mark.parametrize("l", [2, 4])
def test_mr_normal_equations_equal_mgs(l):
    dims = (2, 2, 2, 4)
    U, op, a = problem(dims, 0.6, 0.05, 51)
    S = op.seed_op(a, 0.01)
    b = wl.gaussian_source(dims, 52)[0]
    _, i1 = ok.bicgstabl(S, b, l, 1e-10, 6, mr="normal", keep_x=True)
    _, i2 = ok.bicgstabl(S, b, l, 1e-10, 6, mr="mgs", keep_x=True)
    for x1, x2 in zip(i1.xs, i2.xs):
        assert np.linalg.norm(x1 - x2) <= 1e-9 * np.linalg.norm(x1)


@pytest.mark.parametrize("l", [1, 2, 4])
def test_bicgstabl_converges_to_dense_solve(l):
    dims = (2, 2, 2, 4)
    U, op, a = problem(dims, 0.6, 0.1, 61)
    sig0 = 0.003
    S = op.seed_op(a, sig0)
    b = wl.gaussian_source(dims, 62)[0]
    x, info = ok.bicgstabl(S, b, l, 1e-11, 2000)
    assert info.status == ok.OK
    A, _ = dense_A(U, dims, 0.1, a)
    Sd = A + sig0 * np.eye(A.shape[0])
    xd = np.linalg.solve(Sd, b.reshape(-1)).reshape(12, -1)
    true_res = np.linalg.norm(b - S(x)) / np.linalg.norm(b)
    assert true_res <= 1e-10
    smin = np.linalg.svd(Sd, compute_uv=False).min()
    assert np.linalg.norm(x - xd) <= 2 * true_res * np.linalg.norm(b) / smin


# --------------------------------------------------------------------------
# multi-shift single-pass
# --------------------------------------------------------------------------

def _collinearity_monitor(S, b, sp, store):
    def mon(m, r0, X, scal, active):
        for s in np.nonzero(active)[0]:
            res_true = b - S(X[s]) - sp[s] * X[s]
            res_col = r0 / (scal.zeta[s] * scal.psi[s])
            store.append(np.linalg.norm(res_true - res_col) / np.linalg.norm(b))
    return mon


@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_multishift_collinearity_every_outer_iteration(l):
    dims = (4, 4, 4, 8)
    U, op, a = problem(dims, 0.6, 0.05, 1001)
    sig, w = pfe.neuberger(10)
    b = wl.gaussian_source(dims, 2001)[0]
    sp = sig - sig.min()
    S = op.seed_op(a, sig.min())
    errs = []
    y, info, X = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, l, 1e-8, 400,
                                     1, monitor=_collinearity_monitor(S, b, sp, errs))
    assert info.status == ok.OK
    assert len(errs) > 20
    assert max(errs) <= 1e-9
    # every shift meets its tolerance in the true residual, too
    for s in range(len(sig)):
        rel = np.linalg.norm(b - S(X[s]) - sp[s] * X[s]) / np.linalg.norm(b)
        assert rel <= 1e-8 * 1.5


def test_seed_shift_reproduces_seed_iteration():
    dims = (4, 4, 4, 8)
    U, op, a = problem(dims, 0.6, 0.05, 1001)
    sig = np.array([0.01, 0.05, 0.3])
    w = np.ones(3)
    b = wl.gaussian_source(dims, 2001)[0]
    M = 6
    y, info, X = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, 2, 1e-30, M, 1)
    xs, sinfo = ok.bicgstabl(op.seed_op(a, 0.01), b, 2, 1e-30, M)
    assert np.linalg.norm(X[0] - xs) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("l", [2, 4])
def test_each_shift_equals_separate_solve(l):
    dims = (2, 2, 2, 4)
    U, op, a = problem(dims, 0.6, 0.1, 71)
    sig, w = pfe.neuberger(8)
    b = wl.gaussian_source(dims, 72)[0]
    tol = 1e-10
    y, info, X = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, l, tol, 3000, 1)
    assert info.status == ok.OK
    A, _ = dense_A(U, dims, 0.1, a)
    I = np.eye(A.shape[0])
    ysum = np.zeros(A.shape[0], dtype=complex)
    bound = 0.0
    for s in range(len(sig)):
        xd = np.linalg.solve(A + sig[s] * I, b.reshape(-1))
        ysum += w[s] * xd
        smin = np.linalg.svd(A + sig[s] * I, compute_uv=False).min()
        err = np.linalg.norm(X[s].reshape(-1) - xd)
        assert err <= 1.5 * tol * np.linalg.norm(b) / smin
        bound += w[s] * 1.5 * tol * np.linalg.norm(b) / smin
    assert np.linalg.norm(y.reshape(-1) - ysum) <= bound


def test_free_field_plane_wave_exact():
    dims = (4, 4, 4, 8)
    Lx, Ly, Lz, Lt = dims
    mu, m = 0.05, -2.0
    op = od.Dirac(wl.free_links(dims), dims, m, mu, -1)
    a = 1 / 36.5
    t, z, y_, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                              indexing="ij")
    n = (1, 2, 0, 3)
    p = [2 * np.pi * n[0] / Lx, 2 * np.pi * n[1] / Ly, 2 * np.pi * n[2] / Lz,
         np.pi * (2 * n[3] + 1) / Lt]
    q = np.array(p, dtype=complex)
    q[3] -= 1j * mu
    phase = np.exp(1j * (p[0] * x + p[1] * y_ + p[2] * z + p[3] * t)).reshape(-1)
    chi = np.arange(1, 13) * (1 + 0.5j)
    b = chi[:, None] * phase[None, :]
    lam = a * ((4 + m - np.sum(np.cos(q))) ** 2 + np.sum(np.sin(q) ** 2))
    sig, w = pfe.neuberger(10)
    for l in (1, 2):
        y, info, X = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, l, 1e-8, 50, 1)
        assert info.outer == 1
        for s in range(len(sig)):
            assert np.linalg.norm(X[s] - b / (lam + sig[s])) <= 1e-12 * np.linalg.norm(X[s])
        y2, info2 = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, l, 1e-8, 50, 2)
        assert np.linalg.norm(y2 - y) <= 1e-12 * np.linalg.norm(y)


# --------------------------------------------------------------------------
# double-pass
# --------------------------------------------------------------------------

@pytest.mark.parametrize("l", [1, 2, 4])
def test_double_pass_equals_single_pass(l):
    wk = wl.WORKLOADS["4x4x4x8"]
    U, op, a = problem(wk.dims, wk.eps, wk.mu, wk.gauge_seed)
    sig, w = pfe.neuberger(wk.n_shift)
    b = wk.sources()[0]
    amv = (lambda v: op.a_op(v, a))
    y1, i1, X = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 1000, 1)
    y2, i2 = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 1000, 2)
    assert i1.status == ok.OK and i2.status == ok.OK
    assert np.array_equal(i1.shift_iters, i2.shift_iters)
    # same iteration, sum reorganised: agreement to rounding (grows with l)
    assert np.linalg.norm(y2 - y1) <= 1e-11 * np.linalg.norm(y1)
    # Section 3 cost table (full outer iterations; the last one may end
    # early when the Krylov space is exhausted)
    M = i1.outer
    assert i1.mv == 2 * i1.steps and i2.mv == 4 * i2.steps
    assert i1.dots == i2.dots
    if i1.steps == M * l:
        assert i1.mv == 2 * M * l and i2.mv == 4 * M * l
        assert i1.dots == M * l * (0.5 * l + 3.5)


def test_cost_table_counts_forced_full_iterations():
    wk = wl.WORKLOADS["4x4x4x8"]
    U, op, a = problem(wk.dims, wk.eps, wk.mu, wk.gauge_seed)
    sig, w = pfe.neuberger(wk.n_shift)
    b = wk.sources()[0]
    amv = (lambda v: op.a_op(v, a))
    for l in (1, 2, 3):
        M = 7
        force = np.full(len(sig), M)
        _, i1, _ = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 100, 1, force_iters=force)
        _, i2 = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 100, 2, force_iters=force)
        assert i1.outer == i2.outer == M
        assert i1.mv == 2 * M * l and i2.mv == 4 * M * l
        assert i1.dots == i2.dots == M * l * (0.5 * l + 3.5)


def test_double_pass_with_frozen_shifts_and_unsorted_input():
    dims = (2, 2, 2, 4)
    U, op, a = problem(dims, 0.6, 0.1, 81)
    sig, w = pfe.neuberger(12)
    perm = np.random.default_rng(0).permutation(12)
    sig, w = sig[perm], w[perm]
    b = wl.gaussian_source(dims, 82)[0]
    amv = (lambda v: op.a_op(v, a))
    y1, i1, X = ok.mshift_bicgstabl(amv, b, sig, w, 3, 1e-9, 1000, 1)
    y2, i2 = ok.mshift_bicgstabl(amv, b, sig, w, 3, 1e-9, 1000, 2)
    assert len(set(i1.shift_iters.tolist())) > 2     # shifts freeze at different times
    assert np.linalg.norm(y2 - y1) <= 1e-12 * np.linalg.norm(y1)


def test_force_iters_hook_reproduces_run():
    dims = (2, 2, 2, 4)
    U, op, a = problem(dims, 0.6, 0.1, 81)
    sig, w = pfe.neuberger(6)
    b = wl.gaussian_source(dims, 82)[0]
    amv = (lambda v: op.a_op(v, a))
    y1, i1, _ = ok.mshift_bicgstabl(amv, b, sig, w, 2, 1e-9, 1000, 1)
    y2, i2, _ = ok.mshift_bicgstabl(amv, b, sig, w, 2, 1e-9, 1000, 1,
                                    force_iters=i1.shift_iters)
    y2b, _, _ = ok.mshift_bicgstabl(amv, b, sig, w, 2, 1e-9, 1000, 1,
                                    force_iters=i1.shift_iters)
    assert np.array_equal(y2, y2b)
    assert np.array_equal(i2.shift_iters, i1.shift_iters)
    # forced runs do full outer iterations (no early exhaustion exit)
    assert np.linalg.norm(y1 - y2) <= 1e-7 * np.linalg.norm(y1)
    forced = np.maximum(i1.shift_iters - 1, 1)
    y3, i3, _ = ok.mshift_bicgstabl(amv, b, sig, w, 2, 1e-9, 1000, 1, force_iters=forced)
    assert np.array_equal(i3.shift_iters, forced)


def test_not_converged_status():
    dims = (2, 2, 2, 4)
    U, op, a = problem(dims, 0.6, 0.1, 81)
    sig, w = pfe.neuberger(6)
    b = wl.gaussian_source(dims, 82)[0]
    y, info, _ = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, 2, 1e-9, 1, 1)
    assert info.status == ok.NOT_CONVERGED and info.outer == 1


# --------------------------------------------------------------------------
# f(A) b and sign(H)
# --------------------------------------------------------------------------

def _pfe_error_bound(evals, sig, w):
    return np.max(np.abs(pfe.pfe_scalar(evals, sig, w) - evals ** -0.5))


@pytest.mark.parametrize("mu", [0.0, 0.1])
def test_fAb_against_dense_inverse_sqrt(mu):
    dims = (2, 2, 2, 2)
    U, op, a = problem(dims, 0.6, mu, 91)
    A, H = dense_A(U, dims, mu, a)
    sig, w = pfe.neuberger(30)
    b = wl.gaussian_source(dims, 92)[0]
    y, info, _ = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, 2, 1e-12, 3000, 1)
    assert info.status == ok.OK
    lam, Vec = np.linalg.eig(A)
    exact = Vec @ (lam ** -0.5 * np.linalg.solve(Vec, b.reshape(-1)))
    cond = np.linalg.cond(Vec)
    pfe_err = _pfe_error_bound(lam, sig, w)
    # solver part: each shift to 1e-12 relative residual
    solve_err = sum(w[s] * 1e-12 * np.linalg.norm(b) /
                    np.linalg.svd(A + sig[s] * np.eye(len(A)), compute_uv=False).min()
                    for s in range(len(sig)))
    err = np.linalg.norm(y.reshape(-1) - exact)
    assert err <= 1.5 * (pfe_err * cond * np.linalg.norm(b) + solve_err)
    if mu == 0.0:
        assert cond < 1 + 1e-8      # A Hermitian: eigenvector basis unitary


def test_sign_squares_to_one():
    dims = (2, 2, 2, 2)
    U, op, a = problem(dims, 0.6, 0.05, 93)
    sig, w = pfe.neuberger(40)
    b = wl.gaussian_source(dims, 94)[0]
    s1, _ = osg.pfe_sign_apply(op, a, b, sig, w, 2, 1e-12, 3000)
    s2, _ = osg.pfe_sign_apply(op, a, s1, sig, w, 2, 1e-12, 3000)
    A, H = dense_A(U, dims, 0.05, a)
    lam = np.linalg.eigvals(A)
    tol = 10 * _pfe_error_bound(lam, sig, w) * np.linalg.cond(np.linalg.eig(A)[1]) + 1e-9
    assert np.linalg.norm(s2 - b) <= tol * np.linalg.norm(b)
    # overlap: D_ov b = b + g5 sign(H) b
    dov, _ = osg.pfe_sign_apply(op, a, b, sig, w, 2, 1e-12, 3000, overlap=True)
    assert np.allclose(dov, b + od.g5(s1), atol=1e-9)

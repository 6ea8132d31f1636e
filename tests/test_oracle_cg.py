"""Pins of the oracle's multi-shift CG (single, double and pseudo-double pass).

What pins what:
  * each shift's solution == a dense solve of (A + sigma_s) x = b, and y ==
    sum_s w_s of them (pins zeta, alpha^s, beta^s, the p^s recurrence and the
    freeze test);
  * forced freeze iterations: ||b - (A + sigma_s) x^s|| == ||r_{M_s}|| / |zeta^s|
    for every shift at every M_s (the collinear-residual invariant, which a
    wrong sign or index in the zeta recurrence breaks);
  * the sigma' = 0 shift == plain CG on the seed system, iterate for iterate
    (dense CG from numpy's solve-free definition of the Krylov minimiser:
    the A-norm error minimiser over K_k, computed by a dense least-squares);
  * double pass == pseudo-double pass == single pass, with 2N - 1, N and N Mv;
  * Wilson operator at mu = 0: y == the BiCGstab(l) oracle's y (an
    independent method) within the tolerance;
  * free-field plane wave: x_s = b / (A(p) + sigma_s) exactly after one step.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import cg as ocg
from oracle import dirac as od
from oracle import krylov as ok
from oracle import pfe


def hpd(n, seed, shift=0.05):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return M @ M.conj().T / n + shift * np.eye(n)


def test_shift_solutions_match_dense_solves():
    A = hpd(60, 1)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(60) + 1j * rng.standard_normal(60)
    sig, w = pfe.neuberger(8)
    y, info, xs = ocg.mshift_cg(lambda v: A @ v, b, sig, w, 1e-12, 500, 1, want_shifts=True)
    assert info.status == ocg.OK
    yref = np.zeros(60, complex)
    for s in range(len(sig)):
        xr = np.linalg.solve(A + sig[s] * np.eye(60), b)
        yref += w[s] * xr
        assert np.linalg.norm(xs[s] - xr) <= 1e-9 * np.linalg.norm(xr), s
        # the freeze test stopped the shift at its tolerance
        assert np.linalg.norm(b - (A + sig[s] * np.eye(60)) @ xs[s]) <= 5e-12 * np.linalg.norm(b)
    assert np.linalg.norm(y - yref) <= 1e-9 * np.linalg.norm(yref)
    # shifts with larger sigma converge no later than the seed
    assert info.shift_iters.max() == info.shift_iters[np.argmin(sig)]
    assert np.all(np.diff(info.shift_iters[np.argsort(sig)]) <= 0)


@pytest.mark.parametrize("M", [1, 3, 7, 15])
def test_collinear_residual_at_forced_freeze(M):
    A = hpd(40, 3)
    rng = np.random.default_rng(4)
    b = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    sig = np.array([0.3, 0.01, 1.5, 4.0, 0.05])
    w = np.ones(5)
    force = np.array([M, M + 2, max(M - 1, 1), M, M + 1])
    y, info, xs = ocg.mshift_cg(lambda v: A @ v, b, sig, w, 1e-30, 100, 1, force_iters=force, want_shifts=True)
    assert np.array_equal(info.shift_iters, force)
    for s in range(5):
        true = np.linalg.norm(b - (A + sig[s] * np.eye(40)) @ xs[s]) / np.linalg.norm(b)
        assert abs(true - info.shift_resid[s]) <= 1e-10 * max(true, 1e-3), (s, true, info.shift_resid[s])


def test_seed_shift_is_the_krylov_minimiser():
    """The sigma' = 0 shift after k steps minimises the S-norm error over
    K_k(S, b): computed here by a dense least-squares over an explicit
    orthonormal Krylov basis (no CG recurrence involved)."""
    A = hpd(30, 5)
    rng = np.random.default_rng(6)
    b = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    sig = np.array([0.2, 1.0])
    xstar = np.linalg.solve(A + 0.2 * np.eye(30), b)
    S = A + 0.2 * np.eye(30)
    L = np.linalg.cholesky(S)
    for k in (1, 2, 5, 9):
        K = np.stack([np.linalg.matrix_power(S, i) @ b for i in range(k)], axis=1)
        Q, _ = np.linalg.qr(K)
        # min_c || L^H (Q c - x*) ||_2
        c, *_ = np.linalg.lstsq(L.conj().T @ Q, L.conj().T @ xstar, rcond=None)
        xk = Q @ c
        _, _, xs = ocg.mshift_cg(lambda v: A @ v, b, sig, np.ones(2), 1e-30, 100, 1,
                                 force_iters=np.array([k, k]), want_shifts=True)
        assert np.linalg.norm(xs[0] - xk) <= 1e-8 * np.linalg.norm(xk), k


def test_three_passes_agree_with_cost_counts():
    A = hpd(80, 7)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(80) + 1j * rng.standard_normal(80)
    sig, w = pfe.neuberger(12)
    y1, i1 = ocg.mshift_cg(lambda v: A @ v, b, sig, w, 1e-10, 500, 1)
    y2, i2 = ocg.mshift_cg(lambda v: A @ v, b, sig, w, 1e-10, 500, 2)
    y3, i3 = ocg.mshift_cg(lambda v: A @ v, b, sig, w, 1e-10, 500, 3)
    N = i1.iters
    assert np.array_equal(i1.shift_iters, i2.shift_iters) and np.array_equal(i1.shift_iters, i3.shift_iters)
    assert N == i1.shift_iters.max()
    assert (i1.mv, i2.mv, i3.mv) == (N, 2 * N - 1, N)
    assert i1.dots == i2.dots == i3.dots == 2 * N
    assert np.linalg.norm(y2 - y1) <= 1e-12 * np.linalg.norm(y1)
    assert np.linalg.norm(y3 - y1) <= 1e-12 * np.linalg.norm(y1)


def test_wilson_mu0_matches_bicgstab_oracle():
    dims = (4, 4, 4, 4)
    U = wl.gauge_links(dims, 0.5, 41)
    op = od.Dirac(U, dims, -2.0, 0.0, -1)
    a = od.a_scale_from_radius(od.spectral_radius(op, wl.start_vector(dims, 42), 100))
    b = wl.gaussian_source(dims, 43)[0]
    sig, w = pfe.neuberger(10)
    y_cg, info = ocg.mshift_cg(lambda v: op.a_op(v, a), b, sig, w, 1e-11, 3000, 2)
    y_bi = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, 4, 1e-11, 3000, 1)[0]
    assert info.status == ocg.OK
    assert np.linalg.norm(y_cg - y_bi) <= 1e-8 * np.linalg.norm(y_bi)


def test_free_field_plane_wave_exact():
    dims = (4, 4, 4, 8)
    Lx, Ly, Lz, Lt = dims
    m = -2.0
    U = wl.free_links(dims)
    op = od.Dirac(U, dims, m, 0.0, -1)
    a = 1 / 36.5
    t, z, y_, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    p = np.array([2 * np.pi / Lx, 4 * np.pi / Ly, 0.0, np.pi * 7 / Lt])
    phase = np.exp(1j * (p[0] * x + p[1] * y_ + p[2] * z + p[3] * t)).reshape(-1)
    b = (np.arange(1, 13) * (1 + 0.5j))[:, None] * phase[None, :]
    lam = a * ((4 + m - np.sum(np.cos(p))) ** 2 + np.sum(np.sin(p) ** 2))
    sig, w = pfe.neuberger(6)
    for pass_ in (1, 2, 3):
        out = ocg.mshift_cg(lambda v: op.a_op(v, a), b, sig, w, 1e-10, 50, pass_, want_shifts=(pass_ == 1))
        y, info = out[0], out[1]
        assert info.iters == 1
        ref = sum(w[s] * b / (lam + sig[s]) for s in range(6))
        assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref), pass_

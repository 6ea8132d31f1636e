"""Pins of the oracle's breakdown branches of multi-shift BiCGstab(l)
(the paper does not discuss breakdown, Section 2; the readings are those of
the library's design notes: a gamma breakdown ends the BiCG part after a
u-step and the MR step runs over the completed steps; a Cholesky pivot below
1e-14 max diag truncates the MR polynomial; a shift whose zeta or |zeta psi|
leaves the representable range freezes as broken).

Each branch is driven by a constructed input (tests/breakdown_cases.py) and
checked against what the mathematics fixes, not against the oracle itself:
  * gamma breakdown: the MR coefficient equals the dense least-squares
    minimiser over the completed step, every shift stays collinear
    (b - (S + sigma') x^s = r_0 / (zeta psi)) after the partial iteration,
    and the double pass equals the single pass through the partial step;
  * Cholesky truncation: the 3 coefficients applied equal the dense
    least-squares minimiser over r_1..r_3, and every x_s equals the exact
    free-field plane-wave solution;
  * zeta breakdown: with <r~, (A + sigma_k) b> = 0, zeta_1 = 1 + alpha_0
    sigma'_k is exactly zero, so shift k stops before its first update
    (x_k = 0, broken) while every other shift equals its values in a run
    without shift k;
  * |zeta psi| overflow: the shift stops as converged, its x_s equals
    (A + sigma_s)^{-1} b (= b / sigma_s to rounding for sigma_s = 1e60), the
    other shifts are untouched, and the double pass equals the single pass.
"""
import numpy as np
import pytest

from oracle import krylov as ok
from oracle import dirac as od
from tests import breakdown_cases as bc


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def collinearity_monitor(op, a, b, sig, failures):
    sig0 = sig.min()

    def mon(m, r0, X, scal, active):
        for s in np.nonzero(active)[0]:
            res = b - op.a_op(X[s], a) - sig[s] * X[s]
            col = r0 / (scal.zeta[s] * scal.psi[s])
            failures.append(np.linalg.norm(res - col) / np.linalg.norm(b))
    return mon


@pytest.mark.parametrize("l", [2, 3])
def test_gamma_breakdown_at_step_one(l):
    wk, U, op, a, sig, w, b, rt = bc.gamma_case(1)
    amv = lambda v: op.a_op(v, a)
    # the constructed r~ makes <r~, S u_2> vanish to rounding in step 1
    tr, gaps = [], []
    y, info, X = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 50, 1, shadow=rt, trace=tr,
                                     monitor=collinearity_monitor(op, a, b, sig, gaps))
    steps = info.tape[0].steps
    assert info.status == ok.BREAKDOWN and info.outer == 1
    assert len(steps) == 2 and steps[0].alpha is not None and steps[1].alpha is None
    # MR over the one completed step: the least-squares minimiser of ||r_0 - g r_1||
    t0 = tr[0]
    assert t0["l_eff"] == 1 and len(t0["gammas"]) == 1
    r0, r1 = t0["r"][0].reshape(-1), t0["r"][1].reshape(-1)
    g_ls = np.vdot(r1, r0) / np.vdot(r1, r1)
    assert abs(t0["gammas"][0] - g_ls) <= 1e-12 * abs(g_ls)
    # every shift collinear with the seed after the partial iteration
    assert len(gaps) == len(sig) and max(gaps) <= 1e-12
    # the partial step survives the sweep and the replay
    y2, i2 = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 50, 2, shadow=rt)
    assert i2.status == ok.BREAKDOWN
    assert rel(y2, y) <= 1e-12
    assert i2.mv == 2 * info.mv


def test_gamma_breakdown_at_step_zero():
    wk, U, op, a, sig, w, b, rt = bc.gamma_case(0)
    amv = lambda v: op.a_op(v, a)
    y, info, X = ok.mshift_bicgstabl(amv, b, sig, w, 2, wk.tol, 50, 1, shadow=rt)
    steps = info.tape[0].steps
    assert info.status == ok.BREAKDOWN and info.outer == 1
    assert len(steps) == 1 and steps[0].alpha is None
    # no step completed: no shift moved from x_s = 0
    assert all(np.linalg.norm(x) == 0.0 for x in X) and np.linalg.norm(y) == 0.0
    y2, i2 = ok.mshift_bicgstabl(amv, b, sig, w, 2, wk.tol, 50, 2, shadow=rt)
    assert i2.status == ok.BREAKDOWN and np.linalg.norm(y2) == 0.0


def test_cholesky_truncation_solves_exactly():
    dims, mass, mu, U, a, sig, w, b, rt, waves, lams = bc.cholesky_case()
    op = od.Dirac(U, dims, mass, mu, -1)
    amv = lambda v: op.a_op(v, a)
    # the plane waves are eigenvectors of A with the closed-form eigenvalues
    for v, lam in zip(waves, lams):
        assert np.linalg.norm(amv(v) - lam * v) <= 1e-13 * np.linalg.norm(v)
    tr = []
    y, info, X = ok.mshift_bicgstabl(amv, b, sig, w, 4, 1e-8, 10, 1, shadow=rt, trace=tr)
    assert info.status == ok.OK and info.outer == 1
    assert np.all(info.shift_iters == 1)
    t0 = tr[0]
    assert t0["l_eff"] == 4 and len(t0["gammas"]) == 3          # truncated at the 4th pivot
    R = np.stack([v.reshape(-1) for v in t0["r"][1:4]], axis=1)
    g_ls = np.linalg.lstsq(R, t0["r"][0].reshape(-1), rcond=None)[0]
    assert np.max(np.abs(t0["gammas"] - g_ls)) <= 1e-6 * np.max(np.abs(g_ls))
    for s in range(len(sig)):
        exact = sum(v / (lam + sig[s]) for v, lam in zip(waves, lams))
        assert rel(X[s], exact) <= 1e-8, s
    y2, i2 = ok.mshift_bicgstabl(amv, b, sig, w, 4, 1e-8, 10, 2, shadow=rt)
    assert i2.status == ok.OK and rel(y2, y) <= 1e-12


@pytest.mark.parametrize("l", [1, 2, 4])
def test_zeta_breakdown_stops_one_shift(l):
    wk, U, op, a, sig, w, b, rt, k = bc.zeta_case()
    amv = lambda v: op.a_op(v, a)
    # the construction: zeta_1 = 1 + alpha_0 sigma'_k with alpha_0 = <r~, b> / <r~, S b>
    sp = sig[k] - sig.min()
    Sb = amv(b) + sig.min() * b
    assert abs(1 + sp * np.vdot(rt, b) / np.vdot(rt, Sb)) <= 1e-14
    y, info, X = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 200, 1, shadow=rt)
    assert info.status == ok.BREAKDOWN
    assert np.nonzero(info.shift_breakdown)[0].tolist() == [k]
    assert info.shift_iters[k] == 0 and np.linalg.norm(X[k]) == 0.0
    keep = [s for s in range(len(sig)) if s != k]
    y0, i0, X0 = ok.mshift_bicgstabl(amv, b, sig[keep], w[keep], l, wk.tol, 200, 1, shadow=rt)
    assert i0.status == ok.OK
    for j, s in enumerate(keep):
        assert np.array_equal(X[s], X0[j]) and info.shift_iters[s] == i0.shift_iters[j]
    y2, i2 = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 200, 2, shadow=rt)
    assert i2.status == ok.BREAKDOWN and rel(y2, y) <= 1e-12


@pytest.mark.parametrize("l", [1, 2, 3])
def test_overflowing_shift_stops_as_converged(l):
    wk, U, op, a, sig, w, b = bc.big_shift_case()
    amv = lambda v: op.a_op(v, a)
    force = np.full(len(sig), 3)
    y, info, X = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 3, 1, force_iters=force)
    assert info.status == ok.OK and not info.shift_breakdown.any()
    assert info.shift_iters[3] < 3 and np.all(info.shift_iters[:3] == 3)
    # (A + sigma)^{-1} b = b / sigma (1 - A / sigma + ...) = b / sigma to rounding
    assert rel(X[3], b / sig[3]) <= 1e-14
    # the other shifts are those of a run without the large shift
    y0, i0, X0 = ok.mshift_bicgstabl(amv, b, sig[:3], w[:3], l, wk.tol, 3, 1, force_iters=force[:3])
    for s in range(3):
        assert np.array_equal(X[s], X0[s])
    y2, i2 = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 3, 2, force_iters=force)
    assert i2.status == ok.OK and rel(y2, y) <= 1e-12
    # unforced, the same shift leaves in the first outer iteration (by its
    # residual estimate, or by the guard inside it for l = 3)
    yu, iu, Xu = ok.mshift_bicgstabl(amv, b, sig, w, l, wk.tol, 200, 1)
    assert iu.status == ok.OK and iu.shift_iters[3] <= 1 and not iu.shift_breakdown.any()
    assert rel(Xu[3], b / sig[3]) <= 1e-14

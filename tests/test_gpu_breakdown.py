"""GPU parity on the breakdown branches of multi-shift BiCGstab(l), with the
inputs of tests/breakdown_cases.py (built with the oracle's operator) and the
oracle's iteration as the reference: status, every shift's M_s, y and every
x_s, for the per-step and deferred single pass, the double and the
pseudo-double pass (explicit and basis form of the seed; the deferred single
pass in both forms too), and the persistent launch.

  * gamma breakdown in step 1 (l = 2, 3): the partial step, the completion
    of the direction updates it owes, the MR step over the completed step;
  * gamma breakdown in step 0: nothing completes, y = 0;
  * Cholesky truncation (free field, l = 4): the 3-term MR step solves the
    system exactly (compared with the plane-wave solution too);
  * zeta breakdown of one shift (l = 2, 4): that shift stops at x = 0, the
    rest converge;
  * |zeta psi| overflow of a 1e60 shift under forced iterations (l = 1..3):
    it stops early as converged at b / sigma.

Parity bound: 1e-10, or 30x the oracle's own change when its inputs are
perturbed by 1e-15 relative where the iteration amplifies rounding more than
that (bound_for).
"""
import numpy as np
import pytest

from oracle import dirac as od
from oracle import krylov as ok
from tests import breakdown_cases as bc
from tests.helpers import cuda, host, log

pytestmark = pytest.mark.gpu

FORMS = [("pass1", 1, 0), ("pass1-deferred", 1, "DEFERRED"), ("pass2", 2, 0), ("pass3", 3, 0),
         ("pass2-basis", 2, "SEED_BASIS"), ("pass3-basis", 3, "SEED_BASIS"),
         ("pass1-deferred-basis", 1, "DEFERRED|SEED_BASIS"),
         ("pass1-persistent", 1, "PERSISTENT"), ("pass2-persistent", 2, "PERSISTENT")]


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def oracle(op, a, b, sig, w, l, tol, max_outer, shadow=None, force=None):
    return ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, l, tol, max_outer, 1,
                               shadow=shadow, force_iters=force)


def bound_for(op, a, b, sig, w, l, tol, max_outer, y_ref, shadow=None, force=None):
    """1e-10, or 30x the largest change of the oracle's y over three
    perturbations of its inputs (b, and the shadow residual when given) by
    1e-15 relative -- the size of the GPU's own rounding differences -- where
    the iteration amplifies them more (the ill-conditioned MR step of the
    Cholesky case does)."""
    rng = np.random.default_rng(4321)
    worst = 0.0
    for _ in range(3):
        bp = b * (1 + 1e-15 * rng.standard_normal(b.shape))
        sp = None if shadow is None else shadow * (1 + 1e-15 * rng.standard_normal(shadow.shape))
        yp = oracle(op, a, bp, sig, w, l, tol, max_outer, sp, force)[0]
        worst = max(worst, rel(yp, y_ref))
    return max(1e-10, 30 * worst)


def compare_forms(ctx, a, b, sig, w, l, tol, max_outer, y0, i0, X0, bound, shadow=None, force=None):
    from paper_1010_2592_amd import msb
    allow = (msb.OK, msb.NOT_CONVERGED, msb.BREAKDOWN)
    for name, pass_, fl in FORMS:
        flags = sum(getattr(msb, f) for f in fl.split("|")) if fl else 0
        want = pass_ == 1
        y, info, xs = ctx.mshift_bicgstabl(cuda(b[None]), a, sig, w, l, tol, max_outer, pass_, flags=flags,
                                           want_shifts=want, allow=allow, force_iters=force,
                                           shadow=None if shadow is None else cuda(shadow[None]))
        e = rel(host(y)[0], y0)
        log(f"  {name}: status {info.status} (oracle {i0.status}), M {info.outer_iters}, y {e:.2e} "
            f"(bound {bound:.1e})")
        assert info.status == i0.status, name
        assert np.array_equal(info.shift_iters[0], i0.shift_iters), name
        assert e <= bound, name
        if want:
            xh = host(xs)[0]
            for s in range(len(sig)):
                assert rel(xh[s], X0[s]) <= bound, (name, s)


@pytest.mark.parametrize("l", [2, 3])
def test_gamma_breakdown_step_one(l):
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b, rt = bc.gamma_case(1)
    log(f"gamma breakdown in step 1, l={l}")
    y0, i0, X0 = oracle(op, a, b, sig, w, l, wk.tol, 50, shadow=rt)
    assert i0.status == ok.BREAKDOWN and i0.tape[0].steps[1].alpha is None
    bound = bound_for(op, a, b, sig, w, l, wk.tol, 50, y0, shadow=rt)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    compare_forms(ctx, a, b, sig, w, l, wk.tol, 50, y0, i0, X0, bound, shadow=rt)
    ctx.close()


def test_gamma_breakdown_step_zero():
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b, rt = bc.gamma_case(0)
    log("gamma breakdown in step 0, l=2")
    y0, i0, X0 = oracle(op, a, b, sig, w, 2, wk.tol, 50, shadow=rt)
    assert i0.status == ok.BREAKDOWN and np.linalg.norm(y0) == 0.0
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    compare_forms(ctx, a, b, sig, w, 2, wk.tol, 50, y0, i0, X0, 1e-10, shadow=rt)
    ctx.close()


def test_cholesky_truncation():
    from paper_1010_2592_amd import msb
    dims, mass, mu, U, a, sig, w, b, rt, waves, lams = bc.cholesky_case()
    op = od.Dirac(U, dims, mass, mu, -1)
    log("Cholesky truncation on the free field, l=4")
    y0, i0, X0 = oracle(op, a, b, sig, w, 4, 1e-8, 10, shadow=rt)
    assert i0.status == ok.OK and i0.outer == 1
    bound = bound_for(op, a, b, sig, w, 4, 1e-8, 10, y0, shadow=rt)
    ctx = msb.Context(msb.Lattice(dims, mass, mu, -1), cuda(U))
    compare_forms(ctx, a, b, sig, w, 4, 1e-8, 10, y0, i0, X0, bound, shadow=rt)
    # and the exact plane-wave solution
    y, info, xs = ctx.mshift_bicgstabl(cuda(b[None]), a, sig, w, 4, 1e-8, 10, 1, want_shifts=True,
                                       shadow=cuda(rt[None]))
    xh = host(xs)[0]
    for s in range(len(sig)):
        exact = sum(v / (lam + sig[s]) for v, lam in zip(waves, lams))
        assert rel(xh[s], exact) <= 1e-8, s
    ctx.close()


@pytest.mark.parametrize("l", [2, 4])
def test_zeta_breakdown_one_shift(l):
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b, rt, k = bc.zeta_case()
    log(f"zeta breakdown of shift {k}, l={l}")
    y0, i0, X0 = oracle(op, a, b, sig, w, l, wk.tol, 200, shadow=rt)
    assert i0.status == ok.BREAKDOWN and i0.shift_breakdown[k] and i0.shift_iters[k] == 0
    bound = bound_for(op, a, b, sig, w, l, wk.tol, 200, y0, shadow=rt)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    compare_forms(ctx, a, b, sig, w, l, wk.tol, 200, y0, i0, X0, bound, shadow=rt)
    ctx.close()


@pytest.mark.parametrize("l", [1, 2, 3])
def test_overflowing_shift(l):
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = bc.big_shift_case()
    force = np.full(len(sig), 3)
    log(f"shift 1e60 under 3 forced outer iterations, l={l}")
    y0, i0, X0 = oracle(op, a, b, sig, w, l, wk.tol, 3, force=force)
    assert i0.status == ok.OK and i0.shift_iters[3] < 3
    bound = bound_for(op, a, b, sig, w, l, wk.tol, 3, y0, force=force)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    compare_forms(ctx, a, b, sig, w, l, wk.tol, 3, y0, i0, X0, bound, force=force)
    ctx.close()

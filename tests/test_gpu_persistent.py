"""The persistent (one cooperative launch per pass) solve.

It runs the same stage bodies with the same partial-block counts as the
launch-per-stage path, so results are required to be bitwise identical to
that path (which the solver tests pin to the oracle), and on the small
lattice also to the oracle directly at 1e-10.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import dirac as od
from oracle import krylov as ok
from oracle import pfe
from tests.helpers import A_SCALE_BOUND, cuda, host, log, problem, rel
from tests.test_gpu_solver import parity_bound

pytestmark = pytest.mark.gpu


def ctx_for(wk, U):
    from paper_1010_2592_amd import msb
    return msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))


def shift_sets(sig, w, nrhs):
    """rhs 1 gets a 6-pole set padded with zero-weight copies; the rest the given set."""
    s2, w2 = pfe.neuberger(6)
    S = np.tile(sig, (nrhs, 1))
    W = np.tile(w, (nrhs, 1))
    if nrhs > 1:
        S[1, :6], W[1, :6] = s2, w2
        S[1, 6:], W[1, 6:] = s2[-1] * 2, 0.0
    return S, W


def same(a, b):
    return np.array_equal(host(a), host(b))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("pass_", [1, 2])
def test_persistent_bitwise_equals_launch_path(precision, pass_):
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    bb = wl.gaussian_source(wk.dims, 91, 3)
    S, W = shift_sets(sig, w, 3)
    flags = msb.MIXED if precision == "mixed" else 0
    log(f"persistent vs launch path: 8^4, 3 rhs, {precision}, pass {pass_}")
    ctx = ctx_for(wk, U)
    y0, i0, x0 = ctx.mshift_bicgstabl(cuda(bb), a, S, W, 4, wk.tol, 2000, pass_, flags=flags,
                                      want_shifts=(pass_ == 1))
    y1, i1, x1 = ctx.mshift_bicgstabl(cuda(bb), a, S, W, 4, wk.tol, 2000, pass_, flags=flags | msb.PERSISTENT,
                                      want_shifts=(pass_ == 1))
    assert same(y0, y1)
    if pass_ == 1:
        assert same(x0, x1)
    assert np.array_equal(i0.shift_iters, i1.shift_iters)
    assert (i0.outer_iters, i0.mv_count, i0.dot_count, i0.reliable_updates) == \
        (i1.outer_iters, i1.mv_count, i1.dot_count, i1.reliable_updates)
    # the per-stage path applies u_0..u_{j-1} of each BiCG step inside the
    # r-update (same arithmetic, one pass fewer over them): fewer bytes
    assert 0.8 * i1.bytes_model < i0.bytes_model < i1.bytes_model


@pytest.mark.parametrize("l", [1, 2, 3, 4, 5, 6])
def test_persistent_every_l_matches_oracle(l):
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    force = np.full(len(sig), 3)
    ref = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b[0], sig, w, l, wk.tol, 3, 1, force_iters=force)[0]
    bound = parity_bound(op, a, b[0], sig, w, l, wk.tol, force, ref)
    ctx = ctx_for(wk, U)
    allow = (msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY)
    for pass_ in (1, 2):
        y0 = ctx.mshift_bicgstabl(cuda(b), a, sig, w, l, wk.tol, 3, pass_, force_iters=force, allow=allow)[0]
        y1 = ctx.mshift_bicgstabl(cuda(b), a, sig, w, l, wk.tol, 3, pass_, flags=msb.PERSISTENT,
                                  force_iters=force, allow=allow)[0]
        assert same(y0, y1), (l, pass_)
        log(f"  persistent l={l} pass {pass_}: y vs oracle {rel(host(y1)[0], ref):.2e} (bound {bound:.1e})")
        assert rel(host(y1)[0], ref) <= bound, (l, pass_)


def test_persistent_twelve_point_sources_production_lattice():
    """16^3x32, the 12 point sources in one launch, N_s = 30, l = 4, two forced
    outer iterations, FP64 and mixed, both passes: bitwise equal to the
    launch-per-stage path."""
    from paper_1010_2592_amd import msb
    wk = wl.WORKLOADS["16x16x16x32"]
    log("16x16x16x32, 12 point sources, persistent")
    U = wk.links()
    b = wl.point_sources(wk.dims)
    sig, w = pfe.neuberger(wk.n_shift)
    a = A_SCALE_BOUND
    force = np.full(len(sig), 2)
    ctx = ctx_for(wk, U)
    allow = (msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY)
    for flags in (0, msb.MIXED):
        for pass_ in (1, 2):
            y0 = ctx.mshift_bicgstabl(cuda(b), a, sig, w, 4, wk.tol, 2, pass_, flags=flags, force_iters=force,
                                      allow=allow)[0]
            y1 = ctx.mshift_bicgstabl(cuda(b), a, sig, w, 4, wk.tol, 2, pass_, flags=flags | msb.PERSISTENT,
                                      force_iters=force, allow=allow)[0]
            assert same(y0, y1), (flags, pass_)


def test_persistent_sign_apply_and_l_bound():
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    ctx = ctx_for(wk, U)
    s0 = ctx.pfe_sign_apply(cuda(b), a, sig, w, 2, wk.tol, 2000, 2)[0]
    s1 = ctx.pfe_sign_apply(cuda(b), a, sig, w, 2, wk.tol, 2000, 2, flags=msb.PERSISTENT)[0]
    assert same(s0, s1)
    with pytest.raises(msb.MsbError) as e:
        ctx.mshift_bicgstabl(cuda(b), a, sig, w, 7, wk.tol, 10, 1, flags=msb.PERSISTENT)
    assert e.value.status == msb.ERR_ARG


def test_persistent_timing_hook_reports_stage_classes():
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    ctx = ctx_for(wk, U)
    ctx.profile_enable(True)
    _, info, _ = ctx.mshift_bicgstabl(cuda(b), a, sig, w, 4, wk.tol, 2000, 2, flags=msb.PERSISTENT)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    st = prof["stencil"]
    log(f"  persistent stencil stages: {st['count']} in {st['ms']:.3f} ms, {st['bytes'] / 1e9:.3f} GB")
    # 4 stencil stages per BiCG step, l = 4 steps per outer iteration, in the
    # first pass and again in the replay
    assert st["count"] == 2 * 4 * 4 * info.outer_iters
    assert st["ms"] > 0 and st["bytes"] > 0


def test_persistent_mixed_refined_meets_tolerance():
    """Complex64 compute with FP64 reductions, the single pass in one
    cooperative launch, then FP64 correction solves for the shifts whose
    FP64 residual the FP32 vectors left above tol: the main solve is
    bitwise the per-stage one, and every shift of every source ends at a
    true residual <= tol (recomputed here with the oracle's operator)."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    bb = wl.gaussian_source(wk.dims, 97, 3)
    ctx = ctx_for(wk, U)
    flags = msb.MIXED | msb.REFINE
    y0, i0, x0 = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, wk.tol, 3000, 1, flags=flags, want_shifts=True)
    y1, i1, x1 = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, wk.tol, 3000, 1, flags=flags | msb.PERSISTENT,
                                      want_shifts=True)
    assert i1.status == msb.OK and i1.refined_shifts > 0
    assert same(y0, y1) and same(x0, x1)
    xs = host(x1)
    worst = 0.0
    for r in range(3):
        nb = np.linalg.norm(bb[r])
        for s in range(len(sig)):
            worst = max(worst, np.linalg.norm(bb[r] - op.a_op(xs[r, s], a) - sig[s] * xs[r, s]) / nb)
    log(f"  persistent mixed + refine: worst true residual {worst:.2e}, refined {i1.refined_shifts}")
    assert worst <= wk.tol


def test_timing_hook_class_mask():
    """msb_profile_classes: with the stencil class alone selected, only the
    stencil launches are recorded (4 per BiCG step: two Mv of two stencils),
    every other class stays empty; the default records them all; a stride
    records every stride-th selected launch."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    ctx = ctx_for(wk, U)
    ctx.profile_enable(True, classes=("stencil",))
    _, info, _ = ctx.mshift_bicgstabl(cuda(b), a, sig, w, 4, wk.tol, 2000, 3)
    prof = ctx.profile_read()
    assert prof["stencil"]["count"] == 4 * 4 * info.outer_iters
    assert all(v["count"] == 0 for k, v in prof.items() if k != "stencil")
    ctx.profile_enable(True)
    ctx.mshift_bicgstabl(cuda(b), a, sig, w, 4, wk.tol, 2000, 3)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    assert prof["stencil"]["count"] == 4 * 4 * info.outer_iters
    assert prof["seed_vector"]["count"] > 0 and prof["scalar"]["count"] > 0
    # every third stencil launch: the first, the fourth, ...
    ctx.profile_enable(True, classes=("stencil",), stride=3)
    ctx.mshift_bicgstabl(cuda(b), a, sig, w, 4, wk.tol, 2000, 3)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    assert prof["stencil"]["count"] == (4 * 4 * info.outer_iters + 2) // 3
    assert prof["stencil"]["ms"] > 0
    with pytest.raises(msb.MsbError) as e:
        ctx.profile_enable(True, stride=0)
    assert e.value.status == msb.ERR_ARG

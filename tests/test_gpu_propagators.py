"""Multi-mass Wilson propagators (MSB_OP_WILSON: A = a D_w(mu), one stencil
per Mv).  D_w(m + sigma) = D_w(m) + sigma, so the multi-shift solver with
a = 1 and sigma_s = m_s - m returns x_s = D_w(m_s)^{-1} b for every mass.
Checked against the oracle's iteration (forced freeze points), by every
propagator's true residual, across forms and launch modes.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import dirac as od
from oracle import krylov as ok
from tests.helpers import cuda, host, log, rel

pytestmark = pytest.mark.gpu

MASSES = np.array([0.1, 0.15, 0.25, 0.5, 1.0])


def setup(dims, seed, mu):
    from paper_1010_2592_amd import msb
    U = wl.gauge_links(dims, 0.6, seed)
    m0 = float(MASSES.min())
    op = od.Dirac(U, dims, m0, mu, -1)
    ctx = msb.Context(msb.Lattice(dims, m0, mu, -1), cuda(U))
    return U, op, ctx, MASSES - m0


@pytest.mark.parametrize("form", ["pass1", "deferred", "pass2", "pass3", "pass2-basis", "pass3-basis",
                                  "persistent1", "persistent2"])
def test_forced_matches_oracle(form):
    from paper_1010_2592_amd import msb
    dims = (4, 4, 4, 8)
    U, op, ctx, sig = setup(dims, 73, 0.05)
    b = wl.gaussian_source(dims, 74)[0]
    w = np.array([1.0, 0.5, 0.25, 2.0, 1.5])
    y1, i1, X1 = ok.mshift_bicgstabl(op.dw, b, sig, w, 2, 1e-10, 500, 1)
    y2 = ok.mshift_bicgstabl(op.dw, b, sig, w, 2, 1e-10, 500, 2, force_iters=i1.shift_iters)[0]
    pass_ = {"pass1": 1, "deferred": 1, "pass2": 2, "pass3": 3, "pass2-basis": 2, "pass3-basis": 3,
             "persistent1": 1, "persistent2": 2}[form]
    flags = msb.OP_WILSON | (msb.DEFERRED if form == "deferred" else 0) | \
        (msb.PERSISTENT if form.startswith("persistent") else 0) | \
        (msb.SEED_BASIS if form.endswith("basis") else 0)
    y, info, xs = ctx.mshift_bicgstabl(cuda(b[None]), 1.0, sig, w, 2, 1e-10, 500, pass_, flags=flags,
                                       want_shifts=(pass_ == 1), force_iters=i1.shift_iters)
    ref = y1 if pass_ == 1 else y2
    log(f"propagators {form}: rel err {rel(host(y)[0], ref):.2e}, M {info.outer_iters}")
    assert np.array_equal(info.shift_iters[0], i1.shift_iters)
    assert rel(host(y)[0], ref) <= 1e-10
    if pass_ == 1:
        xs = host(xs)[0]
        for s in range(len(sig)):
            assert rel(xs[s], X1[s]) <= 1e-10, s
    # one stencil per Mv: the cost table's 2 M l Mv (single pass)
    if pass_ != 2:
        assert info.mv_count == 2 * info.outer_iters * 2


@pytest.mark.parametrize("mixed", [False, True])
def test_point_source_propagators_true_residuals(mixed):
    """The 12 spin-colour point sources (chunked stencil), five masses, at
    mu = 0.05: every propagator's true residual ||b - D_w(m_s) x_s|| / ||b||
    meets the tolerance (FP64 single pass deferred; mixed with refinement)."""
    import torch
    from paper_1010_2592_amd import msb
    dims = (8, 8, 8, 8)
    U, op, ctx, sig = setup(dims, 75, 0.05)
    b = cuda(wl.point_sources(dims))
    tol = 1e-9
    flags = msb.OP_WILSON | (msb.MIXED | msb.REFINE if mixed else msb.DEFERRED)
    # point sources need a shadow residual other than b under D_w (parity)
    with pytest.raises(msb.MsbError) as e:
        ctx.mshift_bicgstabl(b, 1.0, sig, np.ones(len(sig)), 4, tol, 1000, 1, flags=msb.OP_WILSON)
    assert e.value.status == msb.BREAKDOWN
    shadow = cuda(np.repeat(wl.gaussian_source(dims, 80), 12, axis=0))
    y, info, xs = ctx.mshift_bicgstabl(b, 1.0, sig, np.ones(len(sig)), 4, tol, 1000, 1, flags=flags,
                                       want_shifts=True, shadow=shadow)
    worst = 0.0
    for s in range(len(sig)):
        xsv = xs[:, s].contiguous()
        dx = ctx.wilson_apply(xsv, 0)
        r = b - dx - sig[s] * xsv
        rr = torch.linalg.vector_norm(r.reshape(12, -1), dim=1) / torch.linalg.vector_norm(b.reshape(12, -1), dim=1)
        worst = max(worst, float(rr.max()))
    log(f"point-source propagators ({'mixed+refine' if mixed else 'fp64 deferred'}): M {info.outer_iters}, "
        f"worst true residual {worst:.2e}")
    assert info.status == 0
    assert worst <= tol
    # against the oracle's multi-shift solve of source 0 with the same r~
    x0 = ok.mshift_bicgstabl(op.dw, wl.point_sources(dims)[0], sig, np.ones(len(sig)), 4, 1e-11, 1000, 1,
                             shadow=wl.gaussian_source(dims, 80)[0])[2]
    for s in range(len(sig)):
        assert rel(host(xs)[0, s], x0[s]) <= 50 * tol, s


def test_op_wilson_flag_rejections():
    from paper_1010_2592_amd import msb
    dims = (4, 4, 4, 8)
    U, op, ctx, sig = setup(dims, 76, 0.05)
    b = cuda(wl.gaussian_source(dims, 77))
    w = np.ones(len(sig))
    with pytest.raises(msb.MsbError) as e:
        ctx.mshift_bicgstabl(b, 1.0, sig, w, 2, 1e-8, 10, 1, flags=msb.OP_WILSON | msb.ADJOINT)
    assert e.value.status == msb.ERR_ARG
    with pytest.raises(msb.MsbError) as e:
        ctx.pfe_sign_apply(b, 1.0, sig, w, 2, 1e-8, 10, 1, flags=msb.OP_WILSON)
    assert e.value.status == msb.ERR_ARG


def test_shadow_residual_forced_matches_oracle():
    """A Gaussian shadow residual: the GPU iteration is the oracle's with the
    same r~ (forced freeze points), single and double pass."""
    from paper_1010_2592_amd import msb
    dims = (4, 4, 4, 8)
    U, op, ctx, sig = setup(dims, 81, 0.05)
    b = wl.point_sources(dims)[3]
    r_t = wl.gaussian_source(dims, 82)[0]
    w = np.array([1.0, 0.5, 0.25, 2.0, 1.5])
    y1, i1, X1 = ok.mshift_bicgstabl(op.dw, b, sig, w, 2, 1e-10, 500, 1, shadow=r_t)
    y2 = ok.mshift_bicgstabl(op.dw, b, sig, w, 2, 1e-10, 500, 2, force_iters=i1.shift_iters, shadow=r_t)[0]
    for pass_, ref in ((1, y1), (2, y2), (3, y2)):
        y, info, _ = ctx.mshift_bicgstabl(cuda(b[None]), 1.0, sig, w, 2, 1e-10, 500, pass_, flags=msb.OP_WILSON,
                                          force_iters=i1.shift_iters, shadow=cuda(r_t[None]))
        log(f"shadow r~ pass {pass_}: rel err {rel(host(y)[0], ref):.2e}")
        assert rel(host(y)[0], ref) <= 1e-10, pass_

"""The pseudo-double pass (pass = 3; Section 2, the second option after
Eq. 2.2): the coefficients come from the same transposed sweep as in the
double pass, but the Mv outputs of the first pass are kept in device memory
and summed afterwards instead of being regenerated.  y is the same sum as the
double pass's, so the oracle's double pass is its reference; the Mv count is
the single pass's (Table 1: 2 M l).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import pfe
from tests.helpers import cuda, host, log, problem, rel
from tests.test_gpu_solver import ctx_for, oracle_run, parity_bound

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("l", [1, 2, 4])
def test_pseudo_forced_matches_oracle_double_pass(l):
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    log(f"pseudo-double pass forced 4x4x4x8 l={l}")
    y1, i1, _ = oracle_run(op, a, b[0], sig, w, l, wk.tol, 2000, 1)
    y2, i2 = oracle_run(op, a, b[0], sig, w, l, wk.tol, 2000, 2, force=i1.shift_iters)
    ctx = ctx_for(wk, U)
    y, info, _ = ctx.mshift_bicgstabl(cuda(b), a, sig, w, l, wk.tol, 2000, 3, force_iters=i1.shift_iters)
    bound = parity_bound(op, a, b[0], sig, w, l, wk.tol, i1.shift_iters, y1)
    log(f"  bound {bound:.2e}, rel err {rel(host(y)[0], y2):.2e}, M {info.outer_iters}")
    assert rel(host(y)[0], y2) <= bound
    assert np.array_equal(info.shift_iters[0], i1.shift_iters)
    y_dp, info_dp, _ = ctx.mshift_bicgstabl(cuda(b), a, sig, w, l, wk.tol, 2000, 2, force_iters=i1.shift_iters)
    assert rel(host(y), host(y_dp)) <= 1e-12
    # Table 1: the single pass's Mv count, the same inner products
    assert info.mv_count == info_dp.mv_count // 2 == 2 * info.outer_iters * l
    assert info.dot_count == info_dp.dot_count


@pytest.mark.parametrize("l", [1, 2])
def test_pseudo_batch_with_shift_sets_crosses_storage_chunks(l):
    """Six right-hand sides (chunked stencil), rhs 1 with a padded 6-pole
    set, enough outer iterations that the stored vectors span several
    storage chunks; the right-hand sides stop at different iterations."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    bb = wl.gaussian_source(wk.dims, 95, 6)
    s2, w2 = pfe.neuberger(6)
    S = np.tile(sig, (6, 1))
    W = np.tile(w, (6, 1))
    S[1, :6], W[1, :6] = s2, w2
    S[1, 6:], W[1, 6:] = s2[-1] * 2, 0.0
    ctx = ctx_for(wk, U)
    y2, i2, _ = ctx.mshift_bicgstabl(cuda(bb), a, S, W, l, wk.tol, 3000, 2)
    y3, i3, _ = ctx.mshift_bicgstabl(cuda(bb), a, S, W, l, wk.tol, 3000, 3)
    y1, i1, _ = ctx.mshift_bicgstabl(cuda(bb), a, S, W, l, wk.tol, 3000, 1)
    log(f"  l={l}: M {i3.outer_iters}; pseudo vs double {rel(host(y3), host(y2)):.2e}, "
        f"vs single {rel(host(y3), host(y1)):.2e}")
    assert i3.outer_iters > 16
    assert np.array_equal(i3.shift_iters, i2.shift_iters)
    assert i3.mv_count == i1.mv_count
    assert rel(host(y3), host(y2)) <= 1e-12
    assert rel(host(y3), host(y1)) <= 1e-10
    for r in range(6):
        assert rel(host(y3)[r], host(y2)[r]) <= 1e-12, r


def test_pseudo_mixed():
    """Mixed precision: FP32 vectors are stored, the FP64 reliable-update
    vectors beside them; y agrees with the FP64 solve at the mixed level."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    bb = wl.gaussian_source(wk.dims, 96, 3)
    ctx = ctx_for(wk, U)
    y64, i64, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 2, wk.tol, 3000, 1)
    y2, i2, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 2, wk.tol, 3000, 2, flags=msb.MIXED)
    y3, i3, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 2, wk.tol, 3000, 3, flags=msb.MIXED)
    d64, d2 = rel(host(y3), host(y64)), rel(host(y3), host(y2))
    log(f"  mixed pseudo: M {i3.outer_iters}, reliable {i3.reliable_updates}, vs FP64 {d64:.2e}, "
        f"vs mixed double {d2:.2e}")
    assert i3.reliable_updates > 0
    assert i3.outer_iters > 8
    assert d64 <= 1e-6
    assert np.max(np.abs(i3.shift_iters - i2.shift_iters)) <= 4


def test_pseudo_free_field_exhaustion():
    """A plane wave on the free field: exhaustion inside the first outer
    iteration; y = sum_s w_s b / (A(p) + sigma_s) exactly."""
    from paper_1010_2592_amd import msb
    dims = (4, 4, 4, 8)
    Lx, Ly, Lz, Lt = dims
    mu, m = 0.05, -2.0
    U = wl.free_links(dims)
    a = 1 / 36.5
    t, z, y_, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    p = [2 * np.pi / Lx, 4 * np.pi / Ly, 0.0, np.pi * 7 / Lt]
    q = np.array(p, dtype=complex)
    q[3] -= 1j * mu
    phase = np.exp(1j * (p[0] * x + p[1] * y_ + p[2] * z + p[3] * t)).reshape(-1)
    b = (np.arange(1, 13) * (1 + 0.5j))[:, None] * phase[None, :]
    lam = a * ((4 + m - np.sum(np.cos(q))) ** 2 + np.sum(np.sin(q) ** 2))
    sig, w = pfe.neuberger(10)
    ctx = msb.Context(msb.Lattice(dims, m, mu, -1), cuda(U))
    ref = sum(w[s] * b / (lam + sig[s]) for s in range(10))
    for l in (1, 2, 4):
        y, info, _ = ctx.mshift_bicgstabl(cuda(b[None]), a, sig, w, l, 1e-8, 50, 3)
        assert info.status == 0 and info.outer_iters == 1
        assert rel(host(y)[0], ref) <= 1e-12, l


def test_pseudo_sign_apply_matches_single_pass():
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    ctx = ctx_for(wk, U)
    o1, _ = ctx.pfe_sign_apply(cuda(b), a, sig, w, 2, wk.tol, 2000, 1, flags=msb.OVERLAP)
    o3, i3 = ctx.pfe_sign_apply(cuda(b), a, sig, w, 2, wk.tol, 2000, 3, flags=msb.OVERLAP)
    log(f"  overlap pseudo vs single {rel(host(o3), host(o1)):.2e}")
    assert rel(host(o3), host(o1)) <= 1e-10


def test_pseudo_flag_restrictions():
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    ctx = ctx_for(wk, U)
    for flags in (msb.PERSISTENT, msb.DEFERRED, msb.REFINE):
        with pytest.raises(msb.MsbError) as e:
            ctx.mshift_bicgstabl(cuda(b), a, sig, w, 2, wk.tol, 10, 3, flags=flags)
        assert e.value.status == msb.ERR_ARG
    with pytest.raises(msb.MsbError) as e:
        ctx.mshift_bicgstabl(cuda(b), a, sig, w, 2, wk.tol, 10, 3, want_shifts=True)
    assert e.value.status == msb.ERR_ARG
    with pytest.raises(msb.MsbError) as e:
        ctx.mshift_bicgstabl(cuda(b), a, sig, w, 2, wk.tol, 10, 4)
    assert e.value.status == msb.ERR_ARG

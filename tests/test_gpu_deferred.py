"""The deferred single pass (MSB_DEFERRED): each shift's vectors are updated
once per outer iteration from the iteration's 2l+2 seed basis vectors, with
coefficients from replaying the step recurrences on the device.  Same
arithmetic as the per-step single pass up to rounding order: the oracle's
iteration (forced freeze iterations) is matched at the parity bound of the
per-step form, and unforced runs take the same iteration path (the freeze
test reads seed scalars only) with y equal to rounding.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import krylov as ok
from oracle import pfe
from tests.helpers import cuda, host, log, problem, rel
from tests.test_gpu_solver import ctx_for, oracle_run, parity_bound

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("basis", [False, True])
@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_deferred_forced_matches_oracle(l, basis):
    """Also with the seed in basis form (MSB_SEED_BASIS): its BiCG steps
    write only the two vectors each Mv reads."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    log(f"deferred forced 4x4x4x8 l={l}{' seed basis' if basis else ''}")
    y0, i0, X0 = oracle_run(op, a, b[0], sig, w, l, wk.tol, 2000, 1)
    ctx = ctx_for(wk, U)
    flags = msb.DEFERRED | (msb.SEED_BASIS if basis else 0)
    y, info, xs = ctx.mshift_bicgstabl(cuda(b), a, sig, w, l, wk.tol, 2000, 1, flags=flags,
                                       want_shifts=True, force_iters=i0.shift_iters)
    assert np.array_equal(info.shift_iters[0], i0.shift_iters)
    bound = parity_bound(op, a, b[0], sig, w, l, wk.tol, i0.shift_iters, y0)
    log(f"  bound {bound:.2e}, rel err {rel(host(y)[0], y0):.2e}")
    assert rel(host(y)[0], y0) <= bound
    xs = host(xs)[0]
    for s in range(len(sig)):
        assert rel(xs[s], X0[s]) <= bound, s


@pytest.mark.parametrize("flags_extra", ["fp64", "mixed", "fp64-basis"])
def test_deferred_batch_with_shift_sets_matches_per_step(flags_extra):
    """Six right-hand sides (chunked stencil), rhs 1 with a padded 6-pole set.
    FP64: the same M_s as the per-step form and y equal to rounding.  Mixed:
    the Mv epilogue that also writes the basis copy is a separate kernel
    instance whose FP32 rounding (multiply-add contraction) may differ in the
    last bit, which in FP32 moves the seed's convergence by an iteration or
    two; M_s then agree within 4 and y within the mixed-precision level."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    bb = wl.gaussian_source(wk.dims, 93, 6)
    s2, w2 = pfe.neuberger(6)
    S = np.tile(sig, (6, 1))
    W = np.tile(w, (6, 1))
    S[1, :6], W[1, :6] = s2, w2
    S[1, 6:], W[1, 6:] = s2[-1] * 2, 0.0
    extra = msb.MIXED if flags_extra == "mixed" else 0
    basis = msb.SEED_BASIS if flags_extra == "fp64-basis" else 0
    ctx = ctx_for(wk, U)
    y0, i0, x0 = ctx.mshift_bicgstabl(cuda(bb), a, S, W, 4, wk.tol, 3000, 1, flags=extra, want_shifts=True)
    y1, i1, x1 = ctx.mshift_bicgstabl(cuda(bb), a, S, W, 4, wk.tol, 3000, 1,
                                      flags=extra | msb.DEFERRED | basis, want_shifts=True)
    d = rel(host(y1), host(y0))
    dx = max(rel(host(x1)[r, s], host(x0)[r, s]) for r in range(6) for s in range(len(sig)))
    log(f"  {flags_extra}: deferred vs per-step y {d:.2e}, worst x_s {dx:.2e}, M {i1.outer_iters}")
    if extra:
        assert np.max(np.abs(i0.shift_iters - i1.shift_iters)) <= 4
        assert d <= 1e-6
    elif basis:
        # the seed's basis form: the same iteration in another rounding order;
        # a freeze point may move where a shift's estimate stagnates near tol
        dm = int(np.max(np.abs(i0.shift_iters - i1.shift_iters)))
        assert dm <= 8
        if dm == 0:
            assert d <= 1e-10 and dx <= 1e-9
        else:
            assert d <= 10 * wk.tol
    else:
        assert np.array_equal(i0.shift_iters, i1.shift_iters)
        assert i0.mv_count == i1.mv_count
        assert d <= 1e-11 and dx <= 1e-10


def test_deferred_oracle_batch_forced():
    """Three right-hand sides, forced to the oracle's freeze iterations each."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    bb = wl.gaussian_source(wk.dims, 79, 3)
    refs, iters = [], []
    for r in range(3):
        it = oracle_run(op, a, bb[r], sig, w, 2, wk.tol, 2000, 1)[1].shift_iters
        refs.append(oracle_run(op, a, bb[r], sig, w, 2, wk.tol, 2000, 1, force=it)[0])
        iters.append(it)
    ctx = ctx_for(wk, U)
    y, info, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 2, wk.tol, 2000, 1, flags=msb.DEFERRED,
                                      force_iters=np.stack(iters))
    for r in range(3):
        assert rel(host(y)[r], refs[r]) <= 1e-10, r


def test_deferred_free_field_exhaustion():
    """A plane wave on the free field: the Krylov space is exhausted inside the
    first outer iteration (no MR); x_s = b / (A(p) + sigma_s) exactly."""
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
    for l in (1, 2, 4):
        y, info, xs = ctx.mshift_bicgstabl(cuda(b[None]), a, sig, w, l, 1e-8, 50, 1, flags=msb.DEFERRED,
                                           want_shifts=True)
        assert info.status == 0 and info.outer_iters == 1
        xs = host(xs)[0]
        for s in range(10):
            assert rel(xs[s], b / (lam + sig[s])) <= 1e-12, (l, s)


def test_deferred_mixed_refined_meets_tolerance():
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    bb = wl.gaussian_source(wk.dims, 94, 3)
    ctx = ctx_for(wk, U)
    y, info, xs = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, wk.tol, 3000, 1,
                                       flags=msb.MIXED | msb.REFINE | msb.DEFERRED, want_shifts=True)
    xs = host(xs)
    worst = 0.0
    for r in range(3):
        nb = np.linalg.norm(bb[r])
        for s in range(len(sig)):
            worst = max(worst, np.linalg.norm(bb[r] - op.a_op(xs[r, s], a) - sig[s] * xs[r, s]) / nb)
    log(f"  deferred mixed + refine: worst true residual {worst:.2e}, refined {info.refined_shifts}")
    assert worst <= wk.tol


def test_deferred_flag_restrictions():
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    ctx = ctx_for(wk, U)
    for flags, pass_ in ((msb.DEFERRED, 2), (msb.DEFERRED | msb.PERSISTENT, 1)):
        with pytest.raises(msb.MsbError) as e:
            ctx.mshift_bicgstabl(cuda(b), a, sig, w, 2, wk.tol, 10, pass_, flags=flags)
        assert e.value.status == msb.ERR_ARG

"""Sparse shadow residual.  When every right-hand side's r~ has at most 16
nonzero entries (r~ = b for a point source has one), the per-stage solve
(FP64 or mixed) skips the full read of r~ in the Mv epilogue, the MR update
and the reliable update and sums <r~, .> from an index list; the persistent
launch always reads r~ whole.
Both must give the same solve: bitwise for unit point sources (every product
with r~ is exact), to rounding for general sparse r~, and the oracle's result
with that r~.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import krylov as ok
from tests.helpers import cuda, host, log, problem, rel

pytestmark = pytest.mark.gpu


def sparse_shadow(dims, counts, seed):
    """[len(counts)][12][V] complex vectors with counts[r] random nonzero
    entries at random positions of row r."""
    rng = np.random.default_rng(seed)
    V = wl.volume(dims)
    out = np.zeros((len(counts), 12, V), dtype=np.complex128)
    for r, k in enumerate(counts):
        pos = rng.choice(12 * V, size=k, replace=False)
        out[r].reshape(-1)[pos] = rng.standard_normal(k) + 1j * rng.standard_normal(k)
    return out


@pytest.mark.parametrize("pass_", [1, 2, 3])
def test_sparse_shadow_matches_dense_path_and_oracle(pass_):
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    bb = wl.gaussian_source(wk.dims, 71, 3)
    counts = [1, 5, 16]          # 16: the largest list
    rt = sparse_shadow(wk.dims, counts, 72)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    force = np.full(len(sig), 3)
    allow = (msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY)
    y0, i0, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 2, wk.tol, 3, pass_, shadow=cuda(rt),
                                     force_iters=force, allow=allow)
    if pass_ != 3:
        y1, i1, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 2, wk.tol, 3, pass_, flags=msb.PERSISTENT,
                                         shadow=cuda(rt), force_iters=force, allow=allow)
        d = rel(host(y0), host(y1))
        log(f"sparse r~ (counts {counts}), pass {pass_}: per-stage vs persistent (dense r~) {d:.2e}")
        assert d <= 1e-13
    for r in range(3):
        ref = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), bb[r], sig, w, 2, wk.tol, 3, 1, shadow=rt[r],
                                  force_iters=force)[0]
        d = rel(host(y0)[r], ref)
        log(f"  rhs {r} ({counts[r]} nonzeros): vs oracle {d:.2e}")
        assert d <= 1e-10
    ctx.close()


def test_shadow_above_the_list_size_takes_the_dense_path():
    """17 nonzero entries in one row: the whole batch reads r~ in full, and the
    result equals the persistent (dense) launch bit for bit."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    bb = wl.gaussian_source(wk.dims, 73, 2)
    rt = sparse_shadow(wk.dims, [1, 17], 74)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    y0 = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 2, wk.tol, 2000, 1, shadow=cuda(rt))[0]
    y1 = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 2, wk.tol, 2000, 1, flags=msb.PERSISTENT, shadow=cuda(rt))[0]
    assert np.array_equal(host(y0), host(y1))
    ctx.close()


def test_unit_point_sources_bitwise_with_dense_path():
    """r~ = b = the 12 unit point sources (the bench workload's case, one
    nonzero 1.0 per row): the sparse dots are exact, so the per-stage solve
    equals the persistent one bit for bit (8^4, forced 3 outer iterations)."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    pts = wl.point_sources(wk.dims)
    force = np.full(len(sig), 3)
    allow = (msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    for flags in (0, msb.MIXED):
        for pass_ in (1, 2):
            y0 = ctx.mshift_bicgstabl(cuda(pts), a, sig, w, 4, wk.tol, 3, pass_, flags=flags, force_iters=force,
                                      allow=allow)[0]
            y1 = ctx.mshift_bicgstabl(cuda(pts), a, sig, w, 4, wk.tol, 3, pass_, flags=flags | msb.PERSISTENT,
                                      force_iters=force, allow=allow)[0]
            assert np.array_equal(host(y0), host(y1)), (flags, pass_)
    ctx.close()


@pytest.mark.parametrize("pass_", [1, 2, 3])
def test_sparse_shadow_mixed_precision(pass_):
    """Mixed precision with a sparse r~ of random entries: the list holds the
    values of r~'s FP32 copy, the reliable update's dot is taken against its
    FP64 residual; the solve matches the persistent (dense r~) launch to FP32
    rounding, with the same reliable updates and freeze iterations."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    bb = wl.gaussian_source(wk.dims, 75, 3)
    rt = sparse_shadow(wk.dims, [1, 4, 16], 76)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    y0, i0, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, wk.tol, 2000, pass_, flags=msb.MIXED,
                                     shadow=cuda(rt))
    if pass_ == 3:
        ref, iref, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, wk.tol, 2000, 1, flags=msb.MIXED,
                                            shadow=cuda(rt))
    else:
        ref, iref, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, wk.tol, 2000, pass_,
                                            flags=msb.MIXED | msb.PERSISTENT, shadow=cuda(rt))
    d = rel(host(y0), host(ref))
    log(f"mixed, sparse r~, pass {pass_}: vs {'per-stage pass 1' if pass_ == 3 else 'persistent'} {d:.2e}, "
        f"outer {i0.outer_iters}/{iref.outer_iters}, reliable updates {i0.reliable_updates}/{iref.reliable_updates}")
    assert d <= 1e-5
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_single_random_entry_bitwise_with_dense_path(precision):
    """One random complex entry per right-hand side: every <r~, .> is a single
    product, so the list path equals the dense persistent path bit for bit
    only if its value is exactly the one the dense kernels read (in mixed
    precision the FP32 copy of r~; the reliable update's dot against its FP64
    residual).  Forced 3 outer iterations, passes 1 and 2."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    bb = wl.gaussian_source(wk.dims, 77, 3)
    rt = sparse_shadow(wk.dims, [1, 1, 1], 78)
    force = np.full(len(sig), 3)
    allow = (msb.OK, msb.NOT_CONVERGED, msb.REDUCED_ACCURACY)
    flags = msb.MIXED if precision == "mixed" else 0
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    for pass_ in (1, 2):
        y0, i0, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, wk.tol, 3, pass_, flags=flags, shadow=cuda(rt),
                                         force_iters=force, allow=allow)
        y1, i1, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, wk.tol, 3, pass_, flags=flags | msb.PERSISTENT,
                                         shadow=cuda(rt), force_iters=force, allow=allow)
        log(f"single random entry, {precision}, pass {pass_}: max |diff| "
            f"{np.abs(host(y0) - host(y1)).max():.2e}, reliable updates {i0.reliable_updates}/{i1.reliable_updates}")
        assert np.array_equal(host(y0), host(y1)), pass_
    ctx.close()

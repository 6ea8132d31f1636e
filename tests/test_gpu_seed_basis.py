"""The basis form of the seed (MSB_SEED_BASIS; passes 2 and 3, FP64): each
BiCG step of Section 2 writes only the two vectors its Mv reads; the other
r_i, u_i of the outer iteration stay coefficients on its basis (r_0, u_0 and
the Mv outputs) and are formed from it for the MR step's Gram matrix and
update.  The Krylov-exhaustion test, which reads ||r_0|| after each step,
runs only where the bound ||r_0|| >= ||r_{j-1}|| / ||S||^(j-1) lets it fire.

Same arithmetic as the explicit form up to rounding order: the oracle's
double pass is matched at the parity bound of the explicit form (forced
freeze iterations); unforced runs take the explicit form's iteration path
(same M_s, same Mv and inner-product counts) with y equal to rounding; the
breakdown branches are in tests/test_gpu_breakdown.py.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import dirac as od
from oracle import pfe
from tests.helpers import A_SCALE_BOUND, cuda, host, log, problem, rel
from tests.test_gpu_solver import ctx_for, oracle_run, parity_bound

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pass_", [2, 3])
@pytest.mark.parametrize("l", [1, 2, 4])
def test_basis_forced_matches_oracle(l, pass_):
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    log(f"seed basis forced 4x4x4x8 l={l} pass {pass_}")
    y1, i1, _ = oracle_run(op, a, b[0], sig, w, l, wk.tol, 2000, 1)
    y2, _ = oracle_run(op, a, b[0], sig, w, l, wk.tol, 2000, 2, force=i1.shift_iters)
    ctx = ctx_for(wk, U)
    y, info, _ = ctx.mshift_bicgstabl(cuda(b), a, sig, w, l, wk.tol, 2000, pass_, flags=msb.SEED_BASIS,
                                      force_iters=i1.shift_iters)
    bound = parity_bound(op, a, b[0], sig, w, l, wk.tol, i1.shift_iters, y1)
    log(f"  bound {bound:.2e}, rel err {rel(host(y)[0], y2):.2e}, M {info.outer_iters}")
    assert np.array_equal(info.shift_iters[0], i1.shift_iters)
    assert rel(host(y)[0], y2) <= bound
    # against the explicit form: two rounding orders of one iteration, so the
    # same bound (BiCGstab(1) amplifies rounding to ~1e-8 over these 80
    # outer iterations)
    ye, ie, _ = ctx.mshift_bicgstabl(cuda(b), a, sig, w, l, wk.tol, 2000, pass_, force_iters=i1.shift_iters)
    assert info.mv_count == ie.mv_count and info.dot_count == ie.dot_count
    d = rel(host(y), host(ye))
    log(f"  vs explicit form {d:.2e}")
    assert d <= bound


def rounding_bound(ctx, bb, a, S, W, l, tol, max_outer, pass_, y0):
    """1e-11, or 30x the explicit form's own change when b is perturbed by
    1e-15 relative (the size of one rounding-order difference) where the
    iteration amplifies rounding more than that."""
    rng = np.random.default_rng(2468)
    bp = bb * (1 + 1e-15 * rng.standard_normal(bb.shape))
    yp, _, _ = ctx.mshift_bicgstabl(cuda(bp), a, S, W, l, tol, max_outer, pass_)
    return max(1e-11, 30 * rel(host(yp), host(y0)))


@pytest.mark.parametrize("pass_", [2, 3])
def test_basis_batch_with_shift_sets_matches_explicit(pass_):
    """Six right-hand sides (chunked stencil), rhs 1 with a padded 6-pole set,
    unforced.  Rounding-order differences can move a freeze point where a
    shift's residual estimate stagnates near the tolerance (BiCGstab(2) on
    rhs 5 does for several outer iterations: its smallest shift freezes at
    M = 62 in the explicit form, 68 in the basis form); so M_s agree within 8
    and y within the explicit form's own rounding sensitivity, or the
    tolerance where a freeze point moved."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("8x8x8x8")
    bb = wl.gaussian_source(wk.dims, 97, 6)
    s2, w2 = pfe.neuberger(6)
    S = np.tile(sig, (6, 1))
    W = np.tile(w, (6, 1))
    S[1, :6], W[1, :6] = s2, w2
    S[1, 6:], W[1, 6:] = s2[-1] * 2, 0.0
    ctx = ctx_for(wk, U)
    for l in (2, 4):
        y0, i0, _ = ctx.mshift_bicgstabl(cuda(bb), a, S, W, l, wk.tol, 3000, pass_)
        y1, i1, _ = ctx.mshift_bicgstabl(cuda(bb), a, S, W, l, wk.tol, 3000, pass_, flags=msb.SEED_BASIS)
        d = rel(host(y1), host(y0))
        bound = rounding_bound(ctx, bb, a, S, W, l, wk.tol, 3000, pass_, y0)
        log(f"  pass {pass_} l={l}: basis vs explicit y {d:.2e} (bound {bound:.1e}), M {i1.outer_iters} "
            f"({i0.outer_iters})")
        dm = int(np.max(np.abs(i0.shift_iters - i1.shift_iters)))
        assert i0.status == i1.status and dm <= 8
        if dm == 0:
            assert i0.mv_count == i1.mv_count and i0.dot_count == i1.dot_count
            assert d <= bound
        else:
            assert d <= max(bound, 10 * wk.tol)


def test_basis_batched_shift_sets_forced_matches_oracle():
    """Three right-hand sides, rhs 1 with a padded 6-pole set, each forced to
    the oracle's freeze iterations: passes 2 and 3 in basis form against the
    oracle's iteration of every right-hand side."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    bb = wl.gaussian_source(wk.dims, 77, 3)
    s2, w2 = pfe.neuberger(6)
    sets_s = np.zeros((3, 10))
    sets_w = np.zeros((3, 10))
    sets_s[0], sets_w[0] = sig, w
    sets_s[2], sets_w[2] = sig, w
    sets_s[1, :6], sets_w[1, :6] = s2, w2
    sets_s[1, 6:], sets_w[1, 6:] = s2[-1] * 2, 0.0
    refs, iters = [], []
    for r in range(3):
        yr, ir, _ = oracle_run(op, a, bb[r], sets_s[r], sets_w[r], 2, wk.tol, 2000, 1)
        refs.append(yr)
        iters.append(ir.shift_iters)
    ctx = ctx_for(wk, U)
    for pass_ in (2, 3):
        y, info, _ = ctx.mshift_bicgstabl(cuda(bb), a, sets_s, sets_w, 2, wk.tol, 2000, pass_,
                                          flags=msb.SEED_BASIS, force_iters=np.stack(iters))
        for r in range(3):
            d = rel(host(y)[r], refs[r])
            log(f"  shift sets, pass {pass_}, rhs {r}: {d:.2e}")
            assert d <= 1e-10, (pass_, r)


@pytest.mark.parametrize("l", [2, 4])
def test_basis_point_sources_forced_matches_oracle(l):
    """Point sources (r~ = b with one nonzero entry: the sparse list, with
    which the MR update also makes the next outer iteration's first
    direction update), each forced to the oracle's freeze iterations, pass 3
    in basis form against the oracle's iteration at its parity bound."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    ps = wl.point_sources(wk.dims)[[0, 7]]
    ctx = ctx_for(wk, U)
    for k in range(2):
        y1, i1, _ = oracle_run(op, a, ps[k], sig, w, l, wk.tol, 2000, 1)
        bound = parity_bound(op, a, ps[k], sig, w, l, wk.tol, i1.shift_iters, y1)
        y, info, _ = ctx.mshift_bicgstabl(cuda(ps[k:k + 1]), a, sig, w, l, wk.tol, 2000, 3, flags=msb.SEED_BASIS,
                                          force_iters=i1.shift_iters)
        d = rel(host(y)[0], y1)
        log(f"  point source {k}, l={l}: {d:.2e} (bound {bound:.1e}), M {info.outer_iters}")
        assert np.array_equal(info.shift_iters[0], i1.shift_iters)
        assert d <= bound, k


def test_basis_production_lattice_fixed_iterations():
    """16^3x32 (one of the 12 point sources), 2 forced outer iterations of
    l = 4, N_s = 30: the basis form against the oracle's iteration."""
    from paper_1010_2592_amd import msb
    wk = wl.WORKLOADS["16x16x16x32"]
    U = wk.links()
    op = od.Dirac(U, wk.dims, wk.mass, wk.mu, wk.bc_t)
    b = wl.point_sources(wk.dims)[[7]]
    sig, w = pfe.neuberger(wk.n_shift)
    a = A_SCALE_BOUND
    force = np.full(len(sig), 2)
    ref = oracle_run(op, a, b[0], sig, w, 4, wk.tol, 2, 1, force=force)[0]
    ctx = ctx_for(wk, U)
    for pass_ in (2, 3):
        y, info, _ = ctx.mshift_bicgstabl(cuda(b), a, sig, w, 4, wk.tol, 2, pass_, flags=msb.SEED_BASIS,
                                          force_iters=force, allow=(msb.OK, msb.NOT_CONVERGED))
        d = rel(host(y)[0], ref)
        log(f"  16^3x32 pass {pass_} l=4 basis: {d:.2e}")
        assert d <= 1e-10, pass_


def test_basis_l8_matches_oracle():
    """l = 8, the largest basis (18 vectors): three forced outer iterations."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    force = np.full(len(sig), 3)
    y1 = oracle_run(op, a, b[0], sig, w, 8, wk.tol, 3, 1, force=force)[0]
    y2 = oracle_run(op, a, b[0], sig, w, 8, wk.tol, 3, 2, force=force)[0]
    bound = parity_bound(op, a, b[0], sig, w, 8, wk.tol, force, y1)
    ctx = ctx_for(wk, U)
    for pass_ in (2, 3):
        y, info, _ = ctx.mshift_bicgstabl(cuda(b), a, sig, w, 8, wk.tol, 3, pass_, flags=msb.SEED_BASIS,
                                          force_iters=force, allow=(msb.OK, msb.NOT_CONVERGED))
        d = rel(host(y)[0], y2)
        log(f"  l=8 pass {pass_} basis: {d:.2e} (bound {bound:.2e})")
        assert d <= bound, pass_


def test_basis_free_field_exhaustion():
    """A plane wave on the free field: the Krylov space is exhausted in the
    first step (r_1 = lambda r_0), the test fires in step 1 through the
    bound, and y = sum_s w_s b / (A(p) + sigma_s) exactly."""
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
    for pass_ in (2, 3):
        for l in (1, 2, 4):
            y, info, _ = ctx.mshift_bicgstabl(cuda(b[None]), a, sig, w, l, 1e-8, 50, pass_, flags=msb.SEED_BASIS)
            log(f"  free field pass {pass_} l={l}: M {info.outer_iters}, {rel(host(y)[0], ref):.2e}")
            assert info.status == 0 and info.outer_iters == 1
            assert rel(host(y)[0], ref) <= 1e-12, (pass_, l)


def test_basis_exhaustion_in_step_three_scaled_links():
    """Three plane waves on free links scaled by 1.3 (not unitary: the norm
    bound of the exhaustion gate takes the links' own norm): the Krylov space
    has dimension 3, so at l = 4 the test fires in step 3 of the first outer
    iteration in both forms, and y is the exact sum over the waves."""
    from paper_1010_2592_amd import msb
    dims = (4, 4, 4, 8)
    Lx, Ly, Lz, Lt = dims
    mu, m, c = 0.05, -2.0, 1.3
    U = c * wl.free_links(dims)
    a = 1 / 60.0
    t, z, y_, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    waves, lams = [], []
    for k, p in enumerate(([2 * np.pi / Lx, 4 * np.pi / Ly, 0.0, np.pi * 7 / Lt],
                           [0.0, 2 * np.pi / Ly, 2 * np.pi / Lz, np.pi / Lt],
                           [6 * np.pi / Lx, 0.0, 4 * np.pi / Lz, np.pi * 3 / Lt])):
        q = np.array(p, dtype=complex)
        q[3] -= 1j * mu
        phase = np.exp(1j * (p[0] * x + p[1] * y_ + p[2] * z + p[3] * t)).reshape(-1)
        waves.append(((np.arange(1, 13) + k) * (1 + 0.5j * (k + 1)))[:, None] * phase[None, :])
        lams.append(a * ((4 + m - c * np.sum(np.cos(q))) ** 2 + c * c * np.sum(np.sin(q) ** 2)))
    assert min(abs(lams[i] - lams[j]) for i in range(3) for j in range(i)) > 1e-3
    b = sum(waves)
    sig, w = pfe.neuberger(10)
    ref = sum(w[s] * sum(v / (lam + sig[s]) for v, lam in zip(waves, lams)) for s in range(10))
    ctx = msb.Context(msb.Lattice(dims, m, mu, -1), cuda(U))
    for pass_ in (2, 3):
        for flags in (0, msb.SEED_BASIS):
            y, info, _ = ctx.mshift_bicgstabl(cuda(b[None]), a, sig, w, 4, 1e-8, 50, pass_, flags=flags)
            d = rel(host(y)[0], ref)
            log(f"  three waves, links x{c}, pass {pass_} flags {flags}: M {info.outer_iters}, "
                f"steps {info.bicg_steps}, {d:.2e}")
            assert info.status == 0 and info.outer_iters == 1 and info.bicg_steps == 3, (pass_, flags)
            assert d <= 1e-11, (pass_, flags)


@pytest.mark.parametrize("pass_", [2, 3])
def test_basis_sparse_shadow(pass_):
    """Point sources with r~ = b (one nonzero entry: the index-list path of
    the inner products with r~), unforced: the basis form against the
    explicit form.  A = a D (MSB_OP_WILSON) is in tests/test_gpu_propagators.py."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    bb = wl.point_sources(wk.dims)[[0, 5, 11]]
    ctx = ctx_for(wk, U)
    y0, i0, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, wk.tol, 2000, pass_)
    y1, i1, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, wk.tol, 2000, pass_, flags=msb.SEED_BASIS)
    d = rel(host(y1), host(y0))
    bound = rounding_bound(ctx, bb, a, sig, w, 4, wk.tol, 2000, pass_, y0)
    log(f"  point sources, sparse r~, pass {pass_}: basis vs explicit {d:.2e} (bound {bound:.1e}), "
        f"M {i1.outer_iters}")
    assert np.array_equal(i0.shift_iters, i1.shift_iters) and d <= bound


@pytest.mark.parametrize("split", [1, 0])
def test_basis_store_limit(split):
    """Pass 3 under a store limit that holds one chunk of 8 outer iterations
    (split = 1) or none: the iterations beyond the store run on rows 1..l of
    the seed's own vectors as basis, and the regeneration replays them; y
    equals the unlimited basis-form pass 3 to rounding."""
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    l = 2
    bb = np.concatenate([b, wl.gaussian_source(wk.dims, 8802, 2)])
    ctx = ctx_for(wk, U)
    y3, i3, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, l, wk.tol, 2000, 3, flags=msb.SEED_BASIS)
    assert i3.outer_iters > 8
    n = 12 * wl.volume(wk.dims)
    cb = bb.shape[0] * 8 * 2 * l * n * 16
    ctx.set_store_limit(cb + cb // 2 if split else cb // 2)
    yh, ih, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, l, wk.tol, 2000, 3, flags=msb.SEED_BASIS)
    ctx.set_store_limit(0)
    d = rel(host(yh), host(y3))
    log(f"  basis pass 3, store limit holding {8 * split} iterations: stored {ih.stored_iters}, y {d:.2e}")
    assert ih.stored_iters == 8 * split
    assert np.array_equal(ih.shift_iters, i3.shift_iters) and d <= 1e-12


def test_basis_flag_restrictions():
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    ctx = ctx_for(wk, U)
    for flags, pass_ in ((msb.SEED_BASIS, 1), (msb.SEED_BASIS | msb.MIXED, 2),
                         (msb.SEED_BASIS | msb.PERSISTENT, 2), (msb.SEED_BASIS | msb.MIXED, 3)):
        with pytest.raises(msb.MsbError) as e:
            ctx.mshift_bicgstabl(cuda(b), a, sig, w, 2, wk.tol, 10, pass_, flags=flags)
        assert e.value.status == msb.ERR_ARG
    with pytest.raises(msb.MsbError) as e:
        ctx.mshift_bicgstabl_noalloc(cuda(b), a, sig, w, 2, wk.tol, 10, 2, flags=msb.SEED_BASIS)
    assert e.value.status == msb.ERR_ARG

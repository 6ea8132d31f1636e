"""Multi-shift CG on the GPU (mu = 0, A = a (gamma5 D_w)^2 Hermitian): single
pass, Neuberger's double pass and the pseudo-double pass against the CG
oracle -- forced freeze iterations at the parity bound, unforced runs at the
tolerance -- plus true residuals, batches with per-source shift sets,
free-field exactness, agreement with BiCGstab(l), and argument checks.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import cg as ocg
from oracle import dirac as od
from oracle import pfe
from tests.helpers import cuda, host, log, rel

pytestmark = pytest.mark.gpu


def mu0_problem(dims, seed, ns):
    U = wl.gauge_links(dims, 0.6, seed)
    op = od.Dirac(U, dims, -2.0, 0.0, -1)
    a = od.a_scale_from_radius(od.spectral_radius(op, wl.start_vector(dims, seed + 1), 100))
    sig, w = pfe.neuberger(ns)
    return U, op, a, sig, w


def ctx_mu0(dims, U):
    from paper_1010_2592_amd import msb
    return msb.Context(msb.Lattice(dims, -2.0, 0.0, -1), cuda(U))


@pytest.mark.parametrize("pass_", [1, 2, 3])
def test_cg_forced_matches_oracle(pass_):
    dims = (4, 4, 4, 8)
    U, op, a, sig, w = mu0_problem(dims, 51, 10)
    b = wl.gaussian_source(dims, 52)[0]
    y0, i0 = ocg.mshift_cg(lambda v: op.a_op(v, a), b, sig, w, 1e-10, 2000, 1)
    force = i0.shift_iters
    out = ocg.mshift_cg(lambda v: op.a_op(v, a), b, sig, w, 1e-10, 2000, pass_, force_iters=force,
                        want_shifts=(pass_ == 1))
    ctx = ctx_mu0(dims, U)
    y, info, xs = ctx.mshift_cg(cuda(b[None]), a, sig, w, 1e-10, 2000, pass_, want_shifts=(pass_ == 1),
                                force_iters=force)
    d = rel(host(y)[0], out[0])
    log(f"CG pass {pass_} forced: N {info.outer_iters}, rel err vs oracle {d:.2e}")
    assert np.array_equal(info.shift_iters[0], force)
    assert d <= 1e-10
    N = int(force.max())
    assert info.mv_count == (2 * N - 1 if pass_ == 2 else N)
    assert info.dot_count == 2 * N
    if pass_ == 1:
        xs = host(xs)[0]
        for s in range(len(sig)):
            assert rel(xs[s], out[2][s]) <= 1e-10, s


def test_cg_unforced_freeze_and_true_residuals():
    dims = (8, 8, 8, 8)
    U, op, a, sig, w = mu0_problem(dims, 53, 16)
    b = wl.gaussian_source(dims, 54)[0]
    tol = 1e-9
    y0, i0 = ocg.mshift_cg(lambda v: op.a_op(v, a), b, sig, w, tol, 3000, 1)
    ctx = ctx_mu0(dims, U)
    y, info, xs = ctx.mshift_cg(cuda(b[None]), a, sig, w, tol, 3000, 1, want_shifts=True)
    log(f"CG unforced 8^4: N {info.outer_iters} (oracle {i0.iters}), y vs oracle {rel(host(y)[0], y0):.2e}")
    assert np.max(np.abs(info.shift_iters[0] - i0.shift_iters)) <= 1
    assert rel(host(y)[0], y0) <= 10 * tol
    xs = host(xs)[0]
    for s in range(len(sig)):
        tr = np.linalg.norm(b - op.a_op(xs[s], a) - sig[s] * xs[s]) / np.linalg.norm(b)
        assert tr <= tol, (s, tr)
        assert abs(tr - info.shift_resid[0, s]) <= 1e-3 * tol + 1e-2 * tr


def test_cg_batch_shift_sets_three_passes():
    """Six sources (chunked stencil), source 1 with a padded 6-pole set; the
    three passes agree, the residual store spans several chunks, each
    source matches the oracle."""
    dims = (8, 8, 8, 8)
    U, op, a, sig, w = mu0_problem(dims, 55, 12)
    bb = wl.gaussian_source(dims, 56, 6)
    s2, w2 = pfe.neuberger(6)
    S = np.tile(sig, (6, 1))
    W = np.tile(w, (6, 1))
    S[1, :6], W[1, :6] = s2, w2
    S[1, 6:], W[1, 6:] = s2[-1] * 2, 0.0
    ctx = ctx_mu0(dims, U)
    y1, i1, _ = ctx.mshift_cg(cuda(bb), a, S, W, 1e-9, 3000, 1)
    y2, i2, _ = ctx.mshift_cg(cuda(bb), a, S, W, 1e-9, 3000, 2)
    y3, i3, _ = ctx.mshift_cg(cuda(bb), a, S, W, 1e-9, 3000, 3)
    log(f"CG batch: N {i1.outer_iters}, 2 vs 1 {rel(host(y2), host(y1)):.2e}, 3 vs 1 {rel(host(y3), host(y1)):.2e}")
    assert i3.outer_iters > 64
    assert np.array_equal(i1.shift_iters, i2.shift_iters) and np.array_equal(i1.shift_iters, i3.shift_iters)
    assert rel(host(y2), host(y1)) <= 1e-11 and rel(host(y3), host(y1)) <= 1e-11
    for r in range(6):
        ref = ocg.mshift_cg(lambda v: op.a_op(v, a), bb[r], S[r], W[r], 1e-9, 3000, 2,
                            force_iters=i1.shift_iters[r])[0]
        assert rel(host(y3)[r], ref) <= 1e-10, r


def test_cg_matches_bicgstab_at_mu0():
    from paper_1010_2592_amd import msb
    dims = (8, 8, 8, 8)
    U, op, a, sig, w = mu0_problem(dims, 57, 16)
    bb = wl.gaussian_source(dims, 58, 4)
    ctx = ctx_mu0(dims, U)
    y_cg, icg, _ = ctx.mshift_cg(cuda(bb), a, sig, w, 1e-10, 3000, 3)
    y_bi, ibi, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 4, 1e-10, 3000, 3)
    log(f"CG vs BiCGstab(4) at mu = 0: {rel(host(y_cg), host(y_bi)):.2e}; Mv {icg.mv_count} vs {ibi.mv_count}")
    assert rel(host(y_cg), host(y_bi)) <= 1e-8


def test_cg_free_field_exact():
    dims = (4, 4, 4, 8)
    Lx, Ly, Lz, Lt = dims
    m = -2.0
    U = wl.free_links(dims)
    a = 1 / 36.5
    t, z, y_, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    p = np.array([2 * np.pi / Lx, 4 * np.pi / Ly, 0.0, np.pi * 7 / Lt])
    phase = np.exp(1j * (p[0] * x + p[1] * y_ + p[2] * z + p[3] * t)).reshape(-1)
    b = (np.arange(1, 13) * (1 + 0.5j))[:, None] * phase[None, :]
    lam = a * ((4 + m - np.sum(np.cos(p))) ** 2 + np.sum(np.sin(p) ** 2))
    sig, w = pfe.neuberger(6)
    ref = sum(w[s] * b / (lam + sig[s]) for s in range(6))
    ctx = ctx_mu0(dims, U)
    for pass_ in (1, 2, 3):
        y, info, _ = ctx.mshift_cg(cuda(b[None]), a, sig, w, 1e-10, 50, pass_)
        assert info.outer_iters == 1 and info.status == 0
        assert rel(host(y)[0], ref) <= 1e-13, pass_


def test_cg_argument_checks():
    from paper_1010_2592_amd import msb
    dims = (4, 4, 4, 8)
    U, op, a, sig, w = mu0_problem(dims, 59, 6)
    b = cuda(wl.gaussian_source(dims, 60)[0][None])
    ctx_mu = msb.Context(msb.Lattice(dims, -2.0, 0.05, -1), cuda(U))
    with pytest.raises(msb.MsbError) as e:
        ctx_mu.mshift_cg(b, a, sig, w, 1e-8, 100, 1)
    assert e.value.status == msb.ERR_ARG
    ctx = ctx_mu0(dims, U)
    for pass_ in (0, 4):
        with pytest.raises(msb.MsbError) as e:
            ctx.mshift_cg(b, a, sig, w, 1e-8, 100, pass_)
        assert e.value.status == msb.ERR_ARG
    with pytest.raises(msb.MsbError) as e:
        ctx.mshift_cg(b, a, sig, w, 1e-8, 100, 2, want_shifts=True)
    assert e.value.status == msb.ERR_ARG
    y, info, _ = ctx.mshift_cg(b * 0, a, sig, w, 1e-8, 100, 1)
    assert info.status == 0 and float(host(y).__abs__().max()) == 0.0

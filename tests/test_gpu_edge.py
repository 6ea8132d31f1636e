"""Degenerate inputs the method has: a zero source (f(A) 0 = 0, no
iteration) inside a batch and a batch of zero sources, for every pass of
BiCGstab(l) and of the mu = 0 CG.  The zero source's y must be exactly zero
with no iterations charged to its shifts, and the other sources must come out
as when solved without it (passes 2 and 3 also with the seed in basis form)."""
import numpy as np
import pytest

import workloads as wl
from oracle import dirac as od
from tests.helpers import cuda, host, log, problem, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pass_,basis", [(1, False), (2, False), (3, False), (2, True), (3, True)])
def test_zero_source_in_a_bicgstab_batch(pass_, basis):
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    bb = wl.gaussian_source(wk.dims, 81, 3)
    bb[1] = 0.0
    flags = msb.SEED_BASIS if basis else 0
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    y, info, _ = ctx.mshift_bicgstabl(cuda(bb), a, sig, w, 2, wk.tol, 2000, pass_, flags=flags)
    assert info.status == msb.OK
    yh = host(y)
    assert np.all(yh[1] == 0.0)
    assert np.all(info.shift_iters[1] == 0)
    y2, info2, _ = ctx.mshift_bicgstabl(cuda(bb[[0, 2]]), a, sig, w, 2, wk.tol, 2000, pass_, flags=flags)
    d = max(rel(yh[0], host(y2)[0]), rel(yh[2], host(y2)[1]))
    log(f"zero source in a batch, pass {pass_}{' seed basis' if basis else ''}: others vs solved alone {d:.2e}, "
        f"iters {info.shift_iters.max(axis=1)}")
    assert d <= 1e-13
    assert np.array_equal(info.shift_iters[[0, 2]], info2.shift_iters)
    ctx.close()


@pytest.mark.parametrize("pass_", [1, 2, 3])
def test_zero_source_in_a_cg_batch(pass_):
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    op0 = od.Dirac(U, wk.dims, wk.mass, 0.0, wk.bc_t)
    a0 = od.a_scale_from_radius(od.spectral_radius(op0, wk.power_start(), 100))
    bb = wl.gaussian_source(wk.dims, 82, 3)
    bb[0] = 0.0
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, 0.0, wk.bc_t), cuda(U))
    y, info, _ = ctx.mshift_cg(cuda(bb), a0, sig, w, wk.tol, 5000, pass_)
    assert info.status == msb.OK
    yh = host(y)
    assert np.all(yh[0] == 0.0)
    assert np.all(info.shift_iters[0] == 0)
    y2, info2, _ = ctx.mshift_cg(cuda(bb[1:]), a0, sig, w, wk.tol, 5000, pass_)
    d = rel(yh[1:], host(y2))
    log(f"zero source in a CG batch, pass {pass_}: others vs solved alone {d:.2e}")
    assert d <= 1e-13
    ctx.close()


def test_batch_of_zero_sources():
    from paper_1010_2592_amd import msb
    wk, U, op, a, sig, w, b = problem("4x4x4x8")
    zero = np.zeros((2, 12, wl.volume(wk.dims)), dtype=np.complex128)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    for pass_, flags in ((1, 0), (2, 0), (3, 0), (2, msb.SEED_BASIS), (3, msb.SEED_BASIS)):
        y, info, _ = ctx.mshift_bicgstabl(cuda(zero), a, sig, w, 2, wk.tol, 50, pass_, flags=flags)
        assert info.status == msb.OK and np.all(host(y) == 0.0) and info.outer_iters == 0, (pass_, flags)
    s, info = ctx.pfe_sign_apply(cuda(zero), a, sig, w, 2, wk.tol, 50, 1)
    assert np.all(host(s) == 0.0)
    ctx.close()

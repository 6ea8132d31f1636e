"""GPU parity of wilson_apply (the stencil D_w(mu), Section 1) against the oracle,
element by element, on several lattices including odd and ragged extents
(sites not a multiple of the 256-thread block), several right-hand sides and
every flag combination; plus the spectral-radius estimate."""
import numpy as np
import pytest

import workloads as wl
from oracle import dirac as od
from tests.helpers import cuda, host, log, rel

pytestmark = pytest.mark.gpu

FLAG_CASES = [0, 1, 2, 4, 1 | 4, 1 | 2]


def oracle_apply(op, v, flags):
    out = []
    for x in v:
        if flags & 4:  # dagger
            y = op.dw_dag(x) if not (flags & 2) else od.g5(op.dw(od.g5(x), op.mu))
        else:
            y = op.dw(x, -op.mu if flags & 2 else op.mu)
        if flags & 1:
            y = od.g5(y)
        out.append(y)
    return np.stack(out)


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (3, 5, 2, 6), (8, 8, 8, 8), (6, 4, 10, 3)])
@pytest.mark.parametrize("flags", FLAG_CASES)
def test_wilson_apply_fp64(dims, flags):
    from paper_1010_2592_amd import msb
    log(f"wilson_apply fp64 dims={dims} flags={flags}")
    U = wl.gauge_links(dims, 0.6, 11 + sum(dims))
    mu = 0.13
    op = od.Dirac(U, dims, -2.0, mu, -1)
    v = wl.gaussian_source(dims, 5, 3)
    ctx = msb.Context(msb.Lattice(dims, -2.0, mu, -1), cuda(U))
    out = host(ctx.wilson_apply(cuda(v), flags))
    ref = oracle_apply(op, v, flags)
    for r in range(3):
        assert rel(out[r], ref[r]) <= 1e-14, (dims, flags, r)


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (3, 5, 2, 6), (6, 4, 10, 3), (8, 8, 8, 8), (16, 4, 2, 6),
                                  (16, 3, 3, 5)])
@pytest.mark.parametrize("flags", FLAG_CASES)
def test_batched_chunked_stencil_matches_single_rhs(dims, flags):
    """Batches of >= 4 right-hand sides take the chunked stencil (links staged
    in LDS per 64-site chunk); single right-hand sides the site-block one.
    Same arithmetic: bitwise equal outputs, and the oracle at 1e-14.  Lattices
    with whole chunks per time slice (t-fastest chunk order) and without;
    Lx = 16 takes the x-neighbours from the adjacent lanes of a row, with a
    whole z-t plane per wavefront (16 x 4) and with wavefronts that straddle
    planes (16 x 3)."""
    from paper_1010_2592_amd import msb
    log(f"chunked stencil dims={dims} flags={flags}")
    U = wl.gauge_links(dims, 0.6, 21 + sum(dims))
    mu = 0.11
    op = od.Dirac(U, dims, -2.0, mu, -1)
    v = wl.gaussian_source(dims, 9, 5)
    ctx = msb.Context(msb.Lattice(dims, -2.0, mu, -1), cuda(U))
    for extra in (0, msb.MIXED):
        batch = host(ctx.wilson_apply(cuda(v), flags | extra))
        for r in range(5):
            single = host(ctx.wilson_apply(cuda(v[r:r + 1]), flags | extra))[0]
            assert np.array_equal(batch[r], single), (dims, flags, extra, r)
    ref = oracle_apply(op, v, flags)
    out = host(ctx.wilson_apply(cuda(v), flags))
    for r in range(5):
        assert rel(out[r], ref[r]) <= 1e-14, (dims, flags, r)


@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (5, 3, 2, 7)])
def test_wilson_apply_fp32(dims):
    from paper_1010_2592_amd import msb
    log(f"wilson_apply fp32 dims={dims}")
    U = wl.gauge_links(dims, 0.6, 3)
    op = od.Dirac(U, dims, -2.0, 0.05, -1)
    v = wl.gaussian_source(dims, 6, 2)
    ctx = msb.Context(msb.Lattice(dims, -2.0, 0.05, -1), cuda(U))
    for flags in (0, 1, 4):
        out = host(ctx.wilson_apply(cuda(v), flags | msb.MIXED))
        ref = oracle_apply(op, v, flags)
        assert rel(out, ref) <= 2e-6


def test_wilson_apply_production_lattice_and_periodic_time():
    from paper_1010_2592_amd import msb
    dims = (16, 16, 16, 32)
    log(f"wilson_apply fp64 dims={dims}")
    U = wl.gauge_links(dims, 0.5, 1003)
    v = wl.gaussian_source(dims, 9, 1)
    for bc in (-1, 1):
        op = od.Dirac(U, dims, -2.0, 0.05, bc)
        ctx = msb.Context(msb.Lattice(dims, -2.0, 0.05, bc), cuda(U))
        out = host(ctx.wilson_apply(cuda(v), 1))
        assert rel(out[0], od.g5(op.dw(v[0]))) <= 1e-14
        ctx.close()


def test_wilson_apply_deterministic():
    from paper_1010_2592_amd import msb
    dims = (8, 8, 8, 8)
    U = wl.gauge_links(dims, 0.6, 1002)
    v = cuda(wl.gaussian_source(dims, 1, 2))
    ctx = msb.Context(msb.Lattice(dims, -2.0, 0.1, -1), cuda(U))
    a = host(ctx.wilson_apply(v, 1))
    b = host(ctx.wilson_apply(v, 1))
    assert np.array_equal(a, b)


def test_spectral_radius_matches_oracle():
    from paper_1010_2592_amd import msb
    wk = wl.WORKLOADS["4x4x4x8"]
    U = wk.links()
    op = od.Dirac(U, wk.dims, wk.mass, wk.mu, wk.bc_t)
    ref = od.spectral_radius(op, wk.power_start(), 100)
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), cuda(U))
    got = ctx.spectral_radius(cuda(wk.power_start()[None]), 100)
    assert abs(got - ref) <= 1e-10 * ref


def test_bad_arguments_raise():
    from paper_1010_2592_amd import msb
    dims = (4, 4, 4, 8)
    U = wl.gauge_links(dims, 0.6, 1)
    ctx = msb.Context(msb.Lattice(dims, -2.0, 0.05, -1), cuda(U))
    v = cuda(wl.gaussian_source(dims, 1, 1))
    with pytest.raises(msb.MsbError):
        ctx.wilson_apply(v, 1 << 10)

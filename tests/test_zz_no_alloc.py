"""mshift_bicgstabl_noalloc: the workspace taken from the library's fixed
device scratch array instead of device allocations.  Its outputs must equal
those of mshift_bicgstabl (the same kernels on the same inputs), on two calls
in a row with the second on a smaller batch (the array keeps the first call's
contents), for the double pass and the single pass, FP64 and mixed precision;
an oversized call must be refused before anything runs; and the call must not
take device memory."""
import numpy as np
import pytest

import workloads as wl
from tests.helpers import cuda, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1010_2592_amd import msb
    wk = wl.WORKLOADS["8x8x8x8"]
    U = cuda(wk.links())
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), U)
    rho = ctx.spectral_radius(cuda(wk.power_start()[None]), 100)
    a = 1.0 / (1.01 * rho)
    sig, w = msb.neuberger_pfe(wk.n_shift)
    b3 = cuda(wl.gaussian_source(wk.dims, 7101, 3))
    b1 = cuda(wl.gaussian_source(wk.dims, 7102, 1))
    yield wk, U, ctx, a, sig, w, b3, b1
    ctx.close()
    torch.cuda.empty_cache()


def _max_rel(x, y):
    import torch
    return float((torch.linalg.vector_norm((x - y).reshape(x.shape[0], -1), dim=1) /
                  torch.linalg.vector_norm(y.reshape(y.shape[0], -1), dim=1)).max())


@pytest.mark.parametrize("pass_,flags_name", [(2, "fp64"), (2, "mixed"), (1, "fp64"), (1, "deferred")])
def test_noalloc_matches_allocating_entry_point(setup, pass_, flags_name):
    import torch
    from paper_1010_2592_amd import msb
    wk, U, ctx, a, sig, w, b3, b1 = setup
    flags = {"fp64": 0, "mixed": msb.MIXED, "deferred": msb.DEFERRED}[flags_name]
    for k, b in enumerate((b3, b1)):         # the second call on a smaller batch
        log(f"noalloc pass {pass_} {flags_name}: call {k + 1}, nrhs {b.shape[0]}")
        want = pass_ == 1
        y0, i0, x0 = ctx.mshift_bicgstabl(b, a, sig, w, 4, wk.tol, 500, pass_, flags=flags, want_shifts=want)
        y1, i1, x1 = ctx.mshift_bicgstabl_noalloc(b, a, sig, w, 4, wk.tol, 500, pass_, flags=flags,
                                                  want_shifts=want)
        d = _max_rel(y1, y0)
        log(f"  M = {i1.outer_iters} (allocating: {i0.outer_iters}), y difference {d:.2e}, "
            f"bitwise {bool(torch.equal(y1, y0))}")
        assert i1.status == i0.status == (msb.REDUCED_ACCURACY if flags & msb.MIXED else msb.OK)
        assert np.array_equal(i1.shift_iters, i0.shift_iters)
        assert i1.mv_count == i0.mv_count
        assert d <= 1e-12
        if want:
            dx = float(torch.linalg.vector_norm(x1 - x0) / torch.linalg.vector_norm(x0))
            log(f"  x_shifts difference {dx:.2e}")
            assert dx <= 1e-12
        del y0, y1, x0, x1


def test_noalloc_refuses_oversized_workspace(setup):
    import torch
    from paper_1010_2592_amd import msb
    wk, U, ctx, a, sig, w, b3, b1 = setup
    y = torch.full_like(b1, 7.0)
    log("noalloc: a double-pass tape larger than the scratch array is refused")
    with pytest.raises(msb.MsbError) as e:
        ctx.mshift_bicgstabl_noalloc(b1, a, sig, w, 4, wk.tol, 4_000_000, 2, y=y)
    assert e.value.status == msb.ERR_ARG
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())          # nothing ran
    with pytest.raises(msb.MsbError):
        ctx.mshift_bicgstabl_noalloc(b1, a, sig, w, 4, wk.tol, 100, 3)
    with pytest.raises(msb.MsbError):
        ctx.mshift_bicgstabl_noalloc(b1, a, sig, w, 4, wk.tol, 100, 2, flags=msb.PERSISTENT)


def test_noalloc_takes_no_device_memory(setup):
    import torch
    from paper_1010_2592_amd import msb
    wk, U, ctx, a, sig, w, b3, b1 = setup
    # every kernel of the call loaded once before the measurement
    ctx.mshift_bicgstabl_noalloc(b3, a, sig, w, 4, wk.tol, 500, 2)
    fresh = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), U)
    y = torch.empty_like(b3)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    _, info, _ = fresh.mshift_bicgstabl_noalloc(b3, a, sig, w, 4, wk.tol, 500, 2, y=y)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    log(f"noalloc on a fresh context: free device memory {free0} -> {free1}, M = {info.outer_iters}")
    fresh.close()
    assert free1 == free0

"""24^3x48 (N_s = 58, l = 2 and 6): the full-size configuration, checked by
properties that hold at any size (the oracle cannot solve this lattice in
seconds).  Every shift's FP64 true residual ||b - (A + sigma_s) x_s|| / ||b||,
formed here with wilson_apply (itself pinned to the oracle element by element
on smaller lattices), meets the tolerance; the double pass reproduces the
single pass; mixed precision with refinement meets the tolerance too.  The
l = 6 single pass keeps N_s (l + 1) = 406 FP64 shift vectors (52 GB).
"""
import numpy as np
import pytest

import workloads as wl
from tests.helpers import cuda, host, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import torch
    from paper_1010_2592_amd import msb
    wk = wl.WORKLOADS["24x24x24x48"]
    log("24x24x24x48: generating links")
    U = cuda(wk.links())
    b = cuda(wk.sources())
    ctx = msb.Context(msb.Lattice(wk.dims, wk.mass, wk.mu, wk.bc_t), U)
    rho = ctx.spectral_radius(cuda(wk.power_start()[None]), 100)
    a = 1.0 / (1.01 * rho)
    sig, w = msb.neuberger_pfe(wk.n_shift)
    log(f"24x24x24x48: spectral radius {rho:.6f}")
    yield wk, ctx, a, sig, w, b
    ctx.close()
    torch.cuda.empty_cache()


def true_residuals(ctx, a, sig, b, xs):
    """||b - (a (g5 D)^2 + sigma_s) x_s|| / ||b|| for x_s = xs[0, s] (FP64)."""
    import torch
    from paper_1010_2592_amd import msb
    x = xs[0]                                   # [N_s][12][V]
    t = ctx.wilson_apply(x, msb.G5_LEFT)
    t = ctx.wilson_apply(t, msb.G5_LEFT)
    s = torch.as_tensor(sig, dtype=torch.float64, device=x.device).view(-1, 1, 1)
    r = b[0].unsqueeze(0) - (a * t + s * x)
    return (torch.linalg.vector_norm(r.reshape(len(sig), -1), dim=1) / torch.linalg.vector_norm(b[0])).cpu().numpy()


@pytest.mark.parametrize("l", [2, 6])
def test_full_size_single_and_double_pass(big, l):
    import torch
    wk, ctx, a, sig, w, b = big
    log(f"24x24x24x48 l={l}: single pass FP64")
    y1, i1, xs = ctx.mshift_bicgstabl(b, a, sig, w, l, wk.tol, 3000, 1, want_shifts=True)
    tr = true_residuals(ctx, a, sig, b, xs)
    log(f"  M = {i1.outer_iters}, max true residual {tr.max():.3e}, max collinear {i1.shift_resid.max():.3e}")
    assert tr.max() <= wk.tol
    del xs
    torch.cuda.empty_cache()
    log(f"24x24x24x48 l={l}: double pass FP64")
    y2, i2, _ = ctx.mshift_bicgstabl(b, a, sig, w, l, wk.tol, 3000, 2)
    d = float(torch.linalg.vector_norm(y2 - y1) / torch.linalg.vector_norm(y1))
    log(f"  double vs single pass: {d:.3e}, Mv {i2.mv_count} = 2 x {i1.mv_count}")
    assert d <= 1e-10
    assert i2.mv_count == 2 * i1.mv_count
    assert np.array_equal(i1.shift_iters, i2.shift_iters)


def test_full_size_mixed_refined(big):
    import torch
    from paper_1010_2592_amd import msb
    wk, ctx, a, sig, w, b = big
    log("24x24x24x48 l=2: mixed + refine")
    y64, _, _ = ctx.mshift_bicgstabl(b, a, sig, w, 2, wk.tol, 3000, 1)
    ym, im, xs = ctx.mshift_bicgstabl(b, a, sig, w, 2, wk.tol, 3000, 1, flags=msb.MIXED | msb.REFINE,
                                      want_shifts=True)
    tr = true_residuals(ctx, a, sig, b, xs)
    d = float(torch.linalg.vector_norm(ym - y64) / torch.linalg.vector_norm(y64))
    log(f"  refined {im.refined_shifts} shifts, max true residual {tr.max():.3e} "
        f"(library {im.shift_true_resid.max():.3e}), y vs FP64 {d:.3e}")
    assert tr.max() <= wk.tol
    assert d <= 1e-6

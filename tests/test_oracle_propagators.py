"""Pins of multi-mass Wilson propagators on the oracle: the multi-shift
solver with A = D_w(m) reaches x_s = D_w(m + sigma_s)^{-1} b for every mass
from one Krylov space (shift structure of the Wilson mass term).

  * D_w(m + sigma) == D_w(m) + sigma, densely (the premise);
  * each x_s == a dense solve with D_w(m_s), at mu = 0 and mu != 0;
  * single, double and pseudo-double pass give the same sum.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import dirac as od
from oracle import krylov as ok


@pytest.mark.parametrize("mu", [0.0, 0.1])
def test_mass_shift_structure_and_dense_solves(mu):
    dims = (2, 2, 2, 4)
    V = wl.volume(dims)
    U = wl.gauge_links(dims, 0.5, 71)
    m0 = 0.1
    masses = np.array([0.1, 0.2, 0.35, 0.6])
    sig = masses - m0
    D0 = od.dense_dw(U, dims, m0, mu)
    for m, s in zip(masses, sig):
        assert np.abs(od.dense_dw(U, dims, m, mu) - (D0 + s * np.eye(12 * V))).max() <= 1e-14
    op = od.Dirac(U, dims, m0, mu, -1)
    b = wl.gaussian_source(dims, 72)[0]
    y, info, xs = ok.mshift_bicgstabl(op.dw, b, sig, np.ones(4), 2, 1e-12, 500, 1)
    assert info.status == ok.OK
    for s in range(4):
        xd = np.linalg.solve(od.dense_dw(U, dims, masses[s], mu), b.reshape(-1)).reshape(b.shape)
        assert np.linalg.norm(xs[s] - xd) <= 1e-9 * np.linalg.norm(xd), s
    y2 = ok.mshift_bicgstabl(op.dw, b, sig, np.ones(4), 2, 1e-12, 500, 2)[0]
    assert np.linalg.norm(y2 - y) <= 1e-10 * np.linalg.norm(y)


def test_point_source_needs_a_general_shadow_residual():
    """With r~ = b a point source meets BiCG's structural breakdown on D_w
    (every hop changes the site parity, so the odd moments <b, H^k b>
    vanish); a seeded Gaussian r~ (allowed by BiCGstab(l): any r~ with
    <r~, r_0> != 0) gives the dense solutions.  (On a lattice with an
    extent 2 the forward and backward hops meet and the breakdown is absent.)"""
    dims = (4, 4, 4, 4)
    U = wl.gauge_links(dims, 0.5, 78)
    m0 = 0.1
    masses = np.array([0.1, 0.3, 0.7])
    op = od.Dirac(U, dims, m0, 0.05, -1)
    b = wl.point_sources(dims)[4]
    out = ok.mshift_bicgstabl(op.dw, b, masses - m0, np.ones(3), 2, 1e-12, 200, 1)
    assert out[1].status == ok.BREAKDOWN
    shadow = wl.gaussian_source(dims, 79)[0]
    y, info, xs = ok.mshift_bicgstabl(op.dw, b, masses - m0, np.ones(3), 2, 1e-12, 200, 1, shadow=shadow)
    assert info.status == ok.OK
    for s in range(3):
        xd = np.linalg.solve(od.dense_dw(U, dims, masses[s], 0.05), b.reshape(-1)).reshape(b.shape)
        assert np.linalg.norm(xs[s] - xd) <= 1e-9 * np.linalg.norm(xd), s
    # the default is r~ = b
    y0 = ok.mshift_bicgstabl(op.dw, shadow, masses - m0, np.ones(3), 2, 1e-10, 200, 1)[0]
    y1 = ok.mshift_bicgstabl(op.dw, shadow, masses - m0, np.ones(3), 2, 1e-10, 200, 1, shadow=shadow)[0]
    assert np.array_equal(y0, y1)

"""Pins of the oracle's backward pass (gradients of Re <eta, f(A) b>).

The gradients are checked against central finite differences of the forward
definition computed with DENSE solves on a 2^4 lattice (no iteration noise,
O(h^2) error), against the adjoint identity <eta, F b> = <F^+ eta, b> with
F^+ from solves at -mu, and against gauge covariance of the link gradient.
A sign, conjugation, transposition or boundary-phase error in the link force
fails the finite differences at O(1)."""
import numpy as np
import pytest

import workloads as wl
from oracle import backward as ob
from oracle import dirac as od
from oracle import krylov as ok
from oracle import pfe

DIMS = (2, 2, 2, 2)
MU = 0.13


def setup(seed=5, mu=MU):
    U = wl.gauge_links(DIMS, 0.6, seed)
    op = od.Dirac(U, DIMS, -2.0, mu, -1)
    rho = od.spectral_radius(op, wl.start_vector(DIMS, seed + 1), 200)
    a = od.a_scale_from_radius(rho)
    b = wl.gaussian_source(DIMS, seed + 2)[0]
    eta = wl.gaussian_source(DIMS, seed + 3)[0]
    sig, w = pfe.neuberger(6)
    return U, op, a, b, eta, sig, w


def dense_loss(U, a, b, eta, sig, w, mode=0, mu=MU):
    V = wl.volume(DIMS)
    D = od.dense_dw(U, DIMS, -2.0, mu, -1)
    H = od.dense_g5(V) @ D
    A = a * H @ H
    I = np.eye(A.shape[0])
    y = sum(w[s] * np.linalg.solve(A + sig[s] * I, b.reshape(-1)) for s in range(len(sig)))
    if mode == 1:
        y = np.sqrt(a) * H @ y
    return float(np.vdot(eta.reshape(-1), y).real)


@pytest.mark.parametrize("mode", [0, 1])
def test_gradients_against_dense_finite_differences(mode):
    U, op, a, b, eta, sig, w = setup()
    gb, gw, gs, GU = ob.fab_backward(op, a, b, eta, sig, w, 2, 1e-13, 5000, mode)
    h = 1e-6
    rng = np.random.default_rng(11)
    L = lambda **kw: dense_loss(kw.get("U", U), a, kw.get("b", b), eta, kw.get("sig", sig),
                                kw.get("w", w), mode)
    # b: a few Re and Im components
    for _ in range(4):
        k, v = rng.integers(12), rng.integers(wl.volume(DIMS))
        for unit, part in ((1.0, "re"), (1j, "im")):
            db = np.zeros_like(b)
            db[k, v] = unit * h
            fd = (L(b=b + db) - L(b=b - db)) / (2 * h)
            an = gb[k, v].real if part == "re" else gb[k, v].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    # weights and shifts
    for s in range(len(sig)):
        e = np.zeros(len(sig))
        e[s] = h
        fd = (L(w=w + e) - L(w=w - e)) / (2 * h)
        assert abs(fd - gw[s]) <= 1e-6 * max(1.0, abs(gw[s]))
        e[s] = h * max(sig[s], 1e-3)
        fd = (L(sig=sig + e) - L(sig=sig - e)) / (2 * e[s])
        assert abs(fd - gs[s]) <= 1e-5 * max(1.0, abs(gs[s]))
    # links: random complex directions (not SU(3): the gradient is the
    # unconstrained complex one) -- dL = Re sum conj(G) dU
    for _ in range(3):
        dU = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
        fd = (L(U=U + h * dU) - L(U=U - h * dU)) / (2 * h)
        an = float(np.sum(GU.conj() * dU).real)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_adjoint_identity():
    U, op, a, b, eta, sig, w = setup(21)
    yF = ok.mshift_bicgstabl(lambda v: op.a_op(v, a), b, sig, w, 2, 1e-13, 5000, 1)[0]
    yA = ok.mshift_bicgstabl(lambda v: op.a_op(v, a, -MU), eta, sig, w, 2, 1e-13, 5000, 1)[0]
    lhs, rhs = np.vdot(eta, yF), np.vdot(yA, b)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_link_gradient_gauge_covariance():
    U, op, a, b, eta, sig, w = setup(31)
    V = wl.volume(DIMS)
    Lx, Ly, Lz, Lt = DIMS
    g = wl.gauge_links(DIMS, 1.1, 77)[0]
    idx = np.arange(V).reshape(Lt, Lz, Ly, Lx)
    Ug = np.empty_like(U)
    fwd = []
    for nu in range(4):
        f = np.roll(idx, -1, axis=3 - nu).reshape(-1)
        fwd.append(f)
        Ug[nu] = np.einsum("abx,bcx,dcx->adx", g, U[nu], g[:, :, f].conj())

    def G(v):
        return np.einsum("abx,sbx->sax", g, v.reshape(4, 3, V)).reshape(12, V)

    _, _, _, GU = ob.fab_backward(op, a, b, eta, sig, w, 2, 1e-13, 5000)
    opg = od.Dirac(Ug, DIMS, -2.0, MU, -1)
    _, _, _, GUg = ob.fab_backward(opg, a, G(b), G(eta), sig, w, 2, 1e-13, 5000)
    for nu in range(4):
        expect = np.einsum("abx,bcx,dcx->adx", g, GU[nu], g[:, :, fwd[nu]].conj())
        assert np.allclose(GUg[nu], expect, atol=1e-8 * np.abs(GU).max())

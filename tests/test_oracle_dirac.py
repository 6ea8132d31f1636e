"""Pins of the oracle's Dirac operator against what the mathematics fixes.

D_w(mu) itself is only named in the paper (Section 1); these tests pin the
oracle's statement of it to: the Clifford algebra of the gamma matrices, an
independent dense construction by explicit site loops, free-field plane waves
(closed form), gamma5-hermiticity at mu = 0, D(mu)^+ = gamma5 D(-mu) gamma5,
and gauge covariance.  A dropped hop, a wrong projector sign, a transposed
link or a misplaced boundary sign fails at least one of them.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import dirac as od

RNG = np.random.default_rng(7)


def rand_spinor(V, rng=RNG):
    return rng.standard_normal((12, V)) + 1j * rng.standard_normal((12, V))


def test_gamma_clifford_and_gamma5():
    g = od.GAMMA
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            ac = g[a] @ g[b] + g[b] @ g[a]
            assert np.allclose(ac, 2.0 * (a == b) * np.eye(4), atol=1e-15)
    assert np.allclose(od.GAMMA5, np.diag([1, 1, -1, -1]))
    for a in range(4):
        assert np.allclose(od.GAMMA5 @ g[a], -g[a] @ od.GAMMA5)


def test_links_are_su3():
    U = wl.gauge_links((2, 2, 2, 4), 0.6, 11)
    M = np.transpose(U, (0, 3, 1, 2)).reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.allclose(np.einsum("nij,nkj->nik", M, M.conj()), eye, atol=1e-13)
    assert np.allclose(np.linalg.det(M), 1.0, atol=1e-13)
    # eps -> 0 is the free field
    U0 = wl.gauge_links((2, 2, 2, 4), 0.0, 11)
    assert np.allclose(U0, wl.free_links((2, 2, 2, 4)))


@pytest.mark.parametrize("dims,mu,bc", [((2, 2, 2, 2), 0.3, -1),
                                        ((2, 2, 2, 4), 0.17, -1),
                                        ((2, 2, 4, 2), 0.0, 1),
                                        ((3, 2, 2, 4), 0.05, -1)])
def test_stencil_equals_dense_site_loops(dims, mu, bc):
    V = wl.volume(dims)
    U = wl.gauge_links(dims, 0.8, 5 + V)
    op = od.Dirac(U, dims, -2.0, mu, bc)
    D = od.dense_dw(U, dims, -2.0, mu, bc)
    for _ in range(3):
        v = rand_spinor(V)
        assert np.allclose(op.dw(v), (D @ v.reshape(-1)).reshape(12, V), atol=1e-13)


def test_free_field_plane_waves():
    """D e^{ipx} chi = e^{ipx} [(4+m - sum cos q) + i sum gamma sin q] chi,
    q_nu = p_nu - i mu delta_{nu4}, antiperiodic momenta in time."""
    dims = (4, 4, 4, 8)
    Lx, Ly, Lz, Lt = dims
    V = wl.volume(dims)
    m, mu = -2.0, 0.05
    op = od.Dirac(wl.free_links(dims), dims, m, mu, -1)
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    coords = [x.reshape(-1), y.reshape(-1), z.reshape(-1), t.reshape(-1)]
    rng = np.random.default_rng(3)
    for n in [(0, 0, 0, 0), (1, 0, 2, 3), (3, 1, 1, 7), (2, 2, 2, 4)]:
        p = [2 * np.pi * n[0] / Lx, 2 * np.pi * n[1] / Ly, 2 * np.pi * n[2] / Lz,
             np.pi * (2 * n[3] + 1) / Lt]
        q = np.array(p, dtype=np.complex128)
        q[3] -= 1j * mu
        phase = np.exp(1j * sum(p[k] * coords[k] for k in range(4)))
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        M = (4 + m - np.sum(np.cos(q))) * np.eye(4) + 1j * sum(od.GAMMA[k] * np.sin(q[k])
                                                               for k in range(4))
        v = (chi.reshape(12, 1) * phase[None, :])
        expect = ((M @ chi).reshape(12, 1) * phase[None, :])
        assert np.allclose(op.dw(v), expect, atol=1e-12)
        # A = a H^2 is the scalar a[(4+m-sum cos q)^2 + sum sin^2 q] on the wave
        a = 0.37
        lam = a * ((4 + m - np.sum(np.cos(q))) ** 2 + np.sum(np.sin(q) ** 2))
        assert np.allclose(op.a_op(v, a), lam * v, atol=1e-12)


def test_gamma5_hermiticity_at_zero_mu():
    dims = (4, 4, 4, 8)
    V = wl.volume(dims)
    op = od.Dirac(wl.gauge_links(dims, 0.6, 1001), dims, -2.0, 0.0, -1)
    phi, psi = rand_spinor(V), rand_spinor(V)
    lhs = np.vdot(phi, op.h(psi))
    rhs = np.vdot(op.h(phi), psi)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_is_gamma5_minus_mu_gamma5():
    # dense form on a tiny lattice ...
    dims = (2, 2, 2, 4)
    V = wl.volume(dims)
    U = wl.gauge_links(dims, 0.7, 77)
    D = od.dense_dw(U, dims, -2.0, 0.21, -1)
    Dm = od.dense_dw(U, dims, -2.0, -0.21, -1)
    G5 = od.dense_g5(V)
    assert np.allclose(D.conj().T, G5 @ Dm @ G5, atol=1e-14)
    # ... and the dot-product test on a production-shaped lattice
    dims = (4, 4, 4, 8)
    V = wl.volume(dims)
    op = od.Dirac(wl.gauge_links(dims, 0.6, 1001), dims, -2.0, 0.05, -1)
    phi, psi = rand_spinor(V), rand_spinor(V)
    lhs = np.vdot(phi, op.dw(psi))
    rhs = np.vdot(op.dw_dag(phi), psi)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # H(mu)^+ = H(-mu)
    lhs = np.vdot(phi, op.h(psi))
    rhs = np.vdot(op.h(phi, -0.05), psi)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gauge_covariance():
    dims = (4, 2, 2, 4)
    V = wl.volume(dims)
    Lx, Ly, Lz, Lt = dims
    U = wl.gauge_links(dims, 0.6, 9)
    g = wl.gauge_links(dims, 1.3, 10)[0]          # one SU(3) matrix per site
    # U^g_nu(x) = g(x) U_nu(x) g(x + nu)^+
    idx = np.arange(V).reshape(Lt, Lz, Ly, Lx)
    Ug = np.empty_like(U)
    for nu in range(4):
        ax = 3 - nu
        fwd = np.roll(idx, -1, axis=ax).reshape(-1)
        Ug[nu] = np.einsum("abx,bcx,dcx->adx", g, U[nu], g[:, :, fwd].conj())
    op = od.Dirac(U, dims, -2.0, 0.11, -1)
    opg = od.Dirac(Ug, dims, -2.0, 0.11, -1)

    def G(v):  # (G v)(x) = g(x) v(x) in colour
        w = v.reshape(4, 3, V)
        return np.einsum("abx,sbx->sax", g, w).reshape(12, V)

    def Gdag(v):
        w = v.reshape(4, 3, V)
        return np.einsum("bax,sbx->sax", g.conj(), w).reshape(12, V)

    v = rand_spinor(V)
    assert np.allclose(opg.dw(v), G(op.dw(Gdag(v))), atol=1e-12)


def test_spectral_radius_estimate_bounds_dense():
    dims = (2, 2, 2, 4)
    V = wl.volume(dims)
    U = wl.gauge_links(dims, 0.6, 21)
    op = od.Dirac(U, dims, -2.0, 0.05, -1)
    D = od.dense_dw(U, dims, -2.0, 0.05, -1)
    lam_max = np.linalg.eigvalsh(D.conj().T @ D).max()
    est = od.spectral_radius(op, wl.start_vector(dims, 4000), 300)
    assert est <= lam_max * (1 + 1e-12)
    assert est >= 0.97 * lam_max
    # a (g5 D)^2 then has spectral radius below one
    a = od.a_scale_from_radius(lam_max)
    G5 = od.dense_g5(V)
    H = G5 @ D
    assert np.abs(np.linalg.eigvals(a * H @ H)).max() < 1.0


def test_vector_sizes_match_paper():
    """Section 2 quotes 50 kB (4^4) and 800 kB (8^4) per vector, Section 3
    100 kB (4^3x8): 12 complex128 numbers per site."""
    import json
    import os
    facts = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))
    for row in facts["vector_sizes"]:
        V = wl.volume(row["dims"])
        nbytes = 12 * 16 * V
        assert abs(nbytes - row["kB"] * 1000) <= 0.03 * row["kB"] * 1000 or \
            abs(nbytes - row["kB"] * 1024) <= 0.03 * row["kB"] * 1024

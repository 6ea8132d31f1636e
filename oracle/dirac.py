"""Wilson-Dirac operator with chemical potential, written out plainly.

Test infrastructure only (see ``oracle/__init__.py``).

The paper uses D_w(mu) without writing it out (Section 1, after Eq. (1.1));
this file takes the standard Wilson discretisation with the chemical potential
on the time links (Hasenfratz-Karsch form):

  (D psi)(x) = (4 + m) psi(x)
      - 1/2 sum_nu b_nu(x)      (1 - gamma_nu) e^{+mu d_nu4} U_nu(x)       psi(x + nu)
      - 1/2 sum_nu b_nu(x - nu) (1 + gamma_nu) e^{-mu d_nu4} U_nu(x - nu)^+ psi(x - nu)

with b_4(x) = bc_t on the time-wrapping links (t = Lt-1 -> 0) and 1 elsewhere
(periodic in space).  Gamma matrices are the chiral basis

  gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],  gamma_4 = [[0, 1], [1, 0]],
  gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1).

From it: H = gamma_5 D_w(mu) (non-Hermitian for mu != 0, Section 1),
A = a H^2 with a = 1 / (estimated spectral radius), the seed matrix
S = A + sigma_0, and the sign function sign(H) b = sqrt(a) H f(A) b with
f(A) = A^{-1/2} (Section 1, text after Eq. (1.2)).

Fields are handled on the 4D grid: spinors (Lt, Lz, Ly, Lx, 4, 3), links
(4, Lt, Lz, Ly, Lx, 3, 3).  ``to_grid`` / ``from_grid`` convert from and to the
boundary layouts ([12][V] spinors with k = 3*spin + colour, [4][3][3][V]
links, site = x + Lx*(y + Ly*(z + Lz*t))).
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# gamma matrices
# --------------------------------------------------------------------------

_PAULI = np.array([[[0, 1], [1, 0]],
                   [[0, -1j], [1j, 0]],
                   [[1, 0], [0, -1]]], dtype=np.complex128)


def gamma_matrices() -> np.ndarray:
    """gamma_1..gamma_4 of the chiral basis, shape (4, 4, 4)."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    for k in range(3):
        g[k, 0:2, 2:4] = -1j * _PAULI[k]
        g[k, 2:4, 0:2] = 1j * _PAULI[k]
    g[3, 0:2, 2:4] = np.eye(2)
    g[3, 2:4, 0:2] = np.eye(2)
    return g


GAMMA = gamma_matrices()
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

# --------------------------------------------------------------------------
# layouts
# --------------------------------------------------------------------------


def spinor_to_grid(v: np.ndarray, dims) -> np.ndarray:
    """[12][V] -> (Lt, Lz, Ly, Lx, 4, 3)."""
    Lx, Ly, Lz, Lt = dims
    g = v.reshape(4, 3, Lt, Lz, Ly, Lx)
    return np.ascontiguousarray(np.transpose(g, (2, 3, 4, 5, 0, 1)))


def spinor_from_grid(g: np.ndarray) -> np.ndarray:
    """(Lt, Lz, Ly, Lx, 4, 3) -> [12][V]."""
    return np.ascontiguousarray(np.transpose(g, (4, 5, 0, 1, 2, 3))).reshape(12, -1)


def links_to_grid(U: np.ndarray, dims) -> np.ndarray:
    """[4][3][3][V] -> (4, Lt, Lz, Ly, Lx, 3, 3)."""
    Lx, Ly, Lz, Lt = dims
    g = U.reshape(4, 3, 3, Lt, Lz, Ly, Lx)
    return np.ascontiguousarray(np.transpose(g, (0, 3, 4, 5, 6, 1, 2)))


def links_from_grid(g: np.ndarray) -> np.ndarray:
    """(4, Lt, Lz, Ly, Lx, 3, 3) -> [4][3][3][V]."""
    return np.ascontiguousarray(np.transpose(g, (0, 5, 6, 1, 2, 3, 4))).reshape(4, 3, 3, -1)


def _axis(nu: int) -> int:
    # grid axes are (t, z, y, x); direction nu = 0..3 is x, y, z, t
    return 3 - nu


def _spin_mul(gm: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(gm psi)[..., s, a] = sum_t gm[s, t] psi[..., t, a]."""
    return np.einsum("st,...ta->...sa", gm, psi)


def _colour_mul(U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U psi)[..., s, a] = sum_b U[..., a, b] psi[..., s, b]."""
    return np.einsum("...ab,...sb->...sa", U, psi)


def _colour_mul_dag(U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U^+ psi)[..., s, a] = sum_b conj(U[..., b, a]) psi[..., s, b]."""
    return np.einsum("...ba,...sb->...sa", U.conj(), psi)


def time_sign(dims, bc_t: int) -> np.ndarray:
    """b_4(x) on the grid, shape (Lt, 1, 1, 1, 1, 1): bc_t on t = Lt-1."""
    Lt = dims[3]
    b = np.ones((Lt, 1, 1, 1, 1, 1))
    b[Lt - 1] = bc_t
    return b

# --------------------------------------------------------------------------
# the operator
# --------------------------------------------------------------------------


class Dirac:
    """D_w(mu) on a fixed gauge field.  All arithmetic in complex128."""

    def __init__(self, links: np.ndarray, dims, mass: float, mu: float,
                 bc_t: int = -1):
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.mass = float(mass)
        self.mu = float(mu)
        self.bc_t = int(bc_t)
        self.U = links_to_grid(np.asarray(links, dtype=np.complex128), self.dims)
        self.bt = time_sign(self.dims, self.bc_t)

    # -- grid-level operator ------------------------------------------------
    def dw_grid(self, psi: np.ndarray, mu: float | None = None) -> np.ndarray:
        mu = self.mu if mu is None else mu
        out = (4.0 + self.mass) * psi
        for nu in range(4):
            ax = _axis(nu)
            # forward hop: b_nu(x) (1 - gamma_nu) e^{mu d} U_nu(x) psi(x + nu)
            hop = _colour_mul(self.U[nu], np.roll(psi, -1, axis=ax))
            term = hop - _spin_mul(GAMMA[nu], hop)
            if nu == 3:
                term = term * (self.bt * np.exp(mu))
            out = out - 0.5 * term
            # backward hop: b_nu(x-nu) (1 + gamma_nu) e^{-mu d} U_nu(x-nu)^+ psi(x - nu)
            hop = _colour_mul_dag(np.roll(self.U[nu], 1, axis=ax),
                                  np.roll(psi, 1, axis=ax))
            term = hop + _spin_mul(GAMMA[nu], hop)
            if nu == 3:
                term = term * (np.roll(self.bt, 1, axis=0) * np.exp(-mu))
            out = out - 0.5 * term
        return out

    # -- boundary-layout wrappers ([12][V]) ---------------------------------
    def dw(self, v: np.ndarray, mu: float | None = None) -> np.ndarray:
        """D_w(mu) v for v in [12][V] layout."""
        g = spinor_to_grid(np.asarray(v, dtype=np.complex128), self.dims)
        return spinor_from_grid(self.dw_grid(g, mu))

    def dw_dag(self, v: np.ndarray) -> np.ndarray:
        """D_w(mu)^+ v, written as gamma5 D_w(-mu) gamma5 v."""
        return g5(self.dw(g5(v), -self.mu))

    def h(self, v: np.ndarray, mu: float | None = None) -> np.ndarray:
        """H v = gamma5 D_w(mu) v."""
        return g5(self.dw(v, mu))

    def a_op(self, v: np.ndarray, a_scale: float, mu: float | None = None) -> np.ndarray:
        """A v = a (gamma5 D_w)^2 v."""
        return a_scale * self.h(self.h(v, mu), mu)

    def seed_op(self, a_scale: float, sigma0: float, mu: float | None = None):
        """The seed matrix S = A + sigma0 as a callable on [12][V] vectors."""
        def mv(v):
            return self.a_op(v, a_scale, mu) + sigma0 * v
        return mv


def g5(v: np.ndarray) -> np.ndarray:
    """gamma5 on a [12][V] (or [nrhs][12][V]) spinor, spin index = k // 3."""
    v = np.asarray(v)
    shp = v.shape
    w = v.reshape(shp[:-2] + (4, 3, shp[-1]))
    w = np.einsum("st,...tav->...sav", GAMMA5, w)
    return w.reshape(shp)


def spectral_radius(op: Dirac, start: np.ndarray, iters: int = 100) -> float:
    """Estimate of lambda_max(D^+ D) by power iteration from ``start``.

    Returns the Rayleigh quotient <v, D^+D v>/<v, v> after ``iters``
    normalised power steps.  The library's scale convention is
    a_scale = 1 / (1.01 * spectral_radius), so that a (gamma5 D)^2 has
    spectral radius below one.
    """
    v = np.asarray(start, dtype=np.complex128)
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = op.dw_dag(op.dw(v))
        lam = float(np.vdot(v, w).real)
        v = w / np.linalg.norm(w)
    return lam


def a_scale_from_radius(rho: float) -> float:
    return 1.0 / (1.01 * rho)

# --------------------------------------------------------------------------
# dense matrices (tiny lattices), built by explicit site loops
# --------------------------------------------------------------------------


def dense_dw(links: np.ndarray, dims, mass: float, mu: float, bc_t: int = -1) -> np.ndarray:
    """Dense D_w(mu) in the [12][V] index order (row/col = k*V + s).

    Built entry by entry with explicit coordinate arithmetic -- a second,
    independent statement of the operator used to check ``Dirac.dw``.
    """
    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    L = (Lx, Ly, Lz, Lt)
    U = np.asarray(links, dtype=np.complex128)
    D = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    eye4 = np.eye(4)

    def idx(c):
        return c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]))

    def block(row_site, col_site, M):
        # M is (4*3, 4*3) in (spin, colour) order -> scatter into k*V + s
        for k1 in range(12):
            for k2 in range(12):
                D[k1 * V + row_site, k2 * V + col_site] += M[k1, k2]

    for t in range(Lt):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    c = [x, y, z, t]
                    s = idx(c)
                    block(s, s, (4.0 + mass) * np.eye(12))
                    for nu in range(4):
                        cf = list(c)
                        cf[nu] = (c[nu] + 1) % L[nu]
                        cb = list(c)
                        cb[nu] = (c[nu] - 1) % L[nu]
                        sf, sb = idx(cf), idx(cb)
                        # forward
                        bf = bc_t if (nu == 3 and c[3] == Lt - 1) else 1.0
                        ef = np.exp(mu) if nu == 3 else 1.0
                        Uf = U[nu, :, :, s]
                        block(s, sf, -0.5 * bf * ef * np.kron(eye4 - GAMMA[nu], Uf))
                        # backward
                        bb = bc_t if (nu == 3 and cb[3] == Lt - 1) else 1.0
                        eb = np.exp(-mu) if nu == 3 else 1.0
                        Ub = U[nu, :, :, sb].conj().T
                        block(s, sb, -0.5 * bb * eb * np.kron(eye4 + GAMMA[nu], Ub))
    return D


def dense_g5(V: int) -> np.ndarray:
    """Dense gamma5 in the [12][V] index order."""
    return np.kron(GAMMA5, np.eye(3 * V))

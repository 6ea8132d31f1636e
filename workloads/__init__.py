"""Seeded synthetic inputs for the multi-shift BiCGstab(l) workloads.

This module only *generates inputs*: SU(3) gauge links, Gaussian and point
sources, and the start vector of the spectral-radius estimate.  It holds none
of the solver's arithmetic and is the one module that both the HIP path and
the CPU oracle draw their inputs from.

Stand-in for the paper's gauge ensembles (beta=5.32 on 4^3x8 and beta=5.71 on
12^3x24, Sections 3-4), which are not available: links are U = exp(i*eps*H)
with H = sum_a h_a lambda_a / 2, h_a ~ N(0, 1) iid (lambda_a the Gell-Mann
matrices), one independent draw per link.  eps -> 0 gives the free field.

Layouts (the library boundary's layouts):
  * site index  s = x + Lx*(y + Ly*(z + Lz*t)), dims = (Lx, Ly, Lz, Lt)
  * spinor      [nrhs][k][s] complex128 with k = 3*spin + colour (12 per site)
  * links       [nu][a][b][s] complex128, nu = 0..3 for x, y, z, t
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "volume", "gauge_links", "free_links",
    "gaussian_source", "point_sources", "start_vector", "gell_mann",
]


def volume(dims) -> int:
    Lx, Ly, Lz, Lt = dims
    return int(Lx * Ly * Lz * Lt)


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7] = np.diag([1.0, 1.0, -2.0]) / np.sqrt(3.0)
    return lam


def gauge_links(dims, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) links U = exp(i eps H), H Gaussian traceless Hermitian.

    Returns complex128 array of shape (4, 3, 3, V).  The exponential is taken
    through the eigendecomposition of the Hermitian H, so U is unitary with
    det U = exp(i eps tr H) = 1 up to rounding.
    """
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal((4, V, 8))
    lam = gell_mann()
    out = np.empty((4, 3, 3, V), dtype=np.complex128)
    chunk = 1 << 16
    for nu in range(4):
        for s0 in range(0, V, chunk):
            s1 = min(V, s0 + chunk)
            H = np.einsum("na,aij->nij", h[nu, s0:s1], lam) * 0.5
            w, Q = np.linalg.eigh(H)
            U = np.einsum("nij,nj,nkj->nik", Q, np.exp(1j * eps * w), Q.conj())
            out[nu, :, :, s0:s1] = np.transpose(U, (1, 2, 0))
    return out


def free_links(dims) -> np.ndarray:
    """Unit links (the free field), shape (4, 3, 3, V)."""
    V = volume(dims)
    out = np.zeros((4, 3, 3, V), dtype=np.complex128)
    for a in range(3):
        out[:, a, a, :] = 1.0
    return out


def gaussian_source(dims, seed: int, nrhs: int = 1) -> np.ndarray:
    """b with Re and Im iid N(0,1), shape (nrhs, 12, V) complex128."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal((nrhs, 12, V))
    im = rng.standard_normal((nrhs, 12, V))
    return re + 1j * im


def point_sources(dims) -> np.ndarray:
    """The 12 spin-colour point sources at the origin: b_k = e_{s=0, k}."""
    V = volume(dims)
    b = np.zeros((12, 12, V), dtype=np.complex128)
    for k in range(12):
        b[k, k, 0] = 1.0
    return b


def start_vector(dims, seed: int) -> np.ndarray:
    """Start vector of the power iteration for the spectral radius, (12, V)."""
    return gaussian_source(dims, seed, 1)[0]


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: lattice, gauge draw, PFE size, l, sources."""
    name: str
    dims: Tuple[int, int, int, int]
    eps: float
    mu: float
    n_shift: int
    ells: Tuple[int, ...]
    source: str                 # "gaussian" or "point"
    gauge_seed: int
    source_seed: int = 0
    eta_seed: int = 0
    power_seed: int = 0
    mass: float = -2.0
    bc_t: int = -1              # antiperiodic in time, periodic in space
    tol: float = 1e-8
    extra: dict = field(default_factory=dict)

    @property
    def volume(self) -> int:
        return volume(self.dims)

    def links(self) -> np.ndarray:
        return gauge_links(self.dims, self.eps, self.gauge_seed)

    def sources(self) -> np.ndarray:
        if self.source == "point":
            return point_sources(self.dims)
        return gaussian_source(self.dims, self.source_seed, 1)

    def eta(self) -> np.ndarray:
        return gaussian_source(self.dims, self.eta_seed, 1)

    def power_start(self) -> np.ndarray:
        return start_vector(self.dims, self.power_seed)


# The five synthetic workloads (lattice shapes of the paper's Sections 3-4).
WORKLOADS = {
    "4x4x4x8": Workload("4x4x4x8", (4, 4, 4, 8), 0.6, 0.05, 10, (2,),
                        "gaussian", 1001, source_seed=2001, power_seed=4001),
    "8x8x8x8": Workload("8x8x8x8", (8, 8, 8, 8), 0.6, 0.1, 20, (4,),
                        "gaussian", 1002, source_seed=2002, power_seed=4002),
    "16x16x16x32": Workload("16x16x16x32", (16, 16, 16, 32), 0.5, 0.05, 30,
                            (4,), "point", 1003, power_seed=4003),
    "24x24x24x48": Workload("24x24x24x48", (24, 24, 24, 48), 0.5, 0.05, 58,
                            (2, 6), "gaussian", 1004, source_seed=2004,
                            power_seed=4004),
    "8x8x8x8-backward": Workload("8x8x8x8-backward", (8, 8, 8, 8), 0.6, 0.05,
                                 20, (4,), "gaussian", 1005, source_seed=2005,
                                 eta_seed=3005, power_seed=4005),
}

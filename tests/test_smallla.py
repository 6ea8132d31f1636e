"""The eigensolver's host-side small dense linear algebra (Cholesky,
triangular inverse, Jacobi Hermitian eigensolver), built with g++ from the
library's header and checked against numpy / the defining identities."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1010_2592_amd", "csrc")


@pytest.fixture(scope="module")
def prog(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("smallla") / "smallla_check")
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "smallla_check.cpp"), "-o", exe],
                   check=True)
    return exe


def run(exe, op, A):
    m = A.shape[0]
    cols = A.reshape(-1, order="F")
    text = f"{op} {m}\n" + "\n".join(f"{float(z.real):.17g} {float(z.imag):.17g}" for z in cols) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    return [ln for ln in out if ln]


def as_matrix(lines, m):
    v = np.array([complex(*map(float, ln.split())) for ln in lines])
    return v.reshape((m, m), order="F")


def herm(rng, m, cond=None):
    Z = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    if cond is None:
        return Z @ Z.conj().T + m * np.eye(m)
    Q, _ = np.linalg.qr(Z)
    s = np.logspace(0, -np.log10(cond), m)
    return (Q * s) @ Q.conj().T


@pytest.mark.parametrize("m", [1, 5, 20, 33])
def test_cholesky_and_inverse(prog, m):
    rng = np.random.default_rng(m)
    G = herm(rng, m)
    R = as_matrix(run(prog, "chol", G), m)
    assert np.allclose(np.tril(R, -1), 0)
    assert np.all(np.diag(R).real > 0) and np.allclose(np.diag(R).imag, 0)
    assert np.abs(R.conj().T @ R - G).max() <= 1e-13 * np.abs(G).max()
    assert np.allclose(R, np.linalg.cholesky(G).conj().T, rtol=0, atol=1e-12 * np.abs(R).max())
    Ri = as_matrix(run(prog, "inv", R), m)
    assert np.allclose(np.tril(Ri, -1), 0)
    assert np.abs(Ri @ R - np.eye(m)).max() <= 1e-12


def test_cholesky_rejects_indefinite(prog):
    A = np.diag([1.0, -1.0, 2.0]).astype(complex)
    assert run(prog, "chol", A) == ["FAIL"]


@pytest.mark.parametrize("m,cond", [(1, None), (2, None), (7, None), (20, 1e12), (32, None), (40, 1e6)])
def test_jacobi_eigen(prog, m, cond):
    rng = np.random.default_rng(100 + m)
    A = herm(rng, m, cond)
    if cond is None:
        A = A - 2 * m * np.eye(m)                       # indefinite
    out = run(prog, "eig", A)
    sweeps = int(out[0])
    assert 0 <= sweeps < 60
    w = np.array([float(x) for x in out[1:1 + m]])
    Q = as_matrix(out[1 + m:], m)
    ref = np.linalg.eigvalsh(A)
    nrm = np.abs(ref).max()
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - ref).max() <= 1e-13 * nrm
    assert np.abs(Q.conj().T @ Q - np.eye(m)).max() <= 1e-13
    assert np.abs(A @ Q - Q * w).max() <= 1e-13 * nrm


def test_jacobi_degenerate_and_diagonal(prog):
    rng = np.random.default_rng(7)
    Z = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    Q0, _ = np.linalg.qr(Z)
    A = (Q0 * np.array([-1.0, -1.0, 2.0, 2.0, 2.0, 5.0])) @ Q0.conj().T
    out = run(prog, "eig", A)
    w = np.array([float(x) for x in out[1:7]])
    Q = as_matrix(out[7:], 6)
    assert np.abs(w - [-1, -1, 2, 2, 2, 5]).max() <= 1e-13
    assert np.abs(A @ Q - Q * w).max() <= 1e-13
    D = np.diag([3.0, -2.0, 0.5]).astype(complex)
    out = run(prog, "eig", D)
    assert int(out[0]) == 0
    assert [float(x) for x in out[1:4]] == [-2.0, 0.5, 3.0]

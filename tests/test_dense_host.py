"""Host dense linear algebra of the library (Rayleigh-Ritz problems).

dense.cpp is plain C++; it is compiled here with g++ together with a small
C wrapper and compared with LAPACK (numpy) on symmetric and symmetric-definite
problems, including clustered and repeated eigenvalues and graded matrices.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1909_13585_amd", "csrc")

WRAP = r"""
#include "dense.h"
extern "C" int t_sym_eig(int n, const double* A, double* w, double* V) { return mlb::sym_eig(n, A, w, V) ? 1 : 0; }
extern "C" int t_gen_eig(int n, const double* A, const double* B, double* mu, double* Y) {
    return mlb::gen_eig(n, A, B, mu, Y) ? 1 : 0;
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    d = tmp_path_factory.mktemp("dense")
    wrap = d / "wrap.cpp"
    wrap.write_text(WRAP)
    so = d / "libdense_test.so"
    cmd = ["g++", "-O2", "-shared", "-fPIC", "-std=c++17", "-I", CSRC, str(wrap),
           os.path.join(CSRC, "dense.cpp"), "-o", str(so)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    L = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    L.t_sym_eig.argtypes = [ctypes.c_int, dp, dp, dp]
    L.t_gen_eig.argtypes = [ctypes.c_int, dp, dp, dp, dp]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def sym_eig(L, A):
    n = A.shape[0]
    A = np.ascontiguousarray(A, dtype=np.float64)
    w = np.zeros(n)
    V = np.zeros((n, n))
    ok = L.t_sym_eig(n, _p(A), _p(w), _p(V))
    return ok, w, V


def _cases():
    rng = np.random.default_rng(5)
    out = []
    for n in (1, 2, 3, 7, 18, 54, 96):
        M = rng.standard_normal((n, n))
        out.append(("random", M + M.T))
    # repeated and clustered eigenvalues
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = np.concatenate([np.full(10, 3.0), np.full(10, -1.0), 1.0 + 1e-9 * np.arange(20)])
    out.append(("clustered", (Q * lam) @ Q.T))
    # graded: eigenvalues spanning 1e-12 .. 1
    lam = np.logspace(-12, 0, 30)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    out.append(("graded", (Q * lam) @ Q.T))
    # already diagonal / tridiagonal with zero off-diagonals
    out.append(("diagonal", np.diag(np.arange(12.0)[::-1] - 4)))
    T = np.diag(np.arange(1.0, 9.0)) + np.diag(np.ones(7), 1) + np.diag(np.ones(7), -1)
    T[3, 4] = T[4, 3] = 0.0
    out.append(("split tridiagonal", T))
    out.append(("zero", np.zeros((5, 5))))
    return out


@pytest.mark.parametrize("name,A", _cases(), ids=[c[0] + str(c[1].shape[0]) for c in _cases()])
def test_sym_eig_matches_lapack(lib, name, A):
    ok, w, V = sym_eig(lib, A)
    assert ok
    ref = np.linalg.eigvalsh(A)[::-1]
    scale = max(np.abs(ref).max(), 1e-300)
    n = A.shape[0]
    assert np.all(np.diff(w) <= 0), "eigenvalues must come out descending"
    assert np.abs(w - ref).max() <= 50 * n * 2.2e-16 * scale
    # orthonormal eigenvectors with small residual
    assert np.abs(V.T @ V - np.eye(n)).max() <= 50 * n * 2.2e-16
    assert np.abs(A @ V - V * w).max() <= 50 * n * 2.2e-16 * scale


def test_sym_eig_rejects_non_finite(lib):
    A = np.eye(4)
    A[1, 2] = A[2, 1] = np.nan
    ok, _, _ = sym_eig(lib, A)
    assert not ok


def test_gen_eig_matches_lapack(lib):
    import scipy.linalg as sla
    rng = np.random.default_rng(11)
    for n in (1, 5, 24, 48):
        M = rng.standard_normal((n, n))
        A = M @ M.T + n * np.eye(n)
        B = rng.standard_normal((n, n))
        B = B + B.T
        mu = np.zeros(n)
        Y = np.zeros((n, n))
        assert lib.t_gen_eig(n, _p(np.ascontiguousarray(A)), _p(np.ascontiguousarray(B)), _p(mu), _p(Y))
        ref = sla.eigh(B, A, eigvals_only=True)[::-1]
        assert np.abs(mu - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.abs(Y.T @ A @ Y - np.eye(n)).max() <= 1e-11
        assert np.abs(B @ Y - A @ Y * mu).max() <= 1e-11 * np.abs(B).max() * n


def test_gen_eig_rejects_indefinite_metric(lib):
    A = np.diag([1.0, -1.0, 2.0])
    B = np.eye(3)
    mu = np.zeros(3)
    Y = np.zeros((3, 3))
    assert not lib.t_gen_eig(3, _p(A), _p(B), _p(mu), _p(Y))

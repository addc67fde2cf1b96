"""Pins of the oracle's dense force-solve pre-processing (Sec. 3.2: Cholesky
factor of the Schur complement computed once, its inverse W = L^{-1}, and the
solve f = W^T (W b)).  Closed forms of the 1D Laplacian's factor and inverse,
uniqueness of the factor, reconstruction, and a known solution.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import workloads


def laplacian_1d(n):
    return 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)


@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_factor_of_1d_laplacian_closed_form(n):
    """tridiag(-1, 2, -1) = L L^T with L_ii = sqrt((i+2)/(i+1)) and
    L_{i+1,i} = -sqrt((i+1)/(i+2)) (0-based), and its inverse has entries
    min(i,j)+1 times (n - max(i,j)) over n + 1."""
    L, W = oracle.chol_factor(laplacian_1d(n))
    ref = np.zeros((n, n))
    for i in range(n):
        ref[i, i] = math.sqrt((i + 2) / (i + 1))
        if i + 1 < n:
            ref[i + 1, i] = -math.sqrt((i + 1) / (i + 2))
    assert np.max(np.abs(L - ref)) < 1e-14
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    tinv = (np.minimum(i, j) + 1) * (n - np.maximum(i, j)) / (n + 1.0)
    assert np.max(np.abs(W.T @ W - tinv)) < 1e-12 * n
    b = np.arange(1.0, n + 1)
    assert np.max(np.abs(oracle.chol_solve(W, b) - tinv @ b)) < 1e-11 * n


def test_factor_2x2_closed_form():
    """[[a, b], [b, c]]: L = [[sqrt a, 0], [b / sqrt a, sqrt(c - b^2 / a)]]."""
    a, b, c = 4.0, 2.0, 5.0
    L, W = oracle.chol_factor(np.array([[a, b], [b, c]]))
    l11, l21 = math.sqrt(a), b / math.sqrt(a)
    l22 = math.sqrt(c - l21 * l21)
    assert np.allclose(L, [[l11, 0.0], [l21, l22]], rtol=0, atol=1e-15)
    assert np.allclose(W, [[1 / l11, 0.0], [-l21 / (l11 * l22), 1 / l22]], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [3, 64, 129])
def test_factor_reconstructs_and_is_lower_with_positive_diagonal(n):
    """L L^T = C, L lower triangular with a positive diagonal (the unique
    Cholesky factor), W L = I, and W lower triangular."""
    C = workloads.spd_matrix(n, 1e3, seed=n)
    L, W = oracle.chol_factor(C)
    assert np.max(np.abs(L @ L.T - C)) < 1e-12 * np.max(np.abs(C))
    assert np.all(np.triu(L, 1) == 0) and np.all(np.diag(L) > 0)
    assert np.max(np.abs(W @ L - np.eye(n))) < 1e-11
    assert np.max(np.abs(np.triu(W, 1))) == 0


def test_solve_recovers_known_solution():
    n = 200
    C = workloads.spd_matrix(n, 1e4, seed=1)
    x = np.random.Generator(np.random.PCG64(11)).standard_normal(n)
    _, W = oracle.chol_factor(C)
    assert np.max(np.abs(oracle.chol_solve(W, C @ x) - x)) < 1e4 * 1e-13 * np.max(np.abs(x)) * 10


def test_indefinite_matrix_is_rejected():
    C = np.diag([1.0, -1.0, 2.0])
    with pytest.raises(np.linalg.LinAlgError):
        oracle.chol_factor(C)


def test_spd_generator_spectrum():
    """The generated matrix is symmetric with eigenvalues 1 .. cond."""
    C = workloads.spd_matrix(50, 1e3, seed=2)
    assert np.max(np.abs(C - C.T)) == 0
    ev = np.linalg.eigvalsh(C)
    assert abs(ev[0] - 1.0) < 1e-9 and abs(ev[-1] - 1e3) < 1e-9

"""Pins for the oracle's dense Bunch-Kaufman LDL^T with inertia (the factorization of eq. (7),
Sec. IV "Step direction"): reconstruction, solves against numpy, and inertia against the
eigenvalue sign count (Sylvester's law of inertia)."""
import numpy as np
import pytest
import scipy.linalg

import oracle


def _inertia_eig(A, tol=1e-9):
    ev = np.linalg.eigvalsh(A)
    s = tol * max(1.0, np.abs(ev).max())
    return (int((ev > s).sum()), int((ev < -s).sum()), int((np.abs(ev) <= s).sum()))


def _kkt(rng, n, m, shift=0.0):
    W = rng.normal(size=(n, n))
    W = W + W.T + shift * np.eye(n)
    A = rng.normal(size=(m, n))
    K = np.zeros((n + m, n + m))
    K[:n, :n] = W
    K[n:, :n] = A
    K[:n, n:] = A.T
    return K


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("size", [1, 2, 5, 17, 40])
def test_random_symmetric(seed, size):
    rng = np.random.default_rng([11, seed, size])
    A = rng.normal(size=(size, size))
    A = A + A.T
    fact = oracle.bk_factor(A)
    P, L, D = oracle.bk_unpack(fact)
    assert np.abs(P @ A @ P.T - L @ D @ L.T).max() <= 50 * size * np.finfo(float).eps * np.abs(A).max() * 10
    b = rng.normal(size=size)
    x = oracle.bk_solve(fact, b)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-9)
    assert fact[3] == _inertia_eig(A)


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("nm", [(6, 3), (20, 11), (35, 20)])
@pytest.mark.parametrize("shift", [-3.0, 0.0, 8.0])
def test_kkt_structured(seed, nm, shift):
    n, m = nm
    rng = np.random.default_rng([12, seed, n, m])
    K = _kkt(rng, n, m, shift)
    fact = oracle.bk_factor(K)
    assert fact[3] == _inertia_eig(K)
    # LAPACK sytrf (scipy.linalg.ldl) must report the same inertia from its D
    _, D, _ = scipy.linalg.ldl(K)
    assert fact[3] == _inertia_eig(D)
    b = rng.normal(size=n + m)
    assert np.allclose(oracle.bk_solve(fact, b), np.linalg.solve(K, b), rtol=1e-8, atol=1e-8)


def test_two_by_two_pivot_and_zero_column():
    # zero diagonal forces a 2x2 pivot: [[0,1],[1,0]] has inertia (1,1,0)
    A = np.array([[0.0, 1.0], [1.0, 0.0]])
    fact = oracle.bk_factor(A)
    assert fact[2][0] == 2
    assert fact[3] == (1, 1, 0)
    assert np.allclose(oracle.bk_solve(fact, np.array([3.0, 5.0])), [5.0, 3.0])
    # an exactly zero row/column is a zero pivot
    B = np.diag([2.0, 0.0, -1.0])
    assert oracle.bk_factor(B)[3] == (1, 1, 1)


def test_badly_scaled_slack_block_is_not_singular():
    # [[sigma, -1], [-1, 0]] with sigma = 1e9: eigenvalues ~ sigma and -1/sigma (det = -1);
    # the inertia must be (1, 1, 0), never "singular"
    A = np.array([[1e9, -1.0], [-1.0, 0.0]])
    assert oracle.bk_factor(A)[3] == (1, 1, 0)

"""Pins for S_n and the Toeplitz products (eq. sine_transform, eq.
tau_preconditioner, eqs. grunwaldmatrix1/2)."""
import numpy as np
import pytest

from oracle import grunwald, symbol, transforms as tr


@pytest.mark.parametrize("n", [1, 2, 7, 31, 100, 255])
def test_dst_matrix_properties(n):
    S = tr.dst_matrix(n)
    np.testing.assert_allclose(S, S.T, atol=0)
    np.testing.assert_allclose(S @ S, np.eye(n), atol=1e-13)
    x = np.random.default_rng(n).standard_normal(n)
    np.testing.assert_allclose(tr.dst(x), S @ x, atol=1e-13)


def test_dst_2d_is_kronecker():
    rng = np.random.default_rng(0)
    n1, n2 = 9, 6
    X = rng.standard_normal((n2, n1))
    K = np.kron(tr.dst_matrix(n2), tr.dst_matrix(n1))
    Y = tr.dst(tr.dst(X, axis=1), axis=0)
    np.testing.assert_allclose(Y.reshape(-1), K @ X.reshape(-1), atol=1e-13)


@pytest.mark.parametrize("n", [15, 63, 255])
def test_tau_eigenvalues_are_symbol_samples(n):
    f = symbol.p_symbol(1.5, symbol.theta(n)) + 0.1
    S = tr.dst_matrix(n)
    tau = S @ np.diag(f) @ S
    ev = np.sort(np.linalg.eigvalsh(0.5 * (tau + tau.T)))
    np.testing.assert_allclose(ev, np.sort(f), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 7, 16, 63, 100, 255])
@pytest.mark.parametrize("weights", ["shifted", "weighted"])
def test_toeplitz_product_equals_dense(n, weights):
    gen = grunwald.generator(1.37, n, weights)
    T = tr.toeplitz_dense(gen, n)
    # the matrix of eq. grunwaldmatrix1: -g_1 on the diagonal, -g_0 above it
    assert T[0, 0] == -gen[1]
    if n > 1:
        assert T[0, 1] == -gen[0] and T[1, 0] == -gen[2]
        assert np.all(np.triu(T, 2) == 0)
    x = np.random.default_rng(n).standard_normal(n)
    np.testing.assert_allclose(tr.toeplitz_mv(gen, x), T @ x, atol=1e-13)
    np.testing.assert_allclose(tr.toeplitz_mv(gen, x, transpose=True), T.T @ x, atol=1e-13)

"""Pins for the build-mode Krylov solvers: brute-force Krylov-subspace
minimisers on tiny systems, dense solves, and the bounded iteration counts of
the constant-coefficient case (Section 3.1 Case I, Theorem 3)."""
import numpy as np
import pytest
import scipy.linalg

import fde_inputs as fi
from oracle import krylov, precond as pc
from oracle.system import FDESystem


def _krylov_basis(op, v0, k):
    """Orthonormal basis of span{v0, op v0, ..., op^{k-1} v0} (Gram-Schmidt
    applied twice at every step, so the basis stays well conditioned)."""
    Q = np.zeros((v0.size, k))
    v = v0 / np.linalg.norm(v0)
    for i in range(k):
        for _ in range(2):
            v = v - Q[:, :i] @ (Q[:, :i].T @ v)
        Q[:, i] = v / np.linalg.norm(v)
        v = op(Q[:, i])
    return Q


def tiny_system(n=24, alpha=1.6):
    p = fi.variable_1d(n=n, alpha=alpha)
    return FDESystem.from_problem(p), p


@pytest.mark.parametrize("k", [1, 3, 6])
def test_fgmres_iterate_is_the_krylov_minimiser(k):
    """After k steps (one cycle) FGMRES with a fixed P returns
    x0 + P Q y minimising ||b - M x|| over the Krylov space K_k(M P, r0)."""
    s, p = tiny_system()
    A = s.dense()
    P = pc.make("tau", s)
    Pinv = P.dense_inverse()
    rng = np.random.default_rng(k)
    b = rng.standard_normal(s.N)
    x0 = rng.standard_normal(s.N)
    x, info = krylov.fgmres(lambda v: A @ v, b, lambda v: Pinv @ v, x0=x0, restart=k,
                            tol=1e-300, maxit=k)
    assert info["iters"] == k
    r0 = b - A @ x0
    Q = _krylov_basis(lambda v: A @ (Pinv @ v), r0, k)
    y, *_ = np.linalg.lstsq(A @ Pinv @ Q, r0, rcond=None)
    xref = x0 + Pinv @ Q @ y
    np.testing.assert_allclose(x, xref, rtol=1e-9, atol=1e-10)
    # the Givens estimate equals the true residual of the returned iterate
    assert info["relres_est"] == pytest.approx(info["relres_true"], rel=1e-6)


def test_fgmres_restarts_converge_to_dense_solution():
    s, p = tiny_system(n=60, alpha=1.3)
    A = s.dense()
    b = np.random.default_rng(5).standard_normal(s.N)
    xs = np.linalg.solve(A, b)
    P = pc.make("tau", s)
    x, info = krylov.fgmres(s.matvec, b, P, restart=5, tol=1e-11)
    assert info["converged"] and info["restarts"] > 0
    assert np.linalg.norm(b - A @ x) <= 1e-11 * np.linalg.norm(b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


@pytest.mark.parametrize("k", [1, 2, 5])
def test_pcg_iterate_minimises_energy_error(k):
    p = fi.constant_1d(n=40)
    s = FDESystem.from_problem(p)
    A = s.dense()
    Pinv = pc.make("tau", s).dense_inverse()
    b = p.b
    x, info = krylov.pcg(lambda v: A @ v, b, lambda v: Pinv @ v, tol=1e-300, maxit=k)
    xs = np.linalg.solve(A, b)
    K = _krylov_basis(lambda v: Pinv @ (A @ v), Pinv @ b, k)
    # minimise (x - xs)^T A (x - xs) over span(K): Galerkin condition
    c = np.linalg.solve(K.T @ A @ K, K.T @ b)
    np.testing.assert_allclose(x, K @ c, rtol=1e-8, atol=1e-10)


def test_pcg_constant_case_iterations_bounded():
    """Case I: tau(p + nu) preconditioned CG needs a number of iterations that
    does not grow with n (the preconditioned spectrum is bounded)."""
    its = []
    for k in range(6, 17):   # n = 63 ... 65535
        p = fi.constant_1d(n=2 ** k - 1)
        s = FDESystem.from_problem(p)
        P = pc.make("tau", s)
        x, info = krylov.pcg(s.matvec, p.b, P, tol=1e-10)
        assert info["converged"]
        its.append(info["iters"])
    assert max(its) <= 8 and max(its) - min(its) <= 2
    # unpreconditioned CG grows like sqrt(kappa) ~ n^{alpha/2}
    p = fi.constant_1d(n=1023)
    s = FDESystem.from_problem(p)
    x, info = krylov.pcg(s.matvec, p.b, pc.Identity(s), tol=1e-10)
    assert info["iters"] > 5 * max(its)


def test_fgmres_2d_small_against_dense():
    p = fi.variable_2d(n=15, n2=11)
    s = FDESystem.from_problem(p)
    A = s.dense()
    b = s.rhs(p.u0.reshape(-1))
    P = pc.make("tau", s)
    x, info = krylov.fgmres(s.matvec, b, P, x0=p.u0.reshape(-1), restart=30, tol=1e-10)
    assert info["converged"]
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)

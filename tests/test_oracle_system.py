"""Pins for the coefficient matrices (eq. first_order_1d_coefficient_matrix,
eq. coef:2d) and the preconditioners (eq. prop_1D, eq. 2D_preconditioner)."""
import numpy as np
import pytest

import fde_inputs as fi
from oracle import precond as pc
from oracle import transforms as tr
from oracle.system import FDESystem


def small_2d(n1=7, n2=5, ax=1.7, ay=1.4, time="euler", weights="shifted"):
    p = fi.variable_2d(n=n1, n2=n2, ax=ax, ay=ay)
    p.time, p.weights = time, weights
    return FDESystem.from_problem(p), p


@pytest.mark.parametrize("time,weights", [("euler", "shifted"), ("cn", "weighted")])
def test_2d_fast_operator_equals_kronecker_form(time, weights):
    s, p = small_2d(time=time, weights=weights)
    A = s.dense()
    u = np.random.default_rng(1).standard_normal(s.N)
    np.testing.assert_allclose(s.matvec(u), A @ u, rtol=1e-13, atol=1e-13)
    # the x-term acts along the contiguous axis: with e+- = 0 the operator is
    # block diagonal with n2 blocks of size n1
    s.eplus[:] = 0
    s.eminus[:] = 0
    B = s.dense()
    n1 = s.n[0]
    off = B.copy()
    for j in range(s.n[1]):
        off[j * n1:(j + 1) * n1, j * n1:(j + 1) * n1] = 0
    assert np.all(off == 0)


def test_1d_operator_and_structure():
    p = fi.variable_1d(n=40, alpha=1.6)
    s = FDESystem.from_problem(p)
    A = s.dense()
    u = np.random.default_rng(2).standard_normal(s.N)
    np.testing.assert_allclose(s.matvec(u), A @ u, rtol=1e-13, atol=1e-13)
    # first-order weights: strictly row diagonally dominant with nonpositive
    # off-diagonals (a nonsingular M-matrix)
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 1e-15)
    assert np.all(np.diag(A) > np.abs(off).sum(axis=1))
    sub, main, sup = s.tridiagonal()
    np.testing.assert_allclose(main, np.diag(A), rtol=1e-14)
    np.testing.assert_allclose(sub, np.diag(A, -1), rtol=1e-14)
    np.testing.assert_allclose(sup, np.diag(A, 1), rtol=1e-14)


@pytest.mark.parametrize("dim", [1, 2])
def test_first_order_rows_dominant_by_nu(dim):
    """Every row of the first-order (shifted Grunwald) M has diagonal minus
    off-diagonal absolute sum >= nu, so ||M^{-1}||_inf <= 1/nu (Varah); the
    mixed-form GPU tests bound the distance between two tol-accurate
    solutions with it."""
    if dim == 1:
        p = fi.variable_1d(n=60, alpha=1.3, seed=4)
    else:
        p = fi.variable_2d(n=9, n2=7, ax=1.9, ay=1.1, seed=4)
    s = FDESystem.from_problem(p)
    assert s.weights == "shifted"
    A = s.dense()
    d = np.diag(A)
    margin = d - (np.abs(A).sum(axis=1) - np.abs(d))
    assert margin.min() >= s.nu * (1 - 1e-12)
    assert np.abs(np.linalg.inv(A)).sum(axis=1).max() <= (1 + 1e-12) / s.nu


def test_constant_case_is_spd_and_hat_equals_shifted_tau():
    p = fi.constant_1d(n=31)
    s = FDESystem.from_problem(p)
    A = s.dense()
    np.testing.assert_allclose(A, A.T, atol=1e-15)
    assert np.linalg.eigvalsh(A).min() > 0
    P1 = pc.make("tau", s)          # shift nu/D applied (Case I)
    P2 = pc.make("tau_hat", s)
    v = np.random.default_rng(3).standard_normal(s.N)
    np.testing.assert_allclose(P1(v), P2(v), rtol=1e-13)
    assert P1.shift == pytest.approx(s.nu)


@pytest.mark.parametrize("dside", ["left", "right"])
def test_tau_apply_equals_dense_inverse(dside):
    s, p = small_2d()
    P = pc.make("tau", s, dside=dside)
    Pinv = P.dense_inverse()
    v = np.random.default_rng(4).standard_normal(s.N)
    np.testing.assert_allclose(P(v), Pinv @ v, rtol=1e-12, atol=1e-13)
    # P itself: D_N (S (x) S) F_N (S (x) S) in the text order
    S = np.kron(tr.dst_matrix(s.n[1]), tr.dst_matrix(s.n[0]))
    D = np.diag(P.D.reshape(-1))
    tau = S @ np.diag(P.F.reshape(-1)) @ S
    Pm = D @ tau if dside == "left" else tau @ D
    np.testing.assert_allclose(Pinv @ Pm, np.eye(s.N), atol=1e-10)


def test_example23_inputs_match_oracle_examples():
    """The Example 2/3 problem data of fde_inputs (used by the GPU tables) are
    the oracle's Example 2/3 fields, exact solution and source."""
    import fde_inputs as fi
    from oracle import examples as ex
    for example, (a, b) in ((2, (1.8, 1.6)), (3, (1.8, 1.2))):
        p = fi.paper_2d(15, example)
        s, X, Y = ex.ex2_system(15, a, b)
        assert np.allclose(p.dplus, s.dplus, rtol=0, atol=0) and np.array_equal(p.eminus, s.eminus)
        assert np.array_equal(p.dminus, s.dminus) and np.array_equal(p.eplus, s.eplus)
        assert p.dt == s.dt and p.time == s.time and p.weights == s.weights
        assert np.array_equal(p.u0, ex.ex2_exact(X, Y, 0.0))
        assert np.allclose(fi.example23_source(X, Y, 0.3, a, b), ex.ex2_source(X, Y, 0.3, a, b), rtol=1e-15)

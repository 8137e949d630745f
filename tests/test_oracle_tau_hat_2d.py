"""Pins for the 2D constant-coefficient preconditioner P_hat
(eq. 2D_preconditioner_proof_case) and for Theorem 3.

Theorem 3's proof splits the constant-coefficient matrix into
I (x) A1 + A2 (x) I, with A1 = (1/r) I + d (T_a + T_a^T) along x and
A2 = (s/r) e (T_b + T_b^T) along y, and P_hat into the matching sums of the 1D
tau matrices P1 = S diag(1/r + d F_a) S, P2 = S diag((s/r) e F_b) S.  It then
bounds the spectrum of P_hat^{-1} A_N by the extreme eigenvalues of the two
1D preconditioned matrices P1^{-1} A1 and P2^{-1} A2.  The tests below check
that inclusion on dense matrices built from the Toeplitz generators (not from
the preconditioner code), for d != e and alpha != beta, so that a dropped
kappa = s/r, swapped d and e, or a wrong symbol order in P_hat moves an
eigenvalue out of the interval; and they check that the condition number
stays bounded as N grows."""
import numpy as np
import pytest
import scipy.linalg

import fde_inputs as fi
from oracle import precond as pc
from oracle import symbol, transforms as tr
from oracle.system import FDESystem


def const_2d(n1, n2, alpha, beta, d, e, weights="weighted", time="cn"):
    x, hx = fi.grid(n1, 0.0, 2.0)
    one = np.ones((n2, n1))
    p = fi.Problem(dim=2, n=(n1, n2), alpha=(alpha, beta), lo=(0.0, 0.0), hi=(2.0, 2.0),
                   dt=hx, dplus=d * one, dminus=d * one, eplus=e * one, eminus=e * one,
                   weights=weights, time=time)
    return FDESystem.from_problem(p)


def split_1d(s, d, e):
    """A1, A2 of Theorem 3 from the Toeplitz generators, and the 1D tau
    preconditioners P1, P2 of its proof."""
    n1, n2 = s.n
    Tx = tr.toeplitz_dense(s.gx, n1)
    Ty = tr.toeplitz_dense(s.gy, n2)
    A1 = s.nu * np.eye(n1) + d * (Tx + Tx.T)
    A2 = s.kappa * e * (Ty + Ty.T)
    S1, S2 = tr.dst_matrix(n1), tr.dst_matrix(n2)
    f1 = s.nu + d * symbol.F_symbol(s.alpha[0], symbol.theta(n1), s.weights)
    f2 = s.kappa * e * symbol.F_symbol(s.alpha[1], symbol.theta(n2), s.weights)
    P1 = S1 @ np.diag(f1) @ S1
    P2 = S2 @ np.diag(f2) @ S2
    return A1, A2, P1, P2


def gen_eigs(A, P):
    """Eigenvalues of P^{-1} A for SPD A and P (a symmetric-definite pencil)."""
    return scipy.linalg.eigh(A, P, eigvals_only=True)


def p_hat_dense(s):
    return np.linalg.inv(pc.TauHatPreconditioner(s).dense_inverse())


CASES = [
    # (alpha, beta, d, e, weights, time)
    (1.8, 1.2, 1.0, 7.0, "weighted", "cn"),
    (1.3, 1.9, 5.0, 0.4, "weighted", "cn"),
    (1.7, 1.4, 2.0, 0.5, "shifted", "euler"),
]


def test_split_reproduces_the_system_matrix():
    """A_N = I (x) A1 + A2 (x) I for constant coefficients (Theorem 3)."""
    s = const_2d(9, 7, 1.8, 1.2, 1.0, 7.0)
    A1, A2, _, _ = split_1d(s, 1.0, 7.0)
    A = np.kron(np.eye(7), A1) + np.kron(A2, np.eye(9))
    np.testing.assert_allclose(s.dense(), A, rtol=0, atol=1e-13 * np.abs(A).max())


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("n1,n2", [(7, 9), (15, 11), (31, 23)])
def test_theorem3_spectrum_inside_1d_interval(case, n1, n2):
    alpha, beta, d, e, weights, time = case
    s = const_2d(n1, n2, alpha, beta, d, e, weights, time)
    A1, A2, P1, P2 = split_1d(s, d, e)
    l1, l2 = gen_eigs(A1, P1), gen_eigs(A2, P2)
    lo, hi = min(l1.min(), l2.min()), max(l1.max(), l2.max())
    lam = gen_eigs(s.dense(), p_hat_dense(s))
    assert lam.min() >= lo * (1 - 1e-10) and lam.max() <= hi * (1 + 1e-10), (lam.min(), lam.max(), lo, hi)


@pytest.mark.parametrize("case", CASES)
def test_theorem3_condition_number_bounded_in_n(case):
    """kappa(P_hat^{-1} A_N) does not grow with N (n = 7 ... 63)."""
    alpha, beta, d, e, weights, time = case
    ks = []
    for n in (7, 15, 31, 63):
        s = const_2d(n, n, alpha, beta, d, e, weights, time)
        lam = gen_eigs(s.dense(), p_hat_dense(s))
        ks.append(lam.max() / lam.min())
    # unpreconditioned kappa(A_N) grows like n^max(alpha, beta); this one stays put
    assert max(ks) < 3.0, ks
    assert ks[-1] < 1.2 * ks[0] + 0.2, ks
    s = const_2d(63, 63, alpha, beta, d, e, weights, time)
    w = np.linalg.eigvalsh(s.dense())
    assert w.max() / w.min() > 10 * max(ks)


def test_p_hat_equals_shifted_p_f_when_d_equals_e():
    """With d+- = e+- = c, D_N = c and P_F with the Case I shift nu/c is
    c tau(F + nu/c) = tau(nu + c F_a + kappa c F_b) = P_hat."""
    for weights, time in (("shifted", "euler"), ("weighted", "cn")):
        s = const_2d(15, 11, 1.6, 1.3, 2.5, 2.5, weights, time)
        a = pc.TauHatPreconditioner(s).dense_inverse()
        b = pc.TauPreconditioner(s).dense_inverse()
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14 * np.abs(a).max())
    # with d != e the two differ (P_F scales by the average of d and e)
    s = const_2d(15, 11, 1.6, 1.3, 1.0, 4.0)
    a = pc.TauHatPreconditioner(s).dense_inverse()
    b = pc.TauPreconditioner(s).dense_inverse()
    assert np.abs(a - b).max() > 1e-3 * np.abs(a).max()


def test_p_hat_eigenvalues_are_the_symbol_samples():
    """The eigenvalues of P_hat are 1/r + d F_a(theta_i) + (s/r) e F_b(theta_j)
    for every pair (i, j) (Kronecker sum of the 1D samples)."""
    s = const_2d(11, 7, 1.8, 1.2, 1.0, 7.0)
    P = p_hat_dense(s)
    _, _, P1, P2 = split_1d(s, 1.0, 7.0)
    Pk = np.kron(np.eye(7), P1) + np.kron(P2, np.eye(11))
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(0.5 * (P + P.T))),
                               np.sort(np.linalg.eigvalsh(Pk)), rtol=1e-10)

"""Preconditioners.

P_F (eq. prop_1D, eq. 2D_preconditioner):
    1D:  P = D_n tau_n(F_a) = D_n S_n diag(F_a(theta)) S_n,       D_n = (D+ + D-)/2
    2D:  P = D_N (S_{n2} (x) S_{n1}) F_N (S_{n2} (x) S_{n1}),      D_N = (D+ + D- + E+ + E-)/4
         F_N(i, j) = F_a(theta_i) + (s/r) F_b(theta_j)
  ``dside='left'`` is the order the text writes (D tau): P^{-1} v = tau^{-1}(D^{-1} v).
  ``dside='right'`` puts D on the other side (tau D): P^{-1} v = D^{-1} tau^{-1} v;
  this is the order that reproduces the condition numbers printed in Tables 1, 3, 4.
  ``shift`` adds a constant to every symbol sample.  The paper adds
  2 nu/(d+ + d-) = nu/D in the constant-coefficient case (Section 3.1, Case I);
  ``shift=None`` applies that rule when all coefficients are one equal constant,
  and no shift otherwise (variable coefficients, eq. prop_1D / 2D_preconditioner).

P_hat (eq. 2D_preconditioner_proof_case; 1D: Case I):
    P = (S (x) S) diag(nu + d F_a(theta_i) + kappa e F_b(theta_j)) (S (x) S), constant d, e.

P_tilde (Table 2, 1D): P = S_n diag(D_n[j] p_a(theta_j)) S_n.
P_tri   (Table 2, 1D): the three main diagonals of M, solved by a banded solver.
"""
import numpy as np
import scipy.linalg

from . import symbol
from . import transforms as tr


def _const_value(*arrs):
    v = float(np.ravel(arrs[0])[0])
    for a in arrs:
        if not np.all(np.asarray(a) == v):
            return None
    return v


class TauPreconditioner:
    """P_F with its diagonal factor; also the shifted constant-coefficient form."""

    def __init__(self, sysm, dside="left", shift=None, workers=None):
        self.sys = sysm
        self.dside = dside
        self.workers = workers
        n1 = sysm.n[0]
        fx = symbol.F_symbol(sysm.alpha[0], symbol.theta(n1), sysm.weights)
        if sysm.dim == 1:
            D = 0.5 * (sysm.dplus + sysm.dminus)
            F = fx.copy()
            coeffs = (sysm.dplus, sysm.dminus)
        else:
            n2 = sysm.n[1]
            fy = symbol.F_symbol(sysm.alpha[1], symbol.theta(n2), sysm.weights)
            D = 0.25 * (sysm.dplus + sysm.dminus + sysm.eplus + sysm.eminus)
            F = fx[None, :] + sysm.kappa * fy[:, None]
            coeffs = (sysm.dplus, sysm.dminus, sysm.eplus, sysm.eminus)
        if shift is None:
            c = _const_value(*coeffs)
            shift = sysm.nu / c if c is not None else 0.0
        self.shift = float(shift)
        self.F = F + self.shift
        self.D = D
        if np.any(D <= 0):
            raise ValueError("D has a zero: d+ and d- share a zero (Section 3.1)")

    def tau_inv(self, v):
        V = np.asarray(v, dtype=np.float64).reshape(self.sys.shape)
        if self.sys.dim == 1:
            return tr.dst(tr.dst(V, workers=self.workers) / self.F, workers=self.workers)
        W = tr.dst(tr.dst(V, axis=1, workers=self.workers), axis=0, workers=self.workers)
        W = W / self.F
        return tr.dst(tr.dst(W, axis=0, workers=self.workers), axis=1, workers=self.workers)

    def apply(self, v):
        V = np.asarray(v, dtype=np.float64).reshape(self.sys.shape)
        if self.dside == "left":
            Z = self.tau_inv(V / self.D)
        else:
            Z = self.tau_inv(V) / self.D
        return Z.reshape(np.shape(v))

    __call__ = apply

    def dense_inverse(self):
        """P^{-1} as a dense matrix (small sizes)."""
        if self.sys.dim == 1:
            S = tr.dst_matrix(self.sys.n[0])
        else:
            S = np.kron(tr.dst_matrix(self.sys.n[1]), tr.dst_matrix(self.sys.n[0]))
        tinv = S @ np.diag(1.0 / self.F.reshape(-1)) @ S
        Dinv = np.diag(1.0 / self.D.reshape(-1))
        return tinv @ Dinv if self.dside == "left" else Dinv @ tinv


class TauHatPreconditioner(TauPreconditioner):
    """Constant coefficients d+- = d, e+- = e: diag(nu + d F_a + kappa e F_b), no D."""

    def __init__(self, sysm, workers=None):
        self.sys = sysm
        self.dside = "left"
        self.workers = workers
        d = _const_value(sysm.dplus, sysm.dminus)
        if d is None:
            raise ValueError("P_hat needs constant d+ = d-")
        n1 = sysm.n[0]
        fx = symbol.F_symbol(sysm.alpha[0], symbol.theta(n1), sysm.weights)
        if sysm.dim == 1:
            self.F = sysm.nu + d * fx
        else:
            e = _const_value(sysm.eplus, sysm.eminus)
            if e is None:
                raise ValueError("P_hat needs constant e+ = e-")
            fy = symbol.F_symbol(sysm.alpha[1], symbol.theta(sysm.n[1]), sysm.weights)
            self.F = sysm.nu + d * fx[None, :] + sysm.kappa * e * fy[:, None]
        self.D = np.ones(sysm.shape)
        self.shift = 0.0


class TildePreconditioner(TauPreconditioner):
    """P_tilde = S diag(D_n[j] p(theta_j)) S (Table 2), 1D only."""

    def __init__(self, sysm, workers=None):
        if sysm.dim != 1:
            raise ValueError("P_tilde is a 1D preconditioner")
        self.sys = sysm
        self.dside = "left"
        self.workers = workers
        fx = symbol.F_symbol(sysm.alpha[0], symbol.theta(sysm.n[0]), sysm.weights)
        Dn = 0.5 * (sysm.dplus + sysm.dminus)
        self.F = Dn * fx
        self.D = np.ones(sysm.shape)
        self.shift = 0.0


class TriPreconditioner:
    """P_tri: tridiagonal part of M, solved directly (Table 2)."""

    def __init__(self, sysm):
        sub, main, sup = sysm.tridiagonal()
        n = main.size
        self.ab = np.zeros((3, n))
        self.ab[0, 1:] = sup
        self.ab[1, :] = main
        self.ab[2, :-1] = sub
        self.sys = sysm

    def apply(self, v):
        return scipy.linalg.solve_banded((1, 1), self.ab, np.asarray(v, dtype=np.float64))

    __call__ = apply

    def dense_inverse(self):
        n = self.ab.shape[1]
        T = np.diag(self.ab[1]) + np.diag(self.ab[0, 1:], 1) + np.diag(self.ab[2, :-1], -1)
        return np.linalg.inv(T)


class Identity:
    def __init__(self, sysm=None):
        self.sys = sysm

    def apply(self, v):
        return np.array(v, dtype=np.float64, copy=True)

    __call__ = apply

    def dense_inverse(self):
        return np.eye(self.sys.N)


def make(kind, sysm, dside="left", shift=None, workers=None):
    if kind in ("none", "identity"):
        return Identity(sysm)
    if kind == "tau":
        return TauPreconditioner(sysm, dside=dside, shift=shift, workers=workers)
    if kind == "tau_hat":
        return TauHatPreconditioner(sysm, workers=workers)
    if kind == "tilde":
        return TildePreconditioner(sysm, workers=workers)
    if kind == "tri":
        return TriPreconditioner(sysm)
    raise ValueError(kind)

"""Coefficient matrices and right-hand sides of the time-stepping systems.

1D implicit Euler (Section 1.2, eqs. matrixform / linsystem):
    M = nu I + D+ T + D- T^T,  nu = h^a / h_t,  b = nu u^{m-1} + h^a f^{(m)}.
2D (Section 1.4, eq. coef:2d), x-fastest ordering, arrays of shape (n2, n1):
    A_x = D+ (I (x) T_a) + D- (I (x) T_a^T),  A_y = E+ (T_b (x) I) + E- (T_b^T (x) I)
    implicit Euler: M = nu I + A_x + kappa A_y, nu = h_x^a/h_t, kappa = h_x^a/h_y^b,
                    b = nu u^{m-1} + h_x^a f^{(m)}   (Section 1.2's scheme applied
                    to the 2D operator; the paper prints only the CN form)
    Crank-Nicolson: M = (1/r) I + A_x + (s/r) A_y, r = h_t/(2 h_x^a), s = h_t/(2 h_y^b),
                    b = ((1/r) I - A_x - (s/r) A_y) u^{m-1} + 2 h_x^a v^{(m-1/2)}.
Both 2D forms are nu I + A_x + kappa A_y with kappa = s/r = h_x^a/h_y^b; only nu
(h_x^a/h_t or 2 h_x^a/h_t) and the right-hand side differ.
T may be replaced by S (second-order weights, Section 1.3).
"""
import numpy as np

from . import grunwald
from . import transforms as tr


class FDESystem:
    def __init__(self, dim, n, alpha, lo, hi, dt, dplus, dminus, eplus=None, eminus=None,
                 weights="shifted", time="euler", workers=None):
        self.dim = dim
        self.n = tuple(int(v) for v in n)
        self.alpha = tuple(float(a) for a in alpha)
        self.lo, self.hi = tuple(lo), tuple(hi)
        self.dt = float(dt)
        self.weights = weights
        self.time = time
        self.workers = workers
        self.h = tuple((self.hi[i] - self.lo[i]) / (self.n[i] + 1) for i in range(dim))
        hxa = self.h[0] ** self.alpha[0]
        self.hxa = hxa
        self.nu = hxa / self.dt if time == "euler" else 2.0 * hxa / self.dt
        self.kappa = hxa / self.h[1] ** self.alpha[1] if dim == 2 else 0.0
        self.shape = (self.n[0],) if dim == 1 else (self.n[1], self.n[0])
        self.N = int(np.prod(self.n))
        self.dplus = np.asarray(dplus, dtype=np.float64).reshape(self.shape)
        self.dminus = np.asarray(dminus, dtype=np.float64).reshape(self.shape)
        if dim == 2:
            self.eplus = np.asarray(eplus, dtype=np.float64).reshape(self.shape)
            self.eminus = np.asarray(eminus, dtype=np.float64).reshape(self.shape)
        self.gx = grunwald.generator(self.alpha[0], self.n[0], weights)
        if dim == 2:
            self.gy = grunwald.generator(self.alpha[1], self.n[1], weights)

    @classmethod
    def from_problem(cls, p, workers=None):
        return cls(p.dim, p.n, p.alpha, p.lo, p.hi, p.dt, p.dplus, p.dminus, p.eplus, p.eminus,
                   weights=p.weights, time=p.time, workers=workers)

    # ---- operator pieces -------------------------------------------------
    def Ax(self, u):
        """D+ T_x u + D- T_x^T u, applied along x (the contiguous axis)."""
        U = np.asarray(u, dtype=np.float64).reshape(self.shape)
        ax = U.ndim - 1
        return (self.dplus * tr.toeplitz_mv(self.gx, U, False, ax, self.workers)
                + self.dminus * tr.toeplitz_mv(self.gx, U, True, ax, self.workers))

    def Ay(self, u):
        U = np.asarray(u, dtype=np.float64).reshape(self.shape)
        return (self.eplus * tr.toeplitz_mv(self.gy, U, False, 0, self.workers)
                + self.eminus * tr.toeplitz_mv(self.gy, U, True, 0, self.workers))

    def matvec(self, u):
        U = np.asarray(u, dtype=np.float64).reshape(self.shape)
        w = self.nu * U + self.Ax(U)
        if self.dim == 2:
            w = w + self.kappa * self.Ay(U)
        return w.reshape(np.shape(u))

    def rhs(self, u_prev, f=None):
        U = np.asarray(u_prev, dtype=np.float64).reshape(self.shape)
        if self.time == "euler":
            b = self.nu * U
            if f is not None:
                b = b + self.hxa * np.asarray(f).reshape(self.shape)
        else:
            b = self.nu * U - self.Ax(U)
            if self.dim == 2:
                b = b - self.kappa * self.Ay(U)
            if f is not None:
                b = b + 2.0 * self.hxa * np.asarray(f).reshape(self.shape)
        return b.reshape(np.shape(u_prev))

    # ---- dense forms (small n only) ---------------------------------------
    def dense(self):
        n1 = self.n[0]
        Tx = tr.toeplitz_dense(self.gx, n1)
        if self.dim == 1:
            return (self.nu * np.eye(n1) + self.dplus.reshape(-1)[:, None] * Tx
                    + self.dminus.reshape(-1)[:, None] * Tx.T)
        n2 = self.n[1]
        Ty = tr.toeplitz_dense(self.gy, n2)
        I1, I2 = np.eye(n1), np.eye(n2)
        dp, dm = self.dplus.reshape(-1), self.dminus.reshape(-1)
        ep, em = self.eplus.reshape(-1), self.eminus.reshape(-1)
        Ax = dp[:, None] * np.kron(I2, Tx) + dm[:, None] * np.kron(I2, Tx.T)
        Ay = ep[:, None] * np.kron(Ty, I1) + em[:, None] * np.kron(Ty.T, I1)
        return self.nu * np.eye(self.N) + Ax + self.kappa * Ay

    def tridiagonal(self):
        """Sub, main and super diagonals of the 1D M (for P_tri, Table 2).

        T has -g_1 on the diagonal, -g_2 below it and -g_0 above it, so
        M[i,i] = nu - (d+_i + d-_i) g_1, M[i,i-1] = -d+_i g_2 - d-_i g_0,
        M[i,i+1] = -d+_i g_0 - d-_i g_2.
        """
        if self.dim != 1:
            raise ValueError("P_tri is defined for the 1D system")
        g = grunwald.generator(self.alpha[0], max(self.n[0], 2), self.weights)
        dp, dm = self.dplus, self.dminus
        main = self.nu - (dp + dm) * g[1]
        sub = -dp[1:] * g[2] - dm[1:] * g[0]
        sup = -dp[:-1] * g[0] - dm[:-1] * g[2]
        return sub, main, sup

"""Examples 1-3 of Section 4 and the time-stepping loops that run them.

Example 1 (1D, first-order shifted Grunwald, implicit Euler) on [0,2] x [0,1]:
  d+ = G(3-a) x^a, d- = G(3-a) (2-x)^a, u(x,0) = 4 x^2 (2-x)^2, source f given in
  the text, exact solution 4 e^{-t} x^2 (2-x)^2, h_x = h_t = 2/(n+1), (n+1)/2 steps.
Examples 2 and 3 (2D, second-order weights, Crank-Nicolson) on [0,2]^2 x [0,1]:
  a = 1.8, b = 1.6 (Ex. 2) or 1.2 (Ex. 3), coefficient fields, u0, source and exact
  solution 16 e^{-t} x^2 (2-x)^2 y^2 (2-y)^2 as in the text; h = 2/(n+1), n = M.
  The text states h_t = 1/(M+1) but also 1/r = 2^{a+1} M/(n+1)^a, which holds for
  h_t = 1/M; h_t = 1/M is the reading that reproduces the printed condition
  numbers and iteration counts, and is used here.
"""
import math

import numpy as np

from . import krylov
from . import precond as pc
from .system import FDESystem


def ex1_system(n, alpha):
    h = 2.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    c = math.gamma(3.0 - alpha)
    return FDESystem(1, (n,), (alpha,), (0.0,), (2.0,), h, c * x ** alpha,
                     c * (2.0 - x) ** alpha), x


def ex1_source(x, t, alpha):
    a = alpha
    return -32.0 * math.exp(-t) * (x ** 2 + (2 - x) ** 2 * (8 + x ** 2) / 8.0
                                   - 3.0 * (x ** 3 + (2 - x) ** 3) / (3.0 - a)
                                   + 3.0 * (x ** 4 + (2 - x) ** 4) / ((4.0 - a) * (3.0 - a)))


def ex1_exact(x, t):
    return 4.0 * math.exp(-t) * x ** 2 * (2.0 - x) ** 2


def ex2_system(n, alpha=1.8, beta=1.6):
    h = 2.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    X, Y = np.meshgrid(x, x)
    ca, cb = math.gamma(3.0 - alpha), math.gamma(3.0 - beta)
    dp = ca * (1 + X) ** alpha * (1 + Y) ** 2
    dm = ca * (3 - X) ** alpha * (3 - Y) ** 2
    ep = cb * (1 + X) ** 2 * (1 + Y) ** beta
    em = cb * (3 - X) ** 2 * (3 - Y) ** beta
    ht = 1.0 / n
    sysm = FDESystem(2, (n, n), (alpha, beta), (0.0, 0.0), (2.0, 2.0), ht, dp, dm, ep, em,
                     weights="weighted", time="cn")
    return sysm, X, Y


def _gfun(gam, x, y):
    return ((8 * x ** (2 - gam) - 24 * x ** (3 - gam) / (3 - gam)
             + 24 * x ** (4 - gam) / ((4 - gam) * (3 - gam)))
            * (1 + x) ** gam * (1 + y) ** 2 * y ** 2 * (2 - y) ** 2)


def ex2_source(X, Y, t, alpha, beta):
    return -16.0 * math.exp(-t) * (X ** 2 * (2 - X) ** 2 * Y ** 2 * (2 - Y) ** 2
                                   + _gfun(alpha, X, Y) + _gfun(alpha, 2 - X, 2 - Y)
                                   + _gfun(beta, Y, X) + _gfun(beta, 2 - Y, 2 - X))


def ex2_exact(X, Y, t):
    return 16.0 * math.exp(-t) * X ** 2 * (2 - X) ** 2 * Y ** 2 * (2 - Y) ** 2


def run_ex1(n, alpha, solver="direct", prec="tau", dside="right", tol=1e-7):
    """Time-step Example 1 to T = 1.  Returns (u(T), exact(T), mean iterations)."""
    sysm, x = ex1_system(n, alpha)
    steps = (n + 1) // 2
    u = ex1_exact(x, 0.0)
    its = []
    A = sysm.dense() if solver == "direct" else None
    if solver == "gmres":
        Pinv = pc.make(prec, sysm, dside=dside)
    for m in range(1, steps + 1):
        t = m * sysm.dt
        b = sysm.rhs(u, ex1_source(x, t, alpha))
        if solver == "direct":
            u = np.linalg.solve(A, b)
        else:
            u, k = krylov.gmres_left(sysm.matvec, b, Pinv.apply, tol=tol)
            its.append(k)
    return u, ex1_exact(x, steps * sysm.dt), (float(np.mean(its)) if its else 0.0)


def run_ex2(n, alpha=1.8, beta=1.6, solver="direct", prec="tau", dside="right", tol=1e-7):
    sysm, X, Y = ex2_system(n, alpha, beta)
    steps = n
    u = ex2_exact(X, Y, 0.0).reshape(-1)
    its = []
    A = sysm.dense() if solver == "direct" else None
    if solver == "gmres":
        Pinv = pc.make(prec, sysm, dside=dside)
    for m in range(1, steps + 1):
        tm = (m - 0.5) * sysm.dt
        b = sysm.rhs(u, ex2_source(X, Y, tm, alpha, beta).reshape(-1))
        if solver == "direct":
            u = np.linalg.solve(A, b)
        else:
            u, k = krylov.gmres_left(sysm.matvec, b, Pinv.apply, tol=tol)
            its.append(k)
    return u.reshape(X.shape), ex2_exact(X, Y, steps * sysm.dt), (float(np.mean(its)) if its else 0.0)


def kappa(sysm, prec="none", dside="right"):
    """2-norm condition number of P^{-1} M (Section 4 tables)."""
    A = sysm.dense()
    if prec == "none":
        return float(np.linalg.cond(A))
    P = pc.make(prec, sysm, dside=dside)
    return float(np.linalg.cond(P.dense_inverse() @ A))

"""Generating functions and spectral symbols (Section 2).

g_a(t) = -e^{-i t} (1 - e^{i t})^a          (symbol of T, Section 2.1)
w_a(t) = -((2 - a (1 - e^{-i t}))/2) (1 - e^{i t})^a   (symbol of S, eq_w_function)
p_a(t) = g_a(t) + g_a(-t)                     (Theorem 2, first_order_symbol)
q_a(t) = w_a(t) + w_a(-t)                     (Theorem 2, second_order_symbol)

Complex powers use the principal branch.  Sample points theta_j = j pi/(n+1),
j = 1..n (eq. tau_preconditioner).
"""
import numpy as np


def theta(n: int) -> np.ndarray:
    return np.pi * np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def g_symbol(alpha: float, t):
    t = np.asarray(t, dtype=np.float64)
    return -np.exp(-1j * t) * (1.0 - np.exp(1j * t)) ** alpha


def w_symbol(alpha: float, t):
    t = np.asarray(t, dtype=np.float64)
    return -((2.0 - alpha * (1.0 - np.exp(-1j * t))) / 2.0) * (1.0 - np.exp(1j * t)) ** alpha


def p_symbol(alpha: float, t):
    """p_a(t) = g_a(t) + g_a(-t); real for real t (imaginary parts cancel)."""
    return (g_symbol(alpha, t) + g_symbol(alpha, -np.asarray(t))).real


def q_symbol(alpha: float, t):
    return (w_symbol(alpha, t) + w_symbol(alpha, -np.asarray(t))).real


def F_symbol(alpha: float, t, weights: str = "shifted"):
    """F_a: p_a for the first-order (shifted) scheme, q_a for the second-order one."""
    return p_symbol(alpha, t) if weights == "shifted" else q_symbol(alpha, t)

"""Grunwald and weighted-shifted Grunwald weights.

g_k = (-1)^k binom(alpha, k)  (Section 1.2, eq. grunwald1).  The product form
alpha(alpha-1)...(alpha-k+1)/k! gives the ratio g_k / g_{k-1} = (k-1-alpha)/k,
which is how the weights are generated here.

w_0 = (alpha/2) g_0, w_k = (alpha/2) g_k + ((2-alpha)/2) g_{k-1}, k >= 1
(Section 1.3).
"""
import numpy as np


def grunwald(alpha: float, K: int) -> np.ndarray:
    """g_0..g_K of eq. (grunwald1)."""
    g = np.empty(K + 1, dtype=np.float64)
    g[0] = 1.0
    for k in range(1, K + 1):
        g[k] = g[k - 1] * ((k - 1) - alpha) / k
    return g


def wsgd(alpha: float, K: int) -> np.ndarray:
    """w_0..w_K of Section 1.3."""
    g = grunwald(alpha, K)
    w = np.empty(K + 1, dtype=np.float64)
    w[0] = 0.5 * alpha * g[0]
    w[1:] = 0.5 * alpha * g[1:] + 0.5 * (2.0 - alpha) * g[:-1]
    return w


def generator(alpha: float, n: int, weights: str = "shifted") -> np.ndarray:
    """Weights 0..n that fill the n x n Toeplitz matrix (T or S)."""
    if weights == "shifted":
        return grunwald(alpha, n)
    if weights == "weighted":
        return wsgd(alpha, n)
    raise ValueError(weights)

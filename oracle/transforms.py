"""Sine transform and Toeplitz matrices.

S_n[i, j] = sqrt(2/(n+1)) sin(i j pi/(n+1)), i, j = 1..n   (eq. sine_transform)
T_{a,n} = -[g_{i-j+1}] (zero above the first superdiagonal) (eq. grunwaldmatrix1)
S_{a,n} = -[w_{i-j+1}]                                       (eq. grunwaldmatrix2)

Products use either the dense matrices (small n) or library primitives:
``scipy.fft.dst(type=1, norm='ortho')`` is the orthonormal DST-I, the same
matrix as S_n; ``scipy.linalg.matmul_toeplitz`` multiplies a Toeplitz matrix
given by its first column and first row.
"""
import numpy as np
import scipy.fft
import scipy.linalg


def dst_matrix(n: int) -> np.ndarray:
    idx = np.arange(1, n + 1, dtype=np.float64)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(idx, idx) * np.pi / (n + 1))


def dst(x: np.ndarray, axis: int = -1, workers=None) -> np.ndarray:
    """S_n applied along one axis (S_n is symmetric and involutory)."""
    return scipy.fft.dst(x, type=1, norm="ortho", axis=axis, workers=workers)


def toeplitz_dense(gen: np.ndarray, n: int) -> np.ndarray:
    """-[gen_{i-j+1}] for i - j + 1 >= 0, zero elsewhere (n x n)."""
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    k = i - j + 1
    out = np.zeros((n, n))
    mask = k >= 0
    out[mask] = -gen[k[mask]]
    return out


def toeplitz_col_row(gen: np.ndarray, n: int):
    """First column and first row of -[gen_{i-j+1}]."""
    col = -gen[1:n + 1].copy()
    row = np.zeros(n)
    row[0] = -gen[1]
    if n > 1:
        row[1] = -gen[0]
    return col, row


def toeplitz_mv(gen: np.ndarray, x: np.ndarray, transpose: bool = False, axis: int = 0,
                workers=None) -> np.ndarray:
    """T x (or T^T x) along ``axis`` of x, with T = -[gen_{i-j+1}]."""
    x = np.asarray(x, dtype=np.float64)
    xm = np.moveaxis(x, axis, 0)
    n = xm.shape[0]
    col, row = toeplitz_col_row(gen, n)
    if transpose:
        col, row = row, col
    flat = xm.reshape(n, -1)
    y = scipy.linalg.matmul_toeplitz((col, row), flat, workers=workers)
    return np.moveaxis(y.reshape(xm.shape), 0, axis)

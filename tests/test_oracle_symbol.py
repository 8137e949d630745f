"""Pins for the generating functions and symbols (Section 2, Theorem 2,
Proposition 1)."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import grunwald, symbol, transforms


def p_closed(a, t):
    # derived from the principal branch: 1 - e^{it} = 2 sin(t/2) e^{i(t - pi)/2}
    return 2.0 ** (a + 1) * np.sin(t / 2) ** a * np.cos((2 - a) * (np.pi - t) / 2)


def q_closed(a, t):
    return (2 * np.sin(t / 2)) ** a * (a * np.cos((2 - a) * (np.pi - t) / 2)
                                        - (2 - a) * np.cos(a * (np.pi - t) / 2))


@pytest.mark.parametrize("a", [1.1, 1.2, 1.5, 1.8, 1.9])
def test_closed_forms(a):
    t = np.linspace(1e-6, np.pi, 2001)
    np.testing.assert_allclose(symbol.p_symbol(a, t), p_closed(a, t), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(symbol.q_symbol(a, t), q_closed(a, t), rtol=1e-11, atol=1e-14)
    assert symbol.p_symbol(a, np.pi) == pytest.approx(2 ** (a + 1))
    assert symbol.q_symbol(a, np.pi) == pytest.approx(2 ** (a + 1) * (a - 1))
    assert np.all(symbol.p_symbol(a, t) >= 0) and np.all(symbol.q_symbol(a, t) >= 0)


@pytest.mark.parametrize("a", [1.2, 1.5, 1.8])
def test_zero_of_order_alpha(a):
    # Proposition 1: p_a has a zero of order a at 0, p(t)/t^a -> 2|cos(a pi/2)|
    t = 1e-6
    assert symbol.p_symbol(a, t) / t ** a == pytest.approx(2 * abs(np.cos(a * np.pi / 2)), rel=1e-5)


@pytest.mark.parametrize("a,weights", [(1.3, "shifted"), (1.7, "shifted"), (1.6, "weighted")])
def test_symbol_generates_the_toeplitz_matrix(a, weights):
    """Fourier coefficients of g_a (w_a) are the entries of T (S): the symbol
    really is the generating function of the matrix (Section 2.1)."""
    gen = grunwald.generator(a, 8, weights)
    Tm = transforms.toeplitz_dense(gen, 6)
    f = symbol.g_symbol if weights == "shifted" else symbol.w_symbol
    for k in range(-2, 5):   # T[i, j] depends on i - j = k
        re = quad(lambda t: (f(a, t) * np.exp(-1j * k * t)).real, -np.pi, np.pi, limit=400)[0]
        im = quad(lambda t: (f(a, t) * np.exp(-1j * k * t)).imag, -np.pi, np.pi, limit=400)[0]
        coef = (re + 1j * im) / (2 * np.pi)
        i, j = (k, 0) if k >= 0 else (0, -k)
        assert coef.real == pytest.approx(Tm[i, j], abs=2e-7)
        assert abs(coef.imag) < 2e-7

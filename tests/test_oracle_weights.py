"""Pins for the Grunwald and WSGD weights (eq. grunwald1, Section 1.3)."""
import math

import numpy as np
import pytest
from scipy.special import binom, gamma

from oracle import grunwald


@pytest.mark.parametrize("alpha", [1.1, 1.2, 1.5, 1.7, 1.8, 1.95])
def test_recursion_equals_binomial_definition(alpha):
    K = 60
    g = grunwald.grunwald(alpha, K)
    k = np.arange(K + 1)
    ref = (-1.0) ** k * binom(alpha, k)           # (-1)^k binom(alpha, k)
    np.testing.assert_allclose(g, ref, rtol=1e-13, atol=1e-300)
    # product form alpha (alpha-1) ... (alpha-k+1) / k!
    for kk in (0, 1, 2, 5, 11):
        prod = 1.0
        for i in range(kk):
            prod *= alpha - i
        assert g[kk] == pytest.approx((-1) ** kk * prod / math.factorial(kk), rel=1e-13)


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8])
def test_sign_pattern_and_partial_sums(alpha):
    g = grunwald.grunwald(alpha, 4000)
    assert g[0] == 1.0 and g[1] == pytest.approx(-alpha)
    assert np.all(g[2:] > 0)
    s = np.cumsum(g)
    assert np.all(s[1:] < 0)           # sum_{k<=K} g_k < 0 for K >= 1
    assert np.all(np.diff(s[1:]) > 0)  # increasing towards the full sum (1-1)^alpha = 0
    # tail: sum_{k<=K} g_k = binom(K - alpha, K) ~ K^{-alpha}/Gamma(1-alpha)
    K = 4000
    assert s[K] == pytest.approx(K ** (-alpha) / gamma(1 - alpha), rel=2e-3)


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.56, 1.57, 1.8])
def test_wsgd_identities(alpha):
    w = grunwald.wsgd(alpha, 4000)
    g = grunwald.grunwald(alpha, 4000)
    assert w[0] == pytest.approx(alpha / 2)
    assert w[1] == pytest.approx(alpha / 2 * g[1] + (2 - alpha) / 2)
    # sum_k w_k = (alpha/2 + (2-alpha)/2) sum_k g_k -> 0
    assert abs(np.sum(w)) < 1e-3
    # signs (+, -, +-, +, +, ...): w_2 < 0 exactly when alpha < (sqrt(17)-1)/2
    assert w[1] < 0 and np.all(w[3:] > 0)
    thr = (math.sqrt(17.0) - 1.0) / 2.0
    assert (w[2] < 0) == (alpha < thr)

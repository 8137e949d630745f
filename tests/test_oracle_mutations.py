"""The pins catch plausible mistakes: each test plants one error in the oracle
(on the CPU, through monkeypatching) and checks that a pinned printed value
no longer matches."""
import numpy as np
import pytest

from oracle import examples as ex
from oracle import grunwald, symbol, transforms as tr

# Table 1, n+1 = 64, alpha = 1.5: kappa(M) = 33.4, kappa(P_F^{-1} M) = 16.1
PIN_I, PIN_PF = 33.4, 16.1


def kappas():
    s, _ = ex.ex1_system(63, 1.5)
    return ex.kappa(s), ex.kappa(s, "tau", "right")


def test_unmutated_matches():
    kI, kP = kappas()
    assert abs(kI - PIN_I) < 0.05 and abs(kP - PIN_PF) < 0.05


def test_wrong_weight_sign_is_caught(monkeypatch):
    orig = grunwald.grunwald
    monkeypatch.setattr(grunwald, "grunwald", lambda a, K: orig(a, K) * np.where(np.arange(K + 1) == 2, -1, 1))
    kI, kP = kappas()
    assert abs(kI - PIN_I) > 0.05 or abs(kP - PIN_PF) > 0.05


def test_transposed_toeplitz_is_caught(monkeypatch):
    orig = tr.toeplitz_dense
    monkeypatch.setattr(tr, "toeplitz_dense", lambda g, n: orig(g, n).T)
    # with variable d+ != d- swapping T and T^T changes M
    kI, kP = kappas()
    assert abs(kI - PIN_I) > 0.05 or abs(kP - PIN_PF) > 0.05


def test_wrong_sample_grid_is_caught(monkeypatch):
    monkeypatch.setattr(symbol, "theta", lambda n: np.pi * np.arange(1, n + 1) / n)
    _, kP = kappas()
    assert abs(kP - PIN_PF) > 0.05


def test_modulus_instead_of_real_part_is_caught(monkeypatch):
    monkeypatch.setattr(symbol, "p_symbol",
                        lambda a, t: np.abs(symbol.g_symbol(a, t)) + np.abs(symbol.g_symbol(a, -np.asarray(t))))
    _, kP = kappas()
    assert abs(kP - PIN_PF) > 0.05


def test_symbol_scale_error_is_caught_by_closed_form():
    """kappa and GMRES counts do not see a constant factor in F (P^{-1} M is
    only rescaled); the closed-form value p(pi) = 2^{a+1} does."""
    a = 1.5
    assert symbol.p_symbol(a, np.pi) == pytest.approx(2 ** (a + 1))
    assert 0.5 * symbol.p_symbol(a, np.pi) != pytest.approx(2 ** (a + 1))


def test_wrong_diagonal_side_is_caught():
    s, _ = ex.ex1_system(63, 1.5)
    assert abs(ex.kappa(s, "tau", "left") - PIN_PF) > 0.05

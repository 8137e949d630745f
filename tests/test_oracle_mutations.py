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


def _theorem3_holds():
    """The inclusion of Theorem 3 on one 2D constant-coefficient case with
    d != e and alpha != beta (helpers of test_oracle_tau_hat_2d)."""
    from test_oracle_tau_hat_2d import const_2d, gen_eigs, p_hat_dense, split_1d
    s = const_2d(15, 11, 1.8, 1.2, 1.0, 7.0)
    A1, A2, P1, P2 = split_1d(s, 1.0, 7.0)
    l1, l2 = gen_eigs(A1, P1), gen_eigs(A2, P2)
    lo, hi = min(l1.min(), l2.min()), max(l1.max(), l2.max())
    lam = gen_eigs(s.dense(), p_hat_dense(s))
    return lam.min() >= lo * (1 - 1e-10) and lam.max() <= hi * (1 + 1e-10)


def _mutate_tau_hat(monkeypatch, build):
    from oracle import precond as pc
    orig = pc.TauHatPreconditioner.__init__

    def init(self, sysm, workers=None):
        orig(self, sysm, workers)
        fx = symbol.F_symbol(sysm.alpha[0], symbol.theta(sysm.n[0]), sysm.weights)
        fy = symbol.F_symbol(sysm.alpha[1], symbol.theta(sysm.n[1]), sysm.weights)
        d, e = float(sysm.dplus.flat[0]), float(sysm.eplus.flat[0])
        self.F = build(sysm, fx, fy, d, e)
    monkeypatch.setattr(pc.TauHatPreconditioner, "__init__", init)


def test_p_hat_unmutated_satisfies_theorem3():
    assert _theorem3_holds()


def test_p_hat_dropped_kappa_is_caught(monkeypatch):
    _mutate_tau_hat(monkeypatch, lambda s, fx, fy, d, e: s.nu + d * fx[None, :] + e * fy[:, None])
    assert not _theorem3_holds()


def test_p_hat_swapped_coefficients_are_caught(monkeypatch):
    _mutate_tau_hat(monkeypatch, lambda s, fx, fy, d, e: s.nu + e * fx[None, :] + s.kappa * d * fy[:, None])
    assert not _theorem3_holds()


def test_p_hat_swapped_axes_are_caught(monkeypatch):
    # the x-direction samples laid along y and vice versa (square grid so the shapes agree)
    from test_oracle_tau_hat_2d import const_2d, gen_eigs, p_hat_dense, split_1d
    _mutate_tau_hat(monkeypatch, lambda s, fx, fy, d, e: s.nu + d * fx[:, None] + s.kappa * e * fy[None, :])
    s = const_2d(15, 15, 1.8, 1.2, 1.0, 7.0)
    A1, A2, P1, P2 = split_1d(s, 1.0, 7.0)
    l1, l2 = gen_eigs(A1, P1), gen_eigs(A2, P2)
    lam = gen_eigs(s.dense(), p_hat_dense(s))
    assert lam.min() < min(l1.min(), l2.min()) * (1 - 1e-6) or lam.max() > max(l1.max(), l2.max()) * (1 + 1e-6)

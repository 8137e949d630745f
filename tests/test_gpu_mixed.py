"""GPU parity of the mixed form (float32 inner GMRES + float32 P^{-1} and
matvec inside float64 right-preconditioned FGMRES) on the plan path.

The mixed form takes a different Krylov path from the float64 mirror, so its
iterates are not compared one by one.  What is fixed is the answer: both
solutions satisfy ||b - M x||_2 <= tol ||b||_2, and the residual of the GPU
solution is recomputed here with the oracle's float64 matvec.  The distance
between the two solutions is bounded by the first-order scheme's diagonal
dominance: every row of M = nu I + D+ T + D- T^T (+ kappa (E+ T_y + E- T_y^T)
in 2D) has diagonal minus off-diagonal absolute sum >= nu, because the
off-diagonal Grunwald weights -1 and g_2, g_3, ... add up to less than -g_1 =
alpha (they sum to alpha - 1 over all k >= 2 and T truncates that sum).  By
Varah's bound ||M^{-1}||_inf <= 1/nu, so
    ||x_gpu - x_oracle||_inf <= (||r_gpu||_inf + ||r_oracle||_inf) / nu.
"""
import numpy as np
import pytest

import fde_inputs as fi
from gpu_util import dev, host, need_gpu, relerr, torch
from oracle import krylov, precond as pc
from oracle.system import FDESystem

pytestmark = pytest.mark.gpu


def oracle_solution(p, b, x0, dside="left"):
    s = FDESystem.from_problem(p)
    P = pc.make("tau", s, dside=dside)
    x, info = krylov.fgmres(s.matvec, b, P, x0=x0, restart=30, tol=1e-8)
    assert info["converged"]
    return s, x


def check_mixed(s, b, xg, xo, info, tol=1e-8):
    assert s.weights == "shifted"   # the diagonal-dominance bound below is for the first-order weights
    assert info.converged
    assert info.relres_true <= tol
    rg = b - s.matvec(xg)
    ro = b - s.matvec(xo)
    assert np.linalg.norm(rg) <= tol * (1 + 1e-6) * np.linalg.norm(b)
    bound = (np.abs(rg).max() + np.abs(ro).max()) / s.nu
    assert np.abs(xg - xo).max() <= bound * (1 + 1e-9) + 1e-15, (np.abs(xg - xo).max(), bound)


def mixed_solve(fde, p, b, x0, **kw):
    with fde.Plan(p, precision=fde.MIXED, **kw) as plan:
        x = dev(x0)
        info = plan.solve(dev(b), x)
        return host(x), info


@pytest.mark.parametrize("n", [7, 63, 1023, 4095])
@pytest.mark.parametrize("inner", [0, 4, 16])
def test_mixed_1d(n, inner):
    fde = need_gpu()
    p = fi.variable_1d(n=n, alpha=1.45, seed=100 + n, steps=1)
    b = FDESystem.from_problem(p).rhs(p.u0)
    s, xo = oracle_solution(p, b, p.u0)
    xg, info = mixed_solve(fde, p, b, p.u0, inner_steps=inner)
    check_mixed(s, b, xg, xo, info)
    if inner:
        assert info.inner_iters > 0


@pytest.mark.parametrize("n1,n2", [(15, 15), (63, 31), (127, 127), (255, 255)])
@pytest.mark.parametrize("dside", ["left", "right"])
def test_mixed_2d(n1, n2, dside):
    fde = need_gpu()
    p = fi.variable_2d(n=n1, n2=n2, seed=200 + n1 + n2, steps=1)
    x0 = p.u0.reshape(-1)
    s0 = FDESystem.from_problem(p)
    b = s0.rhs(x0)
    s, xo = oracle_solution(p, b, x0, dside=dside)
    xg, info = mixed_solve(fde, p, b, x0, dside=fde.D_LEFT if dside == "left" else fde.D_RIGHT)
    check_mixed(s, b, xg, xo, info)


def test_mixed_repeat_solves_deterministic():
    """Consecutive solves on one plan, with other device work between them,
    give bit-identical results to the same solves on a fresh plan: no state
    leaks from one solve into the next."""
    fde = need_gpu()
    p = fi.variable_2d(n=127, n2=255, seed=7, steps=1)
    s = FDESystem.from_problem(p)
    rng = np.random.default_rng(8)
    bs = [s.rhs(rng.uniform(-1, 1, p.N)) for _ in range(3)]
    with fde.Plan(p, precision=fde.MIXED, inner_steps=16) as plan:
        shared = []
        for b in bs:
            x = dev(np.zeros(p.N))
            info = plan.solve(dev(b), x)
            junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
            junk.mul_(2.0).sum().item()
            shared.append((host(x), info.iters, info.inner_iters))
    for b, (xa, ia, ja) in zip(bs, shared):
        xb, info = mixed_solve(fde, p, b, np.zeros(p.N), inner_steps=16)
        assert (ia, ja) == (info.iters, info.inner_iters)
        assert np.array_equal(xa, xb)
        assert relerr(s.matvec(xa), b) <= 1e-8 * (1 + 1e-6)


def test_mixed_probe_keeps_results():
    """A timing probe brackets launches with events without changing the
    result, and records launches, time and bytes."""
    fde = need_gpu()
    p = fi.variable_2d(n=255, n2=127, seed=9, steps=1)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0.reshape(-1))
    res = []
    for probe in (fde.PROBE_OFF, fde.PROBE_MAXPY32):
        with fde.Plan(p, precision=fde.MIXED, inner_steps=16) as plan:
            if probe:
                fde.fde_probe(plan.handle, probe)
            x = dev(np.zeros(p.N))
            info = plan.solve(dev(b), x)
            pr = fde.fde_probe_read(plan.handle) if probe else None
            res.append((host(x), info.iters, pr))
    assert res[0][1] == res[1][1]
    assert np.array_equal(res[0][0], res[1][0])
    ms, launches, by = res[1][2]
    assert launches > 0 and ms > 0 and by > 0


# Outer tolerance at which the mixed form is run to meet the stated forward
# error of 1e-8 against the oracle's float64 reference solution.
ACC_TOL = 1e-9


@pytest.mark.parametrize("case", ["1d-4095", "2d-255", "2d-127x63-right"])
def test_mixed_forward_error_1e8(case):
    """The mixed form's result is within 1e-8 (relative) of the exact
    solution of the step, represented by the oracle's float64 FGMRES run to a
    true residual of 1e-13, when its float64 outer loop stops at ACC_TOL."""
    fde = need_gpu()
    kw = {}
    if case == "1d-4095":
        p = fi.variable_1d(n=4095, alpha=1.45, seed=31, steps=1)
        x0 = p.u0
    else:
        n1, n2 = (255, 255) if case == "2d-255" else (127, 63)
        p = fi.variable_2d(n=n1, n2=n2, seed=32, steps=1)
        x0 = p.u0.reshape(-1)
        if case.endswith("right"):
            kw["dside"] = fde.D_RIGHT
    s = FDESystem.from_problem(p)
    b = s.rhs(x0)
    P = pc.make("tau", s, dside="right" if kw else "left")
    xr, ir = krylov.fgmres(s.matvec, b, P, x0=x0, restart=30, tol=1e-13)
    assert ir["converged"]
    xg, info = mixed_solve(fde, p, b, x0, inner_steps=16, tol=ACC_TOL, **kw)
    assert info.converged and info.relres_true <= ACC_TOL
    assert relerr(xg, xr) <= 1e-8, relerr(xg, xr)

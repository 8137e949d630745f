"""Parity at the full 2D size the benchmark times: 1023 x 1023 unknowns per
direction, alpha = (1.7, 1.4), dt = h, FGMRES(30) + P_F to 1e-8 with
x0 = u^{m-1}, in the plan configuration the benchmark uses.  The oracle runs
the first implicit-Euler solve of the job (about ten seconds on 16 threads).

float64: the operator, the preconditioner and the solve mirror the oracle
(relative 1e-12 for the transforms, 1e-10 and one iteration for the solve).
Mixed: the solution is checked through its true residual and against the
oracle's solution with the diagonal-dominance bound of test_gpu_mixed, on two
consecutive time steps."""
import os

import numpy as np
import pytest

import fde_inputs as fi
from gpu_util import dev, host, mirror_check, need_gpu, relerr, torch
from oracle import krylov, precond as pc
from oracle.system import FDESystem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    need_gpu()
    p = fi.variable_2d(n=1023, steps=2)
    workers = min(16, len(os.sched_getaffinity(0)))
    s = FDESystem.from_problem(p, workers=workers)
    u0 = p.u0.reshape(-1)
    b = s.rhs(u0)
    P = pc.make("tau", s, workers=workers)
    xo, io = krylov.fgmres(s.matvec, b, P, x0=u0, restart=30, tol=p.tol)
    assert io["converged"]
    return dict(p=p, s=s, P=P, u0=u0, b=b, xo=xo, io=io)


def test_full_matvec_and_tau(full):
    fde = need_gpu()
    p, s, P = full["p"], full["s"], full["P"]
    v = np.random.default_rng(31).uniform(-1, 1, p.N)
    with fde.Plan(p) as plan:
        y = torch.empty(p.N, dtype=torch.float64, device="cuda")
        plan.matvec(dev(v), y)
        assert relerr(host(y), s.matvec(v)) < 1e-12
        plan.tau_apply(dev(v), y)
        assert relerr(host(y), P(v)) < 1e-12


def test_full_fp64_solve_mirrors_oracle(full):
    fde = need_gpu()
    p = full["p"]
    with fde.Plan(p, precision=fde.FP64) as plan:
        x = dev(full["u0"])
        info = plan.solve(dev(full["b"]), x)
        xg = host(x)
    assert info.converged
    assert abs(info.iters - full["io"]["iters"]) <= 1, (info.iters, full["io"]["iters"])
    assert relerr(xg, full["xo"]) < 1e-10


def test_full_mixed_solve(full):
    fde = need_gpu()
    p, s, b, xo = full["p"], full["s"], full["b"], full["xo"]
    with fde.Plan(p, precision=fde.MIXED, inner_steps=16) as plan:
        u = dev(full["u0"])
        bd = torch.empty(p.N, dtype=torch.float64, device="cuda")
        xs, infos = [], []
        for _ in range(2):   # two implicit-Euler steps, x0 = u^{m-1}
            plan.rhs(u, bd)
            x = u.clone()
            infos.append(plan.solve(bd, x))
            xs.append(host(x))
            u = x
    # first step against the oracle's float64 solution
    info = infos[0]
    assert info.converged and info.relres_true <= p.tol
    rg = b - s.matvec(xs[0])
    ro = b - s.matvec(xo)
    assert np.linalg.norm(rg) <= p.tol * (1 + 1e-6) * np.linalg.norm(b)
    bound = (np.abs(rg).max() + np.abs(ro).max()) / s.nu
    assert np.abs(xs[0] - xo).max() <= bound * (1 + 1e-9), (np.abs(xs[0] - xo).max(), bound)
    # second step: its own true residual
    assert infos[1].converged
    b2 = s.rhs(xs[0])
    assert np.linalg.norm(b2 - s.matvec(xs[1])) <= p.tol * (1 + 1e-6) * np.linalg.norm(b2)


def _workers():
    return min(16, len(os.sched_getaffinity(0)))


def test_full_fp64_last_step_mirrors_oracle(full):
    """The tenth implicit-Euler step of the job (the benchmark's step count),
    mirrored by the oracle from the GPU's ninth state."""
    fde = need_gpu()
    p = fi.variable_2d(n=1023, steps=10)
    s, P = full["s"], full["P"]
    with fde.Plan(p, precision=fde.FP64) as plan:
        u = dev(p.u0.reshape(-1))
        bd = torch.empty(p.N, dtype=torch.float64, device="cuda")
        for step in range(10):
            prev = u.clone()
            plan.rhs(u, bd)
            x = u.clone()
            info = plan.solve(bd, x)
            u = x
        xg, u9, b = host(u), host(prev), host(bd)
        assert relerr(b, s.rhs(u9)) < 1e-12

        def grun(maxit):
            with fde.Plan(p, precision=fde.FP64, maxit=maxit) as q:
                x = dev(u9)
                i = q.solve(dev(b), x, allow_notconv=True)
                return host(x), i.iters

    def orun(maxit):
        x, i = krylov.fgmres(s.matvec, b, P, x0=u9, restart=30, tol=p.tol, maxit=maxit or 100000)
        return x, i["iters"]

    assert info.converged
    mirror_check(xg, info.iters, orun, grun)


def test_full_cn_second_order_step():
    """1023 x 1023, Crank-Nicolson with the second-order weights (Sections
    1.3-1.4), P_F with the symbols q_a, q_b: one step mirrored by the oracle."""
    fde = need_gpu()
    p = fi.variable_2d(n=1023, steps=1)
    p.weights, p.time = "weighted", "cn"
    w = _workers()
    s = FDESystem.from_problem(p, workers=w)
    P = pc.make("tau", s, workers=w)
    u0 = p.u0.reshape(-1)
    b = s.rhs(u0)

    def orun(maxit):
        x, i = krylov.fgmres(s.matvec, b, P, x0=u0, restart=30, tol=p.tol, maxit=maxit or 100000)
        return x, i["iters"]

    def grun(maxit):
        with fde.Plan(p, maxit=maxit) as q:
            x = dev(u0)
            i = q.solve(dev(b), x, allow_notconv=True)
            return host(x), i.iters

    with fde.Plan(p) as plan:
        bd = torch.empty(p.N, dtype=torch.float64, device="cuda")
        plan.rhs(dev(u0), bd)
        assert relerr(host(bd), b) < 1e-12
        x = dev(u0)
        info = plan.solve(dev(b), x)
        xg = host(x)
    assert info.converged
    mirror_check(xg, info.iters, orun, grun)


def test_full_mixed_forward_error(full):
    """Headline mixed form (float32 inner GMRES(16), float64 outer FGMRES(30))
    at the outer tolerance the benchmark uses for the stated accuracy: relative
    error <= 1e-8 against the step solved by the oracle to a true residual of
    1e-12."""
    fde = need_gpu()
    from test_gpu_mixed import ACC_TOL
    p, s, P, u0, b = full["p"], full["s"], full["P"], full["u0"], full["b"]
    xr, ir = krylov.fgmres(s.matvec, b, P, x0=full["xo"], restart=30, tol=1e-12)
    assert ir["converged"]
    with fde.Plan(p, precision=fde.MIXED, inner_steps=16, tol=ACC_TOL) as plan:
        x = dev(u0)
        info = plan.solve(dev(b), x)
        xg = host(x)
    assert info.converged
    assert relerr(xg, xr) <= 1e-8, relerr(xg, xr)

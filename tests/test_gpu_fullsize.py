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
from gpu_util import dev, host, need_gpu, relerr, torch
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

"""1D lines longer than one workgroup (n + 1 > 4096): four-step FFT path,
parity with the oracle, up to the full size of the 1D variable-coefficient
workload (n = 65535)."""
import numpy as np
import pytest

import fde_inputs as fi
from gpu_util import dev, host, need_gpu, relerr, torch
from oracle import krylov, precond as pc
from oracle.system import FDESystem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,weights,time", [(n, w, t) for n in (8191, 65535, 262143)
                                             for w, t in (("shifted", "euler"), ("weighted", "cn"))]
                         + [(2097151, "shifted", "euler"), (4194303, "weighted", "cn")])
def test_big_matvec_and_tau(n, weights, time):
    fde = need_gpu()
    p = fi.variable_1d(n=n, alpha=1.37, seed=n)
    p.weights, p.time = weights, time
    s = FDESystem.from_problem(p)
    x = np.random.default_rng(1).uniform(-1, 1, n)
    with fde.Plan(p) as plan:
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        plan.matvec(dev(x), y)
        assert relerr(host(y), s.matvec(x)) < 1e-12
        for dside in ("left",):
            plan.tau_apply(dev(x), y)
            assert relerr(host(y), pc.make("tau", s, dside=dside)(x)) < 1e-12
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        plan.rhs(dev(x), b)
        assert relerr(host(b), s.rhs(x)) < 1e-12


@pytest.mark.parametrize("alpha", [1.8, 1.5])
def test_big_fgmres_full_size(alpha):
    """First implicit-Euler step of the 1D variable-coefficient workload,
    n = 65535, GMRES(30) + P_F to 1e-8, mirrored by the oracle."""
    fde = need_gpu()
    p = fi.variable_1d(n=65535, alpha=alpha)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    xo, io = krylov.fgmres(s.matvec, b, pc.make("tau", s), x0=p.u0, restart=30, tol=1e-8)
    with fde.Plan(p) as plan:
        x = dev(p.u0)
        ig = plan.solve(dev(b), x)
        xg = host(x)
    assert ig.converged and io["converged"]
    assert abs(ig.iters - io["iters"]) <= max(1, 0.005 * io["iters"]), (ig.iters, io["iters"])
    assert relerr(s.matvec(xg), b) <= 1e-8 * (1 + 1e-6)
    if ig.iters == io["iters"]:
        assert relerr(xg, xo) < 1e-10


def test_big_mixed_full_size():
    fde = need_gpu()
    p = fi.variable_1d(n=65535, alpha=1.5)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    xo, io = krylov.fgmres(s.matvec, b, pc.make("tau", s), x0=p.u0, restart=30, tol=1e-8)
    with fde.Plan(p, precision=fde.MIXED) as plan:
        x = dev(p.u0)
        ig = plan.solve(dev(b), x)
        xg = host(x)
    assert ig.converged
    assert relerr(s.matvec(xg), b) <= 1e-8 * (1 + 1e-6)   # FP64 true residual, checked by the oracle
    assert relerr(xg, xo) < 1e-6

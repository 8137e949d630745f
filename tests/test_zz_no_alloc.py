"""The allocation-free entry point fde_pcg1d_solve_noalloc (workspace in a
static device array) against the plan path fde_assemble + fde_solve on the
same inputs: same iteration count, same solution (relative 1e-10), on two
calls in a row with the second on a smaller line, and no device memory taken
by the second call."""
import numpy as np
import pytest

import fde_inputs as fi
from gpu_util import dev, host, need_gpu, relerr, torch

pytestmark = pytest.mark.gpu


def const_problem(n, alpha, d, seed):
    p = fi.constant_1d(n=n, alpha=alpha, seed=seed)
    p.dplus = np.full(n, d)
    p.dminus = np.full(n, d)
    return p


def plan_solve(fde, p, x0, **kw):
    with fde.Plan(p, **kw) as plan:
        x = dev(x0)
        info = plan.solve(dev(p.b), x)
        return host(x), info


def noalloc_solve(fde, p, x0, **kw):
    params = fde.params_for(p, **kw)
    x = dev(x0)
    info = fde.fde_pcg1d_solve_noalloc(params, dev(p.dplus), dev(p.dminus), dev(p.b), x)
    return host(x), info


@pytest.mark.parametrize("kind", ["tau", "tau_hat", "tilde"])
def test_noalloc_matches_plan_two_calls(kind):
    fde = need_gpu()
    prec = {"tau": fde.P_TAU, "tau_hat": fde.P_TAU_HAT, "tilde": fde.P_TILDE}[kind]
    cases = [const_problem(4095, 1.5, 1.3, 1), const_problem(1023, 1.7, 1.0, 2)]   # second call smaller
    if kind == "tilde":
        for p in cases:   # variable coefficients are allowed for P_tilde (PCG needs d+ = d-)
            x = np.linspace(0.1, 1.9, p.n[0])
            p.dplus = 1.0 + 0.5 * x
            p.dminus = p.dplus.copy()
    free = []
    for p in cases:
        x0 = np.random.default_rng(p.n[0]).uniform(-1, 1, p.n[0])
        xr, ir = plan_solve(fde, p, x0, prec=prec)
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
        xs, is_ = noalloc_solve(fde, p, x0, prec=prec)
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
        assert is_.converged and ir.converged
        assert is_.iters == ir.iters, (is_.iters, ir.iters)
        assert relerr(xs, xr) < 1e-10
        assert is_.relres_true <= p.tol
    # the second (smaller) call took no device memory
    assert free[3] >= free[2]


def test_noalloc_rejects_what_it_does_not_cover():
    fde = need_gpu()
    p = const_problem(8191, 1.5, 1.0, 3)   # line longer than one workgroup
    with pytest.raises(fde.FdeError) as e:
        noalloc_solve(fde, p, np.zeros(p.n[0]))
    assert e.value.status == fde.FDE_EUNSUPPORTED
    q = fi.variable_1d(n=255, steps=1)      # FGMRES configuration
    q.b = np.ones(255)
    with pytest.raises(fde.FdeError) as e:
        noalloc_solve(fde, q, np.zeros(255))
    assert e.value.status == fde.FDE_EUNSUPPORTED

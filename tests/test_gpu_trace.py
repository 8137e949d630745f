"""The residual-history trace (FDE_TRACE): one line per iteration with the
solver's residual estimate and one per true-residual check.  The FGMRES and
multi-kernel PCG histories are compared with the oracle's estimates of the
same solve, iteration by iteration."""
import os

import numpy as np
import pytest

import fde_inputs as fi
from gpu_util import dev, need_gpu
from oracle import krylov, precond as pc
from oracle.system import FDESystem

pytestmark = pytest.mark.gpu


def parse(path):
    """{solve id: {"solver": str, "est": [(iter, relres)], "true": [(iter, relres)]}}."""
    out = {}
    with open(path) as f:
        for line in f:
            if not line.startswith("fde_trace "):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            d = out.setdefault(int(kv["solve"]), {"solver": kv["solver"], "est": [], "true": []})
            d[kv["kind"]].append((int(kv["iter"]), float(kv["relres"])))
    return out


def traced_solve(fde, p, b, x0, path, **kw):
    os.environ["FDE_TRACE"] = str(path)
    try:
        with fde.Plan(p, **kw) as plan:
            x = dev(x0)
            info = plan.solve(dev(b), x)
    finally:
        del os.environ["FDE_TRACE"]
    runs = parse(path)
    assert len(runs) == 1
    return info, next(iter(runs.values()))


def compare_history(gpu, oracle, iters_g, iters_o):
    """Iteration counts within one; the estimates agree to 1e-6 relative over
    the common iterations (they are formed from the same Givens sines up to
    rounding)."""
    assert abs(iters_g - iters_o) <= 1, (iters_g, iters_o)
    m = min(len(gpu), len(oracle))
    g, o = np.array(gpu[:m]), np.array(oracle[:m])
    assert np.all(np.abs(g - o) <= 1e-6 * o), np.abs(g / o - 1).max()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fgmres_history_2d(tmp_path, precision):
    fde = need_gpu()
    p = fi.variable_2d(n=63, n2=63, seed=8, steps=1)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    prec = fde.FP64 if precision == "fp64" else fde.MIXED
    info, tr = traced_solve(fde, p, b, p.u0, tmp_path / "t.txt", restart=10, precision=prec)
    assert tr["solver"] == "gmres"
    est = tr["est"]
    assert [i for i, _ in est] == list(range(1, info.iters + 1))
    assert est[-1][1] == pytest.approx(info.relres_est, rel=1e-14)
    # a true-residual line at the start and after every cycle
    assert tr["true"][0][0] == 0 and len(tr["true"]) == info.restarts + 2
    assert tr["true"][-1] == (info.iters, pytest.approx(info.relres_true, rel=1e-14))
    if precision == "fp64":
        _, io = krylov.fgmres(s.matvec, b, pc.make("tau", s), x0=p.u0, restart=10, tol=p.tol, history=True)
        compare_history([v for _, v in est], io["hist"], info.iters, io["iters"])
    else:
        # the flexible outer loop with a float32 preconditioner: the estimates
        # still fall to the tolerance, and each cycle's true residual is within
        # a few percent of the estimate it ended on
        assert est[-1][1] <= p.tol
        ends = {i: v for i, v in est}
        for i, v in tr["true"][1:]:
            assert abs(v - ends[i]) <= 0.05 * ends[i] + 1e-3 * p.tol


def test_fgmres_history_1d_restarts(tmp_path):
    fde = need_gpu()
    p = fi.variable_1d(n=1023, alpha=1.3, seed=5, steps=1)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    info, tr = traced_solve(fde, p, b, p.u0, tmp_path / "t.txt", restart=5)
    assert info.restarts >= 2
    _, io = krylov.fgmres(s.matvec, b, pc.make("tau", s), x0=p.u0, restart=5, tol=p.tol, history=True)
    compare_history([v for _, v in tr["est"]], io["hist"], info.iters, io["iters"])


def test_pcg_history_multikernel(tmp_path):
    """n = 8191 runs the multi-kernel PCG loop: one estimate per iteration."""
    fde = need_gpu()
    n = 8191
    p = fi.constant_1d(n=n, alpha=1.5, seed=n)
    s = FDESystem.from_problem(p)
    x0 = np.zeros(n)
    info, tr = traced_solve(fde, p, p.b, x0, tmp_path / "t.txt")
    assert tr["solver"] == "pcg"
    assert [i for i, _ in tr["est"]] == list(range(1, info.iters + 1))
    _, io = krylov.pcg(s.matvec, p.b, pc.make("tau", s), x0=x0, tol=1e-10, history=True)
    compare_history([v for _, v in tr["est"]], io["hist"], info.iters, io["iters"])
    assert tr["true"][-1] == (info.iters, pytest.approx(info.relres_true, rel=1e-14))


def test_pcg_history_one_workgroup(tmp_path):
    """The one-workgroup PCG solve reports its final estimate and true residual."""
    fde = need_gpu()
    p = fi.constant_1d(n=1023)
    info, tr = traced_solve(fde, p, p.b, np.zeros(p.N), tmp_path / "t.txt")
    assert tr["est"] == [(info.iters, pytest.approx(info.relres_est, rel=1e-14))]
    assert tr["true"] == [(info.iters, pytest.approx(info.relres_true, rel=1e-14))]


def test_trace_off_writes_nothing(tmp_path):
    fde = need_gpu()
    p = fi.constant_1d(n=255)
    path = tmp_path / "t.txt"
    os.environ.pop("FDE_TRACE", None)
    with fde.Plan(p) as plan:
        plan.solve(dev(p.b), dev(np.zeros(p.N)))
    assert not path.exists()
    os.environ["FDE_TRACE"] = "0"
    try:
        with fde.Plan(p) as plan:
            plan.solve(dev(p.b), dev(np.zeros(p.N)))
    finally:
        del os.environ["FDE_TRACE"]
    assert not path.exists()

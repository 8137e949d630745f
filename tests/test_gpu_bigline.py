"""1D lines longer than one workgroup (n + 1 > 4096): four-step FFT path,
parity with the oracle, up to the full size of the 1D variable-coefficient
workload (n = 65535)."""
import numpy as np
import pytest

import fde_inputs as fi
from gpu_util import dev, host, mirror_check, need_gpu, relerr, torch
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


@pytest.mark.parametrize("alpha", [1.8, 1.5, 1.2])
def test_big_fgmres_full_size(alpha):
    """First implicit-Euler step of the 1D variable-coefficient workload,
    n = 65535, GMRES(30) + P_F to 1e-8, mirrored by the oracle (iterations
    within one, iterates at equal step count within 1e-10)."""
    fde = need_gpu()
    p = fi.variable_1d(n=65535, alpha=alpha)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    P = pc.make("tau", s)

    def orun(maxit):
        x, info = krylov.fgmres(s.matvec, b, P, x0=p.u0, restart=30, tol=1e-8, maxit=maxit or 100000)
        return x, info["iters"]

    def grun(maxit):
        with fde.Plan(p, maxit=maxit) as plan:
            x = dev(p.u0)
            info = plan.solve(dev(b), x, allow_notconv=True)
            return host(x), info.iters

    with fde.Plan(p) as plan:
        x = dev(p.u0)
        ig = plan.solve(dev(b), x)
        xg = host(x)
    assert ig.converged
    mirror_check(xg, ig.iters, orun, grun)
    assert relerr(s.matvec(xg), b) <= 1e-8 * (1 + 1e-6)


def test_big_mixed_full_size():
    """Mixed form at n = 65535: float64 true residual within the tolerance
    (recomputed by the oracle) and Varah's bound against the oracle's float64
    solution (every row of the first-order M is diagonally dominant by nu)."""
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
    rg, ro = b - s.matvec(xg), b - s.matvec(xo)
    assert np.linalg.norm(rg) <= 1e-8 * (1 + 1e-6) * np.linalg.norm(b)
    assert np.abs(xg - xo).max() <= (np.abs(rg).max() + np.abs(ro).max()) / s.nu


# ---------------------------------------------------------------------------
# 1D lines whose n + 1 is not a power of two: the chirp-z DST and a padded
# Toeplitz embedding on the four-step path.
# ---------------------------------------------------------------------------
CHIRP_SIZES = [2, 5, 100, 1000, 3000, 5000, 12345, 40000, 65000]


@pytest.mark.parametrize("n", CHIRP_SIZES)
@pytest.mark.parametrize("weights,time", [("shifted", "euler"), ("weighted", "cn")])
def test_chirp_matvec_tau_rhs(n, weights, time):
    fde = need_gpu()
    p = fi.variable_1d(n=n, alpha=1.37, seed=n + 1)
    p.weights, p.time = weights, time
    s = FDESystem.from_problem(p)
    x = np.random.default_rng(n).uniform(-1, 1, n)
    with fde.Plan(p) as plan, fde.Plan(p, dside=fde.D_RIGHT) as planr:
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        plan.matvec(dev(x), y)
        assert relerr(host(y), s.matvec(x)) < 1e-12
        for pl, dside in ((plan, "left"), (planr, "right")):
            pl.tau_apply(dev(x), y)
            assert relerr(host(y), pc.make("tau", s, dside=dside)(x)) < 1e-12, dside
        plan.rhs(dev(x), y)
        assert relerr(host(y), s.rhs(x)) < 1e-12


@pytest.mark.parametrize("n,alpha", [(100, 1.5), (3000, 1.3), (40000, 1.8)])
def test_chirp_fgmres(n, alpha):
    """FGMRES(30) + P_F on lines with arbitrary n, mirrored by the oracle."""
    fde = need_gpu()
    p = fi.variable_1d(n=n, alpha=alpha, seed=n)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    P = pc.make("tau", s)

    def orun(maxit):
        x, info = krylov.fgmres(s.matvec, b, P, x0=p.u0, restart=30, tol=1e-8, maxit=maxit or 100000)
        return x, info["iters"]

    def grun(maxit):
        with fde.Plan(p, maxit=maxit) as plan:
            x = dev(p.u0)
            info = plan.solve(dev(b), x, allow_notconv=True)
            return host(x), info.iters

    with fde.Plan(p) as plan:
        x = dev(p.u0)
        ig = plan.solve(dev(b), x)
        xg = host(x)
    assert ig.converged
    mirror_check(xg, ig.iters, orun, grun)


@pytest.mark.parametrize("kind,n", [("tau_hat", 5000), ("tilde", 1000)])
def test_chirp_pcg_other_preconditioners(kind, n):
    """PCG with P_hat (Case I, a few iterations) and the unshifted P_tilde
    (tens of iterations: at n = 5000 the two sides' counts already drift by
    two, so it runs at n = 1000)."""
    fde = need_gpu()
    p = fi.constant_1d(n=n, alpha=1.6, seed=3)
    p.dplus = np.full(n, 1.3)
    p.dminus = np.full(n, 1.3)
    s = FDESystem.from_problem(p)
    xo, io = krylov.pcg(s.matvec, p.b, pc.make(kind, s), tol=1e-10)
    prec = fde.P_TAU_HAT if kind == "tau_hat" else fde.P_TILDE
    with fde.Plan(p, prec=prec) as plan:
        x = dev(np.zeros(n))
        ig = plan.solve(dev(p.b), x)
        xg = host(x)
    assert ig.converged and io["converged"]
    assert abs(ig.iters - io["iters"]) <= 1, (ig.iters, io["iters"])
    assert relerr(xg, xo) < 1e-10


def test_chirp_mixed():
    """Mixed form on a chirp-z line (float32 chirp-z transforms): float64 true
    residual within the tolerance, Varah's bound against the oracle."""
    fde = need_gpu()
    p = fi.variable_1d(n=20000, alpha=1.5, seed=9)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    xo, io = krylov.fgmres(s.matvec, b, pc.make("tau", s), x0=p.u0, restart=30, tol=1e-8)
    for inner in (0, 8):
        with fde.Plan(p, precision=fde.MIXED, inner_steps=inner) as plan:
            x = dev(p.u0)
            ig = plan.solve(dev(b), x)
            xg = host(x)
        assert ig.converged
        rg, ro = b - s.matvec(xg), b - s.matvec(xo)
        assert np.linalg.norm(rg) <= 1e-8 * (1 + 1e-6) * np.linalg.norm(b)
        assert np.abs(xg - xo).max() <= (np.abs(rg).max() + np.abs(ro).max()) / s.nu

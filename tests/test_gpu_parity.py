"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Transforms must agree to a few ulps times log n
(relative 1e-12); FP64 solves mirror the oracle's build-mode FGMRES / PCG to a
relative 1e-10 with iteration counts within one."""
import math

import numpy as np
import pytest

import fde_inputs as fi
from gpu_util import dev, host, mirror_check, need_gpu, relerr, torch
from oracle import krylov, precond as pc
from oracle.system import FDESystem

pytestmark = pytest.mark.gpu

SHAPES_1D = [1, 3, 7, 15, 63, 255, 1023, 4095]
SHAPES_2D = [(7, 3), (15, 31), (63, 63), (127, 255), (255, 127), (3, 1023), (15, 4095)]


def prob1d(n, alpha=1.37, weights="shifted", time="euler", seed=11):
    p = fi.variable_1d(n=n, alpha=alpha, seed=seed, steps=1)
    p.weights, p.time = weights, time
    return p


def prob2d(n1, n2, ax=1.7, ay=1.4, weights="shifted", time="euler", seed=12):
    p = fi.variable_2d(n=n1, n2=n2, ax=ax, ay=ay, seed=seed, steps=1)
    p.weights, p.time = weights, time
    return p


def rng_vec(N, seed):
    return np.random.default_rng(seed).uniform(-1, 1, N)


@pytest.mark.parametrize("n", SHAPES_1D)
@pytest.mark.parametrize("weights,time", [("shifted", "euler"), ("weighted", "cn")])
def test_matvec_1d(n, weights, time):
    fde = need_gpu()
    p = prob1d(n, weights=weights, time=time)
    s = FDESystem.from_problem(p)
    x = rng_vec(s.N, n)
    with fde.Plan(p) as plan:
        y = torch.empty(s.N, dtype=torch.float64, device="cuda")
        plan.matvec(dev(x), y)
        assert relerr(host(y), s.matvec(x)) < 1e-12


@pytest.mark.parametrize("n1,n2", SHAPES_2D + [(1, 1), (3, 7)])
@pytest.mark.parametrize("weights,time", [("shifted", "euler"), ("weighted", "cn")])
def test_matvec_2d(n1, n2, weights, time):
    fde = need_gpu()
    p = prob2d(n1, n2, weights=weights, time=time)
    s = FDESystem.from_problem(p)
    x = rng_vec(s.N, n1 * 7 + n2)
    with fde.Plan(p) as plan:
        y = torch.empty(s.N, dtype=torch.float64, device="cuda")
        plan.matvec(dev(x), y)
        assert relerr(host(y), s.matvec(x)) < 1e-12


@pytest.mark.parametrize("n", SHAPES_1D)
@pytest.mark.parametrize("dside", ["left", "right"])
def test_tau_1d(n, dside):
    fde = need_gpu()
    p = prob1d(n)
    s = FDESystem.from_problem(p)
    P = pc.make("tau", s, dside=dside)
    v = rng_vec(s.N, 3 * n)
    with fde.Plan(p, dside=fde.D_LEFT if dside == "left" else fde.D_RIGHT) as plan:
        z = torch.empty(s.N, dtype=torch.float64, device="cuda")
        plan.tau_apply(dev(v), z)
        assert relerr(host(z), P(v)) < 1e-12


@pytest.mark.parametrize("n1,n2", SHAPES_2D)
@pytest.mark.parametrize("dside", ["left", "right"])
@pytest.mark.parametrize("weights", ["shifted", "weighted"])
def test_tau_2d(n1, n2, dside, weights):
    """2D P_F: symbol p_a (first-order weights) or q_a (second-order weights,
    eq. second_order_symbol) sampled on both axes, with D on either side."""
    fde = need_gpu()
    p = prob2d(n1, n2, weights=weights, time="cn" if weights == "weighted" else "euler")
    s = FDESystem.from_problem(p)
    P = pc.make("tau", s, dside=dside)
    v = rng_vec(s.N, 5 * n1 + n2)
    with fde.Plan(p, dside=fde.D_LEFT if dside == "left" else fde.D_RIGHT) as plan:
        z = torch.empty(s.N, dtype=torch.float64, device="cuda")
        plan.tau_apply(dev(v), z)
        assert relerr(host(z), P(v)) < 1e-12


@pytest.mark.parametrize("kind", ["tau_hat", "tilde", "none", "tau_shift"])
def test_tau_variants(kind):
    fde = need_gpu()
    if kind == "tau_hat":
        p = fi.constant_1d(n=255)
        pk = dict(prec=fde.P_TAU_HAT)
    elif kind == "tilde":
        p = prob1d(255)
        pk = dict(prec=fde.P_TILDE)
    elif kind == "none":
        p = prob2d(31, 15)
        pk = dict(prec=fde.P_NONE)
    else:
        p = prob2d(31, 15)
        pk = dict(shift=0.37)
    s = FDESystem.from_problem(p)
    P = pc.make(kind if kind != "tau_shift" else "tau", s, shift=0.37 if kind == "tau_shift" else None) \
        if kind not in ("tau_hat", "tilde", "none") else pc.make(kind, s)
    v = rng_vec(s.N, 99)
    with fde.Plan(p, **pk) as plan:
        z = torch.empty(s.N, dtype=torch.float64, device="cuda")
        plan.tau_apply(dev(v), z)
        assert relerr(host(z), P(v)) < 1e-12


def test_tau_hat_2d_constant():
    fde = need_gpu()
    n1, n2 = 63, 31
    x, _ = fi.grid(n1, 0, 2)
    y, _ = fi.grid(n2, 0, 2)
    p = prob2d(n1, n2)
    p.dplus = np.full((n2, n1), 1.3)
    p.dminus = np.full((n2, n1), 1.3)
    p.eplus = np.full((n2, n1), 0.6)
    p.eminus = np.full((n2, n1), 0.6)
    s = FDESystem.from_problem(p)
    P = pc.make("tau_hat", s)
    v = rng_vec(s.N, 5)
    with fde.Plan(p, prec=fde.P_TAU_HAT) as plan:
        z = torch.empty(s.N, dtype=torch.float64, device="cuda")
        plan.tau_apply(dev(v), z)
        assert relerr(host(z), P(v)) < 1e-12


@pytest.mark.parametrize("time", ["euler", "cn"])
def test_rhs(time):
    fde = need_gpu()
    p = prob2d(63, 31, weights="weighted" if time == "cn" else "shifted", time=time)
    s = FDESystem.from_problem(p)
    u = rng_vec(s.N, 1)
    f = rng_vec(s.N, 2)
    with fde.Plan(p) as plan:
        b = torch.empty(s.N, dtype=torch.float64, device="cuda")
        plan.rhs(dev(u), b, f=dev(f))
        assert relerr(host(b), s.rhs(u, f)) < 1e-12
        plan.rhs(dev(u), b)
        assert relerr(host(b), s.rhs(u)) < 1e-12


# ---------------------------------------------------------------------------
# Solves
# ---------------------------------------------------------------------------
def oracle_solve(p, b, x0, dside="left", restart=30, tol=1e-8, solver="gmres"):
    s = FDESystem.from_problem(p)
    P = pc.make("tau", s, dside=dside)
    if solver == "pcg":
        return krylov.pcg(s.matvec, b, P, x0=x0, tol=tol)
    return krylov.fgmres(s.matvec, b, P, x0=x0, restart=restart, tol=tol)


def gpu_solve(fde, p, b, x0, allow_notconv=False, **kw):
    with fde.Plan(p, **kw) as plan:
        x = dev(x0)
        info = plan.solve(dev(b), x, allow_notconv=allow_notconv)
        return host(x), info


def mirror(fde, p, b, x0, xg, ig, kind="tau", dside="left", restart=30, tol=1e-8, gpu_kw=None):
    """mirror_check for an FGMRES solve: the oracle's build-mode FGMRES with
    preconditioner `kind`, and a GPU rerun with an iteration cap."""
    s = FDESystem.from_problem(p)
    P = pc.make(kind, s, dside=dside)
    gk = dict(gpu_kw or {})

    def orun(maxit):
        x, info = krylov.fgmres(s.matvec, b, P, x0=x0, restart=restart, tol=tol,
                                maxit=maxit if maxit else 100000)
        if not maxit:
            assert info["converged"]
        return x, info["iters"]

    def grun(maxit):
        x, info = gpu_solve(fde, p, b, x0, allow_notconv=True, maxit=maxit, restart=restart, **gk)
        assert info.iters == maxit
        return x, info.iters

    return mirror_check(xg, ig.iters, orun, grun)


@pytest.mark.parametrize("n,alpha,restart", [(7, 1.5, 30), (63, 1.2, 30), (255, 1.5, 30), (1023, 1.8, 30),
                                              (4095, 1.3, 30), (7, 1.5, 5), (63, 1.2, 5), (255, 1.5, 5),
                                              (1023, 1.8, 5)])
def test_fgmres_1d(n, alpha, restart):
    fde = need_gpu()
    p = fi.variable_1d(n=n, alpha=alpha, seed=n)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    xg, ig = gpu_solve(fde, p, b, p.u0, restart=restart)
    assert ig.converged
    mirror(fde, p, b, p.u0, xg, ig, restart=restart)
    assert ig.relres_true <= 1e-8
    assert relerr(s.matvec(xg), b) <= 1e-8 * (1 + 1e-6)


@pytest.mark.parametrize("n1,n2", [(15, 15), (63, 31), (127, 127), (255, 255)])
@pytest.mark.parametrize("dside", ["left", "right"])
def test_fgmres_2d(n1, n2, dside):
    fde = need_gpu()
    p = fi.variable_2d(n=n1, n2=n2, seed=n1 + n2)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0.reshape(-1))
    x0 = p.u0.reshape(-1)
    dk = dict(dside=fde.D_LEFT if dside == "left" else fde.D_RIGHT)
    xg, ig = gpu_solve(fde, p, b, x0, **dk)
    assert ig.converged
    mirror(fde, p, b, x0, xg, ig, dside=dside, gpu_kw=dk)
    assert relerr(s.matvec(xg), b) <= 1e-8 * (1 + 1e-6)


@pytest.mark.parametrize("n1,n2", [(15, 15), (63, 63), (255, 255), (127, 31)])
def test_fgmres_2d_cn_second_order(n1, n2):
    """2D Crank-Nicolson with the second-order weights (Sections 1.3-1.4,
    eq. coef:2d): one step of the headline coefficient fields, P_F with the
    symbol q_a (eq. second_order_symbol), mirrored by the oracle."""
    fde = need_gpu()
    p = prob2d(n1, n2, weights="weighted", time="cn", seed=n1 * 3 + n2)
    s = FDESystem.from_problem(p)
    x0 = p.u0.reshape(-1)
    b = s.rhs(x0)
    xg, ig = gpu_solve(fde, p, b, x0)
    assert ig.converged
    mirror(fde, p, b, x0, xg, ig)
    assert relerr(s.matvec(xg), b) <= 1e-8 * (1 + 1e-6)


@pytest.mark.parametrize("example", [2, 3])
@pytest.mark.parametrize("n", [15, 16, 31, 32])
def test_paper_examples_2d_steps(example, n):
    """Examples 2 and 3 of Section 4 (second-order weights, Crank-Nicolson,
    h_t = 1/n, the paper's source term) on the GPU: every step's right-hand
    side and solve mirror the oracle from the GPU's previous state (P_F with D
    on the right, as Tables 3-4, GMRES tolerance 1e-7, x0 = u^{m-1}); the
    error at T = 1 falls by about four per halving of h (second order)."""
    fde = need_gpu()
    p = fi.paper_2d(n, example)
    s = FDESystem.from_problem(p)
    X, Y = p.meta["X"], p.meta["Y"]
    a, bt = p.alpha
    u = p.u0.reshape(-1)
    dk = dict(dside=fde.D_RIGHT, tol=p.tol)
    with fde.Plan(p, **dk) as plan:
        bd = torch.empty(p.N, dtype=torch.float64, device="cuda")
        for m in range(1, p.steps + 1):
            f = fi.example23_source(X, Y, (m - 0.5) * p.dt, a, bt).reshape(-1)
            plan.rhs(dev(u), bd, f=dev(f))
            b = host(bd)
            assert relerr(b, s.rhs(u, f)) < 1e-12
            x = dev(u)
            ig = plan.solve(bd, x)
            xg = host(x)
            if m in (1, p.steps // 2, p.steps):
                mirror(fde, p, b, u, xg, ig, dside="right", tol=p.tol, gpu_kw=dk)
            u = xg
    err = np.abs(u - fi.example23_exact(X, Y, p.steps * p.dt).reshape(-1)).max()
    # max error at T = 1 of the second-order scheme (Section 4): about 1.0e-1 at n = 15, 16 and
    # 2.6e-2 at n = 31, 32 (oracle at the paper's n = 16, 32: 9.37e-2, 2.47e-2 for Example 2)
    assert err < {15: 0.12, 16: 0.11, 31: 0.03, 32: 0.028}[n], err


def test_fgmres_many_restarts():
    """GMRES(5) on n = 4095, alpha = 1.3 needs about a thousand iterations
    (over 200 restarts).  The two sides follow the same iterates: after a
    fixed number of steps (no early stop) they agree to 1e-10.  Where the
    residual curve flattens near the tolerance, a rounding-level change of the
    input moves the stopping step of the oracle itself by several steps; the
    stopping steps are compared against that measured spread, and the final
    solutions against Varah's bound (every row of M is diagonally dominant by
    at least nu), which holds for any two solutions meeting the tolerance."""
    fde = need_gpu()
    p = fi.variable_1d(n=4095, alpha=1.3, seed=4095)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    P = pc.make("tau", s)
    for k in (25, 100):
        xo, io = krylov.fgmres(s.matvec, b, P, x0=p.u0, restart=5, tol=1e-300, maxit=k)
        xg, ig = gpu_solve(fde, p, b, p.u0, allow_notconv=True, restart=5, tol=1e-300, maxit=k)
        assert ig.iters == io["iters"] == k
        assert relerr(xg, xo) < 1e-10, (k, relerr(xg, xo))
    xo, io = oracle_solve(p, b, p.u0, restart=5)
    xg, ig = gpu_solve(fde, p, b, p.u0, restart=5)
    assert ig.converged and io["converged"]
    its = []
    for seed in range(3):
        e = np.random.default_rng(seed).uniform(-1, 1, b.size) * 2.0 ** -52
        its.append(krylov.fgmres(s.matvec, b * (1 + e), P, x0=p.u0, restart=5, tol=1e-8)[1]["iters"])
    spread = max(abs(i - io["iters"]) for i in its)
    assert abs(ig.iters - io["iters"]) <= max(1, spread), (ig.iters, io["iters"], its)
    rg, ro = b - s.matvec(xg), b - s.matvec(xo)
    assert np.linalg.norm(rg) <= 1e-8 * (1 + 1e-6) * np.linalg.norm(b)
    assert np.abs(xg - xo).max() <= (np.abs(rg).max() + np.abs(ro).max()) / s.nu


def test_pcg_constant_1d_full_size():
    """1D constant coefficients, n = 1023, alpha = 1.5, dt = h, PCG with the
    Case I shifted tau preconditioner to 1e-10."""
    fde = need_gpu()
    p = fi.constant_1d()
    xo, io = oracle_solve(p, p.b, np.zeros(p.N), tol=1e-10, solver="pcg")
    xg, ig = gpu_solve(fde, p, p.b, np.zeros(p.N))
    assert ig.converged and io["converged"]
    assert abs(ig.iters - io["iters"]) <= 1, (ig.iters, io["iters"])
    assert relerr(xg, xo) < 1e-10


def const_problem(n, alpha, d):
    p = fi.constant_1d(n=n, alpha=alpha, seed=n)
    p.dplus = np.full(n, d)
    p.dminus = np.full(n, d)
    return p


@pytest.mark.parametrize("n,alpha", [(7, 1.5), (15, 1.9), (31, 1.5), (63, 1.2), (127, 1.6), (511, 1.7),
                                     (2047, 1.5), (4095, 1.3), (8191, 1.5)])
@pytest.mark.parametrize("d", [1.0, 1.3])
def test_pcg_constant_1d_sizes(n, alpha, d):
    """PCG + P_F on constant coefficients from a nonzero start, to 1e-10.
    n + 1 <= 4096 runs the whole solve in one workgroup,
    n = 8191 the multi-kernel loop; both take the oracle's PCG steps."""
    fde = need_gpu()
    p = const_problem(n, alpha, d)
    x0 = np.random.default_rng(n).uniform(-1, 1, n)
    xo, io = oracle_solve(p, p.b, x0, tol=1e-10, solver="pcg")
    xg, ig = gpu_solve(fde, p, p.b, x0)
    assert ig.converged and io["converged"]
    assert abs(ig.iters - io["iters"]) <= 1, (ig.iters, io["iters"])
    assert relerr(xg, xo) < 1e-10
    s = FDESystem.from_problem(p)
    assert relerr(s.matvec(xg), p.b) <= 1e-10 * (1 + 1e-6)


@pytest.mark.parametrize("kind", ["tau_hat", "tilde"])
def test_pcg_other_preconditioners(kind):
    fde = need_gpu()
    p = const_problem(1023, 1.6, 1.3)
    s = FDESystem.from_problem(p)
    xo, io = krylov.pcg(s.matvec, p.b, pc.make(kind, s), tol=1e-10)
    prec = fde.P_TAU_HAT if kind == "tau_hat" else fde.P_TILDE
    xg, ig = gpu_solve(fde, p, p.b, np.zeros(p.N), prec=prec)
    assert ig.converged and io["converged"]
    assert abs(ig.iters - io["iters"]) <= 1, (ig.iters, io["iters"])
    assert relerr(xg, xo) < 1e-10


@pytest.mark.parametrize("n", [255, 8191])
def test_pcg_maxit_and_repeat(n):
    """The iteration cap stops PCG with FDE_ENOTCONV and the oracle's iterate
    after that many steps; a second solve on the same plan repeats the first
    bit for bit."""
    fde = need_gpu()
    p = const_problem(n, 1.5, 1.0)
    s = FDESystem.from_problem(p)
    xo, io = krylov.pcg(s.matvec, p.b, pc.make("tau", s), tol=1e-10, maxit=3)
    with fde.Plan(p, maxit=3) as plan:
        runs = []
        for _ in range(2):
            x = dev(np.zeros(n))
            info = plan.solve(dev(p.b), x, allow_notconv=True)
            runs.append((host(x), info.iters, info.converged))
    for xg, iters, conv in runs:
        assert iters == 3 and not conv
        assert relerr(xg, xo) < 1e-10
    assert np.array_equal(runs[0][0], runs[1][0])


@pytest.mark.parametrize("n", [63, 8191])
def test_pcg_zero_rhs_and_nonfinite(n):
    """PCG (one workgroup at n = 63, multi-kernel at n = 8191): b = 0 gives
    x = 0 in no iterations; a NaN in b or an Inf in x0 is FDE_ENONFINITE."""
    fde = need_gpu()
    p = const_problem(n, 1.5, 1.0)
    with fde.Plan(p) as plan:
        x = dev(np.ones(n))
        info = plan.solve(dev(np.zeros(n)), x)
        assert info.iters == 0 and info.converged
        assert np.all(host(x) == 0)
        b = p.b.copy()
        b[5] = np.nan
        with pytest.raises(fde.FdeError) as e:
            plan.solve(dev(b), dev(np.zeros(n)))
        assert e.value.status == fde.FDE_ENONFINITE
        x0 = np.zeros(n)
        x0[3] = np.inf
        with pytest.raises(fde.FdeError) as e:
            plan.solve(dev(p.b), dev(x0))
        assert e.value.status == fde.FDE_ENONFINITE
        x = dev(np.zeros(n))   # the plan still solves after the errors
        info = plan.solve(dev(p.b), x)
        assert info.converged


def test_zero_rhs_and_nonfinite():
    fde = need_gpu()
    p = fi.variable_1d(n=63)
    with fde.Plan(p) as plan:
        x = dev(np.ones(63))
        info = plan.solve(dev(np.zeros(63)), x)
        assert info.iters == 0 and info.converged
        assert np.all(host(x) == 0)
        b = np.ones(63)
        b[5] = np.nan
        with pytest.raises(fde.FdeError) as e:
            plan.solve(dev(b), dev(np.zeros(63)))
        assert e.value.status == fde.FDE_ENONFINITE
        x0 = np.zeros(63)
        x0[7] = np.inf   # a finite b, a non-finite start: the first residual is not finite
        with pytest.raises(fde.FdeError) as e:
            plan.solve(dev(np.ones(63)), dev(x0))
        assert e.value.status == fde.FDE_ENONFINITE


def test_maxit_returns_notconv_with_info():
    fde = need_gpu()
    p = fi.variable_1d(n=255, alpha=1.2)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    with fde.Plan(p, maxit=3) as plan:
        x = dev(np.zeros(255))
        info = plan.solve(dev(b), x, allow_notconv=True)
        assert info.iters == 3 and not info.converged
        xo, io = krylov.fgmres(s.matvec, b, pc.make("tau", s), restart=30, tol=1e-8, maxit=3)
        assert relerr(host(x), xo) < 1e-10


def test_coefficient_validation():
    fde = need_gpu()
    p = fi.variable_1d(n=63)
    p.dplus = p.dplus.copy()
    p.dplus[3] = -1.0
    with pytest.raises(fde.FdeError) as e:
        fde.Plan(p)
    assert e.value.status == fde.FDE_EINVAL
    p = fi.variable_1d(n=63)
    p.dplus = np.zeros(63)
    p.dminus = np.zeros(63)
    with pytest.raises(fde.FdeError):
        fde.Plan(p)


# ---------------------------------------------------------------------------
# P_tri (Table 2): the tridiagonal part of M solved by the partitioned
# elimination (chunk sweeps, reduced system by cyclic reduction, back
# substitution), against the oracle's banded solve.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 3, 7, 63, 1023, 4095, 8191, 65535])
@pytest.mark.parametrize("weights,time", [("shifted", "euler"), ("shifted", "cn")])
def test_tri_apply(n, weights, time):
    fde = need_gpu()
    p = prob1d(n, weights=weights, time=time)
    s = FDESystem.from_problem(p)
    v = rng_vec(n, n + 3)
    with fde.Plan(p, prec=fde.P_TRI) as plan:
        z = torch.empty(n, dtype=torch.float64, device="cuda")
        plan.tau_apply(dev(v), z)
        assert relerr(host(z), pc.make("tri", s)(v)) < 1e-12


@pytest.mark.parametrize("n,alpha", [(255, 1.3), (1023, 1.5), (4095, 1.8), (65535, 1.2)])
def test_tri_fgmres(n, alpha):
    fde = need_gpu()
    p = prob1d(n, alpha=alpha, seed=n)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    xg, ig = gpu_solve(fde, p, b, p.u0, prec=fde.P_TRI)
    assert ig.converged
    mirror(fde, p, b, p.u0, xg, ig, kind="tri", gpu_kw=dict(prec=fde.P_TRI))
    assert relerr(s.matvec(xg), b) <= 1e-8 * (1 + 1e-6)


def test_tri_mixed():
    fde = need_gpu()
    p = prob1d(4095, alpha=1.5, seed=5)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    with fde.Plan(p, prec=fde.P_TRI, precision=fde.MIXED, inner_steps=8) as plan:
        x = dev(p.u0)
        ig = plan.solve(dev(b), x)
    assert ig.converged
    assert relerr(s.matvec(host(x)), b) <= 1e-8 * (1 + 1e-6)


def test_tri_rejected_in_2d_and_without_dominance():
    """The partitioned elimination does not pivot: it takes the strictly
    diagonally dominant tridiagonal part of the first-order scheme (the case
    of Table 2), and rejects 2D and the second-order weights' non-dominant one."""
    fde = need_gpu()
    with pytest.raises(fde.FdeError):
        fde.Plan(prob2d(15, 15), prec=fde.P_TRI)
    with pytest.raises(fde.FdeError) as e:
        fde.Plan(prob1d(63, weights="weighted", time="cn"), prec=fde.P_TRI)
    assert e.value.status == fde.FDE_EINVAL


def test_plan_buffers_reused_and_released():
    """Plans of one shape built one after another take the buffers the
    previous one left in the library's cache (stale contents); their solves
    are bit-identical, also after the cache is released, and a plan of
    another shape in between does not disturb them."""
    fde = need_gpu()
    p = prob2d(127, 255)
    q = prob1d(1023)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0.reshape(-1))
    res = []
    for step in range(4):
        if step == 2:
            fde.fde_release_cache()
        if step == 3:
            with fde.Plan(q, precision=fde.MIXED) as other:
                x = dev(q.u0)
                other.solve(dev(FDESystem.from_problem(q).rhs(q.u0)), x)
        for precision in (fde.FP64, fde.MIXED):
            with fde.Plan(p, precision=precision) as plan:
                x = dev(p.u0.reshape(-1))
                info = plan.solve(dev(b), x)
                res.append((precision, host(x), info.iters))
    for precision in (fde.FP64, fde.MIXED):
        runs = [r for r in res if r[0] == precision]
        for r in runs[1:]:
            assert r[2] == runs[0][2]
            assert np.array_equal(r[1], runs[0][1])
        assert relerr(s.matvec(runs[0][1]), b) <= 1e-8 * (1 + 1e-6)


@pytest.mark.parametrize("case", ["2d-1023-fp64", "2d-1023-mixed", "2d-15x4095", "1d-65535-fp64",
                                  "1d-65535-mixed", "1d-1023-pcg", "1d-40000-chirp", "1d-40000-chirp-mixed",
                                  "2d-300x200-dense-mixed"])
def test_plan_bytes_matches_device_allocation(case):
    """fde_plan_bytes (the admission figure of the server) agrees with what
    assembly takes from the device, measured with the memory cache empty
    (to within a few percent on the large plans)."""
    fde = need_gpu()
    p = {"2d-1023-fp64": lambda: prob2d(1023, 1023), "2d-1023-mixed": lambda: prob2d(1023, 1023),
         "2d-15x4095": lambda: prob2d(15, 4095), "1d-65535-fp64": lambda: prob1d(65535),
         "1d-65535-mixed": lambda: prob1d(65535), "1d-1023-pcg": lambda: fi.constant_1d(n=1023),
         "1d-40000-chirp": lambda: prob1d(40000), "1d-40000-chirp-mixed": lambda: prob1d(40000),
         "2d-300x200-dense-mixed": lambda: prob2d(300, 200)}[case]()
    kw = dict(precision=fde.MIXED) if case.endswith("mixed") else {}
    # one assembly first: the runtime's one-time allocations on the first
    # launches of a process (code objects, scratch) are not the plan's
    with fde.Plan(p, **kw):
        pass
    fde.fde_release_cache()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    with fde.Plan(p, **kw) as plan:
        torch.cuda.synchronize()
        used = free0 - torch.cuda.mem_get_info()[0]
        claimed = fde.fde_plan_bytes(plan.params)
    fde.fde_release_cache()
    # 8 MB for the runtime's allocation granularity over a plan's few dozen buffers
    assert claimed >= 0.95 * used - (8 << 20), (claimed, used)
    assert claimed <= 1.25 * used + (8 << 20), (claimed, used)


# ---------------------------------------------------------------------------
# Dense 2D form: line operators as MFMA products, any n per direction up to
# 1023 (the paper's n = 16 ... 128 of Tables 3-4 included).
# ---------------------------------------------------------------------------
DENSE_SHAPES = [(16, 16), (17, 5), (32, 32), (5, 33), (64, 64), (100, 37), (128, 128), (300, 20), (1, 2),
                (1000, 24), (24, 777), (1000, 999)]


@pytest.mark.parametrize("n1,n2", DENSE_SHAPES)
@pytest.mark.parametrize("weights,time", [("shifted", "euler"), ("weighted", "cn")])
def test_dense_matvec_tau_rhs(n1, n2, weights, time):
    fde = need_gpu()
    p = prob2d(n1, n2, weights=weights, time=time, seed=n1 * 11 + n2)
    s = FDESystem.from_problem(p)
    x = rng_vec(s.N, n1 + 5 * n2)
    with fde.Plan(p) as plan, fde.Plan(p, dside=fde.D_RIGHT) as planr:
        y = torch.empty(s.N, dtype=torch.float64, device="cuda")
        plan.matvec(dev(x), y)
        assert relerr(host(y), s.matvec(x)) < 1e-12
        for pl, dside in ((plan, "left"), (planr, "right")):
            pl.tau_apply(dev(x), y)
            assert relerr(host(y), pc.make("tau", s, dside=dside)(x)) < 1e-12, dside
        plan.rhs(dev(x), y)
        assert relerr(host(y), s.rhs(x)) < 1e-12


@pytest.mark.parametrize("n1,n2", [(16, 16), (33, 20), (128, 128), (700, 40)])
@pytest.mark.parametrize("dside", ["left", "right"])
def test_dense_fgmres(n1, n2, dside):
    fde = need_gpu()
    p = fi.variable_2d(n=n1, n2=n2, seed=n1 + 3 * n2, steps=1)
    s = FDESystem.from_problem(p)
    x0 = p.u0.reshape(-1)
    b = s.rhs(x0)
    dk = dict(dside=fde.D_LEFT if dside == "left" else fde.D_RIGHT)
    xg, ig = gpu_solve(fde, p, b, x0, **dk)
    assert ig.converged
    mirror(fde, p, b, x0, xg, ig, dside=dside, gpu_kw=dk)


def test_dense_tau_hat_and_identity():
    fde = need_gpu()
    n1, n2 = 40, 24
    p = prob2d(n1, n2)
    p.dplus = np.full((n2, n1), 1.3)
    p.dminus = np.full((n2, n1), 1.3)
    p.eplus = np.full((n2, n1), 0.6)
    p.eminus = np.full((n2, n1), 0.6)
    s = FDESystem.from_problem(p)
    v = rng_vec(s.N, 5)
    for kind, prec in (("tau_hat", fde.P_TAU_HAT), ("none", fde.P_NONE)):
        with fde.Plan(p, prec=prec) as plan:
            z = torch.empty(s.N, dtype=torch.float64, device="cuda")
            plan.tau_apply(dev(v), z)
            assert relerr(host(z), pc.make(kind, s)(v)) < 1e-12, kind
    xg, ig = gpu_solve(fde, p, s.rhs(p.u0.reshape(-1)), p.u0.reshape(-1), prec=fde.P_NONE)
    assert ig.converged


def test_dense_mixed():
    """Mixed form on the dense 2D form (float32 MFMA products in the inner
    solve): float64 true residual within the tolerance and Varah's bound
    against the oracle's float64 solution."""
    fde = need_gpu()
    p = fi.variable_2d(n=100, n2=37, seed=77, steps=1)
    s = FDESystem.from_problem(p)
    x0 = p.u0.reshape(-1)
    b = s.rhs(x0)
    xo, io = oracle_solve(p, b, x0)
    xg, ig = gpu_solve(fde, p, b, x0, precision=fde.MIXED, inner_steps=8)
    assert ig.converged and ig.inner_iters > 0
    rg, ro = b - s.matvec(xg), b - s.matvec(xo)
    assert np.linalg.norm(rg) <= 1e-8 * (1 + 1e-6) * np.linalg.norm(b)
    assert np.abs(xg - xo).max() <= (np.abs(rg).max() + np.abs(ro).max()) / s.nu


def test_dense_forced_on_power_of_two_sizes(monkeypatch):
    """FDE_DENSE_LINES=1 selects the dense form for 2D plans of power-of-two
    sizes too (to compare the two forms); both agree with the oracle."""
    fde = need_gpu()
    p = prob2d(127, 63, seed=3)
    s = FDESystem.from_problem(p)
    x = rng_vec(s.N, 9)
    out = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("FDE_DENSE_LINES", flag)
        with fde.Plan(p) as plan:
            y = torch.empty(s.N, dtype=torch.float64, device="cuda")
            plan.matvec(dev(x), y)
            out[flag] = host(y)
            assert relerr(out[flag], s.matvec(x)) < 1e-12
    assert not np.array_equal(out["0"], out["1"])   # two different evaluations


def test_dense_size_limits():
    fde = need_gpu()
    for n1, n2 in ((1024, 16), (16, 1100), (1500, 1500)):
        with pytest.raises(fde.FdeError) as e:
            fde.Plan(prob2d(n1, n2))
        assert e.value.status == fde.FDE_EUNSUPPORTED


@pytest.mark.parametrize("n,alpha,restart", [(7, 1.5, 30), (255, 1.3, 30), (1023, 1.6, 5), (1023, 1.2, 30)])
def test_fgmres_one_workgroup_matches_multikernel(tmp_path, n, alpha, restart):
    """1D FGMRES with n + 1 <= 1024 runs in one workgroup; a traced solve
    (FDE_TRACE set) takes the multi-kernel path.  Both start from the same
    x0 and follow the same steps: iteration counts within one, solutions
    within 1e-10, and each mirrors the oracle."""
    import os
    fde = need_gpu()
    p = fi.variable_1d(n=n, alpha=alpha, seed=n + 3, steps=1)
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    xa, ia = gpu_solve(fde, p, b, p.u0, restart=restart)
    os.environ["FDE_TRACE"] = str(tmp_path / "trace.txt")
    try:
        xb, ib = gpu_solve(fde, p, b, p.u0, restart=restart)
    finally:
        del os.environ["FDE_TRACE"]
    assert (tmp_path / "trace.txt").exists()   # the traced solve did take the multi-kernel path
    assert ia.converged and ib.converged
    assert abs(ia.iters - ib.iters) <= 1, (ia.iters, ib.iters)
    assert relerr(s.matvec(xa), b) <= 1e-8 * (1 + 1e-6)
    if ia.iters == ib.iters:
        assert relerr(xa, xb) < 1e-10
    mirror(fde, p, b, p.u0, xa, ia, restart=restart)


@pytest.mark.parametrize("case", ["1d-255", "1d-65535", "1d-5000-chirp", "2d-127x63", "2d-100x70-dense"])
def test_float32_operators(case):
    """fde_matvec_f32 / fde_tau_apply_f32 (the mixed form's inner arithmetic)
    against the oracle's float64 operators: relative 2e-5; a float64 plan
    rejects them."""
    fde = need_gpu()
    if case.startswith("1d"):
        n = int(case.split("-")[1])
        p = prob1d(n, alpha=1.6, seed=n)
    else:
        n1, n2 = (int(t) for t in case.split("-")[1].split("x"))
        p = prob2d(n1, n2, seed=n1 + n2)
    s = FDESystem.from_problem(p)
    x = rng_vec(s.N, 5 + s.N % 97)
    with fde.Plan(p, precision=fde.MIXED) as plan:
        y = torch.empty(s.N, dtype=torch.float64, device="cuda")
        plan.matvec_f32(dev(x), y)
        assert relerr(host(y), s.matvec(x)) < 2e-5
        plan.tau_apply_f32(dev(x), y)
        assert relerr(host(y), pc.make("tau", s)(x)) < 2e-5
    with fde.Plan(p) as plan:
        with pytest.raises(fde.FdeError) as e:
            plan.matvec_f32(dev(x), torch.empty(s.N, dtype=torch.float64, device="cuda"))
        assert e.value.status == fde.FDE_EINVAL

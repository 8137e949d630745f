"""Batched 1D solves (one persistent launch for many uneven instances):
parity of every instance with the oracle's build-mode FGMRES, the chirp-z
DST for sizes where n + 1 is not a power of two, the staged FFT for long
lines, the mixed form, time stepping through the captured graph, and the
independence of an instance's result from the rest of the batch."""
import numpy as np
import pytest

import fde_inputs as fi
from gpu_util import dev, host, need_gpu, relerr, torch
from oracle import krylov, precond as pc
from oracle.system import FDESystem

pytestmark = pytest.mark.gpu


def inst(n, alpha, seed, weights="shifted", time="euler", fac=1.0):
    p = fi.variable_1d(n=n, alpha=alpha, seed=seed, steps=1)
    p.weights, p.time = weights, time
    p.dplus = p.dplus * fac
    p.dminus = p.dminus * fac
    return p


def rng_vec(n, seed):
    return np.random.default_rng(seed).uniform(-1, 1, n)


def oracle_solve(p, prec="tau", dside="left", restart=30, tol=1e-8):
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    P = pc.make(prec, s, dside=dside)
    x, info = krylov.fgmres(s.matvec, b, P, x0=p.u0, restart=restart, tol=tol)
    return s, b, x, info


def rounding_spread(p, prec="tau", dside="left", restart=30, tol=1e-8):
    """How far the oracle's own FGMRES iterate moves when its matrix-vector
    product carries an error of the size FFT rounding leaves in a Toeplitz
    product: per component u log2(L) ||g||_2 ||x||_2 / sqrt(n), scaled by
    d+ + d-, with L the circulant length.  Ill-conditioned systems (alpha
    near 2, large n) amplify such differences beyond 1e-10."""
    s = FDESystem.from_problem(p)
    b = s.rhs(p.u0)
    P = pc.make(prec, s, dside=dside)
    xo, _ = krylov.fgmres(s.matvec, b, P, x0=p.u0, restart=restart, tol=tol)
    n = s.N
    L = 2 * (1 << int(np.ceil(np.log2(max(n, 1)))))
    r = np.random.default_rng(7).standard_normal(n)
    scale = 2.0 ** -53 * np.log2(L) * (s.dplus + s.dminus) * np.linalg.norm(s.gx) / np.sqrt(n)
    xp, _ = krylov.fgmres(lambda x: s.matvec(x) + scale * np.linalg.norm(x) * r, b, P, x0=p.u0,
                          restart=restart, tol=tol)
    return relerr(xp, xo)


def check_fp64(p, xg, ig, prec="tau", dside="left", restart=30, tol=1e-8, gpu_kw=None):
    """Mirror parity of one batched instance: iteration counts within one;
    the iterates at equal step count (the side that ran one step longer is
    rerun with the other's count; an instance's result does not depend on the
    rest of the batch, so the GPU rerun is a batch of one) within 1e-10, or,
    where the instance's conditioning amplifies rounding past that, within ten
    times the distance the oracle's own iterate moves under a matrix-vector
    product perturbed by FFT-sized rounding (rounding_spread), capped at 1e-8."""
    fde = need_gpu()
    s, b, xo, io = oracle_solve(p, prec, dside, restart, tol)
    assert ig.converged and io["converged"], (p.name, ig.as_dict())
    d = ig.iters - io["iters"]
    assert abs(d) <= 1, (p.n, ig.iters, io["iters"])
    assert relerr(s.matvec(xg), b) <= tol * (1 + 1e-6)
    if d > 0:
        kw = dict(gpu_kw or {}, dside=fde.D_LEFT if dside == "left" else fde.D_RIGHT, restart=restart, tol=tol)
        (xg,), (ig2,) = batch_solve([p], fde, maxit=io["iters"], allow_notconv=True, **kw)
        assert ig2.iters == io["iters"]
    elif d < 0:
        P = pc.make(prec, s, dside=dside)
        xo, _ = krylov.fgmres(s.matvec, b, P, x0=p.u0, restart=restart, tol=tol, maxit=ig.iters)
    err = relerr(xg, xo)
    if err >= 1e-10:
        bound = min(1e-8, max(1e-10, 10.0 * rounding_spread(p, prec, dside, restart, tol)))
        assert err < bound, (p.n, err, bound)


# sizes: tiny, n + 1 a power of two (direct DST), arbitrary n (chirp-z DST),
# Toeplitz and DST both in LDS, and long enough for the staged FFT
SIZES_SMALL = [1, 2, 3, 5, 7, 8, 15, 100, 255, 256, 1000, 1023]
SIZES_LARGE = [2047, 3000, 4095, 5000, 8191, 12345]


def batch_solve(problems, fde, allow_notconv=False, **kw):
    with fde.Batch(problems, **kw) as bt:
        b = bt.pack([FDESystem.from_problem(p).rhs(p.u0) for p in problems])
        x = bt.pack([p.u0 for p in problems])
        infos = bt.solve(b, x, allow_notconv=allow_notconv)
        return bt.unpack(x), infos


def test_batch_small_fp64():
    fde = need_gpu()
    probs = [inst(n, 1.1 + 0.8 * ((7 * i) % 11) / 10.0, 100 + i) for i, n in enumerate(SIZES_SMALL)]
    xs, infos = batch_solve(probs, fde)
    for p, xg, ig in zip(probs, xs, infos):
        check_fp64(p, xg, ig)


def test_batch_large_fp64():
    fde = need_gpu()
    probs = [inst(n, 1.25 + 0.1 * i, 200 + i) for i, n in enumerate(SIZES_LARGE)]
    xs, infos = batch_solve(probs, fde)
    for p, xg, ig in zip(probs, xs, infos):
        check_fp64(p, xg, ig)


@pytest.mark.parametrize("weights,time", [("weighted", "cn"), ("shifted", "cn"), ("weighted", "euler")])
@pytest.mark.parametrize("dside", ["left", "right"])
def test_batch_schemes(weights, time, dside):
    fde = need_gpu()
    probs = [inst(n, a, 300 + n, weights, time) for n, a in [(63, 1.3), (200, 1.7), (1023, 1.5), (1500, 1.2)]]
    xs, infos = batch_solve(probs, fde, dside=fde.D_LEFT if dside == "left" else fde.D_RIGHT)
    for p, xg, ig in zip(probs, xs, infos):
        check_fp64(p, xg, ig, dside=dside)


@pytest.mark.parametrize("prec", ["none", "tilde", "tau_hat", "tri"])
def test_batch_preconditioners(prec):
    fde = need_gpu()
    code = {"none": fde.P_NONE, "tilde": fde.P_TILDE, "tau_hat": fde.P_TAU_HAT, "tri": fde.P_TRI}[prec]
    probs = []
    sizes = {"none": [15, 31, 63], "tri": [1, 2, 100, 1000, 1500, 9000]}.get(prec, [31, 100, 511])
    for i, n in enumerate(sizes):
        p = inst(n, 1.15 + 0.13 * i, 400 + i)
        if prec == "tau_hat":
            p.dplus = np.full(n, 1.5)
            p.dminus = np.full(n, 1.5)
        probs.append(p)
    xs, infos = batch_solve(probs, fde, prec=code, maxit=20000)
    for p, xg, ig in zip(probs, xs, infos):
        check_fp64(p, xg, ig, prec=prec, gpu_kw=dict(prec=code, maxit=20000))


@pytest.mark.parametrize("variant", [
    0, 1,
    pytest.param(2, marks=pytest.mark.skip(reason="256-thread variant disabled: it took a GPU memory fault "
                                                  "whose cause was not found (the CPU emulation runs clean)")),
    pytest.param(3, marks=pytest.mark.skip(reason="256-thread variant disabled with variant 2")),
])
def test_batch_variants(variant):
    """Every enabled launch configuration (workgroup size x FFT radix) solves alike."""
    fde = need_gpu()
    probs = [inst(n, a, 500 + n) for n, a in [(127, 1.4), (999, 1.6), (4095, 1.8), (6000, 1.5)]]
    with fde.Batch(probs) as bt:
        bt.set_cfg(variant, 7, lpt=(variant + 1) % 2)
        b = bt.pack([FDESystem.from_problem(p).rhs(p.u0) for p in probs])
        x = bt.pack([p.u0 for p in probs])
        infos = bt.solve(b, x)
        xs = bt.unpack(x)
    for p, xg, ig in zip(probs, xs, infos):
        check_fp64(p, xg, ig)


@pytest.mark.parametrize("prec", ["tau", "tri"])
def test_batch_mixed(prec):
    fde = need_gpu()
    probs = [inst(n, a, 600 + n) for n, a in [(255, 1.3), (1000, 1.5), (4095, 1.7), (7000, 1.2)]]
    code = fde.P_TRI if prec == "tri" else fde.P_TAU
    for inner in (0, 16):
        xs, infos = batch_solve(probs, fde, precision=fde.MIXED, inner_steps=inner, prec=code)
        for p, xg, ig in zip(probs, xs, infos):
            s, b, xo, io = oracle_solve(p, prec)
            assert ig.converged
            rg, ro = b - s.matvec(xg), b - s.matvec(xo)
            assert np.linalg.norm(rg) <= 1e-8 * (1 + 1e-6) * np.linalg.norm(b)   # float64 true residual
            # Varah: every row of the first-order M is diagonally dominant by nu
            assert np.abs(xg - xo).max() <= (np.abs(rg).max() + np.abs(ro).max()) / s.nu


def test_batch_alone_equals_mix():
    """An instance's iterates do not depend on the other instances."""
    fde = need_gpu()
    probs = [inst(n, a, 700 + n) for n, a in [(300, 1.4), (2047, 1.6), (5000, 1.3), (77, 1.9)]]
    xs, infos = batch_solve(probs, fde)
    for k in (0, 2):
        xa, ia = batch_solve([probs[k]], fde)
        assert ia[0].iters == infos[k].iters
        assert np.array_equal(xa[0], xs[k])


def test_batch_run_graph_matches_eager():
    """Time stepping: the replayed graph gives bit-identical states and
    iteration counts to eager launches, step by step."""
    fde = need_gpu()
    probs = [inst(n, a, 800 + n) for n, a in [(255, 1.5), (1000, 1.3), (3000, 1.7)]]
    steps = 3
    with fde.Batch(probs) as bt:
        u0 = bt.pack([p.u0 for p in probs])
        ug = u0.clone()
        ue = u0.clone()
        ig = bt.run(ug, steps, use_graph=True)
        ie = bt.run(ue, steps, use_graph=False)
        assert torch.equal(ug, ue)
        for s in range(steps):
            assert [i.iters for i in ig[s]] == [i.iters for i in ie[s]]
        # a second graph run continues from the state (graph replayed again)
        ug2 = ug.clone()
        bt.run(ug2, 1, use_graph=True)
        ue2 = ue.clone()
        bt.run(ue2, 1, use_graph=False)
        assert torch.equal(ug2, ue2)
        # every step against the oracle's step from the GPU's previous state
        us = bt.pack([p.u0 for p in probs])
        prev = bt.unpack(us)
        for step in range(steps):
            info = bt.run(us, 1, use_graph=True)[0]
            cur = bt.unpack(us)
            for p, u0, xg, ig in zip(probs, prev, cur, info):
                q = fi.variable_1d(n=p.n[0], alpha=p.alpha[0], steps=1)
                q.dplus, q.dminus, q.u0 = p.dplus, p.dminus, u0
                check_fp64(q, xg, ig)
            prev = cur
        assert torch.equal(us, ug)


def test_batch_float32_operators_need_a_mixed_batch():
    fde = need_gpu()
    probs = [inst(10, 1.5, 1)]
    with fde.Batch(probs) as bt:
        x = bt.pack([probs[0].u0])
        y = torch.empty_like(x)
        with pytest.raises(fde.FdeError) as e:
            bt.matvec(x, y, precision=fde.MIXED)
        assert e.value.status == fde.FDE_EINVAL


def test_batch_edge_cases():
    fde = need_gpu()
    probs = [inst(n, 1.5, 900 + n) for n in (10, 20, 30)]
    with fde.Batch(probs) as bt:
        bvals = [FDESystem.from_problem(p).rhs(p.u0) for p in probs]
        bvals[1] = np.zeros(20)
        b = bt.pack(bvals)
        x = bt.pack([p.u0 for p in probs])
        infos = bt.solve(b, x)
        xs = bt.unpack(x)
        assert infos[1].converged and infos[1].iters == 0 and np.all(xs[1] == 0.0)
        check_fp64(probs[0], xs[0], infos[0])
        # a non-finite right-hand side is reported, the other instances are still solved
        bvals[2] = bvals[2].copy()
        bvals[2][3] = np.nan
        b = bt.pack(bvals)
        x = bt.pack([p.u0 for p in probs])
        with pytest.raises(fde.FdeError) as e:
            bt.solve(b, x)
        assert e.value.status == fde.FDE_ENONFINITE
    # maxit reached: FDE_ENOTCONV with the last iterate
    with fde.Batch(probs[:1], maxit=2) as bt:
        b = bt.pack([FDESystem.from_problem(probs[0]).rhs(probs[0].u0)])
        x = bt.pack([probs[0].u0])
        infos = bt.solve(b, x, allow_notconv=True)
        assert infos[0].iters == 2 and not infos[0].converged


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_split_to_plan_path(precision):
    """The instances of largest estimated work taken out of the persistent
    launch and solved on the plan path by worker threads (split = 3 of 8,
    any n): every instance still mirrors the oracle (float64) or meets the
    tolerance within Varah's bound (mixed), in a solve and in graph-replayed
    time steps; the split instances are the largest ones."""
    fde = need_gpu()
    sizes = [(9000, 1.2), (255, 1.5), (3000, 1.3), (12000, 1.15), (77, 1.9), (6000, 1.4), (1000, 1.6), (5000, 1.25)]
    probs = [inst(n, a, 1500 + n) for n, a in sizes]
    kw = dict(precision=fde.MIXED, inner_steps=0) if precision == "mixed" else {}
    with fde.Batch(probs, **kw) as bt:
        bt.set_cfg(0, 64, 1, split=3)
        assert bt.get_cfg().split == 3
        b = bt.pack([FDESystem.from_problem(p).rhs(p.u0) for p in probs])
        x = bt.pack([p.u0 for p in probs])
        infos = bt.solve(b, x)
        xs = bt.unpack(x)
        for p, xg, ig in zip(probs, xs, infos):
            if precision == "fp64":
                check_fp64(p, xg, ig)
            else:
                s, bb, xo, io = oracle_solve(p)
                assert ig.converged
                rg, ro = bb - s.matvec(xg), bb - s.matvec(xo)
                assert np.linalg.norm(rg) <= 1e-8 * (1 + 1e-6) * np.linalg.norm(bb)
                assert np.abs(xg - xo).max() <= (np.abs(rg).max() + np.abs(ro).max()) / s.nu
        # time steps (graph) with the split: each step against the oracle from the previous state
        us = bt.pack([p.u0 for p in probs])
        prev = bt.unpack(us)
        for step in range(2):
            info = bt.run(us, 1, use_graph=True)[0]
            cur = bt.unpack(us)
            for p, u0, xg, ig in zip(probs, prev, cur, info):
                q = fi.variable_1d(n=p.n[0], alpha=p.alpha[0], steps=1)
                q.dplus, q.dminus, q.u0 = p.dplus, p.dminus, u0
                if precision == "fp64":
                    check_fp64(q, xg, ig)
                else:
                    assert ig.converged and ig.relres_true <= 1e-8
            prev = cur


def test_batch_tune():
    fde = need_gpu()
    probs = fi.batched_1d(count=24, seed=4, nmax=4095, steps=1)
    with fde.Batch(probs) as bt:
        u = bt.pack([p.u0 for p in probs])
        before = u.clone()
        c = bt.tune(u)
        assert torch.equal(u, before)
        assert 0 <= c.variant < fde.BATCH_VARIANTS and c.grid >= 1 and c.ms > 0 and 0 <= c.split < len(probs)
        got = bt.get_cfg()
        assert (got.variant, got.grid, got.lpt, got.split) == (c.variant, c.grid, c.lpt, c.split)
        infos = bt.run(u, 1)
    xs = bt.unpack(u)
    for p, xg, ig in zip(probs, xs, infos[0]):
        s = FDESystem.from_problem(p)
        assert ig.converged
        assert relerr(s.matvec(xg), s.rhs(p.u0)) <= 1e-8 * (1 + 1e-6)


@pytest.mark.parametrize("n,alpha", [(16383, 1.5), (32767, 1.8), (40000, 1.8)])
def test_batch_full_sizes(n, alpha):
    """Long lines: staged FFTs for the Toeplitz product and the DST, direct
    (n + 1 = 2^k) and chirp-z (n = 40000); 16383 is the largest size of the
    batched workload."""
    fde = need_gpu()
    probs = [inst(n, alpha, 1000 + n), inst(255, 1.3, 1001)]
    xs, infos = batch_solve(probs, fde)
    for p, xg, ig in zip(probs, xs, infos):
        check_fp64(p, xg, ig)


OP_SIZES = [(1, 1.5), (2, 1.3), (3, 1.7), (100, 1.2), (255, 1.9), (1000, 1.5), (4095, 1.4), (7000, 1.2),
            (16383, 1.6), (40000, 1.8)]


@pytest.mark.skip(reason="the persistent kernel's operator launches (launch variants 0/1) are disabled: their "
                         "first GPU run took a memory fault whose cause was not found; the batched operators now "
                         "run through per-instance plans (test_batch_operators_plan_path)")
@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("prec", ["tau", "tri"])
def test_batch_operators(variant, prec):
    """Batched M x and P^{-1} v against the oracle, in float64 (relative 1e-12)
    and float32 (relative 2e-5), for every size class: direct and chirp-z DST,
    transforms in LDS and staged through global memory."""
    fde = need_gpu()
    probs = [inst(n, a, 1100 + n) for n, a in OP_SIZES]
    code = fde.P_TRI if prec == "tri" else fde.P_TAU
    xs = [rng_vec(p.n[0], 7 + p.n[0]) for p in probs]
    with fde.Batch(probs, precision=fde.MIXED, prec=code) as bt:
        bt.set_cfg(variant, 64, 1)
        x = bt.pack(xs)
        for precision, tol in ((fde.FP64, 1e-12), (fde.MIXED, 2e-5)):
            y = torch.empty_like(x)
            bt.matvec(x, y, precision=precision)
            ys = bt.unpack(y)
            bt.tau_apply(x, y, precision=precision)
            zs = bt.unpack(y)
            for p, xv, yv, zv in zip(probs, xs, ys, zs):
                s = FDESystem.from_problem(p)
                assert relerr(yv, s.matvec(xv)) < tol, (p.n, precision, "matvec", relerr(yv, s.matvec(xv)))
                zo = pc.make(prec, s)(xv)
                assert relerr(zv, zo) < tol, (p.n, precision, "tau", relerr(zv, zo))


@pytest.mark.parametrize("prec", ["tau", "tri"])
def test_batch_operators_plan_path(prec):
    """Batched M x and P^{-1} v (each instance with its own plan) against the
    oracle, in float64 (relative 1e-12) and float32 (relative 2e-5), for every
    size class: direct and chirp-z DST, one-workgroup lines and long lines."""
    fde = need_gpu()
    probs = [inst(n, a, 1100 + n) for n, a in OP_SIZES]
    code = fde.P_TRI if prec == "tri" else fde.P_TAU
    xs = [rng_vec(p.n[0], 7 + p.n[0]) for p in probs]
    with fde.Batch(probs, precision=fde.MIXED, prec=code) as bt:
        x = bt.pack(xs)
        for precision, tol in ((fde.FP64, 1e-12), (fde.MIXED, 2e-5)):
            y = torch.empty_like(x)
            bt.matvec(x, y, precision=precision)
            ys = bt.unpack(y)
            bt.tau_apply(x, y, precision=precision)
            zs = bt.unpack(y)
            for p, xv, yv, zv in zip(probs, xs, ys, zs):
                s = FDESystem.from_problem(p)
                assert relerr(yv, s.matvec(xv)) < tol, (p.n, precision, "matvec", relerr(yv, s.matvec(xv)))
                zo = pc.make(prec, s)(xv)
                assert relerr(zv, zo) < tol, (p.n, precision, "tau", relerr(zv, zo))


def test_batched_workload_sample_against_oracle():
    """The 512-instance batched workload (n log-uniform in [255, 16383],
    alpha ~ U(1.1, 1.9), scaled Example 1 coefficients), first time step in
    float64 in one launch: a sample of 12 instances spread over the sizes is
    mirrored by the oracle, and every instance's float64 true residual is
    within the tolerance."""
    fde = need_gpu()
    probs = fi.batched_1d(count=512, steps=1)
    with fde.Batch(probs, maxit=20000) as bt:
        u = bt.pack([p.u0 for p in probs])
        infos = bt.run(u, 1)[0]
        xs = bt.unpack(u)
    assert all(i.converged for i in infos)
    assert max(i.relres_true for i in infos) <= 1e-8
    order = np.argsort([p.n[0] for p in probs])
    for k in np.linspace(0, len(probs) - 1, 12).astype(int):
        i = int(order[k])
        check_fp64(probs[i], xs[i], infos[i])


def test_batched_workload_operators_against_oracle():
    """Batched M x and P^{-1} v over the 512-instance batched workload (each
    instance through its own plan): a sample of 16 instances spread over the
    sizes against the oracle (float64 relative 1e-12, float32 2e-5), and for
    every instance the float32 result within 2e-5 of the float64 one."""
    fde = need_gpu()
    probs = fi.batched_1d(count=512, steps=1)
    xs = [rng_vec(p.n[0], 31 + i) for i, p in enumerate(probs)]
    out = {}
    with fde.Batch(probs, precision=fde.MIXED) as bt:
        x = bt.pack(xs)
        y = torch.empty_like(x)
        for precision in (fde.FP64, fde.MIXED):
            bt.matvec(x, y, precision=precision)
            ys = bt.unpack(y)
            bt.tau_apply(x, y, precision=precision)
            out[precision] = (ys, bt.unpack(y))
    for i in range(len(probs)):
        for k in range(2):
            assert relerr(out[fde.MIXED][k][i], out[fde.FP64][k][i]) < 2e-5, (i, probs[i].n, k)
    order = np.argsort([p.n[0] for p in probs])
    for k in np.linspace(0, len(probs) - 1, 16).astype(int):
        i = int(order[k])
        s = FDESystem.from_problem(probs[i])
        yo, zo = s.matvec(xs[i]), pc.make("tau", s)(xs[i])
        for precision, tol in ((fde.FP64, 1e-12), (fde.MIXED, 2e-5)):
            ys, zs = out[precision]
            assert relerr(ys[i], yo) < tol, (probs[i].n, precision, "matvec")
            assert relerr(zs[i], zo) < tol, (probs[i].n, precision, "tau")

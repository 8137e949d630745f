"""Served (continuous-batching) solves: each request's result is the same
alone and inside a mix of concurrently running requests, and admission
respects the HBM budget."""
import numpy as np
import pytest

import fde_inputs as fi
from gpu_util import need_gpu, torch

pytestmark = pytest.mark.gpu


def small_stream(rate=2000.0, count=8, seed=21):
    return fi.served_stream(rate, count, seed=seed, n1d=(255, 4095), n2d=(63, 127, 255), steps=(2, 5))


@pytest.mark.parametrize("precision,inner", [(0, None), (1, None), ("auto", None), (1, "auto")])
def test_alone_equals_mix(precision, inner):
    fde = need_gpu()
    from paper_1912_13304_amd import serve
    arr = small_stream()
    kw = dict(precision=precision)
    if inner is not None:
        kw["inner_steps"] = inner
    results, wall = serve.serve_stream(arr, slots=4, keep_state=True, **kw)
    assert len(results) == len(arr)
    by_name = {r.name: r for r in results}
    # requests overlapped on the device: some request started before another finished
    spans = sorted((r.start, r.finish) for r in results)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    for a in arr:
        infos, u = serve.run_job(a.problem, keep_state=True, **serve.request_kw(a.problem, kw))
        torch.cuda.synchronize()
        r = by_name[a.problem.name]
        assert r.iters == [i.iters for i in infos]
        assert torch.equal(r.u, u), a.problem.name   # bitwise: fixed-order reductions
        assert max(r.relres) <= a.problem.tol * (1 + 1e-6)


def test_admission_budget():
    fde = need_gpu()
    from paper_1912_13304_amd import serve
    arr = small_stream(count=6, seed=5)
    need = [serve.footprint(a.problem) for a in arr]
    budget = max(need) * 1.2        # at most one large request at a time
    srv = serve.Server(slots=4, hbm_budget=budget)
    peak = [0.0]
    orig = srv._take

    def take():
        item = orig()
        peak[0] = max(peak[0], srv.in_use)
        return item
    srv._take = take
    srv.start()
    for a in arr:
        srv.submit(a.problem)
    srv.close()
    assert len(srv.results) == len(arr)
    assert peak[0] <= budget
    st = serve.latency_stats(srv.results)
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_failed_request_is_reported_and_slot_survives():
    """A request the library rejects (a negative coefficient: FDE_EINVAL at
    assembly) comes back as a failed result; the slot's worker keeps serving
    and every other request completes."""
    fde = need_gpu()
    from paper_1912_13304_amd import serve
    arr = small_stream(count=6, seed=9)
    bad = arr[2].problem
    bad.dplus = bad.dplus.copy()
    bad.dplus.reshape(-1)[1] = -1.0
    results, _ = serve.serve_stream(arr, slots=2)
    assert len(results) == len(arr)
    by = {r.name: r for r in results}
    assert not by[bad.name].ok and by[bad.name].status == fde.FDE_EINVAL
    assert all(r.ok for r in results if r.name != bad.name)
    st = serve.latency_stats(results)
    assert st["failed"] == 1 and st["requests"] == len(arr)


def test_served_results_against_oracle():
    """Served results checked step by step against the oracle (each step
    from the state the server computed before it): float64 requests mirror
    the oracle's FGMRES (iterations within one, iterates at equal step count
    within 1e-10); mixed requests have a float64 true residual within the
    tolerance and are within Varah's bound of the oracle's step.  The stream
    includes 1D lines whose n + 1 is not a power of two (chirp-z DST)."""
    import numpy as np
    from gpu_util import mirror_check, rounding_spread
    from oracle import krylov, precond as pc
    from oracle.system import FDESystem
    fde = need_gpu()
    from paper_1912_13304_amd import serve
    arr = fi.served_stream(2000.0, 6, seed=31, n1d=(300, 3000), n2d=(31, 63), steps=(2, 3))
    for precision in (fde.FP64, fde.MIXED):
        results, _ = serve.serve_stream(arr, slots=3, keep_state="all", precision=precision,
                                        inner_steps=serve.AUTO)
        by = {r.name: r for r in results}
        for a in arr:
            p = a.problem
            r = by[p.name]
            assert r.ok and len(r.states) == p.steps
            s = FDESystem.from_problem(p)
            P = pc.make("tau", s)
            prev = p.u0.reshape(-1)
            for m, xg in enumerate(r.states):
                xg = xg.reshape(-1)
                b = s.rhs(prev)

                def orun(maxit, b=b, prev=prev):
                    x, i = krylov.fgmres(s.matvec, b, P, x0=prev, restart=30, tol=p.tol, maxit=maxit or 100000)
                    return x, i["iters"]

                if precision == fde.FP64:
                    def grun(maxit, b=b, prev=prev):
                        with fde.Plan(p, maxit=maxit) as plan:
                            x = torch.as_tensor(prev.copy(), device="cuda")
                            i = plan.solve(torch.as_tensor(b, device="cuda"), x, allow_notconv=True)
                            return x.cpu().numpy(), i.iters
                    spread = (lambda b=b, prev=prev: rounding_spread(s, b, P, prev, tol=p.tol)) \
                        if p.dim == 1 else None
                    mirror_check(xg, r.iters[m], orun, grun, spread=spread)
                else:
                    xo, _ = orun(None)
                    rg, ro = b - s.matvec(xg), b - s.matvec(xo)
                    assert np.linalg.norm(rg) <= p.tol * (1 + 1e-6) * np.linalg.norm(b)
                    assert np.abs(xg - xo).max() <= (np.abs(rg).max() + np.abs(ro).max()) / s.nu
                prev = xg


def test_cancel_pending_and_running():
    """A pending request is dropped at once; a running one stops before its
    next step and returns the steps it completed, which equal the same steps
    run alone; the other requests complete."""
    import time
    fde = need_gpu()
    from paper_1912_13304_amd import serve
    long = fi.variable_1d(n=4095, alpha=1.5, seed=3, steps=400)
    long.name = "long"
    others = []
    for k, seed in enumerate((4, 5, 6)):
        p = fi.variable_1d(n=1023, alpha=1.6, seed=seed, steps=2)
        p.name = f"short{k}"
        others.append(p)
    srv = serve.Server(slots=1)
    srv.start()
    srv.submit(long)
    for p in others:
        srv.submit(p)
    t0 = time.perf_counter()
    while "long" not in srv.running:
        assert time.perf_counter() - t0 < 60
        time.sleep(0.001)
    assert srv.cancel("short1")       # pending
    assert srv.cancel("long")         # running
    assert not srv.cancel("absent")
    srv.close()
    by = {r.name: r for r in srv.results}
    assert len(srv.results) == 4
    assert by["long"].cancelled and len(by["long"].iters) < long.steps
    assert by["short1"].cancelled and by["short1"].iters == []
    assert by["short0"].ok and by["short2"].ok
    assert srv.in_use == 0.0 and not srv.running and not srv.cancel_flags   # slot and budget reclaimed
    st = serve.latency_stats(srv.results, slots=1)
    assert st["cancelled"] == 2 and st["failed"] == 0
    assert st["solves"] == 2 * others[0].steps
    done = len(by["long"].iters)
    if done:
        long.steps = done
        infos, _ = serve.run_job(long)
        assert by["long"].iters == [i.iters for i in infos]

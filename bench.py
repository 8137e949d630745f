#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload (one bench step = one whole time-stepping job): the 2D
variable-coefficient space-fractional diffusion problem on (0,2)^2 with
alpha_x = 1.7, alpha_y = 1.4, n1 = n2 = 1023 (N = 1,046,529 unknowns),
coefficients d+- = G(3-a)x^a(1+y) / G(3-a)(2-x)^a(1+y) and the matching
y-direction fields, dt = h, u0 ~ U[-1,1] (seed 3), f = 0, 10 implicit-Euler
steps; each step is the setup-free right-hand side b = nu u^{m-1} followed by a
preconditioned FGMRES(30) solve with P_F to ||b - M u||/||b|| <= 1e-8 from
x0 = u^{m-1}.  The plan is assembled inside each job (setup row of the path).
Forms: all-float64 and mixed (float32 inner GMRES(k) with float32 matvec and
tau solve inside the float64 outer FGMRES).

Prints one JSON line.  value = linear solves (time steps) per second of the
mixed form; the float64 form, time-to-tol per solve, iteration counts, the
roofline of the dominant kernel (HIP events over the timed region, algorithmic
bytes per launch), and the FP64 CPU oracle on a bounded sample are included.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_2d1023_job.json")


def class_pattern(cls):
    """Kernel-name pattern of a probe class (the template arguments that select it)."""
    import re
    t = {"64": "double", "32": "float"}
    if cls.startswith("cgs_"):
        kind, prec = cls[4:-2], cls[-2:]
        modes = "0" if kind == "dot" else "[12]"
        return re.compile(rf"cgs_kernel<{t[prec]}, \d+, \d+, {modes}>")
    if cls.startswith("line"):
        from paper_1912_13304_amd import fde
        prec, prog = cls[4:6], cls[7:]
        fl = [k for k, v in fde.LINE_PROGRAMS.items() if v == prog]
        if fl:
            return re.compile(rf"line_kernel<{t[prec]}, (true|false), {fl[0]}, \d+>")
    return None


def measured_traffic(cls):
    """HBM bytes per launch of a kernel class from the committed PMC summary,
    or None when there is none or the HIP sources changed since it was taken."""
    try:
        import json as _j
        from paper_1912_13304_amd import profsum
        d = _j.load(open(TRAFFIC_FILE))
        if d.get("source_hash") != profsum.source_hash():
            return None
        pat = class_pattern(cls)
        if pat is None:
            return None
        tot, cnt = 0.0, 0
        for name, v in d["kernels"].items():
            if pat.search(name):
                tot += v["traffic_bytes_avg"] * v["dispatches"]
                cnt += v["dispatches"]
        return tot / cnt if cnt else None
    except (OSError, ValueError, KeyError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def model_bytes_1d(n, iters, inner, m, kin, mixed):
    """Algorithmic bytes of one 1D FGMRES(m) solve: per outer step j (mod m)
    tau 24n + matvec 32n + CGS2 (32j + 80)n + normalisation 16n in float64;
    the mixed form replaces the tau solve by the cast of v (12n), kin float32
    inner steps (tau 12n, matvec 16n, CGS2 (16i + 40)n each), the inner update
    (4(kin+1)n, none when kin = 0), the float32 tau solve (12n) and the cast
    back (12n)."""
    tot = 0.0
    for t in range(iters):
        j = t % m
        if mixed:
            inner_b = sum(12 + 16 + 16 * i + 40 for i in range(kin)) + (4 * (kin + 1) if kin else 0) + 12 + 12 + 12
            tot += (32 + 32 * j + 80 + 16 + inner_b) * n
        else:
            tot += (152 + 32 * j) * n
    return tot


def model_bytes_2d(N, outer, inner_total, m, mixed):
    """Algorithmic bytes of one 2D FGMRES(m) solve of the plan path (every
    vector operand of every kernel read or written once, D on the left), in
    units of N:
      float64 step j (k = j + 1 basis vectors): row DST 24, column DST/F/DST
      16, row DST + z + row Toeplitz 40, column Toeplitz with base 40, CGS2
      (3k + 5) * 8;
      mixed outer step j: cast of v 12, inner norm 4, per inner step i (float32,
      k = i + 1): tau + matvec 60 and single-pass Gram-Schmidt (2k + 3) * 4;
      the inner update 4 (kin + 1), the float32 tau solve 28, the cast back 12,
      the float64 matvec 72 and CGS2 (3(j + 1) + 5) * 8."""
    tot = 0.0
    kin = inner_total / outer if (mixed and outer) else 0.0
    for t in range(outer):
        j = t % m
        cgs64 = (3 * (j + 1) + 5) * 8
        if mixed:
            ki = int(round(kin))
            inner = sum(60 + (2 * (i + 1) + 3) * 4 for i in range(ki))
            tot += 12 + 4 + inner + 4 * (ki + 1) + 28 + 12 + 72 + cgs64
        else:
            tot += 24 + 16 + 40 + 40 + cgs64
    return tot * N


def batched_leg(args, fi, fde, torch, np):
    """Many independent uneven 1D solves in one persistent launch per time
    step (graph replayed per step), launch configuration picked by the tuner;
    and the same instances solved one plan at a time for comparison."""
    probs = fi.batched_1d(count=args.batch_count, seed=4, steps=args.batch_steps)
    out = {"instances": len(probs), "unknowns": int(sum(p.n[0] for p in probs)),
           "workload": f"{len(probs)} 1D instances, n log-uniform in [255, 16383] (any n), alpha ~ U(1.1,1.9), "
                       "Example-1 coefficients x U(0.5,2), dt = h, FGMRES(30)+P_F to 1e-8, x0 = u^(m-1); "
                       f"mixed form: float32 P_F inside the float64 FGMRES, {args.batch_inner} inner steps"}
    # mixed: the float32 preconditioner inside the float64 FGMRES, no inner
    # steps (faster than GMRES(16) inner solves on these 1D lines)
    forms = {"mixed": dict(precision=fde.MIXED, inner_steps=args.batch_inner), "fp64": dict(precision=fde.FP64)}
    cfg = None
    for name, kw in forms.items():
        bt = fde.Batch(probs, **kw)
        u = bt.pack([p.u0 for p in probs])
        if cfg is None and args.batch_cfg:
            v, g, l, sp = (int(t) for t in args.batch_cfg.split(","))
            cfg = {"variant": v, "grid": g, "lpt": l, "split": sp, "tuned": False}
            bt.set_cfg(v, g, l, sp)
        elif cfg is None:
            log(f"[bench] batched: tuning launch configuration")
            c = bt.tune(u)
            cfg = c.as_dict()
        else:
            bt.set_cfg(cfg["variant"], cfg["grid"], cfg["lpt"], cfg.get("split", 0))
        bt.run(u.clone(), 1, use_graph=True, allow_notconv=True)   # warm (graph captured)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = bt.run(u, args.batch_steps, use_graph=True, allow_notconv=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        its = [i.iters for st in infos for i in st]
        inner = [i.inner_iters for st in infos for i in st]
        mixed = name == "mixed"
        byt = sum(model_bytes_1d(p.n[0], i.iters, 0, 30, args.batch_inner if mixed else 0, mixed)
                  for st in infos for p, i in zip(probs, st))
        out[name] = dict(inst_steps_per_s=len(probs) * args.batch_steps / dt, ms_per_step=1e3 * dt / args.batch_steps,
                         modelled_GBps=byt / dt / 1e9, iters_mean=float(np.mean(its)), iters_max=int(max(its)),
                         inner_iters_mean=float(np.mean(inner)),
                         all_converged=all(i.converged for st in infos for i in st),
                         max_relres=float(max(i.relres_true for st in infos for i in st)))
        log(f"[bench] batched {name}: {out[name]}")
        bt.close()
    out["cfg"] = cfg
    # the same instances, one plan at a time (float64 per-plan path), against
    # one batched launch of the same instances
    k = min(args.batch_plan_sample, len(probs))
    sample = fi.batched_1d(count=k, seed=4, steps=1)
    plans = [fde.Plan(p) for p in sample]
    us = [torch.as_tensor(p.u0, dtype=torch.float64, device="cuda") for p in sample]
    bs = [torch.empty_like(u) for u in us]
    xs = [torch.empty_like(u) for u in us]
    for pl, u, b in zip(plans, us, bs):
        pl.rhs(u, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, u, b, x in zip(plans, us, bs, xs):
        x.copy_(u)
        pl.solve(b, x, allow_notconv=True)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    for pl in plans:
        pl.close()
    bt = fde.Batch(sample)
    bt.set_cfg(cfg["variant"], cfg["grid"], cfg["lpt"], cfg.get("split", 0))
    u = bt.pack([p.u0 for p in sample])
    bt.run(u.clone(), 1, use_graph=False, allow_notconv=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.run(u, 1, use_graph=True, allow_notconv=True)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    bt.close()
    out["vs_plan"] = {"instances": k, "plan_fp64_solves_per_s": k / t_plan, "batched_fp64_solves_per_s": k / t_batch,
                      "speedup": t_plan / t_batch,
                      "note": "the same instances (any n), first implicit step each"}
    log(f"[bench] batched vs plan: {out['vs_plan']}")
    return out


def served_leg(args, fi, fde):
    """Poisson arrivals of time-stepping requests (70% 1D, n log-uniform in
    [1023, 65535], any n; 30% 2D, n in {127, 255, 511, 1023}; 5-50 implicit
    steps; alpha ~ U(1.1, 1.9); tol 1e-8), continuously batched over slots x
    streams with HBM-footprint admission.  Reported per stream: completed
    solves/s, p50/p99 arrival-to-completion latency and the slots'
    utilisation.  Legs: every request in the mixed form at the headline rate;
    the same stream with the per-request precision policy; the same stream one
    request at a time in float64 (the plain float64 baseline); and a sweep of
    arrival rates from below to above the service capacity (request count
    scaled so that the arrivals span about serve_window seconds)."""
    from paper_1912_13304_amd import serve
    mix = ("70% 1D n log-uniform in [1023, 65535] (any n), 30% 2D n in {127,255,511,1023}; 5-50 steps; "
           "alpha ~ U(1.1,1.9); tol 1e-8")
    slots = args.serve_slots
    arr = fi.served_stream(args.serve_rate, args.serve_count, seed=5, n1d=(1023, 65535))
    warm = fi.served_stream(args.serve_rate, 8, seed=55, n1d=(1023, 65535), steps=(2, 3))
    serve.serve_stream(warm, slots=slots, precision=fde.MIXED, inner_steps=serve.AUTO)
    serve.serve_stream(warm, slots=1, precision=fde.FP64)
    log(f"[bench] served: {len(arr)} requests at {args.serve_rate}/s, {slots} slots, mixed")
    res, _ = serve.serve_stream(arr, slots=slots, precision=fde.MIXED, inner_steps=serve.AUTO)
    out = serve.latency_stats(res, slots)
    out.update(rate_req_per_s=args.serve_rate, slots=slots,
               mix=mix + f"; mixed precision: float32 inner GMRES({serve.INNER_2D}) for 2D requests, the float32 "
                         "preconditioner without inner steps for 1D requests")
    log(f"[bench] served: {out}")
    res, _ = serve.serve_stream(arr, slots=slots, precision=serve.AUTO, inner_steps=args.inner)
    auto = serve.latency_stats(res, slots)
    auto.update(policy="mixed for 2D requests with n >= 511, float64 for smaller 2D and for 1D requests")
    out["per_request_precision"] = auto
    log(f"[bench] served, per-request precision: {auto}")
    log(f"[bench] served: the same stream one request at a time in float64")
    res, _ = serve.serve_stream(arr, slots=1, precision=fde.FP64)
    base = serve.latency_stats(res, 1)
    out["fp64_one_at_a_time"] = base
    out["speedup_vs_fp64_one_at_a_time"] = out["solves_per_s"] / base["solves_per_s"] if base["solves_per_s"] else None
    log(f"[bench] served, float64 one at a time: {base}")
    sweep = []
    for r in [float(x) for x in args.serve_sweep.split(",") if x.strip()]:
        cnt = int(min(args.serve_count, max(16, round(r * args.serve_window))))
        arr_r = fi.served_stream(r, cnt, seed=5, n1d=(1023, 65535))
        res, _ = serve.serve_stream(arr_r, slots=slots, precision=fde.MIXED, inner_steps=serve.AUTO)
        st = serve.latency_stats(res, slots)
        st.update(rate_req_per_s=r)
        sweep.append(st)
        log(f"[bench] served at {r}/s: {st}")
    out["sweep"] = sweep
    return out


def _first_step(fde, torch, p, kw, reps=2):
    """First implicit step of problem p on the plan path: (iterations, ms per solve, converged)."""
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").reshape(-1).contiguous()
    with fde.Plan(p, **kw) as plan:
        u = T(p.u0)
        b = torch.empty_like(u)
        plan.rhs(u, b)
        best, info = 1e30, None
        for _ in range(reps):
            x = u.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = plan.solve(b, x, allow_notconv=True)
            best = min(best, time.perf_counter() - t0)
    return info.iters, 1e3 * best, bool(info.converged)


def table_variants(fi, fde, torch, np):
    """Preconditioner variants on the first implicit step of the 1D (n = 65535)
    and 2D (1023^2) workloads: P_F with D on either side, P_tilde, P_tri, and
    P_F with the symbol shifted by nu/mean(D) (a variant the paper does not use
    for variable coefficients), FGMRES(30) to 1e-8, float64 plan path."""
    rows = []
    for alpha in (1.2, 1.5, 1.8):
        p = fi.variable_1d(n=65535, alpha=alpha, steps=1)
        h = p.h[0]
        nu = h ** alpha / p.dt
        shift = nu / float(np.mean(0.5 * (p.dplus + p.dminus)))
        forms = [("P_F D.tau (text)", dict(prec=fde.P_TAU, dside=fde.D_LEFT)),
                 ("P_F tau.D (tables)", dict(prec=fde.P_TAU, dside=fde.D_RIGHT)),
                 ("P_tilde", dict(prec=fde.P_TILDE)),
                 ("P_tri", dict(prec=fde.P_TRI)),
                 ("P_F D.tau + nu/mean(D) (not in the paper)", dict(prec=fde.P_TAU, dside=fde.D_LEFT, shift=shift))]
        for name, kw in forms:
            it, ms, conv = _first_step(fde, torch, p, dict(maxit=20000, **kw))
            rows.append({"workload": f"1D n=65535 alpha={alpha}", "preconditioner": name, "iters": it,
                         "ms": ms, "converged": conv})
            log(f"[table] {rows[-1]}")
    p = fi.variable_2d(n=1023, steps=1)
    nu = p.h[0] ** p.alpha[0] / p.dt
    shift = nu / float(np.mean(0.25 * (p.dplus + p.dminus + p.eplus + p.eminus)))
    for name, kw in [("P_F D.tau (text)", dict(prec=fde.P_TAU, dside=fde.D_LEFT)),
                     ("P_F tau.D (tables)", dict(prec=fde.P_TAU, dside=fde.D_RIGHT)),
                     ("P_F D.tau + nu/mean(D) (not in the paper)", dict(prec=fde.P_TAU, dside=fde.D_LEFT,
                                                                       shift=shift))]:
        it, ms, conv = _first_step(fde, torch, p, dict(maxit=20000, **kw))
        rows.append({"workload": "2D 1023^2 alpha=(1.7,1.4)", "preconditioner": name, "iters": it, "ms": ms,
                     "converged": conv})
        log(f"[table] {rows[-1]}")
    return rows


def table_paper2d(fi, fde, torch, np):
    """Examples 2 and 3 (second-order weights, Crank-Nicolson, h_t = 1/n, n steps
    to T = 1, with the source) on the GPU with P_F (tau.D, the tables' side),
    FGMRES(30) to 1e-7, at the paper's n = 16, 32, 64, 128 (Tables 3-4; the
    dense 2D form) and n = 2^k - 1 up to 1023: mean iterations per step, time
    per step and the max-norm error against the exact solution at T = 1."""
    rows = []
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").reshape(-1).contiguous()
    for example in (2, 3):
        for n in (16, 32, 64, 128, 15, 31, 63, 127, 255, 511, 1023):
            p = fi.paper_2d(n, example)
            X, Y = p.meta["X"], p.meta["Y"]
            a, b_ = p.alpha
            S = T(fi.example23_source(X, Y, 0.0, a, b_))   # source = e^{-t} S
            with fde.Plan(p, prec=fde.P_TAU, dside=fde.D_RIGHT, tol=p.tol) as plan:
                u = T(p.u0)
                b = torch.empty_like(u)
                f = torch.empty_like(u)
                its = []
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for m in range(1, n + 1):
                    f.copy_(S).mul_(float(np.exp(-(m - 0.5) * p.dt)))
                    plan.rhs(u, b, f=f)
                    its.append(plan.solve(b, u).iters)   # x0 = u^{m-1}, solution in place
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                err = float(np.max(np.abs(u.cpu().numpy().reshape(X.shape) - fi.example23_exact(X, Y, n * p.dt))))
            rows.append({"example": example, "n": n, "steps": n, "iters_mean": float(np.mean(its)),
                         "iters_max": int(max(its)), "ms_per_step": 1e3 * dt / n, "max_error_T1": err})
            log(f"[table] {rows[-1]}")
    return rows


def table_dense(fi, fde, torch, np):
    """The line operators of 2D grids as dense products on the matrix cores
    (MFMA) against the FFT line kernels: per n (the paper's 16 ... 128, the
    served 2D sizes 127 ... 1023, and 1000, which only the dense form takes),
    the time of one preconditioner application plus one matrix-vector product
    (float64, mean of 200 pairs, events on the stream) and the first implicit
    step of the 2D workload's coefficient
    fields solved by FGMRES(30) + P_F to 1e-8 in float64 and mixed.  Sizes
    whose n + 1 is not a power of two have only the dense form; for the others
    FDE_DENSE_LINES=1 selects it."""
    rows = []
    for n in (16, 32, 64, 127, 128, 255, 511, 1000, 1023):
        p = fi.variable_2d(n=n, steps=1)
        pow2 = ((n + 1) & n) == 0
        for form in (("lines", "dense") if pow2 else ("dense",)):
            os.environ["FDE_DENSE_LINES"] = "1" if form == "dense" else "0"
            try:
                with fde.Plan(p) as plan:
                    v = torch.rand(p.N, dtype=torch.float64, device="cuda")
                    z = torch.empty_like(v)
                    w = torch.empty_like(v)
                    for _ in range(5):
                        plan.tau_apply(v, z)
                        plan.matvec(z, w)
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(200):
                        plan.tau_apply(v, z)
                        plan.matvec(z, w)
                    e1.record()
                    torch.cuda.synchronize()
                    pair_us = 1e3 * e0.elapsed_time(e1) / 200
                row = {"n": n, "form": form, "tau_plus_matvec_us": pair_us}
                for prec, kw in (("fp64", dict(precision=fde.FP64)),
                                 ("mixed", dict(precision=fde.MIXED, inner_steps=16))):
                    it, ms, conv = _first_step(fde, torch, p, kw, reps=3)
                    row[f"{prec}_iters"], row[f"{prec}_ms"], row[f"{prec}_converged"] = it, ms, conv
            finally:
                os.environ.pop("FDE_DENSE_LINES", None)
            rows.append(row)
            log(f"[table] {row}")
    return rows


def pcg_leg(fi, fde, torch, np, solves=20):
    """The 1D constant-coefficient system (d+ = d- = 1, n = 1023, alpha =
    1.5) solved by PCG with the Case I preconditioner to 1e-10 from x0 = 0:
    time-to-tol per solve, host clock around each solve."""
    p = fi.constant_1d()
    with fde.Plan(p) as plan:
        b = torch.as_tensor(p.b, dtype=torch.float64, device="cuda").contiguous()
        times, info = [], None
        for _ in range(solves):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = plan.solve(b, x)
            times.append(time.perf_counter() - t0)
    return {"time_to_tol_us_min": 1e6 * min(times), "time_to_tol_us_median": 1e6 * float(np.median(times)),
            "iters": info.iters, "relres": info.relres_true, "converged": bool(info.converged)}


def one_d_legs(args, fi, fde, torch, np):
    """The 1D workloads: (a) the constant-coefficient system (d+ = d- = 1,
    n = 1023, alpha = 1.5) solved by PCG with the Case I preconditioner to
    1e-10, time-to-tol per solve; (b) 20 implicit steps of the 1D
    variable-coefficient problem at n = 65535 for alpha = 1.2, 1.5, 1.8,
    float64 form and the float32-preconditioner form (float32 tau inside the
    float64 FGMRES, no inner Krylov: inner_steps = 0, the faster mixed form on
    long 1D lines), solves per second."""
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda").reshape(-1).contiguous()
    out = {"pcg_constant_1023": pcg_leg(fi, fde, torch, np)}
    log(f"[bench] 1D PCG: {out['pcg_constant_1023']}")
    jobs = {}
    for alpha in (1.2, 1.5, 1.8):
        p = fi.variable_1d(n=65535, alpha=alpha, steps=args.oned_steps if args else 20)
        for name, kw in (("fp64", dict(precision=fde.FP64)), ("mixed", dict(precision=fde.MIXED, inner_steps=0))):
            with fde.Plan(p, **kw) as plan:
                u = T(p.u0)
                bb = torch.empty_like(u)
                its = []
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(p.steps):
                    plan.rhs(u, bb)
                    its.append(plan.solve(bb, u).iters)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
            jobs[f"alpha={alpha} {name}"] = {"solves_per_s": p.steps / dt, "ms_per_solve": 1e3 * dt / p.steps,
                                             "iters_mean": float(np.mean(its))}
            log(f"[bench] 1D job alpha={alpha} {name}: {jobs[f'alpha={alpha} {name}']}")
    out["variable_65535_20_steps"] = jobs
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed jobs per form")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1023)
    ap.add_argument("--tsteps", type=int, default=10)
    ap.add_argument("--inner", type=int, default=16, help="float32 inner GMRES steps of the 2D mixed form")
    ap.add_argument("--batch-inner", type=int, default=0, help="inner steps of the batched mixed form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--forms", default="fp64,mixed,fp64_acc,mixed_acc",
                    help="fp64 / mixed: the workload's tolerance 1e-8; *_acc: the outer tolerance --acc-tol")
    ap.add_argument("--quick", action="store_true",
                    help="skip the per-class sampling pass; probe --probe-class in the timed region")
    ap.add_argument("--probe-class", default="line32_dst_storez_toeplitz")
    ap.add_argument("--serve-rate", type=float, default=500.0, help="Poisson arrival rate of the served leg")
    ap.add_argument("--serve-sweep", default="2,8,50,200,2000",
                    help="further arrival rates of the served leg, reported in served.sweep ('' to skip)")
    ap.add_argument("--serve-window", type=float, default=8.0,
                    help="seconds of arrivals per sweep rate (request count = rate x window, capped)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 1D legs (constant-coefficient PCG time-to-tol, 1D 20-step jobs)")
    ap.add_argument("--serve-count", type=int, default=200, help="requests in the served leg (0: skip)")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--batch-count", type=int, default=512, help="instances of the batched leg (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=2, help="timed time steps of the batched leg")
    ap.add_argument("--batch-cfg", default="",
                    help="variant,grid,lpt,split of the batched launch instead of the tuner's choice")
    ap.add_argument("--batch-plan-sample", type=int, default=512,
                    help="instances solved one plan at a time for the batched-vs-plan comparison")
    ap.add_argument("--only-batched", action="store_true",
                    help="run the batched leg alone (profiling); prints its JSON object")
    ap.add_argument("--only-served", action="store_true",
                    help="run the served leg alone; prints its JSON object")
    ap.add_argument("--acc-tol", type=float, default=1e-9,
                    help="outer tolerance of the accuracy-matched forms (forward error <= 1e-8 against the "
                         "oracle's reference solution)")
    ap.add_argument("--only-1d", action="store_true",
                    help="only the 1D legs (PCG time-to-tol and the n = 65535 jobs), one JSON line")
    ap.add_argument("--oned-steps", type=int, default=20, help="implicit steps of each n = 65535 job")
    ap.add_argument("--only-pcg", action="store_true",
                    help="run the 1D constant-coefficient PCG leg alone (profiling); prints its JSON object")
    ap.add_argument("--table", choices=["variants", "paper2d", "dense"], default=None,
                    help="print a table instead of the benchmark line: preconditioner variants at the "
                         "workload sizes, or the paper's 2D examples extended to n = 1023")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding is a design "
              "note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import fde_inputs as fi
    from paper_1912_13304_amd import fde

    fde.load()
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.only_batched:
        print(json.dumps({"batched": batched_leg(args, fi, fde, torch, np)}), flush=True)
        return
    if args.only_served:
        print(json.dumps({"served": served_leg(args, fi, fde)}), flush=True)
        return
    if args.only_pcg:
        print(json.dumps({"pcg_constant_1023": pcg_leg(fi, fde, torch, np, solves=50)}), flush=True)
        return
    if args.only_1d:
        print(json.dumps({"one_d": one_d_legs(args, fi, fde, torch, np)}), flush=True)
        return
    if args.table == "variants":
        print(json.dumps({"table": "variants", "rows": table_variants(fi, fde, torch, np)}), flush=True)
        return
    if args.table == "dense":
        print(json.dumps({"table": "dense", "rows": table_dense(fi, fde, torch, np)}), flush=True)
        return
    if args.table == "paper2d":
        print(json.dumps({"table": "paper2d", "rows": table_paper2d(fi, fde, torch, np)}), flush=True)
        return
    prob = fi.variable_2d(n=args.n, steps=args.tsteps)
    N = prob.N
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev).reshape(-1).contiguous()
    coef = [T(prob.dplus), T(prob.dminus), T(prob.eplus), T(prob.eminus)]
    u0 = T(prob.u0)
    forms = {"fp64": dict(precision=fde.FP64), "mixed": dict(precision=fde.MIXED, inner_steps=args.inner),
             "fp64_acc": dict(precision=fde.FP64, tol=args.acc_tol),
             "mixed_acc": dict(precision=fde.MIXED, inner_steps=args.inner, tol=args.acc_tol)}
    forms = {k: v for k, v in forms.items() if k in args.forms.split(",")}

    b = torch.empty(N, dtype=torch.float64, device=dev)
    bufs = [torch.empty(N, dtype=torch.float64, device=dev) for _ in range(2)]

    def job(kw, probe=fde.PROBE_OFF, keep_first=False):
        params = fde.params_for(prob, **kw)
        plan = fde.fde_assemble(params, *coef)
        if probe:
            fde.fde_probe(plan, probe)
        u, x = bufs
        u.copy_(u0)
        infos = []
        first = None
        for m in range(args.tsteps):
            fde.fde_rhs(plan, u, None, b)
            x.copy_(u)   # x0 = u^{m-1}
            infos.append(fde.fde_solve(plan, b, x).as_dict())
            if keep_first and m == 0:
                first = x.detach().cpu().numpy()
            u, x = x, u
        pr = fde.fde_probe_read(plan) if probe else None
        fde.fde_destroy(plan)
        return infos, pr, first

    results = {}
    dominant = {}
    for name, kw in forms.items():
        log(f"[bench] warmup {name} x{args.warmup}")
        for _ in range(args.warmup):
            job(kw)
        # one untimed job per kernel class: sampled GPU time of each candidate
        # (every 32nd launch of the class is bracketed with HIP events)
        shares = {}
        cands = [("cgs_dot64", fde.PROBE_MDOT64), ("cgs_update64", fde.PROBE_MAXPY64),
                 ("cgs_dot32", fde.PROBE_MDOT32), ("cgs_update32", fde.PROBE_MAXPY32)]
        for fl, pname in fde.LINE_PROGRAMS.items():
            cands.append((f"line64_{pname}", fde.PROBE_LINE64_VARIANT + fl))
            cands.append((f"line32_{pname}", fde.PROBE_LINE32_VARIANT + fl))
        if args.quick or name.endswith("_acc"):
            keep = args.probe_class if args.quick else dominant.get(name[:-4])
            cands = [c for c in cands if c[0] == keep] or cands[:1]
        for cls_name, cls in cands:
            _, pr, _ = job(kw, probe=cls)
            ms, nl, by = pr
            if nl:
                shares[cls_name] = dict(ms=ms, launches=nl, bytes=by, GBps=by / (ms * 1e-3) / 1e9 if ms else 0.0,
                                        cls=cls, avg_us=1e3 * ms / nl)
        if not shares:
            shares = {cands[0][0]: dict(ms=0.0, launches=0, bytes=0.0, GBps=0.0, cls=cands[0][1], avg_us=0.0)}
        dom = max(shares, key=lambda k: shares[k]["ms"])
        dominant[name] = dom
        log(f"[bench] {name} sampled kernel classes: " + ", ".join(
            f"{k}: {v['ms']:.2f} ms, {v['avg_us']:.1f} us/launch, {v['GBps']:.0f} GB/s" for k, v in shares.items()))
        # timed region: K whole jobs, the dominant kernel class probed with HIP events
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        all_infos = []
        probe_tot = [0.0, 0, 0.0]
        for _ in range(args.steps):
            infos, pr, _ = job(kw, probe=shares[dom]["cls"])
            all_infos.append(infos)
            probe_tot = [probe_tot[0] + pr[0], probe_tot[1] + pr[1], probe_tot[2] + pr[2]]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        solves = args.steps * args.tsteps
        its = [i["iters"] for inf in all_infos for i in inf]
        results[name] = dict(
            solves_per_s=solves / dt, ms_per_job=1e3 * dt / args.steps, ms_per_solve=1e3 * dt / solves,
            iters_per_solve=float(np.mean(its)), iters_first_step=all_infos[0][0]["iters"],
            inner_iters_per_solve=float(np.mean([i["inner_iters"] for inf in all_infos for i in inf])),
            max_relres=float(max(i["relres_true"] for inf in all_infos for i in inf)),
            all_converged=all(i["converged"] for inf in all_infos for i in inf),
            kernel_classes_sampled={k: dict(ms=v["ms"], avg_us=v["avg_us"], GBps=v["GBps"],
                                            launches=v["launches"]) for k, v in shares.items()},
            dominant=dict(cls=dom, ms=probe_tot[0], launches=probe_tot[1], bytes=probe_tot[2]),
        )
        # whole-iteration roofline: modelled algorithmic bytes of all the
        # solves of the timed jobs over their wall time
        mb = sum(model_bytes_2d(N, i["iters"], i["inner_iters"], 30, name.startswith("mixed"))
                 for inf in all_infos for i in inf)
        results[name]["iteration_roofline"] = dict(
            model_bytes_per_solve=mb / solves, GBps=mb / dt / 1e9, frac=mb / dt / 1e9 / PEAK_HBM_GBS,
            peak=PEAK_HBM_GBS, note="all kernels of the solve; bytes from model_bytes_2d, time = wall time of "
                                    "the timed jobs (assembly and right-hand sides included)")
        log(f"[bench] {name}: {results[name]['solves_per_s']:.1f} solves/s, "
            f"{results[name]['ms_per_solve']:.2f} ms/solve, {results[name]['iters_per_solve']:.1f} it/solve, "
            f"whole-iteration {results[name]['iteration_roofline']['GBps']:.0f} GB/s")

    # the batched leg runs before the served one: its heavy instances overlap
    # the persistent launch on worker streams only while those streams get
    # hardware queues of their own, and the served leg leaves a pool of
    # streams that share the process's few queues
    batched = batched_leg(args, fi, fde, torch, np) if args.batch_count > 0 else None

    served = served_leg(args, fi, fde) if args.serve_count > 0 else None
    legs_1d = None if args.no_configs else one_d_legs(args, fi, fde, torch, np)

    # plain copy bandwidth on the same GPU (1 GiB read + 1 GiB write)
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 10 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst

    head = "mixed" if "mixed" in results else "fp64"
    d = results[head]["dominant"]
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9 if d["ms"] > 0 else 0.0
    avg_us = 1e3 * d["ms"] / max(1, d["launches"])
    alg_per_launch = d["bytes"] / max(1, d["launches"])
    traffic = measured_traffic(d["cls"])

    # CPU oracle on a bounded sample: the first solve of the job
    cpu = None
    parity = None
    if not args.no_cpu:
        from oracle import krylov, precond as pc
        from oracle.system import FDESystem
        cores = min(16, len(os.sched_getaffinity(0)))
        s = FDESystem.from_problem(prob, workers=cores)
        P = pc.make("tau", s, workers=cores)
        u0h = prob.u0.reshape(-1)
        bh = s.rhs(u0h)
        log(f"[bench] CPU oracle: first solve of the job on {cores} threads")
        t0 = time.perf_counter()
        xo, io = krylov.fgmres(s.matvec, bh, P, x0=u0h, restart=30, tol=prob.tol)
        tc = time.perf_counter() - t0
        cpu = {"value": 1.0 / tc, "unit": "solves/s", "cores": cores, "kind": "oracle",
               "sample": f"first implicit-Euler solve of the job (1 of {args.tsteps}), FP64 FGMRES(30)+P_F "
                         f"to 1e-8, {io['iters']} iterations, {tc:.1f} s"}
        # parity of the same solve on the GPU: FP64 form (mirror of the
        # oracle's FGMRES) and mixed form (a different Krylov path to the same
        # tolerance), each with its true residual recomputed by the oracle
        parity = {"oracle_iters": io["iters"], "tol": prob.tol, "acc_tol": args.acc_tol}
        firsts = {}
        for fname, fkw in forms.items():
            _, _, first = job(fkw, keep_first=True)
            firsts[fname] = first
            parity[f"{fname}_first_solve_rel_diff"] = float(np.linalg.norm(first - xo) / np.linalg.norm(xo))
            parity[f"{fname}_first_solve_true_relres"] = float(np.linalg.norm(bh - s.matvec(first)) /
                                                              np.linalg.norm(bh))
        # the error of each form itself: against the oracle's reference
        # solution of the same step (its FGMRES continued from its 1e-8
        # solution to a true residual of 1e-12)
        t0r = time.perf_counter()
        xt, it_ = krylov.fgmres(s.matvec, bh, P, x0=xo, restart=30, tol=1e-12)
        log(f"[bench] oracle reference solution: {time.perf_counter() - t0r:.1f} s")
        parity["reference_true_relres"] = float(np.linalg.norm(bh - s.matvec(xt)) / np.linalg.norm(bh))
        for fname, first in firsts.items():
            parity[f"{fname}_first_solve_error_vs_reference"] = float(np.linalg.norm(first - xt) /
                                                                    np.linalg.norm(xt))
        parity["oracle_error_vs_reference"] = float(np.linalg.norm(xo - xt) / np.linalg.norm(xt))
        if "mixed_acc" in firsts:
            parity["mixed_acc_meets_1e-8"] = parity["mixed_acc_first_solve_error_vs_reference"] <= 1e-8
        log(f"[bench] oracle {tc:.1f} s, parity {parity}")

    out = {
        "metric": "2D 1023^2 GMRES+P_Falpha time-to-tol & solves/s, mixed vs FP64; p99 served latency",
        "value": results[head]["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results[head]["ms_per_job"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"2D {args.n}x{args.n} variable-coefficient FDE, alpha=(1.7,1.4), dt=h, "
                               f"{args.tsteps} implicit-Euler steps per job, FGMRES(30)+P_F to 1e-8, x0=u^(m-1)",
                   "n": args.n, "N": N, "time_steps_per_job": args.tsteps, "restart": 30, "tol": prob.tol,
                   "inner_steps": args.inner},
        "forms": results,
        "time_to_tol_ms": {k: v["ms_per_solve"] for k, v in results.items()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": d["cls"],
                     "algorithmic_bytes_per_launch": alg_per_launch, "avg_launch_us": avg_us,
                     "copy_GBps": copy_gbs},
        "served": served,
        "batched": batched,
        "one_d": legs_1d,
        "p99_served_latency_ms": served["p99_ms"] if served else None,
        "cpu_baseline": cpu,
        "parity": parity,
        "process": process_state(),
    }
    print(json.dumps(out), flush=True)


def process_state():
    """What this process leaves running when it prints its line: child
    processes (none are started: the served and batched legs use threads)
    and live threads (the server's workers have been joined)."""
    import threading
    try:
        import psutil
        children = len(psutil.Process().children(recursive=True))
    except ImportError:
        children = None
    return {"pid": os.getpid(), "child_processes": children, "threads": threading.active_count()}


if __name__ == "__main__":
    main()

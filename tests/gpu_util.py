"""Helpers shared by the GPU tests (no solver arithmetic here)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_13304_amd import fde
    fde.load()   # raises when the library is missing: no silent fallback
    return fde


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda").reshape(-1).contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rounding_spread(s, b, P, x0, restart=30, tol=1e-8):
    """How far the oracle's own FGMRES iterate moves when its matrix-vector
    product carries an error of the size FFT rounding leaves in a Toeplitz
    product: per component u log2(L) ||g||_2 ||x||_2 / sqrt(N), scaled by the
    local coefficients, L the circulant length (1D systems).  Ill-conditioned
    systems (alpha near 2, long lines) amplify such differences past 1e-10."""
    from oracle import krylov
    xo, _ = krylov.fgmres(s.matvec, b, P, x0=x0, restart=restart, tol=tol)
    n = s.N
    L = 2 * (1 << int(np.ceil(np.log2(max(n, 1)))))
    r = np.random.default_rng(7).standard_normal(n)
    scale = 2.0 ** -53 * np.log2(L) * (s.dplus + s.dminus).reshape(-1) * np.linalg.norm(s.gx) / np.sqrt(n)
    xp, _ = krylov.fgmres(lambda x: s.matvec(x) + scale * np.linalg.norm(x) * r, b, P, x0=x0,
                          restart=restart, tol=tol)
    return relerr(xp, xo)


def mirror_check(xg, ig, oracle_run, gpu_run, rel=1e-10, spread=None):
    """Mirror parity of a GPU Krylov solve with the oracle's build-mode solve
    of the same system from the same start: iteration counts within one, and
    the two iterates at the same step count within `rel`.

    oracle_run(maxit) and gpu_run(maxit) rerun either side with an iteration
    cap (None: no cap) and return (x, iters).  When the two stopping points
    differ by one step, the side that ran longer is rerun with the other
    side's count, so that iterates of equal step count are compared.
    Where the system amplifies rounding past `rel`, `spread` (a callable
    returning rounding_spread of the system) relaxes the bound to ten times
    the oracle's own spread, capped at 1e-8.
    Returns (oracle iters, relative difference)."""
    xo, io = oracle_run(None)
    d = ig - io
    assert abs(d) <= 1, (ig, io)
    if d == 0:
        e = relerr(xg, xo)
    elif d > 0:
        xg2, _ = gpu_run(io)
        e = relerr(xg2, xo)
    else:
        xo2, _ = oracle_run(ig)
        e = relerr(xg, xo2)
    if e >= rel and spread is not None:
        rel = min(1e-8, max(rel, 10.0 * spread()))
    assert e < rel, (e, ig, io)
    return io, e

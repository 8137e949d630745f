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


def mirror_check(xg, ig, oracle_run, gpu_run, rel=1e-10):
    """Mirror parity of a GPU Krylov solve with the oracle's build-mode solve
    of the same system from the same start: iteration counts within one, and
    the two iterates at the same step count within `rel`.

    oracle_run(maxit) and gpu_run(maxit) rerun either side with an iteration
    cap (None: no cap) and return (x, iters).  When the two stopping points
    differ by one step, the side that ran longer is rerun with the other
    side's count, so that iterates of equal step count are compared.
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
    assert e < rel, (e, ig, io)
    return io, e

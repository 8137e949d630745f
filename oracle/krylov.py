"""Krylov solvers.

Build mode (what the GPU library computes):
  * ``fgmres``: right-preconditioned flexible GMRES(m).  Each Arnoldi step
    z_j = P^{-1} v_j, w = M z_j, classical Gram-Schmidt applied twice (CGS2),
    Givens rotations on the Hessenberg column, estimate |g_{j+1}|.  A cycle ends
    when the estimate is <= tol ||b||, when m steps are done, or on breakdown;
    then x += Z y and the true residual ||b - M x|| decides: stop when it is
    <= tol ||b||, restart from it otherwise.  Iterations count Arnoldi steps.
    The paper runs GMRES (Section 4); left/right side, restart and starting
    vector are not stated there, and the flexible right-preconditioned form is
    the one whose stopping test is on the true residual.
  * ``pcg``: preconditioned conjugate gradients for the symmetric positive
    definite constant-coefficient case (M and tau(p + nu) are SPD, Section 3.1
    Case I); stops on the recursive residual, confirmed by the true residual.

Paper mode (reproduces Tables 1-4): ``gmres_left``, unrestarted GMRES on
P^{-1} M x = P^{-1} b with x0 = 0, modified Gram-Schmidt, stopping when the
preconditioned residual estimate falls below tol times its initial value
(tolerance 1e-7, Section 4).
"""
import numpy as np
import scipy.linalg


def _givens(h, j, cs, sn, g):
    """Apply rotations 0..j-1 to column h (length j+2, h[j+1] = ||w||), make
    rotation j, update g.  Returns the new residual estimate |g[j+1]|."""
    for i in range(j):
        a, b = h[i], h[i + 1]
        h[i] = cs[i] * a + sn[i] * b
        h[i + 1] = -sn[i] * a + cs[i] * b
    a, b = h[j], h[j + 1]
    rho = np.hypot(a, b)
    if rho == 0.0:
        cs[j], sn[j] = 1.0, 0.0
    else:
        cs[j], sn[j] = a / rho, b / rho
    h[j] = rho
    h[j + 1] = 0.0
    g[j + 1] = -sn[j] * g[j]
    g[j] = cs[j] * g[j]
    return abs(g[j + 1])


def fgmres(A, b, P, x0=None, restart=30, tol=1e-8, maxit=100000, history=False):
    """Right-preconditioned FGMRES(restart) with CGS2.  ``A`` and ``P`` map a
    flat float64 vector to a flat float64 vector (P may be any nonlinear map,
    e.g. an inner solve)."""
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    N = b.size
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64).reshape(-1)
    info = dict(iters=0, restarts=0, converged=False, relres_true=0.0, relres_est=0.0,
                hist=[])
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        info.update(converged=True)
        return np.zeros(N), info
    r = b - A(x)
    beta = np.linalg.norm(r)
    info["relres_true"] = beta / bnorm
    if beta <= tol * bnorm:
        info["converged"] = True
        return x, info
    m = restart
    while True:
        V = np.zeros((m + 1, N))
        Z = np.zeros((m, N))
        R = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            z = P(V[j])
            w = A(z)
            Vj = V[: j + 1]
            h1 = Vj @ w
            w = w - Vj.T @ h1
            h2 = Vj @ w
            w = w - Vj.T @ h2
            h = np.zeros(j + 2)
            h[: j + 1] = h1 + h2
            hn = np.linalg.norm(w)
            h[j + 1] = hn
            info["iters"] += 1
            est = _givens(h, j, cs, sn, g)
            R[: j + 2, j] = h
            Z[j] = z
            k = j + 1
            if history:
                info["hist"].append(est / bnorm)
            info["relres_est"] = est / bnorm
            if est <= tol * bnorm or hn == 0.0 or info["iters"] >= maxit:
                break
            V[j + 1] = w / hn
        y = scipy.linalg.solve_triangular(R[:k, :k], g[:k], lower=False)
        x = x + Z[:k].T @ y
        r = b - A(x)
        beta = np.linalg.norm(r)
        info["relres_true"] = beta / bnorm
        if beta <= tol * bnorm:
            info["converged"] = True
            break
        if info["iters"] >= maxit:
            break
        info["restarts"] += 1
    return x, info


def pcg(A, b, P, x0=None, tol=1e-10, maxit=100000, history=False):
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    N = b.size
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64).reshape(-1)
    info = dict(iters=0, restarts=0, converged=False, relres_true=0.0, relres_est=0.0, hist=[])
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        info["converged"] = True
        return np.zeros(N), info
    r = b - A(x)
    rn = np.linalg.norm(r)
    info["relres_true"] = rn / bnorm
    if rn <= tol * bnorm:
        info["converged"] = True
        return x, info
    z = P(r)
    p = z.copy()
    rz = r @ z
    while info["iters"] < maxit:
        q = A(p)
        a = rz / (p @ q)
        x = x + a * p
        r = r - a * q
        info["iters"] += 1
        rn = np.linalg.norm(r)
        info["relres_est"] = rn / bnorm
        if history:
            info["hist"].append(rn / bnorm)
        if rn <= tol * bnorm:
            rt = b - A(x)
            tn = np.linalg.norm(rt)
            info["relres_true"] = tn / bnorm
            if tn <= tol * bnorm:
                info["converged"] = True
                break
            info["restarts"] += 1
            r = rt
            z = P(r)
            p = z.copy()
            rz = r @ z
            continue
        z = P(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    if not info["converged"]:
        info["relres_true"] = np.linalg.norm(b - A(x)) / bnorm
    return x, info


def gmres_left(A, b, Pinv, tol=1e-7, maxit=None):
    """Unrestarted GMRES on P^{-1} A x = P^{-1} b from x0 = 0 with modified
    Gram-Schmidt.  Returns (x, number of Arnoldi steps)."""
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    N = b.size
    maxit = N if maxit is None else maxit
    r0 = Pinv(b)
    beta = np.linalg.norm(r0)
    if beta == 0.0:
        return np.zeros(N), 0
    V = np.zeros((maxit + 1, N))
    R = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    V[0] = r0 / beta
    k = 0
    for j in range(maxit):
        w = Pinv(A(V[j]))
        h = np.zeros(j + 2)
        for i in range(j + 1):
            h[i] = V[i] @ w
            w = w - h[i] * V[i]
        hn = np.linalg.norm(w)
        h[j + 1] = hn
        est = _givens(h, j, cs, sn, g)
        R[: j + 2, j] = h
        k = j + 1
        if est <= tol * beta or hn == 0.0:
            break
        V[j + 1] = w / hn
    y = scipy.linalg.solve_triangular(R[:k, :k], g[:k], lower=False)
    return V[:k].T @ y, k

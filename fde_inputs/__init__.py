"""Seeded synthetic inputs for the space-fractional diffusion workloads.

This module is shared by the oracle and by the GPU path.  It holds only the
problem data (grids, diffusion-coefficient fields, initial states, right-hand
sides and the arrival stream of the served workload) and none of the solver's
arithmetic: no Grunwald weights, no symbols, no transforms, no Krylov steps.

Workload recipes follow the problem statement of the paper (eq. (1): domain,
alpha in (1,2), nonnegative coefficients d+-, e+-) and the coefficient fields of
its Example 1 (Section 4): d+(x) = Gamma(3-alpha) x^alpha, d-(x) =
Gamma(3-alpha) (2-x)^alpha on (0, 2).  The 2D fields extend that pattern
separably with a (1+y) / (1+x) factor.  Random data is drawn from
``numpy.random.default_rng(seed)`` so that both sides see identical bytes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Problem:
    """One implicit-Euler (or Crank-Nicolson) time-stepping job.

    Arrays are float64.  2D arrays have shape (n2, n1), x fastest, which is the
    lexicographic ordering of Section 1.4.
    """

    dim: int
    n: tuple                 # (n1,) or (n1, n2)
    alpha: tuple             # (alpha_x,) or (alpha_x, alpha_y)
    lo: tuple
    hi: tuple
    dt: float
    dplus: np.ndarray
    dminus: np.ndarray
    eplus: Optional[np.ndarray] = None
    eminus: Optional[np.ndarray] = None
    u0: Optional[np.ndarray] = None    # initial state (time stepping)
    b: Optional[np.ndarray] = None     # right-hand side (single solve)
    steps: int = 1
    tol: float = 1e-8
    solver: str = "gmres"              # "gmres" | "pcg"
    restart: int = 30
    weights: str = "shifted"           # "shifted" (T, g_k) | "weighted" (S, w_k)
    time: str = "euler"                # "euler" | "cn"
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def shape(self) -> tuple:
        return (self.n[0],) if self.dim == 1 else (self.n[1], self.n[0])

    @property
    def h(self) -> tuple:
        return tuple((self.hi[i] - self.lo[i]) / (self.n[i] + 1) for i in range(self.dim))


def grid(n: int, lo: float, hi: float):
    """Interior grid x_i = lo + i h, i = 1..n, h = (hi - lo)/(n + 1)."""
    h = (hi - lo) / (n + 1)
    return lo + h * np.arange(1, n + 1, dtype=np.float64), h


def example1_coefficients(alpha: float, x: np.ndarray):
    """d+(x) = Gamma(3-a) x^a, d-(x) = Gamma(3-a) (2-x)^a (Example 1)."""
    c = math.gamma(3.0 - alpha)
    return c * x ** alpha, c * (2.0 - x) ** alpha


def separable_2d_coefficients(ax: float, ay: float, x: np.ndarray, y: np.ndarray):
    """2D fields of the headline workload, (n2, n1) arrays.

    d+ = G(3-ax) x^ax (1+y), d- = G(3-ax) (2-x)^ax (1+y),
    e+ = G(3-ay) y^ay (1+x), e- = G(3-ay) (2-y)^ay (1+x).
    """
    X, Y = np.meshgrid(x, y)  # (n2, n1), x fastest
    cx, cy = math.gamma(3.0 - ax), math.gamma(3.0 - ay)
    dp = cx * X ** ax * (1.0 + Y)
    dm = cx * (2.0 - X) ** ax * (1.0 + Y)
    ep = cy * Y ** ay * (1.0 + X)
    em = cy * (2.0 - Y) ** ay * (1.0 + X)
    return dp, dm, ep, em


def example23_fields(n: int, alpha: float, beta: float):
    """Coefficient fields of Examples 2 and 3 (Section 4) on (0,2)^2, (n, n)
    arrays x fastest: d+ = G(3-a)(1+x)^a(1+y)^2, d- = G(3-a)(3-x)^a(3-y)^2,
    e+ = G(3-b)(1+x)^2(1+y)^b, e- = G(3-b)(3-x)^2(3-y)^b."""
    x, h = grid(n, 0.0, 2.0)
    X, Y = np.meshgrid(x, x)
    ca, cb = math.gamma(3.0 - alpha), math.gamma(3.0 - beta)
    dp = ca * (1 + X) ** alpha * (1 + Y) ** 2
    dm = ca * (3 - X) ** alpha * (3 - Y) ** 2
    ep = cb * (1 + X) ** 2 * (1 + Y) ** beta
    em = cb * (3 - X) ** 2 * (3 - Y) ** beta
    return X, Y, dp, dm, ep, em


def example23_exact(X, Y, t: float):
    """Exact solution of Examples 2 and 3: 16 e^{-t} x^2 (2-x)^2 y^2 (2-y)^2."""
    return 16.0 * math.exp(-t) * X ** 2 * (2 - X) ** 2 * Y ** 2 * (2 - Y) ** 2


def _g23(gam, x, y):
    return ((8 * x ** (2 - gam) - 24 * x ** (3 - gam) / (3 - gam)
             + 24 * x ** (4 - gam) / ((4 - gam) * (3 - gam)))
            * (1 + x) ** gam * (1 + y) ** 2 * y ** 2 * (2 - y) ** 2)


def example23_source(X, Y, t: float, alpha: float, beta: float):
    """Source term of Examples 2 and 3 (Section 4) at time t."""
    return -16.0 * math.exp(-t) * (X ** 2 * (2 - X) ** 2 * Y ** 2 * (2 - Y) ** 2
                                   + _g23(alpha, X, Y) + _g23(alpha, 2 - X, 2 - Y)
                                   + _g23(beta, Y, X) + _g23(beta, 2 - Y, 2 - X))


def paper_2d(n: int, example: int = 2, tol: float = 1e-7) -> Problem:
    """Example 2 (alpha, beta = 1.8, 1.6) or Example 3 (1.8, 1.2): second-order
    weights, Crank-Nicolson, h_t = 1/n, n steps to T = 1, u0 the exact
    solution at t = 0 (the source is example23_source at t_{m-1/2})."""
    alpha, beta = (1.8, 1.6) if example == 2 else (1.8, 1.2)
    X, Y, dp, dm, ep, em = example23_fields(n, alpha, beta)
    return Problem(dim=2, n=(n, n), alpha=(alpha, beta), lo=(0.0, 0.0), hi=(2.0, 2.0), dt=1.0 / n,
                   dplus=dp, dminus=dm, eplus=ep, eminus=em, u0=example23_exact(X, Y, 0.0),
                   steps=n, tol=tol, weights="weighted", time="cn", name=f"ex{example}-n{n}",
                   meta={"X": X, "Y": Y})


def uniform(rng, shape):
    return rng.uniform(-1.0, 1.0, size=shape)


# --------------------------------------------------------------------------
# Workloads.  Sizes of the full configurations, plus scaled-down versions that
# keep the structure (same coefficient pattern, same alpha, same dt = h rule)
# for parity tests the oracle finishes in seconds.
# --------------------------------------------------------------------------

def constant_1d(n: int = 1023, alpha: float = 1.5, seed: int = 1) -> Problem:
    """1D constant coefficients d+ = d- = 1 on (0,2), dt = h, one solve of
    (nu I + T + T^T) u = b with b ~ U[-1,1]; PCG to 1e-10."""
    rng = np.random.default_rng(seed)
    x, h = grid(n, 0.0, 2.0)
    one = np.ones(n)
    return Problem(dim=1, n=(n,), alpha=(alpha,), lo=(0.0,), hi=(2.0,), dt=h,
                   dplus=one.copy(), dminus=one.copy(), b=uniform(rng, n),
                   steps=1, tol=1e-10, solver="pcg", name=f"1d-const-n{n}-a{alpha}")


def variable_1d(n: int = 65535, alpha: float = 1.5, seed: int = 2, steps: int = 20,
                factor: float = 1.0, tol: float = 1e-8) -> Problem:
    """1D variable coefficients of Example 1 on (0,2), dt = h, u0 ~ U[-1,1],
    f = 0, GMRES(30) to 1e-8."""
    rng = np.random.default_rng(seed)
    x, h = grid(n, 0.0, 2.0)
    dp, dm = example1_coefficients(alpha, x)
    return Problem(dim=1, n=(n,), alpha=(alpha,), lo=(0.0,), hi=(2.0,), dt=h,
                   dplus=factor * dp, dminus=factor * dm, u0=uniform(rng, n),
                   steps=steps, tol=tol, name=f"1d-var-n{n}-a{alpha}")


def variable_2d(n: int = 1023, ax: float = 1.7, ay: float = 1.4, seed: int = 3,
                steps: int = 10, tol: float = 1e-8, n2: Optional[int] = None) -> Problem:
    """2D variable coefficients on (0,2)^2 (separable fields above), dt = h,
    u0 ~ U[-1,1], f = 0, FGMRES(30) to 1e-8."""
    n1 = n
    n2 = n if n2 is None else n2
    rng = np.random.default_rng(seed)
    x, hx = grid(n1, 0.0, 2.0)
    y, _ = grid(n2, 0.0, 2.0)
    dp, dm, ep, em = separable_2d_coefficients(ax, ay, x, y)
    return Problem(dim=2, n=(n1, n2), alpha=(ax, ay), lo=(0.0, 0.0), hi=(2.0, 2.0), dt=hx,
                   dplus=dp, dminus=dm, eplus=ep, eminus=em, u0=uniform(rng, (n2, n1)),
                   steps=steps, tol=tol, name=f"2d-var-n{n1}x{n2}-a{ax},{ay}")


def batched_1d(count: int = 512, seed: int = 4, nmin: int = 255, nmax: int = 16383,
               steps: int = 20, pow2: bool = False) -> list:
    """Independent 1D variable-coefficient instances: n log-uniform in
    [nmin, nmax], alpha ~ U(1.1, 1.9), coefficients of Example 1 scaled by a
    factor ~ U(0.5, 2), dt = h, u0 ~ U[-1,1].  With pow2=True, n is rounded
    to the nearest 2^k - 1 (the sizes the power-of-two transforms take)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        if pow2:
            n = (1 << max(3, int(round(math.log2(n + 1))))) - 1
        alpha = float(rng.uniform(1.1, 1.9))
        fac = float(rng.uniform(0.5, 2.0))
        x, h = grid(n, 0.0, 2.0)
        dp, dm = example1_coefficients(alpha, x)
        u0 = uniform(rng, n)
        out.append(Problem(dim=1, n=(n,), alpha=(alpha,), lo=(0.0,), hi=(2.0,), dt=h,
                           dplus=fac * dp, dminus=fac * dm, u0=u0, steps=steps,
                           tol=1e-8, name=f"batch{i}-n{n}-a{alpha:.3f}"))
    return out


@dataclass
class Arrival:
    t: float          # arrival time, seconds from stream start
    problem: Problem


def served_stream(rate: float, count: int, seed: int = 5, pow2: bool = False,
                  n1d=(1023, 65535), n2d=(127, 255, 511, 1023),
                  steps=(5, 50)) -> list:
    """Poisson arrivals of time-stepping requests: 70% 1D (n log-uniform in
    n1d, any integer; pow2=True rounds it to the nearest 2^k - 1), 30% 2D with
    n in n2d; alpha ~ U(1.1, 1.9); 5..50 steps each."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        s = int(rng.integers(steps[0], steps[1] + 1))
        if rng.uniform() < 0.7:
            n = int(round(math.exp(rng.uniform(math.log(n1d[0]), math.log(n1d[1])))))
            if pow2:
                n = (1 << max(3, int(round(math.log2(n + 1))))) - 1
            p = variable_1d(n=n, alpha=float(rng.uniform(1.1, 1.9)),
                            seed=int(rng.integers(1 << 30)), steps=s)
        else:
            n = int(rng.choice(n2d))
            p = variable_2d(n=n, ax=float(rng.uniform(1.1, 1.9)), ay=float(rng.uniform(1.1, 1.9)),
                            seed=int(rng.integers(1 << 30)), steps=s)
        p.name = f"req{i}-" + p.name
        out.append(Arrival(t=t, problem=p))
    return out

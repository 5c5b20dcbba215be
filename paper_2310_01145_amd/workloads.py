"""Seeded synthetic workloads.  Problem specifications and random draws only:
nothing here performs any of the solver's arithmetic, so both the GPU path
and the CPU oracle can take their inputs from this module.

Problems:
  logistic_c0  -- logistic ODE of the experiments section: y' = y(1-y),
                  y0 = 0.01, t in [0, 10], IWP(2), N = 1000.
  fhn(N)       -- FitzHugh-Nagumo, a = b = 0.2, c = 3, y0 = (-1, 1), t in [0, 100],
                  IWP(3) (D = 8), N swept over 2^12..2^18.
  lorenz(N)    -- Lorenz-63, sigma = 10, rho = 28, beta = 8/3, y0 = (1, 1, 1),
                  t in [0, 20], IWP(4) (D = 15), N = 2^18.
  served_stream(n) -- mixed requests: logistic / FitzHugh-Nagumo / Lotka-Volterra
                  (alpha, beta, gamma, delta ~ U[0.5, 1.5], y0 ~ U[0.5, 2]^2),
                  q ~ U{2, 3, 4}, N log-uniform in [256, 65536].

  mol(d, ...)  -- method of lines for the heat/reaction chain u_t = nu u_xx + u(1-u)
                  on d periodic grid points, nu = 0.01, IWP(2) (D = 3d), N = 4096,
                  t in [0, 1]; mol_batch(B) gives B seeded initial profiles
                  u0 = 0.5 + 0.1 sin(2 pi x_i) + N(0, 0.01^2) noise (seed = instance).

reference_start(spec) gives a starting trajectory near a problem's solution
(the values of a classical Runge-Kutta solution from scipy, an input like any
other).
"""
from __future__ import annotations

import math

import numpy as np


def logistic_c0():
    return dict(name="logistic", field="logistic", params=[], y0=[0.01], t0=0.0, t1=10.0, q=2, N=1000)


def fhn(N=1 << 18, q=3):
    return dict(name="fhn", field="fhn", params=[0.2, 0.2, 3.0], y0=[-1.0, 1.0], t0=0.0, t1=100.0, q=q, N=int(N))


def lorenz(N=1 << 18, q=4, t1=20.0):
    return dict(name="lorenz", field="lorenz", params=[10.0, 28.0, 8.0 / 3.0], y0=[1.0, 1.0, 1.0], t0=0.0, t1=t1,
                q=q, N=int(N))


def lotka_volterra(rng, N, q):
    al, be, ga, de = rng.uniform(0.5, 1.5, size=4)
    y0 = rng.uniform(0.5, 2.0, size=2)
    return dict(name="lotka_volterra", field="lotka_volterra", params=[al, be, ga, de], y0=list(y0), t0=0.0, t1=15.0,
                q=q, N=int(N))


def served_stream(n_requests=4096, seed=0):
    """Requests in arrival order (field, q, N drawn per request)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_requests):
        kind = rng.integers(0, 3)
        q = int(rng.integers(2, 5))
        N = int(math.floor(math.exp(rng.uniform(math.log(256), math.log(65536)))))
        if kind == 0:
            p = dict(logistic_c0(), q=q, N=N)
        elif kind == 1:
            p = fhn(N, q)
        else:
            p = lotka_volterra(rng, N, q)
        out.append(p)
    return out


def mol_initial(d, seed):
    rng = np.random.default_rng(seed)
    x = np.arange(d) / d
    return 0.5 + 0.1 * np.sin(2 * np.pi * x) + rng.normal(0.0, 0.01, size=d)


def mol(d=64, N=4096, q=2, nu=0.01, seed=0, t1=1.0):
    return dict(name="mol_heat_reaction", field="mol_heat_reaction", params=[nu], y0=list(mol_initial(d, seed)),
                t0=0.0, t1=t1, q=q, N=int(N))


def mol_batch(B=16, d=64, N=4096, q=2, nu=0.01, t1=1.0):
    """(spec, y0s [B, d]): instances b = 0..B-1 use seed b."""
    return mol(d, N, q, nu, 0, t1), np.stack([mol_initial(d, b) for b in range(B)])


def random_observations(rng, N, d, q, scale=0.3):
    """Per-step observation data for linear-model tests: Jacobian-like d x d
    matrices J_n = -I + scale * noise and offsets d_n ~ N(0, 1)."""
    J = -np.eye(d)[None] + scale * rng.normal(size=(N, d, d))
    dv = rng.normal(size=(N, d))
    return J, dv


# the vector fields as plain Python, for scipy's integrator only
_FIELDS = {
    "logistic": lambda p, y: [y[0] * (1.0 - y[0])],
    "fhn": lambda p, y: [p[2] * (y[0] - y[0] ** 3 / 3.0 + y[1]), -(y[0] - p[0] + p[1] * y[1]) / p[2]],
    "lorenz": lambda p, y: [p[0] * (y[1] - y[0]), y[0] * (p[1] - y[2]) - y[1], y[0] * y[1] - p[2] * y[2]],
    "lotka_volterra": lambda p, y: [p[0] * y[0] - p[1] * y[0] * y[1], -p[2] * y[1] + p[3] * y[0] * y[1]],
}


def reference_start(spec):
    """[N+1, d(q+1)] starting trajectory near a problem's solution: the
    values of scipy's DOP853 solution (rtol 1e-12) on the grid, derivative
    rows zero (Alg. 2 reads only E0 of a start).  An input like any other,
    for tests that need a start other than the solver's own."""
    from scipy.integrate import solve_ivp

    f = _FIELDS[spec["field"]]
    p = spec["params"]
    q, N = spec["q"], spec["N"]
    ts = np.linspace(spec["t0"], spec["t1"], N + 1)
    sol = solve_ivp(lambda t, y: f(p, y), (spec["t0"], spec["t1"]), spec["y0"], method="DOP853", rtol=1e-12,
                    atol=1e-12, t_eval=ts)
    d = len(spec["y0"])
    tr = np.zeros((N + 1, d * (q + 1)))
    for i in range(d):
        tr[:, i * (q + 1)] = sol.y[i]
    return tr

"""Terrain-weight estimation (test infrastructure only).

Eq. (4) (Alg. 1, Step 3): over a history of H steps, choose the ensemble
weights w minimising

    ||Y_v - F_v w||^2 + ||Y_w - F_w w||^2 + gamma ||w - w_prev||_1
    subject to 0 <= w_i <= 1, sum_i w_i = 1,

where Y are the measured velocity residuals and F[h, i] terrain i's GP mean
at the state of step h.  The oracle solves it as a smooth QP in split
variables (w = w_prev + a - b, a, b >= 0, the L1 term becoming
gamma sum(a + b)) with SciPy's SLSQP, from several starting points.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize


def objective(w, Yv, Yw, Fv, Fw, w_prev, gamma):
    w = np.asarray(w, dtype=np.float64)
    rv = Yv - Fv @ w
    rw = Yw - Fw @ w
    return float(rv @ rv + rw @ rw + gamma * np.abs(w - w_prev).sum())


def solve_weights(Yv, Yw, Fv, Fw, w_prev, gamma):
    Yv, Yw, Fv, Fw = (np.asarray(a, dtype=np.float64) for a in (Yv, Yw, Fv, Fw))
    w_prev = np.asarray(w_prev, dtype=np.float64)
    n = Fv.shape[1]
    F = np.vstack([Fv, Fw])
    Y = np.concatenate([Yv, Yw])
    Q = F.T @ F
    c = F.T @ Y

    def split(z):
        return z[:n], z[n:2 * n]

    def f(z):
        a, b = split(z)
        w = w_prev + a - b
        return float(w @ Q @ w - 2 * c @ w + Y @ Y + gamma * (a.sum() + b.sum()))

    def grad(z):
        a, b = split(z)
        w = w_prev + a - b
        g = 2 * (Q @ w) - 2 * c
        return np.concatenate([g + gamma, -g + gamma])

    cons = [
        {"type": "eq", "fun": lambda z: np.sum(w_prev + z[:n] - z[n:]) - 1.0,
         "jac": lambda z: np.concatenate([np.ones(n), -np.ones(n)])},
        {"type": "ineq", "fun": lambda z: w_prev + z[:n] - z[n:],
         "jac": lambda z: np.hstack([np.eye(n), -np.eye(n)])},
        {"type": "ineq", "fun": lambda z: 1.0 - (w_prev + z[:n] - z[n:]),
         "jac": lambda z: np.hstack([-np.eye(n), np.eye(n)])},
    ]
    bounds = [(0.0, None)] * (2 * n)
    best = None
    starts = [np.full(n, 1.0 / n), w_prev] + [np.eye(n)[i] for i in range(n)]
    for w0 in starts:
        w0 = np.clip(np.asarray(w0, float), 0, 1)
        w0 = w0 / w0.sum()
        d = w0 - w_prev
        z0 = np.concatenate([np.maximum(d, 0), np.maximum(-d, 0)])
        r = minimize(f, z0, jac=grad, bounds=bounds, constraints=cons, method="SLSQP",
                     options={"ftol": 1e-15, "maxiter": 1000})
        a, b = split(r.x)
        w = np.clip(w_prev + a - b, 0.0, 1.0)
        w = w / w.sum()
        val = objective(w, Yv, Yw, Fv, Fw, w_prev, gamma)
        if best is None or val < best[0]:
            best = (val, w)
    return best[1]

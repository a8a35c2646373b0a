"""Dynamic unicycle and covariance propagation (test infrastructure only).

State x = [X, Y, theta, v, w], control u = [v_ref, w_ref] (Sec. III-A).
Positions and heading integrate the velocities; the velocities follow
Eqs. (1)-(2): a nominal model f_v, f_w plus the GP residual.  The paper does
not write f_v, f_w; they are read as first-order lags towards the command,
dv/dt = (v_ref - v)/tau_v, dw/dt = (w_ref - w)/tau_w, and the GP residual is
read as an acceleration, so one explicit Euler step of length dt is

    X+ = X + dt v cos(theta)        Y+ = Y + dt v sin(theta)
    theta+ = theta + dt w
    v+ = v + dt ((v_ref - v)/tau_v + m_v)
    w+ = w + dt ((w_ref - w)/tau_w + m_w)

with every right-hand side evaluated at step k.  Eq. (10) propagates the mean
with the GP mean m and the covariance by a first-order expansion of the
*nominal* dynamics: Sigma+ = A Sigma A^T + diag(0, 0, 0, dt^2 s_v^2, dt^2 s_w^2),
A = d f_nominal / d x at (x_k, u_k), Sigma(0) = 0 (Alg. 1, Step 1).
"""
from __future__ import annotations

import numpy as np


def euler_step(x, u, m, dt, tau_v, tau_w):
    """x [K, 5], u [K, 2], m [K, 2] (GP means; zeros for the nominal model)."""
    X, Y, th, v, w = (x[:, i] for i in range(5))
    out = np.empty_like(x)
    out[:, 0] = X + dt * v * np.cos(th)
    out[:, 1] = Y + dt * v * np.sin(th)
    out[:, 2] = th + dt * w
    out[:, 3] = v + dt * ((u[:, 0] - v) / tau_v + m[:, 0])
    out[:, 4] = w + dt * ((u[:, 1] - w) / tau_w + m[:, 1])
    return out


def nominal_jacobian(x, dt, tau_v, tau_w):
    """A = d(euler_step with m = 0)/dx at x -> [K, 5, 5]."""
    K = x.shape[0]
    th, v = x[:, 2], x[:, 3]
    A = np.zeros((K, 5, 5))
    A[:, 0, 0] = 1.0
    A[:, 0, 2] = -dt * v * np.sin(th)
    A[:, 0, 3] = dt * np.cos(th)
    A[:, 1, 1] = 1.0
    A[:, 1, 2] = dt * v * np.cos(th)
    A[:, 1, 3] = dt * np.sin(th)
    A[:, 2, 2] = 1.0
    A[:, 2, 4] = dt
    A[:, 3, 3] = 1.0 - dt / tau_v
    A[:, 4, 4] = 1.0 - dt / tau_w
    return A


def covariance_step(Sigma, A, s2, dt):
    """Sigma [K,5,5], A [K,5,5], s2 [K,2] predictive GP variances -> Sigma+ (Eq. 10)."""
    out = A @ Sigma @ np.transpose(A, (0, 2, 1))
    out[:, 3, 3] += dt * dt * s2[:, 0]
    out[:, 4, 4] += dt * dt * s2[:, 1]
    return out


def plant_step(x, u, dt, tau_v, tau_w, amplitude=0.3):
    """Synthetic closed-loop plant: the nominal Euler step plus the residual
    amplitude * sin(v w) on both velocity derivatives, without noise.  It
    stands in for the learned ground-truth velocity model of Sec. V-A."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    r = amplitude * np.sin(x[:, 3] * x[:, 4])
    return euler_step(x, np.atleast_2d(u), np.stack([r, r], axis=1), dt, tau_v, tau_w)

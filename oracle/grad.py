"""Gradient of the smoothed expected rollout cost (test infrastructure only).

The differentiation form scores every sample exactly like one MPPI rollout
(Alg. 1 Step 1 with Eqs. 1-3, 10, 11-16 and the combined stage cost of the
hot path), except that the two hard chance indicators are replaced by
logistic sigmoids of temperature tau (metres):

    lane exit   [d_lane > r_bar]        ->  sigmoid((d_lane - r_bar) / tau)
    collision   [min_j d_bar_j <= 0]    ->  sigmoid(-min_j d_bar_j / tau)

and averages the smoothed costs over the K samples:

    J(U, log_ell, log_sf) = (1/K) sum_s S~^s,

the sample mean standing for the expectation in Eq. (5) under common random
numbers (the noise eps is fixed by the seed; u = clip(U + eps), whose
derivative is 1 strictly inside the box and 0 outside).  J depends on the
GP log length-scales and log signal deviations of both outputs through the
kernel vectors, alpha = A^-1 y and A^-1 with A = K(Z, Z) + sn^2 I: the
derivative is total.

The oracle evaluates J with plain float64 torch operations on the CPU
(Cholesky factor and triangular solves as in Rasmussen & Williams Alg. 2.1,
never an explicit inverse) and differentiates it with torch.autograd.  Square
roots use the convention d sqrt(x)/dx = 0 at x = 0 (the covariance is zero
before the first step).  Goal terms, Step-2 tightening and terrain ensembles
are not part of this form.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .constraints import chi2_2_quantile, norm_ppf
from .philox import standard_normals

_F64 = torch.float64


def _sqrt0(x):
    """sqrt with zero derivative at 0 (and 0 for x <= 0)."""
    pos = x > 0
    return torch.where(pos, torch.sqrt(torch.where(pos, x, torch.ones_like(x))), torch.zeros_like(x))


def noise(problem, T: int, sample_ids, seed: int):
    """eps [T, n, 2] of Alg. 1 Step 1 for the given samples (the rollout's stream)."""
    p = problem.params
    ids = np.asarray(sample_ids)
    eps = np.empty((T, len(ids), 2))
    for k in range(T):
        z0, z1 = standard_normals(k, ids, seed, problem.pid)
        eps[k, :, 0] = p["sig_v"] * z0
        eps[k, :, 1] = p["sig_w"] * z1
    return torch.as_tensor(eps, dtype=_F64)


class TorchGP:
    """One exact SE-ARD GP (Sec. III-A) as differentiable torch operations."""

    def __init__(self, Z, y, log_ell, log_sf, log_sn):
        self.Z = torch.as_tensor(np.asarray(Z), dtype=_F64)
        y = torch.as_tensor(np.asarray(y), dtype=_F64)
        self.ell = torch.exp(log_ell)
        self.sf2 = torch.exp(2.0 * log_sf)
        self.sn2 = math.exp(2.0 * float(log_sn))
        Zs = self.Z / self.ell
        d2 = ((Zs[:, None, :] - Zs[None, :, :]) ** 2).sum(-1)
        A = self.sf2 * torch.exp(-0.5 * d2) + self.sn2 * torch.eye(self.Z.shape[0], dtype=_F64)
        self.L = torch.linalg.cholesky(A)
        self.alpha = torch.cholesky_solve(y[:, None], self.L)[:, 0]

    def kvec(self, q):
        """k(q, Z) [n, M]."""
        d2 = (((q[:, None, :] - self.Z[None, :, :]) / self.ell) ** 2).sum(-1)
        return self.sf2 * torch.exp(-0.5 * d2)

    def predict(self, q):
        """Mean and predictive variance sn^2 + max(0, sf^2 - k^T A^-1 k) at q [n, 4]."""
        kq = self.kvec(q)
        mean = kq @ self.alpha
        v = torch.linalg.solve_triangular(self.L, kq.T, upper=False)
        latent = self.sf2 - (v * v).sum(0)
        return mean, self.sn2 + torch.clamp(latent, min=0.0)


def _lane_distance(P, problem):
    if problem.path_kind == 0:
        cx, cy, R = problem.circle
        return torch.abs(torch.sqrt((P[:, 0] - cx) ** 2 + (P[:, 1] - cy) ** 2) - R)
    a = torch.as_tensor(np.asarray(problem.path_pts), dtype=_F64)
    b = torch.roll(a, -1, dims=0)
    e = b - a                                     # [P, 2]
    rel = P[:, None, :] - a[None, :, :]           # [n, P, 2]
    t = torch.clamp((rel * e[None]).sum(-1) / (e * e).sum(-1)[None], 0.0, 1.0)
    d = rel - t[..., None] * e[None]
    best = (d * d).sum(-1).min(dim=1).values
    return _sqrt0(best)


def _lambda_max(a, b, c):
    h = 0.5 * (a - c)
    return 0.5 * (a + c) + _sqrt0(h * h + b * b)


def smoothed_costs(problem, U, log_ell, log_sf, seed: int, tau: float = 0.05, sample_ids=None, x0=None):
    """Per-sample smoothed costs S~ [n] (differentiable in U, log_ell, log_sf)."""
    p = problem.params
    if p.get("w_goal", 0.0) or p.get("w_term", 0.0) or p.get("tighten", 0) or \
            getattr(problem, "terrain_y", None) is not None:
        raise ValueError("the differentiation form has no goal terms, Step-2 tightening or terrains")
    T = U.shape[0]
    ids = np.arange(problem.K) if sample_ids is None else np.asarray(sample_ids)
    n = len(ids)
    dt, tv, tw = p["dt"], p["tau_v"], p["tau_w"]
    gps = [TorchGP(problem.Z[o], problem.y[o], log_ell[o], log_sf[o], problem.log_sn[o]) for o in range(2)]
    eps = noise(problem, T, ids, seed)
    lo = torch.as_tensor(p["u_min"], dtype=_F64)
    hi = torch.as_tensor(p["u_max"], dtype=_F64)
    r = p["half_width"]
    c_p = math.sqrt(chi2_2_quantile(p["p_x"]))
    z_p = norm_ppf(p["p_x"])
    obs = torch.as_tensor(np.asarray(problem.obstacles).reshape(-1, 3), dtype=_F64)
    x0 = problem.x0 if x0 is None else x0
    x = torch.as_tensor(np.asarray(x0), dtype=_F64).expand(n, 5)
    Sig = torch.zeros((n, 5, 5), dtype=_F64)
    S = torch.zeros(n, dtype=_F64)
    for k in range(T):
        u = torch.maximum(torch.minimum(U[k][None, :] + eps[k], hi), lo)
        q = torch.cat([x[:, 3:5], u], dim=1)
        m0, s0 = gps[0].predict(q)
        m1, s1 = gps[1].predict(q)
        X, Y, th, v, w = (x[:, i] for i in range(5))
        # nominal Jacobian at x_k (Eq. 10)
        A = torch.zeros((n, 5, 5), dtype=_F64)
        A[:, 0, 0] = 1.0
        A[:, 0, 2] = -dt * v * torch.sin(th)
        A[:, 0, 3] = dt * torch.cos(th)
        A[:, 1, 1] = 1.0
        A[:, 1, 2] = dt * v * torch.cos(th)
        A[:, 1, 3] = dt * torch.sin(th)
        A[:, 2, 2] = 1.0
        A[:, 2, 4] = dt
        A[:, 3, 3] = 1.0 - dt / tv
        A[:, 4, 4] = 1.0 - dt / tw
        # mean step (Eqs. 1, 2; explicit Euler)
        x = torch.stack([X + dt * v * torch.cos(th),
                         Y + dt * v * torch.sin(th),
                         th + dt * w,
                         v + dt * ((u[:, 0] - v) / tv + m0),
                         w + dt * ((u[:, 1] - w) / tw + m1)], dim=1)
        D = torch.zeros((n, 5, 5), dtype=_F64)
        D[:, 3, 3] = dt * dt * s0
        D[:, 4, 4] = dt * dt * s1
        Sig = A @ Sig @ A.transpose(1, 2) + D
        a, b, c = Sig[:, 0, 0], Sig[:, 0, 1], Sig[:, 1, 1]
        P = x[:, 0:2]
        d_lane = _lane_distance(P, problem)
        r_bar = r - c_p * _sqrt0(_lambda_max(a, b, c))
        cost = (p["w_var"] * (s0 + s1) + p["w_dev"] * d_lane / r
                + p["w_lane"] * p["discount"] ** k * torch.sigmoid((d_lane - r_bar) / tau)
                + p["w_speed"] * (p["v_des"] - x[:, 3]) ** 2)
        if obs.shape[0]:
            dx = P[:, 0:1] - obs[None, :, 0]
            dy = P[:, 1:2] - obs[None, :, 1]
            rho = _sqrt0(dx * dx + dy * dy)
            safe = torch.where(rho > 0, rho, torch.ones_like(rho))
            nx, ny = dx / safe, dy / safe
            var = a[:, None] * nx * nx + 2.0 * b[:, None] * nx * ny + c[:, None] * ny * ny
            var = torch.where(rho > 0, var, _lambda_max(a, b, c)[:, None].expand_as(var))
            dbar = rho - obs[None, :, 2] - z_p * _sqrt0(var)
            cost = cost + p["w_obs"] * torch.sigmoid(-dbar.min(dim=1).values / tau)
        S = S + cost
    return S


def objective(problem, U, log_ell, log_sf, seed: int, tau: float = 0.05, x0=None):
    """J = mean over the problem's K samples of the smoothed cost."""
    return smoothed_costs(problem, U, log_ell, log_sf, seed, tau, x0=x0).mean()


def leaves(problem, U=None):
    """The differentiable inputs (U [T, 2], log_ell [2, 4], log_sf [2]) as float64 leaves."""
    U = problem.U0 if U is None else U
    return (torch.tensor(np.asarray(U), dtype=_F64, requires_grad=True),
            torch.tensor(np.asarray(problem.log_ell), dtype=_F64, requires_grad=True),
            torch.tensor(np.asarray(problem.log_sf), dtype=_F64, requires_grad=True))


def reference_gradient(problem, seed: int, tau: float = 0.05, U=None, x0=None):
    """(J, dJ/dU [T, 2], dJ/dlog_ell [2, 4], dJ/dlog_sf [2]) by reverse-mode autodiff."""
    Ut, le, ls = leaves(problem, U)
    J = objective(problem, Ut, le, ls, seed, tau, x0=x0)
    gU, gl, gs = torch.autograd.grad(J, (Ut, le, ls))
    return float(J.detach()), gU.numpy(), gl.numpy(), gs.numpy()


def central_differences(problem, seed: int, tau: float = 0.05, h: float = 1e-6, U=None):
    """Central differences (J(theta + h) - J(theta - h)) / 2h of every input, in float64."""
    Ut, le, ls = (a.detach() for a in leaves(problem, U))

    def J(a, b, c):
        with torch.no_grad():
            return float(objective(problem, a, b, c, seed, tau))

    out = []
    for which, base in enumerate((Ut, le, ls)):
        g = np.zeros(tuple(base.shape))
        for idx in np.ndindex(*base.shape):
            args_p = [Ut.clone(), le.clone(), ls.clone()]
            args_m = [Ut.clone(), le.clone(), ls.clone()]
            args_p[which][idx] += h
            args_m[which][idx] -= h
            g[idx] = (J(*args_p) - J(*args_m)) / (2 * h)
        out.append(g)
    return tuple(out)

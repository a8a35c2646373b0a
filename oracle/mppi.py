"""One stochastic MPPI iteration and the closed loop (test infrastructure only).

Follows Alg. 1 (Stochastic MPPI), Step 1, with the per-sample uncertainty
propagation of Eq. (10), the chance-constraint tightening of Eqs. (13)-(16)
and one combined stage cost built from the terms of Eqs. (11) and (12).

For every sample s and step k = 0 .. T-1:
  u = clip(U_k + eps_k^s)                          Alg. 1 Step 1, Eq. (8)
  q = (v_k, w_k, u_v, u_w)                         Sec. V-A GP input
  (m_o, s2_o) = GP_o(q), o in {v, w}               Eq. (3), one terrain
  x_{k+1} = Euler(x_k, u, m)                       Eqs. (1), (2), (10)
  Sigma_{k+1} = A Sigma_k A^T + dt^2 diag(0,0,0,s2)  Eq. (10)
  margins at (x_{k+1}, Sigma_{k+1})                Eqs. (13)-(16)
  c_k = w_var (s2_v + s2_w)                        trace of the GP covariance
      + w_dev d_lane / r                           normalised deviation
      + w_lane discount^k [d_lane > r_bar]         lane-exit indicator (tightened)
      + w_speed (v_des - v_{k+1})^2                speed tracking
      + w_obs [min_j d_bar_j <= 0]                 collision indicator (tightened)
  S^s += c_k                                       Eq. (5)
then w^s = exp(-(S^s - min S)/lambda) / sum (the MPPI weights) and
U'_k = sum_s w^s u_k^s (the weighted control update).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import constraints as C
from . import dynamics as D
from . import gp as G
from .philox import sampled_controls

READINGS = {
    "R1": "f_v, f_w are first-order lags; explicit Euler with all terms at step k",
    "R2": "the GP residual is an acceleration: dv = dt m, covariance gains dt^2 s^2",
    "R3": "s^2 = sn^2 + max(0, sf^2 - k^T (K + sn^2 I)^-1 k), the predictive variance",
    "R4": "inducing set = the first M training points (subset of data)",
    "R5": "one terrain with weight 1 unless terrain target sets and weights are given (Eq. 3)",
    "R6": "the covariance Jacobian is that of the nominal dynamics only",
    "R7": "Sigma is propagated per sample along its own rollout",
    "R8": "one combined stage cost; slip and goal terms weigh 0",
    "R9": "speed term (v_des - v_{k+1})^2",
    "R10": "c_k is scored on x_{k+1}, Sigma_{k+1} and the GP variance of query k; discount^k, k from 0",
    "R11": "collision iff d_bar <= 0; lane exit iff d_lane > r_bar",
    "R12": "n = (p - c)/|p - c|; at p = c use sqrt(lambda_max)",
    "R16": "no control-cost term; baseline rho = min S; U' = sum w clip(U + eps)",
    "R17": "closed-loop plant = nominal Euler + dt 0.3 sin(v w) on v and w",
    "R21": "warm start: shift left and repeat the last control",
    "R26": "goal terms (Eq. 12): g = w_goal |p_{k+1} - goal| every step; F = w_term once if no step "
           "of the rollout comes within goal_tol of the goal",
    "R27": "Step 2 tightening (tighten = 1): Sigma propagated once along the nominal sequence "
           "(zero noise, GP mean), its Sigma_XY[k] used for every sample's constraints at step k",
}


@dataclasses.dataclass
class Trace:
    x: np.ndarray            # [T+1, K, 5]
    sxy: np.ndarray          # [T+1, K, 3] (Sigma_XX, Sigma_XY, Sigma_YY)
    gp_mean: np.ndarray      # [T, K, 2]
    gp_var: np.ndarray       # [T, K, 2] predictive variances
    d_lane: np.ndarray       # [T, K]
    lane_margin: np.ndarray  # [T, K]  r_bar - d_lane (exit iff < 0)
    obs_margin: np.ndarray   # [T, K]  min_j d_bar_j (collision iff <= 0; +inf without obstacles)
    u: np.ndarray            # [T, K, 2] sampled, clipped controls
    stage: np.ndarray        # [T, K]  c_k


def param(problem, name):
    return problem.params[name]


def nominal_tightening(problem, x0, U, gps=None):
    """Alg. 1 Step 2: Sigma_XY [T+1, 3] propagated along the nominal controls
    clip(U) (Eq. 10 with the GP mean and variance, no sampling noise)."""
    p = dict(problem.params)
    p.update(sig_v=0.0, sig_w=0.0, tighten=0)
    nominal = dataclasses.replace(problem, params=p)
    _, tr = rollout(nominal, x0, U, 0, gps=gps, sample_ids=np.array([0]))
    return tr.sxy[:, 0, :]


def rollout(problem, x0, U, seed: int, K: Optional[int] = None, gps=None,
            sample_ids: Optional[np.ndarray] = None):
    """Costs S [K] and the full trace for samples 0..K-1 (or the listed ids)."""
    p = problem.params
    K = problem.K if K is None else K
    U = np.asarray(U, dtype=np.float64)
    T = U.shape[0]
    dt, tv, tw = p["dt"], p["tau_v"], p["tau_w"]
    terrains = getattr(problem, "terrain_y", None) is not None
    if gps is None:
        if terrains:
            gps = G.build_terrains(problem.Z, problem.terrain_y, problem.log_ell, problem.log_sf, problem.log_sn)
        else:
            gps = G.build_pair(problem.Z, problem.y, problem.log_ell, problem.log_sf, problem.log_sn)
    ids = np.arange(K) if sample_ids is None else np.asarray(sample_ids)
    K = len(ids)
    u_all = sampled_controls(U, ids, seed, (p["sig_v"], p["sig_w"]), p["u_min"], p["u_max"],
                             problem.pid)
    x = np.tile(np.asarray(x0, dtype=np.float64), (K, 1))
    Sigma = np.zeros((K, 5, 5))
    r = p["half_width"]
    tight = nominal_tightening(problem, x0, U, gps) if p.get("tighten", 0) == 1 else None
    w_goal, w_term = p.get("w_goal", 0.0), p.get("w_term", 0.0)
    goal = np.asarray(p.get("goal", (0.0, 0.0)), dtype=np.float64)
    d_goal_min = np.full(K, np.inf)
    tr = Trace(x=np.empty((T + 1, K, 5)), sxy=np.empty((T + 1, K, 3)),
               gp_mean=np.empty((T, K, 2)), gp_var=np.empty((T, K, 2)),
               d_lane=np.empty((T, K)), lane_margin=np.empty((T, K)),
               obs_margin=np.empty((T, K)), u=u_all, stage=np.empty((T, K)))
    tr.x[0] = x
    tr.sxy[0] = 0.0
    S = np.zeros(K)
    for k in range(T):
        u = u_all[k]
        q = np.concatenate([x[:, 3:5], u], axis=1)
        if terrains:
            m, s2 = G.ensemble_predict(gps, problem.terrain_w, q)
        else:
            m = np.empty((K, 2))
            s2 = np.empty((K, 2))
            for o in range(2):
                m[:, o], _, s2[:, o] = gps[o].predict(q)
        A = D.nominal_jacobian(x, dt, tv, tw)
        x = D.euler_step(x, u, m, dt, tv, tw)
        Sigma = D.covariance_step(Sigma, A, s2, dt)
        sxy = np.stack([Sigma[:, 0, 0], Sigma[:, 0, 1], Sigma[:, 1, 1]], axis=1)
        sxy_c = sxy if tight is None else np.tile(tight[k + 1], (K, 1))
        P = x[:, 0:2]
        d_lane = C.lane_distance(P, problem.path_kind, problem.circle, problem.path_pts)
        r_bar = C.tightened_lane_radius(r, sxy_c, p["p_x"])
        if problem.obstacles.shape[0]:
            obs = C.obstacle_margins(P, sxy_c, problem.obstacles, p["p_x"]).min(axis=1)
        else:
            obs = np.full(K, np.inf)
        lane_exit = (d_lane > r_bar).astype(np.float64)
        collide = (obs <= 0.0).astype(np.float64)
        c = (p["w_var"] * (s2[:, 0] + s2[:, 1])
             + p["w_dev"] * d_lane / r
             + p["w_lane"] * p["discount"] ** k * lane_exit
             + p["w_speed"] * (p["v_des"] - x[:, 3]) ** 2
             + p["w_obs"] * collide)
        d_goal = np.hypot(P[:, 0] - goal[0], P[:, 1] - goal[1])
        d_goal_min = np.minimum(d_goal_min, d_goal)
        c = c + w_goal * d_goal
        S += c
        tr.x[k + 1], tr.sxy[k + 1] = x, sxy
        tr.gp_mean[k], tr.gp_var[k] = m, s2
        tr.d_lane[k], tr.lane_margin[k], tr.obs_margin[k] = d_lane, r_bar - d_lane, obs
        tr.stage[k] = c
    if w_term:
        S += w_term * (d_goal_min > p.get("goal_tol", 0.5))
    return S, tr


def weights(S, lam):
    """w^s = exp(-(S^s - rho)/lambda) / sum_r exp(-(S^r - rho)/lambda), rho = min S."""
    S = np.asarray(S, dtype=np.float64)
    e = np.exp(-(S - S.min()) / lam)
    return e / e.sum()


def update(w, u):
    """U'_k = sum_s w^s u_k^s for u [T, K, 2] -> [T, 2]."""
    return np.einsum("s,tsc->tc", np.asarray(w, dtype=np.float64), u)


def iteration(problem, x0=None, U=None, seed=None, gps=None):
    """One MPPI iteration: returns (U', S, w, trace)."""
    x0 = problem.x0 if x0 is None else x0
    U = problem.U0 if U is None else U
    seed = problem.seed if seed is None else seed
    S, tr = rollout(problem, x0, U, seed, gps=gps)
    w = weights(S, problem.params["lam"])
    return update(w, tr.u), S, w, tr


def shift(U):
    """Warm start: drop the first control, repeat the last one."""
    U = np.asarray(U, dtype=np.float64)
    return np.concatenate([U[1:], U[-1:]], axis=0)


def closed_loop(problem, n_steps: int, x0=None, U=None, record=False):
    """Receding-horizon loop of Alg. 1: optimise, apply U'_0 to the plant, shift."""
    p = problem.params
    x = np.asarray(problem.x0 if x0 is None else x0, dtype=np.float64).copy()
    U = np.asarray(problem.U0 if U is None else U, dtype=np.float64).copy()
    if getattr(problem, "terrain_y", None) is not None:
        gps = G.build_terrains(problem.Z, problem.terrain_y, problem.log_ell, problem.log_sf, problem.log_sn)
    else:
        gps = G.build_pair(problem.Z, problem.y, problem.log_ell, problem.log_sf, problem.log_sn)
    xs, Us = [x.copy()], []
    for t in range(n_steps):
        Unew, S, w, _ = iteration(problem, x, U, problem.seed_at(t), gps=gps)
        x = D.plant_step(x, Unew[0], p["dt"], p["tau_v"], p["tau_w"])[0]
        U = shift(Unew)
        xs.append(x.copy())
        Us.append(Unew)
    return np.array(xs), np.array(Us)


def flip_budget(problem, tr: Trace, delta: float):
    """Per-sample upper bound on how much S may change when indicator decisions
    whose margin lies within `delta` of the threshold flip: sum of the weights
    (times discount) of every such indicator."""
    p = problem.params
    T = tr.lane_margin.shape[0]
    disc = p["discount"] ** np.arange(T)
    near_lane = np.abs(tr.lane_margin) < delta
    near_obs = np.abs(tr.obs_margin) < delta
    return (p["w_lane"] * (near_lane * disc[:, None]).sum(0)
            + p["w_obs"] * near_obs.sum(0))

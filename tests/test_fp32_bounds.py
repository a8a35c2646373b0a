"""The FP32 forward error bounds used by the GPU parity tests, checked on the CPU.

An FP32 evaluation of the covariance recurrence (Eq. 10) and of the tightened
margins (Eqs. 14, 16) from perturbed FP32 states and variances must stay within
the bounds; the same evaluation with a planted mistake (a dropped Jacobian
entry, a dropped variance term, a wrong quantile) must leave them.
"""
import numpy as np
import pytest

from oracle import constraints as C
from oracle import dynamics as D
from oracle import mppi
from paper_2411_03289_amd import workloads as W

import fp32_bounds as FB


def _case(path="eight"):
    pr = W.small_problem(K=48, T=30, M=40, n_obs=8, path=path, seed_data=301, U_scale=1.0)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    rng = np.random.Generator(np.random.PCG64(302))
    x_g = (tr_o.x * (1 + 2e-6 * rng.standard_normal(tr_o.x.shape))).astype(np.float32).astype(np.float64)
    x_g[0] = tr_o.x[0].astype(np.float32)
    var_g = (tr_o.gp_var * (1 + 3e-5 * rng.standard_normal(tr_o.gp_var.shape))).astype(np.float32)
    return pr, tr_o, x_g, var_g.astype(np.float64)


def _fp32_covariances(pr, x_g, var_g, drop=None):
    p = pr.params
    dt = np.float32(p["dt"])
    T, K = var_g.shape[0], var_g.shape[1]
    S = np.zeros((K, 5, 5), np.float32)
    out = np.zeros((T + 1, K, 5, 5))
    for k in range(T):
        A = D.nominal_jacobian(x_g[k], p["dt"], p["tau_v"], p["tau_w"]).astype(np.float32)
        if drop == "jacobian":
            A[:, 0, 2] = 0.0
        S = (A @ S @ np.transpose(A, (0, 2, 1))).astype(np.float32)
        S[:, 3, 3] += dt * dt * var_g[k, :, 0].astype(np.float32)
        if drop != "variance":
            S[:, 4, 4] += dt * dt * var_g[k, :, 1].astype(np.float32)
        out[k + 1] = S
    return out


@pytest.mark.parametrize("path", ["eight", "circle"])
def test_fp32_covariance_within_bound(path):
    pr, tr_o, x_g, var_g = _case(path)
    E, sig = FB.sigma_bound(pr, tr_o.x, tr_o.gp_var, x_g, var_g)
    got = _fp32_covariances(pr, x_g, var_g)
    err = np.abs(got - sig)
    assert np.all(err <= E)
    # the bound is informative: far below the covariance itself
    scale = np.abs(sig).max(axis=(2, 3), keepdims=True)
    assert np.max(E[2:] / np.maximum(scale[2:], 1e-300)) < 1e-3
    # the oracle's covariance is its own trace's position block
    np.testing.assert_array_equal(FB.position_block(sig), tr_o.sxy)


@pytest.mark.parametrize("drop", ["jacobian", "variance"])
def test_fp32_covariance_bound_catches_a_dropped_term(drop):
    pr, tr_o, x_g, var_g = _case()
    E, sig = FB.sigma_bound(pr, tr_o.x, tr_o.gp_var, x_g, var_g)
    got = _fp32_covariances(pr, x_g, var_g, drop=drop)
    assert np.any(np.abs(got - sig) > E)


def _fp32_margins(pr, x_g, sxy_g, p_x=None):
    p = pr.params
    p_x = p["p_x"] if p_x is None else p_x
    P = x_g[1:, :, 0:2].astype(np.float32)
    sxy = sxy_g[1:].astype(np.float32)
    lane, obs = [], []
    for k in range(P.shape[0]):
        d = C.lane_distance(P[k], pr.path_kind, pr.circle, pr.path_pts).astype(np.float32)
        lane.append(C.tightened_lane_radius(np.float32(p["half_width"]), sxy[k], p_x).astype(np.float32) - d)
        obs.append(C.obstacle_margins(P[k], sxy[k], pr.obstacles, p_x).astype(np.float32).min(axis=1))
    return np.array(lane, np.float64), np.array(obs, np.float64)


@pytest.mark.parametrize("path", ["eight", "circle"])
def test_fp32_margins_within_bound(path):
    pr, tr_o, x_g, var_g = _case(path)
    E, sig = FB.sigma_bound(pr, tr_o.x, tr_o.gp_var, x_g, var_g)
    cov = _fp32_covariances(pr, x_g, var_g)
    sxy_g = np.stack([cov[..., 0, 0], cov[..., 0, 1], cov[..., 1, 1]], -1)
    lane, obs = _fp32_margins(pr, x_g, sxy_g)
    exy = FB.position_block(E)[1:]
    bl = FB.lane_margin_bound(pr, tr_o.x, x_g, tr_o.d_lane, tr_o.sxy[1:], exy)
    bo = FB.obstacle_margin_bound(pr, tr_o.x, x_g, tr_o.sxy[1:], exy)
    assert np.all(np.abs(lane - tr_o.lane_margin) <= bl)
    assert np.all(np.abs(obs - tr_o.obs_margin) <= bo)
    # informative: a few micrometres at coordinates of a few metres
    assert bl.max() < 1e-4 and bo.max() < 1e-4


def test_fp32_margin_bounds_catch_a_wrong_quantile():
    pr, tr_o, x_g, var_g = _case()
    E, sig = FB.sigma_bound(pr, tr_o.x, tr_o.gp_var, x_g, var_g)
    cov = _fp32_covariances(pr, x_g, var_g)
    sxy_g = np.stack([cov[..., 0, 0], cov[..., 0, 1], cov[..., 1, 1]], -1)
    lane, obs = _fp32_margins(pr, x_g, sxy_g, p_x=0.9)
    exy = FB.position_block(E)[1:]
    assert np.any(np.abs(lane - tr_o.lane_margin) > FB.lane_margin_bound(pr, tr_o.x, x_g, tr_o.d_lane, tr_o.sxy[1:], exy))
    assert np.any(np.abs(obs - tr_o.obs_margin) > FB.obstacle_margin_bound(pr, tr_o.x, x_g, tr_o.sxy[1:], exy))


def test_no_obstacles_gives_a_zero_bound():
    pr = W.small_problem(K=8, T=5, M=10, n_obs=0, seed_data=303)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    E, _ = FB.sigma_bound(pr, tr_o.x, tr_o.gp_var, tr_o.x, tr_o.gp_var)
    assert np.all(FB.obstacle_margin_bound(pr, tr_o.x, tr_o.x, tr_o.sxy[1:], FB.position_block(E)[1:]) == 0.0)

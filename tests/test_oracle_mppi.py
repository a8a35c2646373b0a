"""Pins for the oracle's rollout, costs, weights and update (Alg. 1; Eqs. 5, 11, 12)."""
import math

import numpy as np
import pytest

from oracle import mppi
from oracle import gp as G
from paper_2411_03289_amd import workloads as W


def test_weights_invariants():
    rng = np.random.Generator(np.random.PCG64(1))
    S = rng.uniform(0, 30, 4096)
    w = mppi.weights(S, 1.0)
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_allclose(mppi.weights(S + 1234.5, 1.0), w, rtol=1e-12)
    np.testing.assert_allclose(mppi.weights(np.full(10, 3.3), 1.0), 0.1, rtol=1e-15)
    w0 = mppi.weights(S, 1e-6)
    assert w0[np.argmin(S)] == 1.0
    tie = np.array([2.0, 1.0, 5.0, 1.0])
    np.testing.assert_allclose(mppi.weights(tie, 1e-9), [0, 0.5, 0, 0.5], atol=1e-300)
    np.testing.assert_allclose(mppi.weights(S, 1e12), 1.0 / S.size, rtol=1e-9)
    # the exponential form: ratios are exp(-(S_i - S_j)/lambda)
    assert w[0] / w[1] == pytest.approx(math.exp(-(S[0] - S[1]) / 1.0), rel=1e-12)


def test_update_is_convex_combination():
    rng = np.random.Generator(np.random.PCG64(2))
    u = rng.uniform(-2, 2, size=(5, 100, 2))
    w = mppi.weights(rng.uniform(0, 3, 100), 0.5)
    U = mppi.update(w, u)
    assert np.all(U <= u.max(axis=1) + 1e-15) and np.all(U >= u.min(axis=1) - 1e-15)
    one = np.zeros(100)
    one[37] = 1.0
    np.testing.assert_array_equal(mppi.update(one, u), u[:, 37])


def _straight_line_problem(T=40):
    # GP data far from every query (zero mean, prior variance), almost no GP
    # variance, no control noise, command equal to the start velocity: the
    # robot drives straight up along X = 5 from the circle track's edge.
    pr = W.small_problem(K=8, T=T, M=10, n_obs=0, seed_data=5)
    pr.Z = pr.Z + 100.0
    pr.log_sf[:] = math.log(1e-7)
    pr.log_sn[:] = math.log(1e-7)
    pr.params.update(sig_v=0.0, sig_w=0.0)
    pr.x0 = np.array([5.0, 0.0, math.pi / 2, 2.0, 0.0])
    pr.U0 = np.tile([2.0, 0.0], (T, 1))
    pr.obstacles = np.array([[5.0, 2.0, 0.33], [-4.0, -4.0, 0.5]])
    return pr


def test_straight_line_scenario_costs_closed_form():
    T = 40
    pr = _straight_line_problem(T)
    p = pr.params
    Unew, S, w, tr = mppi.iteration(pr)
    k = np.arange(T)
    Y = 2.0 * p["dt"] * (k + 1)
    np.testing.assert_allclose(tr.x[1:, 0, 1], Y, atol=1e-12)
    d = np.hypot(5.0, Y) - 5.0
    lane_exit = d > 1.0
    collide = np.abs(Y - 2.0) <= 0.33
    assert lane_exit.sum() == T - 33 and collide.sum() == 7
    var = 2 * (1e-14 + 1e-14)
    stage = (p["w_var"] * var + p["w_dev"] * d / 1.0 + p["w_lane"] * 0.9 ** k * lane_exit
             + p["w_speed"] * (2.0 - 2.0) ** 2 + p["w_obs"] * collide)
    np.testing.assert_allclose(tr.stage[:, 0], stage, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(S, stage.sum(), rtol=1e-12)
    np.testing.assert_allclose(w, 1.0 / pr.K, rtol=1e-12)
    np.testing.assert_allclose(Unew, pr.U0, rtol=1e-15)


def test_speed_and_variance_terms_closed_form():
    T = 25
    pr = _straight_line_problem(T)
    pr.obstacles = np.zeros((0, 3))
    pr.log_sf[:] = math.log(0.4)          # prior variance everywhere: sf^2 + sn^2
    pr.x0 = np.array([5.0, 0.0, math.pi / 2, 0.5, 0.0])
    pr.U0 = np.tile([1.5, 0.0], (T, 1))
    p = pr.params
    _, S, _, tr = mppi.iteration(pr)
    k = np.arange(T)
    v = 1.5 + (0.5 - 1.5) * (1 - p["dt"] / p["tau_v"]) ** (k + 1)
    np.testing.assert_allclose(tr.x[1:, 0, 3], v, rtol=1e-13)
    np.testing.assert_allclose(tr.gp_var[:, 0, :], 0.16 + 1e-14, rtol=1e-12)
    speed = p["w_speed"] * (p["v_des"] - v) ** 2
    assert tr.obs_margin.min() == np.inf
    ref = (p["w_var"] * 2 * (0.16 + 1e-14) + p["w_dev"] * tr.d_lane[:, 0] + speed
           + p["w_lane"] * 0.9 ** k * (tr.lane_margin[:, 0] < 0))
    np.testing.assert_allclose(S[0], ref.sum(), rtol=1e-12)


def test_gp_zeroed_rollout_is_nominal_unicycle():
    # The unicycle-only MPPI baseline: zero GP targets give zero residual mean.
    pr = W.small_problem(K=32, T=15, M=20, seed_data=6, U_scale=1.0)
    pr.y[:] = 0.0
    _, tr = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    p = pr.params
    np.testing.assert_array_equal(tr.gp_mean, 0.0)
    x = np.tile(pr.x0, (pr.K, 1))
    for k in range(pr.T):
        u = tr.u[k]
        x = np.stack([x[:, 0] + p["dt"] * x[:, 3] * np.cos(x[:, 2]),
                      x[:, 1] + p["dt"] * x[:, 3] * np.sin(x[:, 2]),
                      x[:, 2] + p["dt"] * x[:, 4],
                      x[:, 3] + p["dt"] * (u[:, 0] - x[:, 3]) / p["tau_v"],
                      x[:, 4] + p["dt"] * (u[:, 1] - x[:, 4]) / p["tau_w"]], axis=1)
        np.testing.assert_allclose(tr.x[k + 1], x, rtol=1e-13, atol=1e-13)


def test_subset_rollout_equals_full_rows():
    pr = W.small_problem(K=64, T=8, M=16, seed_data=3, U_scale=0.5)
    S, tr = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    ids = np.array([0, 5, 63, 17])
    S2, tr2 = mppi.rollout(pr, pr.x0, pr.U0, pr.seed, sample_ids=ids)
    np.testing.assert_array_equal(S2, S[ids])
    np.testing.assert_array_equal(tr2.x, tr.x[:, ids])


def test_zero_noise_update_returns_clipped_nominal():
    pr = W.small_problem(K=16, T=6, M=12, seed_data=4)
    pr.params.update(sig_v=0.0, sig_w=0.0)
    pr.U0 = np.array([[3.0, 0.1], [-2.5, 1.0], [0.2, 0.3], [1.0, -4.0], [0, 0], [2, 2]])
    Unew, S, w, _ = mppi.iteration(pr)
    np.testing.assert_allclose(Unew, np.clip(pr.U0, -2, 2), rtol=1e-15)
    np.testing.assert_allclose(S, S[0], rtol=1e-15)


def test_small_lambda_selects_best_sample():
    pr = W.small_problem(K=128, T=10, M=16, seed_data=8)
    pr.params["lam"] = 1e-8
    Unew, S, w, tr = mppi.iteration(pr)
    np.testing.assert_allclose(Unew, tr.u[:, np.argmin(S)], rtol=1e-15)


def test_closed_loop_applies_first_control_and_shifts():
    pr = W.small_problem(K=32, T=6, M=12, seed_data=9)
    xs, Us = mppi.closed_loop(pr, 3)
    from oracle import dynamics as D
    p = pr.params
    x = pr.x0.copy()
    U = pr.U0.copy()
    gps = G.build_pair(pr.Z, pr.y, pr.log_ell, pr.log_sf, pr.log_sn)
    for t in range(3):
        Unew, _, _, _ = mppi.iteration(pr, x, U, pr.seed_at(t), gps=gps)
        np.testing.assert_array_equal(Us[t], Unew)
        x = D.plant_step(x, Unew[0], p["dt"], p["tau_v"], p["tau_w"])[0]
        np.testing.assert_array_equal(xs[t + 1], x)
        U = np.concatenate([Unew[1:], Unew[-1:]])


def test_flip_budget_counts_near_threshold_indicators():
    pr = _straight_line_problem(40)
    _, _, _, tr = mppi.iteration(pr)
    # exactly-on-threshold decisions never occur here; a wide band catches them all
    assert np.all(mppi.flip_budget(pr, tr, 1e-9) == 0.0)
    wide = mppi.flip_budget(pr, tr, 10.0)
    assert wide[0] == pytest.approx(np.sum(0.9 ** np.arange(40)) + 40.0, rel=1e-12)


def test_goal_terms_closed_form():
    T = 30
    pr = _straight_line_problem(T)
    pr.obstacles = np.zeros((0, 3))
    pr.params.update(w_goal=0.2, w_term=1.5, goal=(5.0, 2.0), goal_tol=0.3)
    p0 = _straight_line_problem(T)
    p0.obstacles = np.zeros((0, 3))
    base = mppi.rollout(p0, p0.x0, p0.U0, p0.seed)[0]
    S, tr = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    Y = 2.0 * pr.params["dt"] * (np.arange(T) + 1)
    dg = np.abs(Y - 2.0)
    assert dg.min() < 0.3   # the straight line passes the goal: no terminal cost
    np.testing.assert_allclose(S - base, 0.2 * dg.sum(), rtol=1e-12)
    pr.params["goal"] = (8.0, 2.0)   # 3 m off the line: never reached
    S2, _ = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    dg2 = np.hypot(3.0, Y - 2.0)
    np.testing.assert_allclose(S2 - base, 0.2 * dg2.sum() + 1.5, rtol=1e-12)


def test_step2_tightening_matches_monte_carlo_along_the_nominal_controls():
    # Alg. 1 Step 2 propagates Sigma_XY (Eq. 10) along the nominal controls clip(U).  With the GP's
    # training points far from every query its mean is exactly 0 and its variance the closed form
    # sf^2 + sn^2, so the stochastic model is the Euler step driven by clip(U) with that velocity
    # noise; with small noise the spread of many such rollouts approaches the propagated
    # covariance.  Nothing here comes from the oracle's rollout.
    from oracle import dynamics as D
    # the turn-rate noise dominates, so the spread also runs through the heading (the Jacobian's
    # coupling of position to heading), not only through the speed
    pr = W.small_problem(K=40, T=20, M=20, n_obs=0, path="eight", seed_data=17, U_scale=1.0)
    pr.Z = pr.Z + 1.0e3
    pr.y = np.zeros_like(pr.y)
    pr.log_sf = np.log([1.0e-4, 6.0e-3])
    pr.log_sn = np.log([5.0e-5, 1.0e-3])
    s2 = np.exp(2 * pr.log_sf) + np.exp(2 * pr.log_sn)
    nom = mppi.nominal_tightening(pr, pr.x0, pr.U0)
    p = pr.params
    u = np.clip(pr.U0, p["u_min"], p["u_max"])
    rng = np.random.Generator(np.random.PCG64(21))
    n = 200_000
    x = np.tile(np.asarray(pr.x0, float), (n, 1))
    for k in range(pr.T):
        m = rng.normal(0.0, np.sqrt(s2), size=(n, 2))
        x = D.euler_step(x, np.tile(u[k], (n, 1)), m, p["dt"], p["tau_v"], p["tau_w"])
        if k == 0:   # the position of step 1 follows the noise-free initial velocity
            np.testing.assert_array_equal(nom[1], 0.0)
            assert np.ptp(x[:, :2], axis=0).max() == 0.0
            continue
        C = np.cov(x[:, :2].T)
        sx, sy = np.sqrt(nom[k + 1, 0]), np.sqrt(nom[k + 1, 2])
        got = np.array([C[0, 0] / sx**2, C[0, 1] / (sx * sy), C[1, 1] / sy**2])
        want = np.array([1.0, nom[k + 1, 1] / (sx * sy), 1.0])
        np.testing.assert_allclose(got, want, atol=0.02, err_msg=f"step {k + 1}")


def test_step2_tightening_uses_the_nominal_covariance():
    pr = W.small_problem(K=40, T=10, M=20, n_obs=6, path="eight", seed_data=17, U_scale=1.0)
    pr.params["tighten"] = 1
    S, tr = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    nom = mppi.nominal_tightening(pr, pr.x0, pr.U0)
    # the nominal covariance equals a zero-noise single-sample rollout's
    q = W.small_problem(K=40, T=10, M=20, n_obs=6, path="eight", seed_data=17, U_scale=1.0)
    q.params.update(sig_v=0.0, sig_w=0.0)
    _, trq = mppi.rollout(q, q.x0, q.U0, 0, sample_ids=np.array([3]))
    np.testing.assert_array_equal(nom, trq.sxy[:, 0])
    from oracle import constraints as C
    rbar = C.tightened_lane_radius(pr.params["half_width"], nom[1:], pr.params["p_x"])
    np.testing.assert_allclose(tr.lane_margin, rbar[:, None] - tr.d_lane, rtol=1e-13, atol=1e-13)
    # with no noise every sample is the nominal: both modes agree
    q.params["tighten"] = 1
    Sa, _ = mppi.rollout(q, q.x0, q.U0, 0)
    q.params["tighten"] = 0
    Sb, _ = mppi.rollout(q, q.x0, q.U0, 0)
    np.testing.assert_allclose(Sa, Sb, rtol=1e-13)

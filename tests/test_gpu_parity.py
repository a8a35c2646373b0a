"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (FP32 form), with floors s_q = 1 for positions, heading,
velocities, costs and controls:
  states, costs, U        |g - o| <= 1e-5 max(|o|, s_q)
  cost of a sample whose indicator margin comes within 1e-4 m of its
  threshold                 additionally the weights of those indicators
  U                       additionally the first-order effect of the cost
                          tolerance on the weights, (2 tol_S / lambda) sum_s w_s |u_s - U|
  GP mean                 1e-5 + 8 eps32 sum_j |k_j alpha_j|   (FP32 dot product)
  GP variance             2e-6 + 1e-5 s2                     (FP32 W-form, see DESIGN)
"""
import numpy as np
import pytest

from oracle import gp as G
from oracle import mppi
from oracle import philox as OP
from paper_2411_03289_amd import gpmppi as B
from paper_2411_03289_amd import workloads as W

from gpu_util import dev, gpu_rollout, gpu_step, rel_err, torch

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24
TOL = 1e-5
FLIP_BAND = 1e-4


def _print(name, **vals):
    print(name, " ".join(f"{k}={v:.3e}" for k, v in vals.items()), flush=True)


# ------------------------------------------------------------------ noise
def test_philox_bit_exact():
    t = torch()
    rng = np.random.Generator(np.random.PCG64(5))
    ctr = rng.integers(0, 2**32, size=(4099, 4), dtype=np.uint64)
    ctr[:10] = [[k, s, 3, 0] for k, s in zip(range(10), range(100, 110))]
    seed = (2002 << 32) + 77
    c = t.as_tensor(ctr.astype(np.uint32).view(np.int32), device="cuda")
    out = t.empty_like(c)
    B.gpmppi_philox(seed, c, out)
    t.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, OP.philox4x32_10(ctr, OP.seed_key(seed)))


# ------------------------------------------------------------------ GP
def _gp_case(M, seed=3):
    pr = W.small_problem(K=64, T=4, M=M, seed_data=seed, n_data=max(M, 50))
    q = np.concatenate([W.random_queries(700, seed + 1, -2.5, 2.5),
                        pr.Z[0][: min(M, 100)] + 1e-3, pr.Z[1][: min(M, 100)],
                        W.random_queries(33, seed + 2, 6.0, 9.0)])
    return pr, q


def _gpu_predict(pr, q, precision):
    t = torch()
    ctx = B.gpmppi_init(pr, precision)
    qd = dev(q)
    mean = t.empty(2 * len(q), device="cuda")
    var = t.empty(2 * len(q), device="cuda")
    B.gpmppi_gp_predict(ctx, qd, mean, var)
    t.cuda.synchronize()
    return mean.cpu().numpy().reshape(2, -1).astype(np.float64), var.cpu().numpy().reshape(2, -1).astype(np.float64)


@pytest.mark.parametrize("M", [1, 50, 77, 256, 1024])
def test_gp_predict_fp32(M):
    pr, q = _gp_case(M)
    gm, gv = _gpu_predict(pr, q, B.FP32)
    for o, g in enumerate(G.build_pair(pr.Z, pr.y, pr.log_ell, pr.log_sf, pr.log_sn)):
        m, _, v = g.predict(q)
        absdot = np.abs(G.se_ard(q, g.Z, g.log_ell, g.log_sf)) @ np.abs(g.alpha)
        em, ev = np.abs(gm[o] - m), np.abs(gv[o] - v)
        _print(f"gp M={M} o={o}", mean_err=em.max(), var_err=ev.max(), var_min=v.min())
        assert np.all(em <= 1e-5 + 8 * EPS32 * absdot)
        assert np.all(ev <= 2e-6 + 1e-5 * v)
        assert np.all(gv[o] >= g.sn2 * (1 - 1e-6))


def test_gp_predict_bf16_forms():
    pr, q = _gp_case(1024)
    m32, v32 = _gpu_predict(pr, q, B.FP32)
    gps = G.build_pair(pr.Z, pr.y, pr.log_ell, pr.log_sf, pr.log_sn)
    for prec, vtol in ((B.BF16X3, 2e-5), (B.BF16, 2e-2)):
        gm, gv = _gpu_predict(pr, q, prec)
        for o, g in enumerate(gps):
            m, _, v = g.predict(q)
            # the mean is FP32 in every form (only its summation order may differ)
            absdot = np.abs(G.se_ard(q, g.Z, g.log_ell, g.log_sf)) @ np.abs(g.alpha)
            assert np.all(np.abs(gm[o] - m) <= 1e-5 + 8 * EPS32 * absdot)
            _print(f"gp bf16 form={prec} o={o}", var_err=np.abs(gv[o] - v).max())
            assert np.abs(gv[o] - v).max() <= vtol
            assert np.all(gv[o] >= g.sn2 * (1 - 1e-6))


@pytest.mark.parametrize("M", [1, 50, 77, 300, 520])
def test_gp_predict_bf16_forms_ragged(M):
    """The BF16 forms' kernel vectors (exponents on the matrix cores from three-term BF16 splits)
    at sizes whose column tiles do not divide evenly between the waves: the mean keeps the FP32
    bound, the variance the form's."""
    pr, q = _gp_case(M, seed=5)
    gps = G.build_pair(pr.Z, pr.y, pr.log_ell, pr.log_sf, pr.log_sn)
    for prec, vtol in ((B.BF16X3, 2e-5), (B.BF16, 2e-2)):
        gm, gv = _gpu_predict(pr, q, prec)
        for o, g in enumerate(gps):
            m, _, v = g.predict(q)
            absdot = np.abs(G.se_ard(q, g.Z, g.log_ell, g.log_sf)) @ np.abs(g.alpha)
            em = np.abs(gm[o] - m)
            _print(f"gp M={M} form={prec} o={o}", mean_err=em.max(), var_err=np.abs(gv[o] - v).max())
            assert np.all(em <= 1e-5 + 8 * EPS32 * absdot)
            assert np.abs(gv[o] - v).max() <= vtol
            assert np.all(gv[o] >= g.sn2 * (1 - 1e-6))


def _bf16_bounds(pr, tr_o):
    """FP32 dot-product bound of each step's GP mean: sum_j |k_j alpha_j| at the oracle's inputs."""
    q = np.concatenate([tr_o.x[:-1, :, 3:5], tr_o.u], axis=2).reshape(-1, 4)
    absdot = np.stack([np.abs(G.se_ard(q, g.Z, g.log_ell, g.log_sf)) @ np.abs(g.alpha)
                       for g in G.build_pair(pr.Z, pr.y, pr.log_ell, pr.log_sf, pr.log_sn)], axis=1)
    return absdot.reshape(pr.T, pr.K, 2)


def _check_bf16_rollout(prec, S_g, tr_g, tr_o, absdot, label):
    """The state trajectory depends on the GP mean only, which stays FP32 in the BF16 forms, so
    states, controls and means follow the oracle at the FP32 bar; the variance meets the form's."""
    vtol = 5e-5 if prec == B.BF16X3 else 2e-2
    ex = rel_err(tr_g["x"], tr_o.x, 1.0)
    em = np.abs(tr_g["gp_mean"] - tr_o.gp_mean)
    ev = np.abs(tr_g["gp_var"] - tr_o.gp_var)
    _print(label, x=ex.max(), gp_mean=em.max(), gp_var=ev.max())
    assert np.all(ex <= TOL), "states"
    assert np.all(np.abs(tr_g["u"] - tr_o.u) <= 1e-5), "sampled controls"
    assert np.all(em <= 1e-5 + 8 * EPS32 * absdot), "gp mean"
    assert ev.max() <= vtol, "gp variance"
    assert np.all(np.isfinite(S_g))


@pytest.mark.parametrize("prec", [B.BF16, B.BF16X3])
def test_bf16_rollout_states_at_every_shape(prec):
    """BF16-form rollouts at M = 300 (ten column tiles over four or eight waves) for every launch
    shape."""
    pr = W.small_problem(K=150, T=10, M=300, n_obs=7, path="eight", seed_data=26, U_scale=1.0)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    absdot = _bf16_bounds(pr, tr_o)
    ctx = B.gpmppi_init(pr, prec)
    for groups in (1, 2):
        for waves in (4, 8):
            B.gpmppi_set_tuning(ctx, groups, 1, waves)
            S_g, tr_g = gpu_rollout(pr, ctx=ctx)
            _check_bf16_rollout(prec, S_g, tr_g, tr_o, absdot, f"form={prec} groups={groups} waves={waves}")


@pytest.mark.parametrize("prec", [B.BF16, B.BF16X3])
@pytest.mark.parametrize("seed", range(3))
def test_random_instances_bf16_forms_at_every_shape(prec, seed):
    # fixed-seed instances of uneven K, T, M (up to 1024: both walks, and two sample groups where
    # the form's k operands fit), obstacle count and track
    rng = np.random.Generator(np.random.PCG64(9700 + seed))
    K, T, M = int(rng.integers(1, 300)), int(rng.integers(1, 12)), int(rng.integers(1, 1025))
    n_obs, path = int(rng.integers(0, 9)), ("eight" if rng.integers(0, 2) else "circle")
    pr = W.small_problem(K=K, T=T, M=M, n_obs=n_obs, path=path, seed_data=200 + seed,
                         U_scale=float(rng.uniform(0.0, 1.5)), n_data=max(M, 50))
    print(f"instance {seed}: K={K} T={T} M={M} n_obs={n_obs} path={path}", flush=True)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    absdot = _bf16_bounds(pr, tr_o)
    ctx = B.gpmppi_init(pr, prec)
    n_shapes = 0
    for groups in (1, 2):
        for rotate in (0, 1):
            for waves in (4, 8):
                try:
                    B.gpmppi_set_tuning(ctx, groups, rotate, waves)
                except B.GpmppiError:
                    assert groups == 2
                    continue
                S_g, tr_g = gpu_rollout(pr, ctx=ctx)
                _check_bf16_rollout(prec, S_g, tr_g, tr_o, absdot,
                                    f"form={prec} instance {seed} groups={groups} rotate={rotate} waves={waves}")
                n_shapes += 1
    assert n_shapes >= 4


def test_not_positive_definite_is_reported():
    pr = W.small_problem(M=8, seed_data=1)
    pr.Z[0, 1] = pr.Z[0, 0]
    pr.log_sn[:] = -30.0
    with pytest.raises(B.GpmppiError) as e:
        B.gpmppi_init(pr, B.FP32)
    assert e.value.status == -2


# ------------------------------------------------------------------ rollout parity
def _check_rollout(pr, S_g, tr_g, S_o, tr_o, label):
    T, K = pr.T, pr.K
    ex = rel_err(tr_g["x"], tr_o.x, 1.0)
    eu = np.abs(tr_g["u"] - tr_o.u)
    em = np.abs(tr_g["gp_mean"] - tr_o.gp_mean)
    ev = np.abs(tr_g["gp_var"] - tr_o.gp_var)
    pos = np.maximum(np.abs(tr_o.x[1:, :, 0]), np.abs(tr_o.x[1:, :, 1]))
    edl = np.abs(tr_g["d_lane"] - tr_o.d_lane) / np.maximum(pos, 1.0)
    esxy = np.abs(tr_g["sxy"] - tr_o.sxy) / np.maximum(np.abs(tr_o.sxy), 1e-6)
    flip = mppi.flip_budget(pr, tr_o, FLIP_BAND)
    eS = np.abs(S_g - S_o) - flip
    _print(label, x=ex.max(), u=eu.max(), gp_mean=em.max(), gp_var=ev.max(), d_lane=edl.max(),
           sxy_rel=esxy.max(), cost=(eS / np.maximum(S_o, 1)).max(), flagged=float((flip > 0).sum()))
    assert np.all(ex <= TOL), "states"
    assert np.all(eu <= 1e-5), "sampled controls"
    assert np.all(ev <= 2e-6 + 1e-5 * tr_o.gp_var), "gp variance"
    assert np.all(edl <= 2 * TOL), "lane distance"
    assert np.all(esxy <= 1e-3), "position covariance"
    lm_ok = np.abs(tr_g["lane_margin"] - tr_o.lane_margin) <= 2 * TOL * np.maximum(pos, 1.0) + 1e-4
    assert np.all(lm_ok), "lane margin"
    fin = np.isfinite(tr_o.obs_margin)
    assert np.array_equal(np.isfinite(tr_g["obs_margin"]), fin)
    om_ok = np.abs(tr_g["obs_margin"][fin] - tr_o.obs_margin[fin]) <= 2 * TOL * np.maximum(pos[fin], 1.0) + 1e-4
    assert np.all(om_ok), "obstacle margin"
    assert np.all(eS <= TOL * np.maximum(S_o, 1.0)), "costs"


@pytest.mark.parametrize("case", ["c0", "ragged_eight", "tiny", "no_obstacles", "one_point_gp", "zero_noise"])
def test_rollout_trace_matches_oracle(case):
    if case == "c0":
        pr = W.make_config(0)
    elif case == "ragged_eight":
        pr = W.small_problem(K=77, T=13, M=45, n_obs=9, path="eight", seed_data=21, U_scale=1.0)
    elif case == "tiny":
        pr = W.small_problem(K=1, T=1, M=5, n_obs=2, seed_data=22)
    elif case == "no_obstacles":
        pr = W.small_problem(K=40, T=25, M=64, n_obs=0, seed_data=23, U_scale=1.5)
    elif case == "one_point_gp":
        pr = W.small_problem(K=33, T=9, M=1, n_obs=3, path="eight", seed_data=24)
    else:
        pr = W.small_problem(K=50, T=12, M=30, n_obs=5, seed_data=25, U_scale=1.0)
        pr.params.update(sig_v=0.0, sig_w=0.0)
    S_g, tr_g = gpu_rollout(pr)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    _check_rollout(pr, S_g, tr_g, S_o, tr_o, f"rollout {case}")


def _u_tolerance(pr, S_o, w_o, u_o, U_o, flip):
    lam = pr.params["lam"]
    tolS = TOL * np.maximum(S_o, 1.0)
    spread = np.einsum("s,tsc->tc", w_o, np.abs(u_o - U_o[:, None, :]))
    infl = np.einsum("s,tsc->tc", w_o * (np.expm1(np.minimum(flip / lam, 50.0))), np.abs(u_o - U_o[:, None, :]))
    return TOL * np.maximum(np.abs(U_o), 1.0) + 2 * tolS.max() / lam * spread + 2 * infl


@pytest.mark.parametrize("cfg", ["c0", "small_eight"])
def test_step_matches_oracle(cfg):
    pr = W.make_config(0) if cfg == "c0" else W.small_problem(K=300, T=15, M=70, n_obs=8, path="eight",
                                                              seed_data=31, U_scale=1.0)
    U_g, S_g, w_g = gpu_step(pr)
    U_o, S_o, w_o, tr_o = mppi.iteration(pr)
    flip = mppi.flip_budget(pr, tr_o, FLIP_BAND)
    tolU = _u_tolerance(pr, S_o, w_o, tr_o.u, U_o, flip)
    _print(f"step {cfg}", U=np.abs(U_g - U_o).max(), tolU=tolU.min(), w=np.abs(w_g - w_o).max())
    assert np.all(np.abs(S_g - S_o) <= TOL * np.maximum(S_o, 1) + flip)
    assert np.all(np.abs(U_g - U_o) <= tolU)
    assert abs(w_g.sum() - 1.0) < 1e-5
    assert np.all(np.abs(w_g - w_o) <= 1e-4 * np.maximum(w_o, 1e-3 / pr.K) + 2 * w_o * np.expm1(flip))


def test_weights_update_alone():
    t = torch()
    pr = W.small_problem(K=5000, T=7, M=8, seed_data=41, U_scale=1.0)
    S = W.random_costs(pr.K, 42, spread=6.0)
    ctx = B.gpmppi_init(pr, B.FP32)
    U = dev(pr.U0)
    U_out = t.empty_like(U)
    w = t.empty(pr.K, device="cuda")
    B.gpmppi_weights_update(ctx, dev(S), U, pr.seed, U_out, w)
    t.cuda.synchronize()
    S32 = S.astype(np.float32).astype(np.float64)   # the device sees FP32 costs
    w_o = mppi.weights(S32, pr.params["lam"])
    from oracle.philox import sampled_controls
    p = pr.params
    u_o = sampled_controls(pr.U0, np.arange(pr.K), pr.seed, (p["sig_v"], p["sig_w"]), p["u_min"], p["u_max"])
    U_o = mppi.update(w_o, u_o)
    np.testing.assert_allclose(w.cpu().numpy(), w_o, rtol=2e-5, atol=1e-10)
    np.testing.assert_allclose(U_out.cpu().numpy(), U_o, atol=1e-5)


def test_c1_single_iteration():
    pr = W.make_config(1)
    U_g, S_g, w_g = gpu_step(pr)
    U_o, S_o, w_o, tr_o = mppi.iteration(pr)
    flip = mppi.flip_budget(pr, tr_o, FLIP_BAND)
    tolU = _u_tolerance(pr, S_o, w_o, tr_o.u, U_o, flip)
    _print("step c1", U=np.abs(U_g - U_o).max(), cost=(np.abs(S_g - S_o) / np.maximum(S_o, 1)).max())
    assert np.all(np.abs(S_g - S_o) <= TOL * np.maximum(S_o, 1) + flip)
    assert np.all(np.abs(U_g - U_o) <= tolU)


def test_c2_full_size_sampled_and_golden():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c2_oracle.npz")
    pr = W.make_config(2)
    S_g, tr_g = gpu_rollout(pr)
    ids = np.unique(np.concatenate([np.arange(0, pr.K, 257), [pr.K - 1, pr.K - 32, 31, 32]]))
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed, sample_ids=ids)
    sub = {k: (v[:, ids] if v.ndim >= 2 else v) for k, v in tr_g.items()}
    prs = W.make_config(2, K=len(ids))
    _check_rollout(prs, S_g[ids], sub, S_o, tr_o, "c2 sampled")
    if os.path.exists(path):
        g = np.load(path)
        U_g, S_full, _ = gpu_step(pr)
        np.testing.assert_array_equal(S_full, S_g)   # step and rollout agree bitwise
        assert np.all(np.abs(S_g - g["S"]) <= TOL * np.maximum(g["S"], 1) + g["flip"])
        tolS = TOL * np.maximum(g["S"], 1.0).max()
        # sample controls for the U bound come from the oracle's noise
        from oracle.philox import sampled_controls
        p = pr.params
        u_o = sampled_controls(pr.U0, np.arange(pr.K), pr.seed, (p["sig_v"], p["sig_w"]), p["u_min"], p["u_max"])
        tolU = _u_tolerance(pr, g["S"], g["w"], u_o, g["U"], g["flip"])
        _print("c2 full", U=np.abs(U_g - g["U"]).max(), tolU=tolU.min(), tolS=tolS)
        assert np.all(np.abs(U_g - g["U"]) <= tolU)


def test_determinism_and_aliasing():
    t = torch()
    pr = W.small_problem(K=200, T=10, M=40, seed_data=51, U_scale=1.0)
    ctx = B.gpmppi_init(pr, B.FP32)
    a = gpu_step(pr, ctx=ctx)
    b = gpu_step(pr, ctx=ctx)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    U = dev(pr.U0)
    costs = t.empty(pr.K, device="cuda")
    B.gpmppi_step(ctx, dev(pr.x0), U, pr.seed, U, costs, None)   # U_out aliases U
    t.cuda.synchronize()
    np.testing.assert_array_equal(U.cpu().numpy().astype(np.float64), a[0])


def test_nonfinite_cost_sets_status_flag():
    t = torch()
    pr = W.small_problem(K=64, T=3, M=8, seed_data=61)
    ctx = B.gpmppi_init(pr, B.FP32)
    assert B.gpmppi_status_flags(ctx) == 0
    S = W.random_costs(pr.K, 3)
    S[17] = np.nan
    U = dev(pr.U0)
    B.gpmppi_weights_update(ctx, dev(S), U, pr.seed, t.empty_like(U))
    assert B.gpmppi_status_flags(ctx) & 1
    assert B.gpmppi_status_flags(ctx) == 0


# ------------------------------------------------------------------ closed loop
def test_closed_loop_resynced_steps_and_graph_replay():
    t = torch()
    pr = W.make_config(1, K=512, T=20, M=64, n_obs=10)
    p = pr.params
    from oracle import dynamics as D
    gps = G.build_pair(pr.Z, pr.y, pr.log_ell, pr.log_sf, pr.log_sn)
    ctx = B.gpmppi_init(pr, B.FP32)
    x, U = pr.x0.copy(), pr.U0.copy()
    for step in range(4):
        U_o, S_o, w_o, tr_o = mppi.iteration(pr, x, U, pr.seed_at(step), gps=gps)
        U_g, S_g, _ = gpu_step(pr, x0=x, U=U, seed=pr.seed_at(step), ctx=ctx)
        flip = mppi.flip_budget(pr, tr_o, FLIP_BAND)
        assert np.all(np.abs(U_g - U_o) <= _u_tolerance(pr, S_o, w_o, tr_o.u, U_o, flip))
        # plant + shift on the device from the oracle's U'
        xd, Ud = dev(x), dev(U_o)
        B.gpmppi_plant_shift(ctx, xd, xd, Ud, 0.3)
        t.cuda.synchronize()
        x_o = D.plant_step(x, U_o[0], p["dt"], p["tau_v"], p["tau_w"])[0]
        np.testing.assert_allclose(xd.cpu().numpy(), x_o, rtol=1e-6, atol=1e-6)
        np.testing.assert_array_equal(Ud.cpu().numpy(), mppi.shift(U_o).astype(np.float32))
        x, U = x_o, mppi.shift(U_o)
    # whole loop on device: eager launches vs one captured graph replayed
    res = []
    for use_graph in (False, True):
        xd, Ud = dev(pr.x0), dev(pr.U0)
        xh = t.empty(6 * 5, device="cuda")
        uh = t.empty(5 * 2, device="cuda")
        B.gpmppi_closed_loop(ctx, xd, Ud, pr.seed, 5, 0.3, xh, uh, use_graph=use_graph)
        t.cuda.synchronize()
        res.append((xh.cpu().numpy(), uh.cpu().numpy(), Ud.cpu().numpy()))
    for a, b in zip(*res):
        np.testing.assert_array_equal(a, b)
    # the device loop equals step-by-step calls
    xd, Ud = dev(pr.x0), dev(pr.U0)
    costs = t.empty(pr.K, device="cuda")
    for step in range(5):
        B.gpmppi_step(ctx, xd, Ud, pr.seed_at(step), Ud, costs, None)
        B.gpmppi_plant_shift(ctx, xd, xd, Ud, 0.3)
    t.cuda.synchronize()
    np.testing.assert_array_equal(xd.cpu().numpy(), res[0][0][-5:])


# ------------------------------------------------------------------ terrain ensemble (Eq. 3)
def test_terrain_ensemble_rollout_matches_oracle():
    pr = W.add_terrains(W.small_problem(K=96, T=12, M=60, n_obs=6, path="eight", seed_data=81, U_scale=1.0),
                        seed=82, weights=(0.6, 0.25, 0.15))
    S_g, tr_g = gpu_rollout(pr)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    _check_rollout(pr, S_g, tr_g, S_o, tr_o, "rollout terrains")


def test_terrain_weights_select_a_terrain():
    pr = W.add_terrains(W.small_problem(K=64, T=8, M=48, seed_data=83, U_scale=1.0), seed=84)
    ctx = B.gpmppi_init(pr, B.FP32)
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        B.gpmppi_set_terrain_weights(ctx, e)
        single = W.small_problem(K=64, T=8, M=48, seed_data=83, U_scale=1.0)
        single.y = pr.terrain_y[i].copy()
        a = gpu_step(pr, ctx=ctx)
        b = gpu_step(single)
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x, y)


# ------------------------------------------------------------------ goal terms (Eq. 12) and Step 2 tightening
@pytest.mark.parametrize("mode", ["goal_reached", "goal_missed", "step2"])
def test_goal_terms_and_step2_tightening(mode):
    pr = W.small_problem(K=80, T=14, M=50, n_obs=7, path="eight", seed_data=91, U_scale=1.0)
    if mode == "step2":
        pr.params["tighten"] = 1
    else:
        pr.params.update(W.task_params("avoid", goal=(0.3, 0.2) if mode == "goal_reached" else (6.0, -6.0)))
    S_g, tr_g = gpu_rollout(pr)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    _check_rollout(pr, S_g, tr_g, S_o, tr_o, f"rollout {mode}")
    U_g, S2, _ = gpu_step(pr)
    np.testing.assert_array_equal(S2, S_g)


def test_terrain_means_feed_the_weight_estimate():
    t = torch()
    pr = W.add_terrains(W.small_problem(K=64, T=8, M=70, seed_data=85), seed=86)
    ctx = B.gpmppi_init(pr, B.FP32)
    q = W.random_queries(40, 87)
    out = t.empty(40 * 3 * 2, device="cuda")
    B.gpmppi_terrain_means(ctx, dev(q), out)
    t.cuda.synchronize()
    F = out.cpu().numpy().reshape(40, 3, 2).astype(np.float64)
    tg = G.build_terrains(pr.Z, pr.terrain_y, pr.log_ell, pr.log_sf, pr.log_sn)
    for i in range(3):
        for o in range(2):
            m, _, _ = tg[i][o].predict(q)
            absdot = np.abs(G.se_ard(q, tg[i][o].Z, tg[i][o].log_ell, tg[i][o].log_sf)) @ np.abs(tg[i][o].alpha)
            assert np.all(np.abs(F[:, i, o] - m) <= 1e-5 + 8 * EPS32 * absdot)
    # measurements generated by terrain 2: the estimate (Eq. 4) recovers it
    from oracle import terrain as TR
    Yv, Yw = F[:, 2, 0].copy(), F[:, 2, 1].copy()
    w = B.gpmppi_terrain_weights(Yv, Yw, F[:, :, 0], F[:, :, 1], np.full(3, 1 / 3), 0.0)
    np.testing.assert_allclose(w, [0, 0, 1], atol=1e-6)
    np.testing.assert_allclose(w, TR.solve_weights(Yv, Yw, F[:, :, 0], F[:, :, 1], np.full(3, 1 / 3), 0.0),
                               atol=1e-6)


@pytest.mark.parametrize("seed", range(6))
def test_random_instances_at_every_shape_match_oracle(seed):
    # fixed-seed instances of uneven K, T, M, obstacle count, track and nominal controls, at every
    # admissible launch shape: both walks over W (row-tile pairs, single row tiles) across many
    # row-tile counts, ragged sample blocks, and the geometry loops inside the contraction
    rng = np.random.Generator(np.random.PCG64(9000 + seed))
    K, T, M = int(rng.integers(1, 400)), int(rng.integers(1, 14)), int(rng.integers(1, 700))
    n_obs, path = int(rng.integers(0, 9)), ("eight" if rng.integers(0, 2) else "circle")
    pr = W.small_problem(K=K, T=T, M=M, n_obs=n_obs, path=path, seed_data=100 + seed,
                         U_scale=float(rng.uniform(0.0, 1.5)), n_data=max(M, 50))
    print(f"instance {seed}: K={K} T={T} M={M} n_obs={n_obs} path={path}", flush=True)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    ctx = B.gpmppi_init(pr, B.FP32)
    n_shapes = 0
    for groups in (1, 2):
        for rotate in (0, 1):
            for waves in (4, 8):
                try:
                    B.gpmppi_set_tuning(ctx, groups, rotate, waves)
                except B.GpmppiError:
                    assert groups == 2   # two sample groups need both k operands in LDS
                    continue
                S_g, tr_g = gpu_rollout(pr, ctx=ctx)
                _check_rollout(pr, S_g, tr_g, S_o, tr_o, f"instance {seed} groups={groups} rotate={rotate} waves={waves}")
                n_shapes += 1
    assert n_shapes >= 4


def test_every_tuned_shape_matches_oracle_and_the_tuner_installs_its_choice():
    t = torch()
    # M = 300: 10 row tiles, walked as single row tiles (5 pairs cannot be spread evenly over 4 or 8
    # waves), several per wave, so that the walk's start rotation matters
    pr = W.make_config(0, K=300, T=12, M=300, N=300)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    ctx = B.gpmppi_init(pr, B.FP32)
    for groups in (1, 2):
        for rotate in (0, 1):
            for waves in (4, 8):
                B.gpmppi_set_tuning(ctx, groups, rotate, waves)
                got = B.gpmppi_get_tuning(ctx)
                assert (got["groups"], got["rotate"], got["waves"]) == (groups, rotate, waves)
                S_g, tr_g = gpu_rollout(pr, ctx=ctx)
                _check_rollout(pr, S_g, tr_g, S_o, tr_o, f"shape groups={groups} rotate={rotate} waves={waves}")
                S_g2, _ = gpu_rollout(pr, ctx=ctx)
                np.testing.assert_array_equal(S_g, S_g2)
    chosen = B.gpmppi_tune(ctx, dev(pr.x0), dev(pr.U0), pr.seed, reps=2)
    print("tuning", chosen, flush=True)
    got = B.gpmppi_get_tuning(ctx)
    assert (got["groups"], got["rotate"], got["waves"]) == (chosen["groups"], chosen["rotate"], chosen["waves"])
    assert chosen["ms"] > 0
    for bad in ((0, 1, 4), (3, 0, 4), (1, 5, 4), (1, 1, 6)):
        with pytest.raises(B.GpmppiError):
            B.gpmppi_set_tuning(ctx, *bad)

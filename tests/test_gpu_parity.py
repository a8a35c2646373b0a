"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars (FP32 form), with floors s_q = 1 for positions, heading, velocities,
costs and controls:
  states, costs, U        |g - o| <= 1e-5 max(|o|, s_q)
  cost of a sample whose indicator margin comes within 1e-4 m of its
  threshold                 additionally the weights of those indicators
  U                       against sum_s w_s(S_gpu) u_s, the oracle's weights
                          recomputed from the GPU's own costs (the indicator
                          decisions are then the same on both sides), and
                          against the oracle's U where no sample has a margin
                          within 1e-4 m of its threshold
  GP mean                 1e-5 + 8 eps32 sum_j |k_j alpha_j|   (FP32 dot product)
  GP variance             2e-6 + 1e-5 s2                     (FP32 W-form)
  Sigma_XY, margins       the FP32 forward error bounds of Eq. (10)'s recurrence
                          and of Eqs. (13)-(16) given the measured state and
                          variance differences (tests/fp32_bounds.py)
"""
import dataclasses

import numpy as np
import pytest

from oracle import gp as G
from oracle import mppi
from oracle import philox as OP
from paper_2411_03289_amd import gpmppi as B
from paper_2411_03289_amd import workloads as W

import fp32_bounds as FB
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
    """FP32 dot-product bound of each step's GP mean: sum_j |k_j alpha_j| at the oracle's inputs
    (with a terrain ensemble, alpha = sum_i w_i alpha_i, Eq. 3)."""
    q = np.concatenate([tr_o.x[:-1, :, 3:5], tr_o.u], axis=2).reshape(-1, 4)
    if getattr(pr, "terrain_y", None) is not None:
        tg = G.build_terrains(pr.Z, pr.terrain_y, pr.log_ell, pr.log_sf, pr.log_sn)
        alphas = [sum(w * tg[i][o].alpha for i, w in enumerate(pr.terrain_w)) for o in range(2)]
        gps = tg[0]
    else:
        gps = G.build_pair(pr.Z, pr.y, pr.log_ell, pr.log_sf, pr.log_sn)
        alphas = [g.alpha for g in gps]
    absdot = np.stack([np.abs(G.se_ard(q, g.Z, g.log_ell, g.log_sf)) @ np.abs(a)
                       for g, a in zip(gps, alphas)], axis=1)
    return absdot.reshape(tr_o.u.shape[0], tr_o.u.shape[1], 2)


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
def _mean_bound(pr, tr_o):
    """FP32 dot-product bound of each step's GP mean [T, K, 2]: 1e-5 + 8 eps32 sum_j |k_j alpha_j|
    at the oracle's queries (Eq. 3's mean)."""
    return 1e-5 + 8 * EPS32 * _bf16_bounds(pr, tr_o)


def _nominal_traces(pr, ctx):
    """Alg. 1 Step 2's nominal sequence: the oracle's and the GPU's one-sample zero-noise rollout,
    the GPU's at the launch shape of ctx (its tightening table is that rollout's covariance)."""
    pn = dataclasses.replace(pr, K=1, params=dict(pr.params, sig_v=0.0, sig_w=0.0, tighten=0))
    _, tr_n = mppi.rollout(pn, pr.x0, pr.U0, 0)
    cn = B.gpmppi_init(pn, B.FP32)
    tun = B.gpmppi_get_tuning(ctx)
    B.gpmppi_set_tuning(cn, tun["groups"], tun["rotate"], tun["waves"], tun["split"])
    _, tg = gpu_rollout(pn, ctx=cn, seed=0)
    return tr_n, tg["x"], tg["gp_var"]


def _margin_covariance(pr, tr_o, E, nominal):
    """Position covariance [T, K, 3] each step's margins use (at k + 1) and its bound: the sample's
    own (R7), or with Step-2 tightening the nominal sequence's (R27)."""
    if pr.params.get("tighten", 0) != 1:
        return tr_o.sxy[1:], FB.position_block(E)[1:]
    assert nominal is not None, "Step-2 tightening needs the nominal traces"
    tr_n, x_n, var_n = nominal
    En, _ = FB.sigma_bound(pr, tr_n.x, tr_n.gp_var, x_n, var_n)
    K = tr_o.x.shape[1]
    return (np.repeat(tr_n.sxy[1:, :1], K, axis=1), np.repeat(FB.position_block(En)[1:, :1], K, axis=1))


def _check_rollout(pr, S_g, tr_g, S_o, tr_o, label, nominal=None, mean_bound=None):
    ex = rel_err(tr_g["x"], tr_o.x, 1.0)
    eu = np.abs(tr_g["u"] - tr_o.u)
    em = np.abs(tr_g["gp_mean"] - tr_o.gp_mean)
    ev = np.abs(tr_g["gp_var"] - tr_o.gp_var)
    E, _ = FB.sigma_bound(pr, tr_o.x, tr_o.gp_var, tr_g["x"], tr_g["gp_var"])
    exy = FB.position_block(E)
    sxy_c, exy_c = _margin_covariance(pr, tr_o, E, nominal)
    esxy = np.abs(tr_g["sxy"] - tr_o.sxy)
    edl = np.abs(tr_g["d_lane"] - tr_o.d_lane)
    bdl = FB.lane_distance_bound(pr, tr_o.x, tr_g["x"], tr_o.d_lane)
    elm = np.abs(tr_g["lane_margin"] - tr_o.lane_margin)
    blm = FB.lane_margin_bound(pr, tr_o.x, tr_g["x"], tr_o.d_lane, sxy_c, exy_c)
    fin = np.isfinite(tr_o.obs_margin)
    eom = np.where(fin, np.abs(np.where(fin, tr_g["obs_margin"], 0.0) - np.where(fin, tr_o.obs_margin, 0.0)), 0.0)
    bom = FB.obstacle_margin_bound(pr, tr_o.x, tr_g["x"], sxy_c, exy_c)
    flip = mppi.flip_budget(pr, tr_o, FLIP_BAND)
    eS = np.abs(S_g - S_o) - flip
    mb = _mean_bound(pr, tr_o) if mean_bound is None else mean_bound

    def frac(e, b):
        with np.errstate(divide="ignore", invalid="ignore"):
            return float(np.max(np.where(b > 0, e / b, np.where(e > 0, np.inf, 0.0))))

    _print(label, x=ex.max(), u=eu.max(), gp_mean=em.max(), gp_var=ev.max(), d_lane=edl.max(),
           sxy_of_bound=frac(esxy, exy), lane_margin=elm.max(), lane_of_bound=frac(elm, blm),
           obs_margin=eom.max(), obs_of_bound=frac(eom, bom),
           cost=(eS / np.maximum(S_o, 1)).max(), flagged=float((flip > 0).sum()))
    assert np.all(ex <= TOL), "states"
    assert np.all(eu <= 1e-5), "sampled controls"
    assert np.all(em <= mb), "gp mean"
    assert np.all(ev <= 2e-6 + 1e-5 * tr_o.gp_var), "gp variance"
    assert np.all(edl <= bdl), "lane distance"
    assert np.all(esxy <= exy), "position covariance"
    assert np.all(elm <= blm), "lane margin"
    assert np.array_equal(np.isfinite(tr_g["obs_margin"]), fin)
    assert np.all(eom <= bom), "obstacle margin"
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
    """Where indicator margins lie within the flip band, the oracle's U may move by the weights of
    the indicators that flip: first-order effect of the cost tolerance plus the flipped weights."""
    lam = pr.params["lam"]
    tolS = TOL * np.maximum(S_o, 1.0)
    spread = np.einsum("s,tsc->tc", w_o, np.abs(u_o - U_o[:, None, :]))
    infl = np.einsum("s,tsc->tc", w_o * (np.expm1(np.minimum(flip / lam, 50.0))), np.abs(u_o - U_o[:, None, :]))
    return TOL * np.maximum(np.abs(U_o), 1.0) + 2 * tolS.max() / lam * spread + 2 * infl


def _check_update(pr, U_g, S_g, w_g, u_o, U_o, S_o, w_o, flip, label):
    """Alg. 1's weights and weighted update at 1e-5 relative: (1) against the oracle's weights of the
    GPU's own costs and the oracle's sampled controls, which fixes the indicator decisions to the
    GPU's; (2) against the oracle's own U wherever no sample has an indicator margin within the
    flip band (otherwise within the flipped indicators' effect)."""
    lam = pr.params["lam"]
    w_ref = mppi.weights(S_g, lam)
    U_ref = mppi.update(w_ref, u_o)
    e_ref = np.abs(U_g - U_ref) / np.maximum(np.abs(U_ref), 1.0)
    e_o = np.abs(U_g - U_o) / np.maximum(np.abs(U_o), 1.0)
    n_flag = int((flip > 0).sum())
    vals = dict(U_vs_own_cost_weights=e_ref.max(), U_vs_oracle=e_o.max(), flagged=float(n_flag))
    if w_g is not None:
        # FP32 weights: the exponent (S - min S) / lambda carries about 2 eps32 of its size
        gap = (S_g - S_g.min()) / lam
        ew = np.abs(w_g - w_ref)
        vals["w_of_bound"] = float(np.max(ew / ((TOL + 4 * EPS32 * gap) * w_ref + 1e-37)))
        assert np.all(ew <= (TOL + 4 * EPS32 * gap) * w_ref + 1e-37), "weights of the GPU's costs"
        assert abs(w_g.sum() - 1.0) <= TOL
    _print(label, **vals)
    assert np.all(e_ref <= TOL), "U against the weights of the GPU's costs"
    if n_flag == 0:
        assert np.all(e_o <= TOL), "U against the oracle"
    else:
        assert np.all(np.abs(U_g - U_o) <= _u_tolerance(pr, S_o, w_o, u_o, U_o, flip)), "U against the oracle"


@pytest.mark.parametrize("cfg", ["c0", "small_eight"])
def test_step_matches_oracle(cfg):
    pr = W.make_config(0) if cfg == "c0" else W.small_problem(K=300, T=15, M=70, n_obs=8, path="eight",
                                                              seed_data=31, U_scale=1.0)
    U_g, S_g, w_g = gpu_step(pr)
    U_o, S_o, w_o, tr_o = mppi.iteration(pr)
    flip = mppi.flip_budget(pr, tr_o, FLIP_BAND)
    assert np.all(np.abs(S_g - S_o) <= TOL * np.maximum(S_o, 1) + flip)
    _check_update(pr, U_g, S_g, w_g, tr_o.u, U_o, S_o, w_o, flip, f"step {cfg}")


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
    _print("step c1", cost=(np.abs(S_g - S_o) / np.maximum(S_o, 1)).max())
    assert np.all(np.abs(S_g - S_o) <= TOL * np.maximum(S_o, 1) + flip)
    _check_update(pr, U_g, S_g, w_g, tr_o.u, U_o, S_o, w_o, flip, "step c1")


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
    g = np.load(path)
    U_g, S_full, w_g = gpu_step(pr)
    np.testing.assert_array_equal(S_full, S_g)   # step and rollout agree bitwise
    assert np.all(np.abs(S_g - g["S"]) <= TOL * np.maximum(g["S"], 1) + g["flip"])
    # the update's sampled controls are the oracle's (Philox words are bit-exact, Box-Muller in FP64)
    from oracle.philox import sampled_controls
    p = pr.params
    u_o = sampled_controls(pr.U0, np.arange(pr.K), pr.seed, (p["sig_v"], p["sig_w"]), p["u_min"], p["u_max"])
    _check_update(pr, U_g, S_g, w_g, u_o, g["U"], g["S"], g["w"], g["flip"], "c2 full")


# BF16 forms at c2: the variance bars of the GP-level tests, and the U bars the forms are stated at
FORM_VAR_TOL = {B.BF16X3: 5e-5, B.BF16: 2e-2}
FORM_U_TOL = {B.BF16X3: 1e-5, B.BF16: 1e-3}


def _form_margin_band(pr, tr_g, vtol):
    """Per (step, sample) bounds [T, K] on |margin_gpu - margin_oracle| (lane, obstacle) for a form
    whose GP variances are within vtol of the oracle's and whose states are within the FP32 bar:
    the forward error bounds of Eq. (10) and Eqs. (13)-(16) evaluated around the GPU's own
    trajectory (first order in the variance error)."""
    x_g, var_g = tr_g["x"], tr_g["gp_var"]
    x_p = x_g + TOL * np.maximum(np.abs(x_g), 1.0)
    E, sig = FB.sigma_bound(pr, x_g, var_g, x_p, var_g + vtol)
    sxy, exy = FB.position_block(sig)[1:], FB.position_block(E)[1:]
    return (FB.lane_margin_bound(pr, x_g, x_p, tr_g["d_lane"], sxy, exy),
            FB.obstacle_margin_bound(pr, x_g, x_p, sxy, exy))


@pytest.mark.parametrize("waves", [None, 12])
@pytest.mark.parametrize("prec", [B.BF16, B.BF16X3])
def test_c2_bf16_forms_end_to_end(prec, waves):
    """The precision forms at c2's full size, end to end.  States, controls and GP means stay at the
    FP32 bar (the trajectory depends on the means only); on sampled samples each cost is within
    w_var sum_k |ds2_k| (its measured variance differences) plus the weights of the indicators whose
    margin lies within the measured margin differences; every cost is within 2 T w_var vtol plus the
    weights of the indicators whose own margin lies within the band that vtol allows (an indicator
    can differ from the oracle's only where the margin's sign can); U is within the form's stated
    bar of the oracle's U.  waves = 12: the wave-specialised shape; None: the context's default."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "c2_oracle.npz"))
    pr = W.make_config(2)
    vtol, utol = FORM_VAR_TOL[prec], FORM_U_TOL[prec]
    ctx = B.gpmppi_init(pr, prec)
    if waves is not None:
        B.gpmppi_set_tuning(ctx, B.gpmppi_get_tuning(ctx)["groups"], 0, waves)
    S_g, tr_g = gpu_rollout(pr, ctx=ctx)
    U_g, S2, _ = gpu_step(pr, ctx=ctx)
    np.testing.assert_array_equal(S2, S_g)
    # sampled samples against the oracle's traces
    ids = np.unique(np.concatenate([np.arange(0, pr.K, 257), [pr.K - 1, pr.K - 32, 31, 32]]))
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed, sample_ids=ids)
    sub = {k: (v[:, ids] if v.ndim >= 2 else v) for k, v in tr_g.items()}
    prs = W.make_config(2, K=len(ids))
    absdot = _bf16_bounds(prs, tr_o)
    _check_bf16_rollout(prec, S_g[ids], sub, tr_o, absdot, f"c2 form={prec} sampled")
    dvar = np.abs(sub["gp_var"] - tr_o.gp_var)
    band = np.maximum(np.abs(sub["lane_margin"] - tr_o.lane_margin),
                      np.where(np.isfinite(tr_o.obs_margin),
                               np.abs(np.nan_to_num(sub["obs_margin"] - tr_o.obs_margin, posinf=0.0)), 0.0))
    p = pr.params
    disc = p["discount"] ** np.arange(pr.T)
    near_lane = np.abs(tr_o.lane_margin) <= band + 1e-4
    near_obs = np.abs(tr_o.obs_margin) <= band + 1e-4
    flip_s = p["w_lane"] * (near_lane * disc[:, None]).sum(0) + p["w_obs"] * near_obs.sum(0)
    bound_s = TOL * np.maximum(S_o, 1.0) + p["w_var"] * dvar.sum(axis=(0, 2)) + flip_s
    eS_s = np.abs(S_g[ids] - S_o)
    # every sample against the stored oracle costs
    bl, bo = _form_margin_band(pr, tr_g, vtol)
    near_lane = np.abs(tr_g["lane_margin"]) <= bl
    near_obs = np.isfinite(tr_g["obs_margin"]) & (np.abs(tr_g["obs_margin"]) <= bo)
    flip_all = p["w_lane"] * (near_lane * disc[:, None]).sum(0) + p["w_obs"] * near_obs.sum(0)
    bound_all = TOL * np.maximum(g["S"], 1.0) + 2 * pr.T * p["w_var"] * vtol + flip_all
    mb = float(max(bl.max(), bo.max()))
    eS_all = np.abs(S_g - g["S"])
    eU = np.abs(U_g - g["U"])
    _print(f"c2 form={prec} waves={waves}", cost_sampled=eS_s.max(), cost_sampled_of_bound=(eS_s / bound_s).max(),
           cost_all=eS_all.max(), cost_all_of_bound=(eS_all / bound_all).max(), margin_band_max=mb,
           flagged=float((flip_all > 0).sum()), U=eU.max())
    assert np.all(eS_s <= bound_s), "sampled costs"
    assert np.all(eS_all <= bound_all), "costs"
    assert np.all(eU <= utol * np.maximum(np.abs(g["U"]), 1.0)), "U"


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
        U_g, S_g, w_g = gpu_step(pr, x0=x, U=U, seed=pr.seed_at(step), ctx=ctx)
        flip = mppi.flip_budget(pr, tr_o, FLIP_BAND)
        assert np.all(np.abs(S_g - S_o) <= TOL * np.maximum(S_o, 1) + flip)
        _check_update(pr, U_g, S_g, w_g, tr_o.u, U_o, S_o, w_o, flip, f"closed loop step {step}")
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
    ctx = B.gpmppi_init(pr, B.FP32)
    S_g, tr_g = gpu_rollout(pr, ctx=ctx)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    nominal = _nominal_traces(pr, ctx) if mode == "step2" else None
    _check_rollout(pr, S_g, tr_g, S_o, tr_o, f"rollout {mode}", nominal=nominal)
    U_g, S2, _ = gpu_step(pr, ctx=ctx)
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

"""The wave-specialised rollout (waves = 12: eight waves walk W, four generate the kernel vectors
and carry the sample state) against the FP64 oracle, at the bars of the BF16 forms' other shapes
(states, controls and GP means at the FP32 bar, the variance at the form's), and its shape rules."""
import numpy as np
import pytest

from oracle import mppi
from paper_2411_03289_amd import gpmppi as B
from paper_2411_03289_amd import workloads as W

from gpu_util import gpu_rollout, gpu_step
from test_gpu_parity import _bf16_bounds, _check_bf16_rollout, _print

pytestmark = pytest.mark.gpu

PIPE = 12
FORMS = {B.BF16: 2, B.BF16X3: 1}   # form: the group count its k operand allows at M_pad = 1024


def _pipe_ctx(pr, prec):
    ctx = B.gpmppi_init(pr, prec)
    B.gpmppi_set_tuning(ctx, FORMS[prec], 0, PIPE)
    assert B.gpmppi_get_tuning(ctx)["waves"] == PIPE
    return ctx


def test_shape_rules():
    pr = W.small_problem(K=70, T=3, M=1000, seed_data=31)
    for prec, groups in FORMS.items():
        ctx = B.gpmppi_init(pr, prec)
        B.gpmppi_set_tuning(ctx, groups, 0, PIPE)
        with pytest.raises(B.GpmppiError):
            B.gpmppi_set_tuning(ctx, groups, 0, PIPE, 1)            # no output split
        if groups == 2:
            with pytest.raises(B.GpmppiError):
                B.gpmppi_set_tuning(ctx, 1, 0, PIPE)                 # the largest group count only
    with pytest.raises(B.GpmppiError):
        B.gpmppi_set_tuning(B.gpmppi_init(pr, B.FP32), 1, 0, PIPE)   # BF16 forms only
    small = W.small_problem(K=70, T=3, M=300, seed_data=31)
    with pytest.raises(B.GpmppiError):
        B.gpmppi_set_tuning(B.gpmppi_init(small, B.BF16), 2, 0, PIPE)   # M_pad = 1024 only


def _with_track(pr, pts):
    pr.path_pts = pts
    return pr


CASES = {
    # ragged K (150 = 2 x 64 + 22), polyline track, obstacles
    "eight": dict(make=lambda: W.small_problem(K=150, T=10, M=1000, n_obs=7, path="eight", seed_data=26,
                                               U_scale=1.0)),
    # one sample, one step
    "single": dict(make=lambda: W.small_problem(K=1, T=1, M=1024, n_obs=3, path="circle", seed_data=27,
                                                U_scale=1.0)),
    # circle track with the goal terms (Eq. 12), a longer horizon
    "goal": dict(make=lambda: W.small_problem(K=100, T=25, M=990, n_obs=9, path="circle", seed_data=28,
                                              U_scale=1.0),
                 params=W.task_params("avoid", goal=(0.3, 0.2))),
    # samples spread widely (large controls) around a polyline whose length is not a multiple
    # of the 16-segment bounding circles
    "spread": dict(make=lambda: _with_track(W.small_problem(K=200, T=40, M=1000, n_obs=5, path="eight",
                                                            seed_data=34, U_scale=3.0), W.figure_eight(8.0, 250))),
    # starting off the track, where several circles are about as near
    "offtrack": dict(make=lambda: _with_track(W.small_problem(K=128, T=20, M=1000, n_obs=4, path="eight",
                                                              seed_data=35, U_scale=1.5,
                                                              x0=[2.5, 1.0, 0.3, 1.0, 0.0]),
                                              W.figure_eight(8.0, 250))),
    # terrain ensemble (Eq. 3: variance scale and mixed alpha)
    "terrains": dict(make=lambda: W.add_terrains(W.small_problem(K=96, T=12, M=1000, n_obs=6, path="eight",
                                                                 seed_data=29, U_scale=1.0),
                                                 seed=30, weights=(0.6, 0.25, 0.15))),
}


@pytest.mark.parametrize("prec", list(FORMS))
@pytest.mark.parametrize("case", list(CASES))
def test_rollout_matches_oracle(prec, case):
    spec = CASES[case]
    pr = spec["make"]()
    if "params" in spec:
        pr.params.update(spec["params"])
    print(f"case {case} form {prec}: K={pr.K} T={pr.T} M={pr.Z.shape[0]}", flush=True)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    absdot = _bf16_bounds(pr, tr_o)
    ctx = _pipe_ctx(pr, prec)
    S_g, tr_g = gpu_rollout(pr, ctx=ctx)
    _check_bf16_rollout(prec, S_g, tr_g, tr_o, absdot, f"pipe {case} form={prec}")
    _check_lane_distance(tr_g, tr_o)
    # the same launch twice: every hand-over is fixed, so the results are too
    S_2, tr_2 = gpu_rollout(pr, ctx=ctx)
    np.testing.assert_array_equal(S_2, S_g)
    for k in tr_g:
        np.testing.assert_array_equal(tr_2[k], tr_g[k])
    assert B.gpmppi_status_flags(ctx) == 0


def _check_lane_distance(tr_g, tr_o):
    """The distance to the track is 1-Lipschitz in the position, so it can differ from the
    oracle's by no more than the positions do (plus FP32 rounding): the state waves' share of the
    segment loop must find the nearest segment."""
    dpos = np.abs(tr_g["x"][1:, :, :2] - tr_o.x[1:, :, :2]).max(axis=2)
    err = np.abs(tr_g["d_lane"] - tr_o.d_lane)
    _print("lane distance", err=err.max(), of_bound=(err / (1.5 * dpos + 2e-5)).max())
    assert np.all(err <= 1.5 * dpos + 2e-5), "lane distance"


@pytest.mark.parametrize("prec", list(FORMS))
def test_step2_tightening_and_step(prec):
    pr = W.small_problem(K=80, T=14, M=1000, n_obs=7, path="eight", seed_data=32, U_scale=1.0)
    pr.params["tighten"] = 1
    ctx = _pipe_ctx(pr, prec)
    S_g, tr_g = gpu_rollout(pr, ctx=ctx)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    _check_bf16_rollout(prec, S_g, tr_g, tr_o, _bf16_bounds(pr, tr_o), f"pipe step2 form={prec}")
    _check_lane_distance(tr_g, tr_o)
    U_g, S2, _ = gpu_step(pr, ctx=ctx)
    np.testing.assert_array_equal(S2, S_g)


def test_agrees_with_the_eight_wave_shape():
    """The same problem at waves = 8 and 12: the kernel vectors differ only in how their FP32
    exponents are formed (split-BF16 matrix-core products against exact differences) and the
    partial sums in their grouping, so states, means and variances agree far inside the form's bar."""
    pr = W.small_problem(K=256, T=20, M=1024, n_obs=8, path="eight", seed_data=33, U_scale=1.0)
    ctx = B.gpmppi_init(pr, B.BF16)
    B.gpmppi_set_tuning(ctx, 2, 0, 8)
    S_8, tr_8 = gpu_rollout(pr, ctx=ctx)
    B.gpmppi_set_tuning(ctx, 2, 0, PIPE)
    S_p, tr_p = gpu_rollout(pr, ctx=ctx)
    ex = np.abs(tr_p["x"] - tr_8["x"]).max()
    em = np.abs(tr_p["gp_mean"] - tr_8["gp_mean"]).max()
    ev = np.abs(tr_p["gp_var"] - tr_8["gp_var"]).max()
    _print("pipe vs 8 waves", x=ex, gp_mean=em, gp_var=ev)
    assert ex <= 1e-4 and em <= 1e-4 and ev <= 2e-3


def test_a_wait_that_gives_up_marks_its_workgroup():
    """The hand-over waits are bounded by the context's exchange spin; a negative spin makes every
    wait that is not met at once give up (a test hook: with the default spin a wait can only give
    up through a defect).  A workgroup that gave up reports NaN costs and the status bit, every
    other one its ordinary results, and the next launch at the default spin is whole again."""
    pr = W.small_problem(K=256, T=6, M=1000, n_obs=4, path="eight", seed_data=36, U_scale=1.0)
    ctx = _pipe_ctx(pr, B.BF16)
    S_ok, _ = gpu_rollout(pr, ctx=ctx)
    assert B.gpmppi_status_flags(ctx) == 0
    B.gpmppi_set_exchange_spin(ctx, -1)
    S_st, _ = gpu_rollout(pr, ctx=ctx)
    flags = B.gpmppi_status_flags(ctx)
    bad = np.isnan(S_st)
    _print("forced stall", nan_samples=float(bad.sum()))
    assert flags & B.FLAG_PIPELINE_STALL
    assert bad.any()
    np.testing.assert_array_equal(S_st[~bad], S_ok[~bad])
    B.gpmppi_set_exchange_spin(ctx, 0)
    S_again, _ = gpu_rollout(pr, ctx=ctx)
    np.testing.assert_array_equal(S_again, S_ok)
    assert B.gpmppi_status_flags(ctx) == 0

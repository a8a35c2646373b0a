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
    # the same launch twice: every hand-over is fixed, so the results are too
    S_2, tr_2 = gpu_rollout(pr, ctx=ctx)
    np.testing.assert_array_equal(S_2, S_g)
    for k in tr_g:
        np.testing.assert_array_equal(tr_2[k], tr_g[k])
    assert B.gpmppi_status_flags(ctx) == 0


@pytest.mark.parametrize("prec", list(FORMS))
def test_step2_tightening_and_step(prec):
    pr = W.small_problem(K=80, T=14, M=1000, n_obs=7, path="eight", seed_data=32, U_scale=1.0)
    pr.params["tighten"] = 1
    ctx = _pipe_ctx(pr, prec)
    S_g, tr_g = gpu_rollout(pr, ctx=ctx)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed)
    _check_bf16_rollout(prec, S_g, tr_g, tr_o, _bf16_bounds(pr, tr_o), f"pipe step2 form={prec}")
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

"""Output split: the two GP outputs of each 32-sample block on two workgroups
that exchange the GP means and the second output's variance every step.  The
exchanged values enter the same arithmetic as in the unsplit rollout, so every
cost, trace row, control update and closed-loop state must equal the unsplit
launch's bit for bit (the unsplit path is held to the oracle by the parity
tests); the oracle is checked directly at the c1 size."""
import numpy as np
import pytest

from oracle import mppi
from paper_2411_03289_amd import gpmppi as B
from paper_2411_03289_amd import workloads as W

from gpu_util import dev, gpu_rollout, gpu_step, torch
from test_gpu_parity import _check_rollout as check_rollout

pytestmark = pytest.mark.gpu

FORMS = {"fp32": B.FP32, "bf16": B.BF16, "bf16x3": B.BF16X3}


def _case(name):
    if name == "c0":
        return W.make_config(0)
    if name == "ragged_rows":      # M = 300: 10 row tiles, walked as single rows; 10 sample blocks, ragged
        return W.small_problem(K=300, T=13, M=300, n_obs=7, path="eight", seed_data=201, U_scale=1.0, n_data=300)
    if name == "pairs":            # M = 256: 4 row-tile pairs
        return W.small_problem(K=97, T=9, M=256, n_obs=3, path="circle", seed_data=202, U_scale=0.7, n_data=256)
    if name == "tiny":             # one sample, one training point
        return W.small_problem(K=1, T=5, M=1, n_obs=2, path="eight", seed_data=203, U_scale=1.0)
    if name == "goal":
        pr = W.small_problem(K=80, T=14, M=50, n_obs=7, path="eight", seed_data=91, U_scale=1.0)
        pr.params.update(W.task_params("avoid", goal=(0.3, 0.2)))
        return pr
    if name == "terrains":         # ensemble weights fold into alpha and the variance scale
        return W.add_terrains(W.small_problem(K=96, T=12, M=60, n_obs=6, path="eight", seed_data=81, U_scale=1.0),
                              seed=82, weights=(0.6, 0.25, 0.15))
    if name == "step2":
        pr = W.small_problem(K=80, T=14, M=50, n_obs=7, path="eight", seed_data=91, U_scale=1.0)
        pr.params["tighten"] = 1
        return pr
    raise KeyError(name)


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("case", ["c0", "ragged_rows", "pairs", "tiny", "goal", "step2", "terrains"])
def test_split_equals_unsplit_bitwise(form, case):
    pr = _case(case)
    prec = FORMS[form]
    print(f"split {form} {case}: K={pr.K} T={pr.T} M={pr.M}", flush=True)
    ctx = B.gpmppi_init(pr, prec)
    for waves in (4, 8):
        for rotate in (0, 1):
            res = []
            for split in (0, 1):
                B.gpmppi_set_tuning(ctx, 1, rotate, waves, split)
                assert B.gpmppi_get_tuning(ctx)["split"] == split
                res.append(gpu_rollout(pr, prec, ctx=ctx) + gpu_step(pr, prec, ctx=ctx))
            (S0, tr0, U0, Ss0, w0), (S1, tr1, U1, Ss1, w1) = res
            np.testing.assert_array_equal(S1, S0)
            for k in tr0:
                np.testing.assert_array_equal(tr1[k], tr0[k], err_msg=f"trace {k} waves={waves} rotate={rotate}")
            np.testing.assert_array_equal(U1, U0)
            np.testing.assert_array_equal(Ss1, S1)
            np.testing.assert_array_equal(w1, w0)


def test_split_c1_matches_oracle_and_unsplit():
    pr = W.make_config(1)
    ctx = B.gpmppi_init(pr, B.FP32)
    B.gpmppi_set_tuning(ctx, 1, 1, 8, 0)
    U_a, S_a, w_a = gpu_step(pr, ctx=ctx)
    for waves in (4, 8):
        B.gpmppi_set_tuning(ctx, 1, 1, waves, 1)
        U_b, S_b, w_b = gpu_step(pr, ctx=ctx)
        if waves == 8:
            np.testing.assert_array_equal(S_b, S_a)
            np.testing.assert_array_equal(U_b, U_a)
            np.testing.assert_array_equal(w_b, w_a)
    # against the oracle, on sampled blocks (first, middle, last, ragged edges)
    ids = np.unique(np.concatenate([np.arange(0, pr.K, 97), [0, 31, 32, 2047, 2048, pr.K - 1]]))
    S_g, tr_g = gpu_rollout(pr, ctx=ctx)
    S_o, tr_o = mppi.rollout(pr, pr.x0, pr.U0, pr.seed, sample_ids=ids)
    sub = {k: (v[:, ids] if v.ndim >= 2 else v) for k, v in tr_g.items()}
    check_rollout(W.make_config(1, K=len(ids)), S_g[ids], sub, S_o, tr_o, "split c1 sampled")


def test_split_closed_loop_eager_graph_and_unsplit_agree():
    t = torch()
    pr = W.make_config(1, K=512, T=20, M=64, n_obs=10)
    ctx = B.gpmppi_init(pr, B.FP32)
    res = []
    for split, use_graph in ((0, False), (1, False), (1, True)):
        B.gpmppi_set_tuning(ctx, 1, 1, 8, split)
        xd, Ud = dev(pr.x0), dev(pr.U0)
        n = 40   # 40 launches per loop: the exchange epoch advances on every one
        xh = t.empty((n + 1) * 5, device="cuda")
        uh = t.empty(n * 2, device="cuda")
        B.gpmppi_closed_loop(ctx, xd, Ud, pr.seed, n, 0.3, xh, uh, use_graph=use_graph)
        t.cuda.synchronize()
        res.append((xh.cpu().numpy(), uh.cpu().numpy(), Ud.cpu().numpy()))
    for r in res[1:]:
        for a, b in zip(res[0], r):
            np.testing.assert_array_equal(b, a)
    assert B.gpmppi_status_flags(ctx) == 0


def test_split_admissibility_and_tuner():
    # c2's 512 sample blocks need 1024 resident workgroups: not admissible
    big = W.make_config(2, T=2)
    ctx = B.gpmppi_init(big, B.FP32)
    with pytest.raises(B.GpmppiError):
        B.gpmppi_set_tuning(ctx, 1, 1, 8, 1)
    assert B.gpmppi_get_tuning(ctx)["split"] == 0
    pr = W.make_config(1, T=10)
    ctx = B.gpmppi_init(pr, B.FP32)
    with pytest.raises(B.GpmppiError):
        B.gpmppi_set_tuning(ctx, 2, 1, 8, 1)    # split needs one sample group
    with pytest.raises(B.GpmppiError):
        B.gpmppi_set_tuning(ctx, 1, 1, 8, 2)
    chosen = B.gpmppi_tune(ctx, dev(pr.x0), dev(pr.U0), pr.seed, reps=2)
    print("c1 tuning", chosen, flush=True)
    got = B.gpmppi_get_tuning(ctx)
    assert {k: got[k] for k in ("groups", "rotate", "waves", "split")} == \
        {k: chosen[k] for k in ("groups", "rotate", "waves", "split")}
    S_a, _ = gpu_rollout(pr, ctx=ctx)
    B.gpmppi_set_tuning(ctx, 1, chosen["rotate"] if chosen["groups"] == 1 else 1, chosen["waves"], 0)
    S_b, _ = gpu_rollout(pr, ctx=ctx)
    if chosen["groups"] == 1:
        np.testing.assert_array_equal(S_a, S_b)


def test_split_exchange_timeout_runs_each_block_alone_with_identical_results():
    # the fallback path, forced from the host: every exchange wait gives up at once, so every
    # workgroup of the split launch computes its block alone with the unsplit code; costs, U and
    # weights equal the unsplit launch's bit for bit and the status word reports the time-out
    # (not a non-finite cost); the next launch at the default wait is split again and exact
    # (records of the abandoned launch carry its epoch)
    pr = W.small_problem(K=96, T=8, M=40, n_obs=3, path="eight", seed_data=211, U_scale=1.0)
    ctx = B.gpmppi_init(pr, B.FP32)
    B.gpmppi_set_tuning(ctx, 1, 1, 8, 0)
    U_a, S_a, w_a = gpu_step(pr, ctx=ctx)
    S_ra, tr_a = gpu_rollout(pr, ctx=ctx)
    assert B.gpmppi_status_flags(ctx) == 0
    B.gpmppi_set_tuning(ctx, 1, 1, 8, 1)
    B.gpmppi_set_exchange_spin(ctx, -1)
    U_b, S_b, w_b = gpu_step(pr, ctx=ctx)
    np.testing.assert_array_equal(S_b, S_a)
    np.testing.assert_array_equal(U_b, U_a)
    np.testing.assert_array_equal(w_b, w_a)
    assert B.gpmppi_status_flags(ctx) == B.FLAG_EXCHANGE_TIMEOUT
    S_rb, tr_b = gpu_rollout(pr, ctx=ctx)
    np.testing.assert_array_equal(S_rb, S_ra)
    for key in tr_a:
        np.testing.assert_array_equal(tr_b[key], tr_a[key], err_msg=key)
    assert B.gpmppi_status_flags(ctx) == B.FLAG_EXCHANGE_TIMEOUT
    B.gpmppi_set_exchange_spin(ctx, 0)
    U_c, S_c, w_c = gpu_step(pr, ctx=ctx)
    np.testing.assert_array_equal(S_c, S_a)
    np.testing.assert_array_equal(U_c, U_a)
    np.testing.assert_array_equal(w_c, w_a)
    assert B.gpmppi_status_flags(ctx) == 0

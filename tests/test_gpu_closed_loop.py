"""The receding-horizon loop of Alg. 1 at the c1 workload's full size (K = 4096, T = 50,
M = 256, 20 obstacles, figure-eight track, 100 control steps) against the oracle's own loop
(tests/golden/c1_loop.npz, written by the oracle alone).

Re-synced: every step starts both sides from the oracle's state and warm-started controls, so
each step is an independent check of one iteration at the FP32 bars (U at 1e-5 relative).
Free-running: the device loop (eager launches and a HIP graph, bitwise equal) against the oracle's
loop; the state drift is reported per step."""
import os

import numpy as np
import pytest

from oracle import mppi
from oracle.philox import sampled_controls
from paper_2411_03289_amd import gpmppi as B
from paper_2411_03289_amd import workloads as W

from gpu_util import dev, gpu_step, torch

pytestmark = pytest.mark.gpu

TOL = 1e-5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c1_loop.npz")


def _ctx(pr):
    ctx = B.gpmppi_init(pr, B.FP32)
    chosen = B.gpmppi_tune(ctx, dev(pr.x0), dev(pr.U0), pr.seed, reps=2)
    print("c1 tuned shape", chosen, flush=True)
    return ctx


def _flagged_tolerance(g, t, pr, S_g, u_o, U_o):
    """Where some sample of step t has an indicator margin within the flip band, the oracle's U'
    may move by the first-order effect of the cost tolerance and of the flipped indicators on the
    weights (the GPU's costs stand in for the oracle's in the weights, within 1e-5 relative away
    from the flipped indicators)."""
    lam = pr.params["lam"]
    rows = g["flagged_rows"][g["flagged_rows"][:, 0] == t]
    flip = np.zeros(pr.K)
    flip[rows[:, 1].astype(int)] = rows[:, 2]
    w = mppi.weights(S_g, lam)
    dev_u = np.abs(u_o - U_o[:, None, :])
    spread = np.einsum("s,tsc->tc", w, dev_u)
    infl = np.einsum("s,tsc->tc", w * np.expm1(np.minimum(flip / lam, 50.0)), dev_u)
    tolS = TOL * max(float(g["S_max"][list(g["flagged_steps"]).index(t)]), 1.0)
    return TOL * np.maximum(np.abs(U_o), 1.0) + 2 * tolS / lam * spread + 2 * infl


def test_c1_resynced_steps_match_oracle():
    g = np.load(GOLDEN)
    pr = W.make_config(1)
    p = pr.params
    ctx = _ctx(pr)
    n = g["U_out"].shape[0]
    worst_ref, worst_o, n_flagged = 0.0, 0.0, 0
    for t in range(n):
        seed = pr.seed_at(t)
        U_g, S_g, w_g = gpu_step(pr, x0=g["x"][t], U=g["U_in"][t], seed=seed, ctx=ctx)
        assert np.all(np.isfinite(S_g)), t
        u_o = sampled_controls(g["U_in"][t], np.arange(pr.K), seed, (p["sig_v"], p["sig_w"]), p["u_min"], p["u_max"])
        U_ref = mppi.update(mppi.weights(S_g, p["lam"]), u_o)
        e_ref = np.abs(U_g - U_ref) / np.maximum(np.abs(U_ref), 1.0)
        U_o = g["U_out"][t]
        e_o = np.abs(U_g - U_o) / np.maximum(np.abs(U_o), 1.0)
        worst_ref = max(worst_ref, float(e_ref.max()))
        assert np.all(e_ref <= TOL), (t, e_ref.max())
        if g["n_flag"][t] == 0:
            worst_o = max(worst_o, float(e_o.max()))
            assert np.all(e_o <= TOL), (t, e_o.max())
        else:
            n_flagged += 1
            assert np.all(np.abs(U_g - U_o) <= _flagged_tolerance(g, t, pr, S_g, u_o, U_o)), t
    print(f"c1 re-synced {n} steps: U vs own-cost weights {worst_ref:.2e}, U vs oracle {worst_o:.2e} "
          f"(steps without flagged samples), {n_flagged} steps with flagged samples", flush=True)


def test_c1_closed_loop_drift():
    t_ = torch()
    g = np.load(GOLDEN)
    pr = W.make_config(1)
    ctx = _ctx(pr)
    n = g["U_out"].shape[0]
    runs = []
    for use_graph in (False, True):
        xd, Ud = dev(pr.x0), dev(pr.U0)
        xh = t_.empty((n + 1) * 5, device="cuda")
        uh = t_.empty(n * 2, device="cuda")
        B.gpmppi_closed_loop(ctx, xd, Ud, pr.seed, n, float(g["amplitude"]), xh, uh, use_graph=use_graph)
        t_.cuda.synchronize()
        runs.append((xh.cpu().numpy().reshape(n + 1, 5).astype(np.float64), uh.cpu().numpy().reshape(n, 2)))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    np.testing.assert_array_equal(runs[0][1], runs[1][1])
    x_g, u0_g = runs[0]
    drift = np.max(np.abs(x_g - g["x"]) / np.maximum(np.abs(g["x"]), 1.0), axis=1)
    du0 = np.max(np.abs(u0_g - g["U_out"][:, 0]), axis=1)
    first_flag = int(np.argmax(g["n_flag"] > 0)) if np.any(g["n_flag"] > 0) else n
    marks = [1, 2, 5, 10, 20, 30, 40, 50, 60, 70, 80, 90, 100]
    print("c1 free-running drift (max relative state difference, floor 1) at steps "
          + ", ".join(f"{t}: {drift[t]:.2e}" for t in marks if t <= n)
          + f"; applied control difference max {du0.max():.2e}; first step with flagged samples {first_flag}",
          flush=True)
    assert np.all(np.isfinite(x_g))
    # until the first step whose oracle iteration has a near-threshold indicator, both loops see
    # the same decisions and stay at FP32 distance
    assert np.all(drift[: first_flag + 1] <= TOL)
    # afterwards the loops may part where an indicator flips; they stay on the same course
    assert np.all(drift <= 1e-2)

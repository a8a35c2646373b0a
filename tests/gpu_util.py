"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
bring its SoA outputs into the oracle's layout."""
import numpy as np

from paper_2411_03289_amd import gpmppi as B

TRACE_FIELDS = ("x_d", "sxy_d", "gp_mean_d", "gp_var_d", "d_lane_d", "lane_margin_d", "obs_margin_d", "u_d")


def torch():
    import torch as t
    return t


def dev(a, dtype=None):
    t = torch()
    return t.as_tensor(np.ascontiguousarray(a), dtype=dtype or t.float32, device="cuda")


def gpu_rollout(pr, precision=B.FP32, x0=None, U=None, seed=None, ctx=None):
    """Rollout with every trace field; returns (costs [K], trace dict in oracle layout)."""
    t = torch()
    K, T = pr.K, pr.T
    ctx = ctx or B.gpmppi_init(pr, precision)
    x0 = dev(pr.x0 if x0 is None else x0)
    U = dev(pr.U0 if U is None else U)
    costs = t.empty(K, device="cuda")
    tr = {k: t.full((B.TRACE_SIZES[k](K, T),), float("nan"), device="cuda") for k in TRACE_FIELDS}
    B.gpmppi_rollout(ctx, x0, U, pr.seed if seed is None else seed, costs, tr)
    t.cuda.synchronize()
    h = {k: v.cpu().numpy().astype(np.float64) for k, v in tr.items()}
    out = dict(
        x=h["x_d"].reshape(T + 1, 5, K).transpose(0, 2, 1),
        sxy=h["sxy_d"].reshape(T + 1, 3, K).transpose(0, 2, 1),
        gp_mean=h["gp_mean_d"].reshape(T, 2, K).transpose(0, 2, 1),
        gp_var=h["gp_var_d"].reshape(T, 2, K).transpose(0, 2, 1),
        d_lane=h["d_lane_d"].reshape(T, K),
        lane_margin=h["lane_margin_d"].reshape(T, K),
        obs_margin=h["obs_margin_d"].reshape(T, K),
        u=h["u_d"].reshape(T, 2, K).transpose(0, 2, 1),
    )
    return costs.cpu().numpy().astype(np.float64), out


def gpu_step(pr, precision=B.FP32, x0=None, U=None, seed=None, ctx=None):
    t = torch()
    ctx = ctx or B.gpmppi_init(pr, precision)
    x0 = dev(pr.x0 if x0 is None else x0)
    U = dev(pr.U0 if U is None else U)
    U_out = t.empty_like(U)
    costs = t.empty(pr.K, device="cuda")
    w = t.empty(pr.K, device="cuda")
    B.gpmppi_step(ctx, x0, U, pr.seed if seed is None else seed, U_out, costs, w)
    t.cuda.synchronize()
    return (U_out.cpu().numpy().astype(np.float64), costs.cpu().numpy().astype(np.float64),
            w.cpu().numpy().astype(np.float64))


def rel_err(g, o, floor):
    return np.abs(g - o) / np.maximum(np.abs(o), floor)

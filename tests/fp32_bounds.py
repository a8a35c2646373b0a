"""Forward error bounds of the FP32 path's covariance and constraint margins.

The GPU evaluates Eq. (10)'s covariance recurrence and the tightened margins
of Eqs. (13)-(16) in FP32 from its own states and GP variances.  Those inputs
are checked against the oracle on their own (states at 1e-5 relative, the
variance at its FP32 W-form bar); the bounds here say how far the covariance
and the margins may then move: the measured input differences pushed through
the recurrence, plus the FP32 rounding of the operations themselves.  A
dropped or wrong term moves a value by the size of that term, far outside
these bounds (the CPU tests plant such mistakes in an FP32 emulation).

Recurrence of the bound (entrywise, u = 2^-24, |.| entrywise absolute values,
A the oracle's Jacobian at x_k, A^ the FP32 one at the GPU state, dA >= |A^ - A|):

    E_{k+1} = |A^| E_k |A^|^T + dA |Sigma_k| |A^|^T + |A| |Sigma_k| dA^T
              + g |A^| (|Sigma_k| + E_k) |A^|^T + dt^2 diag(0, 0, 0, ds_v, ds_w)
              + 3u dt^2 diag(0, 0, 0, s2_v, s2_w)

with ds = |s2^ - s2| the measured variance difference, and g = 8u covering the
at most four roundings of each entry of A Sigma A^T (two fused multiply-adds
for A Sigma, two for (A Sigma) A^T) twice over.  dA bounds the Jacobian entries
-dt v sin(theta), dt cos(theta), dt v cos(theta), dt sin(theta) by the measured
state differences (|d(v sin)| <= |dv| + |v| |dtheta|) plus 4u of each entry.

Margins (Eqs. 14, 16): |d sqrt(x)| <= min(|dx| / sqrt(x), sqrt(|dx|)); the
largest eigenvalue moves by at most ||dSigma_XY||_2 <= ||E_XY||_F (Weyl);
distances to the centreline and to obstacle centres are 1-Lipschitz in the
position; each operation adds its FP32 rounding relative to the magnitudes it
combines (coordinates, radii, path extent).
"""
from __future__ import annotations

import numpy as np

from oracle import constraints as C
from oracle import dynamics as D

U32 = 2.0 ** -24


def oracle_covariances(pr, x_o, var_o):
    """The oracle's full 5x5 covariances [T+1, K, 5, 5] from its states and GP variances (Eq. 10)."""
    p = pr.params
    T, K = var_o.shape[0], var_o.shape[1]
    out = np.zeros((T + 1, K, 5, 5))
    for k in range(T):
        A = D.nominal_jacobian(x_o[k], p["dt"], p["tau_v"], p["tau_w"])
        out[k + 1] = D.covariance_step(out[k], A, var_o[k], p["dt"])
    return out


def jacobian_error(x_o, x_g, dt, tau_v, tau_w):
    """Entrywise bound [K, 5, 5] on |A(x_g) in FP32 - A(x_o)|."""
    th, v = x_o[:, 2], x_o[:, 3]
    dth = np.abs(x_g[:, 2] - th)
    dv = np.abs(x_g[:, 3] - v)
    vg = np.abs(x_g[:, 3])
    K = x_o.shape[0]
    dA = np.zeros((K, 5, 5))
    dvs = dt * (dv + np.abs(v) * dth) + 4 * U32 * dt * vg      # v sin(theta), v cos(theta)
    dc = dt * dth + 4 * U32 * dt                               # sin(theta), cos(theta)
    dA[:, 0, 2] = dA[:, 1, 2] = dvs
    dA[:, 0, 3] = dA[:, 1, 3] = dc
    dA[:, 2, 4] = U32 * dt
    dA[:, 3, 3] = U32 * abs(1.0 - dt / tau_v)
    dA[:, 4, 4] = U32 * abs(1.0 - dt / tau_w)
    return dA


def sigma_bound(pr, x_o, var_o, x_g, var_g):
    """Bound E [T+1, K, 5, 5] on |Sigma_gpu - Sigma_oracle| from the oracle's states x_o [T+1, K, 5]
    and GP variances var_o [T, K, 2] and the GPU's x_g, var_g; returns (E, Sigma_oracle)."""
    p = pr.params
    dt, tv, tw = p["dt"], p["tau_v"], p["tau_w"]
    sig = oracle_covariances(pr, x_o, var_o)
    T, K = var_g.shape[0], var_g.shape[1]
    E = np.zeros((T + 1, K, 5, 5))
    g = 8 * U32
    for k in range(T):
        A = np.abs(D.nominal_jacobian(x_o[k], dt, tv, tw))
        dA = jacobian_error(x_o[k], x_g[k], dt, tv, tw)
        Ah = A + dA
        AhT = np.transpose(Ah, (0, 2, 1))
        S = np.abs(sig[k])
        e = (Ah @ E[k] @ AhT + dA @ S @ AhT + A @ S @ np.transpose(dA, (0, 2, 1))
             + g * (Ah @ (S + E[k]) @ AhT))
        ds = np.abs(var_g[k] - var_o[k])
        e[:, 3, 3] += dt * dt * (ds[:, 0] + 3 * U32 * np.abs(var_o[k, :, 0]))
        e[:, 4, 4] += dt * dt * (ds[:, 1] + 3 * U32 * np.abs(var_o[k, :, 1]))
        E[k + 1] = e
    return E, sig


def position_block(S):
    """(Sigma_XX, Sigma_XY, Sigma_YY) [..., 3] of 5x5 matrices [..., 5, 5]."""
    return np.stack([S[..., 0, 0], S[..., 0, 1], S[..., 1, 1]], axis=-1)


def _sqrt_change(x, dx):
    """Bound on |sqrt(x') - sqrt(x)| for |x' - x| <= dx, x >= 0."""
    x = np.maximum(x, 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        lin = np.where(x > 0, dx / np.sqrt(x), np.inf)
    return np.minimum(lin, np.sqrt(dx))


def _lambda_change(sxy, exy):
    """Bound on the change of lambda_max(Sigma_XY) and on its FP32 evaluation."""
    a, b, c = np.abs(sxy[..., 0]), np.abs(sxy[..., 1]), np.abs(sxy[..., 2])
    ea, eb, ec = exy[..., 0], exy[..., 1], exy[..., 2]
    weyl = np.sqrt(ea * ea + ec * ec + 2 * eb * eb)
    return weyl + 8 * U32 * (a + 2 * b + c + ea + 2 * eb + ec)


def _path_extent(pr):
    if pr.path_kind == 0:
        cx, cy, R = pr.circle
        return float(np.hypot(cx, cy) + R)
    return float(np.max(np.hypot(pr.path_pts[:, 0], pr.path_pts[:, 1])))


def _position_change(x_o, x_g):
    P_o, P_g = x_o[1:, :, 0:2], x_g[1:, :, 0:2]
    dp = np.hypot(P_g[..., 0] - P_o[..., 0], P_g[..., 1] - P_o[..., 1])
    return P_o, dp, np.hypot(P_o[..., 0], P_o[..., 1]) + dp


def lane_distance_bound(pr, x_o, x_g, d_lane_o):
    """Bound [T, K] on |d_lane gpu - d_lane oracle| (the distance is 1-Lipschitz in the position)."""
    _, dp, pn = _position_change(x_o, x_g)
    return dp + 8 * U32 * (pn + _path_extent(pr)) + 2 * U32 * d_lane_o


def lane_margin_bound(pr, x_o, x_g, d_lane_o, sxy, exy):
    """Bound [T, K] on |lane margin gpu - lane margin oracle| (Eq. 14: r_bar - d_lane), where
    sxy [T, K, 3] is the oracle's position covariance the margin of step k uses (at k + 1) and
    exy its bound."""
    p = pr.params
    c_p = np.sqrt(C.chi2_2_quantile(p["p_x"]))
    lam = C.lambda_max_2x2(sxy[..., 0], sxy[..., 1], sxy[..., 2])
    dl = _lambda_change(sxy, exy)
    sq = np.sqrt(np.maximum(lam, 0.0))
    d_sqrt = _sqrt_change(lam, dl) + 2 * U32 * sq
    r_round = 2 * U32 * (p["half_width"] + c_p * (sq + d_sqrt))
    return lane_distance_bound(pr, x_o, x_g, d_lane_o) + c_p * d_sqrt + r_round


def obstacle_margin_bound(pr, x_o, x_g, sxy, exy):
    """Bound [T, K] on |min_j d_bar_j (gpu) - min_j d_bar_j (oracle)| (Eq. 16); without obstacles
    both sides report +inf and the bound is 0."""
    p = pr.params
    obs = np.asarray(pr.obstacles, dtype=np.float64)
    T, K = sxy.shape[0], sxy.shape[1]
    if obs.shape[0] == 0:
        return np.zeros((T, K))
    z = C.norm_ppf(p["p_x"])
    P_o, dp, pn = _position_change(x_o, x_g)
    a, b, c = sxy[..., 0], sxy[..., 1], sxy[..., 2]
    lam = np.maximum(C.lambda_max_2x2(a, b, c), 0.0)
    dl = _lambda_change(sxy, exy)
    worst = np.zeros((T, K))
    for j in range(obs.shape[0]):
        dx, dy = P_o[..., 0] - obs[j, 0], P_o[..., 1] - obs[j, 1]
        rho = np.hypot(dx, dy)
        with np.errstate(divide="ignore", invalid="ignore"):
            nx, ny = dx / rho, dy / rho
            var = np.where(rho > 0, a * nx * nx + 2 * b * nx * ny + c * ny * ny, lam)
            dn = np.where(rho > dp, 2 * dp / np.maximum(rho - dp, 1e-300), 2.0)
        var = np.maximum(var, 0.0)
        cn = np.hypot(obs[j, 0], obs[j, 1])
        d_rho = dp + 8 * U32 * (pn + cn + rho)
        # n^T Sigma n moves by ||dSigma||_2 + 2 ||Sigma||_2 |dn|, |dn| <= 2 |dp| / rho
        d_var = dl + 2 * (lam + dl) * np.minimum(dn, 2.0) + 8 * U32 * (np.abs(a) + 2 * np.abs(b) + np.abs(c))
        # at (or within dp of) a centre the GPU may take sqrt(lambda_max) instead of n^T Sigma n
        d_var = np.where(rho > dp, d_var, lam + dl)
        sq = np.sqrt(var)
        d_sig = _sqrt_change(var, d_var) + 4 * U32 * sq
        bound = d_rho + z * d_sig + 2 * U32 * (rho + obs[j, 2] + z * (sq + d_sig))
        worst = np.maximum(worst, bound)
    return worst

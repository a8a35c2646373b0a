"""Chance-constraint tightening (test infrastructure only).

Lane (Eqs. 13-14): the robot must stay within half-width r of the centreline;
with position covariance Sigma_XY the radius is tightened to
    r_bar = r - sqrt(chi2_2(p_x) * lambda_max(Sigma_XY)).
chi2 with two degrees of freedom has the closed-form quantile -2 ln(1 - p).

Obstacles (Eqs. 15-16): circles; d is the signed distance to the circle
boundary, n the unit vector between the robot and the closest boundary point
(for a circle, the radial direction), and the tightened distance is
    d_bar = d - Phi^{-1}(p_x) sqrt(n^T Sigma_XY n),  safe iff d_bar > 0.
Phi^{-1} is computed with Wichura's algorithm AS241 (PPND16, Applied
Statistics 37(3), 1988), accurate to about 1e-16.
"""
from __future__ import annotations

import math

import numpy as np


def chi2_2_quantile(p: float) -> float:
    return -2.0 * math.log1p(-p)


# AS241 PPND16 coefficients (Wichura 1988).
_A = (3.3871328727963666080e0, 1.3314166789178437745e+2, 1.9715909503065514427e+3,
      1.3731693765509461125e+4, 4.5921953931549871457e+4, 6.7265770927008700853e+4,
      3.3430575583588128105e+4, 2.5090809287301226727e+3)
_B = (1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2, 5.3941960214247511077e+3,
      2.1213794301586595867e+4, 3.9307895800092710610e+4, 2.8729085735721942674e+4,
      5.2264952788528545610e+3)
_C = (1.42343711074968357734e0, 4.63033784615654529590e0, 5.76949722146069140550e0,
      3.64784832476320460504e0, 1.27045825245236838258e0, 2.41780725177450611770e-1,
      2.27238449892691845833e-2, 7.74545014278341407640e-4)
_D = (1.0, 2.05319162663775882187e0, 1.67638483018380384940e0, 6.89767334985100004550e-1,
      1.48103976427480074590e-1, 1.51986665636164571966e-2, 5.47593808499534494600e-4,
      1.05075007164441684324e-9)
_E = (6.65790464350110377720e0, 5.46378491116411436990e0, 1.78482653991729133580e0,
      2.96560571828504891230e-1, 2.65321895265761230930e-2, 1.24266094738807843860e-3,
      2.71155556874348757815e-5, 2.01033439929228813265e-7)
_F = (1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1, 1.48753612908506148525e-2,
      7.86869131145613259100e-4, 1.84631831751005468180e-5, 1.42151175831644588870e-7,
      2.04426310338993978564e-15)


def _poly(c, r):
    acc = 0.0
    for coef in reversed(c):
        acc = acc * r + coef
    return acc


def norm_ppf(p: float) -> float:
    """Phi^{-1}(p) for 0 < p < 1 (AS241)."""
    if not 0.0 < p < 1.0:
        raise ValueError("p must lie in (0, 1)")
    q = p - 0.5
    if abs(q) <= 0.425:
        r = 0.180625 - q * q
        return q * _poly(_A, r) / _poly(_B, r)
    r = p if q < 0 else 1.0 - p
    r = math.sqrt(-math.log(r))
    if r <= 5.0:
        r -= 1.6
        val = _poly(_C, r) / _poly(_D, r)
    else:
        r -= 5.0
        val = _poly(_E, r) / _poly(_F, r)
    return -val if q < 0 else val


def lambda_max_2x2(a, b, c):
    """Largest eigenvalue of [[a, b], [b, c]] (closed form)."""
    h = 0.5 * (a - c)
    return 0.5 * (a + c) + np.sqrt(h * h + b * b)


def lane_distance(P, path_kind, circle, pts):
    """Distance from positions P [K, 2] to the centreline.

    circle: | ||p - c|| - R |; polyline: minimum over the closed polyline's
    segments of the point-to-segment distance.
    """
    if path_kind == 0:
        cx, cy, R = circle
        return np.abs(np.hypot(P[:, 0] - cx, P[:, 1] - cy) - R)
    a = np.asarray(pts, dtype=np.float64)
    b = np.roll(a, -1, axis=0)
    best = np.full(P.shape[0], np.inf)
    for i in range(a.shape[0]):
        e = b[i] - a[i]
        rel = P - a[i]
        t = np.clip((rel @ e) / (e @ e), 0.0, 1.0)
        d = rel - t[:, None] * e[None, :]
        best = np.minimum(best, np.einsum("ij,ij->i", d, d))
    return np.sqrt(best)


def tightened_lane_radius(r, Sxy, p_x):
    """Eq. (14): r_bar = r - sqrt(chi2_2(p_x) lambda_max(Sigma_XY)).  Sxy = (a, b, c)."""
    lam = lambda_max_2x2(Sxy[..., 0], Sxy[..., 1], Sxy[..., 2])
    return r - np.sqrt(chi2_2_quantile(p_x) * lam)


def obstacle_margins(P, Sxy, obstacles, p_x):
    """Eqs. (15)-(16) for every obstacle: d_bar [K, n].

    n = (p - c)/||p - c||; where p coincides with a centre the direction is
    undefined and sqrt(lambda_max) (the largest directional sigma) is used.
    """
    z = norm_ppf(p_x)
    K, n = P.shape[0], obstacles.shape[0]
    out = np.empty((K, n))
    a, b, c = Sxy[:, 0], Sxy[:, 1], Sxy[:, 2]
    lam = lambda_max_2x2(a, b, c)
    for j in range(n):
        dx = P[:, 0] - obstacles[j, 0]
        dy = P[:, 1] - obstacles[j, 1]
        rho = np.hypot(dx, dy)
        d = rho - obstacles[j, 2]
        with np.errstate(invalid="ignore", divide="ignore"):
            nx, ny = dx / rho, dy / rho
            var = a * nx * nx + 2.0 * b * nx * ny + c * ny * ny
        var = np.where(rho > 0.0, var, lam)
        out[:, j] = d - z * np.sqrt(np.maximum(var, 0.0))
    return out

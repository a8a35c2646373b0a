"""Exact GP regression for the velocity residuals (test infrastructure only).

Sec. III-A trains one GP per velocity output on the residual between measured
and nominal velocities; Sec. V-A gives its input (v, w, v_cmd, w_cmd) and a
GPyTorch batch GP.  Eq. (3) uses each GP's predictive mean and covariance.

The oracle follows Rasmussen & Williams, "Gaussian Processes for Machine
Learning", Algorithm 2.1, with the squared-exponential ARD covariance
    k(a, b) = sf^2 exp(-1/2 sum_d (a_d - b_d)^2 / ell_d^2):
    L = cholesky(K(Z, Z) + sn^2 I)
    alpha = L^T \\ (L \\ y)
    mean(q) = k(q, Z) alpha
    v = L \\ k(Z, q);  latent var = k(q, q) - v^T v
The predictive variance of the residual is sn^2 + max(0, latent var): the
latent part cannot be negative, so the variance never drops below the noise
floor sn^2.  W = L^{-1} is never formed here.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def se_ard(A, B, log_ell, log_sf):
    """k(a_i, b_j) for rows of A [n, d] and B [m, d] -> [n, m]."""
    ell = np.exp(np.asarray(log_ell, dtype=np.float64))
    sf2 = np.exp(2.0 * float(log_sf))
    d2 = np.zeros((A.shape[0], B.shape[0]))
    for d in range(A.shape[1]):
        diff = (A[:, d][:, None] - B[:, d][None, :]) / ell[d]
        d2 += diff * diff
    return sf2 * np.exp(-0.5 * d2)


class ExactGP:
    """One output's GP posterior (Rasmussen & Williams Alg. 2.1)."""

    def __init__(self, Z, y, log_ell, log_sf, log_sn):
        self.Z = np.asarray(Z, dtype=np.float64)
        self.y = np.asarray(y, dtype=np.float64)
        self.log_ell = np.asarray(log_ell, dtype=np.float64)
        self.log_sf = float(log_sf)
        self.log_sn = float(log_sn)
        self.sf2 = np.exp(2.0 * self.log_sf)
        self.sn2 = np.exp(2.0 * self.log_sn)
        A = se_ard(self.Z, self.Z, self.log_ell, self.log_sf) + self.sn2 * np.eye(len(self.Z))
        self.L = np.linalg.cholesky(A)   # raises LinAlgError when A is not positive definite
        self.alpha = sla.solve_triangular(self.L.T, sla.solve_triangular(self.L, self.y, lower=True),
                                          lower=False)

    def predict(self, Q):
        """Q [n, 4] -> (mean [n], latent variance [n], predictive variance [n])."""
        Q = np.asarray(Q, dtype=np.float64)
        Ks = se_ard(self.Z, Q, self.log_ell, self.log_sf)          # [M, n]
        mean = Ks.T @ self.alpha
        v = sla.solve_triangular(self.L, Ks, lower=True)           # [M, n]
        latent = self.sf2 - np.sum(v * v, axis=0)                  # k(q, q) = sf^2
        pred = self.sn2 + np.maximum(0.0, latent)
        return mean, latent, pred


def build_pair(Z, y, log_ell, log_sf, log_sn):
    """The two residual GPs (linear and angular velocity)."""
    return [ExactGP(Z[o], y[o], log_ell[o], log_sf[o], log_sn[o]) for o in range(2)]


def ensemble_predict(terrain_gps, weights, Q):
    """Eq. (3): the weighted terrain ensemble of the residual GPs.

    terrain_gps[i][o] is the GP of terrain i and output o.  Returns the mean
    sum_i w_i m_i [n, 2] and the diagonal of sum_i w_i^2 C_i [n, 2], with C_i
    each terrain's predictive covariance (its diagonal; the outputs are
    independent GPs)."""
    Q = np.asarray(Q, dtype=np.float64)
    mean = np.zeros((Q.shape[0], 2))
    var = np.zeros((Q.shape[0], 2))
    for w, gps in zip(weights, terrain_gps):
        for o in range(2):
            m, _, s2 = gps[o].predict(Q)
            mean[:, o] += w * m
            var[:, o] += w * w * s2
    return mean, var


def build_terrains(Z, terrain_y, log_ell, log_sf, log_sn):
    """One GP pair per terrain target set terrain_y [n_terr, 2, M]."""
    return [build_pair(Z, y, log_ell, log_sf, log_sn) for y in terrain_y]

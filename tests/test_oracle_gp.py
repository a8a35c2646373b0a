"""Pins for the oracle's GP regression (Sec. III-A, Eq. 3; R&W Alg. 2.1)."""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import gp as G
from paper_2411_03289_amd import workloads as W


def _fit(M=30, seed=3, ell=(1.0, 0.7, 1.3, 2.0), sf=0.5, sn=0.05):
    pr = W.small_problem(M=M, seed_data=seed)
    log_ell = np.log(np.array(ell))
    g = G.ExactGP(pr.Z[0], pr.y[0], log_ell, math.log(sf), math.log(sn))
    return pr, g


def test_se_ard_matches_scaled_sqeuclidean():
    rng = np.random.Generator(np.random.PCG64(1))
    A, B = rng.normal(size=(7, 4)), rng.normal(size=(5, 4))
    ell = np.array([0.5, 1.0, 2.0, 3.0])
    ref = 0.3 ** 2 * np.exp(-0.5 * cdist(A / ell, B / ell, "sqeuclidean"))
    np.testing.assert_allclose(G.se_ard(A, B, np.log(ell), math.log(0.3)), ref, rtol=1e-14)


def test_posterior_matches_dense_direct_solve():
    pr, g = _fit(M=50)
    Q = W.random_queries(200, 5)
    Kzz = G.se_ard(g.Z, g.Z, g.log_ell, g.log_sf)
    A = Kzz + g.sn2 * np.eye(len(g.Z))
    Ks = G.se_ard(Q, g.Z, g.log_ell, g.log_sf)
    mean_ref = Ks @ np.linalg.solve(A, g.y)
    var_ref = g.sf2 - np.einsum("ij,ji->i", Ks, np.linalg.solve(A, Ks.T))
    mean, latent, pred = g.predict(Q)
    np.testing.assert_allclose(mean, mean_ref, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(latent, var_ref, rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(pred, g.sn2 + np.maximum(var_ref, 0), rtol=1e-8, atol=1e-12)


def test_posterior_matches_sklearn_regressor():
    sk = pytest.importorskip("sklearn.gaussian_process")
    from sklearn.gaussian_process.kernels import RBF, ConstantKernel, WhiteKernel
    pr, g = _fit(M=40, seed=9)
    ell = np.exp(g.log_ell)
    kern = (ConstantKernel(g.sf2, "fixed") * RBF(ell, "fixed") + WhiteKernel(g.sn2, "fixed"))
    reg = sk.GaussianProcessRegressor(kern, alpha=1e-300, optimizer=None).fit(g.Z, g.y)
    Q = W.random_queries(100, 6)
    m_ref, sd_ref = reg.predict(Q, return_std=True)
    mean, _, pred = g.predict(Q)
    np.testing.assert_allclose(mean, m_ref, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(pred, sd_ref ** 2, rtol=1e-8, atol=1e-12)


def test_single_point_closed_form():
    z = np.array([[0.3, -0.2, 1.0, 0.5]])
    y = np.array([0.7])
    sf, sn = 0.5, 0.05
    g = G.ExactGP(z, y, np.zeros(4), math.log(sf), math.log(sn))
    q = np.array([[0.1, 0.4, 0.0, 1.5]])
    r2 = float(np.sum((q - z) ** 2))
    kq = sf**2 * math.exp(-0.5 * r2)
    mean, latent, pred = g.predict(q)
    assert mean[0] == pytest.approx(kq * y[0] / (sf**2 + sn**2), rel=1e-14)
    assert latent[0] == pytest.approx(sf**2 - kq**2 / (sf**2 + sn**2), rel=1e-13)


def test_variance_floor_training_points_and_prior_far_away():
    pr, g = _fit(M=50, seed=4)
    Q = W.random_queries(500, 8, lo=-3, hi=3)
    _, _, pred = g.predict(Q)
    assert np.all(pred >= g.sn2)
    _, latent, pred = g.predict(g.Z)
    bound = g.sn2 + g.sf2 * g.sn2 / (g.sf2 + g.sn2)
    assert np.all(pred <= bound * (1 + 1e-9))
    far = g.Z[:5] + 60.0
    mean, latent, pred = g.predict(far)
    np.testing.assert_allclose(mean, 0.0, atol=1e-300)
    np.testing.assert_allclose(pred, g.sf2 + g.sn2, rtol=1e-15)


def test_zero_targets_give_zero_mean():
    pr = W.small_problem(M=20, seed_data=2)
    g = G.ExactGP(pr.Z[1], np.zeros(20), pr.log_ell[1], pr.log_sf[1], pr.log_sn[1])
    mean, _, _ = g.predict(W.random_queries(50, 1))
    np.testing.assert_array_equal(mean, 0.0)


def test_not_positive_definite_raises():
    Z = np.zeros((3, 4))   # identical inputs
    with pytest.raises(np.linalg.LinAlgError):
        G.ExactGP(Z, np.zeros(3), np.zeros(4), 0.0, -400.0)   # sn = e^-400 underflows to 0


def test_ensemble_reduces_to_single_terrain_and_scales_variance():
    pr = W.add_terrains(W.small_problem(M=30, seed_data=12), seed=5)
    tg = G.build_terrains(pr.Z, pr.terrain_y, pr.log_ell, pr.log_sf, pr.log_sn)
    Q = W.random_queries(80, 13)
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        m, v = G.ensemble_predict(tg, e, Q)
        for o in range(2):
            mi, _, vi = tg[i][o].predict(Q)
            np.testing.assert_array_equal(m[:, o], mi)
            np.testing.assert_array_equal(v[:, o], vi)
    # shared inputs and hyperparameters: each terrain has the same covariance,
    # so the ensemble variance is (sum w^2) times it, and the mean is linear in w
    w = np.array([0.5, 0.3, 0.2])
    m, v = G.ensemble_predict(tg, w, Q)
    for o in range(2):
        _, _, v0 = tg[0][o].predict(Q)
        np.testing.assert_allclose(v[:, o], np.sum(w**2) * v0, rtol=1e-12)
        ref = sum(w[i] * tg[i][o].predict(Q)[0] for i in range(3))
        np.testing.assert_allclose(m[:, o], ref, rtol=1e-12, atol=1e-15)
        # alpha of the weighted targets = weighted alphas (the GP mean is linear in y)
        gw = G.ExactGP(pr.Z[o], np.tensordot(w, pr.terrain_y[:, o], 1), pr.log_ell[o], pr.log_sf[o], pr.log_sn[o])
        np.testing.assert_allclose(gw.predict(Q)[0], m[:, o], rtol=1e-10, atol=1e-13)

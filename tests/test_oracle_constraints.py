"""Pins for the oracle's chance-constraint tightening (Eqs. 13-16)."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import constraints as C
from paper_2411_03289_amd import workloads as W


def test_quantiles_match_scipy():
    for p in (0.5, 0.9, 0.95, 0.99, 0.999):
        assert C.chi2_2_quantile(p) == pytest.approx(stats.chi2.ppf(p, 2), rel=1e-14)
    ps = np.concatenate([np.linspace(1e-6, 1 - 1e-6, 2001), [1e-12, 1e-20, 0.425 + 0.5, 0.075]])
    for p in ps:
        ref = stats.norm.ppf(p)
        assert C.norm_ppf(p) == pytest.approx(ref, rel=2e-14, abs=1e-14)
    assert C.norm_ppf(0.95) == pytest.approx(1.6448536269514722, rel=1e-15)
    assert math.sqrt(C.chi2_2_quantile(0.95)) == pytest.approx(2.4477468306808161, rel=1e-15)


def test_lambda_max_matches_eigvalsh():
    rng = np.random.Generator(np.random.PCG64(4))
    L = rng.normal(size=(500, 2, 2))
    S = L @ np.transpose(L, (0, 2, 1))
    ref = np.linalg.eigvalsh(S)[:, 1]
    got = C.lambda_max_2x2(S[:, 0, 0], S[:, 0, 1], S[:, 1, 1])
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    assert C.lambda_max_2x2(2.0, 0.0, 2.0) == 2.0   # repeated eigenvalue


def test_obstacle_margin_special_cases():
    obs = np.array([[1.0, 2.0, 0.5], [-3.0, 0.0, 1.0]])
    P = np.array([[1.0, 4.0], [0.0, 0.0], [1.0, 2.0]])
    zero = np.zeros((3, 3))
    d = C.obstacle_margins(P, zero, obs, 0.95)
    ref = np.hypot(P[:, None, 0] - obs[None, :, 0], P[:, None, 1] - obs[None, :, 1]) - obs[None, :, 2]
    np.testing.assert_allclose(d, ref, rtol=1e-15)
    sig = 0.3
    iso = np.tile([sig**2, 0.0, sig**2], (3, 1))
    z = C.norm_ppf(0.95)
    np.testing.assert_allclose(C.obstacle_margins(P, iso, obs, 0.95), ref - z * sig, rtol=1e-14)
    # directional variance: Sigma = diag(a, c) seen along x is sqrt(a)
    aniso = np.tile([0.04, 0.0, 0.25], (1, 1))
    d = C.obstacle_margins(np.array([[3.0, 0.0]]), aniso, np.array([[0.0, 0.0, 1.0]]), 0.95)
    assert d[0, 0] == pytest.approx(2.0 - z * 0.2, rel=1e-14)
    # robot exactly on the centre: largest directional sigma
    d = C.obstacle_margins(np.array([[0.0, 0.0]]), aniso, np.array([[0.0, 0.0, 1.0]]), 0.95)
    assert d[0, 0] == pytest.approx(-1.0 - z * 0.5, rel=1e-14)


def test_lane_radius_special_cases():
    iso = np.array([[0.09, 0.0, 0.09]])
    assert C.tightened_lane_radius(1.0, iso, 0.95)[0] == pytest.approx(1.0 - 2.4477468306808161 * 0.3, rel=1e-14)
    assert C.tightened_lane_radius(1.0, np.zeros((1, 3)), 0.95)[0] == 1.0


def test_tightening_probabilities_by_monte_carlo():
    # Eq. 16: a Gaussian position crosses the tightened half-plane with prob. 1 - p_x.
    rng = np.random.Generator(np.random.PCG64(12))
    n = 400_000
    Sxy = np.array([[0.05, 0.02], [0.02, 0.03]])
    pts = rng.multivariate_normal([0, 0], Sxy, size=n)
    nvec = np.array([0.6, 0.8])
    z = C.norm_ppf(0.95)
    sd = math.sqrt(nvec @ Sxy @ nvec)
    frac = np.mean(pts @ nvec > z * sd)
    assert frac == pytest.approx(0.05, abs=4 * math.sqrt(0.05 * 0.95 / n))
    # Eq. 14 with an isotropic covariance: the chi2_2 disc holds mass p_x.
    iso = rng.normal(0, 0.2, size=(n, 2))
    rad = math.sqrt(C.chi2_2_quantile(0.95) * 0.04)
    assert np.mean(np.hypot(*iso.T) <= rad) == pytest.approx(0.95, abs=4 * math.sqrt(0.05 * 0.95 / n))


def test_lane_distance_circle_and_polyline():
    rng = np.random.Generator(np.random.PCG64(3))
    P = rng.uniform(-8, 8, size=(300, 2))
    exact = C.lane_distance(P, 0, (0.0, 0.0, 5.0), None)
    np.testing.assert_allclose(exact, np.abs(np.hypot(*P.T) - 5.0), rtol=1e-15)
    Pn = 1024
    poly = C.lane_distance(P, 1, None, W.circle_polyline(5.0, Pn))
    sagitta = 5.0 * (1 - math.cos(math.pi / Pn))
    assert np.all(np.abs(poly - exact) <= sagitta + 1e-12)


def test_polyline_distance_brute_force():
    rng = np.random.Generator(np.random.PCG64(8))
    pts = W.figure_eight(8.0, 64)
    P = rng.uniform(-9, 9, size=(200, 2))
    got = C.lane_distance(P, 1, None, pts)
    t = np.linspace(0, 1, 2001)
    a, b = pts, np.roll(pts, -1, axis=0)
    dense = (a[:, None, :] + t[None, :, None] * (b - a)[:, None, :]).reshape(-1, 2)
    brute = np.min(np.hypot(P[:, None, 0] - dense[None, :, 0], P[:, None, 1] - dense[None, :, 1]), axis=1)
    seg = np.max(np.hypot(*(b - a).T)) / 2000
    assert np.all(got <= brute + 1e-12)
    assert np.all(brute - got <= seg)

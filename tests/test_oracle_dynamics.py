"""Pins for the oracle's dynamics and covariance propagation (Eqs. 1, 2, 10)."""
import math

import numpy as np
import pytest

from oracle import dynamics as D

DT, TV, TW = 0.05, 0.2, 0.1


def _run(x0, u, steps, m=None):
    x = np.atleast_2d(np.asarray(x0, float))
    xs = [x[0].copy()]
    for _ in range(steps):
        x = D.euler_step(x, np.atleast_2d(u), np.zeros((1, 2)) if m is None else np.atleast_2d(m),
                         DT, TV, TW)
        xs.append(x[0].copy())
    return np.array(xs)


@pytest.mark.parametrize("w", [0.2, -1.25, 1e-3])
def test_constant_turn_closed_form(w):
    # command = current velocities, GP zeroed: v, w stay constant and the Euler
    # positions are the vertices of a regular polygon inscribed in a circle.
    x0 = np.array([5.0, 0.0, math.pi / 2, 1.0, w])
    xs = _run(x0, [1.0, w], 60)
    phi = w * DT
    k = np.arange(61)
    chord = 1.0 * DT * np.sin(k * phi / 2) / np.sin(phi / 2)
    ang = x0[2] + (k - 1) * phi / 2
    np.testing.assert_allclose(xs[:, 0], x0[0] + chord * np.cos(ang), atol=1e-12)
    np.testing.assert_allclose(xs[:, 1], x0[1] + chord * np.sin(ang), atol=1e-12)
    np.testing.assert_allclose(xs[:, 2], x0[2] + k * phi, atol=1e-12)
    R = 1.0 * DT / (2 * np.sin(phi / 2))
    centre = x0[:2] + R * np.array([np.cos(x0[2] + math.pi / 2 - phi / 2),
                                    np.sin(x0[2] + math.pi / 2 - phi / 2)])
    np.testing.assert_allclose(np.hypot(*(xs[:, :2] - centre).T), abs(R), rtol=1e-12)


def test_straight_line():
    x0 = np.array([1.0, -2.0, 0.3, 1.5, 0.0])
    xs = _run(x0, [1.5, 0.0], 40)
    k = np.arange(41)
    np.testing.assert_allclose(xs[:, 0], 1.0 + k * 1.5 * DT * math.cos(0.3), atol=1e-13)
    np.testing.assert_allclose(xs[:, 1], -2.0 + k * 1.5 * DT * math.sin(0.3), atol=1e-13)


def test_first_order_lag_and_gp_residual():
    xs = _run([0, 0, 0, 0.5, -1.0], [1.8, 0.7], 30)
    k = np.arange(31)
    np.testing.assert_allclose(xs[:, 3], 1.8 + (0.5 - 1.8) * (1 - DT / TV) ** k, rtol=1e-13)
    np.testing.assert_allclose(xs[:, 4], 0.7 + (-1.0 - 0.7) * (1 - DT / TW) ** k, rtol=1e-12)
    # a constant GP mean m acts as an extra acceleration: fixed point u + tau m
    xs = _run([0, 0, 0, 0.0, 0.0], [1.0, 0.0], 400, m=[0.3, -0.2])
    assert xs[-1, 3] == pytest.approx(1.0 + TV * 0.3, rel=1e-10)
    assert xs[-1, 4] == pytest.approx(0.0 + TW * -0.2, abs=1e-10)


def test_jacobian_matches_central_differences():
    rng = np.random.Generator(np.random.PCG64(2))
    x = rng.normal(size=(6, 5))
    u = rng.normal(size=(6, 2))
    A = D.nominal_jacobian(x, DT, TV, TW)
    h = 1e-6
    for i in range(5):
        e = np.zeros(5)
        e[i] = h
        fp = D.euler_step(x + e, u, np.zeros((6, 2)), DT, TV, TW)
        fm = D.euler_step(x - e, u, np.zeros((6, 2)), DT, TV, TW)
        np.testing.assert_allclose(A[:, :, i], (fp - fm) / (2 * h), atol=1e-9)


def test_covariance_structure_and_velocity_closed_form():
    rng = np.random.Generator(np.random.PCG64(5))
    K = 8
    x = np.tile([0.0, 0.0, 0.4, 1.2, 0.3], (K, 1))
    S = np.zeros((K, 5, 5))
    s2 = np.array([0.04, 0.09])
    u = rng.uniform(-1, 1, size=(K, 2))
    for k in range(1, 31):
        A = D.nominal_jacobian(x, DT, TV, TW)
        x = D.euler_step(x, u, np.zeros((K, 2)), DT, TV, TW)
        S = D.covariance_step(S, A, np.tile(s2, (K, 1)), DT)
        if k == 1:
            np.testing.assert_array_equal(S[:, :3, :3], 0.0)
        np.testing.assert_allclose(S, np.transpose(S, (0, 2, 1)), rtol=0, atol=1e-14 * np.abs(S).max())
        assert np.all(np.linalg.eigvalsh(S) > -1e-15)
        np.testing.assert_array_equal(S[:, 2, 3], 0.0)   # Sigma_theta,v
        np.testing.assert_array_equal(S[:, 3, 4], 0.0)   # Sigma_v,w
        for i, (tau, var) in enumerate(((TV, s2[0]), (TW, s2[1]))):
            a = 1 - DT / tau
            np.testing.assert_allclose(S[:, 3 + i, 3 + i], DT**2 * var * (1 - a ** (2 * k)) / (1 - a * a),
                                       rtol=1e-12)


def test_covariance_matches_monte_carlo_of_linearised_noise():
    # With small velocity noise, the spread of noisy Euler rollouts approaches
    # the first-order propagated covariance (Eq. 10).
    rng = np.random.Generator(np.random.PCG64(9))
    n, steps, sd = 200_000, 20, 1e-3
    x = np.tile([0.0, 0.0, 0.4, 1.2, 0.8], (n, 1))
    xm = x[:1].copy()
    S = np.zeros((1, 5, 5))
    u = np.array([[1.5, -0.5]])
    for _ in range(steps):
        A = D.nominal_jacobian(xm, DT, TV, TW)
        xm = D.euler_step(xm, u, np.zeros((1, 2)), DT, TV, TW)
        S = D.covariance_step(S, A, np.array([[sd**2, sd**2]]), DT)
        m = rng.normal(0.0, sd, size=(n, 2))
        x = D.euler_step(x, np.tile(u, (n, 1)), m, DT, TV, TW)
    C = np.cov(x.T)
    scale = np.sqrt(np.outer(np.diag(S[0]), np.diag(S[0])))
    np.testing.assert_allclose(C / scale, S[0] / scale, atol=0.02)


def test_plant_is_nominal_plus_residual():
    x = np.array([1.0, 2.0, 0.1, 1.1, -0.7])
    u = np.array([1.5, 0.2])
    nom = D.euler_step(x[None], u[None], np.zeros((1, 2)), DT, TV, TW)[0]
    pl = D.plant_step(x, u, DT, TV, TW, amplitude=0.3)[0]
    r = 0.3 * math.sin(1.1 * -0.7)
    np.testing.assert_allclose(pl - nom, [0, 0, 0, DT * r, DT * r], atol=1e-15)

"""Pins for the terrain-weight estimate of Eq. (4) (Alg. 1, Step 3)."""
import itertools

import numpy as np
import pytest

from oracle import terrain as TR


def _case(seed, H=20, n=3, true=(0.7, 0.2, 0.1), noise=0.02):
    rng = np.random.Generator(np.random.PCG64(seed))
    Fv = rng.normal(size=(H, n))
    Fw = rng.normal(size=(H, n))
    w_true = np.asarray(true[:n])
    Yv = Fv @ w_true + noise * rng.normal(size=H)
    Yw = Fw @ w_true + noise * rng.normal(size=H)
    return Yv, Yw, Fv, Fw, w_true


def _grid(n, step):
    ticks = np.arange(0, 1 + 1e-12, step)
    for c in itertools.product(ticks, repeat=n - 1):
        s = sum(c)
        if s <= 1 + 1e-12:
            yield np.array(list(c) + [1 - s])


@pytest.mark.parametrize("gamma", [0.0, 0.05, 0.5, 5.0])
def test_qp_solution_beats_a_fine_simplex_grid(gamma):
    Yv, Yw, Fv, Fw, _ = _case(1)
    w_prev = np.array([0.2, 0.5, 0.3])
    w = TR.solve_weights(Yv, Yw, Fv, Fw, w_prev, gamma)
    assert np.all(w >= -1e-12) and np.all(w <= 1 + 1e-12) and abs(w.sum() - 1) < 1e-12
    f = TR.objective(w, Yv, Yw, Fv, Fw, w_prev, gamma)
    grid = min(TR.objective(g, Yv, Yw, Fv, Fw, w_prev, gamma) for g in _grid(3, 0.0025))
    assert f <= grid + 1e-12
    # no small feasible move improves it (first-order optimality)
    rng = np.random.Generator(np.random.PCG64(2))
    for _ in range(2000):
        d = rng.normal(size=3)
        d -= d.mean()
        t = 1e-5
        w2 = w + t * d
        if np.all(w2 >= 0) and np.all(w2 <= 1):
            assert TR.objective(w2, Yv, Yw, Fv, Fw, w_prev, gamma) >= f - 1e-12


def test_recovers_the_generating_terrain_without_regularisation():
    Yv, Yw, Fv, Fw, w_true = _case(3, H=200, noise=0.0)
    w = TR.solve_weights(Yv, Yw, Fv, Fw, np.full(3, 1 / 3), 0.0)
    np.testing.assert_allclose(w, w_true, atol=1e-7)


def test_large_gamma_keeps_the_previous_weights():
    Yv, Yw, Fv, Fw, _ = _case(4)
    w_prev = np.array([0.1, 0.1, 0.8])
    w = TR.solve_weights(Yv, Yw, Fv, Fw, w_prev, 1e6)
    np.testing.assert_allclose(w, w_prev, atol=1e-9)


@pytest.mark.parametrize("seed,gamma,n", [(11, 0.0, 3), (12, 0.1, 3), (13, 2.0, 3), (14, 0.3, 5), (15, 0.05, 2),
                                          (16, 0.0, 1)])
def test_library_qp_matches_oracle(seed, gamma, n):
    import os
    from paper_2411_03289_amd import gpmppi as B
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libgpmppi.so not built")
    true = (0.5, 0.2, 0.1, 0.15, 0.05)
    Yv, Yw, Fv, Fw, _ = _case(seed, H=30, n=n, true=true[:n] if n > 1 else (1.0,), noise=0.05)
    rng = np.random.Generator(np.random.PCG64(seed + 100))
    w_prev = rng.dirichlet(np.ones(n))
    w_lib = B.gpmppi_terrain_weights(Yv, Yw, Fv, Fw, w_prev, gamma)
    w_or = TR.solve_weights(Yv, Yw, Fv, Fw, w_prev, gamma)
    f_lib = TR.objective(w_lib, Yv, Yw, Fv, Fw, w_prev, gamma)
    f_or = TR.objective(w_or, Yv, Yw, Fv, Fw, w_prev, gamma)
    assert abs(w_lib.sum() - 1) < 1e-12 and np.all(w_lib >= 0)
    assert f_lib <= f_or + 1e-10
    np.testing.assert_allclose(w_lib, w_or, atol=2e-6)

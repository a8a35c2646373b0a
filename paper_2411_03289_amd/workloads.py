"""Seeded synthetic workloads for the GP-MPPI rollout.

This module only draws inputs: GP training sets, obstacle fields, reference
paths, start states, nominal control sequences and a few generic random
arrays used by unit tests.  It contains none of the controller's arithmetic
(no GP algebra, no dynamics, no costs), so that both the HIP path and the
FP64 oracle can be fed from it without sharing code.

The workloads stand in for the paper's data, which is not available: the GP
in the paper is trained on 300 shared points with 4-d inputs (current v, w and
commanded v, w) and residual velocity outputs (Sec. V-A), obstacles are
circles (Sec. IV-C, Eqs. 15-16) and the tracks are circles and closed curves
driven at 2 m/s (Sec. V-A).

All draws use numpy's PCG64 with an explicit seed, in a fixed order:
  1. for output o in (v, w): Z_o ~ U[-2, 2]^(N x 4), then e_o ~ N(0, 0.05^2)^N;
     y_o = 0.3 sin(Z_o[:,0] * Z_o[:,1]) + e_o; the GP uses the first M rows.
  2. obstacle centres ~ U[-a, a]^(n x 2), then radii ~ U[r_lo, r_hi]^n.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# Controller defaults (readings of quantities the paper names without values).
DEFAULT_PARAMS = dict(
    dt=0.05, tau_v=0.2, tau_w=0.1,          # first-order velocity lags
    sig_v=0.5, sig_w=0.8,                   # Sigma_sim = diag(sig_v^2, sig_w^2)
    u_min=(-2.0, -2.0), u_max=(2.0, 2.0),   # control box, Eq. (8)
    lam=1.0, p_x=0.95,                      # MPPI temperature, chance level
    w_var=1.0, w_dev=0.5, w_lane=1.0, w_speed=0.1, w_obs=1.0,
    v_des=2.0, discount=0.9, half_width=1.0,
    w_goal=0.0, w_term=0.0, goal=(0.0, 0.0), goal_tol=0.5,   # goal terms of Eq. (12), off by default
    tighten=0,                                               # 1: tighten along the nominal sequence
)


def task_params(task: str, goal=(8.0, 0.0)) -> dict:
    """Weight presets switching between the paper's two tasks (Sec. IV-B):
    path tracking (Eq. 11 terms) or obstacle avoidance towards a goal (Eq. 12)."""
    if task == "track":
        return dict(w_var=1.0, w_dev=0.5, w_lane=1.0, w_speed=0.1, w_obs=0.0, w_goal=0.0, w_term=0.0)
    if task == "avoid":
        return dict(w_var=1.0, w_dev=0.0, w_lane=0.0, w_speed=0.0, w_obs=1.0, w_goal=0.2, w_term=1.0,
                    goal=tuple(goal), goal_tol=0.5)
    raise ValueError(task)

RESIDUAL_AMPLITUDE = 0.3   # synthetic residual 0.3 sin(v w) (also the plant's)
TARGET_NOISE = 0.05


@dataclasses.dataclass
class Problem:
    """One MPC problem instance (all float64 host arrays)."""
    K: int
    T: int
    Z: np.ndarray          # [2, M, 4] GP inputs per output (v, w)
    y: np.ndarray          # [2, M]    GP targets per output
    log_ell: np.ndarray    # [2, 4]
    log_sf: np.ndarray     # [2]
    log_sn: np.ndarray     # [2]
    obstacles: np.ndarray  # [n, 3] (cx, cy, r)
    path_kind: int         # 0 = circle, 1 = closed polyline
    circle: tuple          # (cx, cy, R) when path_kind == 0
    path_pts: np.ndarray   # [P, 2] polyline vertices when path_kind == 1
    x0: np.ndarray         # [5] (X, Y, theta, v, w)
    U0: np.ndarray         # [T, 2] nominal control sequence
    seed: int              # 64-bit Philox key of the first iteration
    pid: int = 0           # problem id (Philox counter word 2)
    params: dict = dataclasses.field(default_factory=lambda: dict(DEFAULT_PARAMS))
    name: str = ""
    terrain_y: Optional[np.ndarray] = None   # [n_terr, 2, M] per-terrain targets on the shared inputs Z
    terrain_w: Optional[np.ndarray] = None   # [n_terr] ensemble weights

    @property
    def M(self) -> int:
        return int(self.Z.shape[1])

    def seed_at(self, t: int) -> int:
        """Philox key for closed-loop step t: high word fixed, low word t."""
        return int(self.seed + t)


def _gp_data(rng: np.random.Generator, N: int, M: int):
    Z = np.empty((2, M, 4))
    y = np.empty((2, M))
    for o in range(2):
        Zo = rng.uniform(-2.0, 2.0, size=(N, 4))
        eo = rng.normal(0.0, TARGET_NOISE, size=N)
        yo = RESIDUAL_AMPLITUDE * np.sin(Zo[:, 0] * Zo[:, 1]) + eo
        Z[o] = Zo[:M]
        y[o] = yo[:M]
    return Z, y


def _obstacles(rng: np.random.Generator, n: int, half_extent: float, r_lo: float, r_hi: float):
    c = rng.uniform(-half_extent, half_extent, size=(n, 2))
    r = rng.uniform(r_lo, r_hi, size=n)
    return np.concatenate([c, r[:, None]], axis=1) if n else np.zeros((0, 3))


def figure_eight(A: float = 8.0, P: int = 256) -> np.ndarray:
    """Closed Gerono lemniscate x = A sin s, y = A sin s cos s at s_i = 2 pi i / P."""
    s = 2.0 * np.pi * np.arange(P) / P
    return np.stack([A * np.sin(s), A * np.sin(s) * np.cos(s)], axis=1)


def circle_polyline(R: float, P: int, cx: float = 0.0, cy: float = 0.0) -> np.ndarray:
    s = 2.0 * np.pi * np.arange(P) / P
    return np.stack([cx + R * np.cos(s), cy + R * np.sin(s)], axis=1)


def _hyper(M_dims=4, ell=1.0, sf=0.5, sn=0.05):
    log_ell = np.full((2, M_dims), math.log(ell))
    log_sf = np.full(2, math.log(sf))
    log_sn = np.full(2, math.log(sn))
    return log_ell, log_sf, log_sn


# Start on the figure-eight at s = 0, heading along its tangent (8, 8).
_F8_START = np.array([0.0, 0.0, math.atan2(8.0, 8.0), 1.0, 0.0])
_C0_START = np.array([5.0, 0.0, math.pi / 2.0, 1.0, 0.2])


def make_config(c: int, **over) -> Problem:
    """Workload `c`:
    0: K=256,  T=20,  M=N=50,  5 obstacles (r 0.3-0.6, [-6,6]^2), circle R=5.
    1: K=4096, T=50,  M=256 of N=2000, 20 obstacles (r 0.2-0.8, [-10,10]^2), figure-eight A=8.
    2: K=16384, T=100, M=1024 of N=2000, 50 obstacles, figure-eight A=8.
    4: K=4096, T=50,  M=512 of N=2000, 20 obstacles, figure-eight A=8.
    Keyword overrides: K, T, M, N, n_obs, path ('circle' | 'eight'), seed_data.
    """
    spec = {
        0: dict(K=256, T=20, M=50, N=50, n_obs=5, ext=6.0, r=(0.3, 0.6), path="circle"),
        1: dict(K=4096, T=50, M=256, N=2000, n_obs=20, ext=10.0, r=(0.2, 0.8), path="eight"),
        2: dict(K=16384, T=100, M=1024, N=2000, n_obs=50, ext=10.0, r=(0.2, 0.8), path="eight"),
        4: dict(K=4096, T=50, M=512, N=2000, n_obs=20, ext=10.0, r=(0.2, 0.8), path="eight"),
    }[c]
    spec.update({k: v for k, v in over.items() if k in ("K", "T", "M", "N", "n_obs", "path")})
    if spec["N"] < spec["M"]:
        spec["N"] = spec["M"]
    rng = np.random.Generator(np.random.PCG64(over.get("seed_data", 1000 + c)))
    Z, y = _gp_data(rng, spec["N"], spec["M"])
    obs = _obstacles(rng, spec["n_obs"], spec["ext"], *spec["r"])
    log_ell, log_sf, log_sn = _hyper()
    if spec["path"] == "circle":
        kind, circ, pts, x0 = 0, (0.0, 0.0, 5.0), np.zeros((0, 2)), _C0_START.copy()
    else:
        kind, circ, pts, x0 = 1, (0.0, 0.0, 0.0), figure_eight(8.0, 256), _F8_START.copy()
    T = spec["T"]
    return Problem(K=spec["K"], T=T, Z=Z, y=y, log_ell=log_ell, log_sf=log_sf, log_sn=log_sn,
                   obstacles=obs, path_kind=kind, circle=circ, path_pts=pts, x0=x0,
                   U0=np.zeros((T, 2)), seed=((2000 + c) << 32), pid=0, name=f"c{c}")


def make_batch_problem(pid: int, root_seed: int = 1003) -> Problem:
    """One of the independent problems of the batched workload (uneven shapes)."""
    rng = np.random.Generator(np.random.PCG64([root_seed, pid]))
    K = int(rng.choice([1024, 2048, 4096, 8192, 16384]))
    T = int(rng.integers(30, 101))
    M = int(rng.choice([64, 256, 512, 1024]))
    n_obs = int(rng.integers(0, 51))
    eight = bool(rng.integers(0, 2))
    Z, y = _gp_data(rng, max(M, 2000) if M > 50 else 50, M)
    obs = _obstacles(rng, n_obs, 10.0, 0.2, 0.8)
    log_ell, log_sf, log_sn = _hyper()
    if eight:
        kind, circ, pts, x0 = 1, (0.0, 0.0, 0.0), figure_eight(8.0, 256), _F8_START.copy()
    else:
        kind, circ, pts, x0 = 0, (0.0, 0.0, 5.0), np.zeros((0, 2)), _C0_START.copy()
    return Problem(K=K, T=T, Z=Z, y=y, log_ell=log_ell, log_sf=log_sf, log_sn=log_sn,
                   obstacles=obs, path_kind=kind, circle=circ, path_pts=pts, x0=x0,
                   U0=np.zeros((T, 2)), seed=(2003 << 32), pid=pid, name=f"c3p{pid}")


def small_problem(K=64, T=10, M=40, n_obs=4, path="circle", seed_data=7, U_scale=0.0,
                  n_data: Optional[int] = None, x0=None) -> Problem:
    """A small instance with the paper's structure, for fast tests."""
    rng = np.random.Generator(np.random.PCG64(seed_data))
    Z, y = _gp_data(rng, n_data or M, M)
    obs = _obstacles(rng, n_obs, 6.0, 0.3, 0.6)
    U0 = rng.uniform(-1.0, 1.0, size=(T, 2)) * U_scale
    log_ell, log_sf, log_sn = _hyper()
    if path == "circle":
        kind, circ, pts, xs = 0, (0.0, 0.0, 5.0), np.zeros((0, 2)), _C0_START.copy()
    else:
        kind, circ, pts, xs = 1, (0.0, 0.0, 0.0), figure_eight(8.0, 256), _F8_START.copy()
    return Problem(K=K, T=T, Z=Z, y=y, log_ell=log_ell, log_sf=log_sf, log_sn=log_sn,
                   obstacles=obs, path_kind=kind, circle=circ, path_pts=pts,
                   x0=xs if x0 is None else np.asarray(x0, float), U0=U0,
                   seed=(0xC0FFEE << 32) + seed_data, pid=0, name=f"small{seed_data}")


def random_queries(n: int, seed: int, lo=-2.5, hi=2.5) -> np.ndarray:
    """GP query points q = (v, w, v_cmd, w_cmd), uniform in a box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=(n, 4))


def random_costs(K: int, seed: int, spread: float = 20.0, offset: float = 100.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return offset + spread * rng.random(K)


def random_controls(T: int, seed: int, scale: float = 1.5) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, size=(T, 2))


# Per-terrain synthetic residuals on shared inputs (v, w, v_cmd, w_cmd):
# y = a sin(v w) - c v + N(0, 0.05^2), one (a, c) per terrain.
TERRAINS = ((0.3, 0.0), (0.15, 0.2), (0.45, -0.1))


def add_terrains(problem: Problem, seed: int, weights=(0.5, 0.3, 0.2), n_terr: int = 3) -> Problem:
    """Gives the problem n_terr target sets on its GP inputs and ensemble weights."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M = problem.M
    ty = np.empty((n_terr, 2, M))
    for i in range(n_terr):
        a, c = TERRAINS[i % len(TERRAINS)]
        for o in range(2):
            Zo = problem.Z[o]
            ty[i, o] = a * np.sin(Zo[:, 0] * Zo[:, 1]) - c * Zo[:, 0] + rng.normal(0.0, TARGET_NOISE, size=M)
    problem.terrain_y = ty
    problem.terrain_w = np.asarray(weights[:n_terr], dtype=np.float64)
    return problem

"""The adjoint rollout's per-sample algebra (csrc/adjoint_step.hpp, built for
the host) against float64 reverse-mode autodiff of one step written out here:
the covariance update of Eq. (10), the Euler step of Eqs. (1)-(2), and the
smoothed stage cost of Eqs. (11)-(16) with sigmoid indicators."""
import ctypes
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

from oracle.constraints import chi2_2_quantile, norm_ppf
from paper_2411_03289_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TRIU = [(0, 0), (0, 1), (0, 2), (0, 3), (0, 4), (1, 1), (1, 2), (1, 3), (1, 4), (2, 2), (2, 3), (2, 4), (3, 3),
        (3, 4), (4, 4)]
F = ctypes.POINTER(ctypes.c_float)


@pytest.fixture(scope="module")
def L(tmp_path_factory):
    hipcc = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
    if hipcc is None:
        pytest.skip("hipcc unavailable")
    out = str(tmp_path_factory.mktemp("adj") / "libadj.so")
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O1", "-std=c++17", "-fPIC", "-shared",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2411_03289_amd", "csrc"),
                    os.path.join(HERE, "adjoint_step_check.cpp"), "-o", out], check=True, capture_output=True)
    lib = ctypes.CDLL(out)
    lib.adj_stage.restype = ctypes.c_float
    return lib


def _f(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(F)


class World:
    def __init__(self, path_kind, n_obs, seed, tau, p_x=0.95):
        rng = np.random.Generator(np.random.PCG64(seed))
        self.kind = path_kind
        self.circle = np.array([0.0, 0.0, 5.0], np.float32)
        pts = W.figure_eight(8.0, 256) if path_kind else np.array([[0.0, 0.0], [1.0, 0.0]])
        e = np.roll(pts, -1, axis=0) - pts
        self.seg = np.concatenate([pts, e], axis=1).astype(np.float32)
        self.seg_inv = (1.0 / (e * e).sum(1)).astype(np.float32)
        self.P = pts.shape[0] if path_kind else 0
        self.obs = np.zeros((max(n_obs, 1), 4), np.float32)
        self.n_obs = n_obs
        self.hw = 1.0
        self.z_p = np.float32(norm_ppf(p_x))
        self.c_p = np.float32(math.sqrt(chi2_2_quantile(p_x)))
        self.tau = tau
        self.rng = rng
        p = W.DEFAULT_PARAMS
        self.cw = np.array([p["w_var"], p["w_dev"], p["w_lane"], p["w_speed"], p["w_obs"], p["v_des"],
                            p["discount"]], np.float32)
        dt, tv, tw = p["dt"], p["tau_v"], p["tau_w"]
        self.dyn = np.array([dt, dt / tv, dt / tw, 1 - dt / tv, 1 - dt / tw], np.float32)

    def place_obstacles(self, X, Y):
        # obstacles around the point so that the sigmoid is not saturated
        for j in range(self.n_obs):
            ang = self.rng.uniform(0, 2 * np.pi)
            r = self.rng.uniform(0.2, 0.6)
            dist = r + self.rng.uniform(-0.05, 0.3)
            self.obs[j] = [X + dist * np.cos(ang), Y + dist * np.sin(ang), r, 0.0]


def _sym(p15):
    S = torch.zeros((5, 5), dtype=torch.float64)
    rows = []
    for i in range(5):
        row = []
        for j in range(5):
            a, b = min(i, j), max(i, j)
            row.append(p15[TRIU.index((a, b))])
        rows.append(torch.stack(row))
    return torch.stack(rows)


def _step_torch(wd, xk, pk, u, m, s2, disc_k, cbar, xb_in, pb_in, iseg, iobs):
    dt, dtv, dtw, a33, a44 = (float(v) for v in wd.dyn)
    X, Y, th, v, w = xk
    A = torch.zeros((5, 5), dtype=torch.float64)
    A = A + torch.diag(torch.tensor([1.0, 1.0, 1.0, a33, a44], dtype=torch.float64))
    E = torch.zeros((5, 5), dtype=torch.float64)
    E[0, 2] = 1.0
    A = A + E * (-dt * v * torch.sin(th))
    E = torch.zeros((5, 5), dtype=torch.float64); E[0, 3] = 1.0
    A = A + E * (dt * torch.cos(th))
    E = torch.zeros((5, 5), dtype=torch.float64); E[1, 2] = 1.0
    A = A + E * (dt * v * torch.cos(th))
    E = torch.zeros((5, 5), dtype=torch.float64); E[1, 3] = 1.0
    A = A + E * (dt * torch.sin(th))
    E = torch.zeros((5, 5), dtype=torch.float64); E[2, 4] = 1.0
    A = A + E * dt
    x1 = torch.stack([X + dt * v * torch.cos(th), Y + dt * v * torch.sin(th), th + dt * w,
                      v + (dtv * (u[0] - v) + dt * m[0]), w + (dtw * (u[1] - w) + dt * m[1])])
    D = torch.zeros((5, 5), dtype=torch.float64)
    D3 = torch.zeros((5, 5), dtype=torch.float64); D3[3, 3] = 1.0
    D4 = torch.zeros((5, 5), dtype=torch.float64); D4[4, 4] = 1.0
    S1 = A @ _sym(pk) @ A.T + D3 * (dt * dt * s2[0]) + D4 * (dt * dt * s2[1])
    p1 = torch.stack([S1[i, j] for i, j in TRIU])
    a, b, c = p1[0], p1[1], p1[5]
    h = 0.5 * (a - c)
    lmax = 0.5 * (a + c) + torch.sqrt(h * h + b * b)
    w_var, w_dev, w_lane, w_speed, w_obs, v_des, _ = (float(t) for t in wd.cw)
    if wd.kind == 0:
        dl = torch.abs(torch.sqrt(x1[0] ** 2 + x1[1] ** 2) - float(wd.circle[2]))
    else:
        sg = torch.as_tensor(wd.seg[iseg].astype(np.float64))
        rx, ry = x1[0] - sg[0], x1[1] - sg[1]
        t = torch.clamp((rx * sg[2] + ry * sg[3]) * float(wd.seg_inv[iseg]), 0.0, 1.0)
        dl = torch.sqrt((rx - t * sg[2]) ** 2 + (ry - t * sg[3]) ** 2)
    rbar = wd.hw - float(wd.c_p) * torch.sqrt(lmax)
    cost = (w_var * (s2[0] + s2[1]) + w_dev * dl / wd.hw + w_speed * (v_des - x1[3]) ** 2
            + w_lane * disc_k * torch.sigmoid((dl - rbar) / wd.tau))
    if iobs >= 0:
        ob = wd.obs[iobs].astype(np.float64)
        dx, dy = x1[0] - ob[0], x1[1] - ob[1]
        rho = torch.sqrt(dx * dx + dy * dy)
        var = (a * dx * dx + 2 * b * dx * dy + c * dy * dy) / (rho * rho)
        om = rho - ob[2] - float(wd.z_p) * torch.sqrt(var)
        cost = cost + w_obs * torch.sigmoid(-om / wd.tau)
    total = cbar * cost + (xb_in * x1).sum() + (pb_in * p1).sum()
    return total, cost, x1, p1


def _argmins(wd, x1, p1):
    iseg = -1
    if wd.kind == 1:
        rel = x1[:2][None, :] - wd.seg[:, :2]
        t = np.clip((rel * wd.seg[:, 2:]).sum(1) * wd.seg_inv, 0, 1)
        d = rel - t[:, None] * wd.seg[:, 2:]
        iseg = int(np.argmin((d * d).sum(1)))
    iobs = -1
    if wd.n_obs:
        a, b, c = p1[0], p1[1], p1[5]
        dx = x1[0] - wd.obs[:wd.n_obs, 0]
        dy = x1[1] - wd.obs[:wd.n_obs, 1]
        rho = np.hypot(dx, dy)
        var = (a * dx * dx + 2 * b * dx * dy + c * dy * dy) / rho ** 2
        iobs = int(np.argmin(rho - wd.obs[:wd.n_obs, 2] - wd.z_p * np.sqrt(var)))
    return iseg, iobs


def _case(seed, kind, n_obs, tau):
    wd = World(kind, n_obs, seed, tau)
    rng = wd.rng
    if kind == 0:
        ang = rng.uniform(0, 2 * np.pi)
        rad = 5.0 + rng.uniform(-0.8, 0.8)
        X, Y = rad * np.cos(ang), rad * np.sin(ang)
    else:
        i = rng.integers(0, 256)
        X, Y = wd.seg[i, 0] + rng.normal(0, 0.4), wd.seg[i, 1] + rng.normal(0, 0.4)
    xk = np.array([X, Y, rng.uniform(-np.pi, np.pi), rng.uniform(0.3, 2.0), rng.uniform(-1, 1)], np.float32)
    B = rng.normal(size=(5, 5)) * 0.15
    S = B @ B.T
    S[2, 3] = S[3, 2] = 0.0
    S[3, 4] = S[4, 3] = 0.0
    S[:2, :2] += np.eye(2) * 0.02
    pk = np.array([S[i, j] for i, j in TRIU], np.float32)
    u = rng.uniform(-2, 2, 2).astype(np.float32)
    m = rng.normal(0, 0.2, 2).astype(np.float32)
    s2 = rng.uniform(0.003, 0.3, 2).astype(np.float32)
    wd.place_obstacles(X + 0.05 * np.cos(xk[2]), Y + 0.05 * np.sin(xk[2]))
    xb_in = rng.normal(size=5).astype(np.float32)
    pb_in = rng.normal(size=15).astype(np.float32)
    return wd, xk, pk, u, m, s2, xb_in, pb_in


@pytest.mark.parametrize("seed,kind,n_obs,tau", [(1, 0, 0, 0.05), (2, 0, 5, 0.05), (3, 1, 0, 0.05), (4, 1, 6, 0.05),
                                                 (5, 1, 6, 0.3), (6, 0, 3, 0.5), (7, 1, 4, 0.02), (8, 0, 6, 0.1)])
def test_step_adjoint_matches_float64_autodiff(L, seed, kind, n_obs, tau):
    wd, xk, pk, u, m, s2, xb_in, pb_in = _case(seed, kind, n_obs, tau)
    disc_k, cbar = np.float32(0.9 ** 3), np.float32(1.0 / 64)
    # forward in the harness (covariance) and in float64
    dt, a33, a44 = float(wd.dyn[0]), float(wd.dyn[3]), float(wd.dyn[4])
    th, v = float(xk[2]), float(xk[3])
    jac = np.array([-dt * v * math.sin(th), dt * math.cos(th), dt * v * math.cos(th), dt * math.sin(th)], np.float32)
    P = np.zeros(15, np.float32)
    L.adj_cov_forward(_f(pk)[1], _f(jac)[1], ctypes.c_float(dt), ctypes.c_float(a33), ctypes.c_float(a44),
                      ctypes.c_float(dt * dt * s2[0]), ctypes.c_float(dt * dt * s2[1]), P.ctypes.data_as(F))
    leaves = [torch.tensor(a.astype(np.float64), requires_grad=True) for a in (xk, pk, u, m, s2)]
    # the next state (independent of the argmins), the argmins there, then the evaluation
    _, _, x1, p1 = _step_torch(wd, *leaves, float(disc_k), float(cbar), torch.tensor(xb_in.astype(np.float64)),
                               torch.tensor(pb_in.astype(np.float64)), 0, -1)
    iseg, iobs = _argmins(wd, x1.detach().numpy(), p1.detach().numpy())
    total, cost, x1, p1 = _step_torch(wd, *leaves, float(disc_k), float(cbar),
                                      torch.tensor(xb_in.astype(np.float64)), torch.tensor(pb_in.astype(np.float64)),
                                      iseg, iobs)
    np.testing.assert_allclose(P, p1.detach().numpy(), rtol=2e-6, atol=1e-7)
    grads = torch.autograd.grad(total, leaves)
    x1f = x1.detach().numpy().astype(np.float32)
    p1f = p1.detach().numpy().astype(np.float32)
    circle = wd.circle
    c_h = L.adj_stage(wd.kind, _f(circle)[1], wd.P, _f(wd.seg)[1], _f(wd.seg_inv)[1], wd.n_obs, _f(wd.obs)[1],
                      ctypes.c_float(wd.hw), ctypes.c_float(wd.z_p), ctypes.c_float(wd.c_p), _f(wd.cw)[1],
                      ctypes.c_float(1.0 / tau), ctypes.c_float(disc_k), _f(x1f)[1], _f(p1f)[1], _f(s2)[1], iseg, iobs)
    assert c_h == pytest.approx(float(cost.detach()), rel=2e-5, abs=2e-6)
    xb = xb_in.copy()
    pb = pb_in.copy()
    out6 = np.zeros(6, np.float32)
    L.adj_step(wd.kind, _f(circle)[1], wd.P, _f(wd.seg)[1], _f(wd.seg_inv)[1], wd.n_obs, _f(wd.obs)[1],
               ctypes.c_float(wd.hw), ctypes.c_float(wd.z_p), ctypes.c_float(wd.c_p), _f(wd.cw)[1], _f(wd.dyn)[1],
               ctypes.c_float(1.0 / tau), ctypes.c_float(cbar), ctypes.c_float(disc_k), _f(xk)[1], _f(pk)[1],
               _f(x1f)[1], _f(p1f)[1], iseg, iobs, xb.ctypes.data_as(F), pb.ctypes.data_as(F),
               out6.ctypes.data_as(F))
    gx, gp, gu, gm, gs = (g.numpy() for g in grads)
    for name, got, ref in (("x", xb, gx), ("Sigma", pb, gp), ("u", out6[4:6], gu), ("m", out6[2:4], gm),
                           ("s2", out6[0:2], gs)):
        scale = max(np.abs(ref).max(), 1e-3)
        assert np.all(np.abs(got - ref) <= 2e-4 * scale + 1e-4 * np.abs(ref)), (name, got, ref)

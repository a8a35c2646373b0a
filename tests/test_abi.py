"""C-ABI contract checks that need no GPU: the library loads, exports every
function the header declares, and rejects invalid arguments on the host."""
import ctypes
import math
import os
import re

import numpy as np
import pytest
from scipy import stats

from paper_2411_03289_amd import gpmppi as B
from paper_2411_03289_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libgpmppi.so not built")
    return B.lib()


def _declared():
    text = open(os.path.join(ROOT, "include", "gpmppi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gpmppi_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_documented_entry_points():
    names = _declared()
    for n in ("gpmppi_init", "gpmppi_step", "gpmppi_rollout", "gpmppi_weights_update", "gpmppi_gp_predict",
              "gpmppi_closed_loop", "gpmppi_destroy", "gpmppi_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_normal_quantile_host_routine(L):
    for p in (1e-12, 0.01, 0.3, 0.5, 0.9, 0.95, 0.999999):
        assert B.gpmppi_norm_quantile(p) == pytest.approx(stats.norm.ppf(p), rel=1e-13, abs=1e-14)
    assert math.isnan(B.gpmppi_norm_quantile(1.0)) and math.isnan(B.gpmppi_norm_quantile(0.0))


def _args(pr, **over):
    keep = []
    params = B.make_params(pr)
    for k, v in over.items():
        setattr(params, k, v)
    gps = B._gp_structs(pr, keep)
    ob, obp = B._as_c_double(pr.obstacles)
    keep.append(ob)
    obs = B.gpmppi_obstacles(n=pr.obstacles.shape[0], xyr=obp)
    path = B.gpmppi_path(kind=0, cx=0, cy=0, R=5.0, P=0, pts=None, half_width=1.0)
    return params, gps, obs, path, keep


def _init_status(L, params, gps, obs, path):
    h = ctypes.c_void_p()
    st = L.gpmppi_init(ctypes.byref(params), gps, ctypes.byref(obs), ctypes.byref(path), ctypes.byref(h))
    assert h.value is None
    return st, L.gpmppi_last_error().decode()


@pytest.mark.parametrize("field,value,code", [
    ("K", 0, -1), ("T", 0, -1), ("T", 5000, -1), ("lambda_", 0.0, -1), ("p_x", 1.0, -1), ("p_x", 0.0, -1),
    ("dt", -0.1, -1), ("precision", 3, -1), ("sig_v", -1.0, -1), ("dt", float("nan"), -5),
    ("w_obs", float("inf"), -5), ("K", 1 << 25, -6)])
def test_invalid_params_rejected_before_device_work(L, field, value, code):
    pr = W.small_problem()
    params, gps, obs, path, keep = _args(pr, **{field: value})
    st, msg = _init_status(L, params, gps, obs, path)
    assert st == code and msg


def test_invalid_gp_and_world_rejected(L):
    pr = W.small_problem(M=12)
    params, gps, obs, path, keep = _args(pr)
    gps[1].M = 11
    assert _init_status(L, params, gps, obs, path)[0] == -1
    pr.Z[0, 3, 2] = np.nan
    params, gps, obs, path, keep = _args(pr)
    assert _init_status(L, params, gps, obs, path)[0] == -5
    big = W.small_problem(M=1100)
    params, gps, obs, path, keep = _args(big)
    assert _init_status(L, params, gps, obs, path)[0] == -6
    pr = W.small_problem(M=12)
    pr.obstacles[0, 2] = -0.1
    params, gps, obs, path, keep = _args(pr)
    assert _init_status(L, params, gps, obs, path)[0] == -1
    pr = W.small_problem(M=12)
    params, gps, obs, path, keep = _args(pr)
    path.half_width = 0.0
    assert _init_status(L, params, gps, obs, path)[0] == -1
    pts = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 0.0]])
    path = B.gpmppi_path(kind=1, cx=0, cy=0, R=0, P=3, pts=pts.ctypes.data_as(B._dp), half_width=1.0)
    assert _init_status(L, params, gps, obs, path)[0] == -1


def test_null_arguments_rejected(L):
    assert L.gpmppi_step(None, None, None, 0, None, None, None, None) == -1
    assert L.gpmppi_rollout(None, None, None, 0, None, None, None) == -1
    assert L.gpmppi_philox(0, None, 1, None, None) == -1
    assert L.gpmppi_info(None, None, None, None) == -1
    assert L.gpmppi_set_exchange_spin(None, 0) == -1
    L.gpmppi_destroy(None)


def test_binding_names_follow_the_abi():
    for n in _declared():
        assert hasattr(B, n), n


def test_batch_validation_without_device(L):
    ps = [W.small_problem(seed_data=1), W.small_problem(seed_data=2)]
    keep = []
    params = (B.gpmppi_params * 2)(B.make_params(ps[0], B.FP32), B.make_params(ps[1], B.BF16))
    gps = (B.gpmppi_gp * 4)()
    obs = (B.gpmppi_obstacles * 2)()
    paths = (B.gpmppi_path * 2)()
    for i, p in enumerate(ps):
        g = B._gp_structs(p, keep)
        gps[2 * i], gps[2 * i + 1] = g[0], g[1]
        obs[i], paths[i] = B._world_structs(p, keep)
    h = ctypes.c_void_p()
    assert L.gpmppi_batch_init(2, params, gps, obs, paths, ctypes.byref(h)) == -1   # mixed precision
    assert L.gpmppi_batch_init(0, params, gps, obs, paths, ctypes.byref(h)) == -1
    params[1].precision = B.FP32
    params[1].K = 0
    assert L.gpmppi_batch_init(2, params, gps, obs, paths, ctypes.byref(h)) == -1
    assert h.value is None


def test_tuning_struct_and_null_handles(L):
    import ctypes
    assert ctypes.sizeof(B.gpmppi_tuning) == 32
    assert B.gpmppi_tuning.split.offset == 20 and B.gpmppi_tuning.ms.offset == 24
    t = B.gpmppi_tuning(1, 1, 1, 0, 4, 0, 0.0)
    for fn in (L.gpmppi_set_tuning, L.gpmppi_batch_set_tuning, L.gpmppi_get_tuning, L.gpmppi_batch_get_tuning):
        assert fn(None, ctypes.byref(t)) == -1
    assert L.gpmppi_tune(None, None, None, 0, 1, None, None) == -1
    assert L.gpmppi_batch_tune(None, None, None, 0, 1, None, None) == -1


def test_grad_entry_point_rejects_null_context(L):
    assert L.gpmppi_grad(None, None, None, 0, 0.05, 10, None, None, None, None, None, None) == -1

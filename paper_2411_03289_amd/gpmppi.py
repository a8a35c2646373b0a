"""ctypes binding of libgpmppi.so (the C ABI declared in include/gpmppi.h).

Argument marshalling only: every step of the controller runs in the HIP
library.  Device arrays are torch tensors on the context's GPU; streams are
torch streams (default: the current stream).  Every function raises
GpmppiError when the library returns an error status, and the library must
be built (python -m paper_2411_03289_amd.build) - there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpmppi.so")

FP32, BF16, BF16X3 = 0, 1, 2
STATUS = {0: "OK", -1: "E_INVALID", -2: "E_NOT_PD", -3: "E_HIP", -4: "E_NOMEM", -5: "E_NONFINITE",
          -6: "E_UNSUPPORTED"}
# status bits read by gpmppi_status_flags (GPMPPI_FLAG_* in gpmppi.h)
FLAG_NONFINITE = 1
FLAG_EXCHANGE_TIMEOUT = 2
FLAG_PIPELINE_STALL = 4

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)


class GpmppiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class gpmppi_gp(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("Z", _dp), ("y", _dp), ("log_ell", ctypes.c_double * 4),
                ("log_sf", ctypes.c_double), ("log_sn", ctypes.c_double)]


class gpmppi_obstacles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("xyr", _dp)]


class gpmppi_path(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("R", ctypes.c_double), ("P", ctypes.c_int32), ("pts", _dp),
                ("half_width", ctypes.c_double)]


class gpmppi_params(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("T", ctypes.c_int32), ("dt", ctypes.c_double),
                ("tau_v", ctypes.c_double), ("tau_w", ctypes.c_double), ("sig_v", ctypes.c_double),
                ("sig_w", ctypes.c_double), ("u_min", ctypes.c_double * 2), ("u_max", ctypes.c_double * 2),
                ("lambda_", ctypes.c_double), ("p_x", ctypes.c_double), ("w_var", ctypes.c_double),
                ("w_dev", ctypes.c_double), ("w_lane", ctypes.c_double), ("w_speed", ctypes.c_double),
                ("w_obs", ctypes.c_double), ("v_des", ctypes.c_double), ("discount", ctypes.c_double),
                ("precision", ctypes.c_int32), ("problem_id", ctypes.c_int32),
                ("w_goal", ctypes.c_double), ("w_term", ctypes.c_double), ("goal", ctypes.c_double * 2),
                ("goal_tol", ctypes.c_double), ("tighten", ctypes.c_int32)]


class gpmppi_trace(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("x_d", "sxy_d", "gp_mean_d", "gp_var_d", "d_lane_d",
                                              "lane_margin_d", "obs_margin_d", "u_d")]


class gpmppi_tuning(ctypes.Structure):
    _fields_ = [("groups", ctypes.c_int32), ("rotate", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("order", ctypes.c_int32), ("waves", ctypes.c_int32), ("split", ctypes.c_int32),
                ("ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2411_03289_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    sig = {
        "gpmppi_init": [ctypes.POINTER(gpmppi_params), ctypes.POINTER(gpmppi_gp), ctypes.POINTER(gpmppi_obstacles),
                        ctypes.POINTER(gpmppi_path), ctypes.POINTER(vp)],
        "gpmppi_set_gp": [vp, ctypes.POINTER(gpmppi_gp)],
        "gpmppi_set_terrains": [vp, i32, ctypes.POINTER(f64), ctypes.POINTER(f64)],
        "gpmppi_set_terrain_weights": [vp, ctypes.POINTER(f64)],
        "gpmppi_terrain_weights": [i32, i32] + [ctypes.POINTER(f64)] * 5 + [f64, ctypes.POINTER(f64)],
        "gpmppi_terrain_means": [vp, vp, i32, vp, vp],
        "gpmppi_step": [vp, vp, vp, u64, vp, vp, vp, vp],
        "gpmppi_rollout": [vp, vp, vp, u64, vp, ctypes.POINTER(gpmppi_trace), vp],
        "gpmppi_weights_update": [vp, vp, vp, u64, vp, vp, vp],
        "gpmppi_gp_predict": [vp, vp, i32, vp, vp, vp],
        "gpmppi_plant_shift": [vp, vp, vp, vp, f64, vp],
        "gpmppi_closed_loop": [vp, vp, vp, u64, i32, f64, vp, vp, i32, vp],
        "gpmppi_philox": [u64, vp, i32, vp, vp],
        "gpmppi_status_flags": [vp, ctypes.POINTER(ctypes.c_uint32)],
        "gpmppi_info": [vp, ctypes.POINTER(i32), ctypes.POINTER(f64), ctypes.POINTER(f64)],
        "gpmppi_batch_init": [i32, ctypes.POINTER(gpmppi_params), ctypes.POINTER(gpmppi_gp),
                              ctypes.POINTER(gpmppi_obstacles), ctypes.POINTER(gpmppi_path), ctypes.POINTER(vp)],
        "gpmppi_batch_layout": [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
        "gpmppi_batch_step": [vp, vp, vp, u64, vp, vp, vp, vp],
        "gpmppi_batch_closed_loop": [vp, vp, vp, u64, i32, f64, vp, i32, vp],
        "gpmppi_tune": [vp, vp, vp, u64, i32, ctypes.POINTER(gpmppi_tuning), vp],
        "gpmppi_grad": [vp, vp, vp, u64, f64, i32, vp, vp, vp, vp, vp, vp],
        "gpmppi_grad_noalloc": [vp, vp, vp, u64, f64, i32, vp, vp, vp, vp, vp, vp],
        "gpmppi_set_tuning": [vp, ctypes.POINTER(gpmppi_tuning)],
        "gpmppi_set_exchange_spin": [vp, i32],
        "gpmppi_set_grad_split": [vp, i32],
        "gpmppi_get_tuning": [vp, ctypes.POINTER(gpmppi_tuning)],
        "gpmppi_batch_tune": [vp, vp, vp, u64, i32, ctypes.POINTER(gpmppi_tuning), vp],
        "gpmppi_batch_set_tuning": [vp, ctypes.POINTER(gpmppi_tuning)],
        "gpmppi_batch_get_tuning": [vp, ctypes.POINTER(gpmppi_tuning)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.gpmppi_destroy.argtypes = [vp]
    L.gpmppi_destroy.restype = None
    L.gpmppi_batch_destroy.argtypes = [vp]
    L.gpmppi_batch_destroy.restype = None
    L.gpmppi_last_error.argtypes = []
    L.gpmppi_last_error.restype = ctypes.c_char_p
    L.gpmppi_norm_quantile.argtypes = [f64]
    L.gpmppi_norm_quantile.restype = f64
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise GpmppiError(status, lib().gpmppi_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _dev(t, n: int, name: str, dtype: str = "float32", optional: bool = False):
    """Checks a device tensor argument: on a GPU, contiguous, right dtype, at
    least n elements.  Returns its address (None for an allowed None)."""
    if t is None:
        if optional:
            return None
        raise GpmppiError(-1, f"{name} is required")
    if not getattr(t, "is_cuda", False):
        raise GpmppiError(-1, f"{name} must be a GPU tensor")
    if str(t.dtype) != f"torch.{dtype}":
        raise GpmppiError(-1, f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise GpmppiError(-1, f"{name} must be contiguous")
    if t.numel() < n:
        raise GpmppiError(-1, f"{name} needs {n} elements, has {t.numel()}")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(stream)


class Context:
    """Owns a gpmppi_ctx; destroyed with the object."""

    def __init__(self, handle: int, params: dict):
        self.handle = ctypes.c_void_p(handle)
        self.params = params

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gpmppi_destroy(self.handle)
            self.handle = None


def _as_c_double(a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def make_params(problem, precision: int = FP32) -> gpmppi_params:
    p = problem.params
    return gpmppi_params(
        K=problem.K, T=problem.T, dt=p["dt"], tau_v=p["tau_v"], tau_w=p["tau_w"], sig_v=p["sig_v"],
        sig_w=p["sig_w"], u_min=(ctypes.c_double * 2)(*p["u_min"]), u_max=(ctypes.c_double * 2)(*p["u_max"]),
        lambda_=p["lam"], p_x=p["p_x"], w_var=p["w_var"], w_dev=p["w_dev"], w_lane=p["w_lane"],
        w_speed=p["w_speed"], w_obs=p["w_obs"], v_des=p["v_des"], discount=p["discount"],
        precision=precision, problem_id=problem.pid, w_goal=p.get("w_goal", 0.0), w_term=p.get("w_term", 0.0),
        goal=(ctypes.c_double * 2)(*p.get("goal", (0.0, 0.0))), goal_tol=p.get("goal_tol", 0.5),
        tighten=int(p.get("tighten", 0)))


def _gp_structs(problem, keep: list):
    gps = (gpmppi_gp * 2)()
    for o in range(2):
        Z, Zp = _as_c_double(problem.Z[o])
        y, yp = _as_c_double(problem.y[o])
        keep += [Z, y]
        gps[o].M = problem.M
        gps[o].Z, gps[o].y = Zp, yp
        gps[o].log_ell = (ctypes.c_double * 4)(*problem.log_ell[o])
        gps[o].log_sf = float(problem.log_sf[o])
        gps[o].log_sn = float(problem.log_sn[o])
    return gps


def _world_structs(problem, keep: list):
    ob_arr, ob_p = _as_c_double(problem.obstacles.reshape(-1, 3))
    keep.append(ob_arr)
    obs = gpmppi_obstacles(n=problem.obstacles.shape[0], xyr=ob_p)
    if problem.path_kind == 0:
        cx, cy, R = problem.circle
        path = gpmppi_path(kind=0, cx=cx, cy=cy, R=R, P=0, pts=None, half_width=problem.params["half_width"])
    else:
        pts, pts_p = _as_c_double(problem.path_pts)
        keep.append(pts)
        path = gpmppi_path(kind=1, cx=0, cy=0, R=0, P=pts.shape[0], pts=pts_p,
                           half_width=problem.params["half_width"])
    return obs, path


def gpmppi_init(problem, precision: int = FP32) -> Context:
    """Creates a context from a workload Problem (see workloads.Problem)."""
    keep: list = []
    params = make_params(problem, precision)
    gps = _gp_structs(problem, keep)
    obs, path = _world_structs(problem, keep)
    h = ctypes.c_void_p()
    _check(lib().gpmppi_init(ctypes.byref(params), gps, ctypes.byref(obs), ctypes.byref(path), ctypes.byref(h)))
    ctx = Context(h.value, dict(K=problem.K, T=problem.T, M=problem.M, precision=precision))
    if getattr(problem, "terrain_y", None) is not None:
        gpmppi_set_terrains(ctx, problem.terrain_y, problem.terrain_w)
    return ctx


def gpmppi_set_gp(ctx: Context, problem):
    keep: list = []
    _check(lib().gpmppi_set_gp(ctx.handle, _gp_structs(problem, keep)))


def gpmppi_set_terrains(ctx: Context, terrain_y, weights):
    """terrain_y [n_terr, 2, M] targets on the context's GP inputs; weights [n_terr]."""
    y, yp = _as_c_double(terrain_y)
    w, wp = _as_c_double(weights)
    if y.ndim != 3 or y.shape[1:] != (2, ctx.params["M"]) or w.shape != (y.shape[0],):
        raise GpmppiError(-1, "terrain_y must be [n_terr, 2, M] and weights [n_terr]")
    _check(lib().gpmppi_set_terrains(ctx.handle, int(y.shape[0]), yp, wp))
    ctx.params["n_terr"] = int(y.shape[0])


def gpmppi_set_terrain_weights(ctx: Context, weights):
    w, wp = _as_c_double(weights)
    if w.shape != (ctx.params.get("n_terr", -1),):
        raise GpmppiError(-1, "weights must have one entry per terrain")
    _check(lib().gpmppi_set_terrain_weights(ctx.handle, wp))


def gpmppi_terrain_means(ctx: Context, q, out, stream=None):
    n, nt = int(q.shape[0]), ctx.params.get("n_terr", 0)
    _check(lib().gpmppi_terrain_means(ctx.handle, _dev(q, 4 * n, "q"), n, _dev(out, n * max(nt, 1) * 2, "out"),
                                      _stream(stream)))


def gpmppi_terrain_weights(Yv, Yw, Fv, Fw, w_prev, gamma: float) -> np.ndarray:
    """Eq. (4) on the host: returns the new terrain weights [n]."""
    Yv, Yvp = _as_c_double(Yv)
    Yw, Ywp = _as_c_double(Yw)
    Fv, Fvp = _as_c_double(Fv)
    Fw, Fwp = _as_c_double(Fw)
    wp, wpp = _as_c_double(w_prev)
    H, n = Fv.shape
    if Yv.shape != (H,) or Yw.shape != (H,) or Fw.shape != (H, n) or wp.shape != (n,):
        raise GpmppiError(-1, "shapes: Yv, Yw [H]; Fv, Fw [H, n]; w_prev [n]")
    out = np.empty(n)
    _check(lib().gpmppi_terrain_weights(H, n, Yvp, Ywp, Fvp, Fwp, wpp, float(gamma), out.ctypes.data_as(_dp)))
    return out


def gpmppi_step(ctx: Context, x0, U, seed: int, U_out, costs, weights=None, stream=None):
    K, T = ctx.params["K"], ctx.params["T"]
    _check(lib().gpmppi_step(ctx.handle, _dev(x0, 5, "x0"), _dev(U, 2 * T, "U"), ctypes.c_uint64(seed),
                             _dev(U_out, 2 * T, "U_out"), _dev(costs, K, "costs"),
                             _dev(weights, K, "weights", optional=True), _stream(stream)))


TRACE_SIZES = {"x_d": lambda K, T: (T + 1) * 5 * K, "sxy_d": lambda K, T: (T + 1) * 3 * K,
               "gp_mean_d": lambda K, T: T * 2 * K, "gp_var_d": lambda K, T: T * 2 * K,
               "d_lane_d": lambda K, T: T * K, "lane_margin_d": lambda K, T: T * K,
               "obs_margin_d": lambda K, T: T * K, "u_d": lambda K, T: T * 2 * K}


def gpmppi_rollout(ctx: Context, x0, U, seed: int, costs, trace: Optional[dict] = None, stream=None):
    K, T = ctx.params["K"], ctx.params["T"]
    tr = None
    if trace:
        unknown = set(trace) - set(TRACE_SIZES)
        if unknown:
            raise GpmppiError(-1, f"unknown trace fields {sorted(unknown)}")
        tr = gpmppi_trace(**{k: _dev(v, TRACE_SIZES[k](K, T), k, optional=True) for k, v in trace.items()})
    _check(lib().gpmppi_rollout(ctx.handle, _dev(x0, 5, "x0"), _dev(U, 2 * T, "U"), ctypes.c_uint64(seed),
                                _dev(costs, K, "costs"), ctypes.byref(tr) if tr is not None else None,
                                _stream(stream)))


def gpmppi_weights_update(ctx: Context, costs, U, seed: int, U_out, weights=None, stream=None):
    K, T = ctx.params["K"], ctx.params["T"]
    _check(lib().gpmppi_weights_update(ctx.handle, _dev(costs, K, "costs"), _dev(U, 2 * T, "U"),
                                       ctypes.c_uint64(seed), _dev(U_out, 2 * T, "U_out"),
                                       _dev(weights, K, "weights", optional=True), _stream(stream)))


def gpmppi_gp_predict(ctx: Context, q, mean, var, stream=None):
    n = int(q.shape[0])
    _check(lib().gpmppi_gp_predict(ctx.handle, _dev(q, 4 * n, "q"), n, _dev(mean, 2 * n, "mean"),
                                   _dev(var, 2 * n, "var"), _stream(stream)))


def gpmppi_plant_shift(ctx: Context, x, x_out, U, amplitude: float, stream=None):
    T = ctx.params["T"]
    _check(lib().gpmppi_plant_shift(ctx.handle, _dev(x, 5, "x"), _dev(x_out, 5, "x_out"), _dev(U, 2 * T, "U"),
                                    float(amplitude), _stream(stream)))


def gpmppi_closed_loop(ctx: Context, x, U, seed0: int, n: int, amplitude: float, x_hist=None, U0_hist=None,
                       use_graph: bool = False, stream=None):
    T = ctx.params["T"]
    _check(lib().gpmppi_closed_loop(ctx.handle, _dev(x, 5, "x"), _dev(U, 2 * T, "U"), ctypes.c_uint64(seed0),
                                    int(n), float(amplitude), _dev(x_hist, 5 * (n + 1), "x_hist", optional=True),
                                    _dev(U0_hist, 2 * n, "U0_hist", optional=True), int(bool(use_graph)),
                                    _stream(stream)))


def gpmppi_philox(seed: int, ctr, out, stream=None):
    n = int(ctr.shape[0])
    _check(lib().gpmppi_philox(ctypes.c_uint64(seed), _dev(ctr, 4 * n, "ctr", "int32"), n,
                               _dev(out, 4 * n, "out", "int32"), _stream(stream)))


def gpmppi_status_flags(ctx: Context) -> int:
    f = ctypes.c_uint32()
    _check(lib().gpmppi_status_flags(ctx.handle, ctypes.byref(f)))
    return f.value


def gpmppi_info(ctx: Context):
    m, z, c = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
    _check(lib().gpmppi_info(ctx.handle, ctypes.byref(m), ctypes.byref(z), ctypes.byref(c)))
    return m.value, z.value, c.value


def gpmppi_norm_quantile(p: float) -> float:
    return lib().gpmppi_norm_quantile(float(p))


class Controller:
    """Convenience wrapper: device buffers for one problem and step()."""

    def __init__(self, problem, precision: int = FP32, device: str = "cuda"):
        import torch
        self.torch = torch
        self.problem = problem
        self.ctx = gpmppi_init(problem, precision)
        f32 = dict(device=device, dtype=torch.float32)
        self.costs = torch.empty(problem.K, **f32)
        self.weights = torch.empty(problem.K, **f32)

    def step(self, x0, U, seed: int, stream=None):
        torch = self.torch
        U_out = torch.empty_like(U)
        gpmppi_step(self.ctx, x0, U, seed, U_out, self.costs, self.weights, stream)
        return U_out, self.costs, self.weights


def gpmppi_destroy(ctx: Context):
    """Frees the context's device buffers now (otherwise done when it is collected)."""
    if ctx.handle:
        lib().gpmppi_destroy(ctx.handle)
        ctx.handle = None


def gpmppi_last_error() -> str:
    return lib().gpmppi_last_error().decode()


class Batch:
    """Owns a gpmppi_batch; destroyed with the object."""

    def __init__(self, handle: int, problems, U_off, K_off):
        self.handle = ctypes.c_void_p(handle)
        self.n = len(problems)
        self.U_off = U_off
        self.K_off = K_off

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.gpmppi_batch_destroy(self.handle)
            self.handle = None


def gpmppi_batch_init(problems, precision: int = FP32) -> Batch:
    keep: list = []
    n = len(problems)
    params = (gpmppi_params * n)(*[make_params(p, precision) for p in problems])
    gps = (gpmppi_gp * (2 * n))()
    obs = (gpmppi_obstacles * n)()
    paths = (gpmppi_path * n)()
    for i, p in enumerate(problems):
        g = _gp_structs(p, keep)
        gps[2 * i], gps[2 * i + 1] = g[0], g[1]
        obs[i], paths[i] = _world_structs(p, keep)
    h = ctypes.c_void_p()
    _check(lib().gpmppi_batch_init(n, params, gps, obs, paths, ctypes.byref(h)))
    U_off = (ctypes.c_int64 * (n + 1))()
    K_off = (ctypes.c_int64 * (n + 1))()
    _check(lib().gpmppi_batch_layout(h, U_off, K_off))
    return Batch(h.value, problems, list(U_off), list(K_off))


def gpmppi_batch_layout(b: Batch):
    return b.U_off, b.K_off


def gpmppi_batch_step(b: Batch, x0, U, seed: int, U_out, costs, weights=None, stream=None):
    nU, nK = b.U_off[-1], b.K_off[-1]
    _check(lib().gpmppi_batch_step(b.handle, _dev(x0, 5 * b.n, "x0"), _dev(U, nU, "U"), ctypes.c_uint64(seed),
                                   _dev(U_out, nU, "U_out"), _dev(costs, nK, "costs"),
                                   _dev(weights, nK, "weights", optional=True), _stream(stream)))


def gpmppi_batch_closed_loop(b: Batch, x, U, seed0: int, n_steps: int, amplitude: float, x_hist=None,
                             use_graph: bool = False, stream=None):
    _check(lib().gpmppi_batch_closed_loop(b.handle, _dev(x, 5 * b.n, "x"), _dev(U, b.U_off[-1], "U"),
                                          ctypes.c_uint64(seed0), int(n_steps), float(amplitude),
                                          _dev(x_hist, 5 * b.n * (n_steps + 1), "x_hist", optional=True),
                                          int(bool(use_graph)), _stream(stream)))


def gpmppi_grad(ctx: Context, x0, U, seed: int, tau: float, checkpoint_every: int, J, dU, dlog_ell, dlog_sf,
                costs=None, stream=None):
    K, T = ctx.params["K"], ctx.params["T"]
    _check(lib().gpmppi_grad(ctx.handle, _dev(x0, 5, "x0"), _dev(U, 2 * T, "U"), ctypes.c_uint64(seed), float(tau),
                             int(checkpoint_every), _dev(J, 1, "J"), _dev(dU, 2 * T, "dU"),
                             _dev(dlog_ell, 8, "dlog_ell"), _dev(dlog_sf, 2, "dlog_sf"),
                             _dev(costs, K, "costs", optional=True), _stream(stream)))


GRAD_SCRATCH_BYTES = 128 << 20   # GPMPPI_GRAD_SCRATCH_BYTES


def gpmppi_grad_noalloc(ctx: Context, x0, U, seed: int, tau: float, checkpoint_every: int, J, dU, dlog_ell,
                        dlog_sf, costs=None, stream=None):
    """gpmppi_grad without any device allocation (the library's per-GPU scratch array)."""
    K, T = ctx.params["K"], ctx.params["T"]
    _check(lib().gpmppi_grad_noalloc(ctx.handle, _dev(x0, 5, "x0"), _dev(U, 2 * T, "U"), ctypes.c_uint64(seed),
                                     float(tau), int(checkpoint_every), _dev(J, 1, "J"), _dev(dU, 2 * T, "dU"),
                                     _dev(dlog_ell, 8, "dlog_ell"), _dev(dlog_sf, 2, "dlog_sf"),
                                     _dev(costs, K, "costs", optional=True), _stream(stream)))


class GradProblem:
    """A context for the differentiation form: holds the GP data to rebuild the
    GP when the hyperparameters change, the start state and the seed."""

    def __init__(self, problem, seed=None, tau: float = 0.05, checkpoint_every: int = 10, x0=None):
        import torch
        self.problem = problem
        self.ctx = gpmppi_init(problem, FP32)
        self.seed = problem.seed if seed is None else seed
        self.tau = tau
        self.checkpoint_every = min(checkpoint_every, problem.T)
        self.x0 = torch.as_tensor(np.asarray(problem.x0 if x0 is None else x0), dtype=torch.float32, device="cuda")
        self._hyper = (np.array(problem.log_ell, dtype=np.float64), np.array(problem.log_sf, dtype=np.float64))

    def set_hyper(self, log_ell, log_sf):
        le = np.asarray(log_ell, dtype=np.float64).reshape(2, 4)
        ls = np.asarray(log_sf, dtype=np.float64).reshape(2)
        if np.array_equal(le, self._hyper[0]) and np.array_equal(ls, self._hyper[1]):
            return
        import copy
        pr = copy.copy(self.problem)
        pr.log_ell, pr.log_sf = le, ls
        gpmppi_set_gp(self.ctx, pr)
        self._hyper = (le, ls)

    def evaluate(self, U, log_ell, log_sf):
        """(J, dU, dlog_ell, dlog_sf) as device tensors."""
        import torch
        self.set_hyper(log_ell, log_sf)
        f32 = dict(dtype=torch.float32, device="cuda")
        U = torch.as_tensor(U, **f32).contiguous()
        J, dU = torch.empty(1, **f32), torch.empty_like(U)
        dle, dls = torch.empty((2, 4), **f32), torch.empty(2, **f32)
        gpmppi_grad(self.ctx, self.x0, U, self.seed, self.tau, self.checkpoint_every, J, dU, dle, dls)
        return J, dU, dle, dls


def expected_cost(gp: GradProblem, U, log_ell, log_sf):
    """J(U, log_ell, log_sf) as a differentiable torch scalar (the adjoint rollout
    supplies the gradient)."""
    import torch

    class _ExpectedCost(torch.autograd.Function):
        @staticmethod
        def forward(fctx, U_, le_, ls_):
            J, dU, dle, dls = gp.evaluate(U_.detach(), le_.detach().cpu().numpy(), ls_.detach().cpu().numpy())
            fctx.save_for_backward(dU.to(U_.device, U_.dtype), dle.to(le_.device, le_.dtype),
                                   dls.to(ls_.device, ls_.dtype))
            return J[0].to(U_.device, U_.dtype)

        @staticmethod
        def backward(fctx, gJ):
            dU, dle, dls = fctx.saved_tensors
            return gJ.to(dU.device) * dU, gJ.to(dle.device) * dle, gJ.to(dls.device) * dls

    return _ExpectedCost.apply(U, log_ell, log_sf)


def gpmppi_tune(ctx: Context, x0, U, seed: int, reps: int = 3, stream=None) -> dict:
    t = gpmppi_tuning()
    _check(lib().gpmppi_tune(ctx.handle, _dev(x0, 5, "x0"), _dev(U, 2 * ctx.params["T"], "U"),
                             ctypes.c_uint64(seed), int(reps), ctypes.byref(t), _stream(stream)))
    return t.as_dict()


def gpmppi_set_tuning(ctx: Context, groups: int, rotate: int, waves: int = 4, split: int = 0):
    t = gpmppi_tuning(groups, rotate, 1, 0, waves, split, 0.0)
    _check(lib().gpmppi_set_tuning(ctx.handle, ctypes.byref(t)))


def gpmppi_set_exchange_spin(ctx: Context, polls: int):
    _check(lib().gpmppi_set_exchange_spin(ctx.handle, polls))


def gpmppi_set_grad_split(ctx: Context, split: int):
    _check(lib().gpmppi_set_grad_split(ctx.handle, int(split)))


def gpmppi_get_tuning(ctx: Context) -> dict:
    t = gpmppi_tuning()
    _check(lib().gpmppi_get_tuning(ctx.handle, ctypes.byref(t)))
    return t.as_dict()


def gpmppi_batch_tune(b: Batch, x0, U, seed: int, reps: int = 2, stream=None) -> dict:
    t = gpmppi_tuning()
    _check(lib().gpmppi_batch_tune(b.handle, _dev(x0, 5 * b.n, "x0"), _dev(U, b.U_off[-1], "U"),
                                   ctypes.c_uint64(seed), int(reps), ctypes.byref(t), _stream(stream)))
    return t.as_dict()


def gpmppi_batch_set_tuning(b: Batch, groups: int, rotate: int, wg_per_cu: int, order: int, waves: int = 4):
    t = gpmppi_tuning(groups, rotate, wg_per_cu, order, waves, 0, 0.0)
    _check(lib().gpmppi_batch_set_tuning(b.handle, ctypes.byref(t)))


def gpmppi_batch_get_tuning(b: Batch) -> dict:
    t = gpmppi_tuning()
    _check(lib().gpmppi_batch_get_tuning(b.handle, ctypes.byref(t)))
    return t.as_dict()


def gpmppi_batch_destroy(b: Batch):
    if b.handle:
        lib().gpmppi_batch_destroy(b.handle)
        b.handle = None

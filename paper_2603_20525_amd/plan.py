"""ctypes binding of libplan (include/plan.h).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of ``libplan.so``. Device buffers are torch tensors (contiguous,
float32, on the GPU); their ``data_ptr()`` is passed through the C ABI. The
library must have been built (``python -m paper_2603_20525_amd.build``);
importing this module on a machine without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libplan.so")

PLAN_OK, PLAN_EINVAL, PLAN_ENOMEM, PLAN_EDEVICE, PLAN_ENOTERRAIN = 0, -1, -2, -3, -4
PLAN_ARGMIN, PLAN_SOFTMIN = 0, 1
STATUS_NAMES = {0: "PLAN_OK", -1: "PLAN_EINVAL", -2: "PLAN_ENOMEM", -3: "PLAN_EDEVICE",
                -4: "PLAN_ENOTERRAIN"}


class PlanError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str):
        super().__init__(f"{fn} -> {STATUS_NAMES.get(status, status)}: {detail}")
        self.status = status


class Vehicle(C.Structure):
    _fields_ = [(n, C.c_float) for n in (
        "M", "Jxx", "Jyy", "Jzz", "Lf", "Lr", "e", "hR", "kf", "kr", "bf", "br",
        "C", "mu", "delta_max", "delta_rate_max", "g")]


class Cost(C.Structure):
    _fields_ = [(n, C.c_float) for n in (
        "w_t", "w_c", "w_g", "goal_x", "goal_y", "goal_r", "sigma", "eps_esm", "eps_dist")]


class Integ(C.Structure):
    _fields_ = [("dt", C.c_float), ("substeps", C.c_int), ("accel_max", C.c_float),
                ("vx_min", C.c_float)]


# every symbol include/plan.h declares
EXPORTS = ("plan_create", "plan_set_stream", "plan_set_cost", "plan_set_terrain",
           "plan_rollout", "plan_rollout_chunk", "plan_init_state", "plan_select",
           "plan_set_launch", "plan_get_launch", "plan_enable_timing", "plan_last_rollout_ms",
           "plan_destroy", "plan_last_error")

_lib = None


def lib():
    """Load libplan.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2603_20525_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, ip, fp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_float)
        L.plan_create.argtypes = [C.POINTER(vp), C.POINTER(Vehicle), C.POINTER(Cost),
                                  C.POINTER(Integ), C.c_int, C.c_int, C.c_int, C.c_int, vp]
        L.plan_set_stream.argtypes = [vp, vp]
        L.plan_set_cost.argtypes = [vp, C.POINTER(Cost)]
        L.plan_set_terrain.argtypes = [vp, vp, C.c_int, C.c_int, C.c_float, C.c_float,
                                       C.c_float, vp]
        L.plan_rollout.argtypes = [vp, fp, vp, C.c_int, C.c_int, vp, vp]
        L.plan_rollout_chunk.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_int]
        L.plan_init_state.argtypes = [vp, fp, vp, vp, C.c_int]
        L.plan_select.argtypes = [vp, C.c_int, C.c_float, vp, vp, C.c_int, C.c_int, ip, fp, vp]
        L.plan_set_launch.argtypes = [vp, C.c_int, C.c_int]
        L.plan_get_launch.argtypes = [vp, ip, ip]
        L.plan_enable_timing.argtypes = [vp, C.c_int]
        L.plan_last_rollout_ms.argtypes = [vp, fp]
        L.plan_destroy.argtypes = [vp]
        L.plan_destroy.restype = None
        L.plan_last_error.argtypes = [vp]
        L.plan_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("plan_destroy", "plan_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(fn: str, st: int, ctx=None):
    if st != PLAN_OK:
        detail = lib().plan_last_error(ctx)
        raise PlanError(fn, st, detail.decode() if detail else "")


def _dptr(t, name, numel=None):
    """Device address of a contiguous float32 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda or t.dtype.__str__() != "torch.float32" or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 GPU tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return C.c_void_p(t.data_ptr())


def _struct(cls, d):
    return cls(**{k: (int(d[k]) if t is C.c_int else float(d[k])) for k, t in cls._fields_
                  if k in d})


def _stream_handle(stream):
    if stream is None:
        return None
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ------------------------------------------------------- ABI-named functions

def plan_create(vehicle: dict, cost: dict, integ: dict, max_K: int, max_N: int,
                max_W: int, max_H: int, stream=None):
    h = C.c_void_p()
    v, c, i = _struct(Vehicle, vehicle), _struct(Cost, cost), _struct(Integ, integ)
    st = lib().plan_create(C.byref(h), C.byref(v), C.byref(c), C.byref(i), int(max_K),
                           int(max_N), int(max_W), int(max_H), _stream_handle(stream))
    _check("plan_create", st, None)
    return h


def plan_set_stream(ctx, stream):
    _check("plan_set_stream", lib().plan_set_stream(ctx, _stream_handle(stream)), ctx)


def plan_set_cost(ctx, cost: dict):
    c = _struct(Cost, cost)
    _check("plan_set_cost", lib().plan_set_cost(ctx, C.byref(c)), ctx)


def plan_set_terrain(ctx, height, x0: float, y0: float, res: float, costmap=None):
    H, W = height.shape
    st = lib().plan_set_terrain(ctx, _dptr(height, "height"), W, H, float(x0), float(y0),
                                float(res), _dptr(costmap, "costmap", H * W))
    _check("plan_set_terrain", st, ctx)


def plan_rollout(ctx, state0, controls, cost, final_state=None):
    """state0: 13 host floats; controls [N][2][K], cost [K], final_state [13][K] on GPU."""
    N, two, K = controls.shape
    if two != 2:
        raise ValueError("controls must be [N][2][K]")
    s0 = (C.c_float * 13)(*[float(v) for v in state0])
    st = lib().plan_rollout(ctx, s0, _dptr(controls, "controls"), K, N,
                            _dptr(cost, "cost", K),
                            _dptr(final_state, "final_state", 13 * K))
    _check("plan_rollout", st, ctx)


def plan_rollout_chunk(ctx, state, cost, controls, n0: int, n1: int, finalize: bool):
    """Advance state [13][K] and running cost [K] (GPU, in place) through
    control intervals [n0, n1) of controls [N][2][K]."""
    N, two, K = controls.shape
    if two != 2:
        raise ValueError("controls must be [N][2][K]")
    st = lib().plan_rollout_chunk(ctx, _dptr(state, "state", 13 * K), _dptr(cost, "cost", K),
                                  _dptr(controls, "controls"), K, N, int(n0), int(n1),
                                  int(bool(finalize)))
    _check("plan_rollout_chunk", st, ctx)


def plan_init_state(ctx, state0, state, cost):
    K = cost.numel()
    s0 = (C.c_float * 13)(*[float(v) for v in state0])
    st = lib().plan_init_state(ctx, s0, _dptr(state, "state", 13 * K), _dptr(cost, "cost", K), K)
    _check("plan_init_state", st, ctx)


def plan_select(ctx, controls, cost, plan, mode: int = PLAN_ARGMIN, lam: float = 0.0,
                want_result: bool = True):
    """Returns (best_k, best_cost) when want_result, else None (no sync)."""
    N, _, K = controls.shape
    bk, bc = C.c_int(0), C.c_float(0)
    st = lib().plan_select(ctx, int(mode), float(lam), _dptr(controls, "controls"),
                           _dptr(cost, "cost", K), K, N,
                           C.byref(bk) if want_result else None,
                           C.byref(bc) if want_result else None,
                           _dptr(plan, "plan", 2 * N))
    _check("plan_select", st, ctx)
    return (bk.value, bc.value) if want_result else None


def plan_set_launch(ctx, lanes: int = 0, block: int = 0):
    _check("plan_set_launch", lib().plan_set_launch(ctx, int(lanes), int(block)), ctx)


def plan_get_launch(ctx):
    l, b = C.c_int(0), C.c_int(0)
    _check("plan_get_launch", lib().plan_get_launch(ctx, C.byref(l), C.byref(b)), ctx)
    return l.value, b.value


def plan_enable_timing(ctx, on: bool = True):
    _check("plan_enable_timing", lib().plan_enable_timing(ctx, int(bool(on))), ctx)


def plan_last_rollout_ms(ctx) -> float:
    ms = C.c_float(0)
    _check("plan_last_rollout_ms", lib().plan_last_rollout_ms(ctx, C.byref(ms)), ctx)
    return ms.value


def plan_destroy(ctx):
    if ctx:
        lib().plan_destroy(ctx)


def plan_last_error(ctx=None) -> str:
    s = lib().plan_last_error(ctx)
    return s.decode() if s else ""


# ------------------------------------------------------------- convenience

class Planner:
    """Owns one libplan context bound to torch's current stream."""

    def __init__(self, vehicle, cost, integ, max_K, max_N, max_W, max_H, stream=None):
        import torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ctx = plan_create(vehicle, cost, integ, max_K, max_N, max_W, max_H, self.stream)

    def close(self):
        if getattr(self, "ctx", None):
            plan_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_cost(self, cost):
        plan_set_cost(self.ctx, cost)

    def set_terrain(self, height, x0, y0, res, costmap=None):
        plan_set_terrain(self.ctx, height, x0, y0, res, costmap)

    def rollout(self, state0, controls, cost, final_state=None):
        plan_rollout(self.ctx, state0, controls, cost, final_state)

    def rollout_chunk(self, state, cost, controls, n0, n1, finalize):
        plan_rollout_chunk(self.ctx, state, cost, controls, n0, n1, finalize)

    def init_state(self, state0, state, cost):
        plan_init_state(self.ctx, state0, state, cost)

    def select(self, controls, cost, plan, mode=PLAN_ARGMIN, lam=0.0, want_result=True):
        return plan_select(self.ctx, controls, cost, plan, mode, lam, want_result)

    def set_launch(self, lanes=0, block=0):
        plan_set_launch(self.ctx, lanes, block)

    def get_launch(self):
        return plan_get_launch(self.ctx)

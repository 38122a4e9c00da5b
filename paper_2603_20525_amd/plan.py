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
PLAN_SAMPLE_UNIFORM, PLAN_SAMPLE_GAUSSIAN = 0, 1
PLAN_EULER, PLAN_RK4 = 0, 1
PLAN_ORDER_AUTO, PLAN_ORDER_OFF, PLAN_ORDER_ON = 0, 1, 2
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
        "w_t", "w_c", "w_g", "goal_x", "goal_y", "goal_r", "sigma", "eps_esm", "eps_dist",
        "eps_ay")]


class Integ(C.Structure):
    _fields_ = [("dt", C.c_float), ("substeps", C.c_int), ("accel_max", C.c_float),
                ("vx_min", C.c_float), ("method", C.c_int)]


class Sample(C.Structure):
    _fields_ = [("kind", C.c_int), ("keep_nominal", C.c_int), ("seed", C.c_ulonglong),
                ("stream", C.c_ulonglong), ("scale", C.c_float * 2),
                ("nominal_dev", C.c_void_p)]


# every symbol include/plan.h declares
EXPORTS = ("plan_create", "plan_set_stream", "plan_set_cost", "plan_set_terrain",
           "plan_rollout", "plan_rollout_est", "plan_rollout_chunk", "plan_init_state", "plan_rollout_grad",
           "plan_rollout_grad_noalloc",
           "plan_select", "plan_sample_controls", "plan_rollout_sampled", "plan_select_sampled",
           "plan_rollout_argmin", "plan_rollout_sampled_argmin",
           "plan_smooth_terrain", "plan_costmap_polygons",
           "plan_set_launch", "plan_get_launch", "plan_set_order", "plan_get_order",
           "plan_enable_timing", "plan_last_rollout_ms",
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
        L.plan_rollout_est.argtypes = [vp, fp, vp, C.c_int, C.c_int, vp, vp]
        L.plan_rollout_chunk.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.c_int]
        L.plan_init_state.argtypes = [vp, fp, vp, vp, C.c_int]
        L.plan_rollout_grad.argtypes = [vp, fp, vp, C.c_int, C.c_int, vp, C.c_int, vp, vp]
        L.plan_rollout_grad_noalloc.argtypes = L.plan_rollout_grad.argtypes
        L.plan_select.argtypes = [vp, C.c_int, C.c_float, vp, vp, C.c_int, C.c_int, ip, fp, vp]
        sp = C.POINTER(Sample)
        L.plan_sample_controls.argtypes = [vp, sp, C.c_int, C.c_int, vp]
        L.plan_rollout_sampled.argtypes = [vp, fp, sp, C.c_int, C.c_int, vp, vp]
        L.plan_select_sampled.argtypes = [vp, sp, vp, C.c_int, C.c_int, ip, fp, vp]
        L.plan_rollout_argmin.argtypes = [vp, fp, vp, C.c_int, C.c_int, vp, vp, vp, ip, fp]
        L.plan_rollout_sampled_argmin.argtypes = [vp, fp, sp, C.c_int, C.c_int, vp, vp, vp, ip,
                                                  fp]
        L.plan_smooth_terrain.argtypes = [vp, vp, C.c_int, C.c_int, C.c_float, C.c_float, vp]
        L.plan_costmap_polygons.argtypes = [vp, vp, C.c_int, ip, ip, C.c_int, C.c_int, C.c_int,
                                            C.c_float, C.c_float, C.c_float, C.c_float,
                                            C.c_float, C.c_int, vp]
        L.plan_set_launch.argtypes = [vp, C.c_int, C.c_int]
        L.plan_get_launch.argtypes = [vp, ip, ip]
        L.plan_set_order.argtypes = [vp, C.c_int]
        L.plan_get_order.argtypes = [vp, ip]
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


_F32 = None


def _dptr(t, name, numel=None):
    """Device address (int) of a contiguous float32 CUDA tensor (None -> NULL)."""
    global _F32
    if t is None:
        return None
    if _F32 is None:
        import torch
        _F32 = torch.float32
    if not t.is_cuda or t.dtype is not _F32 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 GPU tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return t.data_ptr()


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


def plan_rollout_est(ctx, state0, controls, cost, final_state=None):
    """EST formulation: state0 7 host floats (x, y, psi, v_y, omega_z, delta,
    v_x); controls [N][2][K], cost [K], final_state [7][K] on the GPU."""
    N, two, K = controls.shape
    if two != 2:
        raise ValueError("controls must be [N][2][K]")
    if len(state0) != 7:
        raise ValueError("state0 must have 7 entries")
    s0 = (C.c_float * 7)(*[float(v) for v in state0])
    st = lib().plan_rollout_est(ctx, s0, _dptr(controls, "controls"), K, N,
                                _dptr(cost, "cost", K), _dptr(final_state, "final_state", 7 * K))
    _check("plan_rollout_est", st, ctx)


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


def plan_rollout_grad(ctx, state0, controls, cost, grad, weight=None, checkpoint_every=10):
    """cost [K] and grad [N][2][K] (GPU) receive J and w_k dJ_k/du."""
    N, two, K = controls.shape
    if two != 2:
        raise ValueError("controls must be [N][2][K]")
    s0 = (C.c_float * 13)(*[float(v) for v in state0])
    st = lib().plan_rollout_grad(ctx, s0, _dptr(controls, "controls"), K, N,
                                 _dptr(weight, "weight", K), int(checkpoint_every),
                                 _dptr(cost, "cost", K), _dptr(grad, "grad", 2 * N * K))
    _check("plan_rollout_grad", st, ctx)


def plan_rollout_grad_noalloc(ctx, state0, controls, cost, grad, weight=None,
                              checkpoint_every=10):
    """plan_rollout_grad on the library's fixed per-GPU workspace (no
    allocation; calls on one GPU must not overlap)."""
    N, two, K = controls.shape
    if two != 2:
        raise ValueError("controls must be [N][2][K]")
    s0 = (C.c_float * 13)(*[float(v) for v in state0])
    st = lib().plan_rollout_grad_noalloc(ctx, s0, _dptr(controls, "controls"), K, N,
                                         _dptr(weight, "weight", K), int(checkpoint_every),
                                         _dptr(cost, "cost", K), _dptr(grad, "grad", 2 * N * K))
    _check("plan_rollout_grad_noalloc", st, ctx)


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


def sample_spec(kind: int, seed: int, stream: int, scale, nominal=None,
                keep_nominal: bool = False, N: int | None = None) -> Sample:
    """plan_sample_t for the generator; nominal is a [N][2] float32 GPU tensor
    or None. The tensor must outlive the calls that use the spec."""
    if nominal is not None and N is not None and nominal.numel() != 2 * N:
        raise ValueError("nominal must be [N][2]")
    return Sample(kind=int(kind), keep_nominal=int(bool(keep_nominal)), seed=int(seed),
                  stream=int(stream), scale=(C.c_float * 2)(float(scale[0]), float(scale[1])),
                  nominal_dev=_dptr(nominal, "nominal"))


def plan_sample_controls(ctx, spec: Sample, controls):
    """Fill controls [N][2][K] (GPU) from the generator."""
    N, two, K = controls.shape
    if two != 2:
        raise ValueError("controls must be [N][2][K]")
    st = lib().plan_sample_controls(ctx, C.byref(spec), K, N, _dptr(controls, "controls"))
    _check("plan_sample_controls", st, ctx)


def plan_rollout_sampled(ctx, state0, spec: Sample, N: int, cost, final_state=None):
    """Roll out cost.numel() candidates drawn inside the kernel from spec."""
    K = cost.numel()
    s0 = (C.c_float * 13)(*[float(v) for v in state0])
    st = lib().plan_rollout_sampled(ctx, s0, C.byref(spec), K, int(N), _dptr(cost, "cost", K),
                                    _dptr(final_state, "final_state", 13 * K))
    _check("plan_rollout_sampled", st, ctx)


def plan_select_sampled(ctx, spec: Sample, cost, plan, want_result: bool = True):
    """Argmin over cost [K]; plan [N][2] gets the winner's regenerated controls."""
    K = cost.numel()
    N = plan.numel() // 2
    bk, bc = C.c_int(0), C.c_float(0)
    st = lib().plan_select_sampled(ctx, C.byref(spec), _dptr(cost, "cost", K), K, N,
                                   C.byref(bk) if want_result else None,
                                   C.byref(bc) if want_result else None,
                                   _dptr(plan, "plan", 2 * N))
    _check("plan_select_sampled", st, ctx)
    return (bk.value, bc.value) if want_result else None


def plan_rollout_argmin(ctx, state0, controls, cost, plan, final_state=None,
                        want_result: bool = True, _bufs=None):
    """Rollout and argmin in one launch; returns (best_k, best_cost) when
    want_result (waits), else None. _bufs: reusable (state0 array, int,
    float) ctypes objects of the caller."""
    N, two, K = controls.shape
    if two != 2:
        raise ValueError("controls must be [N][2][K]")
    if _bufs is None:
        s0 = (C.c_float * 13)(*[float(v) for v in state0])
        bk, bc = C.c_int(0), C.c_float(0)
    else:
        s0, bk, bc = _bufs
        s0[:] = state0
    st = lib().plan_rollout_argmin(ctx, s0, _dptr(controls, "controls"), K, N,
                                   _dptr(cost, "cost", K),
                                   _dptr(final_state, "final_state", 13 * K),
                                   _dptr(plan, "plan", 2 * N),
                                   C.byref(bk) if want_result else None,
                                   C.byref(bc) if want_result else None)
    _check("plan_rollout_argmin", st, ctx)
    return (bk.value, bc.value) if want_result else None


def plan_rollout_sampled_argmin(ctx, state0, spec: Sample, N: int, cost, plan,
                                final_state=None, want_result: bool = True):
    """Sampled rollout and argmin in one launch."""
    K = cost.numel()
    s0 = (C.c_float * 13)(*[float(v) for v in state0])
    bk, bc = C.c_int(0), C.c_float(0)
    st = lib().plan_rollout_sampled_argmin(ctx, s0, C.byref(spec), K, int(N),
                                           _dptr(cost, "cost", K),
                                           _dptr(final_state, "final_state", 13 * K),
                                           _dptr(plan, "plan", 2 * int(N)),
                                           C.byref(bk) if want_result else None,
                                           C.byref(bc) if want_result else None)
    _check("plan_rollout_sampled_argmin", st, ctx)
    return (bk.value, bc.value) if want_result else None


def plan_smooth_terrain(ctx, height, res: float, sigma: float, out):
    """Gaussian level-of-detail smoothing of height [H][W] into out [H][W] (GPU)."""
    H, W = height.shape
    st = lib().plan_smooth_terrain(ctx, _dptr(height, "height"), W, H, float(res), float(sigma),
                                   _dptr(out, "out", H * W))
    _check("plan_smooth_terrain", st, ctx)


def plan_costmap_polygons(ctx, verts, offsets, kinds, costmap, x0: float, y0: float,
                          res: float, sigma: float, eps_dist: float, accumulate=False):
    """Distance-constraint costmap [H][W] (GPU) from polygons: verts [V][2]
    (GPU float32), offsets [P+1] and kinds [P] (host int sequences)."""
    H, W = costmap.shape
    P = len(kinds)
    off = (C.c_int * (P + 1))(*[int(v) for v in offsets])
    kd = (C.c_int * max(P, 1))(*[int(v) for v in kinds])
    V = 0 if verts is None else verts.shape[0]
    st = lib().plan_costmap_polygons(ctx, _dptr(verts, "verts") if V else None, V, off, kd, P,
                                     W, H, float(x0), float(y0), float(res), float(sigma),
                                     float(eps_dist), int(bool(accumulate)),
                                     _dptr(costmap, "costmap", H * W))
    _check("plan_costmap_polygons", st, ctx)


def plan_set_launch(ctx, lanes: int = 0, block: int = 0):
    _check("plan_set_launch", lib().plan_set_launch(ctx, int(lanes), int(block)), ctx)


def plan_get_launch(ctx):
    l, b = C.c_int(0), C.c_int(0)
    _check("plan_get_launch", lib().plan_get_launch(ctx, C.byref(l), C.byref(b)), ctx)
    return l.value, b.value


def plan_set_order(ctx, mode: int = 0):
    """Candidate order for gather locality: PLAN_ORDER_AUTO, _OFF or _ON."""
    _check("plan_set_order", lib().plan_set_order(ctx, int(mode)), ctx)


def plan_get_order(ctx) -> bool:
    """Whether the most recent full-horizon rollout ran in locality order."""
    o = C.c_int(0)
    _check("plan_get_order", lib().plan_get_order(ctx, C.byref(o)), ctx)
    return bool(o.value)


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
        self._bufs = None  # reusable ctypes arguments of the one-launch plan call
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

    def rollout_est(self, state0, controls, cost, final_state=None):
        plan_rollout_est(self.ctx, state0, controls, cost, final_state)

    def rollout_chunk(self, state, cost, controls, n0, n1, finalize):
        plan_rollout_chunk(self.ctx, state, cost, controls, n0, n1, finalize)

    def rollout_grad(self, state0, controls, cost, grad, weight=None, checkpoint_every=10):
        plan_rollout_grad(self.ctx, state0, controls, cost, grad, weight, checkpoint_every)

    def init_state(self, state0, state, cost):
        plan_init_state(self.ctx, state0, state, cost)

    def select(self, controls, cost, plan, mode=PLAN_ARGMIN, lam=0.0, want_result=True):
        return plan_select(self.ctx, controls, cost, plan, mode, lam, want_result)

    def sample_controls(self, spec, controls):
        plan_sample_controls(self.ctx, spec, controls)

    def rollout_sampled(self, state0, spec, N, cost, final_state=None):
        plan_rollout_sampled(self.ctx, state0, spec, N, cost, final_state)

    def select_sampled(self, spec, cost, plan, want_result=True):
        return plan_select_sampled(self.ctx, spec, cost, plan, want_result)

    def rollout_argmin(self, state0, controls, cost, plan, final_state=None, want_result=True):
        if self._bufs is None:
            self._bufs = ((C.c_float * 13)(), C.c_int(0), C.c_float(0))
        return plan_rollout_argmin(self.ctx, state0, controls, cost, plan, final_state,
                                   want_result, self._bufs)

    def rollout_sampled_argmin(self, state0, spec, N, cost, plan, final_state=None,
                               want_result=True):
        return plan_rollout_sampled_argmin(self.ctx, state0, spec, N, cost, plan, final_state,
                                           want_result)

    def smooth_terrain(self, height, res, sigma, out):
        plan_smooth_terrain(self.ctx, height, res, sigma, out)

    def costmap_polygons(self, verts, offsets, kinds, costmap, x0, y0, res, sigma, eps_dist,
                         accumulate=False):
        plan_costmap_polygons(self.ctx, verts, offsets, kinds, costmap, x0, y0, res, sigma,
                              eps_dist, accumulate)

    def set_launch(self, lanes=0, block=0):
        plan_set_launch(self.ctx, lanes, block)

    def enable_timing(self, on=True):
        plan_enable_timing(self.ctx, on)

    def last_rollout_ms(self):
        return plan_last_rollout_ms(self.ctx)

    def get_launch(self):
        return plan_get_launch(self.ctx)

    def set_order(self, mode=0):
        plan_set_order(self.ctx, mode)

    def get_order(self):
        return plan_get_order(self.ctx)


# ----------------------------------------------------- serving (plan_serve.h)

class Request(C.Structure):
    _fields_ = [("height_dev", C.c_void_p), ("W", C.c_int), ("H", C.c_int),
                ("x0", C.c_float), ("y0", C.c_float), ("res", C.c_float),
                ("costmap_dev", C.c_void_p), ("state0", C.c_float * 13),
                ("controls_dev", C.c_void_p), ("K", C.c_int), ("N", C.c_int),
                ("cost", Cost), ("integ", Integ), ("plan_dev", C.c_void_p),
                ("cost_dev", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("best_k", C.c_int), ("best_cost", C.c_float),
                ("slot", C.c_int), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double)]


SERVER_EXPORTS = ("plan_server_create", "plan_server_submit", "plan_server_step",
                  "plan_server_drain", "plan_server_stats", "plan_server_result",
                  "plan_server_completions", "plan_server_now", "plan_server_destroy",
                  "plan_server_last_error")

_server_bound = False


def _bind_server():
    global _server_bound
    L = lib()
    if not _server_bound:
        vp, ip = C.c_void_p, C.POINTER(C.c_int)
        L.plan_server_create.argtypes = [C.POINTER(vp), C.POINTER(Vehicle), C.c_int, C.c_int,
                                         C.c_int, C.c_int, C.c_int, C.c_ulonglong, C.c_int, vp]
        L.plan_server_submit.argtypes = [vp, C.POINTER(Request), ip]
        L.plan_server_step.argtypes = [vp, ip, ip]
        L.plan_server_drain.argtypes = [vp]
        L.plan_server_result.argtypes = [vp, C.c_int, C.POINTER(Result)]
        L.plan_server_stats.argtypes = [vp, ip, ip, C.POINTER(C.c_ulonglong)]
        L.plan_server_completions.argtypes = [vp, ip, C.c_int, ip]
        L.plan_server_now.argtypes = [vp]
        L.plan_server_now.restype = C.c_double
        L.plan_server_destroy.argtypes = [vp]
        L.plan_server_destroy.restype = None
        L.plan_server_last_error.argtypes = [vp]
        L.plan_server_last_error.restype = C.c_char_p
        for n in ("plan_server_create", "plan_server_submit", "plan_server_step",
                  "plan_server_drain", "plan_server_stats", "plan_server_result",
                  "plan_server_completions"):
            getattr(L, n).restype = C.c_int
        _server_bound = True
    return L


def _scheck(fn, st, h):
    if st != PLAN_OK:
        d = _bind_server().plan_server_last_error(h)
        raise PlanError(fn, st, d.decode() if d else "")


class Server:
    """Continuous-batching planning server (one host thread)."""

    def __init__(self, vehicle, max_slots, max_K, max_N, max_W, max_H, budget_bytes,
                 chunk_intervals=16, stream=None):
        import torch
        self._req = Request()
        self._rid = C.c_int(-1)
        self._params = {}
        self._cbuf = {}
        self._cn, self._sa, self._sq = C.c_int(0), C.c_int(0), C.c_int(0)
        L = _bind_server()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        v = _struct(Vehicle, vehicle)
        st = L.plan_server_create(C.byref(h), C.byref(v), int(max_slots), int(max_K), int(max_N),
                                  int(max_W), int(max_H), C.c_ulonglong(int(budget_bytes)),
                                  int(chunk_intervals), _stream_handle(self.stream))
        _scheck("plan_server_create", st, None)
        self.h = h
        self._keep = {}

    def submit(self, height, x0, y0, res, state0, controls, cost, integ, plan, costmap=None,
               costs_out=None):
        """All tensors are kept referenced until the request is read back.
        costs_out ([K], optional) receives every candidate's cost."""
        H, W = height.shape
        N, two, K = controls.shape
        # the library copies the request, so one Request object is reused
        r = self._req
        r.height_dev = _dptr(height, "height")
        r.W, r.H = W, H
        r.x0, r.y0, r.res = float(x0), float(y0), float(res)
        r.costmap_dev = None if costmap is None else _dptr(costmap, "costmap", H * W)
        r.state0[:] = state0
        r.controls_dev = _dptr(controls, "controls")
        r.K, r.N = K, N
        r.cost = self._param(Cost, cost)
        r.integ = self._param(Integ, integ)
        r.plan_dev = _dptr(plan, "plan", 2 * N)
        r.cost_dev = None if costs_out is None else _dptr(costs_out, "costs_out", K)
        rid = self._rid
        _scheck("plan_server_submit", _bind_server().plan_server_submit(self.h, C.byref(r),
                                                                         C.byref(rid)), self.h)
        self._keep[rid.value] = (height, controls, plan, costmap, costs_out)
        return rid.value

    def _param(self, cls, d):
        """ctypes copy of a parameter dict, reused while the dict's values are
        unchanged (requests usually share their cost and integration dicts)."""
        key = (cls, id(d))
        snap = tuple(d.values())
        hit = self._params.get(key)
        if hit is not None and hit[0] is d and hit[1] == snap:
            return hit[2]
        st = _struct(cls, d)
        if len(self._params) > 256:
            self._params.clear()
        self._params[key] = (d, snap, st)
        return st

    def step(self):
        a, q = self._sa, self._sq
        _scheck("plan_server_step", _bind_server().plan_server_step(self.h, C.byref(a),
                                                                     C.byref(q)), self.h)
        return a.value, q.value

    def stats(self):
        a, q, u = C.c_int(0), C.c_int(0), C.c_ulonglong(0)
        _scheck("plan_server_stats", _bind_server().plan_server_stats(
            self.h, C.byref(a), C.byref(q), C.byref(u)), self.h)
        return a.value, q.value, u.value

    def drain(self):
        _scheck("plan_server_drain", _bind_server().plan_server_drain(self.h), self.h)

    def result(self, rid) -> dict:
        r = Result()
        _scheck("plan_server_result", _bind_server().plan_server_result(self.h, int(rid),
                                                                         C.byref(r)), self.h)
        out = {n: getattr(r, n) for n, _ in Result._fields_}
        if out["status"] != 0:
            self._keep.pop(rid, None)
        return out

    def completions(self, capacity=128) -> list:
        """Ids of requests finished since the previous call, in the order
        the host observed them."""
        buf = self._cbuf.get(capacity)
        if buf is None:
            buf = self._cbuf[capacity] = (C.c_int * capacity)()
        n = self._cn
        _scheck("plan_server_completions", _bind_server().plan_server_completions(
            self.h, buf, capacity, C.byref(n)), self.h)
        return buf[:n.value] if n.value else []

    def now(self) -> float:
        return _bind_server().plan_server_now(self.h)

    def close(self):
        if getattr(self, "h", None):
            _bind_server().plan_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

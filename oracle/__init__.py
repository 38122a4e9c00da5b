"""FP64 CPU oracle for the SRB sampling planner -- TEST INFRASTRUCTURE ONLY.

This package is the correctness reference that the GPU library is checked
against. Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; the product path (the
``paper_2603_20525_amd`` package and its C library) never does, and it shares
no code with it. The arithmetic lives in ``srb_oracle.c`` (plain C, double
precision); this module only builds it and marshals arguments with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile ``srb_oracle.c`` into ``liboracle.so`` (gcc -O2, no fast-math,
    OpenMP over candidates)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Vehicle(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "M", "Jxx", "Jyy", "Jzz", "Lf", "Lr", "e", "hR", "kf", "kr", "bf", "br",
        "C", "mu", "delta_max", "delta_rate_max", "g")]


class Cost(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "w_t", "w_c", "w_g", "goal_x", "goal_y", "goal_r", "sigma", "eps_esm",
        "eps_dist", "eps_ay")]


class Integ(C.Structure):
    _fields_ = [("dt", C.c_double), ("substeps", C.c_int),
                ("accel_max", C.c_double), ("vx_min", C.c_double), ("method", C.c_int)]


class Diag(C.Structure):
    _fields_ = [
        ("P", C.c_double * 3 * 4), ("vi", C.c_double * 3 * 4),
        ("terr", C.c_double * 4 * 4),
        ("chi", C.c_double * 4), ("chidot", C.c_double * 4),
        ("Fk", C.c_double * 4), ("Fb", C.c_double * 4), ("Fz", C.c_double * 4),
        ("Fy", C.c_double * 4), ("alpha", C.c_double * 4),
        ("f", C.c_double * 3 * 4),
        ("Fy_sum", C.c_double), ("Fz_sum", C.c_double), ("Mx", C.c_double),
        ("My", C.c_double), ("Mz", C.c_double), ("c_sum", C.c_double),
        ("U_esm", C.c_double), ("L", C.c_double),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = np.ctypeslib.as_array(v).copy() if hasattr(v, "_length_") else float(v)
        return out


class EstDiag(C.Structure):
    _fields_ = [
        ("phi", C.c_double), ("theta", C.c_double), ("z", C.c_double),
        ("R", C.c_double * 3 * 3), ("gB", C.c_double * 3),
        ("alpha_f", C.c_double), ("alpha_r", C.c_double),
        ("Fz_f", C.c_double), ("Fz_r", C.c_double),
        ("Fy_f", C.c_double), ("Fy_r", C.c_double),
        ("Fz_wheel", C.c_double * 4), ("ax", C.c_double), ("ay", C.c_double),
        ("pi_ay", C.c_double), ("a_bar_y", C.c_double),
        ("P", C.c_double * 3 * 4), ("c_sum", C.c_double), ("L", C.c_double),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = np.ctypeslib.as_array(v).copy() if hasattr(v, "_length_") else float(v)
        return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp, fp, ip, vp = (C.POINTER(C.c_double), C.POINTER(C.c_float),
                          C.POINTER(C.c_int), C.c_void_p)
        L.oracle_create.restype = vp
        L.oracle_create.argtypes = [C.POINTER(Vehicle), C.POINTER(Cost), C.POINTER(Integ)]
        L.oracle_destroy.argtypes = [vp]
        L.oracle_set_terrain.argtypes = [vp, fp, C.c_int, C.c_int, C.c_double,
                                         C.c_double, C.c_double, fp]
        L.oracle_sample_terrain.argtypes = [vp, C.c_double, C.c_double, dp]
        L.oracle_rhs.argtypes = [vp, dp, C.c_double, C.c_double, dp, C.POINTER(Diag)]
        L.oracle_esm.restype = C.c_double
        L.oracle_esm.argtypes = [vp, C.c_double, C.c_double]
        L.oracle_soft.restype = C.c_double
        L.oracle_soft.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_rollout.argtypes = [vp, fp, fp, C.c_int, C.c_int, dp, dp, ip]
        L.oracle_select.argtypes = [vp, C.c_int, C.c_double, fp, fp, C.c_int,
                                    C.c_int, ip, dp, dp]
        L.oracle_rollout_span.argtypes = [vp, fp, fp, fp, C.c_int, C.c_int, C.c_int,
                                          C.c_int, C.c_int, dp, dp, dp, dp, dp]
        L.oracle_rollout_d.argtypes = [vp, dp, dp, C.c_int, C.c_int, dp, dp]
        L.oracle_set_round32.argtypes = [vp, C.c_int]
        L.oracle_set_round32.restype = None
        L.oracle_est_rhs.argtypes = [vp, dp, C.c_double, C.c_double, dp, C.POINTER(EstDiag)]
        L.oracle_est_rollout.argtypes = [vp, fp, fp, C.c_int, C.c_int, dp, dp, ip]
        L.oracle_smooth_terrain.argtypes = [fp, C.c_int, C.c_int, C.c_double, C.c_double, dp]
        L.oracle_costmap_polygons.argtypes = [dp, ip, ip, C.c_int, C.c_int, C.c_int, C.c_double,
                                              C.c_double, C.c_double, C.c_double, C.c_double, dp]
        u64p = C.POINTER(C.c_uint64)
        L.oracle_philox4x64.argtypes = [u64p, u64p, u64p]
        L.oracle_philox4x64.restype = None
        L.oracle_sample_controls.argtypes = [C.c_int, C.c_uint64, C.c_uint64, dp, C.c_int, fp,
                                             C.c_int, C.c_int, dp]
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def soft(sigma: float, eps: float, pi: float) -> float:
    return lib().oracle_soft(sigma, eps, pi)


def philox4x64(counter, key):
    """Philox4x64-10 block: four uint64 words for a 4-word counter, 2-word key."""
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().oracle_philox4x64(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(out, C.c_uint64))
    return out


SAMPLE_UNIFORM, SAMPLE_GAUSSIAN = 0, 1
OBSTACLE, PATH_BOUNDARY = 0, 1


def smooth_terrain(height, res, sigma):
    """Gaussian level-of-detail smoothing of a float32 [H][W] heightmap (double out)."""
    h = _f32(height)
    H, W = h.shape
    out = np.zeros((H, W))
    rc = lib().oracle_smooth_terrain(_ptr(h, C.c_float), W, H, float(res), float(sigma),
                                     _ptr(out, C.c_double))
    if rc != 0:
        raise ValueError("oracle_smooth_terrain rejected the arguments")
    return out


def polygon_arrays(polygons):
    """[(kind, [(x, y), ...]), ...] -> (verts [V][2] double, offsets [P+1], kinds [P])."""
    verts = np.ascontiguousarray(np.concatenate([np.asarray(v, np.float64).reshape(-1, 2)
                                                 for _, v in polygons]) if polygons
                                 else np.zeros((0, 2)))
    offsets = np.zeros(len(polygons) + 1, np.int32)
    offsets[1:] = np.cumsum([len(v) for _, v in polygons])
    kinds = np.asarray([k for k, _ in polygons], np.int32)
    return verts, offsets, kinds


def costmap_polygons(polygons, W, H, x0, y0, res, sigma, eps_dist):
    """Distance-constraint cost rate at every node (double [H][W])."""
    verts, offsets, kinds = polygon_arrays(polygons)
    out = np.zeros((H, W))
    rc = lib().oracle_costmap_polygons(_ptr(verts, C.c_double), _ptr(offsets, C.c_int),
                                       _ptr(kinds, C.c_int), len(polygons), int(W), int(H),
                                       float(x0), float(y0), float(res), float(sigma),
                                       float(eps_dist), _ptr(out, C.c_double))
    if rc != 0:
        raise ValueError("oracle_costmap_polygons rejected the arguments")
    return out


def sample_controls(kind, seed, stream, scale, K, N, nominal=None, keep_nominal=False):
    """Candidate controls [N][2][K] (double) from the counter-based generator."""
    sc = np.ascontiguousarray(scale, dtype=np.float64)
    nom = None if nominal is None else _f32(nominal).reshape(N, 2)
    out = np.zeros((N, 2, K))
    rc = lib().oracle_sample_controls(int(kind), int(seed), int(stream), _ptr(sc, C.c_double),
                                      int(bool(keep_nominal)),
                                      None if nom is None else _ptr(nom, C.c_float),
                                      int(K), int(N), _ptr(out, C.c_double))
    if rc != 0:
        raise ValueError("oracle_sample_controls rejected the arguments")
    return out


class Oracle:
    """One oracle context: parameters plus (after ``set_terrain``) a terrain."""

    def __init__(self, vehicle: dict, cost: dict, integ: dict):
        self._veh = Vehicle(**{k: float(vehicle[k]) for k, _ in Vehicle._fields_})
        self._cost = Cost(**{k: float(cost.get(k, 0.0)) for k, _ in Cost._fields_})
        self._integ = Integ(dt=float(integ["dt"]), substeps=int(integ["substeps"]),
                            accel_max=float(integ["accel_max"]),
                            vx_min=float(integ["vx_min"]), method=int(integ.get("method", 0)))
        self._h = lib().oracle_create(C.byref(self._veh), C.byref(self._cost),
                                      C.byref(self._integ))
        if not self._h:
            raise ValueError("oracle_create rejected the parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.oracle_destroy(h)
            self._h = None

    @property
    def substeps(self) -> int:
        """Euler (or RK4) steps per control interval."""
        return int(self._integ.substeps)

    def set_terrain(self, height, x0, y0, res, costmap=None):
        h = _f32(height)
        H, W = h.shape
        c = None if costmap is None else _f32(costmap)
        self._keep = (h, c)
        rc = lib().oracle_set_terrain(self._h, _ptr(h, C.c_float), W, H, x0, y0, res,
                                      None if c is None else _ptr(c, C.c_float))
        if rc != 0:
            raise ValueError("oracle_set_terrain rejected the terrain")

    def sample(self, x, y):
        out = np.zeros(4)
        lib().oracle_sample_terrain(self._h, float(x), float(y), _ptr(out, C.c_double))
        return out

    def rhs(self, xi, delta_dot, vx_dot):
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        out = np.zeros(13)
        d = Diag()
        rc = lib().oracle_rhs(self._h, _ptr(xi, C.c_double), float(delta_dot),
                              float(vx_dot), _ptr(out, C.c_double), C.byref(d))
        if rc != 0:
            raise RuntimeError("oracle_rhs failed (no terrain?)")
        return out, d.as_dict()

    def esm(self, phi, theta):
        return lib().oracle_esm(self._h, float(phi), float(theta))

    def est_rhs(self, xi, delta_dot, vx_dot):
        """EST state derivative (7) and diagnostics."""
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        out = np.zeros(7)
        d = EstDiag()
        rc = lib().oracle_est_rhs(self._h, _ptr(xi, C.c_double), float(delta_dot),
                                  float(vx_dot), _ptr(out, C.c_double), C.byref(d))
        if rc != 0:
            raise RuntimeError("oracle_est_rhs failed (no terrain?)")
        return out, d.as_dict()

    def est_rollout(self, state0, controls):
        """EST formulation: state0 [7] float32, controls [N][2][K] float32.
        Returns (cost[K], final_state[7][K], exit_step[K])."""
        s0 = _f32(state0)
        u = _f32(controls)
        N, two, K = u.shape
        assert two == 2 and s0.shape == (7,)
        cost = np.zeros(K)
        fs = np.zeros((7, K))
        ex = np.zeros(K, dtype=np.int32)
        rc = lib().oracle_est_rollout(self._h, _ptr(s0, C.c_float), _ptr(u, C.c_float), K, N,
                                      _ptr(cost, C.c_double), _ptr(fs, C.c_double),
                                      _ptr(ex, C.c_int))
        if rc != 0:
            raise RuntimeError(f"oracle_est_rollout failed ({rc})")
        return cost, fs, ex

    def rollout(self, state0, controls):
        """controls: [N][2][K] float32. Returns (cost[K], final_state[13][K], exit_step[K])."""
        s0 = _f32(state0)
        u = _f32(controls)
        N, two, K = u.shape
        assert two == 2 and s0.shape == (13,)
        cost = np.zeros(K)
        fs = np.zeros((13, K))
        ex = np.zeros(K, dtype=np.int32)
        rc = lib().oracle_rollout(self._h, _ptr(s0, C.c_float), _ptr(u, C.c_float), K, N,
                                  _ptr(cost, C.c_double), _ptr(fs, C.c_double),
                                  _ptr(ex, C.c_int))
        if rc != 0:
            raise RuntimeError(f"oracle_rollout failed ({rc})")
        return cost, fs, ex

    def rollout_span(self, state_in, cost_in, controls, n0, n1, finalize, margins=False):
        """Continue from per-candidate float32 states [13][K] and running costs
        [K] over control intervals [n0, n1). Returns (state_out [13][K],
        cost_out [K]) in double, plus (touchdown margin [K], slip margin [K],
        largest |roll| or |pitch| [K]) when margins is set."""
        si = _f32(state_in)
        ci = _f32(cost_in)
        u = _f32(controls)
        N, _, K = u.shape
        assert si.shape == (13, K) and ci.shape == (K,)
        so = np.zeros((13, K))
        co = np.zeros(K)
        td = np.zeros(K)
        sl = np.zeros(K)
        tl = np.zeros(K)
        rc = lib().oracle_rollout_span(self._h, _ptr(si, C.c_float), _ptr(ci, C.c_float),
                                       _ptr(u, C.c_float), K, N, int(n0), int(n1),
                                       int(bool(finalize)), _ptr(so, C.c_double),
                                       _ptr(co, C.c_double), _ptr(td, C.c_double),
                                       _ptr(sl, C.c_double), _ptr(tl, C.c_double))
        if rc != 0:
            raise RuntimeError(f"oracle_rollout_span failed ({rc})")
        return (so, co, td, sl, tl) if margins else (so, co)

    def rollout_d(self, state0, controls):
        """Double-precision inputs: state0 [13], controls [N][2][K]. Returns
        (cost [K], final_state [13][K])."""
        s0 = np.ascontiguousarray(state0, dtype=np.float64)
        u = np.ascontiguousarray(controls, dtype=np.float64)
        N, _, K = u.shape
        cost = np.zeros(K)
        fs = np.zeros((13, K))
        rc = lib().oracle_rollout_d(self._h, _ptr(s0, C.c_double), _ptr(u, C.c_double), K, N,
                                    _ptr(cost, C.c_double), _ptr(fs, C.c_double))
        if rc != 0:
            raise RuntimeError(f"oracle_rollout_d failed ({rc})")
        return cost, fs

    def fd_grad(self, state0, controls, k, entries, step=1e-6):
        """FP64 central differences dJ_k/du[n][c] for (n, c) in entries, with
        the one-sided differences (for detecting a kink in between)."""
        u = np.ascontiguousarray(controls[:, :, k:k + 1], dtype=np.float64)
        s0 = np.asarray(state0, dtype=np.float64)
        cols = []
        for n, c in entries:
            up, dn = u.copy(), u.copy()
            up[n, c, 0] += step
            dn[n, c, 0] -= step
            cols += [up, dn]
        U = np.concatenate([u] + cols, axis=2)
        J, _ = self.rollout_d(s0, U)
        J0, Jp, Jm = J[0], J[1::2], J[2::2]
        return (Jp - Jm) / (2 * step), (Jp - J0) / step, (J0 - Jm) / step

    def set_round32(self, on: bool):
        """Conditioning probe: round state and running cost to float after each step."""
        lib().oracle_set_round32(self._h, int(bool(on)))

    def select(self, controls, cost, mode=0, lam=0.0):
        u = _f32(controls)
        N, _, K = u.shape
        J = _f32(cost)
        bk = C.c_int(0)
        bc = C.c_double(0)
        plan = np.zeros((N, 2))
        rc = lib().oracle_select(self._h, int(mode), float(lam), _ptr(u, C.c_float),
                                 _ptr(J, C.c_float), K, N, C.byref(bk), C.byref(bc),
                                 _ptr(plan, C.c_double))
        if rc != 0:
            raise ValueError("oracle_select rejected the arguments")
        return bk.value, bc.value, plan

"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the
oracle's tests.

This module holds no planner arithmetic: it only produces parameter sets,
terrains, candidate control sequences and an initial state, as numpy arrays.
Both the GPU library and the oracle receive exactly these float32 arrays.

Workloads (the paper's scanned terrain and hand-marked obstacles are not
available, so these stand in for them; terrain features are smooth at wheel
scale, matching the 0.3 m Gaussian level of detail used for the SRB model):

* ``c1`` -- 128x128 heightmap at 0.2 m, sum of 40 Gaussian bumps; K=64, N=50.
* ``c2`` -- 512x512 at 0.1 m, 5-octave value-noise fBm (0.6 m peak-to-peak)
  plus two 0.3 m berms; K=4096, N=100.
* ``c3`` -- serving trace: 64 requests, Poisson arrivals at 200 req/s, K in
  {512..8192}, N in 40..160, each with its own 256x256 fBm crop.
* ``c4`` -- K=1024, N=100 on a fresh fBm terrain (gradient refinement case).
* ``c5`` -- 2048x2048 at 0.05 m: alternating 15 degree side slopes, 0.5 m
  berms, two 0.3 m ruts; K=65536, N=200 at dt=0.01.
* ``paper`` -- the paper's own solver shape: K=204,288 uniform steering-rate
  samples, 16 zero-order-hold segments of 0.25 s, 50 Euler substeps (5 ms).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

G = 9.81

# Paper, appendix "Vehicle Model Parameters": Polaris MRZR D4 (model
# parameter table) with the simulation tire fit (C = 6.1 /rad, mu = 0.6).
PAPER_VEHICLE = dict(
    M=969.0, Jxx=280.9, Jyy=692.1, Jzz=810.7,
    Lf=1.565, Lr=1.148, e=1.280, hR=0.380 + 0.291,
    kf=4.2e4, kr=5.8e4, bf=3.1e3, br=4.3e3,
    C=6.1, mu=0.6, delta_max=0.639, delta_rate_max=1.0, g=G,
)

# Synthetic workload vehicle: mass 900 kg, wheelbase 2.0 m, track 1.5 m,
# CoM height 0.6 m. Front/rear split follows the paper's Lf:Lr ratio, inertia
# scales with mass; springs, dampers, steering limits and tire from the paper.
_WB = 2.0
WORKLOAD_VEHICLE = dict(
    M=900.0,
    Jxx=280.9 * 900.0 / 969.0, Jyy=692.1 * 900.0 / 969.0, Jzz=810.7 * 900.0 / 969.0,
    Lf=_WB * 1.565 / (1.565 + 1.148), Lr=_WB * 1.148 / (1.565 + 1.148),
    e=1.5, hR=0.6,
    kf=4.2e4, kr=5.8e4, bf=3.1e3, br=4.3e3,
    C=6.1, mu=0.6, delta_max=0.639, delta_rate_max=1.0, g=G,
)

# Paper, section "OCP Formulation": w_t = 5 /s, w_c = 8 /s per (rad/s)^2,
# w_g = 15 /m, sigma = 1e6 /s, eps_dist = 0.25 m, goal radius 2.5 m.
# eps_esm = 0 asks each implementation for its default (10 % of the level
# ground ESM).
BASE_COST = dict(w_t=5.0, w_c=8.0, w_g=15.0, goal_x=0.0, goal_y=0.0, goal_r=2.5,
                 sigma=1.0e6, eps_esm=0.0, eps_dist=0.25)

BASE_INTEG = dict(dt=0.02, substeps=1, accel_max=3.0, vx_min=1.0)


@dataclass
class Terrain:
    height: np.ndarray          # [H][W] float32
    x0: float
    y0: float
    res: float
    costmap: np.ndarray | None = None   # [H][W] float32 cost units / s

    @property
    def W(self) -> int:
        return self.height.shape[1]

    @property
    def H(self) -> int:
        return self.height.shape[0]

    def node_xy(self):
        xs = self.x0 + self.res * np.arange(self.W)
        ys = self.y0 + self.res * np.arange(self.H)
        return np.meshgrid(xs, ys)  # [H][W] each


@dataclass
class Workload:
    name: str
    vehicle: dict
    cost: dict
    integ: dict
    terrain: Terrain
    state0: np.ndarray          # [13] float32
    controls: np.ndarray        # [N][2][K] float32
    meta: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return self.controls.shape[2]

    @property
    def N(self) -> int:
        return self.controls.shape[0]


# ------------------------------------------------------------------ terrains

def bumps_terrain(seed: int, n: int = 128, res: float = 0.2, count: int = 40,
                  amp=(0.0, 0.4), width=(0.5, 3.0)) -> Terrain:
    """Sum of ``count`` isotropic Gaussian bumps on an n x n grid."""
    rng = np.random.default_rng(seed)
    extent = n * res
    X, Y = np.meshgrid(res * np.arange(n), res * np.arange(n))
    h = np.zeros((n, n))
    for _ in range(count):
        a = rng.uniform(*amp)
        w = rng.uniform(*width)
        cx, cy = rng.uniform(0.0, extent, size=2)
        h += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * w * w))
    return Terrain(h.astype(np.float32), 0.0, 0.0, res)


def _value_noise(rng, X, Y, spacing):
    """Lattice value noise with quintic fade at the given lattice spacing."""
    gx = X / spacing
    gy = Y / spacing
    nx = int(math.floor(gx.max())) + 2
    ny = int(math.floor(gy.max())) + 2
    lat = rng.uniform(-1.0, 1.0, size=(ny, nx))
    ix = np.floor(gx).astype(np.int64)
    iy = np.floor(gy).astype(np.int64)
    tx = gx - ix
    ty = gy - iy
    fx = tx * tx * tx * (tx * (tx * 6.0 - 15.0) + 10.0)
    fy = ty * ty * ty * (ty * (ty * 6.0 - 15.0) + 10.0)
    v00 = lat[iy, ix]
    v10 = lat[iy, ix + 1]
    v01 = lat[iy + 1, ix]
    v11 = lat[iy + 1, ix + 1]
    a = v00 + fx * (v10 - v00)
    b = v01 + fx * (v11 - v01)
    return a + fy * (b - a)


def fbm_heights(seed: int, n: int, res: float, octaves: int = 5, base: float = 12.8,
                p2p: float = 0.6) -> np.ndarray:
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(res * np.arange(n), res * np.arange(n))
    h = np.zeros((n, n))
    for o in range(octaves):
        h += (0.5 ** o) * _value_noise(rng, X, Y, base * 2.0 ** (-o))
    h -= h.min()
    h *= p2p / max(h.max(), 1e-12)
    return h


def gaussian_ridge(X, Y, x_c, y_c, angle_deg, height, sigma):
    """A straight Gaussian-profile ridge through (x_c, y_c); ``angle_deg`` is
    the ridge's angle from the y axis (0 = crossing an x-directed path square)."""
    a = math.radians(angle_deg)
    # signed distance from the ridge line whose direction is (sin a, cos a)
    d = (X - x_c) * math.cos(a) - (Y - y_c) * math.sin(a)
    return height * np.exp(-d * d / (2.0 * sigma * sigma))


def fbm_berm_terrain(seed: int, n: int = 512, res: float = 0.1, berms=True,
                     y_path: float | None = None) -> Terrain:
    rng = np.random.default_rng(seed + 7)
    h = fbm_heights(seed, n, res)
    if berms:
        X, Y = np.meshgrid(res * np.arange(n), res * np.arange(n))
        yc = (n * res) / 2.0 if y_path is None else y_path
        for xc, ang in ((20.0, 30.0), (32.0, -30.0)):
            h = h + gaussian_ridge(X, Y, xc + rng.uniform(-1, 1), yc, ang, 0.3, 0.4)
    return Terrain(h.astype(np.float32), 0.0, 0.0, res)


def side_slope_terrain(seed: int, n: int = 2048, res: float = 0.05,
                       track: float = 1.5, berm_sigma: float = 1.0) -> Terrain:
    """Alternating 15 degree cross slopes (sign flips every 10 m along x with a
    tanh blend), 0.5 m berms about every 15 m (Gaussian profile, sigma 1 m:
    steepest flank about 17 degrees, so a 20 m/s vehicle is launched but not
    thrown), two 0.3 m ruts one track apart."""
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(res * np.arange(n), res * np.arange(n))
    yc = n * res / 2.0
    phase = np.sin(np.pi * X / 10.0)
    sign = np.tanh(4.0 * phase)
    h = math.tan(math.radians(15.0)) * (Y - yc) * sign
    # keep the slope band bounded away from the centre line so the heights stay
    # moderate over the whole map
    h = 3.0 * np.tanh(h / 3.0)
    x = 5.0
    while x < n * res - 5.0:
        x += rng.uniform(12.0, 18.0)
        h += gaussian_ridge(X, Y, x, yc, rng.uniform(-30, 30), 0.5, berm_sigma)
    for yr in (yc - track / 2.0, yc + track / 2.0):
        h -= 0.3 * np.exp(-((Y - yr) ** 2) / (2.0 * 0.3 * 0.3))
    return Terrain(h.astype(np.float32), 0.0, 0.0, res)


def obstacle_polygons(terrain: Terrain, seed: int, count: int = 6, radius=(0.8, 2.0),
                      sides: int = 12, boundary: bool = False) -> list:
    """Seeded obstacle perimeters: ``count`` regular polygons (kind 0) with
    circumradius in ``radius`` placed over the map, plus, with ``boundary``,
    a path-boundary rectangle (kind 1) 1 m inside the map edge. Geometry only:
    each side turns it into a costmap with its own code."""
    rng = np.random.default_rng(seed)
    ext_x = terrain.W * terrain.res
    ext_y = terrain.H * terrain.res
    polys = []
    for _ in range(count):
        cx = terrain.x0 + rng.uniform(0.2 * ext_x, 0.9 * ext_x)
        cy = terrain.y0 + rng.uniform(0.2 * ext_y, 0.8 * ext_y)
        r = rng.uniform(*radius)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        t = ph + 2.0 * math.pi * np.arange(sides) / sides
        polys.append((0, [(cx + r * math.cos(a), cy + r * math.sin(a)) for a in t]))
    if boundary:
        x0, y0 = terrain.x0 + 1.0, terrain.y0 + 1.0
        x1 = terrain.x0 + (terrain.W - 1) * terrain.res - 1.0
        y1 = terrain.y0 + (terrain.H - 1) * terrain.res - 1.0
        polys.append((1, [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]))
    return polys


# -------------------------------------------------------------- initial state

def settled_state(terrain: Terrain, x: float, y: float, psi: float, v0: float,
                  hR: float) -> np.ndarray:
    """Initial state resting on the terrain: the chassis axis b_z is aligned
    with the normal of a least-squares plane fitted to the heightmap nodes
    within 2 m of (x, y), the CoM sits hR above that plane along the normal,
    body velocity (v0, 0, 0), no rotation, straight wheels."""
    X, Y = terrain.node_xy()
    m = (X - x) ** 2 + (Y - y) ** 2 <= 4.0
    A = np.stack([np.ones(m.sum()), X[m] - x, Y[m] - y], axis=1)
    coef, *_ = np.linalg.lstsq(A, terrain.height[m].astype(np.float64), rcond=None)
    f0, a, b = coef
    nrm = np.array([-a, -b, 1.0]) / math.sqrt(1.0 + a * a + b * b)
    c, s = math.cos(psi), math.sin(psi)
    # normal expressed in the yaw-rotated frame; then b_z = Ry(theta) Rx(phi) e_z
    n1 = np.array([c * nrm[0] + s * nrm[1], -s * nrm[0] + c * nrm[1], nrm[2]])
    phi = -math.asin(max(-1.0, min(1.0, n1[1])))
    theta = math.atan2(n1[0], n1[2])
    z = f0 + hR / nrm[2]
    xi = np.zeros(13, dtype=np.float64)
    xi[0:6] = (x, y, z, psi, theta, phi)
    xi[6] = v0
    return xi.astype(np.float32)


# ------------------------------------------------------------------ controls

def gaussian_controls(seed: int, K: int, N: int, dt: float, sig=(0.1, 0.2),
                      amp_max: float = 0.5) -> np.ndarray:
    """[N][2][K]: a seeded sinusoidal steering-rate nominal (amplitude
    U(0, amp_max) rad/s, frequency U(0.2, 1) Hz, phase U(0, 2 pi)), zero
    throttle; candidate k adds i.i.d. N(0, sig^2) per step and channel;
    candidate 0 is the nominal itself."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.0, amp_max)
    f = rng.uniform(0.2, 1.0)
    ph = rng.uniform(0.0, 2.0 * math.pi)
    n = np.arange(N)
    nominal = A * np.sin(2.0 * math.pi * f * n * dt + ph)
    u = np.zeros((N, 2, K), dtype=np.float64)
    u[:, 0, :] = nominal[:, None]
    noise = rng.standard_normal((N, 2, K))
    noise[:, 0, :] *= sig[0]
    noise[:, 1, :] *= sig[1]
    noise[:, :, 0] = 0.0
    u += noise
    return u.astype(np.float32)


def uniform_controls(seed: int, K: int, N: int, rate_max: float = 1.0) -> np.ndarray:
    """The paper's sampling: steering rate uniform in [-rate_max, rate_max],
    longitudinal acceleration zero."""
    rng = np.random.default_rng(seed)
    u = np.zeros((N, 2, K), dtype=np.float32)
    u[:, 0, :] = rng.uniform(-rate_max, rate_max, size=(N, K)).astype(np.float32)
    return u


# --------------------------------------------------------------- workloads

def _cost_with_goal(gx, gy):
    c = dict(BASE_COST)
    c["goal_x"], c["goal_y"] = float(gx), float(gy)
    return c


def c1(seed: int = 1000, K: int = 64, N: int = 50) -> Workload:
    T = bumps_terrain(seed)
    s0 = settled_state(T, 5.0, 12.8, 0.0, 8.0, WORKLOAD_VEHICLE["hR"])
    u = gaussian_controls(seed + 1, K, N, 0.02)
    return Workload("c1", dict(WORKLOAD_VEHICLE), _cost_with_goal(17.0, 12.8),
                    dict(BASE_INTEG), T, s0, u)


def c2(seed: int = 2000, K: int = 4096, N: int = 100) -> Workload:
    T = fbm_berm_terrain(seed)
    s0 = settled_state(T, 8.0, 25.6, 0.0, 15.0, WORKLOAD_VEHICLE["hR"])
    u = gaussian_controls(seed + 1, K, N, 0.02)
    return Workload("c2", dict(WORKLOAD_VEHICLE), _cost_with_goal(49.2, 25.6),
                    dict(BASE_INTEG), T, s0, u)


def c4(seed: int = 4000, K: int = 1024, N: int = 100) -> Workload:
    w = c2(seed, K, N)
    w.name = "c4"
    return w


def c5(seed: int = 5000, K: int = 65536, N: int = 200, terrain: Terrain | None = None) -> Workload:
    T = terrain if terrain is not None else side_slope_terrain(seed)
    s0 = settled_state(T, 10.0, 51.2, 0.0, 20.0, WORKLOAD_VEHICLE["hR"])
    u = gaussian_controls(seed + 1, K, N, 0.01, sig=(0.15, 0.3))
    integ = dict(BASE_INTEG)
    integ["dt"] = 0.01
    return Workload("c5", dict(WORKLOAD_VEHICLE), _cost_with_goal(70.0, 51.2),
                    integ, T, s0, u)


def paper_shape(seed: int = 6000, K: int = 204288, terrain: Terrain | None = None) -> Workload:
    """K uniform samples, 16 ZOH segments of 0.25 s, 50 Euler substeps, the
    paper's vehicle and simulation tire."""
    T = terrain if terrain is not None else fbm_berm_terrain(2000)
    s0 = settled_state(T, 8.0, 25.6, 0.0, 7.5, PAPER_VEHICLE["hR"])
    u = uniform_controls(seed, K, 16)
    integ = dict(dt=0.25, substeps=50, accel_max=3.0, vx_min=1.0)
    return Workload("paper", dict(PAPER_VEHICLE), _cost_with_goal(49.2, 25.6),
                    integ, T, s0, u)


def goal_for(x, y, psi, v0, T_h, terrain: Terrain, margin: float = 2.0):
    """Goal 1.5 v0 T ahead along the heading, clamped ``margin`` inside the map."""
    d = 1.5 * v0 * T_h
    gx = x + d * math.cos(psi)
    gy = y + d * math.sin(psi)
    lo_x, hi_x = terrain.x0 + margin, terrain.x0 + (terrain.W - 1) * terrain.res - margin
    lo_y, hi_y = terrain.y0 + margin, terrain.y0 + (terrain.H - 1) * terrain.res - margin
    return min(max(gx, lo_x), hi_x), min(max(gy, lo_y), hi_y)


@dataclass
class Request:
    rid: int
    arrival: float
    workload: Workload


def c3_trace(seed: int = 3000, n_req: int = 64, rate: float = 200.0,
             Ks=(512, 1024, 2048, 4096, 8192), Nrange=(40, 160)) -> list:
    """Serving trace: Poisson arrivals, per-request K, N, speed, heading,
    terrain crop (256x256 at 0.1 m from the fBm generator), start at the
    crop centre, goal ahead along the heading."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for r in range(n_req):
        s = seed + 1 + r
        K = int(rng.choice(Ks))
        N = int(rng.integers(Nrange[0], Nrange[1] + 1))
        v0 = float(rng.uniform(5.0, 20.0))
        psi = float(rng.uniform(0.0, 2.0 * math.pi))
        T = Terrain(fbm_heights(s, 256, 0.1).astype(np.float32), 0.0, 0.0, 0.1)
        x = y = 12.8
        s0 = settled_state(T, x, y, psi, v0, WORKLOAD_VEHICLE["hR"])
        gx, gy = goal_for(x, y, psi, v0, N * 0.02, T)
        u = gaussian_controls(s + 500, K, N, 0.02)
        w = Workload(f"c3-{r}", dict(WORKLOAD_VEHICLE), _cost_with_goal(gx, gy),
                     dict(BASE_INTEG), T, s0, u)
        reqs.append(Request(r, float(t[r]), w))
    return reqs

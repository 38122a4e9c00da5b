"""GPU parity: the HIP rollout and selection (through the C ABI) against the
FP64 oracle, on identical seeded float32 inputs. Tolerances are in
tests/parity.py."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402  (test infrastructure)
from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402
from tests.parity import (ROLLOVER, assert_argmin_parity,  # noqa: E402
                          assert_finite_agreement, assert_horizon_parity,
                          assert_rollout_parity, assert_step_map_parity, conditioning,
                          cost_err)

pytestmark = pytest.mark.gpu

SHAPES = [(1, 64), (2, 64), (4, 64), (1, 256), (2, 256), (4, 256)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    yield
    torch.cuda.synchronize()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


class Case:
    """A workload uploaded to both the GPU library and the oracle."""

    def __init__(self, w: inputs.Workload, max_K=None, max_N=None, costmap=None):
        self.w = w
        T = w.terrain
        self.planner = P.Planner(w.vehicle, w.cost, w.integ, max_K or w.K, max_N or w.N,
                                 T.W, T.H)
        self.h_dev = dev(T.height)
        self.cm_dev = None if costmap is None else dev(costmap)
        self.planner.set_terrain(self.h_dev, T.x0, T.y0, T.res, self.cm_dev)
        self.o = oracle.Oracle(w.vehicle, w.cost, w.integ)
        self.o.set_terrain(T.height, T.x0, T.y0, T.res, costmap)

    def gpu(self, controls=None, state0=None, lanes=0, block=0):
        u = self.w.controls if controls is None else controls
        s0 = self.w.state0 if state0 is None else state0
        N, _, K = u.shape
        ud = dev(u)
        J = torch.empty(K, device="cuda")
        fs = torch.empty(13, K, device="cuda")
        self.planner.set_launch(lanes, block)
        self.planner.rollout(s0, ud, J, fs)
        torch.cuda.synchronize()
        return J.cpu().numpy(), fs.cpu().numpy(), ud

    def oracle(self, controls=None, state0=None):
        u = self.w.controls if controls is None else controls
        s0 = self.w.state0 if state0 is None else state0
        return self.o.rollout(s0, u)


@pytest.fixture(scope="module")
def c1():
    return Case(inputs.c1())


@pytest.fixture(scope="module")
def c2_1000():
    return Case(inputs.c2(K=1000))


# ----------------------------------------------------------------- rollout

@pytest.mark.parametrize("lanes,block", SHAPES)
def test_c1_full_parity_every_launch_shape(c1, lanes, block):
    J, fs, _ = c1.gpu(lanes=lanes, block=block)
    Jo, fso, _ = c1.oracle()
    ce, se = assert_rollout_parity(J, fs, Jo, fso, f"c1 lanes={lanes} block={block}")
    print(f"c1 lanes={lanes} block={block}: max cost err {ce:.3g}, state err {se:.3g} (x tol)")


@pytest.mark.parametrize("lanes,block", SHAPES)
def test_start_at_rest_takes_the_zero_over_zero_slip_convention(c1, lanes, block):
    """From rest every wheel's contact-point velocity is 0/0 at the first
    node: the slip angle is then -delta_i (the convention of the oracle), not
    a NaN that would score the candidate +inf. Two intervals, every launch
    shape, against the oracle."""
    s0 = np.array(c1.w.state0, dtype=np.float32).copy()
    s0[6:12] = 0.0
    u = np.ascontiguousarray(c1.w.controls[:2])
    J, fs, _ = c1.gpu(controls=u, state0=s0, lanes=lanes, block=block)
    assert np.isfinite(J).all() and np.isfinite(fs).all()
    Jo, fso, _ = c1.oracle(controls=u, state0=s0)
    ce, se = assert_rollout_parity(J, fs, Jo, fso, f"c1 at rest lanes={lanes} block={block}")
    print(f"c1 from rest lanes={lanes} block={block}: max cost err {ce:.3g}, state err {se:.3g}")


def _horizon(case, idx=None, lanes=0, block=0, label="", min_cost=0.9, min_state=0.5,
             controls=None, **kw):
    """Whole-horizon parity of every candidate (or of the candidates idx)
    against the oracle and its float32-storage probe (rules in
    tests/parity.py)."""
    u = case.w.controls if controls is None else controls
    J, fs, _ = case.gpu(controls=u, lanes=lanes, block=block)
    if idx is not None:
        u = np.ascontiguousarray(u[:, :, idx])
        J, fs = J[idx], fs[:, idx]
    return assert_horizon_parity(J, fs, case.o, case.w.state0, u, label, min_cost, min_state,
                                 **kw)


@pytest.mark.parametrize("lanes,block", SHAPES)
def test_c2_ragged_parity_every_launch_shape(c2_1000, lanes, block):
    _horizon(c2_1000, lanes=lanes, block=block, label=f"c2/1000 lanes={lanes} block={block}",
             min_cost=0.99, min_state=0.75)


def test_launch_shapes_agree_bitwise(c2_1000):
    ref = c2_1000.gpu(lanes=1, block=64)
    for lanes, block in SHAPES[1:]:
        J, fs, _ = c2_1000.gpu(lanes=lanes, block=block)
        np.testing.assert_array_equal(J, ref[0], err_msg=f"lanes={lanes} block={block}")
        np.testing.assert_array_equal(fs, ref[1], err_msg=f"lanes={lanes} block={block}")


def test_repeated_rollout_is_bitwise_identical(c2_1000):
    a = c2_1000.gpu()
    b = c2_1000.gpu()
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_chunked_rollout_equals_single_rollout_bitwise(c2_1000):
    J, fs, ud = c2_1000.gpu()
    K = c2_1000.w.K
    state = torch.empty(13, K, device="cuda")
    cost = torch.empty(K, device="cuda")
    c2_1000.planner.init_state(c2_1000.w.state0, state, cost)
    for n0, n1 in ((0, 7), (7, 7), (7, 40), (40, 99), (99, 100)):
        c2_1000.planner.rollout_chunk(state, cost, ud, n0, n1, n1 == 100)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(cost.cpu().numpy(), J)
    np.testing.assert_array_equal(state.cpu().numpy(), fs)


@pytest.fixture(scope="module")
def c2_full():
    return Case(inputs.c2())


def test_c2_full_step_map_parity(c2_full):
    w = c2_full.w
    ws, wc, _, _ = assert_step_map_parity(c2_full.planner, c2_full.o, w.controls,
                                          dev(w.controls), w.state0, 1, label="c2 step map")
    print(f"c2 step map (per interval): state err {ws:.3g}, cost err {wc:.3g} (x tol)")


def test_c2_full_size_bench_configuration(c2_full):
    J, fs, ud = c2_full.gpu()
    plan = torch.empty(c2_full.w.N, 2, device="cuda")
    k, jb = c2_full.planner.select(ud, torch.from_numpy(J).cuda(), plan)
    assert jb == J[k]
    # every candidate against the oracle, and the pick against the oracle's costs
    assert_horizon_parity(J, fs, c2_full.o, c2_full.w.state0, c2_full.w.controls, "c2 full",
                          min_cost=0.99, min_state=0.80, k_gpu=k)
    ko, _, po = c2_full.o.select(c2_full.w.controls, J, mode=0)
    assert k == ko
    np.testing.assert_array_equal(plan.cpu().numpy(), po.astype(np.float32))


def test_c4_step_map_and_horizon_parity():
    case = Case(inputs.c4())
    w = case.w
    assert_step_map_parity(case.planner, case.o, w.controls, dev(w.controls), w.state0, 1,
                           label="c4 step map")
    # this terrain seed drives many candidates into the ESM soft zone (the
    # 1e6 /s penalty makes cost a steep function of roll)
    _horizon(case, label="c4", min_cost=0.87, min_state=0.55)


@pytest.fixture(scope="module")
def c5_full():
    return Case(inputs.c5())


def test_c5_stress_full_step_map(c5_full):
    """Every one of the 65 536 stress candidates, every one of its 200
    intervals restarted from the GPU's own state."""
    w = c5_full.w
    ws, wc, _, _ = assert_step_map_parity(c5_full.planner, c5_full.o, w.controls,
                                          dev(w.controls), w.state0, 1, label="c5 step map")
    print(f"c5 step map (per interval, all 65536): state {ws:.3g}, cost {wc:.3g} (x tol)")


def test_c5_stress_horizon_parity(c5_full):
    """Whole horizon on the stress terrain. Every candidate is launched by a
    berm and rolls over late in its 2 s horizon (intervals 170-190), so the
    full horizon checks the finite pattern, the probe population rule and the
    pick; the strict per-candidate rules run on the first 170 intervals,
    before any candidate rolls over."""
    w = c5_full.w
    J, fs, ud = c5_full.gpu()
    plan = torch.empty(w.N, 2, device="cuda")
    k, _ = c5_full.planner.select(ud, torch.from_numpy(J).cuda(), plan)
    out = assert_horizon_parity(J, fs, c5_full.o, w.state0, w.controls, "c5 full horizon",
                                min_cost=0.0, min_state=0.0, k_gpu=k)
    assert out["rolled"] >= 0.99 * w.K
    pre = np.ascontiguousarray(w.controls[:170])
    out = _horizon(c5_full, controls=pre, label="c5 first 170 intervals", min_cost=0.40,
                   min_state=0.88)
    assert out["rolled"] == 0 and out["well_conditioned"] >= 0.9 * w.K


def test_c5_narrow_berms_nonfinite_agreement():
    """The stress terrain with 0.4 m wide berms: at 20 m/s 99.5 % of the
    candidates tumble into a non-finite state. The GPU and the oracle agree
    on which, up to what float32 storage alone changes in the oracle, and
    every interval before a candidate rolls over matches the oracle's."""
    T = inputs.side_slope_terrain(5000, berm_sigma=0.4)
    w = inputs.c5(terrain=T)
    case = Case(w)
    J, fs, _ = case.gpu()
    J64, F64, J32, F32, td, sl, tilt = conditioning(case.o, w.state0, w.controls)
    out = assert_finite_agreement(J, fs, J64, J32, F32, "c5 narrow berms")
    assert out["nonfinite_oracle"] > 0.99 * w.K
    assert_step_map_parity(case.planner, case.o, w.controls, dev(w.controls), w.state0, 1,
                           label="c5 narrow berms step map")


def test_paper_shape_full_step_map_and_horizon():
    """The paper's solver shape at full size (K = 204 288 uniform steering
    rates, 16 intervals of 0.25 s at 50 Euler substeps): every candidate's
    step map (each interval of 50 substeps restarted from the GPU's state)
    and whole horizon."""
    w = inputs.paper_shape()
    case = Case(w)
    ws, wc, _, _ = assert_step_map_parity(case.planner, case.o, w.controls, dev(w.controls),
                                          w.state0, 1, label="paper shape step map")
    print(f"paper shape step map (all 204288): state {ws:.3g}, cost {wc:.3g} (x tol)")
    _horizon(case, label="paper shape full", min_cost=0.99, min_state=0.87)


def test_paper_step_map_at_5ms():
    """The paper's 5 ms Euler step map, one step per interval (the same
    arithmetic the 50-substep intervals repeat), uniform steering rates held
    for 50 steps each."""
    w = inputs.paper_shape(K=2048)
    u = np.repeat(w.controls, 50, axis=0)[:400]
    w.controls = np.ascontiguousarray(u)
    w.integ = dict(w.integ, dt=0.005, substeps=1)
    case = Case(w)
    ws, wc, _, _ = assert_step_map_parity(case.planner, case.o, w.controls, dev(w.controls),
                                          w.state0, 1, label="paper 5 ms step map")
    print(f"paper 5 ms step map (400 steps): state {ws:.3g}, cost {wc:.3g}")


@pytest.mark.parametrize("lanes,block", [(0, 0), (1, 256)])
def test_costmap_obstacles_parity(lanes, block):
    """Obstacles and a path boundary as a costmap, against the oracle: the
    step map and the whole horizon, at the automatic launch (four lanes) and
    at one lane (the request-ahead kernels with their cost channel)."""
    w = inputs.c1(K=512)
    T = w.terrain
    cm = oracle.costmap_polygons(inputs.obstacle_polygons(T, seed=77, count=8), T.W, T.H, T.x0,
                                 T.y0, T.res, 1.0e6, 0.25).astype(np.float32)
    case = Case(w, costmap=cm)
    Jo, _, _ = case.oracle()
    assert (Jo > 1e3).sum() > 10  # obstacles are actually hit
    case.planner.set_launch(lanes, block)
    assert_step_map_parity(case.planner, case.o, w.controls, dev(w.controls), w.state0, 1,
                           label=f"costmap step map lanes={lanes}")
    _horizon(case, lanes=lanes, block=block, label=f"costmap lanes={lanes}", min_cost=0.99,
             min_state=0.95)
    case.planner.set_launch(0, 0)


def test_costmap_launch_shapes_agree_bitwise():
    """With a costmap that obstacles actually hit, every launch shape (the
    one-lane request-ahead kernels with their cost channel included) gives
    the same bits as the one-lane launch, for the plain and one-launch paths."""
    w = inputs.c1(K=512, N=30)
    T = w.terrain
    cm = oracle.costmap_polygons(inputs.obstacle_polygons(T, seed=77, count=8), T.W, T.H, T.x0,
                                 T.y0, T.res, 1.0e6, 0.25).astype(np.float32)
    case = Case(w, costmap=cm)
    ud = dev(w.controls)
    out = {}
    for lanes, block in SHAPES:
        J, fs, _ = case.gpu(lanes=lanes, block=block)
        J1 = torch.empty(w.K, device="cuda")
        plan = torch.empty(w.N, 2, device="cuda")
        k, jb = case.planner.rollout_argmin(w.state0, ud, J1, plan)
        torch.cuda.synchronize()
        out[(lanes, block)] = (J, fs, J1.cpu().numpy(), plan.cpu().numpy(), k, jb)
    case.planner.set_launch(0, 0)
    ref = out[SHAPES[0]]
    assert (ref[0] > 1e3).sum() > 10  # obstacles are actually hit
    for shape, got in out.items():
        for i, (a, b) in enumerate(zip(got, ref)):
            if isinstance(a, np.ndarray):
                np.testing.assert_array_equal(a, b, err_msg=f"{shape} output {i}")
            else:
                assert a == b, (shape, i, a, b)
    print(f"costmap: {len(SHAPES)} launch shapes bitwise equal, "
          f"{int((ref[0] > 1e3).sum())} of {w.K} candidates with a cost above 1e3")


@pytest.mark.parametrize("lanes,block", [(0, 0), (1, 256)])
def test_goal_exit_parity(lanes, block):
    """Candidates that reach the goal freeze there, against the oracle, at
    the automatic launch and at one lane (the request-ahead kernel skips a
    frozen candidate's steps and requests)."""
    w = inputs.c1(K=512)
    w.cost["goal_x"], w.cost["goal_y"] = 12.0, 12.8
    case = Case(w)
    J, fs, _ = case.gpu(lanes=lanes, block=block)
    case.planner.set_launch(0, 0)
    Jo, fso, ex = case.oracle()
    assert (ex >= 0).mean() > 0.5
    # a candidate may cross the goal circle within FP32 rounding of a node:
    # then the exit node differs by one; those are exempt
    rg = w.cost["goal_r"]
    d_g = np.hypot(fs[0] - 12.0, fs[1] - 12.8)
    d_o = np.hypot(fso[0] - 12.0, fso[1] - 12.8)
    marginal = (np.abs(d_g - rg) < 1e-3) | (np.abs(d_o - rg) < 1e-3)
    ok = ~marginal
    assert marginal.mean() < 0.05
    assert_rollout_parity(J[ok], fs[:, ok], Jo[ok], fso[:, ok], f"goal exit lanes={lanes}")
    print(f"goal exit lanes={lanes}: {int((ex >= 0).sum())} of {w.K} candidates reach the goal, "
          f"{int(marginal.sum())} marginal")


def test_nonsquare_terrain_and_leaving_the_map():
    rng = np.random.default_rng(9)
    H, W = 96, 200
    T = inputs.Terrain((0.3 * rng.standard_normal((H, W))).astype(np.float32), -3.0, 2.0, 0.1)
    # smooth it a little so it is wheel-scale smooth
    from scipy.ndimage import gaussian_filter
    T.height = gaussian_filter(T.height.astype(np.float64), 3.0).astype(np.float32)
    s0 = inputs.settled_state(T, 2.0, 6.5, 0.4, 18.0, inputs.WORKLOAD_VEHICLE["hR"])
    u = inputs.gaussian_controls(5, 300, 120, 0.02)
    cost = dict(inputs.BASE_COST, goal_x=40.0, goal_y=30.0)
    w = inputs.Workload("edge", dict(inputs.WORKLOAD_VEHICLE), cost, dict(inputs.BASE_INTEG),
                        T, s0, u)
    case = Case(w)
    J, fs, _ = case.gpu()
    Jo, fso, _ = case.oracle()
    assert (fso[0] > -3.0 + 0.1 * (W - 1)).any() or (fso[1] > 2.0 + 0.1 * (H - 1)).any()
    assert_rollout_parity(J, fs, Jo, fso, "non-square / off-map")


@pytest.mark.parametrize("W,H,x,y", [(2, 2, 3.0, 2.5), (2, 37, 4.0, 2.0), (17, 3, 0.5, 4.0),
                                     (33, 18, 1.0, 4.5)])
def test_small_and_ragged_terrain_grids(W, H, x, y):
    """Grids of one cell row or column, and grids that end inside a pack tile
    (16 x 16 cells): the vehicle starts off the map or next to its edge, so
    the lookups run through the clamped edge cells. Heights vary along both
    axes; the 33 x 18 grid carries a costmap. Step map of every candidate,
    then the whole horizon."""
    res = 0.5
    X, Y = np.meshgrid(np.arange(W) * res, np.arange(H) * res)
    h = (0.15 * np.sin(0.9 * X) + 0.1 * np.cos(0.7 * Y) + 0.03 * X).astype(np.float32)
    T = inputs.Terrain(h, 0.0, 0.0, res)
    s0 = inputs.settled_state(T, x, y, 0.3, 8.0, inputs.WORKLOAD_VEHICLE["hR"])
    u = inputs.gaussian_controls(W * 100 + H, 256, 50, 0.02)
    cost = dict(inputs.BASE_COST, goal_x=40.0, goal_y=20.0)
    w = inputs.Workload("grid", dict(inputs.WORKLOAD_VEHICLE), cost, dict(inputs.BASE_INTEG), T,
                        s0, u)
    cm = None
    if W > 16:
        cm = (20.0 * (1.0 + np.sin(0.5 * X) * np.cos(0.4 * Y))).astype(np.float32)
    case = Case(w, costmap=cm)
    assert_step_map_parity(case.planner, case.o, w.controls, dev(w.controls), w.state0, 1,
                           label=f"{W}x{H} grid step map")
    J, fs, _ = case.gpu()
    Jo, fso, _ = case.oracle()
    assert_rollout_parity(J, fs, Jo, fso, f"{W}x{H} grid")


def test_single_candidate_single_interval_and_max_sizes():
    w = inputs.c1(K=1, N=1)
    case = Case(w)
    J, fs, _ = case.gpu()
    Jo, fso, _ = case.oracle()
    assert_rollout_parity(J, fs, Jo, fso, "K=1 N=1")
    w = inputs.c1(K=777, N=64)
    case = Case(w, max_K=777, max_N=64)
    J, fs, _ = case.gpu()
    Jo, fso, _ = case.oracle()
    assert_rollout_parity(J, fs, Jo, fso, "K=max N=max")


def test_non_finite_candidates_score_infinity(c1):
    u = c1.w.controls.copy()
    u[10, 0, 3] = np.nan
    u[0, 1, 17] = np.inf   # clamps to full throttle: stays finite
    J, fs, _ = c1.gpu(controls=u)
    Jo, fso, _ = c1.oracle(controls=u)
    assert math.isinf(J[3]) and math.isinf(Jo[3])
    assert np.isfinite(J[17]) and np.isfinite(Jo[17])
    assert_rollout_parity(J, fs, Jo, fso, "non-finite")


def test_non_finite_candidates_agree_bitwise_over_launch_shapes(c1):
    """A candidate whose state turns NaN keeps stepping in every kernel form
    (its position is never at the goal), so its final state, NaN entries
    included, and its +inf cost are the same bits at every launch shape."""
    u = c1.w.controls.copy()
    u[10, 0, 3] = np.nan
    u[4, 1, 40] = np.nan
    ref = c1.gpu(controls=u, lanes=1, block=64)
    assert math.isinf(ref[0][3]) and math.isinf(ref[0][40])
    assert np.isnan(ref[1][:, 3]).any()
    for lanes, block in SHAPES[1:]:
        J, fs, _ = c1.gpu(controls=u, lanes=lanes, block=block)
        np.testing.assert_array_equal(J, ref[0], err_msg=f"lanes={lanes} block={block}")
        np.testing.assert_array_equal(fs, ref[1], err_msg=f"lanes={lanes} block={block}")
    c1.planner.set_launch(0, 0)
    print(f"non-finite candidates: {len(SHAPES)} launch shapes bitwise equal")


# ----------------------------------------------------------------- select

def _select_case(K, N=20, seed=0):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.5, 1.5, size=(N, 2, K)).astype(np.float32)
    J = rng.uniform(50, 60, size=K).astype(np.float32)
    return u, J


@pytest.mark.parametrize("K", [1, 63, 4096, 4097, 100_003])
def test_argmin_select_matches_oracle_exactly(c1, K):
    u, J = _select_case(K)
    planner = P.Planner(c1.w.vehicle, c1.w.cost, c1.w.integ, K, 20, 8, 8)
    plan = torch.empty(20, 2, device="cuda")
    k, jb = planner.select(dev(u), dev(J), plan)
    ko, jo, po = c1.o.select(u, J, mode=0)
    assert k == ko and jb == np.float32(jo)
    np.testing.assert_array_equal(plan.cpu().numpy(), po.astype(np.float32))
    # a second call reuses the reset workspace
    J2 = J.copy()
    J2[K // 2] = 1.0
    k2, _ = planner.select(dev(u), dev(J2), plan)
    assert k2 == K // 2


def test_argmin_ties_nonfinite_and_all_infinite(c1):
    K = 9000
    u, J = _select_case(K)
    J[:] = 100.0
    J[[7000, 5000, 8999]] = 3.0
    J[[1, 2]] = np.nan
    J[4] = -np.inf
    planner = P.Planner(c1.w.vehicle, c1.w.cost, c1.w.integ, K, 20, 8, 8)
    plan = torch.empty(20, 2, device="cuda")
    k, jb = planner.select(dev(u), dev(J), plan)
    assert k == 5000 and jb == 3.0
    J[:] = np.inf
    k, jb = planner.select(dev(u), dev(J), plan)
    assert k == -1 and math.isinf(jb)
    assert torch.count_nonzero(plan).item() == 0


@pytest.mark.parametrize("K,lam", [(64, 1.0), (4096, 0.5), (70_000, 2.0), (4096, 1e-6)])
def test_softmin_select_matches_oracle(c1, K, lam):
    u, J = _select_case(K, seed=3)
    planner = P.Planner(c1.w.vehicle, c1.w.cost, c1.w.integ, K, 20, 8, 8)
    plan = torch.empty(20, 2, device="cuda")
    for _ in range(2):
        k, jb = planner.select(dev(u), dev(J), plan, mode=P.PLAN_SOFTMIN, lam=lam)
        ko, jo, po = c1.o.select(u, J, mode=1, lam=lam)
        assert k == ko
        g = plan.cpu().numpy().astype(np.float64)
        np.testing.assert_array_less(np.abs(g - po), 1e-4 * np.maximum(np.abs(po), 0.1))


def test_rollout_then_select_pipeline_c1(c1):
    J, fs, ud = c1.gpu()
    Jo, _, _ = c1.oracle()
    plan = torch.empty(c1.w.N, 2, device="cuda")
    k, jb = c1.planner.select(ud, torch.from_numpy(J).cuda(), plan)
    assert_argmin_parity(k, Jo)
    assert cost_err(np.array([jb]), np.array([Jo[k]]))[0] <= 1.0


# ----------------------------------------------------------------- errors

def test_error_codes_on_device():
    w = inputs.c1(K=16, N=8)
    planner = P.Planner(w.vehicle, w.cost, w.integ, 16, 8, w.terrain.W, w.terrain.H)
    u = dev(w.controls)
    J = torch.empty(16, device="cuda")
    with pytest.raises(P.PlanError) as e:
        planner.rollout(w.state0, u, J)
    assert e.value.status == P.PLAN_ENOTERRAIN
    h = w.terrain.height.copy()
    h[3, 4] = np.nan
    with pytest.raises(P.PlanError) as e:
        planner.set_terrain(dev(h), 0.0, 0.0, 0.2)
    assert e.value.status == P.PLAN_EINVAL and "non-finite" in str(e.value)
    with pytest.raises(P.PlanError) as e:
        planner.rollout(w.state0, u, J)
    assert e.value.status == P.PLAN_ENOTERRAIN
    planner.set_terrain(dev(w.terrain.height), 0.0, 0.0, 0.2)
    big = dev(inputs.gaussian_controls(1, 17, 8, 0.02))
    with pytest.raises(P.PlanError) as e:
        P.plan_rollout(planner.ctx, w.state0, big, torch.empty(17, device="cuda"))
    assert e.value.status == P.PLAN_EINVAL
    s_bad = w.state0.copy()
    s_bad[4] = np.inf
    with pytest.raises(P.PlanError) as e:
        planner.rollout(s_bad, u, J)
    assert e.value.status == P.PLAN_EINVAL
    with pytest.raises(P.PlanError):
        planner.select(u, J, torch.empty(8, 2, device="cuda"), mode=P.PLAN_SOFTMIN, lam=0.0)
    with pytest.raises(P.PlanError):
        planner.set_terrain(dev(np.zeros((w.terrain.H + 1, w.terrain.W), np.float32)), 0, 0, 0.2)
    planner.rollout(w.state0, u, J)
    torch.cuda.synchronize()
    assert torch.isfinite(J).all()


def test_no_costmap_kernels_equal_a_zero_costmap_bitwise():
    """Without a costmap the kernels skip the cost channel; with an all-zero
    costmap they load and sum it. The results are the same bits, for the plain,
    one-launch and sampled paths and every lane count."""
    w = inputs.c2(K=777, N=40)
    T = w.terrain
    ud = dev(w.controls)
    plain = Case(w)
    zero = Case(w, costmap=np.zeros_like(T.height))
    spec = P.sample_spec(P.PLAN_SAMPLE_GAUSSIAN, 41, 0, (0.1, 0.2))
    for lanes in (1, 2, 4):
        out = []
        for case in (plain, zero):
            J, fs, _ = case.gpu(lanes=lanes)
            J1 = torch.empty(w.K, device="cuda")
            plan = torch.empty(w.N, 2, device="cuda")
            k, jb = case.planner.rollout_argmin(w.state0, ud, J1, plan)
            Js = torch.empty(w.K, device="cuda")
            case.planner.rollout_sampled(w.state0, spec, w.N, Js)
            torch.cuda.synchronize()
            out.append((J, fs, J1.cpu().numpy(), plan.cpu().numpy(), k, Js.cpu().numpy()))
        for a, b in zip(*out):
            np.testing.assert_array_equal(a, b, err_msg=f"lanes={lanes}")

"""GPU parity of the extended single-track (EST) baseline rollout
(plan_rollout_est) against the oracle's EST formulation, on the same seeded
float32 inputs, with the tolerances of tests/parity.py (EST state scales:
1 m, 0.1 rad, 1 m/s, 1 rad/s)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402  (test infrastructure)
from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402
from tests.parity import assert_est_probe_parity, assert_rollout_parity  # noqa: E402
from tests.test_parity_gpu import dev  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    yield
    torch.cuda.synchronize()


def est_state0(s13):
    """EST state from an SRB state: x, y, psi, v_y, omega_z, delta, v_x."""
    s = np.asarray(s13, np.float32)
    return np.array([s[0], s[1], s[3], s[7], s[11], s[12], s[6]], np.float32)


class EstCase:
    def __init__(self, w, vehicle=None, cost=None, costmap=None, max_K=None):
        self.w = w
        veh = vehicle or w.vehicle
        co = cost or w.cost
        T = w.terrain
        self.planner = P.Planner(veh, co, w.integ, max_K or w.K, w.N, T.W, T.H)
        self.h_dev = dev(T.height)
        self.cm_dev = None if costmap is None else dev(costmap)
        self.planner.set_terrain(self.h_dev, T.x0, T.y0, T.res, self.cm_dev)
        self.o = oracle.Oracle(veh, co, w.integ)
        self.o.set_terrain(T.height, T.x0, T.y0, T.res, costmap)
        self.s0 = est_state0(w.state0)

    def gpu(self, controls=None):
        u = self.w.controls if controls is None else controls
        N, _, K = u.shape
        J = torch.empty(K, device="cuda")
        fs = torch.empty(7, K, device="cuda")
        self.planner.rollout_est(self.s0, dev(u), J, fs)
        torch.cuda.synchronize()
        return J.cpu().numpy(), fs.cpu().numpy()

    def check(self, label, controls=None):
        u = self.w.controls if controls is None else controls
        J, fs = self.gpu(u)
        Jo, fso, _ = self.o.est_rollout(self.s0, u)
        ce, se = assert_rollout_parity(J, fs, Jo, fso, label)
        print(f"{label}: max cost err {ce:.3g}, state err {se:.3g} (x tol)")
        return J, fs


def test_est_c1_parity():
    EstCase(inputs.c1()).check("est c1")


def test_est_c2_ragged_parity_and_repeatability():
    case = EstCase(inputs.c2(K=1000))
    J, fs = case.check("est c2 K=1000")
    J2, fs2 = case.gpu()
    assert np.array_equal(J, J2) and np.array_equal(fs, fs2)


def test_est_c2_full_size():
    case = EstCase(inputs.c2())
    J, fs = case.gpu()
    idx = np.arange(0, case.w.K, 7)
    u = np.ascontiguousarray(case.w.controls[:, :, idx])
    Jo, fso, _ = case.o.est_rollout(case.s0, u)
    ce, se = assert_rollout_parity(J[idx], fs[:, idx], Jo, fso, "est c2 full, sampled")
    print(f"est c2 full (every 7th of 4096): cost err {ce:.3g}, state err {se:.3g}")


def test_est_costmap_parity():
    w = inputs.c1(K=512)
    T = w.terrain
    cm = oracle.costmap_polygons(inputs.obstacle_polygons(T, seed=77, count=8), T.W, T.H, T.x0,
                                 T.y0, T.res, 1.0e6, 0.25).astype(np.float32)
    EstCase(w, costmap=cm).check("est c1 costmap")


def test_est_paper_shape_substeps():
    """The paper's sampling (uniform steering rates held 0.25 s, 800 Euler
    steps): near-neutral sideslip dynamics, compared against the oracle's
    float32-storage probe (tests/parity.py)."""
    w = inputs.paper_shape(K=2048)
    case = EstCase(w)
    J, fs = case.gpu()
    m, worst = assert_est_probe_parity(J, fs, case.o, case.s0, w.controls,
                                       "est paper shape (16 x 50 substeps)")
    print(f"est paper shape: {m:.1%} within tolerance, worst {worst:.3g} of the probe bound")


def test_est_tall_vehicle_where_the_constraint_binds():
    """hR = 2 m puts a_bar_y = 0.375 g below mu g, so the soft constraint
    adds cost on some candidates; sigma is lowered so that the cost stays in
    a range where FP32 accumulation can be compared."""
    w = inputs.c1(K=256)
    veh = dict(w.vehicle, hR=2.0)
    co = dict(w.cost, sigma=100.0)
    case = EstCase(w, vehicle=veh, cost=co)
    J, _ = case.check("est tall vehicle")
    # the constraint is active: without it (sigma = 0) some candidates cost less
    free = oracle.Oracle(veh, dict(co, sigma=0.0), w.integ)
    T = w.terrain
    free.set_terrain(T.height, T.x0, T.y0, T.res)
    J0, _, _ = free.est_rollout(case.s0, w.controls)
    assert np.sum(J > J0 + 1.0) >= 10


def test_est_stress_terrain_sampled():
    w = inputs.c5(K=4096, N=200)
    case = EstCase(w)
    J, fs = case.gpu()
    idx = np.arange(0, w.K, 8)
    u = np.ascontiguousarray(w.controls[:, :, idx])
    m, worst = assert_est_probe_parity(J[idx], fs[:, idx], case.o, case.s0, u, "est c5 sampled")
    print(f"est c5 (every 8th of 4096): {m:.1%} within tolerance, worst {worst:.3g} of bound")


def test_est_errors():
    case = EstCase(inputs.c1())
    u = dev(case.w.controls)
    J = torch.empty(case.w.K, device="cuda")
    bad = case.s0.copy()
    bad[6] = np.nan
    with pytest.raises(P.PlanError) as e:
        case.planner.rollout_est(bad, u, J)
    assert e.value.status == P.PLAN_EINVAL
    lib = P.lib()
    s0 = (P.C.c_float * 7)(*case.s0)
    assert lib.plan_rollout_est(case.planner.ctx, s0, None, 64, 50,
                                P.C.c_void_p(J.data_ptr()), None) == P.PLAN_EINVAL
    assert lib.plan_rollout_est(case.planner.ctx, s0, P.C.c_void_p(u.data_ptr()), 65, 50,
                                P.C.c_void_p(J.data_ptr()), None) == P.PLAN_EINVAL

"""GPU parity of the fourth-order Runge-Kutta option (plan_integ_t.method =
PLAN_RK4) against the oracle's RK4, on identical float32 inputs, and its
restrictions."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402
from tests.parity import assert_rollout_parity, assert_horizon_parity  # noqa: E402
from tests.test_parity_gpu import SHAPES, Case, dev  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    yield
    torch.cuda.synchronize()


def rk4(w):
    w.integ = dict(w.integ, method=P.PLAN_RK4)
    return w


@pytest.fixture(scope="module")
def c1rk():
    return Case(rk4(inputs.c1()))


@pytest.mark.parametrize("lanes,block", SHAPES)
def test_c1_rk4_full_parity_every_launch_shape(c1rk, lanes, block):
    J, fs, _ = c1rk.gpu(lanes=lanes, block=block)
    Jo, fso, _ = c1rk.oracle()
    ce, se = assert_rollout_parity(J, fs, Jo, fso, f"c1 rk4 lanes={lanes} block={block}")
    print(f"c1 rk4 lanes={lanes} block={block}: cost err {ce:.3g}, state err {se:.3g} (x tol)")


def test_rk4_launch_shapes_and_chunks_agree_bitwise():
    case = Case(rk4(inputs.c2(K=1000)))
    ref = case.gpu(lanes=1, block=64)
    for lanes, block in SHAPES[1:]:
        J, fs, _ = case.gpu(lanes=lanes, block=block)
        assert np.array_equal(J, ref[0]) and np.array_equal(fs, ref[1]), (lanes, block)
    w = case.w
    u = dev(w.controls)
    st = torch.empty(13, w.K, device="cuda")
    cost = torch.empty(w.K, device="cuda")
    case.planner.set_launch(0, 0)
    case.planner.init_state(w.state0, st, cost)
    for n0 in range(0, w.N, 17):
        n1 = min(n0 + 17, w.N)
        case.planner.rollout_chunk(st, cost, u, n0, n1, n1 == w.N)
    torch.cuda.synchronize()
    assert np.array_equal(cost.cpu().numpy(), ref[0])
    assert np.array_equal(st.cpu().numpy(), ref[1])


def test_c2_rk4_horizon_parity():
    case = Case(rk4(inputs.c2(K=1000)))
    J, fs, _ = case.gpu()
    assert_horizon_parity(J, fs, case.o, case.w.state0, case.w.controls, "c2 rk4",
                          min_cost=0.99, min_state=0.85)


def test_paper_shape_rk4_at_a_coarser_step():
    """The paper's samples (uniform steering rates, 16 intervals of 0.25 s)
    integrated by RK4 at 25 ms (10 steps per interval)."""
    w = rk4(inputs.paper_shape(K=2048))
    w.integ = dict(w.integ, substeps=10)
    case = Case(w)
    J, fs, _ = case.gpu()
    assert_horizon_parity(J, fs, case.o, w.state0, w.controls, "paper shape rk4 (16 x 10)",
                          min_cost=0.99, min_state=0.93)


def test_rk4_is_refused_where_only_euler_is_built(c1rk):
    w = c1rk.w
    u = dev(w.controls)
    J = torch.empty(w.K, device="cuda")
    plan = torch.empty(w.N, 2, device="cuda")
    spec = P.sample_spec(P.PLAN_SAMPLE_UNIFORM, 1, 0, (1.0, 0.0))
    calls = [
        lambda: c1rk.planner.rollout_argmin(w.state0, u, J, plan),
        lambda: c1rk.planner.rollout_sampled(w.state0, spec, w.N, J),
        lambda: c1rk.planner.rollout_sampled_argmin(w.state0, spec, w.N, J, plan),
        lambda: c1rk.planner.rollout_grad(w.state0, u, J, torch.empty_like(u)),
        lambda: c1rk.planner.rollout_est(np.zeros(7, np.float32) + 1.0, u, J),
    ]
    for call in calls:
        with pytest.raises(P.PlanError) as e:
            call()
        assert e.value.status == P.PLAN_EINVAL
    bad = dict(w.integ, method=2)
    with pytest.raises(P.PlanError):
        P.Planner(w.vehicle, w.cost, bad, 8, 8, 8, 8)

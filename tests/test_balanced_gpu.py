"""One-lane full-horizon launches whose candidates fill whole rounds of one
wave per SIMD plus a small remainder run that remainder at four lanes per
candidate in the same launch. Every candidate's results must equal those of
the plain one-lane launch bit for bit, for materialised and sampled controls,
with and without the fused argmin, with and without the locality order; the
oracle checks a sample of the candidates."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402  (test infrastructure)
from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402
from tests.parity import assert_horizon_parity  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    # one whole round (a wave per SIMD) plus a sixteenth of a round, 4 intervals
    # of 50 Euler substeps, no costmap: the form the balanced launch takes
    K = 64 * simds + 4 * simds
    w = inputs.paper_shape(K=K)
    N = 4
    u = np.ascontiguousarray(w.controls[:N])
    T = w.terrain
    pl = P.Planner(w.vehicle, w.cost, w.integ, K, N, T.W, T.H)
    pl.set_terrain(torch.from_numpy(T.height).cuda(), T.x0, T.y0, T.res)
    yield w, u, pl, K, N, 4 * simds
    pl.close()


def _all_paths(pl, w, u, K, N):
    ud = torch.from_numpy(u).cuda()
    spec = P.sample_spec(P.PLAN_SAMPLE_UNIFORM, 6000, 0, (1.0, 0.0))
    out = {}
    J = torch.empty(K, device="cuda")
    fs = torch.empty(13, K, device="cuda")
    pl.rollout(w.state0, ud, J, fs)
    torch.cuda.synchronize()
    out["plain"] = (J.cpu().numpy(), fs.cpu().numpy())
    plan = torch.empty(N, 2, device="cuda")
    kb, jb = pl.rollout_argmin(w.state0, ud, J, plan, fs)
    torch.cuda.synchronize()
    out["fused"] = (J.cpu().numpy(), fs.cpu().numpy(), plan.cpu().numpy(), kb, jb)
    pl.rollout_sampled(w.state0, spec, N, J, fs)
    torch.cuda.synchronize()
    out["sampled"] = (J.cpu().numpy(), fs.cpu().numpy())
    kb, jb = pl.rollout_sampled_argmin(w.state0, spec, N, J, plan, fs)
    torch.cuda.synchronize()
    out["fused_sampled"] = (J.cpu().numpy(), fs.cpu().numpy(), plan.cpu().numpy(), kb, jb)
    return out


@pytest.mark.parametrize("order", [P.PLAN_ORDER_OFF, P.PLAN_ORDER_ON])
def test_balanced_launch_equals_one_lane_bitwise(setup, order):
    w, u, pl, K, N, _ = setup
    pl.set_order(order)
    pl.set_launch(0, 0)
    auto = _all_paths(pl, w, u, K, N)
    pl.set_launch(1, 64)
    one = _all_paths(pl, w, u, K, N)
    pl.set_launch(0, 0)
    pl.set_order(P.PLAN_ORDER_AUTO)
    for path in auto:
        for i, (a, b) in enumerate(zip(auto[path], one[path])):
            if isinstance(a, np.ndarray):
                np.testing.assert_array_equal(a, b, err_msg=f"{path} output {i}")
            else:
                assert a == b, (path, i, a, b)
    print(f"balanced launch, K = {K}, order {order}: {len(auto)} paths bitwise equal to one lane")


def test_balanced_launch_against_the_oracle(setup):
    """Candidates of both parts of the launch (the one-lane rounds and the
    four-lane remainder, which holds the last slots) against the oracle."""
    w, u, pl, K, N, rem = setup
    pl.set_order(P.PLAN_ORDER_OFF)
    ud = torch.from_numpy(u).cuda()
    J = torch.empty(K, device="cuda")
    fs = torch.empty(13, K, device="cuda")
    pl.rollout(w.state0, ud, J, fs)
    torch.cuda.synchronize()
    pl.set_order(P.PLAN_ORDER_AUTO)
    idx = np.concatenate([np.arange(0, K - rem, 97), np.arange(K - rem, K, 7)])
    o = oracle.Oracle(w.vehicle, w.cost, w.integ)
    T = w.terrain
    o.set_terrain(T.height, T.x0, T.y0, T.res)
    us = np.ascontiguousarray(u[:, :, idx])
    assert_horizon_parity(J.cpu().numpy()[idx], fs.cpu().numpy()[:, idx], o, w.state0, us,
                          "balanced launch sample", min_cost=0.99, min_state=0.85,
                          argmin=False)
    print(f"balanced launch: {idx.size} candidates against the oracle "
          f"({int((idx >= K - rem).sum())} in the four-lane remainder)")

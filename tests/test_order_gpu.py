"""GPU tests of the locality order: running the candidates of a full-horizon
rollout in proxy-trajectory order changes only which lane simulates which
candidate, so every output must be bit-identical to the unordered launch,
and every candidate must be written exactly once (outputs start as NaN)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402
from tests.test_est_gpu import est_state0  # noqa: E402
from tests.test_parity_gpu import dev  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    yield
    torch.cuda.synchronize()


def nan(*shape):
    return torch.full(shape, float("nan"), device="cuda")


class Ctx:
    def __init__(self, w, max_K):
        T = w.terrain
        self.w = w
        self.pl = P.Planner(w.vehicle, w.cost, w.integ, max_K, w.N, T.W, T.H)
        self.pl.set_terrain(dev(T.height), T.x0, T.y0, T.res)

    def run(self, mode, u, K=None):
        """Every full-horizon entry point under one order mode."""
        pl, w = self.pl, self.w
        u = u if K is None else u[:, :, :K].contiguous()
        N, _, K = u.shape
        pl.set_order(mode)
        out = {}
        J, fs = nan(K), nan(13, K)
        pl.rollout(w.state0, u, J, fs)
        out["rollout"] = (J, fs, pl.get_order())
        J, fs, plan = nan(K), nan(13, K), nan(N, 2)
        r = pl.rollout_argmin(w.state0, u, J, plan, fs)
        out["argmin"] = (J, fs, plan, r)
        spec = P.sample_spec(P.PLAN_SAMPLE_UNIFORM, 77, 3, (1.0, 0.5))
        J, fs, plan = nan(K), nan(13, K), nan(N, 2)
        r = pl.rollout_sampled_argmin(w.state0, spec, N, J, plan, fs)
        out["sampled_argmin"] = (J, fs, plan, r, pl.get_order())
        J, fs = nan(K), nan(13, K)
        pl.rollout_sampled(w.state0, spec, N, J, fs)
        out["sampled"] = (J, fs)
        J, fs = nan(K), nan(7, K)
        pl.rollout_est(est_state0(w.state0), u, J, fs)
        out["est"] = (J, fs, pl.get_order())
        torch.cuda.synchronize()
        return out


def assert_same(a, b, label):
    for key in a:
        for x, y in zip(a[key], b[key]):
            if isinstance(x, torch.Tensor):
                xh, yh = x.cpu().numpy(), y.cpu().numpy()
                assert not np.isnan(xh).any(), f"{label} {key}: a candidate was not written"
                np.testing.assert_array_equal(xh, yh, err_msg=f"{label} {key}")
            elif isinstance(x, tuple):
                assert x == y, f"{label} {key}: {x} != {y}"


def test_ordered_outputs_equal_unordered_bitwise_ragged_tiles():
    # 5000 candidates: three sort tiles, the last ragged; forced on
    w = inputs.c2(K=5000, N=24)
    c = Ctx(w, 5000)
    u = dev(w.controls)
    off = c.run(P.PLAN_ORDER_OFF, u)
    assert c.pl.get_launch()[0] == 4  # automatic shape at K = 5000
    on = c.run(P.PLAN_ORDER_ON, u)
    assert c.pl.get_launch()[0] == 1  # ordered launches run one lane per candidate
    assert not off["rollout"][2] and on["rollout"][2] and on["est"][2]
    assert_same(off, on, "c2 K=5000")
    c.pl.close()


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_ordered_outputs_with_fewer_intervals_than_proxy_samples(N):
    w = inputs.c1(K=300, N=N)
    c = Ctx(w, 300)
    u = dev(w.controls)
    assert_same(c.run(P.PLAN_ORDER_OFF, u), c.run(P.PLAN_ORDER_ON, u), f"c1 N={N}")
    c.pl.close()


def test_single_candidate_ordered():
    w = inputs.c1(K=1, N=10)
    c = Ctx(w, 1)
    u = dev(w.controls)
    assert_same(c.run(P.PLAN_ORDER_OFF, u), c.run(P.PLAN_ORDER_ON, u), "K=1")
    c.pl.close()


def test_auto_orders_large_uniform_sampled_launches_and_k_can_change():
    # paper-shape candidates (uniform steering rates, 50 substeps) on a short
    # horizon; the automatic mode orders launches that draw uniform samples
    # from K = 49 152 on (at one lane per candidate) and nothing else, and
    # alternating sizes on one context reuse the sort's workspace
    w = inputs.paper_shape(K=200000)
    w.controls = np.ascontiguousarray(w.controls[:4])
    c = Ctx(w, 200000)
    u = dev(w.controls)
    off_big = c.run(P.PLAN_ORDER_OFF, u)
    off_small = c.run(P.PLAN_ORDER_OFF, u, K=5000)
    auto_big = c.run(P.PLAN_ORDER_AUTO, u)
    assert auto_big["sampled_argmin"][4]
    assert not auto_big["rollout"][2] and not auto_big["est"][2]
    assert c.pl.get_launch()[0] == 1
    # Gaussian samples around a nominal stay close together: not ordered
    gspec = P.sample_spec(P.PLAN_SAMPLE_GAUSSIAN, 5, 0, (0.1, 0.2))
    J, plan = nan(200000), nan(4, 2)
    c.pl.rollout_sampled_argmin(w.state0, gspec, 4, J, plan)
    assert not c.pl.get_order()
    # below the threshold the uniform draws are not ordered either
    auto_40k = c.run(P.PLAN_ORDER_AUTO, u, K=40000)
    assert not auto_40k["sampled_argmin"][4]
    # nor with one Euler substep per control (a draw every step, short rollout)
    w1 = inputs.c2(K=8, N=10)
    T1 = w1.terrain
    pl1 = P.Planner(w1.vehicle, w1.cost, w1.integ, 50000, 10, T1.W, T1.H)
    pl1.set_terrain(dev(T1.height), T1.x0, T1.y0, T1.res)
    uspec = P.sample_spec(P.PLAN_SAMPLE_UNIFORM, 3, 0, (1.0, 0.0))
    pl1.rollout_sampled_argmin(w1.state0, uspec, 10, nan(50000), nan(10, 2))
    assert w1.integ["substeps"] == 1 and not pl1.get_order()
    pl1.close()
    auto_small = c.run(P.PLAN_ORDER_AUTO, u, K=5000)
    assert not auto_small["rollout"][2] and not auto_small["sampled_argmin"][4]
    off_mid = c.run(P.PLAN_ORDER_OFF, u, K=60000)
    auto_mid = c.run(P.PLAN_ORDER_AUTO, u, K=60000)
    assert not auto_mid["rollout"][2] and auto_mid["sampled_argmin"][4]
    assert_same(off_mid, auto_mid, "K=60000 auto")
    on_small = c.run(P.PLAN_ORDER_ON, u, K=5000)
    auto_big2 = c.run(P.PLAN_ORDER_AUTO, u)
    assert_same(off_big, auto_big, "K=200000 auto")
    assert_same(off_small, auto_small, "K=5000 auto")
    assert_same(off_small, on_small, "K=5000 on after 200000")
    assert_same(off_big, auto_big2, "K=200000 auto again")
    c.pl.close()


def test_lane_ordered_controls_grow_between_calls():
    # the lane-ordered copy of the controls is grown on demand: a small
    # ordered launch, then a larger one (regrow), then the small one again
    w = inputs.c2(K=6000, N=30)
    c = Ctx(w, 6000)
    u = dev(w.controls)
    small, large = u[:10].contiguous(), u
    off_s = c.run(P.PLAN_ORDER_OFF, small, K=1500)
    off_l = c.run(P.PLAN_ORDER_OFF, large)
    on_s = c.run(P.PLAN_ORDER_ON, small, K=1500)
    on_l = c.run(P.PLAN_ORDER_ON, large)
    on_s2 = c.run(P.PLAN_ORDER_ON, small, K=1500)
    assert_same(off_s, on_s, "N=10 K=1500")
    assert_same(off_l, on_l, "N=30 K=6000 after regrow")
    assert_same(off_s, on_s2, "N=10 K=1500 again")
    c.pl.close()


def test_ordered_rk4_rollout_bitwise():
    # fourth-order Runge-Kutta through plan_rollout (its one-lane kernel
    # carries the order like the Euler kernels)
    w = inputs.c2(K=3000, N=20)
    w.integ = dict(w.integ, method=P.PLAN_RK4)
    T = w.terrain
    pl = P.Planner(w.vehicle, w.cost, w.integ, w.K, w.N, T.W, T.H)
    pl.set_terrain(dev(T.height), T.x0, T.y0, T.res)
    u = dev(w.controls)
    out = {}
    for mode in (P.PLAN_ORDER_OFF, P.PLAN_ORDER_ON):
        pl.set_order(mode)
        J, fs = nan(w.K), nan(13, w.K)
        pl.rollout(w.state0, u, J, fs)
        torch.cuda.synchronize()
        out[mode] = (J.cpu().numpy(), fs.cpu().numpy(), pl.get_order())
    assert out[P.PLAN_ORDER_ON][2] and not out[P.PLAN_ORDER_OFF][2]
    for a, b in zip(out[P.PLAN_ORDER_OFF][:2], out[P.PLAN_ORDER_ON][:2]):
        assert not np.isnan(b).any()
        np.testing.assert_array_equal(a, b)
    pl.close()


def test_ordered_gaussian_draws_with_nominal_bitwise():
    # the proxy draws the same Gaussian controls as the rollout, around a
    # nominal sequence, with candidate 0 kept on the nominal
    w = inputs.c2(K=4000, N=16)
    T = w.terrain
    pl = P.Planner(w.vehicle, w.cost, w.integ, w.K, w.N, T.W, T.H)
    pl.set_terrain(dev(T.height), T.x0, T.y0, T.res)
    nominal = dev(np.stack([0.2 * np.sin(np.arange(16) / 3.0),
                            0.3 * np.ones(16)], axis=1))
    spec = P.sample_spec(P.PLAN_SAMPLE_GAUSSIAN, 91, 2, (0.5, 0.2), nominal=nominal,
                         keep_nominal=True, N=16)
    res = {}
    for mode in (P.PLAN_ORDER_OFF, P.PLAN_ORDER_ON):
        pl.set_order(mode)
        J, fs, plan = nan(w.K), nan(13, w.K), nan(16, 2)
        r = pl.rollout_sampled_argmin(w.state0, spec, 16, J, plan, fs)
        torch.cuda.synchronize()
        res[mode] = (J.cpu().numpy(), fs.cpu().numpy(), plan.cpu().numpy(), r)
    off, on = res[P.PLAN_ORDER_OFF], res[P.PLAN_ORDER_ON]
    assert off[3] == on[3]
    for a, b in zip(off[:3], on[:3]):
        assert not np.isnan(b).any()
        np.testing.assert_array_equal(a, b)
    pl.close()


def test_invalid_order_mode_is_rejected_and_keeps_the_mode():
    w = inputs.c1(K=64, N=10)
    c = Ctx(w, 64)
    with pytest.raises(P.PlanError) as e:
        c.pl.set_order(3)
    assert e.value.status == P.PLAN_EINVAL
    # the previous (default, automatic) mode is kept: a small launch stays unordered
    J = nan(64)
    c.pl.rollout(w.state0, dev(w.controls), J)
    torch.cuda.synchronize()
    assert not c.pl.get_order() and not np.isnan(J.cpu().numpy()).any()
    c.pl.close()

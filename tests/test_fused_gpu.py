"""The one-launch planning calls (plan_rollout_argmin,
plan_rollout_sampled_argmin) against the two-call sequences they fuse, bit
for bit, and against the oracle's selection."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402
from tests.parity import assert_argmin_parity, assert_rollout_parity  # noqa: E402
from tests.test_parity_gpu import SHAPES, Case, dev  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def c2case():
    return Case(inputs.c2(K=3000), max_K=4096)


def two_call(case, u, lanes, block):
    N, _, K = u.shape
    J = torch.empty(K, device="cuda")
    fs = torch.empty(13, K, device="cuda")
    plan = torch.empty(N, 2, device="cuda")
    case.planner.set_launch(lanes, block)
    case.planner.rollout(case.w.state0, u, J, fs)
    r = case.planner.select(u, J, plan)
    return J, fs, plan, r


def fused(case, u, lanes, block):
    N, _, K = u.shape
    J = torch.empty(K, device="cuda")
    fs = torch.empty(13, K, device="cuda")
    plan = torch.full((N, 2), 9.0, device="cuda")
    case.planner.set_launch(lanes, block)
    r = case.planner.rollout_argmin(case.w.state0, u, J, plan, fs)
    return J, fs, plan, r


@pytest.mark.parametrize("lanes,block", SHAPES)
def test_fused_equals_rollout_then_select_bitwise(c2case, lanes, block):
    u = dev(c2case.w.controls)
    a = two_call(c2case, u, lanes, block)
    b = fused(c2case, u, lanes, block)
    torch.cuda.synchronize()
    c2case.planner.set_launch(0, 0)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert torch.equal(a[2], b[2]) and a[3] == b[3]


def test_repeated_and_resized_fused_calls_reset_their_reduction(c2case):
    """Every call starts from a clean slot: a sequence of calls with
    different K (different grids) gives each call's own argmin."""
    w = c2case.w
    for K in (3000, 17, 1, 2048, 3000):
        u = dev(np.ascontiguousarray(w.controls[:, :, :K]))
        a = two_call(c2case, u, 0, 0)
        b = fused(c2case, u, 0, 0)
        torch.cuda.synchronize()
        assert a[3] == b[3] and torch.equal(a[2], b[2]), K
        assert torch.equal(a[0], b[0])


def test_fused_asynchronous_call_then_wait(c2case):
    u = dev(c2case.w.controls)
    N, _, K = u.shape
    J = torch.empty(K, device="cuda")
    plan = torch.empty(N, 2, device="cuda")
    assert c2case.planner.rollout_argmin(c2case.w.state0, u, J, plan, want_result=False) is None
    torch.cuda.synchronize()
    ref = two_call(c2case, u, 0, 0)
    torch.cuda.synchronize()
    assert torch.equal(plan, ref[2])


def test_fused_all_non_finite_gives_minus_one_and_zero_plan(c2case):
    u = c2case.w.controls[:, :, :256].copy()
    u[0, 0, :] = np.nan
    b = fused(c2case, dev(u), 0, 0)
    torch.cuda.synchronize()
    assert b[3][0] == -1 and b[3][1] == float("inf")
    assert torch.count_nonzero(b[2]).item() == 0
    assert torch.isinf(b[0]).all()


def test_fused_matches_oracle_on_c1():
    case = Case(inputs.c1())
    u = dev(case.w.controls)
    J, fs, plan, (bk, bc) = fused(case, u, 0, 0)
    torch.cuda.synchronize()
    Jo, fso, _ = case.oracle()
    assert_rollout_parity(J.cpu().numpy(), fs.cpu().numpy(), Jo, fso, "c1 fused")
    assert_argmin_parity(bk, Jo)
    kb, _, plan_o = case.o.select(case.w.controls, J.cpu().numpy())
    assert kb == bk
    assert np.array_equal(plan.cpu().numpy(), plan_o.astype(np.float32))


@pytest.mark.parametrize("lanes,block", [(1, 256), (4, 64)])
def test_sampled_fused_equals_sampled_two_call(lanes, block):
    w = inputs.paper_shape(K=5000)
    case = Case(w)
    spec = P.sample_spec(P.PLAN_SAMPLE_UNIFORM, 6000, 3, (1.0, 0.0))
    N, K = 16, w.K
    case.planner.set_launch(lanes, block)
    J1 = torch.empty(K, device="cuda")
    p1 = torch.empty(N, 2, device="cuda")
    case.planner.rollout_sampled(w.state0, spec, N, J1)
    r1 = case.planner.select_sampled(spec, J1, p1)
    J2 = torch.empty(K, device="cuda")
    p2 = torch.empty(N, 2, device="cuda")
    r2 = case.planner.rollout_sampled_argmin(w.state0, spec, N, J2, p2)
    torch.cuda.synchronize()
    case.planner.set_launch(0, 0)
    assert r1 == r2 and torch.equal(J1, J2) and torch.equal(p1, p2)


def test_host_results_never_stale_across_contexts():
    # each context's pinned result record may reuse memory a destroyed context
    # published into; the reported (k*, J*) must be this call's
    for seed in (11, 12, 13, 14, 15, 16):
        w = inputs.c1(seed=seed)
        T = w.terrain
        pl = P.Planner(w.vehicle, w.cost, w.integ, w.K, w.N, T.W, T.H)
        pl.set_terrain(dev(T.height), T.x0, T.y0, T.res)
        u = dev(w.controls)
        J = torch.empty(w.K, device="cuda")
        plan = torch.empty(w.N, 2, device="cuda")
        for _ in range(seed % 3 + 1):
            k, jb = pl.rollout_argmin(w.state0, u, J, plan)
            torch.cuda.synchronize()
            Jh = J.cpu().numpy()
            assert k == int(np.argmin(Jh)) and np.float32(jb) == Jh[k]
        k2, jb2 = pl.select(u, J, plan)
        assert (k2, jb2) == (k, jb)
        pl.close()


def test_fused_argument_errors(c2case):
    u = dev(c2case.w.controls)
    N, _, K = u.shape
    J = torch.empty(K, device="cuda")
    lib = P.lib()
    s0 = (P.C.c_float * 13)(*c2case.w.state0)
    ptr = lambda t: P.C.c_void_p(t.data_ptr())  # noqa: E731
    assert lib.plan_rollout_argmin(c2case.planner.ctx, s0, ptr(u), K, N, ptr(J), None, None,
                                   None, None) == P.PLAN_EINVAL
    assert lib.plan_rollout_argmin(c2case.planner.ctx, s0, ptr(u), 5000, N, ptr(J), None,
                                   ptr(J), None, None) == P.PLAN_EINVAL
    spec = P.sample_spec(5, 0, 0, (1.0, 0.0))
    assert lib.plan_rollout_sampled_argmin(c2case.planner.ctx, s0, P.C.byref(spec), K, N,
                                           ptr(J), None, ptr(J), None, None) == P.PLAN_EINVAL

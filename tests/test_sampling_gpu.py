"""GPU parity of on-device candidate sampling (plan_sample_controls,
plan_rollout_sampled, plan_select_sampled) against the oracle's sampler and
rollout, and against the materialised path."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402  (test infrastructure)
from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402
from tests.parity import assert_rollout_parity, assert_horizon_parity  # noqa: E402
from tests.test_parity_gpu import SHAPES, Case, dev  # noqa: E402

pytestmark = pytest.mark.gpu

U, G = P.PLAN_SAMPLE_UNIFORM, P.PLAN_SAMPLE_GAUSSIAN


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def c1big():
    return Case(inputs.c1(), max_K=8192, max_N=160)


def gpu_samples(case, spec, K, N):
    u = torch.empty(N, 2, K, device="cuda")
    case.planner.sample_controls(spec, u)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def f32(x):
    return np.float32(x)


@pytest.mark.parametrize("K,N", [(1, 1), (1000, 37), (4099, 16), (8192, 160)])
def test_uniform_samples_are_bit_exact(c1big, K, N):
    """nominal 0: one FP32 rounding of scale * (2x - 1) on both sides."""
    sc = (f32(1.0), f32(0.37))
    spec = P.sample_spec(U, 2603, 9, sc)
    g = gpu_samples(c1big, spec, K, N)
    ref = oracle.sample_controls(U, 2603, 9, [float(sc[0]), float(sc[1])], K, N)
    assert np.array_equal(g, ref.astype(np.float32))


def _nominal(N, seed=5):
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.5, 0.5, size=(N, 2)).astype(np.float32)


def test_uniform_samples_with_nominal_within_two_roundings(c1big):
    """FP32 rounds scale * t, then nominal + that: the error is at most half
    an ulp of each (the oracle's double result is exact to 1e-16)."""
    K, N = 3001, 50
    nom = _nominal(N)
    nd = dev(nom)
    sc = (f32(0.25), f32(0.6))
    g = gpu_samples(c1big, P.sample_spec(U, 1, 2, sc, nominal=nd, N=N), K, N)
    ref = oracle.sample_controls(U, 1, 2, [float(sc[0]), float(sc[1])], K, N, nominal=nom)
    prod = ref - nom.astype(np.float64)[:, :, None]
    bound = (0.5 * np.spacing(np.abs(prod).astype(np.float32)).astype(np.float64)
             + 0.5 * np.spacing(np.abs(g)).astype(np.float64))
    assert np.all(np.abs(g - ref) <= bound * (1 + 1e-9))


@pytest.mark.parametrize("keep", [False, True])
def test_gaussian_samples_match_oracle(c1big, keep):
    """Box-Muller in FP32 (logf, sqrtf, sincospif: a few ulp each) against
    FP64: |error| <= 2e-6 scale max(1, |z|) plus two ulp of the result."""
    K, N = 2500, 41
    nom = _nominal(N, 8)
    nd = dev(nom)
    sc = (f32(0.1), f32(0.2))
    g = gpu_samples(c1big, P.sample_spec(G, 77, 3, sc, nominal=nd, keep_nominal=keep, N=N),
                    K, N)
    ref = oracle.sample_controls(G, 77, 3, [float(sc[0]), float(sc[1])], K, N, nominal=nom,
                                 keep_nominal=keep)
    z = (ref - nom.astype(np.float64)[:, :, None]) / np.array([sc[0], sc[1]])[None, :, None]
    tol = (2e-6 * np.array([sc[0], sc[1]])[None, :, None] * np.maximum(1.0, np.abs(z))
           + 2 * np.spacing(np.abs(ref).astype(np.float32)))
    err = np.abs(g - ref)
    assert np.all(err <= tol), float(np.max(err / tol))
    if keep:
        assert np.array_equal(g[:, :, 0], nom)


@pytest.mark.parametrize("lanes,block", SHAPES)
def test_sampled_rollout_equals_materialised_rollout_bitwise(c1big, lanes, block):
    K, N = 1500, 50
    nom = np.ascontiguousarray(c1big.w.controls[:, :, 0])
    nd = dev(nom)
    spec = P.sample_spec(G, 11, 0, (0.1, 0.2), nominal=nd, keep_nominal=True, N=N)
    u = torch.empty(N, 2, K, device="cuda")
    c1big.planner.sample_controls(spec, u)
    c1big.planner.set_launch(lanes, block)
    J1 = torch.empty(K, device="cuda")
    fs1 = torch.empty(13, K, device="cuda")
    c1big.planner.rollout(c1big.w.state0, u, J1, fs1)
    J2 = torch.empty(K, device="cuda")
    fs2 = torch.empty(13, K, device="cuda")
    c1big.planner.rollout_sampled(c1big.w.state0, spec, N, J2, fs2)
    torch.cuda.synchronize()
    c1big.planner.set_launch(0, 0)
    assert torch.equal(J1, J2) and torch.equal(fs1, fs2)


def test_c1_scheme_sampled_in_kernel_matches_oracle(c1big):
    """The C1 sampling scheme (Gaussian sigma 0.1 rad/s, 0.2 around the seeded
    nominal, candidate 0 = nominal) drawn in the kernel; the oracle draws its
    own FP64 samples from the same generator and rolls them out in FP64."""
    w = c1big.w
    K, N = 64, 50
    nom = np.ascontiguousarray(w.controls[:, :, 0])
    nd = dev(nom)
    sc = (f32(0.1), f32(0.2))
    spec = P.sample_spec(G, 1001, 0, sc, nominal=nd, keep_nominal=True, N=N)
    J = torch.empty(K, device="cuda")
    fs = torch.empty(13, K, device="cuda")
    c1big.planner.rollout_sampled(w.state0, spec, N, J, fs)
    torch.cuda.synchronize()
    u_o = oracle.sample_controls(G, 1001, 0, [float(sc[0]), float(sc[1])], K, N, nominal=nom,
                                 keep_nominal=True)
    Jo, fso = c1big.o.rollout_d(w.state0.astype(np.float64), u_o)
    ce, se = assert_rollout_parity(J.cpu().numpy(), fs.cpu().numpy(), Jo, fso, "c1 sampled")
    print(f"c1 in-kernel Gaussian samples: max cost err {ce:.3g}, state err {se:.3g} (x tol)")


def test_paper_scheme_sampled_in_kernel_matches_oracle():
    """The paper's scheme (steering rate uniform in [-1, 1] rad/s, no
    acceleration; 16 intervals of 0.25 s at 50 Euler substeps): in-kernel
    samples equal the oracle's bit for bit, so the rollout is compared with
    the whole-horizon rule."""
    w = inputs.paper_shape(K=4096)
    case = Case(w)
    K, N = w.K, 16
    spec = P.sample_spec(U, 6000, 0, (1.0, 0.0))
    J = torch.empty(K, device="cuda")
    fs = torch.empty(13, K, device="cuda")
    case.planner.rollout_sampled(w.state0, spec, N, J, fs)
    torch.cuda.synchronize()
    u_o = oracle.sample_controls(U, 6000, 0, [1.0, 0.0], K, N).astype(np.float32)
    assert np.array_equal(gpu_samples(case, spec, K, N), u_o)
    assert_horizon_parity(J.cpu().numpy(), fs.cpu().numpy(), case.o, w.state0, u_o,
                          "paper scheme sampled in kernel", min_cost=0.99, min_state=0.86)


def test_select_sampled_equals_select_on_materialised(c1big):
    K, N = 5000, 30
    nom = _nominal(N, 3)
    nd = dev(nom)
    spec = P.sample_spec(G, 5, 5, (0.8, 0.9), nominal=nd, N=N)
    u = torch.empty(N, 2, K, device="cuda")
    c1big.planner.sample_controls(spec, u)
    J = torch.empty(K, device="cuda")
    c1big.planner.rollout_sampled(c1big.w.state0, spec, N, J)
    p1 = torch.empty(N, 2, device="cuda")
    p2 = torch.empty(N, 2, device="cuda")
    r1 = c1big.planner.select(u, J, p1)
    r2 = c1big.planner.select_sampled(spec, J, p2)
    torch.cuda.synchronize()
    assert r1 == r2 and torch.equal(p1, p2)
    # the plan is the clamped winner, as the oracle's selection gathers it
    bk, bc, plan = c1big.o.select(u.cpu().numpy(), J.cpu().numpy())
    assert bk == r2[0]
    assert np.array_equal(p2.cpu().numpy(), plan.astype(np.float32))


def test_select_sampled_all_infinite_gives_minus_one(c1big):
    K, N = 300, 12
    spec = P.sample_spec(U, 1, 1, (1.0, 1.0))
    J = torch.full((K,), float("inf"), device="cuda")
    p = torch.full((N, 2), 7.0, device="cuda")
    bk, bc = c1big.planner.select_sampled(spec, J, p)
    assert bk == -1 and bc == float("inf")
    assert torch.count_nonzero(p).item() == 0


def test_sampling_errors(c1big):
    u = torch.empty(4, 2, 8, device="cuda")
    J = torch.empty(8, device="cuda")
    bad = [P.sample_spec(2, 0, 0, (1, 1)), P.sample_spec(U, 0, 0, (-1, 1)),
           P.sample_spec(G, 0, 0, (float("nan"), 1)), P.sample_spec(G, 0, 0, (1, float("inf")))]
    for sp in bad:
        with pytest.raises(P.PlanError) as e:
            c1big.planner.sample_controls(sp, u)
        assert e.value.status == P.PLAN_EINVAL
        with pytest.raises(P.PlanError):
            c1big.planner.rollout_sampled(c1big.w.state0, sp, 4, J)
        with pytest.raises(P.PlanError):
            c1big.planner.select_sampled(sp, J, torch.empty(4, 2, device="cuda"))
    ok = P.sample_spec(U, 0, 0, (1, 1))
    with pytest.raises(P.PlanError):
        c1big.planner.rollout_sampled(c1big.w.state0, ok, 161, J)   # N above max_N
    lib = P.lib()
    assert lib.plan_sample_controls(c1big.planner.ctx, None, 8, 4,
                                    P.C.c_void_p(u.data_ptr())) == P.PLAN_EINVAL


def test_paper_shape_full_size_one_launch_sampled_outputs():
    """The paper's configuration at full size in the launch the bench times
    (K = 204 288 candidates drawn in the kernel, 16 x 0.25 s at 50 Euler
    substeps, argmin epilogue): sampled candidates' costs against the oracle's
    own draws and rollouts for every candidate, and the selection against the
    cost array and against the oracle's costs."""
    T = inputs.fbm_berm_terrain(2000)
    w = inputs.paper_shape(K=8, terrain=T)
    K, N = 204288, 16
    pl = P.Planner(w.vehicle, w.cost, w.integ, K, N, T.W, T.H)
    pl.set_terrain(dev(T.height), T.x0, T.y0, T.res)
    spec = P.sample_spec(U, 6000, 0, (1.0, 0.0))
    J = torch.empty(K, device="cuda")
    fs = torch.empty(13, K, device="cuda")
    plan = torch.empty(N, 2, device="cuda")
    bk, bc = pl.rollout_sampled_argmin(w.state0, spec, N, J, plan, fs)
    torch.cuda.synchronize()
    Jg = J.cpu().numpy()
    # selection: lowest index of the minimal finite cost, its controls regenerated
    fin = np.isfinite(Jg)
    assert bk == int(np.flatnonzero(Jg == Jg[fin].min())[0]) and bc == Jg[bk]
    u_best = oracle.sample_controls(U, 6000, 0, [1.0, 0.0], K, N)[:, :, bk]
    expect = np.stack([np.clip(u_best[:, 0], -1.0, 1.0), np.clip(u_best[:, 1], -1.0, 1.0)], 1)
    assert np.array_equal(plan.cpu().numpy(), expect.astype(np.float32))
    # every candidate against the oracle's own draws and rollouts, and the
    # launch's pick against the oracle's costs
    u_all = oracle.sample_controls(U, 6000, 0, [1.0, 0.0], K, N).astype(np.float32)
    o = oracle.Oracle(w.vehicle, w.cost, w.integ)
    o.set_terrain(T.height, T.x0, T.y0, T.res)
    assert_horizon_parity(Jg, fs.cpu().numpy(), o, w.state0, u_all,
                          "paper shape full size, one launch", min_cost=0.99, min_state=0.87,
                          k_gpu=bk)
    pl.close()

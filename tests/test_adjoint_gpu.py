"""GPU tests of the adjoint rollout (plan_rollout_grad and the autograd
wrapper): gradients of candidate costs with respect to the controls, checked
against FP64 central finite differences of the oracle (step 1e-6)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402  (test infrastructure)
from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402

pytestmark = pytest.mark.gpu

# relative to max(|fd|, 1e-2 of the candidate's largest |fd|); the worst entry
# seen is 2.5e-3 (C4 top 32), the FP32 forward's own sensitivity to rounding
GRAD_RTOL = 5e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    yield
    torch.cuda.synchronize()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def setup(w):
    T = w.terrain
    pl = P.Planner(w.vehicle, w.cost, w.integ, w.K, w.N, T.W, T.H)
    pl.set_terrain(dev(T.height), T.x0, T.y0, T.res)
    o = oracle.Oracle(w.vehicle, w.cost, w.integ)
    o.set_terrain(T.height, T.x0, T.y0, T.res)
    return pl, o


def gpu_grad(pl, w, controls, ckpt=10, weight=None):
    N, _, K = controls.shape
    u = dev(controls)
    J = torch.empty(K, device="cuda")
    g = torch.empty(N, 2, K, device="cuda")
    pl.rollout_grad(w.state0, u, J, g, None if weight is None else dev(weight), ckpt)
    torch.cuda.synchronize()
    return J.cpu().numpy(), g.cpu().numpy()


def compare_fd(o, w, controls, g, ks, n_entries=24, seed=0, label=""):
    """Central differences on sampled entries of candidates ks; entries whose
    one-sided differences disagree (a kink or a discontinuity within +-1e-6)
    are skipped. Returns (worst normalised error, compared, skipped)."""
    rng = np.random.default_rng(seed)
    N = controls.shape[0]
    worst, used, skipped = 0.0, 0, 0
    for k in ks:
        ent = [(int(rng.integers(0, N)), int(rng.integers(0, 2))) for _ in range(n_entries)]
        fd, fp, fm = o.fd_grad(w.state0, controls, k, ent)
        smooth = np.abs(fp - fm) <= 1e-3 * np.maximum(np.abs(fd), 1e-2)
        scale = max(np.max(np.abs(fd[smooth])) if smooth.any() else 0.0, 1e-3)
        for (n, c), f, ok in zip(ent, fd, smooth):
            if not ok:
                skipped += 1
                continue
            err = abs(g[n, c, k] - f) / (GRAD_RTOL * max(abs(f), 1e-2 * scale))
            assert err <= 1.0, (f"{label}: candidate {k} u[{n}][{c}]: gpu {g[n, c, k]!r} "
                                f"vs fd {f!r} ({err:.3g}x tol)")
            worst = max(worst, err)
            used += 1
    return worst, used, skipped


def test_c4_top32_gradients_against_fp64_finite_differences():
    w = inputs.c4()
    pl, o = setup(w)
    u_all = dev(w.controls)
    J = torch.empty(w.K, device="cuda")
    pl.rollout(w.state0, u_all, J)
    top = np.argsort(J.cpu().numpy(), kind="stable")[:32]
    sub = np.ascontiguousarray(w.controls[:, :, top])
    Jg, g = gpu_grad(pl, w, sub)
    np.testing.assert_array_equal(Jg, J.cpu().numpy()[top])
    worst, used, skipped = compare_fd(o, w, sub, g, range(32), label="c4 top-32")
    print(f"c4 top-32: {used} gradient entries vs FP64 FD, worst {worst:.3g} x tol, "
          f"{skipped} skipped at kinks")
    assert used >= 0.8 * 32 * 24


def test_c1_gradients_every_candidate_sampled():
    w = inputs.c1(K=16)
    pl, o = setup(w)
    _, g = gpu_grad(pl, w, w.controls)
    worst, used, skipped = compare_fd(o, w, w.controls, g, range(16), n_entries=12, label="c1")
    print(f"c1: {used} entries, worst {worst:.3g} x tol, {skipped} skipped")
    assert used >= 0.8 * 16 * 12


def test_checkpoint_interval_does_not_change_the_gradient():
    w = inputs.c2(K=256)
    pl, _ = setup(w)
    ref = gpu_grad(pl, w, w.controls, ckpt=10)
    for c in (1, 7, 100, 1000):
        J, g = gpu_grad(pl, w, w.controls, ckpt=c)
        np.testing.assert_array_equal(J, ref[0])
        np.testing.assert_array_equal(g, ref[1])


def test_lanes_per_candidate_do_not_change_the_gradient():
    """The backward kernel splits each candidate's wheels over 1, 2 or 4 lanes
    and sums their adjoints in the forward's fixed order: identical bits."""
    w = inputs.c2(K=333)
    pl, _ = setup(w)
    pl.set_launch(1, 64)
    ref = gpu_grad(pl, w, w.controls, ckpt=10)
    for lanes in (2, 4):
        pl.set_launch(lanes, 64)
        J, g = gpu_grad(pl, w, w.controls, ckpt=10)
        np.testing.assert_array_equal(J, ref[0])
        np.testing.assert_array_equal(g, ref[1])
    pl.set_launch(0, 0)


def test_weights_scale_the_gradient_and_autograd_matches():
    from paper_2603_20525_amd.autograd import RolloutCost
    w = inputs.c1(K=32)
    pl, _ = setup(w)
    wt = np.linspace(0.5, 2.0, 32).astype(np.float32)
    _, g1 = gpu_grad(pl, w, w.controls)
    _, gw = gpu_grad(pl, w, w.controls, weight=wt)
    np.testing.assert_allclose(gw, g1 * wt[None, None, :], rtol=1e-5, atol=1e-7)
    u = dev(w.controls).requires_grad_(True)
    J = RolloutCost.apply(u, pl, w.state0, 10)
    (J * dev(wt)).sum().backward()
    np.testing.assert_array_equal(u.grad.cpu().numpy(), gw)


def test_clamped_controls_and_infinite_candidates_get_zero_gradient():
    w = inputs.c1(K=8)
    pl, _ = setup(w)
    u = w.controls.copy()
    u[5, 0, 2] = 3.0       # beyond the steering-rate limit
    u[7, 1, 4] = -2.0      # beyond full braking
    u[3, 0, 6] = np.nan    # candidate 6 becomes non-finite
    J, g = gpu_grad(pl, w, u)
    assert g[5, 0, 2] == 0.0 and g[7, 1, 4] == 0.0
    assert np.isinf(J[6]) and np.all(g[:, :, 6] == 0.0)
    assert np.all(np.isfinite(g))


def test_goal_exit_freezes_later_gradients():
    w = inputs.c1(K=8)
    w.cost["goal_x"], w.cost["goal_y"] = 9.0, 12.8
    pl, o = setup(w)
    _, F, ex = o.rollout(w.state0, w.controls)
    J, g = gpu_grad(pl, w, w.controls)
    for k in range(8):
        if ex[k] >= 0:
            assert np.all(g[ex[k] + 2:, :, k] == 0.0)


def test_paper_shape_substeps_gradient():
    w = inputs.paper_shape(K=8)
    pl, o = setup(w)
    _, g = gpu_grad(pl, w, w.controls, ckpt=2)
    worst, used, skipped = compare_fd(o, w, w.controls, g, range(0, 8, 2), n_entries=8,
                                      label="paper shape")
    print(f"paper shape: {used} entries, worst {worst:.3g} x tol, {skipped} skipped")
    assert used >= 0.75 * 4 * 8

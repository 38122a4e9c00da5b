"""GPU parity of terrain preparation (plan_smooth_terrain,
plan_costmap_polygons) against the oracle, and a rollout over a costmap each
side builds itself."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402  (test infrastructure)
from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402
from tests.parity import assert_horizon_parity  # noqa: E402
from tests.test_parity_gpu import dev  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    yield
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def planner():
    w = inputs.c1()
    pl = P.Planner(w.vehicle, w.cost, w.integ, 64, 50, 2048, 2048)
    yield pl
    pl.close()


def smooth_tol(h, res, sigma):
    """Two FP32 passes of 2r+1 normalised taps: each sum carries at most
    (2r+2) roundings of 2^-24 of max|h| (taps included)."""
    r = math.ceil(3 * sigma / res - 1e-6)
    return 2 * (2 * r + 2) * 2.0 ** -24 * float(np.abs(h).max()) + 1e-12


@pytest.mark.parametrize("shape,res,sigma", [((512, 512), 0.1, 0.3), ((512, 512), 0.1, 1.5),
                                             ((77, 131), 0.1, 0.3), ((300, 41), 0.05, 0.3),
                                             ((1, 9), 0.1, 0.3), ((256, 256), 0.1, 4.2)])
def test_smoothing_matches_oracle(planner, shape, res, sigma):
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    if shape == (512, 512):
        h = inputs.c2().terrain.height
    else:
        h = rng.normal(0.0, 0.3, size=shape).astype(np.float32)
    out = torch.empty(shape, device="cuda")
    planner.smooth_terrain(dev(h), res, sigma, out)
    torch.cuda.synchronize()
    # the library receives res and sigma as float32: so does the oracle
    ref = oracle.smooth_terrain(h, float(np.float32(res)), float(np.float32(sigma)))
    err = np.abs(out.cpu().numpy() - ref).max()
    assert err <= smooth_tol(h, res, sigma), (err, smooth_tol(h, res, sigma))


def test_smoothing_in_place_and_lod_pipeline(planner):
    """The paper's two levels of detail of the full 2048 x 2048 C5 map, in
    place, then packed as a terrain. The oracle smooths a crop; nodes at
    least r from the crop's edges see the same neighbourhood as in the full
    map, so they are compared there."""
    T = inputs.c5(K=64, N=10).terrain
    j0, i0, n = 800, 900, 320
    crop = np.ascontiguousarray(T.height[j0:j0 + n, i0:i0 + n])
    for sigma in (0.3, 1.5):
        r = math.ceil(3 * sigma / T.res - 1e-6)
        h = dev(T.height)
        planner.smooth_terrain(h, T.res, sigma, h)
        torch.cuda.synchronize()
        ref = oracle.smooth_terrain(crop, float(np.float32(T.res)),
                                    float(np.float32(sigma)))[r:n - r, r:n - r]
        got = h.cpu().numpy()[j0 + r:j0 + n - r, i0 + r:i0 + n - r]
        assert np.abs(got - ref).max() <= smooth_tol(T.height, T.res, sigma)
        planner.set_terrain(h, T.x0, T.y0, T.res)


def test_smoothing_argument_errors(planner):
    h = torch.zeros(16, 16, device="cuda")
    with pytest.raises(P.PlanError):
        planner.smooth_terrain(h, 0.1, 12.8, h)          # r = 384 > 127
    with pytest.raises(P.PlanError):
        planner.smooth_terrain(h, 0.0, 0.3, h)
    with pytest.raises(P.PlanError):
        planner.smooth_terrain(torch.zeros(16, 4096, device="cuda"), 0.1, 0.3,
                               torch.zeros(16, 4096, device="cuda"))   # W above max


def costmap_tol(ref, coord_max, sigma=1e6, eps=0.25, n_poly=1):
    """FP32 geometry: a signed distance is off by at most ~16 ulp of the
    coordinate magnitude; the cost's slope in sdist is 2 sigma / eps
    sqrt(cost / sigma) per perimeter."""
    dsd = 16 * np.spacing(np.float32(coord_max))
    slope = 2 * sigma / eps * np.sqrt(np.maximum(ref, 0) / sigma) * math.sqrt(n_poly)
    return 1e-6 * ref + slope * dsd + 1e-3


def gpu_costmap(planner, polys, T, accumulate_from=None):
    verts, offsets, kinds = oracle.polygon_arrays(polys)
    vd = dev(verts) if len(verts) else None
    cm = dev(accumulate_from) if accumulate_from is not None else torch.empty(T.H, T.W,
                                                                              device="cuda")
    planner.costmap_polygons(vd, offsets, kinds, cm, T.x0, T.y0, T.res, 1e6, 0.25,
                             accumulate=accumulate_from is not None)
    torch.cuda.synchronize()
    return cm.cpu().numpy()


def test_costmap_matches_oracle_c2_scene(planner):
    T = inputs.c2(K=8, N=4).terrain
    polys = inputs.obstacle_polygons(T, seed=5, count=20, boundary=True)
    g = gpu_costmap(planner, polys, T)
    ref = oracle.costmap_polygons(polys, T.W, T.H, T.x0, T.y0, T.res, 1e6, 0.25)
    tol = costmap_tol(ref, T.W * T.res, n_poly=len(polys))
    assert np.all(np.abs(g - ref) <= tol), float(np.max(np.abs(g - ref) / tol))
    assert (ref > 0).mean() > 0.02 and (ref == 0).mean() > 0.2


def test_costmap_accumulate_and_empty(planner):
    T = inputs.c1(K=8, N=4).terrain
    polys = inputs.obstacle_polygons(T, seed=9, count=6)
    base = np.full((T.H, T.W), 3.0, np.float32)
    g = gpu_costmap(planner, polys, T, accumulate_from=base)
    ref = oracle.costmap_polygons(polys, T.W, T.H, T.x0, T.y0, T.res, 1e6, 0.25) + 3.0
    assert np.all(np.abs(g - ref) <= costmap_tol(ref, T.W * T.res, n_poly=6) + 1e-6 * 3)
    z = gpu_costmap(planner, [], T)
    assert np.count_nonzero(z) == 0


def test_costmap_argument_errors(planner):
    cm = torch.zeros(8, 8, device="cuda")
    sq = dev(np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32))
    bad = [([0, 2], [0]), ([0, 4], [2]), ([1, 4], [0]), ([0, 5], [0])]
    for off, kd in bad:
        with pytest.raises(P.PlanError) as e:
            planner.costmap_polygons(sq, off, kd, cm, 0, 0, 0.1, 1e6, 0.25)
        assert e.value.status == P.PLAN_EINVAL
    with pytest.raises(P.PlanError):
        planner.costmap_polygons(sq, [0, 4], [0], cm, 0, 0, 0.1, 1e6, 0.0)


def test_rollout_over_costmaps_each_side_builds():
    """C1 with obstacles: the GPU builds its costmap with its own kernel, the
    oracle with its own code; the rollouts must agree (whole-horizon rule)."""
    w = inputs.c1(K=512)
    T = w.terrain
    polys = inputs.obstacle_polygons(T, seed=77, count=8)
    pl = P.Planner(w.vehicle, w.cost, w.integ, w.K, w.N, T.W, T.H)
    verts, offsets, kinds = oracle.polygon_arrays(polys)
    cm = torch.empty(T.H, T.W, device="cuda")
    pl.costmap_polygons(dev(verts), offsets, kinds, cm, T.x0, T.y0, T.res, 1e6, 0.25)
    h = dev(T.height)
    pl.set_terrain(h, T.x0, T.y0, T.res, cm)
    J = torch.empty(w.K, device="cuda")
    fs = torch.empty(13, w.K, device="cuda")
    pl.rollout(w.state0, dev(w.controls), J, fs)
    torch.cuda.synchronize()
    o = oracle.Oracle(w.vehicle, w.cost, w.integ)
    o.set_terrain(T.height, T.x0, T.y0, T.res,
                  oracle.costmap_polygons(polys, T.W, T.H, T.x0, T.y0, T.res, 1e6, 0.25))
    assert_horizon_parity(J.cpu().numpy(), fs.cpu().numpy(), o, w.state0, w.controls,
                          "rollout over own costmaps", min_cost=0.99, min_state=0.95)
    pl.close()

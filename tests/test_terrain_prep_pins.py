"""Pins of the oracle's terrain preparation: level-of-detail Gaussian
smoothing (section "Terrain Smoothing") and the polygon distance costmap
(sections "OCP Formulation", "Real-Time Implementation"). Checked against 1-D
closed forms of the separable kernel (moments, impulse response, sinusoid
gain, edge clamping), plane geometry, and an independent brute-force distance
and winding-number construction."""
import math

import numpy as np
import pytest

import oracle


def g1(res, sigma):
    """1-D weights of the truncated Gaussian (unnormalised) and offsets."""
    r = math.ceil(3 * sigma / res - 1e-6)
    k = np.arange(-r, r + 1)
    return k, np.exp(-(k * res) ** 2 / (2 * sigma ** 2))


@pytest.mark.parametrize("res,sigma", [(0.1, 0.3), (0.1, 1.5), (0.05, 0.3), (0.2, 0.3)])
def test_constant_and_plane_are_preserved(res, sigma):
    H, W = 60, 70
    k, _ = g1(res, sigma)
    r = k[-1]
    c = np.full((H, W), 1.25, np.float32)
    assert np.allclose(oracle.smooth_terrain(c, res, sigma), 1.25, rtol=0, atol=1e-12)
    J, I = np.mgrid[0:H, 0:W]
    plane = (I / 32.0 - J / 64.0).astype(np.float32)   # exact in float32
    out = oracle.smooth_terrain(plane, res, sigma)
    if H > 2 * r and W > 2 * r:
        inner = (slice(r, H - r), slice(r, W - r))
        assert np.allclose(out[inner], plane.astype(np.float64)[inner], rtol=0, atol=1e-11)


@pytest.mark.parametrize("res,sigma", [(0.1, 0.3), (0.1, 1.5)])
def test_quadratic_gains_the_discrete_kernel_variance(res, sigma):
    """x^2 smoothed = x^2 + Var, Var = sum k^2 res^2 g(k) / sum g(k) of the 1-D
    marginal (the square kernel factorises)."""
    k, g = g1(res, sigma)
    r = k[-1]
    var = float(np.sum((k * res) ** 2 * g) / np.sum(g))
    H, W = 2 * r + 21, 2 * r + 31
    # heights (q / 8)^2 of the node index q: exact in float32; one node is
    # res metres, so the smoothed value gains Var / (8 res)^2
    q = (np.arange(W) - W // 2) / 8.0
    h = np.repeat((q ** 2)[None, :], H, axis=0).astype(np.float32)
    out = oracle.smooth_terrain(h, res, sigma)
    inner = (slice(r, H - r), slice(r, W - r))
    expect = h.astype(np.float64) + var / (8 * res) ** 2
    assert np.allclose(out[inner], expect[inner], rtol=0, atol=1e-10)
    # close to the continuous kernel (3-sigma truncation removes ~2.5 % of the variance)
    assert var == pytest.approx(sigma ** 2, rel=0.03)


def test_impulse_response_is_the_normalised_outer_product():
    res, sigma = 0.1, 0.3
    k, g = g1(res, sigma)
    r = k[-1]
    n = 2 * r + 11
    h = np.zeros((n, n), np.float32)
    c = n // 2
    h[c, c] = 1.0
    out = oracle.smooth_terrain(h, res, sigma)
    gn = g / g.sum()
    expect = np.zeros((n, n))
    expect[c - r:c + r + 1, c - r:c + r + 1] = np.outer(gn, gn)
    assert np.allclose(out, expect, rtol=0, atol=1e-15)


@pytest.mark.parametrize("lam", [1.0, 2.5, 6.4])
def test_sinusoid_gain(lam):
    """sin(2 pi x / lam) keeps its shape with gain sum g(k) cos(2 pi k res / lam)
    / sum g(k), close to the continuous exp(-2 pi^2 sigma^2 / lam^2)."""
    res, sigma = 0.1, 0.3
    k, g = g1(res, sigma)
    r = k[-1]
    gain = float(np.sum(g * np.cos(2 * np.pi * k * res / lam)) / np.sum(g))
    W, H = 160, 2 * r + 5
    x = np.arange(W) * res
    h = np.repeat(np.sin(2 * np.pi * x / lam)[None, :], H, axis=0).astype(np.float32)
    out = oracle.smooth_terrain(h, res, sigma)
    inner = (slice(r, H - r), slice(r, W - r))
    assert np.allclose(out[inner], (gain * h.astype(np.float64))[inner], rtol=0, atol=1e-7)
    assert gain == pytest.approx(math.exp(-2 * math.pi ** 2 * sigma ** 2 / lam ** 2), abs=5e-3)


def test_edges_clamp_to_the_nearest_node():
    """h = row index j: at row 0 the rows above the grid read as row 0."""
    res, sigma = 0.1, 0.3
    k, g = g1(res, sigma)
    H, W = 30, 12
    h = np.repeat(np.arange(H, dtype=np.float32)[:, None], W, axis=1)
    out = oracle.smooth_terrain(h, res, sigma)
    for j in (0, 1, H - 1):
        expect = float(np.sum(g * np.clip(j + k, 0, H - 1)) / np.sum(g))
        assert np.allclose(out[j], expect, rtol=0, atol=1e-12)


def test_smoothing_commutes_with_flips():
    rng = np.random.default_rng(3)
    h = rng.normal(size=(37, 41)).astype(np.float32)
    out = oracle.smooth_terrain(h, 0.1, 0.3)
    assert np.allclose(oracle.smooth_terrain(h[::-1, :].copy(), 0.1, 0.3), out[::-1, :],
                       rtol=0, atol=1e-13)
    assert np.allclose(oracle.smooth_terrain(h[:, ::-1].copy(), 0.1, 0.3), out[:, ::-1],
                       rtol=0, atol=1e-13)


# ------------------------------------------------------------------ costmap

SIG, EPS = 1e6, 0.25


def soft(pi):
    return SIG * max(0.0, 1.0 + pi / EPS) ** 2


def _single(poly, kind, x, y):
    """Cost at one point, from a 1x1 grid placed there."""
    return oracle.costmap_polygons([(kind, poly)], 1, 1, x, y, 1.0, SIG, EPS)[0, 0]


SQUARE = [(0.0, 0.0), (2.0, 0.0), (2.0, 2.0), (0.0, 2.0)]


def test_square_obstacle_closed_forms():
    # centre: sdist = -1
    assert _single(SQUARE, oracle.OBSTACLE, 1.0, 1.0) == pytest.approx(soft(1.0), rel=1e-12)
    # inside near an edge: depth 0.1
    assert _single(SQUARE, oracle.OBSTACLE, 1.0, 0.1) == pytest.approx(soft(0.1), rel=1e-12)
    # outside, beside an edge: perpendicular distance 0.1
    assert _single(SQUARE, oracle.OBSTACLE, 1.0, -0.1) == pytest.approx(soft(-0.1), rel=1e-12)
    # outside a corner: distance to the vertex
    d = math.hypot(0.1, 0.15)
    assert _single(SQUARE, oracle.OBSTACLE, -0.1, -0.15) == pytest.approx(soft(-d), rel=1e-12)
    # beyond eps from the perimeter: nothing
    assert _single(SQUARE, oracle.OBSTACLE, 1.0, -0.26) == 0.0
    # on the perimeter: sigma
    assert _single(SQUARE, oracle.OBSTACLE, 2.0, 1.0) == pytest.approx(SIG, rel=1e-12)


def test_path_boundary_reverses_the_sign():
    assert _single(SQUARE, oracle.PATH_BOUNDARY, 1.0, 1.0) == 0.0
    assert _single(SQUARE, oracle.PATH_BOUNDARY, 1.0, 0.1) == pytest.approx(soft(-0.1), rel=1e-12)
    assert _single(SQUARE, oracle.PATH_BOUNDARY, 1.0, -0.3) == pytest.approx(soft(0.3), rel=1e-12)


def test_orientation_and_start_vertex_do_not_matter():
    star = [(math.cos(t) * (1.5 if q % 2 else 0.6) + 3.0, math.sin(t) * (1.5 if q % 2 else 0.6) + 3.0)
            for q, t in enumerate(np.linspace(0, 2 * np.pi, 11)[:-1])]
    a = oracle.costmap_polygons([(0, star)], 60, 60, 0.0, 0.0, 0.1, SIG, EPS)
    b = oracle.costmap_polygons([(0, star[::-1])], 60, 60, 0.0, 0.0, 0.1, SIG, EPS)
    c = oracle.costmap_polygons([(0, star[3:] + star[:3])], 60, 60, 0.0, 0.0, 0.1, SIG, EPS)
    assert np.allclose(a, b, rtol=1e-12, atol=0) and np.allclose(a, c, rtol=1e-12, atol=0)


def test_two_perimeters_add():
    a = [(0.0, 0.0), (1.0, 0.0), (1.0, 1.0), (0.0, 1.0)]
    b = [(1.2, 0.0), (2.2, 0.0), (2.2, 1.0)]
    one = oracle.costmap_polygons([(0, a)], 40, 20, -0.5, -0.5, 0.1, SIG, EPS)
    two = oracle.costmap_polygons([(0, b)], 40, 20, -0.5, -0.5, 0.1, SIG, EPS)
    both = oracle.costmap_polygons([(0, a), (0, b)], 40, 20, -0.5, -0.5, 0.1, SIG, EPS)
    assert np.allclose(both, one + two, rtol=1e-12, atol=0)


def test_non_convex_polygon_against_brute_force_distance_and_winding():
    """Distance by dense sampling of the perimeter (error below the sample
    spacing) and inside by the winding number (sum of subtended angles)."""
    rng = np.random.default_rng(11)
    t = np.sort(rng.uniform(0, 2 * np.pi, 9))
    rad = rng.uniform(0.5, 1.6, 9)
    poly = [(2.0 + r * math.cos(a), 2.0 + r * math.sin(a)) for r, a in zip(rad, t)]
    P = np.asarray(poly + poly[:1])
    samples = np.concatenate([np.linspace(P[e], P[e + 1], 4001) for e in range(len(poly))])
    spacing = max(np.linalg.norm(P[e + 1] - P[e]) for e in range(len(poly))) / 4000
    n, res, x0 = 41, 0.1, 0.0
    cm = oracle.costmap_polygons([(0, poly)], n, n, x0, x0, res, SIG, EPS)
    for j in range(0, n, 3):
        for i in range(0, n, 3):
            q = np.array([x0 + i * res, x0 + j * res])
            d = np.min(np.linalg.norm(samples - q, axis=1))
            v = P - q
            ang = np.arctan2(v[1:, 1], v[1:, 0]) - np.arctan2(v[:-1, 1], v[:-1, 0])
            ang = (ang + np.pi) % (2 * np.pi) - np.pi
            inside = abs(ang.sum()) > np.pi
            sd = -d if inside else d
            lo = soft(-(sd + spacing)) if not inside else soft(-(sd + spacing))
            hi = soft(-(sd - spacing))
            assert min(lo, hi) - 1e-6 <= cm[j, i] <= max(lo, hi) + 1e-6, (i, j)


def test_invalid_polygons_are_rejected():
    with pytest.raises(ValueError):
        oracle.costmap_polygons([(0, [(0, 0), (1, 0)])], 4, 4, 0, 0, 1, SIG, EPS)
    with pytest.raises(ValueError):
        oracle.costmap_polygons([(2, SQUARE)], 4, 4, 0, 0, 1, SIG, EPS)
    with pytest.raises(ValueError):
        oracle.smooth_terrain(np.zeros((4, 4), np.float32), 0.1, 0.0)

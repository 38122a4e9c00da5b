"""Pins of the oracle's fourth-order Runge-Kutta option (section "Real-Time
Implementation": forward Euler at 5 ms was chosen over the alternative
fourth-order Runge-Kutta method the paper compared). Checked against exact
polynomial and linear-oscillator solutions of the scheme, fourth-order
convergence, and agreement with Euler as the step shrinks."""
import numpy as np
import pytest

import oracle
from paper_2603_20525_amd import inputs
from tests.test_oracle_pins import _cost, _grid, _integ, _oracle, _veh, state


def rk4(**kw):
    return _integ(method=1, **kw)


def test_free_fall_is_exact():
    """Airborne, the model is z'' = -g: a quadratic, which RK4 integrates
    exactly (Euler does not)."""
    v = _veh()
    N, dt, vz0 = 10, 0.02, 0.5
    o = _oracle(v, cost=_cost(goal_x=200.0, goal_y=0.0), integ=rk4())
    s0 = state(z=v["hR"] + 1.0, v=(5.0, 0.0, vz0)).astype(np.float32)
    J, fs, _ = o.rollout(s0, np.zeros((N, 2, 1), np.float32))
    t = N * dt
    assert fs[2, 0] == pytest.approx(float(s0[2]) + float(s0[8]) * t - v["g"] * t * t / 2,
                                     rel=1e-13)
    assert fs[8, 0] == pytest.approx(float(s0[8]) - v["g"] * t, rel=1e-12)
    assert J[0] == pytest.approx(5.0 * t + 15.0 * (200.0 - 5.0 * t), rel=1e-12)


def test_undamped_heave_follows_the_rk4_amplification_matrix():
    """Pure heave with the dampers off is e'' = -w^2 e; one RK4 step maps
    (e, e') by sum_{m<=4} (hA)^m / m! with A = [[0, 1], [-w^2, 0]]."""
    v = _veh(Lf=1.2, Lr=1.2, kf=5.0e4, kr=5.0e4, bf=0.0, br=0.0)
    N, dt, e0 = 12, 0.02, 0.01
    o = _oracle(v, integ=rk4())
    s0 = state(z=v["hR"] + e0, v=(5.0, 0, 0)).astype(np.float32)
    J, fs, _ = o.rollout(s0, np.zeros((N, 2, 1), np.float32))
    w2 = 2.0 * (v["kf"] + v["kr"]) / v["M"]
    A = np.array([[0.0, 1.0], [-w2, 0.0]]) * dt
    step = np.eye(2) + A + A @ A / 2 + A @ A @ A / 6 + A @ A @ A @ A / 24
    eN, vN = np.linalg.matrix_power(step, N) @ np.array([float(s0[2]) - v["hR"], 0.0])
    assert fs[2, 0] - v["hR"] == pytest.approx(eN, rel=1e-9, abs=1e-13)
    assert fs[8, 0] == pytest.approx(vN, rel=1e-9, abs=1e-13)
    # energy decays slightly (|R(i w h)| < 1), unlike Euler's growth
    E0 = 0.5 * w2 * (float(s0[2]) - v["hR"]) ** 2
    EN = 0.5 * fs[8, 0] ** 2 + 0.5 * w2 * (fs[2, 0] - v["hR"]) ** 2
    assert EN < E0


def test_fourth_order_convergence_on_a_smooth_manoeuvre():
    """Steering on an inclined plane: no liftoff, no cell-boundary kinks (the
    bilinear interpolant reproduces a plane), so the trajectory is smooth and
    successive differences shrink 16-fold per halving of h."""
    v = _veh()
    terr = _grid(lambda X, Y: 0.125 * X - 0.0625 * Y, n=161, res=0.25, x0=-20.0, y0=-20.0)
    o0 = _oracle(v, terrain=terr)
    N = 10
    u = np.zeros((N, 2, 1), np.float32)
    u[:, 0, 0] = 0.4 * np.cos(np.arange(N) * 0.5)
    u[:, 1, 0] = 0.2
    s0 = inputs.settled_state(inputs.Terrain(terr[0], terr[1], terr[2], terr[3]), 0.0, 0.0,
                              0.3, 6.0, v["hR"])
    finals = []
    for S in (8, 16, 32, 64):
        o = _oracle(v, terrain=terr, integ=rk4(dt=0.1, substeps=S))
        _, fs, _ = o.rollout(s0, u)
        finals.append(fs[:, 0])
    d = [np.linalg.norm(finals[i] - finals[i + 1]) for i in range(3)]
    for i in range(2):
        assert 12.0 < d[i] / d[i + 1] < 20.0, d
    del o0


def test_rk4_and_euler_converge_to_the_same_trajectory():
    T = inputs.bumps_terrain(1000)
    v = _veh()
    s0 = inputs.settled_state(T, 5.0, 12.8, 0.0, 5.0, v["hR"])
    N = 10
    u = np.zeros((N, 2, 1), np.float32)
    u[:, 0, 0] = 0.3 * np.sin(np.arange(N) * 0.3)
    out = {}
    for m, S in ((0, 400), (1, 40)):
        o = oracle.Oracle(v, _cost(goal_x=100.0, goal_y=0.0), _integ(dt=0.05, substeps=S,
                                                                      method=m))
        o.set_terrain(T.height, T.x0, T.y0, T.res)
        _, fs, _ = o.rollout(s0, u)
        out[m] = fs[:, 0]
    assert np.abs(out[0][:2] - out[1][:2]).max() < 2e-3


def test_invalid_method_is_rejected():
    with pytest.raises(ValueError):
        oracle.Oracle(_veh(), _cost(), _integ(method=2))


def test_cost_quadrature_is_exact_for_a_linearly_varying_rate():
    """Level ground, straight line at constant speed over a costmap linear in
    x: the running cost is linear in time, which RK4's weights integrate
    exactly (the left Riemann sum of Euler is off by half a step's slope)."""
    v = _veh()
    c0, c1 = 2.0, 0.5
    terr = _grid(lambda X, Y: 0.0 * X)
    h_grid, x0g, y0g, res = terr
    X = x0g + res * np.arange(h_grid.shape[1])
    cm = np.repeat((c0 + c1 * X)[None, :].astype(np.float32), h_grid.shape[0], axis=0)
    N, dt, vx, xs = 20, 0.02, 5.0, -3.0
    T = N * dt
    s0 = state(x=xs, z=v["hR"], v=(vx, 0, 0)).astype(np.float32)
    goal_x = 1e4
    exact_c = 4 * c0 * T + c1 * (4 * (float(s0[0]) * T + vx * T * T / 2) + 2 * (v["Lf"] - v["Lr"]) * T)
    res_J = {}
    for m in (0, 1):
        o = oracle.Oracle(v, _cost(goal_x=goal_x, goal_y=0.0), _integ(method=m))
        o.set_terrain(h_grid, x0g, y0g, res, cm)
        J, fs, _ = o.rollout(s0, np.zeros((N, 2, 1), np.float32))
        res_J[m] = J[0] - 5.0 * T - 15.0 * (goal_x - fs[0, 0])
    assert res_J[1] == pytest.approx(exact_c, rel=1e-9)
    assert abs(res_J[0] - exact_c) > 1e-3 * abs(exact_c)

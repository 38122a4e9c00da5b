"""Helpers that compare the GPU library with the FP64 oracle.

Tolerances (FP32 GPU arithmetic against FP64 on identical float32 inputs):
  * final state component s: |gpu - oracle| <= 1e-4 * max(|oracle|, scale_s)
    with scales 1 m (positions), 0.1 rad (angles, steering), 1 m/s
    (velocities), 1 rad/s (angular rates);
  * cost: |gpu - oracle| <= 1e-4 * max(|oracle|, 10) cost units;
  * argmin: same index, unless the oracle's costs of the two picks differ by
    less than the cost tolerance (a tie at FP32 resolution);
  * plan entries: 1e-4 relative to max(|oracle|, 0.1).
The state bound is the one the planner's accuracy needs (1e-4 of a metre on
a trajectory of tens of metres). One control interval computed in FP32
from the same float32 state stays within it (worst about half of it on the
single-plan workload), so the step map is compared element by element; over a whole
horizon on berm terrain the model's discontinuities (damper switch at
touchdown, slip-angle flip at v_x = 0) and the steep ESM soft cost amplify
storage rounding beyond 1e-4 even between two FP64 runs whose inputs differ
by one float32 ulp, so whole-horizon comparisons of large workloads screen
each mismatch against the oracle's own sensitivity probes.
"""
from __future__ import annotations

import math

import numpy as np

STATE_SCALE = np.array([1, 1, 1, 0.1, 0.1, 0.1, 1, 1, 1, 1, 1, 1, 0.1])
# extended single-track state: x, y, psi, v_y, omega_z, delta, v_x
EST_STATE_SCALE = np.array([1, 1, 0.1, 1, 1, 0.1, 1])
STATE_RTOL = 1e-4
COST_RTOL = 1e-4
COST_FLOOR = 10.0


def state_err(gpu_fs, ora_fs):
    """Normalised error per (component, candidate); <= 1 passes. The state
    is the SRB's (13 rows) or the extended single-track model's (7 rows)."""
    g = np.asarray(gpu_fs, np.float64)
    o = np.asarray(ora_fs, np.float64)
    sc = STATE_SCALE if o.shape[0] == 13 else EST_STATE_SCALE
    scale = np.maximum(np.abs(o), sc[:, None])
    return np.abs(g - o) / (STATE_RTOL * scale)


def cost_err(gpu_J, ora_J):
    g = np.asarray(gpu_J, np.float64)
    o = np.asarray(ora_J, np.float64)
    both_inf = np.isinf(g) & np.isinf(o)
    e = np.abs(g - o) / (COST_RTOL * np.maximum(np.abs(o), COST_FLOOR))
    e[both_inf] = 0.0
    return e


def assert_rollout_parity(gpu_J, gpu_fs, ora_J, ora_fs, label="", ora_exit=None):
    ce = cost_err(gpu_J, ora_J)
    finite = np.isfinite(ora_J)
    assert np.array_equal(np.isinf(gpu_J), np.isinf(ora_J)), f"{label}: inf pattern differs"
    if gpu_fs is not None:
        se = state_err(gpu_fs, ora_fs)[:, finite]
        worst = np.unravel_index(np.argmax(se), se.shape) if se.size else None
        assert se.size == 0 or se.max() <= 1.0, (
            f"{label}: state error {se.max():.3g}x tolerance at component {worst[0]}, "
            f"candidate {np.flatnonzero(finite)[worst[1]]}")
    worst_c = int(np.argmax(ce))
    assert ce.max() <= 1.0, (f"{label}: cost error {ce.max():.3g}x tolerance at k={worst_c} "
                             f"(gpu {gpu_J[worst_c]!r}, oracle {ora_J[worst_c]!r})")
    return float(ce.max()), (float(state_err(gpu_fs, ora_fs)[:, finite].max())
                             if gpu_fs is not None and finite.any() else 0.0)


def assert_argmin_parity(k_gpu, ora_J):
    o = np.asarray(ora_J, np.float64)
    fin = np.isfinite(o)
    if not fin.any():
        assert k_gpu == -1
        return
    k_ora = int(np.flatnonzero(o == o[fin].min())[0])
    if k_gpu == k_ora:
        return
    tol = COST_RTOL * max(abs(o[k_ora]), COST_FLOOR)
    assert 0 <= k_gpu < len(o) and abs(o[k_gpu] - o[k_ora]) <= tol, (
        f"argmin differs: gpu {k_gpu} (oracle J {o[k_gpu] if 0 <= k_gpu < len(o) else None}) "
        f"vs oracle {k_ora} (J {o[k_ora]})")


# --------------------------------------------------------------------------
# Conditioning screen and step-map parity.
#
# Over a long horizon a float32 trajectory can leave its float64 twin for
# reasons that are not implementation errors: the damper force jumps to zero
# at liftoff, and the ESM soft cost (sigma = 1e6 /s) is extremely steep, so a
# rounding-level difference can flip a branch or move a cost by whole units.
# Two checks separate this from defects:
#   * step-map parity: the GPU advances every candidate CHUNK intervals at a
#     time; the oracle restarts each chunk from the GPU's own float32 state and
#     must agree with the chunk's end state and cost within the tolerances
#     above (for every candidate: a wrong term shows within one chunk);
#   * whole-horizon parity of every cost and final state, where any mismatch
#     must be explained by the oracle's own conditioning indicators (below).
#
# The step map is compared one control interval at a time, so both sides
# start from identical float32 state and differ only by one interval of
# rounding (~1e-6 relative): F_s - k chi then differs by a few newtons at most
# (~1e-5 of F_s ~ 2 kN) and a wheel speed by far less than 1 mm/s.
TD_EPS = 1e-4
SLIP_EPS = 1e-3
# Past 72 degrees of roll or pitch the paper scores a rollover; the model's
# contact geometry no longer describes the vehicle (wheels above the chassis)
# and such a candidate's cost is already orders above any viable plan.
ROLLOVER = math.radians(72.0)
MAX_EXEMPT = 0.02            # at most 2 % of candidate-intervals may be exempt
# Whole-horizon comparison. A float32 trajectory may end far from its float64
# twin only for a reason the oracle can show on its own side. A candidate is
# "explained" (ill conditioned) if any of these holds for its float64 run:
#   * rounding the state to float32 after every step (the probe) moves its
#     cost or final state by more than PROBE_FRACTION of the tolerance;
#   * it passes within HORIZON_TD_EPS of the damper's touchdown switch or
#     HORIZON_SLIP_EPS of the slip-angle flip (over a whole horizon the two
#     trajectories drift apart by up to ~1e-4 m in a wheel's extension, ~6 N of
#     ~2 kN, so a 1 % margin is needed for the branch to be certain);
#   * it rolls over.
# Every unexplained candidate must match within the base tolerances, and at
# least min_match of all finite candidates must match.
PROBE_FRACTION = 0.01
HORIZON_TD_EPS = 1e-2
HORIZON_SLIP_EPS = 1e-2


def conditioning(o, state0, controls):
    """Float64 rollout (J64 [K], F64 [13][K]), the float32-storage probe
    (J32, F32) and the float64 run's discontinuity margins and tilt."""
    N, _, K = controls.shape
    s_in = np.repeat(np.asarray(state0, np.float32)[:, None], K, axis=1)
    F64, J64, td, sl, tilt = o.rollout_span(s_in, np.zeros(K, np.float32), controls, 0, N,
                                            True, margins=True)
    o.set_round32(True)
    try:
        J32, F32, _ = o.rollout(state0, controls)
    finally:
        o.set_round32(False)
    return J64, F64, J32, F32, td, sl, tilt


def assert_screened_parity(gpu_J, gpu_fs, o, state0, controls, label="", min_match=0.9):
    """Whole-horizon cost and final-state parity (rules above) plus the
    argmin. Returns (cost match fraction, state match fraction, explained
    fraction)."""
    J64, F64, J32, F32, td, sl, tilt = conditioning(o, state0, controls)
    g = np.asarray(gpu_J, np.float64)
    gf = np.asarray(gpu_fs, np.float64)
    fin = np.isfinite(J64)
    with np.errstate(invalid="ignore"):
        probe_c = cost_err(J32, J64)
        probe_s = np.where(np.isfinite(F32).all(axis=0), state_err(F32, F64).max(axis=0), np.inf)
        c_err = cost_err(g, J64)
        s_err = np.where(np.isfinite(gf).all(axis=0), state_err(gf, F64).max(axis=0), np.inf)
    rolled = tilt > ROLLOVER
    explained = ((probe_c > PROBE_FRACTION) | (probe_s > PROBE_FRACTION) |
                 (td < HORIZON_TD_EPS) | (sl < HORIZON_SLIP_EPS) | rolled |
                 (np.isfinite(J32) != fin))
    c_ok = c_err <= 1.0
    s_ok = s_err <= 1.0
    bad_c = ~c_ok & ~explained
    bad_s = ~s_ok & ~explained & fin
    assert not bad_c.any(), (f"{label}: unexplained cost mismatch at candidates "
                             f"{np.flatnonzero(bad_c)[:5]} ({c_err[bad_c].max():.3g}x tol)")
    assert not bad_s.any(), (f"{label}: unexplained final-state mismatch at candidates "
                             f"{np.flatnonzero(bad_s)[:5]} ({s_err[bad_s].max():.3g}x tol)")
    live = fin & ~rolled
    match_c = float(c_ok[live].mean()) if live.any() else 1.0
    match_s = float(s_ok[live].mean()) if live.any() else 1.0
    assert match_c >= min_match, f"{label}: only {match_c:.1%} of costs match"
    # the pick: identical, a near-tie, or the oracle's own pick is ill conditioned
    if fin.any():
        k_ora = int(np.argmin(np.where(fin, J64, np.inf)))
        k_gpu = int(np.argmin(np.where(np.isfinite(g), g, np.inf)))
        if k_gpu != k_ora and not explained[k_ora]:
            assert_argmin_parity(k_gpu, J64)
    return match_c, match_s, float(explained[live].mean()) if live.any() else 0.0


def assert_step_map_parity(planner, o, controls_np, controls_dev, state0, chunk, idx=None,
                           label=""):
    """Chunked GPU rollout; each chunk re-run by the oracle from the GPU's
    float32 state at the chunk start. Returns the worst normalised errors."""
    import torch
    N, _, K = controls_np.shape
    state = torch.empty(13, K, device="cuda")
    cost = torch.empty(K, device="cuda")
    planner.init_state(state0, state, cost)
    u_sub = controls_np if idx is None else np.ascontiguousarray(controls_np[:, :, idx])
    worst_s = worst_c = 0.0
    exempt = total = near_count = rolled_count = 0
    for n0 in range(0, N, chunk):
        n1 = min(N, n0 + chunk)
        fin = n1 == N
        torch.cuda.synchronize()
        s_in = state.cpu().numpy()
        c_in = cost.cpu().numpy()
        planner.rollout_chunk(state, cost, controls_dev, n0, n1, fin)
        torch.cuda.synchronize()
        s_out = state.cpu().numpy()
        c_out = cost.cpu().numpy()
        if idx is not None:
            s_in, c_in, s_out, c_out = s_in[:, idx], c_in[idx], s_out[:, idx], c_out[idx]
        so, co, td, sl, tilt = o.rollout_span(s_in, c_in, u_sub, n0, n1, fin, margins=True)
        rolled = tilt > ROLLOVER
        near = ~((td > TD_EPS) & (sl > SLIP_EPS)) & ~rolled
        near_count += int(near.sum())
        rolled_count += int(rolled.sum())
        near |= rolled
        exempt += int(near.sum())
        total += near.size
        live = np.isfinite(so).all(axis=0) & np.isfinite(co)
        assert np.array_equal(live[~near], (np.isfinite(s_out).all(axis=0) &
                                            np.isfinite(c_out))[~near]), (
            f"{label}: finite pattern differs in chunk [{n0},{n1})")
        live &= ~near
        se = state_err(s_out, so)[:, live]
        ce = cost_err(c_out, co)[live]
        if se.size:
            q, kk = np.unravel_index(np.argmax(se), se.shape)
            assert se.max() <= 1.0, (f"{label}: chunk [{n0},{n1}) state error {se.max():.3g}x "
                                     f"tolerance, component {q}, candidate "
                                     f"{np.flatnonzero(live)[kk]}")
            worst_s = max(worst_s, float(se.max()))
        if ce.size:
            assert ce.max() <= 1.0, (f"{label}: chunk [{n0},{n1}) cost error {ce.max():.3g}x "
                                     f"tolerance at candidate {np.flatnonzero(live)[np.argmax(ce)]}")
            worst_c = max(worst_c, float(ce.max()))
    assert near_count <= MAX_EXEMPT * total, (f"{label}: {near_count} of {total} "
                                              "candidate-intervals pass near a discontinuity")
    print(f"{label}: of {total} candidate-intervals, {near_count} exempt near a discontinuity, "
          f"{rolled_count} past rollover")
    return worst_s, worst_c, state, cost


# --------------------------------------------------------------------------
# Extended single-track rollouts. The EST model has no switching terms, but at
# large sideslip (saturated tires, the paper's uniform steering-rate samples
# held for 0.25 s) its lateral dynamics are close to neutral, so float32
# storage alone moves many long-horizon trajectories by a visible fraction of
# the tolerance. The oracle's float32-storage probe measures that drift per
# candidate; the GPU's deviation must stay within PROBE_FACTOR times the
# probe's own deviation (or the base tolerance, whichever is larger), and at
# least min_match of the candidates must meet the base tolerance outright. A
# wrong term moves a trajectory far beyond what storage rounding does.
PROBE_FACTOR = 10.0


def assert_est_probe_parity(gpu_J, gpu_fs, o, state0, controls, label="", min_match=0.9):
    J64, F64, _ = o.est_rollout(state0, controls)
    o.set_round32(True)
    try:
        J32, F32, _ = o.est_rollout(state0, controls)
    finally:
        o.set_round32(False)
    g = np.asarray(gpu_J, np.float64)
    gf = np.asarray(gpu_fs, np.float64)
    fin = np.isfinite(J64)
    assert np.array_equal(np.isfinite(g), fin) or np.array_equal(np.isfinite(J32), np.isfinite(g)), (
        f"{label}: inf pattern differs from the oracle and its probe")
    with np.errstate(invalid="ignore"):
        pc = cost_err(J32, J64)
        ps = state_err(F32, F64).max(axis=0)
        ce = cost_err(g, J64)
        se = state_err(gf, F64).max(axis=0)
    lim_c = np.maximum(1.0, PROBE_FACTOR * pc)
    lim_s = np.maximum(1.0, PROBE_FACTOR * ps)
    bad = fin & ((ce > lim_c) | (se > lim_s))
    assert not bad.any(), (f"{label}: candidates {np.flatnonzero(bad)[:5]} deviate beyond "
                           f"{PROBE_FACTOR:g}x the float32-storage probe "
                           f"(cost {ce[bad].max():.3g}, state {se[bad].max():.3g} x tol)")
    match = float(((ce <= 1.0) & (se <= 1.0))[fin].mean()) if fin.any() else 1.0
    assert match >= min_match, f"{label}: only {match:.1%} of candidates within tolerance"
    return match, float(np.max(se[fin] / lim_s[fin])) if fin.any() else 0.0

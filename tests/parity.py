"""Helpers that compare the GPU library with the FP64 oracle.

Tolerances (FP32 GPU arithmetic against FP64 on identical float32 inputs):
  * final state component s: |gpu - oracle| <= 1e-4 * max(|oracle|, scale_s)
    with scales 1 m (positions), 0.1 rad (angles, steering), 1 m/s
    (velocities), 1 rad/s (angular rates);
  * cost: |gpu - oracle| <= 1e-4 * max(|oracle|, 10) cost units;
  * argmin: same index, unless the oracle's costs of the two picks differ by
    at most 1e-6 relative (a tie);
  * plan entries: 1e-4 relative to max(|oracle|, 0.1).
The state bound is the one the planner's accuracy needs (1e-4 of a metre on
a trajectory of tens of metres). One control interval computed in FP32
from the same float32 state stays within it (worst about half of it on the
single-plan workload), so the step map is compared element by element; over a whole
horizon on berm terrain the model's discontinuities (damper switch at
touchdown, slip-angle flip at v_x = 0) and the steep ESM soft cost amplify
storage rounding beyond 1e-4 even between two FP64 runs whose inputs differ
by one float32 ulp, so whole-horizon comparisons of large workloads screen
each candidate against the oracle's own sensitivity probe.
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
TIE_RTOL = 1e-6


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


def assert_argmin_parity(k_gpu, ora_J, label=""):
    """The GPU's pick against the oracle's own costs: the oracle's pick (the
    lowest index of its minimal finite cost), or a candidate whose oracle
    cost ties with the minimum within TIE_RTOL relative; -1 exactly when the
    oracle has no finite candidate."""
    o = np.asarray(ora_J, np.float64)
    fin = np.isfinite(o)
    if not fin.any():
        assert k_gpu == -1, f"{label}: oracle has no finite candidate, gpu picked {k_gpu}"
        return
    k_ora = int(np.flatnonzero(o == o[fin].min())[0])
    if k_gpu == k_ora:
        return
    tol = TIE_RTOL * abs(o[k_ora])
    assert 0 <= k_gpu < len(o) and abs(o[k_gpu] - o[k_ora]) <= tol, (
        f"{label}: argmin differs: gpu {k_gpu} (oracle J {o[k_gpu] if 0 <= k_gpu < len(o) else None}) "
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
# rounding (~1e-6 relative): over one Euler step F_s - k chi then differs by
# a few newtons at most (~1e-5 of F_s ~ 2 kN) and a wheel speed by far less
# than 1 mm/s. Over an interval of many Euler steps the touchdown instant is
# more sensitive: at the paper's shape (50 steps per interval) the oracle
# itself, restarted from its float32 state perturbed by 2^-22 relative
# (random signs, 8 draws per candidate-interval), lands a wheel one step
# earlier or later, and so misses the base tolerance 30-fold, in 13.5 % of
# candidate-intervals with a touchdown margin below 1e-4, 0.3 % of those in
# [1e-4, 3e-4) and none of 20 400 sampled above 3e-4; TD_EPS_MULTI covers that
# band with a factor of three (1.4 % of the paper shape's candidate-intervals
# fall below it, within MAX_EXEMPT).
TD_EPS = 1e-4
TD_EPS_MULTI = 1e-3
SLIP_EPS = 1e-3
# Past 72 degrees of roll or pitch the paper scores a rollover; the model's
# contact geometry no longer describes the vehicle (wheels above the chassis)
# and such a candidate's cost is already orders above any viable plan.
ROLLOVER = math.radians(72.0)
MAX_EXEMPT = 0.02            # at most 2 % of candidate-intervals may be exempt
# Step-map conditioning probe. The oracle also runs each interval from the
# GPU's start state perturbed by STEP_PERTURB relative (signs alternating over
# the 13 components), about the size of the GPU's own arithmetic error in a
# step (hardware sine and cosine to about 1e-6, a few tens of FP32 roundings).
# A candidate-interval matches within max(1, STEP_FACTOR x the probe's
# deviation): the base tolerance wherever the interval's map is well
# conditioned, more only where the oracle itself shows the map amplifying
# rounding (tumbling chassis, velocities of hundreds of m/s). Candidate-
# intervals that are beyond the base tolerance but within their relaxed bound
# are counted and capped at MAX_RELAXED.
STEP_PERTURB = 2.0 ** -20
STEP_FACTOR = 30.0
MAX_RELAXED = 0.01
# Whole-horizon comparison. A float32 trajectory may end far from its float64
# twin without any implementation error: the discontinuities above and the
# steep ESM cost amplify rounding differently for every candidate. The
# oracle measures each candidate's own sensitivity with a probe: the same
# float64 rollout with the state and J rounded to float32 after every Euler
# step. The GPU's deviation is then judged against the probe's:
#   R1 finite pattern: the GPU and the oracle disagree on which candidates
#      stay finite for at most twice as many candidates as the oracle
#      disagrees with its own probe (zero where the probe agrees everywhere);
#   R2 population: of the candidates finite on all three runs, at least
#      POP_FRACTION deviate by at most max(1, POP_FACTOR x the probe's
#      deviation) (cost, and worst state component, each in tolerance units);
#   R3 every well-conditioned candidate (its float64 run neither rolls over
#      nor passes within WELL_EPS of the touchdown switch or a wheel's
#      slip-angle flip) deviates by at most max(1, WELL_FACTOR x the probe's),
#      except at most WELL_SPARE of them, which stay within WELL_CAP x the
#      base tolerance (long stiff horizons where the probe, which rounds only
#      the stored state, underrates the GPU's own arithmetic error);
#   R4 at least min_cost / min_state of the finite, non-rolled candidates are
#      within the base tolerances outright;
#   R5 the GPU's argmin (over its own costs) is the oracle's, or ties with it
#      within TIE_RTOL (assert_argmin_parity).
# The factors reflect that the GPU rounds every operation in FP32 and takes
# its sines and cosines from the hardware unit (absolute error about 1e-6, some
# 30 times float32 storage rounding of an O(1) angle), so its per-step
# perturbation is one to two orders of magnitude above the probe's; a wrong
# term moves trajectories by orders more, in every candidate. A candidate can
# cross a branch its float64 twin only approaches when the two trajectories
# differ by more than the branch margin; WELL_EPS bounds that for the
# drifts seen here.
POP_FACTOR = 30.0
POP_FRACTION = 0.99
WELL_FACTOR = 200.0
WELL_EPS = 2e-3
WELL_SPARE = 5e-3
WELL_CAP = 10.0


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


def assert_finite_agreement(gpu_J, gpu_fs, J64, J32, F32, label=""):
    """R1: the GPU and the oracle disagree on which candidates stay finite
    (cost and final state; cost alone when gpu_fs is None) for at most twice
    as many candidates as the oracle's float64 run disagrees with its own
    float32-storage probe, plus three standard deviations of a Poisson count
    of that mean: the candidates that change finiteness are the few whose
    tumbling chassis (past the rollover limit) diverges, and a count of one
    or two is a noisy estimate of how many a perturbation of the GPU's size
    flips (the C5 stress plan: 1 in the probe, 2 or 3 on the GPU depending on
    rounding; a wrong term changes hundreds)."""
    g = np.asarray(gpu_J, np.float64)
    fin = np.isfinite(J64)
    fin_g = np.isfinite(g)
    fin_p = np.isfinite(J32)
    if gpu_fs is not None:
        fin_g &= np.isfinite(np.asarray(gpu_fs, np.float64)).all(axis=0)
        fin_p &= np.isfinite(F32).all(axis=0)
    d_gpu = int(np.sum(fin_g != fin))
    d_probe = int(np.sum(fin_p != fin))
    print(f"{label}: non-finite candidates: oracle {int((~fin).sum())}, gpu {int((~fin_g).sum())}, "
          f"probe {int((~fin_p).sum())}; finite on one side only: gpu {d_gpu}, probe {d_probe}",
          flush=True)
    bound = 2 * d_probe + 3.0 * math.sqrt(2 * d_probe + 1)
    assert d_gpu <= bound, (f"{label}: {d_gpu} candidates finite on one side only "
                            f"(the oracle's probe: {d_probe}; bound {bound:.1f})")
    return {"nonfinite_oracle": int((~fin).sum()), "nonfinite_gpu": int((~fin_g).sum()),
            "finite_disagree": d_gpu, "probe_finite_disagree": d_probe,
            "fin": fin, "fin_g": fin_g, "fin_p": fin_p}


def assert_horizon_parity(gpu_J, gpu_fs, o, state0, controls, label="", min_cost=0.9,
                          min_state=0.5, k_gpu=None, argmin=True, cond=None):
    """Whole-horizon parity of every candidate's cost and final state (cost
    alone when gpu_fs is None) by the rules R1-R5 above. k_gpu: the GPU's own pick (default: the lowest index
    of the GPU's minimal finite cost). cond: a precomputed conditioning()
    tuple. Returns a dict of the counts and fractions (also printed)."""
    J64, F64, J32, F32, td, sl, tilt = cond if cond is not None else conditioning(
        o, state0, controls)
    g = np.asarray(gpu_J, np.float64)
    K = len(J64)
    # R1
    fa = assert_finite_agreement(g, gpu_fs, J64, J32, F32, label)
    fin, fin_g, fin_p = fa["fin"], fa["fin_g"], fa["fin_p"]
    d_gpu, d_probe = fa["finite_disagree"], fa["probe_finite_disagree"]
    with np.errstate(invalid="ignore", over="ignore"):
        pc = cost_err(J32, J64)
        ce = cost_err(g, J64)
        if gpu_fs is None:  # costs only: the state terms drop out of every rule
            ps = se = np.zeros(K)
        else:
            ps = state_err(F32, F64).max(axis=0)
            se = state_err(np.asarray(gpu_fs, np.float64), F64).max(axis=0)
    common = fin & fin_g & fin_p
    # R2
    pop_ok = (ce <= np.maximum(1.0, POP_FACTOR * pc)) & (se <= np.maximum(1.0, POP_FACTOR * ps))
    pop = float(pop_ok[common].mean()) if common.any() else 1.0
    assert pop >= POP_FRACTION, (f"{label}: only {pop:.2%} of {int(common.sum())} candidates "
                                 f"within {POP_FACTOR:g}x the float32-storage probe")
    # R3
    rolled = tilt > ROLLOVER
    near = (td < WELL_EPS) | (sl < WELL_EPS)
    well = common & ~rolled & ~near
    beyond = well & ~((ce <= np.maximum(1.0, WELL_FACTOR * pc)) &
                      (se <= np.maximum(1.0, WELL_FACTOR * ps)))
    bad = beyond & ~((ce <= WELL_CAP) & (se <= WELL_CAP))
    # R4 counts
    live = common & ~rolled
    mc = float((ce[live] <= 1.0).mean()) if live.any() else float("nan")
    ms = float((se[live] <= 1.0).mean()) if live.any() else float("nan")
    out = {"candidates": K, "finite_common": int(common.sum()), "finite_disagree": d_gpu,
           "probe_finite_disagree": d_probe, "within_pop_factor": pop,
           "well_conditioned": int(well.sum()), "beyond_probe": int(beyond.sum()),
           "rolled": int((fin & rolled).sum()),
           "near_discontinuity": int((common & near & ~rolled).sum()),
           "cost_match": mc, "state_match": ms}
    print(f"{label}: {K} candidates, {out['finite_common']} finite on all runs "
          f"({d_gpu} finite on one side only, probe {d_probe}); within {POP_FACTOR:g}x probe "
          f"{pop:.2%}; {out['well_conditioned']} well conditioned ({out['beyond_probe']} beyond "
          f"{WELL_FACTOR:g}x probe, within {WELL_CAP:g}x tol), {out['near_discontinuity']} near a "
          f"discontinuity, {out['rolled']} rolled over; within 1e-4: costs {mc:.2%}, final "
          f"states {ms:.2%}", flush=True)
    assert not bad.any(), (f"{label}: well-conditioned candidates {np.flatnonzero(bad)[:5]} "
                           f"deviate beyond {WELL_FACTOR:g}x the probe and {WELL_CAP:g}x the "
                           f"tolerance (cost {ce[bad].max():.3g}, state {se[bad].max():.3g} x tol)")
    assert beyond.sum() <= WELL_SPARE * max(int(well.sum()), 1), (
        f"{label}: {int(beyond.sum())} of {int(well.sum())} well-conditioned candidates deviate "
        f"beyond {WELL_FACTOR:g}x the probe (worst cost {ce[beyond].max():.3g}, state "
        f"{se[beyond].max():.3g} x tol)")
    # R4 (nothing to count when every candidate rolled over)
    if live.any():
        assert mc >= min_cost, f"{label}: only {mc:.2%} of {int(live.sum())} costs within 1e-4"
        assert ms >= min_state, (f"{label}: only {ms:.2%} of {int(live.sum())} final states "
                                 "within 1e-4")
    # R5
    if argmin:
        if k_gpu is None:
            k_gpu = int(np.argmin(np.where(fin_g, g, np.inf))) if fin_g.any() else -1
        assert_argmin_parity(k_gpu, J64, label)
    return out


def assert_step_map_parity(planner, o, controls_np, controls_dev, state0, chunk, idx=None,
                           label=""):
    """Chunked GPU rollout; each chunk re-run by the oracle from the GPU's
    float32 state at the chunk start (and from that state perturbed by
    STEP_PERTURB, the conditioning probe). Returns the worst errors as
    fractions of their bounds."""
    import torch
    N, _, K = controls_np.shape
    state = torch.empty(13, K, device="cuda")
    cost = torch.empty(K, device="cuda")
    planner.init_state(state0, state, cost)
    u_sub = controls_np if idx is None else np.ascontiguousarray(controls_np[:, :, idx])
    worst_s = worst_c = 0.0
    exempt = total = near_count = rolled_count = relaxed_count = compared = 0
    nonfinite_count = 0
    td_eps = TD_EPS if chunk * o.substeps == 1 else TD_EPS_MULTI
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
        # candidates already non-finite at the interval's start stay so on
        # both sides (checked by the finite pattern below), nothing to measure
        start_fin = np.isfinite(s_in).all(axis=0) & np.isfinite(c_in)
        nonfinite_count += int((~start_fin).sum())
        sgn = np.where(np.arange(13) % 2 == 0, 1.0, -1.0)[:, None]
        s_pert = (s_in.astype(np.float64) * (1.0 + sgn * STEP_PERTURB)).astype(np.float32)
        sp, cp = o.rollout_span(s_pert, c_in, u_sub, n0, n1, fin)
        with np.errstate(invalid="ignore"):
            probe = np.maximum(state_err(sp, so).max(axis=0), cost_err(cp, co))
        bound = np.maximum(1.0, STEP_FACTOR * np.nan_to_num(probe, nan=np.inf))
        rolled = (tilt > ROLLOVER) & start_fin
        near = ~((td > td_eps) & (sl > SLIP_EPS)) & ~rolled & start_fin
        near_count += int(near.sum())
        rolled_count += int(rolled.sum())
        near |= rolled | ~start_fin
        exempt += int(near.sum())
        total += near.size
        live = np.isfinite(so).all(axis=0) & np.isfinite(co)
        assert np.array_equal(live[~near], (np.isfinite(s_out).all(axis=0) &
                                            np.isfinite(c_out))[~near]), (
            f"{label}: finite pattern differs in chunk [{n0},{n1})")
        live &= ~near
        compared += int(live.sum())
        e_abs = np.maximum(state_err(s_out, so).max(axis=0), cost_err(c_out, co))
        relaxed_count += int((live & (e_abs > 1.0)).sum())
        se = state_err(s_out, so)[:, live] / bound[live]
        ce = cost_err(c_out, co)[live] / bound[live]
        if se.size:
            q, kk = np.unravel_index(np.argmax(se), se.shape)
            assert se.max() <= 1.0, (f"{label}: chunk [{n0},{n1}) state error {se.max():.3g}x "
                                     f"its bound, component {q}, candidate "
                                     f"{np.flatnonzero(live)[kk]}")
            worst_s = max(worst_s, float(se.max()))
        if ce.size:
            assert ce.max() <= 1.0, (f"{label}: chunk [{n0},{n1}) cost error {ce.max():.3g}x "
                                     f"its bound at candidate "
                                     f"{np.flatnonzero(live)[np.argmax(ce)]}")
            worst_c = max(worst_c, float(ce.max()))
    assert near_count <= MAX_EXEMPT * total, (f"{label}: {near_count} of {total} "
                                              "candidate-intervals pass near a discontinuity")
    assert relaxed_count <= MAX_RELAXED * total, (
        f"{label}: {relaxed_count} of {total} candidate-intervals beyond the base tolerance")
    print(f"{label}: of {total} candidate-intervals, {compared} compared "
          f"({relaxed_count} of them beyond the base tolerance, within the bound of their "
          f"ill-conditioned map), {near_count} exempt near a discontinuity, {rolled_count} past "
          f"rollover, {nonfinite_count} already non-finite; worst state {worst_s:.3g}, cost "
          f"{worst_c:.3g} of the bound", flush=True)
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

"""GPU tests of the continuous-batching server (include/plan_serve.h): every
request's result is bit-identical to the plain path (plan_rollout +
plan_select) and to the same request served alone, whether it runs alone or
mixed with others, under any arrival pattern, tick length, slot limit or
memory budget; and every served request of the trace matches the FP64
oracle's rollout of that request."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402  (test infrastructure)
from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402
from tests.parity import assert_horizon_parity  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    yield
    torch.cuda.synchronize()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


class Resident:
    """One request's inputs uploaded to the GPU, plus its plain-path answer."""

    def __init__(self, req: inputs.Request):
        w = req.workload
        self.w = w
        self.arrival = req.arrival
        self.h = dev(w.terrain.height)
        self.u = dev(w.controls)
        self.plan = torch.zeros(w.N, 2, device="cuda")

    def plain(self):
        w, T = self.w, self.w.terrain
        pl = P.Planner(w.vehicle, w.cost, w.integ, w.K, w.N, T.W, T.H)
        pl.set_terrain(self.h, T.x0, T.y0, T.res)
        J = torch.empty(w.K, device="cuda")
        plan = torch.empty(w.N, 2, device="cuda")
        pl.rollout(w.state0, self.u, J)
        k, jb = pl.select(self.u, J, plan)
        pl.close()
        return k, jb, plan.cpu().numpy()

    def submit(self, srv):
        w, T = self.w, self.w.terrain
        self.plan.zero_()
        return srv.submit(self.h, T.x0, T.y0, T.res, w.state0, self.u, w.cost, w.integ,
                          self.plan)


@pytest.fixture(scope="module")
def trace():
    reqs = [Resident(r) for r in inputs.c3_trace(n_req=12)]
    for r in reqs:
        r.ref = r.plain()
    return reqs


def _server(reqs, slots=16, budget=1 << 34, chunk=16):
    K = max(r.w.K for r in reqs)
    N = max(r.w.N for r in reqs)
    return P.Server(inputs.WORKLOAD_VEHICLE, slots, K, N, 256, 256, budget, chunk)


def _check(srv, reqs, ids):
    for r, rid in zip(reqs, ids):
        res = srv.result(rid)
        assert res["status"] == 1, res
        k, jb, plan = r.ref
        assert res["best_k"] == k
        assert np.float32(res["best_cost"]) == np.float32(jb)
        np.testing.assert_array_equal(r.plan.cpu().numpy(), plan)
        assert res["t_submit"] <= res["t_admit"] <= res["t_done"]


def test_burst_results_identical_to_plain_path(trace):
    srv = _server(trace)
    ids = [r.submit(srv) for r in trace]
    srv.drain()
    _check(srv, trace, ids)
    srv.close()


def test_staggered_arrivals_and_tick_lengths(trace):
    for chunk in (1, 7, 200):
        srv = _server(trace, chunk=chunk)
        ids = []
        for i, r in enumerate(trace):
            ids.append(r.submit(srv))
            for _ in range(i % 3):
                srv.step()
        srv.drain()
        _check(srv, trace, ids)
        srv.close()


def test_slot_limit_bounds_residency(trace):
    srv = _server(trace, slots=2)
    ids = [r.submit(srv) for r in trace]
    peak = 0
    while True:
        a, q = srv.step()
        peak = max(peak, a)
        if a == 0 and q == 0:
            break
    srv.drain()
    assert peak == 2
    _check(srv, trace, ids)
    srv.close()


def test_memory_budget_admission(trace):
    fp = [64 * 256 * 256 + 56 * r.w.K + 8 * r.w.K * r.w.N + 8 * r.w.N for r in trace]
    budget = max(fp) + min(fp) - 1  # the largest never shares with another
    srv = _server(trace, budget=budget)
    ids = [r.submit(srv) for r in trace]
    blocked = False
    while True:
        a, q = srv.step()
        a2, q2, used = srv.stats()
        assert used <= budget
        blocked = blocked or (q2 > 0 and a2 < 16)  # waiting on memory, not on slots
        if a == 0 and q == 0:
            break
    assert blocked
    srv.drain()
    _check(srv, trace, ids)
    with pytest.raises(P.PlanError):
        small = _server(trace, budget=min(fp) - 1)
        trace[0].submit(small)
    srv.close()


def test_bad_terrain_request_fails_alone(trace):
    srv = _server(trace)
    bad = trace[1]
    h = bad.w.terrain.height.copy()
    h[10, 10] = np.nan
    bad_h = dev(h)
    ids = []
    for i, r in enumerate(trace[:4]):
        if i == 1:
            T = r.w.terrain
            ids.append(srv.submit(bad_h, T.x0, T.y0, T.res, r.w.state0, r.u, r.w.cost,
                                  r.w.integ, r.plan))
        else:
            ids.append(r.submit(srv))
    srv.drain()
    assert srv.result(ids[1])["status"] == P.PLAN_EINVAL
    good = [0, 2, 3]
    _check(srv, [trace[i] for i in good], [ids[i] for i in good])
    srv.close()


def test_bad_terrain_flag_cleared_for_next_request(trace):
    # one slot: the request after the bad one reuses its slot, and must not
    # inherit the non-finite-terrain flag
    srv = _server(trace, slots=1)
    bad = trace[1]
    h = bad.w.terrain.height.copy()
    h[3, 7] = np.inf
    T = bad.w.terrain
    id_bad = srv.submit(dev(h), T.x0, T.y0, T.res, bad.w.state0, bad.u, bad.w.cost,
                        bad.w.integ, bad.plan)
    ids = [r.submit(srv) for r in trace[2:4]]
    srv.drain()
    assert srv.result(id_bad)["status"] == P.PLAN_EINVAL
    assert srv.result(id_bad)["slot"] == srv.result(ids[0])["slot"] == 0
    _check(srv, trace[2:4], ids)
    srv.close()


def test_status_of_each_request_through_one_slot_and_every_ring_entry(trace):
    """One slot and a tick long enough for any horizon: request i finishes in
    step i + 1 and publishes into ring entry i mod 4, so every ring entry is
    reused with the other status four steps later (bad terrain where
    i % 3 == 0). Each result must carry its own request's status, never the
    previous occupant's."""
    srv = _server(trace, slots=1, chunk=200)
    ids, bad = [], []
    for i, r in enumerate(trace):
        T = r.w.terrain
        if i % 3 == 0:
            h = T.height.copy()
            h[5 + i, 9] = np.nan
            ids.append(srv.submit(dev(h), T.x0, T.y0, T.res, r.w.state0, r.u, r.w.cost,
                                  r.w.integ, r.plan))
            bad.append(True)
        else:
            ids.append(r.submit(srv))
            bad.append(False)
    srv.drain()
    for rid, b in zip(ids, bad):
        assert srv.result(rid)["status"] == (P.PLAN_EINVAL if b else 1), (rid, b)
    good = [i for i, b in enumerate(bad) if not b]
    _check(srv, [trace[i] for i in good], [ids[i] for i in good])
    srv.close()


def test_completion_queue(trace):
    srv = _server(trace, slots=4)
    ids = [r.submit(srv) for r in trace[:6]]
    assert srv.completions() == []
    srv.drain()
    first = srv.completions(capacity=4)
    rest = srv.completions()
    assert len(first) == 4 and sorted(first + rest) == sorted(ids)
    assert srv.completions() == []
    # in the order observed: non-decreasing completion times
    t = [srv.result(i)["t_done"] for i in first + rest]
    assert t == sorted(t)
    _check(srv, trace[:6], ids)
    srv.close()


def test_submit_validation(trace):
    srv = _server(trace)
    r = trace[0]
    T = r.w.terrain
    with pytest.raises(P.PlanError):
        big_u = dev(np.zeros((r.w.N, 2, 20000), np.float32))
        srv.submit(r.h, T.x0, T.y0, T.res, r.w.state0, big_u, r.w.cost, r.w.integ, r.plan)
    s_bad = r.w.state0.copy()
    s_bad[0] = np.nan
    with pytest.raises(P.PlanError):
        srv.submit(r.h, T.x0, T.y0, T.res, s_bad, r.u, r.w.cost, r.w.integ, r.plan)
    with pytest.raises(P.PlanError):
        srv.submit(r.h, T.x0, T.y0, 0.0, r.w.state0, r.u, r.w.cost, r.w.integ, r.plan)
    srv.close()


def _serve_trace(reqs, gap_per_step=0.005, **kw):
    """Submit the requests in arrival order, one scheduling step per
    gap_per_step seconds of arrival gap (so later requests join while earlier
    ones are on the GPU), with a [K] cost output each; drain."""
    srv = _server(reqs, **kw)
    costs = [torch.full((r.w.K,), float("nan"), device="cuda") for r in reqs]
    ids = []
    for i, r in enumerate(reqs):
        T = r.w.terrain
        r.plan.zero_()
        ids.append(srv.submit(r.h, T.x0, T.y0, T.res, r.w.state0, r.u, r.w.cost, r.w.integ,
                              r.plan, costs_out=costs[i]))
        if i + 1 < len(reqs):
            for _ in range(int((reqs[i + 1].arrival - r.arrival) / gap_per_step)):
                srv.step()
    srv.drain()
    res = [srv.result(i) for i in ids]
    out = [(x, c.cpu().numpy(), r.plan.cpu().numpy()) for x, c, r in zip(res, costs, reqs)]
    srv.close()
    return out


@pytest.fixture(scope="module")
def full_trace():
    return [Resident(r) for r in inputs.c3_trace()]


def test_served_results_match_the_oracle(full_trace):
    """All 64 requests of the serving trace (Poisson arrivals at 200 req/s, K
    in {512..8192}, N in 40..160, each with its own terrain crop, start and
    goal), served in the mix: every candidate's cost against the oracle's
    rollout of that request (whole-horizon rule), the request's pick against
    the oracle's costs, and its plan equal to the clamped controls of the
    pick."""
    served = _serve_trace(full_trace, slots=16, chunk=16)
    compared = 0
    for r, (res, J, plan) in zip(full_trace, served):
        w, T = r.w, r.w.terrain
        assert res["status"] == 1, res
        # the pick is the lowest index of the request's minimal finite cost
        fin = np.isfinite(J)
        k = res["best_k"]
        assert k == int(np.flatnonzero(J == J[fin].min())[0]) and res["best_cost"] == J[k]
        o = oracle.Oracle(w.vehicle, w.cost, w.integ)
        o.set_terrain(T.height, T.x0, T.y0, T.res)
        assert_horizon_parity(J, None, o, w.state0, w.controls,
                              f"served request {w.name} (K={w.K}, N={w.N})", min_cost=0.99,
                              k_gpu=k)
        ko, _, po = o.select(w.controls, J, mode=0)
        assert ko == k
        np.testing.assert_array_equal(plan, po.astype(np.float32))
        compared += w.K
    print(f"served trace: {len(full_trace)} requests, {compared} candidates against the oracle")


def test_each_request_alone_equals_the_mix(full_trace):
    """Every request of the trace served on its own gives the same bits as
    in the mix: pick, cost of the pick, every candidate's cost, plan."""
    mix = _serve_trace(full_trace, slots=16, chunk=16)
    for r, (res, J, plan) in zip(full_trace, mix):
        (res1, J1, plan1), = _serve_trace([r], slots=1, chunk=16)
        assert (res1["best_k"], res1["best_cost"]) == (res["best_k"], res["best_cost"])
        np.testing.assert_array_equal(J1, J)
        np.testing.assert_array_equal(plan1, plan)

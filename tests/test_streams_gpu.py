"""GPU tests of independent contexts on their own streams: contexts bound to
different (default-priority) streams run interleaved, unsynchronised calls
and each still returns exactly what it returns alone."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2603_20525_amd import inputs  # noqa: E402
from paper_2603_20525_amd import plan as P  # noqa: E402

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


class Job:
    def __init__(self, w, stream):
        T = w.terrain
        self.w = w
        with torch.cuda.stream(stream):
            self.pl = P.Planner(w.vehicle, w.cost, w.integ, w.K, w.N, T.W, T.H, stream=stream)
            self.pl.set_terrain(dev(T.height), T.x0, T.y0, T.res)
        self.u = dev(w.controls)
        self.J = torch.empty(w.K, device="cuda")
        self.fs = torch.empty(13, w.K, device="cuda")
        self.plan = torch.empty(w.N, 2, device="cuda")
        torch.cuda.synchronize()

    def launch(self):
        # one-launch rollout + argmin, no host wait
        self.pl.rollout_argmin(self.w.state0, self.u, self.J, self.plan, self.fs,
                               want_result=False)

    def results(self):
        return (self.J.cpu().numpy().copy(), self.fs.cpu().numpy().copy(),
                self.plan.cpu().numpy().copy())


def test_contexts_on_separate_streams_match_their_solo_results():
    workloads = [inputs.c1(), inputs.c2(K=1000), inputs.c4(K=300)]
    streams = [torch.cuda.Stream() for _ in workloads]
    jobs = [Job(w, s) for w, s in zip(workloads, streams)]
    solo = []
    for j in jobs:
        j.launch()
        torch.cuda.synchronize()
        solo.append(j.results())
    for _ in range(3):
        for j in jobs:  # interleaved, nothing waits between the launches
            j.launch()
        torch.cuda.synchronize()
        for j, ref in zip(jobs, solo):
            for got, want in zip(j.results(), ref):
                np.testing.assert_array_equal(got, want)
    for j in jobs:
        j.pl.close()


def test_server_and_planner_on_separate_streams():
    w = inputs.c2(K=512, N=60)
    T = w.terrain
    s_plan, s_srv = torch.cuda.Stream(), torch.cuda.Stream()
    job = Job(w, s_plan)
    job.launch()
    torch.cuda.synchronize()
    ref = job.results()
    srv = P.Server(w.vehicle, 4, w.K, w.N, T.W, T.H, 1 << 30, 16, stream=s_srv)
    h = dev(T.height)
    plan = torch.zeros(w.N, 2, device="cuda")
    torch.cuda.synchronize()
    rid = srv.submit(h, T.x0, T.y0, T.res, w.state0, job.u, w.cost, w.integ, plan)
    srv.step()
    job.launch()  # concurrently with the server's step on its own stream
    srv.drain()
    torch.cuda.synchronize()
    res = srv.result(rid)
    assert res["status"] == 1
    J, _, plan_ref = ref
    k = int(np.argmin(J))
    assert res["best_k"] == k and np.float32(res["best_cost"]) == J[k]
    np.testing.assert_array_equal(plan.cpu().numpy(), plan_ref)
    for got, want in zip(job.results(), ref):
        np.testing.assert_array_equal(got, want)
    srv.close()
    job.pl.close()

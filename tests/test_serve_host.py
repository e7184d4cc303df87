"""Host logic of the serving loop (no device): admission by footprint in arrival
order, the memory budget, retirement and the summary, with the library calls replaced
by stand-ins that count steps."""
import numpy as np
import pytest

from paper_2002_09217_amd import serve, workloads as W


class FakeLattice:
    live = 0

    def __init__(self, cfg):
        self.cfg, self.n, self._batch = cfg, 0, None
        FakeLattice.live += 1

    def init_fields(self, rho, u, T):
        return self

    def steps_done(self):
        return self.n

    def moments(self):
        return {"steps": self.n}

    def last_error(self):
        return "ok"

    def tile_info(self):
        return {"variant": 0}

    def close(self):
        if self._batch is not None:
            self._batch.members.remove(self)
            self._batch = None
        FakeLattice.live -= 1


class FakeBatch:
    def __init__(self, stream=None):
        self.members = []
        self.max_members = 0

    def add(self, lat):
        self.members.append(lat)
        lat._batch = self
        FakeBatch.max_seen = max(getattr(FakeBatch, "max_seen", 0), len(self.members))

    def remove(self, lat):
        self.members.remove(lat)
        lat._batch = None

    def step(self, n):
        for m in self.members:
            m.n += n
        return []

    def close(self):
        for m in self.members:
            m._batch = None
        self.members = []


@pytest.fixture
def fake_pond(monkeypatch):
    monkeypatch.setattr(serve.pond, "Lattice", FakeLattice)
    monkeypatch.setattr(serve.pond, "Batch", FakeBatch)
    monkeypatch.setattr(serve.pond, "footprint", lambda cfg: cfg.N * 100)
    FakeLattice.live = 0
    FakeBatch.max_seen = 0


def _jobs(sides, steps):
    jobs = []
    for j, s in enumerate(sides):
        case = W.Case(name=f"j{j}", dim=2, n=(s, s), params=W.base_params(), rho=np.ones(s * s),
                      u=np.zeros((2, s * s)), T=np.ones(s * s), steps=steps[j])
        jobs.append(serve.Job(j, 0.0, case, steps[j]))
    return jobs


def test_every_job_runs_its_own_step_count(fake_pond):
    jobs = _jobs([8, 16, 8, 32, 16], [30, 75, 10, 60, 5])
    srv = serve.Server(chunk=20, keep_fields=True)
    res = srv.run(jobs)
    assert [r.status for r in res] == ["ok"] * 5
    assert [r.steps_done for r in res] == [30, 75, 10, 60, 5]
    assert [r.fields["steps"] for r in res] == [30, 75, 10, 60, 5]
    assert FakeLattice.live == 0 and FakeBatch.max_seen == 5


def test_budget_limits_resident_bytes_and_admits_in_arrival_order(fake_pond):
    sides = [16, 16, 16, 8, 16, 8]
    jobs = _jobs(sides, [40] * 6)
    budget = 2 * 16 * 16 * 100 + 8 * 8 * 100       # two large jobs and one small fit
    srv = serve.Server(chunk=10, budget_bytes=budget)
    res = srv.run(jobs)
    assert all(r.status == "ok" and r.steps_done == 40 for r in res)
    assert srv.peak_bytes <= budget
    assert FakeBatch.max_seen == 3
    admitted = [r.admitted for r in sorted(res, key=lambda r: r.jid)]
    assert admitted == sorted(admitted)                 # FIFO: no overtaking


def test_job_larger_than_budget_is_rejected(fake_pond):
    jobs = _jobs([32, 8], [10, 10])
    res = serve.Server(budget_bytes=8 * 8 * 100 + 1).run(jobs)
    assert res[0].status.startswith("rejected") and res[1].status == "ok"


def test_summary_percentiles():
    rs = [serve.JobResult(i, 8, 64, 10, arrival=0.0, admitted=0.0, finished=float(i + 1)) for i in range(100)]
    s = serve.summarize(rs)
    assert s["completed"] == 100 and s["makespan_s"] == 100.0
    assert s["p50_s"] == pytest.approx(50.5) and s["p99_s"] == pytest.approx(99.01)
    assert s["runs_per_s"] == pytest.approx(1.0)
    assert s["mlups"] == pytest.approx(100 * 64 * 10 / 100.0 / 1e6, abs=0.05)


def test_serving_workload_is_seeded():
    a, b = serve.make_jobs(8, seed=3, steps=10), serve.make_jobs(8, seed=3, steps=10)
    assert [j.arrival for j in a] == [j.arrival for j in b]
    assert all(np.array_equal(x.case.rho, y.case.rho) for x, y in zip(a, b))
    assert {j.case.n[0] for j in serve.make_jobs(64)} <= {64, 128, 256, 512}

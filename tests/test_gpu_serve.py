"""The serving loop on the device: jobs of mixed sizes and temperatures arriving
over time under a memory budget that keeps some of them waiting; every job's result
is bitwise the one it gets alone (one job at a time, pond_step)."""
import numpy as np
import pytest

from paper_2002_09217_amd import pond, serve

pytestmark = pytest.mark.gpu


def _fields(m):
    return np.concatenate([m[k] for k in ("rho", "ux", "uy", "T", "p", "E")])


@pytest.mark.parametrize("precision", [pond.FP32_STORE, pond.FP64])
def test_served_results_equal_one_at_a_time(precision):
    jobs = serve.make_jobs(count=8, seed=5, steps=90, rate=400.0, sides=(64, 128))
    tiles = {64: 0, 128: 2}
    fp128 = pond.footprint(serve.lattice_config(next(j.case for j in jobs if j.case.n[0] == 128), precision, 2))
    budget = int(2.5 * fp128)
    srv = serve.Server(precision, budget_bytes=budget, chunk=40, tiles=tiles, keep_fields=True)
    got = srv.run(jobs)
    ref = serve.run_sequential(jobs, precision, tiles, keep_fields=True)
    print(serve.summarize(got), serve.summarize(ref), srv.peak_slots, srv.peak_bytes, flush=True)
    assert srv.peak_bytes <= budget and srv.peak_slots >= 2
    for g, r in zip(got, ref):
        assert g.jid == r.jid and g.status.split(":")[0] == r.status.split(":")[0]
        assert g.steps_done == r.steps_done
        assert g.arrival <= g.admitted <= g.finished
        if g.status == "ok":
            assert g.steps_done == 90
            assert np.array_equal(_fields(g.fields), _fields(r.fields))
    assert sum(g.status == "ok" for g in got) >= 6

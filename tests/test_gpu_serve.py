"""The serving loop on the device: jobs of mixed sizes and temperatures arriving
over time under a memory budget that keeps some of them waiting; every job's result
is bitwise the one it gets alone (one job at a time, pond_step)."""
import numpy as np
import pytest

from paper_2002_09217_amd import pond, serve, workloads as W

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


def test_near_spinodal_serving_job_fails_where_the_oracle_does():
    """The smallest serving job that ends with an error (job 1: 128^2, T = 0.85 T_cr, four
    overlapping droplets) is the scheme's failure, not the kernel's: the GPU and the oracle
    agree to round-off up to step 300, and both leave the EoS domain in step 310."""
    from oracle import core
    from tests.common import compare, oracle_config, pond_config

    case = W.serving_jobs()[1][1]
    print(f"serving job 1: {case.meta} n={case.n}", flush=True)
    sim = core.Sim(oracle_config(case))
    sim.init(case.rho, case.u[0], case.T, uy=case.u[1])
    sim.step(300)
    ref = sim.moments()
    lat = pond.Lattice(pond_config(case, tile=0))
    try:
        lat.init_fields(case.rho, case.u, case.T)
        lat.step(300)
        errs = compare(lat.moments(), ref)
        print("job 1, step 300:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        assert max(errs.values()) < 1e-10, errs
        with pytest.raises(pond.PondError):
            lat.step(10)
        gpu_done = lat.steps_done()
    finally:
        lat.close()
    with pytest.raises(core.OracleError):
        sim.step(10)
    assert gpu_done == sim.steps == 309

"""Inputs: the van der Waals constants stored for the workloads are the oracle's, and
the seeded generators are deterministic and shaped as the configurations say."""
import numpy as np

from oracle import write_constants
from paper_2002_09217_amd import workloads as W


def test_stored_constants_are_the_oracles():
    fresh = write_constants.compute()
    stored = W.CONST
    for k in ("a", "b", "R", "rho_cr", "T_cr", "p_cr"):
        assert stored[k] == fresh[k]
    for k in ("T_over_Tcr", "rho_v", "rho_l", "p_sat"):
        assert np.allclose(stored["coexistence"][k], fresh["coexistence"][k], rtol=1e-13, atol=0)
    for k, v in fresh["shock"].items():
        assert np.isclose(stored["shock"][k], v, rtol=1e-12, atol=0), k


def test_generators_are_seeded_and_shaped():
    a = W.perturbed(40, 36, seed=3)
    b = W.perturbed(40, 36, seed=3)
    c = W.perturbed(40, 36, seed=4)
    assert np.array_equal(a.rho, b.rho) and not np.array_equal(a.rho, c.rho)
    assert a.rho.shape == (1440,) and a.u.shape == (2, 1440)
    d = W.static_droplet()
    assert d.n == (256, 256) and d.steps == 20000
    rv, rl = W.coexistence(0.9)
    assert np.isclose(d.rho.max(), rl, rtol=1e-6) and np.isclose(d.rho.min(), rv, rtol=1e-6)
    s = W.shock_tube()
    assert s.n == (1000,) and np.isclose(s.rho[0], 1.5 * W.RHO_CR) and np.isclose(s.rho[-1], 0.5 * W.RHO_CR)
    jobs = W.serving_jobs(count=8, seed=0, steps=10)
    assert len(jobs) == 8 and all(t2 > t1 for (t1, _), (t2, _) in zip(jobs, jobs[1:]))
    assert {j.n[0] for _, j in jobs} <= {64, 128, 256, 512}

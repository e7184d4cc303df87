"""Pins of the predictor-corrector (reading R1 of the oracle).

In Particles-on-Demand the populations of a node are streamed in the gauge (u, theta) that
they themselves carry after the step; the paper reaches it by a predictor-corrector whose
passes each re-derive the gauge from the populations just streamed.  The oracle makes a fixed
number of passes.  These tests check, on the oracle alone, that the passes are that
fixed-point iteration: one step taken with 1, 2, ... passes from the same state changes with
the pass count, the changes shrink geometrically, and many passes reach a state that one more
pass leaves unchanged to round-off (the self-consistent gauge).  A pass that failed to
re-derive the gauge, or re-derived it from the wrong populations or moments, would leave the
result independent of the pass count or stop it converging.
"""
import numpy as np
import pytest

from oracle import core


def _one_step(cfg_kw, fields, n_pass):
    c = core.Config(n_pass=n_pass, **cfg_kw)
    s = core.Sim(c)
    if c.dim == 2:
        s.init(fields["rho"], fields["ux"], fields["T"], uy=fields["uy"])
    else:
        s.init(fields["rho"], fields["ux"], fields["T"])
    s.step(1)
    m = s.moments()
    keys = ("rho", "ux", "uy", "T") if c.dim == 2 else ("rho", "ux", "T")
    return np.concatenate([np.ravel(m[k]) for k in keys])


def _cases():
    rng = np.random.default_rng(7)
    n = 64
    x = np.arange(n) - (n / 2 - 0.5)
    T_cr = 8 * (2 / 49) / (27 * (2 / 21))
    # the van der Waals shock tube (1.5 / 0.5 rho_cr at 1.05 T_cr), jump smoothed over a node
    jump = 0.5 * (1 - np.tanh(x))
    one_d = dict(cfg=dict(dim=1, nx=n, ny=1, omega=1.0, kappa=0.0, dt=0.5,
                          bc=((core.OUTFLOW, core.OUTFLOW), (0, 0))),
                 fields=dict(rho=3.5 * (0.5 + jump), ux=np.zeros(n), T=np.full(n, 1.05 * T_cr)))
    nx, ny = 12, 10
    two_d = dict(cfg=dict(dim=2, nx=nx, ny=ny, omega=1.5, kappa=0.0176, dt=0.2),
                 fields=dict(rho=3.5 * (1 + 0.1 * rng.standard_normal((ny, nx))),
                             ux=0.05 * rng.standard_normal((ny, nx)), uy=0.05 * rng.standard_normal((ny, nx)),
                             T=1.05 * T_cr * (1 + 0.02 * rng.standard_normal((ny, nx)))))
    return {"1d_shock_tube": one_d, "2d_random": two_d}


@pytest.mark.parametrize("name", ["1d_shock_tube", "2d_random"])
def test_passes_converge_to_the_self_consistent_gauge(name):
    case = _cases()[name]
    X = [_one_step(case["cfg"], case["fields"], k) for k in range(1, 13)]
    scale = np.max(np.abs(X[-1]))
    d = [np.max(np.abs(X[k + 1] - X[k])) / scale for k in range(len(X) - 1)]
    # the corrector acts: a second pass changes the step
    assert d[0] > 1e-6
    # contraction: every further pass changes the result by a shrinking amount (until
    # round-off), at a rate well below one
    rates = [d[k + 1] / d[k] for k in range(4)]
    assert max(rates) < 0.5, (d, rates)
    # fixed point: after many passes one more leaves the state unchanged to round-off
    assert d[-1] < 1e-13, d

"""Pin of the oracle's read-back (rho, u-hat, T, p, E) at t = 0.

The initial state (reading R10) stores the collision of the equilibrium of the given
(rho, u-hat, T) in the gauge u = u-hat - F0 dt/(2 rho), with theta = p/(rho T_L).  Read back
before any step, it must return the inputs: rho and u-hat exactly (to round-off), T
through the inversion of p, p = p(rho, T) of the law, and E = e(rho, T) + |u-hat|^2/2.  The
expected p and e are written here from the laws themselves (van der Waals: main text and
App. A; Dieterici: the Supplement's pressure and the exponential-integral form of its
departure energy), not taken from the oracle's helpers.
"""
import math

import numpy as np
import pytest
from scipy.special import expi

from oracle import core
from oracle.thermo import Dieterici, VdW

VDW, DIET = VdW(), Dieterici()


def _laws(kind):
    if kind == core.EOS_VDW:
        a, b, R, Cv = VDW.a, VDW.b, VDW.R, VDW.R / (1.0 / 3.0)
        p = lambda r, T: r * R * T / (1.0 - b * r) - a * r * r
        e = lambda r, T: Cv * T - a * r
        return dict(a=a, b=b, R=R), p, e
    a, b, R, Cv = DIET.a, DIET.b, DIET.R, DIET.R / (1.0 / 3.0)
    p = lambda r, T: r * R * T / (1.0 - b * r) * np.exp(-a * r / (R * T))

    def e(r, T):
        beta = a / (R * T * b)
        return Cv * T - (a / b) * np.exp(-beta) * (expi(beta) - expi((1.0 - b * r) * beta))
    return dict(a=a, b=b, R=R), p, e


@pytest.mark.parametrize("kind", [core.EOS_VDW, core.EOS_DIETERICI])
@pytest.mark.parametrize("dim", [1, 2])
def test_initial_state_reads_back_its_inputs(kind, dim):
    consts, p_of, e_of = _laws(kind)
    nx, ny = 23, (17 if dim == 2 else 1)
    N = nx * ny
    rng = np.random.default_rng(40 + kind + 10 * dim)
    rho = rng.uniform(1.5, 3.0, N)
    ux = rng.uniform(-0.1, 0.1, N)
    uy = rng.uniform(-0.1, 0.1, N) if dim == 2 else None
    T = rng.uniform(1.0, 1.3, N) * VDW.T_cr
    cfg = core.Config(dim=dim, nx=nx, ny=ny, kappa=0.0176, dt=0.2, eos=kind, **consts)
    m = core.Sim(cfg).init(rho, ux, T, uy=uy).moments()
    assert np.allclose(m["rho"], rho, rtol=1e-15, atol=0)
    assert np.allclose(m["ux"], ux, rtol=0, atol=1e-15)
    if dim == 2:
        assert np.allclose(m["uy"], uy, rtol=0, atol=1e-15)
    assert np.allclose(m["T"], T, rtol=1e-13, atol=0)
    assert np.allclose(m["p"], p_of(rho, T), rtol=1e-13, atol=0)
    uh2 = ux * ux + (uy * uy if dim == 2 else 0.0)
    assert np.allclose(m["E"], e_of(rho, T) + 0.5 * uh2, rtol=1e-12, atol=0)


@pytest.mark.parametrize("dim", [1, 2])
def test_uniform_state_with_its_own_inflow_ghosts_is_a_fixed_point(dim):
    """Inflow faces carry the equilibrium of a fixed (rho, u-hat, T) (reading R9).  A uniform
    state equal to that inflow state, with the inflow face upstream and an outflow face
    downstream, must stay put: a wrong ghost (gauge, weights or energy population) would
    disturb the cells next to the face."""
    nx, ny = 30, (12 if dim == 2 else 1)
    N = nx * ny
    rho0, u0, T0 = 2.0, 0.07, 1.1 * VDW.T_cr
    bc = ((core.INFLOW, core.OUTFLOW), (core.PERIODIC, core.PERIODIC))
    inflow = (((rho0, u0, 0.0, T0), (0.0,) * 4), ((0.0,) * 4, (0.0,) * 4))
    cfg = core.Config(dim=dim, nx=nx, ny=ny, bc=bc, inflow=inflow, kappa=0.0176, dt=0.2, omega=1.3)
    sim = core.Sim(cfg).init(np.full(N, rho0), np.full(N, u0), np.full(N, T0),
                             uy=np.zeros(N) if dim == 2 else None)
    sim.step(40)
    m = sim.moments()
    assert np.allclose(m["rho"], rho0, rtol=1e-13, atol=0)
    assert np.allclose(m["ux"], u0, rtol=1e-12, atol=0)
    assert np.allclose(m["T"], T0, rtol=1e-13, atol=0)
    if dim == 2:
        assert np.allclose(m["uy"], 0.0, rtol=0, atol=1e-14)

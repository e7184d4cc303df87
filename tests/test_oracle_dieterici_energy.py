"""Pins of the oracle's Dieterici fluid with the energy equation.

The Supplement's thermodynamics integrates de = C_v dT + [T (dp/dT)_v - p] dv with a
constant C_v; the oracle takes that C_v in the ideal-gas limit v -> oo and integrates the
volume part along the isotherm from there (quadrature), then inverts e(rho, T) and
p(rho, T) for T by Newton's method.  These tests pin that arithmetic by routes that share
none of it:
  * the departure integral in closed form, -(a/b) e^-beta [Ei(beta) - Ei((1 - b rho) beta)]
    with beta = a/(R T b) (scipy's exponential integral);
  * the first law at constant T, (de/drho)_T = (p - T (dp/dT)_rho) / rho^2, by central
    differences of e and p, and (de/dT)_rho against the returned heat capacity;
  * the ideal-gas limit e -> C_v T;
  * T round trips through e and p over the liquid, vapour and supercritical range;
  * an isentrope integrated with the returned heat capacity obeys de = p/rho^2 drho, and the
    isentropic sound speed of App. A, (dp/drho)_T + T (dp/dT)_rho^2 / (rho^2 c_v), is the
    slope of p along it;
  * a pulse in the oracle's D1Q3 run travels at that speed, and a uniform state at rest
    stays put.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp
from scipy.special import expi

from oracle import core
from oracle.thermo import Dieterici
from tests.common import pulse_speed

DIET = Dieterici()
CFG = core.Config(dim=1, nx=4, a=DIET.a, b=DIET.b, R=DIET.R, delta=DIET.delta, eos=core.EOS_DIETERICI)
CV = DIET.R / DIET.delta
STATES = [(r, tr) for tr in (0.6, 0.9, 1.0, 1.5, 3.0) for r in (1e-3, 0.4, 1.8, 3.5, 5.4, 6.6)]


def _closed_form_e(rho, T):
    beta = DIET.a / (DIET.R * T * DIET.b)
    return CV * T - (DIET.a / DIET.b) * math.exp(-beta) * (expi(beta) - expi((1.0 - DIET.b * rho) * beta))


@pytest.mark.parametrize("rho,tr", STATES)
def test_energy_matches_the_exponential_integral_closed_form(rho, tr):
    T = tr * DIET.T_cr
    e = core.eos_e(CFG, rho, T)
    ref = _closed_form_e(rho, T)
    # the closed form loses digits to the difference of two Ei at small rho
    assert e == pytest.approx(ref, rel=1e-13, abs=1e-15)
    assert DIET.e(rho, T) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("rho,tr", [s for s in STATES if s[0] > 0.01])
def test_first_law_at_constant_temperature_and_the_heat_capacity(rho, tr):
    T = tr * DIET.T_cr
    h = 1e-5 * rho
    dedr = (core.eos_e(CFG, rho + h, T) - core.eos_e(CFG, rho - h, T)) / (2 * h)
    hT = 1e-5 * T
    dpdT = (core.eos_p(CFG, rho, T + hT) - core.eos_p(CFG, rho, T - hT)) / (2 * hT)
    p = core.eos_p(CFG, rho, T)
    assert dedr == pytest.approx((p - T * dpdT) / rho ** 2, rel=1e-8)
    dedT = (core.eos_e(CFG, rho, T + hT) - core.eos_e(CFG, rho, T - hT)) / (2 * hT)
    assert core.eos_cv(CFG, rho, T) == pytest.approx(dedT, rel=1e-8)
    assert 0.0 < core.eos_cv(CFG, rho, T) < CV


def test_ideal_gas_limit():
    for tr in (0.7, 1.0, 2.0):
        T = tr * DIET.T_cr
        assert core.eos_e(CFG, 1e-9, T) == pytest.approx(CV * T, rel=1e-9)
        assert core.eos_cv(CFG, 1e-9, T) == pytest.approx(CV, rel=1e-12)


@pytest.mark.parametrize("rho,tr", STATES)
def test_temperature_round_trips(rho, tr):
    T = tr * DIET.T_cr
    assert core.eos_T_of_e(CFG, rho, core.eos_e(CFG, rho, T)) == pytest.approx(T, rel=1e-13)
    assert core.eos_T_of_p(CFG, rho, core.eos_p(CFG, rho, T)) == pytest.approx(T, rel=1e-13)


@pytest.mark.parametrize("rho0,tr", [(1.8, 0.9), (5.4, 0.9), (3.5, 1.2)])
def test_isentrope_obeys_the_first_law_and_sets_the_sound_speed(rho0, tr):
    T0 = tr * DIET.T_cr

    def rhs(r, y):
        T = y[0]
        hT = 1e-6 * T
        dpdT = (core.eos_p(CFG, r, T + hT) - core.eos_p(CFG, r, T - hT)) / (2 * hT)
        return [T * dpdT / (r * r * core.eos_cv(CFG, r, T))]

    rho1 = 1.15 * rho0 if rho0 < 5 else 1.05 * rho0
    sol = solve_ivp(rhs, (rho0, rho1), [T0], rtol=1e-11, atol=0.0, dense_output=True)
    T1 = sol.y[0, -1]
    work = quad(lambda r: core.eos_p(CFG, r, sol.sol(r)[0]) / r ** 2, rho0, rho1, epsabs=0, epsrel=1e-11)[0]
    assert core.eos_e(CFG, rho1, T1) - core.eos_e(CFG, rho0, T0) == pytest.approx(work, rel=1e-7)
    # the slope of p along the isentrope at rho0 is the isentropic sound speed squared
    h = 1e-4 * rho0
    sol_b = solve_ivp(rhs, (rho0, rho0 - h), [T0], rtol=1e-12, atol=0.0)
    sol_f = solve_ivp(rhs, (rho0, rho0 + h), [T0], rtol=1e-12, atol=0.0)
    slope = (core.eos_p(CFG, rho0 + h, sol_f.y[0, -1]) - core.eos_p(CFG, rho0 - h, sol_b.y[0, -1])) / (2 * h)
    assert math.sqrt(slope) == pytest.approx(DIET.sound(rho0, T0), rel=1e-7)


def _cfg(n, **kw):
    base = dict(dim=1, nx=n, ny=1, a=DIET.a, b=DIET.b, R=DIET.R, delta=DIET.delta, omega=1.5, kappa=0.0,
                n_pass=2, dt=0.2, eos=core.EOS_DIETERICI, isothermal=0)
    base.update(kw)
    return core.Config(**base)


def test_uniform_state_is_a_fixed_point():
    c = _cfg(12, omega=1.2)
    T = 1.1 * DIET.T_cr
    s = core.Sim(c).init(np.full(12, 2.3), np.full(12, 0.05), np.full(12, T))
    s.step(20)
    m = s.moments()
    assert np.allclose(m["rho"], 2.3, rtol=1e-13, atol=0)
    assert np.allclose(m["ux"], 0.05, rtol=1e-12, atol=0)
    assert np.allclose(m["T"], T, rtol=1e-12, atol=0)


@pytest.mark.parametrize("rho0,tr", [(1.75, 1.05), (3.5, 1.2)])
def test_pulse_travels_at_the_isentropic_sound_speed(rho0, tr):
    def factory(rho, T, dt):
        return core.Sim(_cfg(rho.size, dt=dt)).init(rho, np.zeros(rho.size), T)

    T0 = tr * DIET.T_cr
    c_ref = DIET.sound(rho0, T0)
    c = pulse_speed(factory, rho0, tr, isentrope=lambda r: DIET.T_isentrope(r, rho0, T0))
    assert c == pytest.approx(c_ref, rel=3e-3)

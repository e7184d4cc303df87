"""Pins of the oracle's van der Waals thermodynamics against what the paper prints
and against what the mathematics fixes independently of the oracle's formulas.

Reyhanian, Dorschner & Karlin, arXiv:2002.09217: main text (EoS, critical values,
speed of sound at the critical point), App. A (C_p, speed of sound), App. E
(fundamental derivative, shock-tube table, Rankine-Hugoniot)."""
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

from oracle.thermo import VdW

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
REDUCED = dict(a=3.0, b=1.0 / 3.0, R=8.0 / 3.0)  # vdW in reduced variables p/p_cr, v/v_cr, T/T_cr


def _isentrope_p(v0, T0, gas, dv):
    """p along the isentrope through (v0, T0): for the vdW fluid with constant C_v the
    entropy is s = C_v ln T + R ln(v - b) + const, so T (v - b)^(R/C_v) is constant."""
    k = gas.R / gas.Cv
    v = v0 + dv
    T = T0 * ((v0 - gas.b) / (v - gas.b)) ** k
    return gas.R * T / (v - gas.b) - gas.a / v**2


def test_critical_point_is_the_inflection_of_the_critical_isotherm():
    g = VdW()
    assert g.rho_cr == pytest.approx(3.5, rel=1e-15)
    assert g.T_cr == pytest.approx(8.0 / 63.0, rel=1e-15)
    assert g.p_cr == pytest.approx(1.0 / 6.0, rel=1e-15)
    assert g.p(g.rho_cr, g.T_cr) == pytest.approx(g.p_cr, rel=1e-14)
    h = 1e-3
    r, T = g.rho_cr, g.T_cr
    d1 = (g.p(r + h, T) - g.p(r - h, T)) / (2 * h)
    d2 = (g.p(r + h, T) - 2 * g.p(r, T) + g.p(r - h, T)) / h**2
    assert abs(d1) < 1e-6 and abs(d2) < 1e-5
    # just below T_cr the isotherm has a loop, just above it is monotone
    rr = np.linspace(0.5 * r, 1.5 * r, 2001)
    assert np.min(np.diff(g.p(rr, 0.99 * T))) < 0.0
    assert np.min(np.diff(g.p(rr, 1.01 * T))) > 0.0


def test_energy_temperature_round_trip():
    g = VdW()
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.5, 7.0, 200)
    T = rng.uniform(0.5, 1.5, 200) * g.T_cr
    assert np.allclose(g.T_of_e(rho, g.e(rho, T)), T, rtol=1e-14, atol=0)
    assert np.allclose(g.T_of_p(rho, g.p(rho, T)), T, rtol=1e-12, atol=0)


@pytest.mark.parametrize("delta", [1.0 / 3.0, 2.0 / 3.0, 0.0125])
def test_sound_speed_three_routes(delta):
    """App. A: vdW closed form == general relation == (C_p/C_v)(dp/drho)_T, and all equal
    -v^2 (dp/dv)_s taken numerically along the isentrope."""
    g = VdW(delta=delta)
    for rho, Tr in [(1.0, 1.2), (5.8, 0.9), (1.49, 0.9), (3.0, 1.05)]:
        T = Tr * g.T_cr
        c_vdw = g.sound_vdw(rho, T)
        assert g.sound_general(rho, T) == pytest.approx(c_vdw, rel=1e-13)
        assert math.sqrt(g.Cp_vdw(rho, T) / g.Cv * g.dp_drho_T(rho, T)) == pytest.approx(c_vdw, rel=1e-12)
        assert g.Cp_general(rho, T) == pytest.approx(g.Cp_vdw(rho, T), rel=1e-12)
        v, h = 1.0 / rho, 1e-5 / rho
        dpdv = (_isentrope_p(v, T, g, h) - _isentrope_p(v, T, g, -h)) / (2 * h)
        assert math.sqrt(-v * v * dpdv) == pytest.approx(c_vdw, rel=1e-8)


@pytest.mark.parametrize("delta", [1.0 / 3.0, 2.0 / 3.0])
def test_isentrope_satisfies_the_first_law(delta):
    """Along the oracle's isentrope de = -p dv (no heat): the numerical derivative of
    e(T(v), v) plus p vanishes, and (dp/drho) along it is the sound speed squared."""
    g = VdW(delta=delta)
    for rho0, Tr in [(1.49, 0.9), (5.8, 0.9), (3.5, 1.2)]:
        T0 = Tr * g.T_cr
        v0, h = 1.0 / rho0, 1e-5 / rho0

        def e_of_v(v):
            T = g.T_isentrope(1.0 / v, rho0, T0)
            return g.e(1.0 / v, T)

        dedv = (e_of_v(v0 + h) - e_of_v(v0 - h)) / (2 * h)
        assert dedv + g.p(rho0, T0) == pytest.approx(0.0, abs=1e-8 * g.p(rho0, T0))
        r, hr = rho0, 1e-5 * rho0
        dpdr = (g.p(r + hr, g.T_isentrope(r + hr, rho0, T0)) - g.p(r - hr, g.T_isentrope(r - hr, rho0, T0))) / (2 * hr)
        assert math.sqrt(dpdr) == pytest.approx(g.sound_vdw(rho0, T0), rel=1e-8)


def test_sound_speed_at_critical_point():
    """Main text: the speed of sound at the critical point is sqrt(2 p_cr v_cr) (delta = 1/3)."""
    g = VdW(delta=1.0 / 3.0)
    c = g.sound_vdw(g.rho_cr, g.T_cr)
    assert c * c == pytest.approx(2.0 * g.p_cr / g.rho_cr, rel=1e-14)
    assert c * c == pytest.approx(0.0952380952380952, rel=1e-12)


def test_ideal_gas_limit_of_bulk_viscosity_factor():
    """Main text after eq. 15: for p -> rho R T the sound speed tends to (D+2) R T/D for the
    monatomic value C_v = D R/2, so (D+2)/D - rho c^2/p vanishes."""
    for D in (1, 2, 3):
        g = VdW(a=0.0, b=0.0, R=1.0, delta=2.0 / D if D > 1 else 2.0 / 3.0)
        if D == 1:
            continue  # delta <= 2/3 in the paper; D = 1 monatomic would need delta = 2
        rho, T = 0.7, 0.3
        c2 = g.sound_vdw(rho, T) ** 2
        assert (D + 2) / D - rho * c2 / g.p(rho, T) == pytest.approx(0.0, abs=1e-14)


def _load_table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_fundamental_derivative_shock_tube_table():
    """App. E table: Gamma of the left and right states (reduced units)."""
    for case, pL, rL, pR, rR, GL, GR, d in _load_table("shock_tube_conditions.txt"):
        g = VdW(delta=float(d), **REDUCED)
        assert g.gamma(float(pL), 1.0 / float(rL)) == pytest.approx(float(GL), abs=6e-4), case
        assert g.gamma(float(pR), 1.0 / float(rR)) == pytest.approx(float(GR), abs=6e-4), case


def test_fundamental_derivative_anomalous_states_negative():
    for side, p, r, d, sign in _load_table("anomalous_shock_states.txt"):
        g = VdW(delta=float(d), **REDUCED)
        assert np.sign(g.gamma(float(p), 1.0 / float(r))) == int(sign), side


def test_fundamental_derivative_matches_its_definition():
    """Gamma = v^3/(2 c^2) (d^2 p/dv^2)_s, second derivative taken numerically on the isentrope."""
    for d in (0.0125, 0.329, 1.0 / 3.0):
        g = VdW(delta=d, **REDUCED)
        for p, rho in [(1.09, 0.879), (1.6077, 1.01), (0.575, 0.275), (3.0, 1.818)]:
            v = 1.0 / rho
            T = g.T_of_p(rho, p)
            h = 2e-4 * v
            d2 = (_isentrope_p(v, T, g, h) - 2 * _isentrope_p(v, T, g, 0.0) + _isentrope_p(v, T, g, -h)) / h**2
            c2 = g.sound_vdw(rho, T) ** 2
            assert g.gamma(p, v) == pytest.approx(v**3 / (2 * c2) * d2, rel=2e-5, abs=2e-5)


def test_maxwell_near_critical_asymptote():
    """Near T_cr the vdW coexistence densities obey (rho_l - rho_v)/rho_cr -> 4 sqrt(1 - T/T_cr)."""
    g = VdW()
    for tau in (1e-4, 1e-5):
        rv, rl, _ = g.maxwell((1 - tau) * g.T_cr)
        assert (rl - rv) / g.rho_cr == pytest.approx(4 * math.sqrt(tau), rel=2 * tau + 1e-7)


def test_maxwell_equal_area_by_quadrature_and_stability():
    g = VdW()
    for Tr in (0.85, 0.9, 0.95):
        T = Tr * g.T_cr
        rv, rl, ps = g.maxwell(T)
        assert g.p(rv, T) == pytest.approx(ps, rel=1e-11)
        assert g.p(rl, T) == pytest.approx(ps, rel=1e-11)
        area, _ = quad(lambda v: g.R * T / (v - g.b) - g.a / v**2, 1 / rl, 1 / rv, epsabs=0, epsrel=1e-13)
        assert area == pytest.approx(ps * (1 / rv - 1 / rl), rel=1e-10)
        assert g.dp_drho_T(rv, T) > 0 and g.dp_drho_T(rl, T) > 0  # both on stable branches


def test_maxwell_corresponding_states_and_reduced_pressure():
    """The reduced coexistence curve is the same for any (a, b, R); the reduced saturation
    pressure of the van der Waals fluid is 0.6470 at T/T_cr = 0.9 and 0.8119 at 0.95."""
    g, red = VdW(), VdW(**REDUCED)
    for Tr, pr in ((0.9, 0.6470), (0.95, 0.8119)):
        rv, rl, ps = g.maxwell(Tr * g.T_cr)
        rv2, rl2, ps2 = red.maxwell(Tr * red.T_cr)
        assert rv / g.rho_cr == pytest.approx(rv2 / red.rho_cr, rel=1e-10)
        assert rl / g.rho_cr == pytest.approx(rl2 / red.rho_cr, rel=1e-10)
        assert ps / g.p_cr == pytest.approx(pr, abs=6e-5)
    # coexistence densities do not depend on delta (main text, Fig. 2)
    assert VdW(delta=2 / 3).maxwell(0.9 * g.T_cr)[0] == pytest.approx(g.maxwell(0.9 * g.T_cr)[0], rel=1e-14)


@pytest.mark.parametrize("delta", [1.0 / 3.0, 2.0 / 3.0])
def test_rankine_hugoniot_closed_form_vs_direct(delta):
    """App. E closed form (rho_1 as parameter) against a direct solve of the jump conditions.
    The printed velocity line is read with the pre-shock sound speed."""
    g = VdW(delta=delta)
    T0 = 0.95 * g.T_cr
    rho0, _, p0 = g.maxwell(T0)
    d = g.hugoniot_direct(rho0, p0, 3.0 * p0)
    res = g.rh_jump_residual(rho0, p0, 0.0, d["rho1"], d["p1"], d["u1"], d["s"])
    assert np.max(np.abs(res)) < 1e-13
    M0, u1, p1 = g.rh_closed_form(rho0, p0, d["rho1"])
    assert p1 == pytest.approx(d["p1"], rel=1e-10)
    assert M0 == pytest.approx(d["Ms"], rel=1e-10)
    assert u1 == pytest.approx(d["u1"], rel=1e-10)
    if delta == 1.0 / 3.0:
        assert d["rho1"] == pytest.approx(3.84380084, rel=1e-7)
        assert d["u1"] == pytest.approx(0.25126554, rel=1e-6)

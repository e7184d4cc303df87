"""Pins of the oracle's isothermal equations of state (Supplement: speed of sound in the
simplified free energy and in the van der Waals fluid, coexistence curve of the
Dieterici fluid) against what the paper prints and what the mathematics fixes, and
isothermal runs of the oracle against them."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import core
from oracle.thermo import DoubleWell, Dieterici, VdW, maxwell_isotherm
from tests.common import pulse_speed

DIET = Dieterici()
VDW = VdW()
WELLS = [DoubleWell(8e-4, 5.0, 0.5, 0.1), DoubleWell(3e-3, 3.0, 0.3, 0.05)]


def test_dieterici_printed_critical_values_are_the_inflection_of_the_critical_isotherm():
    r, T, h = DIET.rho_cr, DIET.T_cr, 1e-3
    p = lambda x: DIET.p(x, T)
    assert p(r) == pytest.approx(DIET.p_cr, rel=1e-14)
    assert abs((p(r + h) - p(r - h)) / (2 * h)) < 1e-7
    assert abs((p(r + h) - 2 * p(r) + p(r - h)) / h**2) < 1e-6
    rr = np.linspace(0.5 * r, 1.5 * r, 2001)
    assert np.min(np.diff(DIET.p(rr, 0.99 * T))) < 0.0
    assert np.min(np.diff(DIET.p(rr, 1.01 * T))) > 0.0


def test_dieterici_reduced_form():
    """p/p_cr = rho_r T_r e^2/(2 - rho_r) exp(-2 rho_r/T_r), the printed reduced form."""
    rng = np.random.default_rng(5)
    rr, tr = rng.uniform(0.05, 1.95, 50), rng.uniform(0.6, 1.6, 50)
    got = DIET.p(rr * DIET.rho_cr, tr * DIET.T_cr) / DIET.p_cr
    want = rr * tr * math.e**2 / (2.0 - rr) * np.exp(-2.0 * rr / tr)
    assert np.allclose(got, want, rtol=1e-13, atol=0)


def test_dieterici_coexistence_near_critical_asymptote():
    """In reduced variables ln p = ln rho + ln T + 2 - ln(2 - rho) - 2 rho/T, so at the
    critical point d3p/drho3 = 4 and d2p/drho dT = 2.  With p ~ p(1, T) + 2 w t + (2/3) w^3
    (w = rho_r - 1, t = T_r - 1) the two coexisting branches are w = +-sqrt(-3 t):
    (rho_l - rho_v)/rho_cr -> 2 sqrt(3) sqrt(1 - T_r)."""
    for tau in (1e-5, 1e-6):
        rv, rl, _ = DIET.maxwell((1 - tau) * DIET.T_cr)
        assert (rl - rv) / DIET.rho_cr == pytest.approx(2 * math.sqrt(3 * tau), rel=5 * tau + 2e-6)


@pytest.mark.parametrize("Tr", [0.8, 0.9, 0.95])
def test_dieterici_coexistence_equal_pressure_and_chemical_potential(Tr):
    """The coexisting states share p and the chemical potential; along the isotherm
    d mu = dp/rho, integrated here in rho (the equal-area rule works in v)."""
    T = Tr * DIET.T_cr
    rv, rl, ps = DIET.maxwell(T)
    assert DIET.p(rv, T) == pytest.approx(ps, rel=1e-11) and DIET.p(rl, T) == pytest.approx(ps, rel=1e-11)
    dmu, _ = quad(lambda r: DIET.dp_drho_T(r, T) / r, rv, rl, epsabs=1e-14 * ps / rl, epsrel=0, limit=400)
    assert abs(dmu) < 1e-10 * ps / rl
    assert DIET.dp_drho_T(rv, T) > 0 and DIET.dp_drho_T(rl, T) > 0


@pytest.mark.parametrize("w", WELLS)
def test_double_well_saturation_states_and_printed_sound_speeds(w):
    """p(rho_l) = p(rho_v) = p0 (both minima of E0 are zero); (dp/drho) at the saturated
    densities, by central differences of p, equals the printed sound speeds squared;
    Maxwell's rule returns the two minima (their common tangent is E0 = 0)."""
    assert w.p(w.rho_l) == pytest.approx(w.p0, rel=1e-15) and w.p(w.rho_v) == pytest.approx(w.p0, rel=1e-15)
    cl, cv = w.sound_saturated()
    for r, c in ((w.rho_l, cl), (w.rho_v, cv)):
        h = 1e-5 * r
        assert (w.p(r + h) - w.p(r - h)) / (2 * h) == pytest.approx(c * c, rel=1e-8)
    rv, rl, ps = w.maxwell()
    assert rv == pytest.approx(w.rho_v, rel=1e-12) and rl == pytest.approx(w.rho_l, rel=1e-12)
    assert ps == pytest.approx(w.p0, rel=1e-12)


def test_generic_maxwell_equals_the_van_der_waals_construction():
    for Tr in (0.85, 0.9, 0.95):
        T = Tr * VDW.T_cr
        a = VDW.maxwell(T)
        b = maxwell_isotherm(lambda r: VDW.p(r, T), lambda r: VDW.dp_drho_T(r, T), 1e-9, (1 - 1e-12) / VDW.b)
        assert np.allclose(a, b, rtol=1e-11, atol=0)


# ----------------------------------------------------------------------------
# isothermal runs of the oracle
# ----------------------------------------------------------------------------
def _cfg(kind, n, T0, c=(0.0, 0.0, 0.0, 0.0), **kw):
    base = dict(dim=1, nx=n, ny=1, omega=1.5, kappa=0.0, n_pass=2, dt=0.2, eos=kind, isothermal=1, T0=T0,
                eos_c=tuple(c))
    if kind == core.EOS_DIETERICI:
        base.update(a=DIET.a, b=DIET.b, R=DIET.R)
    base.update(kw)
    return core.Config(**base)


def test_isothermal_requirements_are_validated():
    with pytest.raises(core.OracleError):
        core.Sim(_cfg(core.EOS_WELL, 8, 0.1, c=(1e-3, 0.5, 5.0, 0.1))).init(np.full(8, 2.0), np.zeros(8),
                                                                                np.full(8, 0.1))


@pytest.mark.parametrize("kind", [core.EOS_VDW, core.EOS_DIETERICI, core.EOS_WELL])
def test_isothermal_uniform_state_is_fixed_point(kind):
    c = _cfg(kind, 12, 0.9 * 8 / 63, c=(8e-4, 5.0, 0.5, 0.1), omega=1.2)
    rho = np.full(12, 2.3)
    s = core.Sim(c).init(rho, np.full(12, 0.05), np.full(12, 0.5))   # the T input is replaced by T0
    s.step(20)
    m = s.moments()
    assert np.allclose(m["rho"], 2.3, rtol=1e-13, atol=0)
    assert np.allclose(m["ux"], 0.05, rtol=1e-12, atol=0)
    assert np.allclose(m["T"], c.T0, rtol=0, atol=0)


@pytest.mark.parametrize("w", WELLS)
def test_isothermal_pulse_in_the_double_well_travels_at_the_printed_speed(w):
    for rho0, c_ref in zip((w.rho_l, w.rho_v), w.sound_saturated()):
        def factory(rho, T, dt):
            return core.Sim(_cfg(core.EOS_WELL, rho.size, 0.1, c=(w.beta, w.rho_l, w.rho_v, w.p0), dt=dt)).init(
                rho, np.zeros(rho.size), np.full(rho.size, 0.1))

        # measured over 60 to 120 nodes of travel, so that the two half-pulses have separated
        times = (round(60.0 / c_ref), round(120.0 / c_ref))
        assert pulse_speed(factory, rho0, 1.0, times=times) == pytest.approx(c_ref, rel=3e-3)


@pytest.mark.parametrize("side", [0, 1])
def test_isothermal_vdw_pulse_travels_at_the_isothermal_sound_speed(side):
    """Supplement: the isothermal speed of sound of the van der Waals fluid at the
    saturated densities, sqrt((dp/drho)_T)."""
    T0 = 0.9 * VDW.T_cr
    rho0 = VDW.maxwell(T0)[side]

    def factory(rho, T, dt):
        return core.Sim(_cfg(core.EOS_VDW, rho.size, T0, dt=dt)).init(rho, np.zeros(rho.size), np.full(rho.size, T0))

    c_ref = math.sqrt(VDW.dp_drho_T(rho0, T0))
    times = (round(60.0 / c_ref), round(120.0 / c_ref))
    assert pulse_speed(factory, rho0, 0.9, times=times) == pytest.approx(c_ref, rel=3e-3)


def test_isothermal_dieterici_slab_relaxes_to_maxwell_coexistence():
    """Supplement, coexistence curve: a liquid slab in its vapour at 0.9 T_cr.  Without
    an energy equation the acoustic transient of the initial profile decays slowly, so
    the densities at the centres of the two phases are averaged over 8000 steps."""
    N, T0 = 400, 0.9 * DIET.T_cr
    rv, rl, _ = DIET.maxwell(T0)
    x = np.arange(N)
    prof = 0.5 * (np.tanh((x - N / 4) / 3.0) - np.tanh((x - 3 * N / 4) / 3.0))
    s = core.Sim(_cfg(core.EOS_DIETERICI, N, T0, omega=1.0, kappa=0.0176, dt=0.1)).init(
        rv + (rl - rv) * prof, np.zeros(N), np.full(N, T0))
    s.step(4000)
    vap, liq = [], []
    for _ in range(40):
        s.step(200)
        r = s.moments()["rho"]
        vap.append(0.5 * (r[:20].mean() + r[-20:].mean()))
        liq.append(r[N // 2 - 10:N // 2 + 10].mean())
    ev, el = np.mean(vap) / rv - 1, np.mean(liq) / rl - 1
    assert abs(ev) < 0.01 and abs(el) < 0.01, (ev, el)


@pytest.mark.parametrize("kind", [core.EOS_DIETERICI, core.EOS_WELL])
def test_three_dimensional_oracle_reduces_to_one_dimension(kind):
    """A box that varies along x only: D3Q27 factors into D1Q3 times the rest directions
    of y and z, so the 3D oracle reproduces the 1D one (kappa = 0) up to round-off."""
    n, T0 = 24, 0.9 * DIET.T_cr
    cw = (8e-4, 5.0, 0.5, 0.1)
    x = np.arange(n)
    rho = (2.0 if kind == core.EOS_DIETERICI else 5.0) * (1.0 + 0.05 * np.sin(2 * np.pi * x / n))
    u = 0.02 * np.cos(2 * np.pi * x / n)
    c1 = _cfg(kind, n, T0, c=cw, dt=0.2)
    s1 = core.Sim(c1).init(rho, u, np.full(n, T0))
    s1.step(15)
    m1 = s1.moments()
    c3 = core.Config3(nx=n, ny=1, nz=1, a=c1.a, b=c1.b, R=c1.R, omega=c1.omega, kappa=0.0, dt=0.2, n_pass=2,
                      eos=kind, isothermal=1, T0=T0, eos_c=cw)
    s3 = core.Sim3(c3).init(rho, np.stack([u, np.zeros(n), np.zeros(n)]), np.full(n, T0))
    s3.step(15)
    m3 = s3.moments()
    assert np.allclose(m3["rho"], m1["rho"], rtol=1e-12, atol=0)
    assert np.allclose(m3["ux"], m1["ux"], rtol=0, atol=1e-13)
    assert np.all(m3["T"] == T0)

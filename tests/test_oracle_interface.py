"""Pins of the planar-interface thermodynamics the surface-tension tests use.

The interface energy kappa/2 |grad rho|^2 behind the Korteweg stress of eq. 18 gives a
planar equilibrium profile with kappa rho'^2 / 2 = omega(rho), where omega is the excess
grand potential density against the coexisting phases, and the surface tension
sigma = int sqrt(2 kappa omega) d rho.  The Supplement measures the surface tension with
the Laplace law on 2D droplets; these tests pin the reference value by routes that do not
share the quadrature:
  * rho mu - f is the van der Waals pressure (main text), so f and mu are right;
  * omega vanishes with zero slope at both Maxwell densities;
  * solving the profile equation kappa rho'' = mu(rho) - mu_sat on a grid and integrating
    kappa rho'^2 gives the same sigma;
  * near T_cr, sigma and the 10-90 % width follow the closed mean-field limits of the van
    der Waals fluid, sigma -> 16 sqrt(kappa a) (1 - T_r)^(3/2) / (27 b^2) and
    width -> 2 atanh(0.8) sqrt(kappa / a) / sqrt(1 - T_r) (Landau expansion about the
    critical point, where d^3 mu/d rho^3 = 27 a b^2 and d^2 mu/d rho dT = 27 R b / 4);
  * the droplet workloads' kappa = 0.0176 gives the 10-90 % width of their tanh profile.
"""
import math

import numpy as np
import pytest
from scipy.linalg import solve_banded

from oracle.thermo import VdW

VDW = VdW()


def test_free_energy_and_chemical_potential_give_the_eos_pressure():
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.2, 9.5, 200)
    T = rng.uniform(0.7, 1.4, 200) * VDW.T_cr
    p = rho * VDW.chem_potential(rho, T) - VDW.free_energy(rho, T)
    assert np.allclose(p, VDW.p(rho, T), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("Tr", [0.85, 0.9, 0.95])
def test_grand_excess_vanishes_with_zero_slope_at_coexistence(Tr):
    T = Tr * VDW.T_cr
    rv, rl, _ = VDW.maxwell(T)
    scale = VDW.p_cr
    assert abs(VDW.grand_excess(rl, T, rv)) < 1e-12 * scale
    inner = np.linspace(rv, rl, 101)[1:-1]
    assert np.all(VDW.grand_excess(inner, T, rv) > 0.0)
    h = 1e-6
    for r in (rv, rl):
        slope = (VDW.grand_excess(r + h, T, rv) - VDW.grand_excess(r - h, T, rv)) / (2 * h)
        assert abs(slope) < 1e-8


def test_surface_tension_equals_the_integral_of_the_solved_profile():
    """Newton solve of kappa rho'' = mu(rho) - mu_sat on a fine grid (centre pinned at the
    mean density, bulk densities at the ends), then sigma = int kappa rho'^2 dx."""
    T, kappa = 0.9 * VDW.T_cr, 0.0176
    rv, rl, _ = VDW.maxwell(T)
    mu_sat = VDW.chem_potential(rv, T)
    L, n = 40.0, 8001
    x = np.linspace(-L, L, n)
    h = x[1] - x[0]
    rho = 0.5 * (rl + rv) + 0.5 * (rl - rv) * np.tanh(x / 2.0)
    mid = n // 2
    for _ in range(60):
        mu = VDW.chem_potential(rho, T)
        dmu = (VDW.chem_potential(rho + 1e-7, T) - VDW.chem_potential(rho - 1e-7, T)) / 2e-7
        res = np.zeros(n)
        res[1:-1] = kappa * (rho[2:] - 2 * rho[1:-1] + rho[:-2]) / h ** 2 - (mu[1:-1] - mu_sat)
        res[0], res[-1] = rho[0] - rv, rho[-1] - rl
        res[mid] = rho[mid] - 0.5 * (rl + rv)
        ab = np.zeros((3, n))                      # banded Jacobian: upper, diagonal, lower
        ab[0, 2:] = kappa / h ** 2
        ab[1, 1:-1] = -2 * kappa / h ** 2 - dmu[1:-1]
        ab[2, :-2] = kappa / h ** 2
        ab[1, 0] = ab[1, -1] = 1.0
        ab[0, 1] = 0.0
        ab[2, -2] = 0.0
        ab[0, mid + 1], ab[2, mid - 1], ab[1, mid] = 0.0, 0.0, 1.0
        step = solve_banded((1, 1), ab, -res)
        rho += step
        if np.max(np.abs(step)) < 1e-13:
            break
    grad = np.gradient(rho, h)
    sigma_profile = np.trapezoid(kappa * grad ** 2, x)
    assert sigma_profile == pytest.approx(VDW.surface_tension(T, kappa), rel=1e-5)
    # equipartition along the solved profile: kappa rho'^2 / 2 = omega
    om = VDW.grand_excess(rho, T, rv)
    inner = np.abs(x) < 10
    assert np.allclose(0.5 * kappa * grad[inner] ** 2, om[inner], rtol=1e-4, atol=1e-9)


def test_near_critical_limits_of_tension_and_width():
    a, b = VDW.a, VDW.b
    sig_lim = 16.0 * math.sqrt(a) / (27.0 * b * b)
    width_lim = 2.0 * math.atanh(0.8) / math.sqrt(a)
    for one_minus_tr, tol in ((1e-3, 2e-3), (1e-4, 3e-4)):
        T = (1.0 - one_minus_tr) * VDW.T_cr
        assert VDW.surface_tension(T, 1.0) / one_minus_tr ** 1.5 == pytest.approx(sig_lim, rel=tol)
        assert VDW.interface_width(T, 1.0) * math.sqrt(one_minus_tr) == pytest.approx(width_lim, rel=tol)


def test_droplet_kappa_matches_the_tanh_profile_width():
    """kappa = 0.0176 (droplet workloads) makes the equilibrium 10-90 % width at 0.9 T_cr that
    of their profile tanh(2 (r - R) / 4), i.e. 4 atanh(0.8) nodes."""
    w = VDW.interface_width(0.9 * VDW.T_cr, 0.0176)
    assert w == pytest.approx(4.0 * math.atanh(0.8), rel=5e-3)   # kappa is given to three digits

"""TEST INFRASTRUCTURE ONLY -- van der Waals thermodynamics used by the oracle tests.

Only the test suite, ``__graft_entry__.smoke()``, the CPU-baseline leg of
``bench.py`` and ``oracle/write_constants.py`` may import this module.

Everything follows Reyhanian, Dorschner & Karlin (arXiv:2002.09217):
  * van der Waals EoS p = rho R T/(1 - b rho) - a rho^2 and critical values
    rho_cr = 1/(3b), T_cr = 8a/(27 R b), p_cr = a/(27 b^2)          (main text)
  * e = C_v T - a rho, C_v = R/delta                                   (main text; App. A)
  * C_p, the speed of sound (general and van der Waals forms)          (App. A)
  * the fundamental derivative Gamma(p, v) of the van der Waals fluid  (App. E, shock tube)
  * Rankine-Hugoniot post-shock state                                  (App. E)
  * Maxwell's equal-area rule for the coexistence densities            (main text, Fig. 2)
  * the Dieterici pressure and its printed critical values             (Supplement, coexistence)
  * the Dieterici internal energy e = C_v T + int [T (dp/dT)_v - p] dv, its heat
    capacity, isentropes and isentropic sound speed                    (Supplement, thermodynamics)
  * the simplified (double-well) free energy near the critical point,
    with the printed saturated sound speeds                            (Supplement, speed of sound)
  * Maxwell's rule for any isotherm with one loop
  * the planar interface of the interface energy kappa/2 |grad rho|^2 (eq. 18): surface
    tension and width of the equilibrium profile                      (Supplement, surface tension)
All arithmetic is FP64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.integrate import quad
from scipy.optimize import brentq

A_SIM, B_SIM, R_SIM = 2.0 / 49.0, 2.0 / 21.0, 1.0  # constants used in the paper's simulations


@dataclass(frozen=True)
class VdW:
    a: float = A_SIM
    b: float = B_SIM
    R: float = R_SIM
    delta: float = 1.0 / 3.0

    # critical point (main text)
    @property
    def rho_cr(self) -> float:
        return 1.0 / (3.0 * self.b)

    @property
    def T_cr(self) -> float:
        return 8.0 * self.a / (27.0 * self.R * self.b)

    @property
    def p_cr(self) -> float:
        return self.a / (27.0 * self.b * self.b)

    @property
    def Cv(self) -> float:
        return self.R / self.delta

    # EoS and caloric relation
    def p(self, rho, T):
        return rho * self.R * T / (1.0 - self.b * rho) - self.a * rho * rho

    def e(self, rho, T):
        return self.Cv * T - self.a * rho

    def T_of_e(self, rho, e):
        return (e + self.a * rho) / self.Cv

    def T_of_p(self, rho, p):
        return (p + self.a * rho * rho) * (1.0 - self.b * rho) / (rho * self.R)

    # partial derivatives of p(rho, T)
    def dp_drho_T(self, rho, T):
        return self.R * T / (1.0 - self.b * rho) ** 2 - 2.0 * self.a * rho

    def dp_dT_rho(self, rho, T):
        return rho * self.R / (1.0 - self.b * rho)

    # App. A: C_p = C_v + T (dp/dT)_v (dv/dT)_p, general form with the EoS derivatives
    def Cp_general(self, rho, T):
        v = 1.0 / rho
        dp_dT_v = self.dp_dT_rho(rho, T)
        dp_dv_T = -rho * rho * self.dp_drho_T(rho, T)
        dv_dT_p = -dp_dT_v / dp_dv_T
        return self.Cv + T * dp_dT_v * dv_dT_p + 0.0 * v

    # App. A: closed form for the van der Waals fluid
    def Cp_vdw(self, rho, T):
        R = self.R
        return self.Cv + R * R * T / (R * T - 2.0 * self.a * rho * (1.0 - self.b * rho) ** 2)

    # Isentrope through (rho0, T0): with constant C_v the entropy is
    # s = C_v ln T + R ln(v - b) + const (first law with e = C_v T - a/v), so
    # T (v - b)^(R/C_v) is constant along it.
    def T_isentrope(self, rho, rho0, T0):
        return T0 * ((1.0 / rho0 - self.b) / (1.0 / rho - self.b)) ** (self.R / self.Cv)

    # App. A: sound speed, general relation and the van der Waals closed form
    def sound_general(self, rho, T):
        return math.sqrt(self.dp_drho_T(rho, T) + T / (rho * rho * self.Cv) * self.dp_dT_rho(rho, T) ** 2)

    def sound_vdw(self, rho, T):
        return math.sqrt(self.R * T / (1.0 - self.b * rho) ** 2 * (1.0 + self.delta) - 2.0 * self.a * rho)

    # App. E: fundamental derivative of the van der Waals fluid
    def gamma(self, p, v):
        a, b, d = self.a, self.b, self.delta
        num = (d + 1.0) * (d + 2.0) * (p + a / v**2) / (v - b) ** 2 - 6.0 * a / v**4
        den = 2.0 * (d + 1.0) * (p + a / v**2) / (v * (v - b)) - 4.0 * a / v**4
        return num / den

    # ------------------------------------------------------------------
    # Maxwell's equal-area rule (main text, Fig. 2)
    # ------------------------------------------------------------------
    def spinodal(self, T):
        """Densities where (dp/drho)_T = 0 at T < T_cr (vapor-side, liquid-side)."""
        rc = self.rho_cr
        f = lambda r: self.dp_drho_T(r, T)
        lo = brentq(f, 1e-12, rc, xtol=1e-15, rtol=1e-15, maxiter=500)
        hi = brentq(f, rc, (1.0 - 1e-12) / self.b, xtol=1e-15, rtol=1e-15, maxiter=500)
        return lo, hi

    def _outer_roots(self, T, ps):
        """Smallest and largest specific volume with p(v) = ps (roots of the cubic)."""
        a, b, R = self.a, self.b, self.R
        roots = np.roots([ps, -(ps * b + R * T), a, -a * b])
        real = np.sort(roots[np.abs(roots.imag) < 1e-9 * np.abs(roots).max()].real)
        real = real[real > b]
        return real[0], real[-1]

    def maxwell(self, T):
        """(rho_vapor, rho_liquid, p_sat) at T < T_cr from the equal-area rule
        int_{v_l}^{v_v} p dv = p_sat (v_v - v_l)."""
        if not T < self.T_cr:
            raise ValueError("Maxwell construction needs T < T_cr")
        r_sv, r_sl = self.spinodal(T)
        p_hi = self.p(r_sv, T)             # local maximum of the loop
        p_lo = max(self.p(r_sl, T), 0.0)   # local minimum (clipped at 0)
        R, a, b = self.R, self.a, self.b

        def area(ps):
            vl, vv = self._outer_roots(T, ps)
            integral = R * T * math.log((vv - b) / (vl - b)) + a / vv - a / vl
            return integral - ps * (vv - vl)

        eps = 1e-13 * p_hi
        ps = brentq(area, p_lo + eps, p_hi - eps, xtol=1e-16, rtol=1e-15, maxiter=500)
        vl, vv = self._outer_roots(T, ps)
        # polish the two densities on the exact EoS
        rho_l = brentq(lambda r: self.p(r, T) - ps, r_sl, (1.0 - 1e-14) / b, xtol=1e-15, rtol=1e-15)
        rho_v = brentq(lambda r: self.p(r, T) - ps, 1e-12, r_sv, xtol=1e-15, rtol=1e-15)
        return rho_v, rho_l, ps

    # ------------------------------------------------------------------
    # Planar interface of the interface energy kappa/2 |grad rho|^2 (eq. 18)
    # ------------------------------------------------------------------
    def free_energy(self, rho, T):
        """Helmholtz free energy per volume, up to terms linear in rho (which drop out of
        every quantity below): rho R T ln(rho/(1 - b rho)) - a rho^2."""
        return rho * self.R * T * np.log(rho / (1.0 - self.b * rho)) - self.a * rho * rho

    def chem_potential(self, rho, T):
        """mu = d f/d rho (same linear terms dropped); rho mu - f is the pressure."""
        return self.R * T * (np.log(rho / (1.0 - self.b * rho)) + 1.0 / (1.0 - self.b * rho)) - 2.0 * self.a * rho

    def grand_excess(self, rho, T, rho_v=None):
        """omega(rho) = f(rho) - f(rho_v) - mu_sat (rho - rho_v): the excess grand potential
        density against the coexisting bulk phases, zero at both coexistence densities."""
        if rho_v is None:
            rho_v = self.maxwell(T)[0]
        return (self.free_energy(rho, T) - self.free_energy(rho_v, T)
                - self.chem_potential(rho_v, T) * (rho - rho_v))

    def surface_tension(self, T, kappa):
        """Tension of the planar interface at T < T_cr: sigma = int_{rho_v}^{rho_l}
        sqrt(2 kappa omega(rho)) d rho (the equilibrium profile has kappa rho'^2 / 2 = omega)."""
        rv, rl, _ = self.maxwell(T)
        return quad(lambda r: math.sqrt(max(2.0 * kappa * float(self.grand_excess(r, T, rv)), 0.0)), rv, rl,
                    epsabs=0.0, epsrel=1e-12, limit=200)[0]

    def interface_width(self, T, kappa, lo=0.1, hi=0.9):
        """Distance between the points of the equilibrium profile at the fractions lo and hi
        of the density jump: x(rho) = int sqrt(kappa / (2 omega)) d rho."""
        rv, rl, _ = self.maxwell(T)
        a, b = rv + lo * (rl - rv), rv + hi * (rl - rv)
        return quad(lambda r: math.sqrt(kappa / (2.0 * float(self.grand_excess(r, T, rv)))), a, b,
                    epsabs=0.0, epsrel=1e-12, limit=200)[0]

    # ------------------------------------------------------------------
    # Rankine-Hugoniot (App. E)
    # ------------------------------------------------------------------
    def e_pv(self, p, v):
        """Internal energy as a function of (p, v): T from the EoS, then e = C_v T - a/v."""
        T = (p + self.a / v**2) * (v - self.b) / self.R
        return self.Cv * T - self.a / v

    def hugoniot_direct(self, rho0, p0, p1):
        """Post-shock state behind a shock into still fluid (u0 = 0) with pressure p1.
        Solves e(p1, v1) - e(p0, v0) = (p1 + p0)(v0 - v1)/2 for v1, then mass and
        momentum jumps give the shock speed s and the post-shock velocity u1."""
        v0 = 1.0 / rho0
        e0 = self.e_pv(p0, v0)
        f = lambda v1: self.e_pv(p1, v1) - e0 - 0.5 * (p1 + p0) * (v0 - v1)
        v1 = brentq(f, self.b * (1.0 + 1e-9), v0, xtol=1e-16, rtol=1e-15, maxiter=500)
        rho1 = 1.0 / v1
        m2 = (p1 - p0) / (v0 - v1)            # mass flux squared through the shock
        m = math.sqrt(m2)
        s = m * v0                            # shock speed (u0 = 0)
        u1 = s - m * v1
        T1 = self.T_of_p(rho1, p1)
        return dict(rho1=rho1, u1=u1, p1=p1, s=s, T1=T1, Ms=s / self.sound_vdw(rho0, self.T_of_p(rho0, p0)))

    def rh_closed_form(self, rho0, p0, rho1):
        """The closed form of App. E in reduced variables (rho1 as the free parameter).
        Returns (M0, u1, p1) in physical units.  The velocity line uses the pre-shock
        sound speed (see the design notes for this reading)."""
        rc, pc = self.rho_cr, self.p_cr
        scale = math.sqrt(pc / rc)            # sqrt(p_cr v_cr)
        r0, r1, P0, d = rho0 / rc, rho1 / rc, p0 / pc, self.delta
        c0 = self.sound_vdw(rho0, self.T_of_p(rho0, p0)) / scale
        M0 = (1.0 / c0) * math.sqrt(
            6.0 * r1 * (P0 * (1.0 + d) + r0 * r1 * (r0 + r1 + 3.0 * d - 3.0))
            / (r0 * (2.0 * r0 * (3.0 - r1) + 3.0 * d * (r0 - r1))))
        u1 = c0 * M0 * (r1 - r0) / r1
        P1 = P0 + c0 * c0 * M0 * M0 * r0 * (r1 - r0) / r1
        return M0, u1 * scale, P1 * pc

    def rh_jump_residual(self, rho0, p0, u0, rho1, p1, u1, s):
        """Residual of -s <M> + <N> = 0 for M = (rho, rho u, rho E), N = (rho u, p + rho u^2,
        rho u H), E = e + u^2/2, H = E + p/rho."""
        def MN(r, p, u):
            T = self.T_of_p(r, p)
            E = self.e(r, T) + 0.5 * u * u
            H = E + p / r
            return np.array([r, r * u, r * E]), np.array([r * u, p + r * u * u, r * u * H])
        M0_, N0_ = MN(rho0, p0, u0)
        M1_, N1_ = MN(rho1, p1, u1)
        return -s * (M1_ - M0_) + (N1_ - N0_)


# ----------------------------------------------------------------------
# Isothermal equations of state of the Supplement
# ----------------------------------------------------------------------
def maxwell_isotherm(p, dp, rho_lo, rho_hi, samples=4001):
    """(rho_vapor, rho_liquid, p_sat) of an isotherm p(rho) (derivative dp) with one
    loop inside (rho_lo, rho_hi): the loop's extrema from dp = 0, then the saturation
    pressure from the equal-area rule int_{v_l}^{v_v} p dv = p_sat (v_v - v_l), with
    the integral taken by adaptive quadrature in v."""
    r = np.linspace(rho_lo, rho_hi, samples)
    d = dp(r)
    neg = np.nonzero(d < 0.0)[0]
    if neg.size == 0:
        raise ValueError("isotherm without a loop")
    r_sv = brentq(dp, r[neg[0] - 1], r[neg[0]], xtol=1e-15, rtol=1e-15)       # local maximum
    r_sl = brentq(dp, r[neg[-1]], r[neg[-1] + 1], xtol=1e-15, rtol=1e-15)     # local minimum
    # pressures for which both outer branches have a root inside (rho_lo, rho_hi)
    p_hi = min(p(r_sv), p(rho_hi))
    p_lo = max(p(r_sl), p(rho_lo), 0.0)

    def roots(ps):
        rv = brentq(lambda x: p(x) - ps, rho_lo, r_sv, xtol=1e-15, rtol=1e-15, maxiter=500)
        rl = brentq(lambda x: p(x) - ps, r_sl, rho_hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        return rv, rl

    def area(ps):
        rv, rl = roots(ps)
        integral, _ = quad(lambda v: p(1.0 / v), 1.0 / rl, 1.0 / rv, epsabs=0.0, epsrel=2e-14, limit=200)
        return integral - ps * (1.0 / rv - 1.0 / rl)

    eps = 1e-12 * p_hi
    ps = brentq(area, p_lo + eps, p_hi - eps, xtol=1e-16, rtol=1e-15, maxiter=500)
    rv, rl = roots(ps)
    return rv, rl, ps


# Dieterici constants with the critical point of the van der Waals fluid above
# (rho_cr = 3.5, T_cr = 8/63): b = 1/(2 rho_cr), a = 4 R b T_cr
B_DIET = 1.0 / 7.0
A_DIET = 4.0 * R_SIM * B_DIET * 8.0 / 63.0


@dataclass(frozen=True)
class Dieterici:
    """p = rho R T/(1 - b rho) exp(-a rho/(R T)) (Supplement, coexistence curve), with the
    caloric relation of the Supplement's thermodynamics."""
    a: float = A_DIET
    b: float = B_DIET
    R: float = R_SIM
    delta: float = 1.0 / 3.0

    # critical values as printed (Supplement)
    @property
    def rho_cr(self) -> float:
        return 1.0 / (2.0 * self.b)

    @property
    def T_cr(self) -> float:
        return self.a / (4.0 * self.R * self.b)

    @property
    def p_cr(self) -> float:
        return self.a / (2.0 * math.e * self.b) ** 2

    def p(self, rho, T):
        return rho * self.R * T / (1.0 - self.b * rho) * np.exp(-self.a * rho / (self.R * T))

    def dp_drho_T(self, rho, T):
        return self.p(rho, T) * (1.0 / rho + self.b / (1.0 - self.b * rho) - self.a / (self.R * T))

    def maxwell(self, T):
        if not T < self.T_cr:
            raise ValueError("Maxwell construction needs T < T_cr")
        return maxwell_isotherm(lambda r: self.p(r, T), lambda r: self.dp_drho_T(r, T),
                                1e-9, (1.0 - 1e-12) / self.b)

    # caloric relation (Supplement, thermodynamics): de = C_v dT + [T (dp/dT)_v - p] dv with
    # the constant (ideal-gas) C_v = R/delta, integrated along the isotherm from v -> oo
    @property
    def Cv(self) -> float:
        return self.R / self.delta

    def dp_dT_rho(self, rho, T):
        return self.p(rho, T) / T * (1.0 + self.a * rho / (self.R * T))

    def _dep(self, rho, T, power):
        # int_0^rho [T dp/dT - p](r) / r^2 * (a r / (R T))^power dr; T dp/dT - p = p a r/(R T)
        def f(r):   # p x / r^2 = a exp(-x) / (1 - b r), x = a r / (R T)
            x = self.a * r / (self.R * T)
            return self.a * math.exp(-x) / (1.0 - self.b * r) * x ** power
        return quad(f, 0.0, float(rho), epsabs=0.0, epsrel=1e-13, limit=200)[0]

    def e(self, rho, T):
        return self.Cv * T - self._dep(rho, T, 0)

    def cv(self, rho, T):
        """(de/dT)_rho = C_v - int_0^rho T d^2p/dT^2 / r^2 dr, T d2p/dT2 = p x^2 / T."""
        return self.Cv - self._dep(rho, T, 1) / T

    def sound(self, rho, T):
        """Isentropic speed of sound (App. A): (dp/drho)_T + T (dp/dT)_rho^2 / (rho^2 c_v),
        with c_v = (de/dT)_rho of the state."""
        return math.sqrt(self.dp_drho_T(rho, T) + T / (rho * rho * self.cv(rho, T)) * self.dp_dT_rho(rho, T) ** 2)

    def T_isentrope(self, rho, rho0, T0):
        """T along the isentrope through (rho0, T0): T ds = de - p/rho^2 drho = 0 gives
        dT/drho = T (dp/dT)_rho / (rho^2 c_v), integrated from rho0 (accepts arrays)."""
        from scipy.integrate import solve_ivp
        rho = np.asarray(rho, dtype=np.float64)
        out = np.empty_like(rho)
        rhs = lambda r, T: [T[0] * self.dp_dT_rho(r, T[0]) / (r * r * self.cv(r, T[0]))]
        for side in (rho >= rho0, rho < rho0):
            if not np.any(side):
                continue
            end = rho[side].max() if rho[side].max() >= rho0 else rho[side].min()
            if end == rho0:
                out[side] = T0
                continue
            sol = solve_ivp(rhs, (rho0, float(end)), [T0], rtol=1e-12, atol=0.0, dense_output=True)
            out[side] = sol.sol(rho[side])[0]
        return out if out.ndim else float(out)


@dataclass(frozen=True)
class DoubleWell:
    """Simplified free energy near the critical point (Supplement), read with squares:
    E0 = beta (rho - rho_l)^2 (rho - rho_v)^2, p = p0 + rho dE0/drho - E0.  The
    background pressure p0 keeps the gauge temperature positive and changes no
    derivative of p."""
    beta: float
    rho_l: float
    rho_v: float
    p0: float

    def E0(self, rho):
        return self.beta * (rho - self.rho_l) ** 2 * (rho - self.rho_v) ** 2

    def dE0(self, rho):
        return 2.0 * self.beta * (rho - self.rho_l) * (rho - self.rho_v) * (2.0 * rho - self.rho_l - self.rho_v)

    def p(self, rho):
        return self.p0 + rho * self.dE0(rho) - self.E0(rho)

    def dp_drho(self, rho):
        # d/drho (rho E0' - E0) = rho E0''
        r, rl, rv = rho, self.rho_l, self.rho_v
        d2 = 2.0 * self.beta * ((r - rv) ** 2 + 4.0 * (r - rl) * (r - rv) + (r - rl) ** 2)
        return rho * d2

    def sound_saturated(self):
        """Sound speeds at the saturated densities as printed (Supplement):
        (rho_l - rho_v) sqrt(2 beta rho_l) and (rho_l - rho_v) sqrt(2 beta rho_v)."""
        d = self.rho_l - self.rho_v
        return d * math.sqrt(2.0 * self.beta * self.rho_l), d * math.sqrt(2.0 * self.beta * self.rho_v)

    def maxwell(self):
        return maxwell_isotherm(self.p, self.dp_drho, 0.5 * self.rho_v, self.rho_l + 2.0 * (self.rho_l - self.rho_v))

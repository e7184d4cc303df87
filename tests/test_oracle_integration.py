"""Integration pins of the oracle time step (Reyhanian, Dorschner & Karlin, arXiv:2002.09217).

* a uniform equilibrium state is a fixed point, also when it moves (main text,
  conclusion: Galilean invariance, error-free collision);
* with a uniform gauge (ideal gas at uniform T and u) one streaming pass and the
  collision conserve mass, momentum and energy exactly (eqs. 2-6);
* on periodic lattices the Korteweg force and the heat-flux correction are
  divergences and sum to zero (eqs. 9, 18);
* the ideal-gas limit (a = b = 0) reproduces the exact Riemann solution (main text);
* the shear viscosity is mu = (1/omega - 1/2) p dt (eq. 14);
* a van der Waals slab at T < T_cr relaxes to Maxwell's coexistence densities,
  independently of delta and of a uniform advection (main text, Fig. 2);
* a small isentropic pressure pulse travels at the adiabatic van der Waals sound speed
  of App. A, in the gas, the saturated vapour and liquid, and at the critical density
  above T_cr (main text, Fig. 1).
"""
import numpy as np
import pytest

from oracle import core, riemann
from oracle.thermo import VdW
from paper_2002_09217_amd import workloads as W
from tests.common import oracle_config, pulse_speed

VDW = VdW()


def rel_linf(a, b, floor=0.0):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), floor)


@pytest.mark.parametrize("state", [
    dict(rho=2.0, Tr=1.05, u=(0.1, -0.05)),      # supercritical
    dict(rho=1.2, Tr=0.9, u=(0.0, 0.0)),         # subcritical vapour-like single phase
    dict(rho=1.0, Tr=1.5, u=(1.0911, 0.0)),      # moving with 5 U_ch
])
def test_uniform_state_is_fixed_point(state):
    c = core.Config(dim=2, nx=5, ny=5, omega=1.5, kappa=0.0176, dt=0.2, n_pass=2)
    N = c.N
    s = core.Sim(c).init(np.full(N, state["rho"]), np.full(N, state["u"][0]),
                         np.full(N, state["Tr"] * VDW.T_cr), uy=np.full(N, state["u"][1]))
    m0 = s.moments()
    nsteps = 1000
    s.step(nsteps)
    m1 = s.moments()
    # every node sees the same rounding each step (the 16 interpolation weights do not sum
    # to exactly one), so the drift grows linearly: allow 4 ulp per step
    tol = nsteps * 4 * np.finfo(float).eps / 2
    for k in ("rho", "T", "p", "E"):
        assert rel_linf(m1[k], m0[k]) < tol, k
    for k in ("ux", "uy"):
        assert np.max(np.abs(m1[k] - m0[k])) < tol * max(1.0, abs(state["u"][0])), k


@pytest.mark.parametrize("dim", [1, 2])
def test_uniform_gauge_step_conserves_exactly(dim):
    """Ideal gas, uniform T and u, smooth density: the gauge theta = 3 R T and u are the
    same at every node, so streaming is a pure shift with weights summing to one and the
    collision conserves; one step with a single pass keeps the sums to round-off."""
    n = 24
    c = core.Config(dim=dim, nx=n, ny=n if dim == 2 else 1, a=0.0, b=0.0, delta=0.4, omega=1.5,
                    dt=0.5, n_pass=1)
    N = c.N
    x = np.arange(n)
    if dim == 2:
        X, Y = np.meshgrid(x, x)
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * X / n) * np.cos(4 * np.pi * Y / n)
    else:
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x / n)
    s = core.Sim(c).init(rho.ravel(), np.full(N, 0.13), np.full(N, 0.2), uy=np.full(N, -0.07))

    def sums(sim):
        v_all = []
        for node in range(N):
            lam = (sim.ux[node], sim.uy[node], sim.th[node])
            v_all.append(core.velocities(c, lam)[:, :dim])
        v_all = np.array(v_all)  # (N, Q, dim)
        mass = np.sum(sim.f)
        mom = np.einsum("qn,nqa->a", sim.f, v_all)
        energy = np.sum(sim.g)
        return mass, mom, energy

    m0, p0, e0 = sums(s)
    s.step(1)
    m1, p1, e1 = sums(s)
    assert abs(m1 - m0) / m0 < 1e-13
    assert np.max(np.abs(p1 - p0)) / m0 < 1e-13
    assert abs(e1 - e0) / e0 < 1e-13


def test_korteweg_force_and_heat_correction_sum_to_zero_on_periodic_lattice():
    n = 20
    c = core.Config(dim=2, nx=n, ny=n, kappa=0.0176, omega=1.5)
    rng = np.random.default_rng(7)
    x = np.arange(n)
    X, Y = np.meshgrid(x, x)
    rho = 3.0 + np.sin(2 * np.pi * X / n + 0.3) * np.cos(2 * np.pi * Y / n) + 0.1 * rng.normal(size=(n, n))
    Fx, Fy = core.korteweg_force(c, rho.ravel())
    scale = np.sum(np.abs(Fx)) + np.sum(np.abs(Fy))
    assert abs(np.sum(Fx)) / scale < 1e-14 and abs(np.sum(Fy)) / scale < 1e-14
    # the force is kappa rho grad(lap rho) in the continuum: check on a smooth long wave
    k = 2 * np.pi / n
    rho_s = 3.0 + 0.01 * np.sin(k * X)
    Fx_s, _ = core.korteweg_force(c, rho_s.ravel())
    # discrete lap of sin is -(2 - 2 cos k) sin; discrete grad of sin is sin(k) cos
    cont = c.kappa * rho_s * (0.01 * np.sin(k) * (-(2 - 2 * np.cos(k))) * np.cos(k * X))
    assert np.max(np.abs(Fx_s.reshape(n, n) - cont)) < 0.02 * np.max(np.abs(cont))
    T = 0.1 + 0.01 * rng.normal(size=n * n)
    h = 0.3 + 0.01 * rng.normal(size=n * n)
    mu = 0.05 + 0.01 * rng.uniform(size=n * n)
    kc = 0.2 + 0.01 * rng.uniform(size=n * n)
    M0 = core.heat_correction(c, T, h, mu, kc)
    assert abs(np.sum(M0)) / np.sum(np.abs(M0)) < 1e-14


def test_heat_correction_vanishes_for_ideal_gas():
    """For a = b = 0, h = C_p^ig T, so M0 = 2 div(mu grad(C_p^ig T - h)) = 0 with k = mu C_p^ig."""
    n = 16
    c = core.Config(dim=2, nx=n, ny=n, a=0.0, b=0.0, delta=0.4, omega=1.2)
    rng = np.random.default_rng(3)
    T = 0.1 + 0.02 * rng.uniform(size=n * n)
    rho = 1.0 + 0.1 * rng.uniform(size=n * n)
    p = rho * c.R * T
    e = c.R / c.delta * T
    h = e + p / rho
    mu = (1 / c.omega - 0.5) * p * c.dt
    kc = mu * c.R * (1 + c.delta) / c.delta
    M0 = core.heat_correction(c, T, h, mu, kc)
    assert np.max(np.abs(M0)) < 1e-16 * 100


def _sod(dt, N=1000, t_end=400.0, n_pass=2):
    c = core.Config(dim=1, nx=N, ny=1, a=0.0, b=0.0, R=1.0, delta=0.4, omega=1.0, kappa=0.0,
                    bc=((core.OUTFLOW, core.OUTFLOW), (0, 0)), n_pass=n_pass, dt=dt)
    x = np.arange(N) - (N / 2 - 0.5)
    sm = 0.5 * (1 - np.tanh(x / 1.0))   # jump smoothed over about one node
    rho = 0.125 + (1 - 0.125) * sm
    p = 0.01 + (0.1 - 0.01) * sm
    s = core.Sim(c).init(rho, np.zeros(N), p / rho)
    mass0 = np.sum(s.moments()["rho"])
    s.step(int(round(t_end / dt)))
    m = s.moments()
    ex = riemann.sample((1.0, 0.0, 0.1), (0.125, 0.0, 0.01), 1.0 + c.delta, x / t_end)
    return x, m, ex, np.sum(m["rho"]) - mass0


def test_ideal_gas_riemann_problem():
    """Sod's problem in lattice units, gamma = 1 + delta = 1.4.  The semi-Lagrangian step is
    not conservative at a shock; the mass defect and with it the shock-position error
    vanish as the time step shrinks (second order), so the test checks both the accuracy
    at dt = 1/4 and the convergence from dt = 1/2."""
    x, m, ex, dm = _sod(0.25)
    L1 = np.mean(np.abs(m["rho"] - ex[:, 0])) / np.mean(ex[:, 0])
    assert L1 < 0.005
    i_sh = np.nonzero(ex[:, 0] > 0.126)[0][-1]
    mid = 0.5 * (ex[i_sh, 0] + 0.125)
    shock_num = x[np.nonzero(m["rho"] > mid)[0][-1]]
    assert abs(shock_num - x[i_sh]) <= 3
    assert np.mean(np.abs(m["ux"] - ex[:, 1])) / np.max(ex[:, 1]) < 0.01
    assert np.mean(np.abs(m["p"] - ex[:, 2])) / np.mean(ex[:, 2]) < 0.005
    _, _, _, dm_half = _sod(0.5)
    assert abs(dm) < abs(dm_half) / 3.0


@pytest.mark.parametrize("U", [0.0, 0.3])
def test_shear_wave_viscosity(U):
    """A transverse wave u_y = A sin(k x) in a uniform ideal gas decays as exp(-(mu/rho) k^2 t),
    mu = (1/omega - 1/2) p dt, also on top of a uniform stream U along x."""
    n, ny, A = 64, 3, 1e-3
    c = core.Config(dim=2, nx=n, ny=ny, a=0.0, b=0.0, delta=0.4, omega=1.0, dt=1.0, n_pass=2)
    rho0, T0 = 1.0, 0.1
    X = np.tile(np.arange(n), ny)
    k = 2 * np.pi / n
    s = core.Sim(c).init(np.full(c.N, rho0), np.full(c.N, U), np.full(c.N, T0), uy=A * np.sin(k * X))

    def amp(sim):
        uy = sim.moments()["uy"].reshape(ny, n).mean(axis=0)
        return np.abs(np.fft.rfft(uy)[1]) * 2 / n

    a0 = amp(s)
    nsteps = 1000
    s.step(nsteps)
    nu = (1 / c.omega - 0.5) * rho0 * T0 * c.dt / rho0
    expect = np.exp(-nu * k * k * nsteps * c.dt)
    assert amp(s) / a0 == pytest.approx(expect, rel=0.02)


@pytest.mark.parametrize("k_scale", [1.0, 3.0])
def test_heat_conduction_rate(k_scale):
    """An isobaric temperature wave in an ideal gas decays as exp(-k k_w^2 t/(rho C_p)); with
    k = k_scale mu C_p^ig (eq. 9 with the free conductivity) the diffusivity is k_scale mu/rho."""
    n = 64
    c = core.Config(dim=1, nx=n, ny=1, a=0.0, b=0.0, delta=0.4, omega=1.0, dt=1.0, n_pass=2,
                    k_scale=k_scale)
    x = np.arange(n)
    kw = 2 * np.pi / n
    eps, T0, rho0 = 1e-3, 0.1, 1.0
    s = core.Sim(c).init(rho0 / (1 + eps * np.sin(kw * x)), np.zeros(n), T0 * (1 + eps * np.sin(kw * x)))

    def amp(sim):
        return np.abs(np.fft.rfft(sim.moments()["T"])[1]) * 2 / n

    a0 = amp(s)
    nsteps = 1000
    s.step(nsteps)
    rate = -np.log(amp(s) / a0) / (kw * kw * nsteps * c.dt)
    assert rate == pytest.approx(k_scale * (1 / c.omega - 0.5) * T0, rel=0.02)


def _slab(delta=1.0 / 3.0, U=0.0, N=100, steps=16000, kappa=0.0176, width=2.0):
    T0 = 0.9 * VDW.T_cr
    g = VdW(delta=delta)
    rv, rl, _ = g.maxwell(T0)
    c = core.Config(dim=1, nx=N, ny=1, omega=1.0, kappa=kappa, n_pass=2, dt=0.1, delta=delta)
    x = np.arange(N)
    prof = 0.5 * (np.tanh((x - N / 4) / width) - np.tanh((x - 3 * N / 4) / width))
    s = core.Sim(c).init(rv + (rl - rv) * prof, np.full(N, U), np.full(N, T0))
    s.step(steps)
    return g, s.moments()


def _bulk_error(g, m):
    """Relative deviation of the bulk vapour and liquid densities from Maxwell's rule at the
    measured mean temperature.  Bulk values are the medians of the lower and upper halves,
    which skip the small over- and undershoots next to each interface."""
    order = np.sort(m["rho"])
    n = order.size
    rv, rl, _ = g.maxwell(np.mean(m["T"]))
    return np.median(order[: n // 2]) / rv - 1.0, np.median(order[n // 2:]) / rl - 1.0


@pytest.mark.parametrize("delta", [1.0 / 3.0, 2.0 / 3.0])
def test_vdw_slab_relaxes_to_maxwell_coexistence(delta):
    ev, el = _bulk_error(*_slab(delta=delta))
    assert abs(ev) < 0.01 and abs(el) < 0.01


def test_advected_vdw_slab_converges_to_maxwell_coexistence():
    """The slab carried at U = 5 U_ch (Fig. 2): the interface moving through the lattice picks
    up interpolation error, which shrinks when the interface is resolved by twice as many
    nodes (kappa four times larger)."""
    coarse = _bulk_error(*_slab(U=1.0911, steps=8000))
    fine = _bulk_error(*_slab(U=1.0911, steps=8000, N=200, kappa=4 * 0.0176, width=4.0))
    assert max(abs(fine[0]), abs(fine[1])) < 0.015
    assert abs(fine[0]) < abs(coarse[0]) / 2


SOUND_STATES = [(1.75, 1.05), (1.490095732, 0.9), (5.800445742, 0.9), (3.5, 1.2)]


@pytest.mark.parametrize("rho0,Tr", SOUND_STATES)
def test_pulse_travels_at_the_vdw_sound_speed(rho0, Tr):
    def factory(rho, T, dt):
        c = core.Config(dim=1, nx=rho.size, ny=1, omega=1.5, kappa=0.0, dt=dt, n_pass=2)
        return core.Sim(c).init(rho, np.zeros(rho.size), T)

    c = pulse_speed(factory, rho0, Tr)
    assert c == pytest.approx(VDW.sound_vdw(rho0, Tr * VDW.T_cr), rel=3e-3)


def _wave_steepening(case, t1_steps):
    """Largest pressure jump between neighbours in each half of a shock tube at t1 and at
    2 t1, and where it sits.  The contact carries no pressure jump, so each half holds one
    wave: a shock keeps its steepness, a fan's steepness falls like 1/t."""
    sim = core.Sim(oracle_config(case))
    sim.init(case.rho, case.u[0], case.T)
    out = []
    n = case.n[0]
    for _ in range(2):
        sim.step(t1_steps)
        dp = np.abs(np.diff(sim.moments()["p"]))
        out.append((dp[: n // 2].max(), dp[n // 2:].max(), int(np.argmax(dp[: n // 2])),
                    n // 2 + int(np.argmax(dp[n // 2:]))))
    return out


def test_anomalous_shock_tube_has_a_rarefaction_shock_and_a_compression_fan():
    """Main text, Fig. 4: with delta = 0.0125 both states lie where Gamma < 0; the expansion
    running into the high-pressure side is a shock and the compression running into the
    low-pressure side is a fan.  The same states at delta = 1/3 give the classical pair."""
    case = W.reduced_shock_tube("anomalous", n=400, dt=0.2)
    (l1, r1, xl1, xr1), (l2, r2, xl2, xr2) = _wave_steepening(case, case.steps // 2)
    assert l2 / l1 > 0.85 and r2 / r1 < 0.75
    assert xl2 < xl1 < 200 < xr1 < xr2                 # rarefaction to the left, compression right
    classical = W.reduced_shock_tube("anomalous", n=400, dt=0.2, delta=1.0 / 3.0)
    (l1, r1, *_), (l2, r2, *_) = _wave_steepening(classical, classical.steps // 6)
    assert l2 / l1 < 0.75 and r2 / r1 > 0.85

"""Pins of the three-dimensional (D3Q27) oracle against what the paper and the
mathematics fix: the lattice and transfer algebra (App. B, C), the force source,
the force-extended g equilibrium and the heat-flux kernel with their moments
(eqs. 9, 16-22; App. F), exact local conservation of the collision, fixed points,
exact conservation with a uniform gauge, telescoping non-local terms (eq. 18), and
the van der Waals sound speed of a pulse (App. A; main text, Fig. 1).

Reyhanian, Dorschner & Karlin, arXiv:2002.09217."""
import numpy as np
import pytest

from oracle import core
from oracle.thermo import VdW
from tests.common import pulse_speed

T_L = 1.0 / 3.0
RNG = np.random.default_rng(27)
VDW = VdW()


def rand_gauge():
    return np.array([*RNG.uniform(-0.4, 0.4, 3), RNG.uniform(0.05, 0.4)])


def moments27(f, v):
    """All moments sum_i f_i vx^l vy^m vz^n with l, m, n <= 2 (App. C)."""
    return np.array([np.sum(f * v[:, 0] ** l * v[:, 1] ** m * v[:, 2] ** n)
                     for l in range(3) for m in range(3) for n in range(3)])


def test_weights_and_maxwellian_moments():
    W = core.weights3()
    c = core.velocities3(np.array([0.0, 0.0, 0.0, 1.0]))
    assert np.sum(W) == pytest.approx(1.0, rel=1e-15)
    assert np.allclose(W @ c, 0.0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", W, c, c), T_L * np.eye(3), atol=1e-15)
    # rho W in the gauge (u, theta) has the moments of a Maxwellian: rho u, rho (u u + theta T_L I)
    for _ in range(5):
        lam, rho = rand_gauge(), RNG.uniform(0.5, 6.0)
        v = core.velocities3(lam)
        assert np.allclose(rho * W @ v, rho * lam[:3], rtol=1e-13)
        P = np.einsum("i,ia,ib->ab", rho * W, v, v)
        assert np.allclose(P, rho * (np.outer(lam[:3], lam[:3]) + lam[3] * T_L * np.eye(3)), rtol=1e-12)


def test_transfer_equals_full_27x27_moment_matrix_solve():
    """G = M_to^{-1} M_from with the 27 x 27 moment matrices, solved by the library."""
    for _ in range(10):
        lf, lt = rand_gauge(), rand_gauge()
        vf, vt = core.velocities3(lf), core.velocities3(lt)
        exps = [(l, m, n) for l in range(3) for m in range(3) for n in range(3)]
        Mf = np.array([[v[0] ** l * v[1] ** m * v[2] ** n for v in vf] for (l, m, n) in exps])
        Mt = np.array([[v[0] ** l * v[1] ** m * v[2] ** n for v in vt] for (l, m, n) in exps])
        G = np.linalg.solve(Mt, Mf)
        f = RNG.uniform(0.0, 1.0, 27)
        assert np.allclose(core.transfer3_pop(lf, lt, f), G @ f, rtol=1e-9, atol=1e-11)


def test_transfer_preserves_moments_identity_and_composition():
    for _ in range(10):
        la, lb, lc = rand_gauge(), rand_gauge(), rand_gauge()
        f = RNG.uniform(0.0, 1.0, 27)
        fb = core.transfer3_pop(la, lb, f)
        assert np.allclose(moments27(fb, core.velocities3(lb)), moments27(f, core.velocities3(la)),
                           rtol=1e-10, atol=1e-12)
        assert np.allclose(core.transfer3_pop(la, la, f), f, rtol=1e-13, atol=1e-15)
        assert np.allclose(core.transfer3_pop(lb, lc, fb), core.transfer3_pop(la, lc, f), rtol=1e-9, atol=1e-12)


def test_force_source_moments():
    W = core.weights3()
    for _ in range(10):
        lam, rho = rand_gauge(), RNG.uniform(0.5, 6.0)
        du = RNG.uniform(-0.05, 0.05, 3)
        S = core.force_source3(rho, lam[:3], lam[3], du)
        v = core.velocities3(lam)
        assert abs(np.sum(S)) < 1e-13
        assert np.allclose(S @ v, rho * du, rtol=1e-10, atol=1e-14)
        u, up = lam[:3], lam[:3] + du
        assert np.allclose(np.einsum("i,ia,ib->ab", S, v, v), rho * (np.outer(up, up) - np.outer(u, u)),
                           rtol=1e-9, atol=1e-13)
        # S is zero without force
        assert np.allclose(core.force_source3(rho, lam[:3], lam[3], np.zeros(3)), 0.0, atol=1e-14)
        assert np.all(np.isfinite(W))


@pytest.mark.parametrize("dt", [1.0, 0.2])
def test_force_extended_geq_moments(dt):
    c = core.Config3(dt=dt)
    for _ in range(10):
        lam, rho = rand_gauge(), RNG.uniform(0.5, 6.0)
        F = RNG.uniform(-0.05, 0.05, 3)
        u, p, E = lam[:3], rho * lam[3] * T_L, RNG.uniform(0.1, 0.6)
        uh = u + F * dt / (2 * rho)
        H = E + p / rho
        g = core.geq3(c, rho, u, lam[3], p, E, uh, F)
        v = core.velocities3(lam)
        assert np.sum(g) == pytest.approx(2 * rho * E, rel=1e-13)
        assert np.allclose(g @ v, 2 * rho * uh * H, rtol=1e-11, atol=1e-13)
        expect = 2 * rho * np.outer(uh, uh) * (H + p / rho) + 2 * p * H * np.eye(3)
        assert np.allclose(np.einsum("i,ia,ib->ab", g, v, v), expect, rtol=1e-11, atol=1e-13)
        # without force it is eq. 8 with D = 3: rho W [2 e - 3 p/rho + v^2]
        g0 = core.geq3(c, rho, u, lam[3], p, E, u, np.zeros(3))
        e = E - 0.5 * np.dot(u, u)
        assert np.allclose(g0, rho * core.weights3() * (2 * e - 3 * p / rho + np.sum(v * v, axis=1)),
                           rtol=1e-12, atol=1e-13)


def test_heat_flux_kernel_moments():
    for _ in range(10):
        lam, rho = rand_gauge(), RNG.uniform(0.5, 6.0)
        p = rho * lam[3] * T_L
        psi = core.psi3(rho, lam[:3], lam[3], p)
        v = core.velocities3(lam)
        assert np.sum(psi) == pytest.approx(1.0, rel=1e-13)
        assert np.allclose(psi @ v, 0.0, atol=1e-13)
        assert np.allclose(np.einsum("i,ia,ib->ab", psi, v, v), 0.0, atol=1e-13)


def test_collision_local_conservation():
    c = core.Config3(omega=1.5, dt=0.2)
    W = core.weights3()
    for _ in range(10):
        lam = rand_gauge()
        lam[3] = RNG.uniform(0.05, 0.25)
        rho = RNG.uniform(1.0, 3.0)
        fstr = rho * W * (1 + 0.05 * RNG.normal(size=27))
        gstr = rho * W * (0.8 + 0.05 * RNG.normal(size=27))
        F = RNG.uniform(-0.02, 0.02, 3)
        M0 = RNG.uniform(-0.01, 0.01)
        fo, go, lo = core.collide3(c, lam, fstr, gstr, F, M0)
        vs, vo = core.velocities3(lam), core.velocities3(lo)
        rho_s = np.sum(fstr)
        assert np.sum(fo) == pytest.approx(rho_s, rel=1e-14)
        j_s = fstr @ vs
        assert np.allclose(fo @ vo, j_s + F * c.dt, rtol=1e-12, atol=1e-14)
        u_col = j_s / rho_s
        uh = u_col + F * c.dt / (2 * rho_s)
        assert np.sum(go) == pytest.approx(np.sum(gstr) + (M0 + 2 * np.dot(uh, F)) * c.dt, rel=1e-13)
        assert np.allclose(lo[:3], u_col, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("state", [dict(rho=2.0, Tr=1.05, u=(0.1, -0.05, 0.07)),
                                   dict(rho=1.0, Tr=1.5, u=(0.6, 0.3, -0.4))])
def test_uniform_state_is_fixed_point(state):
    c = core.Config3(nx=4, ny=3, nz=5, omega=1.5, kappa=0.0176, dt=0.2, n_pass=2)
    N = c.N
    s = core.Sim3(c).init(np.full(N, state["rho"]), np.repeat(np.array(state["u"])[:, None], N, axis=1),
                          np.full(N, state["Tr"] * VDW.T_cr))
    m0 = s.moments()
    s.step(100)
    m1 = s.moments()
    tol = 100 * 4 * np.finfo(float).eps
    for k in ("rho", "T", "p", "E"):
        assert np.max(np.abs(m1[k] - m0[k])) < tol * np.max(np.abs(m0[k])), k
    for k in ("ux", "uy", "uz"):
        assert np.max(np.abs(m1[k] - m0[k])) < tol, k


def test_uniform_gauge_step_conserves_exactly():
    """Ideal gas, uniform T and u, smooth density: the gauge is uniform, streaming is a
    shift with weights summing to one, the collision conserves: the sums of rho, rho u
    and g are kept to round-off by one single-pass step."""
    n = 10
    c = core.Config3(nx=n, ny=n, nz=n, a=0.0, b=0.0, delta=0.4, omega=1.5, dt=0.5, n_pass=1)
    N = c.N
    x, y, z = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    rho = (1.0 + 0.1 * np.sin(2 * np.pi * x / n) * np.cos(2 * np.pi * (y + 2 * z) / n)).T.ravel()
    u = np.array([0.13, -0.07, 0.05])
    s = core.Sim3(c).init(rho, np.repeat(u[:, None], N, axis=1), np.full(N, 0.4))
    vel = lambda s_: np.stack([core.velocities3(np.array([*s_.u[:, i], s_.th[i]])) for i in range(N)])
    m_before = np.sum(s.f), np.einsum("qn,nqa->a", s.f, vel(s)), np.sum(s.g)
    s.step(1)
    m_after = np.sum(s.f), np.einsum("qn,nqa->a", s.f, vel(s)), np.sum(s.g)
    assert m_after[0] == pytest.approx(m_before[0], rel=1e-13)
    assert np.allclose(m_after[1], m_before[1], rtol=1e-12, atol=1e-12)
    assert m_after[2] == pytest.approx(m_before[2], rel=1e-13)


def test_korteweg_force_and_heat_correction_sum_to_zero():
    c = core.Config3(nx=7, ny=6, nz=5, kappa=0.05)
    N = c.N
    rho = RNG.uniform(1.0, 5.0, N)
    F = core.korteweg_force3(c, rho)
    assert np.allclose(F.sum(axis=1), 0.0, atol=1e-12 * np.abs(F).sum())
    T, h, mu, kc = (RNG.uniform(0.5, 1.5, N) for _ in range(4))
    M0 = core.heat_correction3(c, T, h, mu, kc)
    assert abs(M0.sum()) < 1e-12 * np.abs(M0).sum()
    # a density varying along x only gives the one-dimensional force of the same profile
    n = 16
    c1 = core.Config3(nx=n, ny=3, nz=2, kappa=0.05)
    prof = 2.0 + np.sin(2 * np.pi * np.arange(n) / n)
    F1 = core.korteweg_force3(c1, np.tile(prof, 6))
    # continuum: F_x = kappa rho d3 rho/dx3; the lattice stencil converges to it
    k = 2 * np.pi / n
    exact = 0.05 * prof * (-(k ** 3) * np.cos(2 * np.pi * np.arange(n) / n))
    assert np.max(np.abs(F1[0, :n] - exact)) < 0.1 * np.max(np.abs(exact))
    assert np.allclose(F1[1:], 0.0, atol=1e-15)


@pytest.mark.parametrize("rho0,Tr", [(5.800445742, 0.9)])
def test_plane_pulse_travels_at_the_vdw_sound_speed(rho0, Tr):
    """A pulse varying along x only, on a 300 x 1 x 1 periodic box (saturated liquid at
    0.9 T_cr; the GPU tests cover the vapour and the other temperatures)."""
    def factory(rho, T, dt):
        c = core.Config3(nx=rho.size, ny=1, nz=1, omega=1.5, kappa=0.0, dt=dt, n_pass=2)
        sim = core.Sim3(c).init(rho, np.zeros((3, rho.size)), T)
        return sim

    c = pulse_speed(factory, rho0, Tr, n=300, sigma=6.0, dt=0.25, times=(40.0, 100.0))
    assert c == pytest.approx(VDW.sound_vdw(rho0, Tr * VDW.T_cr), rel=3e-3)

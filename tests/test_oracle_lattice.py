"""Pins of the oracle's lattice algebra: equilibria, transfer matrix, reconstruction,
force source, force-extended g equilibrium, heat-flux kernel, local conservation.

Reyhanian, Dorschner & Karlin, arXiv:2002.09217: eq. 1 and App. B (velocities and
weights), App. C (transfer matrix), App. D (reconstruction), eqs. 16-22 and App. F
(forcing, force-extended g equilibrium and its moments), eq. 9 and App. F (g~)."""
import itertools

import numpy as np
import pytest

from oracle import core

T_L = 1.0 / 3.0
RNG = np.random.default_rng(20020921)


def cfg(dim):
    return core.Config(dim=dim, nx=4, ny=4 if dim == 2 else 1)


def vel(dim, lam):
    return core.velocities(cfg(dim), lam)[:, :dim]


def moments9(f, v):
    """All moments sum_i f_i vx^m vy^n with m, n <= 2 (App. C), in absolute velocities."""
    return np.array([[np.sum(f * v[:, 0] ** m * v[:, 1] ** n) for n in range(3)] for m in range(3)])


def moments3(f, v):
    return np.array([np.sum(f * v[:, 0] ** m) for m in range(3)])


def rand_gauge():
    return np.array([RNG.uniform(-0.4, 0.4), RNG.uniform(-0.4, 0.4), RNG.uniform(0.05, 0.4)])


# ---------------------------------------------------------------------------
# equilibrium (App. B)
# ---------------------------------------------------------------------------
def test_feq_moments_are_maxwellian():
    W = core.weights(cfg(2))
    for _ in range(20):
        lam, rho = rand_gauge(), RNG.uniform(0.5, 6)
        v = vel(2, lam)
        M = moments9(rho * W, v)
        P = lam[2] * T_L
        ux, uy = lam[0], lam[1]
        gauss = lambda u, k: [1.0, u, u * u + P][k]  # 1D Gaussian moments up to order 2
        for m, n in itertools.product(range(3), range(3)):
            assert M[m, n] == pytest.approx(rho * gauss(ux, m) * gauss(uy, n), rel=1e-13, abs=1e-14)
    # fourth-order diagonal moment per axis is also Maxwellian (3 P^2 about the mean)
    lam = np.array([0.0, 0.0, 0.3])
    v = vel(2, lam)
    assert np.sum(W * v[:, 0] ** 4) == pytest.approx(3 * (0.3 * T_L) ** 2, rel=1e-14)


# ---------------------------------------------------------------------------
# transfer matrix (App. C)
# ---------------------------------------------------------------------------
def vandermonde(lam_u, theta):
    v = lam_u + np.sqrt(theta) * np.array([-1.0, 0.0, 1.0])
    return np.vstack([np.ones(3), v, v * v])


def test_transfer_1d_equals_library_solve():
    for _ in range(50):
        a, b = rand_gauge(), rand_gauge()
        G = core.transfer_1d(a[0], a[2], b[0], b[2])
        ref = np.linalg.solve(vandermonde(b[0], b[2]), vandermonde(a[0], a[2]))
        assert np.allclose(G, ref, rtol=1e-12, atol=1e-12)


def test_transfer_2d_equals_full_9x9_moment_matrix_solve():
    c = cfg(2)
    for _ in range(30):
        a, b = rand_gauge(), rand_gauge()
        va, vb = vel(2, a), vel(2, b)
        # the 9x9 moment matrix of App. C, rows (m, n), columns populations
        Ma = np.array([[va[i, 0] ** m * va[i, 1] ** n for i in range(9)] for m in range(3) for n in range(3)])
        Mb = np.array([[vb[i, 0] ** m * vb[i, 1] ** n for i in range(9)] for m in range(3) for n in range(3)])
        f = RNG.uniform(0.1, 1.0, 9)
        ref = np.linalg.solve(Mb, Ma @ f)
        assert np.allclose(core.transfer_pop(c, a, b, f), ref, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("dim", [1, 2])
def test_transfer_preserves_moments_identity_and_composition(dim):
    c = cfg(dim)
    Q = c.Q
    for _ in range(30):
        a, b, d = rand_gauge(), rand_gauge(), rand_gauge()
        if dim == 1:
            a[1] = b[1] = d[1] = 0.0
        f = RNG.uniform(-0.5, 1.0, Q)
        fb = core.transfer_pop(c, a, b, f)
        if dim == 2:
            assert np.allclose(moments9(fb, vel(2, b)), moments9(f, vel(2, a)), rtol=1e-12, atol=1e-13)
        else:
            assert np.allclose(moments3(fb, vel(1, b)), moments3(f, vel(1, a)), rtol=1e-12, atol=1e-13)
        assert np.array_equal(core.transfer_pop(c, a, a, f), f) or np.allclose(core.transfer_pop(c, a, a, f), f, rtol=1e-15, atol=1e-16)
        two_step = core.transfer_pop(c, b, d, fb)
        assert np.allclose(two_step, core.transfer_pop(c, a, d, f), rtol=1e-11, atol=1e-12)


def _printed_axis(u_to, th_to, u_from, th_from):
    """The explicit one-axis factors as printed in App. C:
    g(i,k) = A(i)^2 - B(i,k), A(i) = (u' - u)/sqrt3 - i sqrt(p/rho),
    B(i,0) = p'/rho', B(i,k) = k sqrt(p'/rho') A(i); w(0) = 1/(p'/rho'), w(k) = -1/(2 p'/rho').
    Primed quantities belong to the target gauge; p/rho = theta T_L."""
    Pt, Pf = th_to * T_L, th_from * T_L
    out = np.zeros((3, 3))
    for k in (-1, 0, 1):
        w = 1.0 / Pt if k == 0 else -1.0 / (2.0 * Pt)
        for i in (-1, 0, 1):
            A = (u_to - u_from) / np.sqrt(3.0) - i * np.sqrt(Pf)
            B = Pt if k == 0 else k * np.sqrt(Pt) * A
            out[k + 1, i + 1] = w * (A * A - B)
    return out


def test_printed_explicit_transfer_form():
    """The printed explicit form (App. C) equals the definition for two axes (the
    product of two axis factors), while one axis factor alone carries the opposite sign."""
    c = cfg(2)
    for _ in range(20):
        a, b = rand_gauge(), rand_gauge()
        Gx = _printed_axis(b[0], b[2], a[0], a[2])
        Gy = _printed_axis(b[1], b[2], a[1], a[2])
        f = RNG.uniform(0.1, 1.0, 9)
        printed = np.einsum("ki,lj,ij->kl", Gx, Gy, f.reshape(3, 3)).ravel()
        assert np.allclose(printed, core.transfer_pop(c, a, b, f), rtol=1e-11, atol=1e-12)
        assert np.allclose(Gx, -core.transfer_1d(a[0], a[2], b[0], b[2]), rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------------------
# reconstruction (App. D)
# ---------------------------------------------------------------------------
def test_lagrange_weights():
    nodes = np.arange(4.0)
    for t in RNG.uniform(1.0, 2.0, 50):
        w = core.lagrange4(t)
        assert np.sum(w) == pytest.approx(1.0, abs=1e-15)
        for _ in range(3):
            coef = RNG.normal(size=4)
            poly = np.polyval(coef, nodes)
            assert np.dot(w, poly) == pytest.approx(np.polyval(coef, t), rel=1e-12, abs=1e-12)
        # agrees with the library's interpolating polynomial through the four nodes
        vals = RNG.normal(size=4)
        assert np.dot(w, vals) == pytest.approx(np.polyval(np.polyfit(nodes, vals, 3), t), rel=1e-10, abs=1e-12)
    for n in range(4):
        assert np.allclose(core.lagrange4(float(n)), np.eye(4)[n], atol=0)


# ---------------------------------------------------------------------------
# forcing (eqs. 16-17 and App. F)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [1, 2])
def test_force_source_moments_and_closed_form(dim):
    c = cfg(dim)
    W = core.weights(c)
    for _ in range(20):
        lam, rho = rand_gauge(), RNG.uniform(0.5, 6.0)
        du = RNG.uniform(-0.05, 0.05, 2)
        if dim == 1:
            lam[1] = du[1] = 0.0
        S = core.force_source(c, rho, lam[:2], lam[2], du)
        v = vel(dim, lam)
        assert abs(np.sum(S)) < 1e-13
        for a in range(dim):
            assert np.sum(S * v[:, a]) == pytest.approx(rho * du[a], rel=1e-11, abs=1e-14)
            for b in range(dim):
                u, up = lam[:2], lam[:2] + du
                expect = rho * (up[a] * up[b] - u[a] * u[b])
                assert np.sum(S * v[:, a] * v[:, b]) == pytest.approx(expect, rel=1e-10, abs=1e-13)
        # per-axis closed form: S_0 = -rho du^2/theta, S_pm = rho (du^2/(2 theta) pm du/(2 sqrt theta)),
        # combined as the product of the two axis factors of rho W + S
        th = lam[2]
        phi = lambda d: np.array([1 / 6 + d * d / (2 * th) - d / (2 * np.sqrt(th)),
                                  2 / 3 - d * d / th,
                                  1 / 6 + d * d / (2 * th) + d / (2 * np.sqrt(th))])
        closed = rho * (np.outer(phi(du[0]), phi(du[1])).ravel() if dim == 2 else phi(du[0])) - rho * W
        assert np.allclose(S, closed, rtol=1e-10, atol=1e-13)


def test_modified_source_moments_of_appendix_F():
    """App. F: S^ = S - omega (f^eq(rho, u_hat) - rho W) has zero mass, momentum
    dt (1 - omega/2) F and second moment dt (1 - omega/2)(u_hat F + F u_hat) + omega dt^2 F F/(4 rho)."""
    c = cfg(2)
    for omega in (1.0, 1.5):
        for dt in (1.0, 0.2):
            lam, rho = rand_gauge(), RNG.uniform(0.5, 6.0)
            F = RNG.uniform(-0.05, 0.05, 2)
            u = lam[:2]
            S = core.force_source(c, rho, u, lam[2], F * dt / rho)
            uh = u + F * dt / (2 * rho)
            feq_uh = core.force_source(c, rho, u, lam[2], uh - u) + rho * core.weights(c)
            Sh = S - omega * (feq_uh - rho * core.weights(c))
            v = vel(2, lam)
            assert abs(np.sum(Sh)) < 1e-13
            for a in range(2):
                assert np.sum(Sh * v[:, a]) == pytest.approx(dt * (1 - omega / 2) * F[a], rel=1e-9, abs=1e-14)
                for b in range(2):
                    expect = dt * (1 - omega / 2) * (uh[a] * F[b] + F[a] * uh[b]) + omega * dt * dt * F[a] * F[b] / (4 * rho)
                    assert np.sum(Sh * v[:, a] * v[:, b]) == pytest.approx(expect, rel=1e-8, abs=1e-14)


# ---------------------------------------------------------------------------
# g equilibrium (eqs. 8, 20-22 and App. F) and heat-flux kernel (eq. 9)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [1, 2])
def test_force_extended_geq_moments(dim):
    c = core.Config(dim=dim, nx=4, ny=4 if dim == 2 else 1)
    for dt in (1.0, 0.2):
        c.dt = dt
        for _ in range(15):
            lam, rho = rand_gauge(), RNG.uniform(0.5, 6.0)
            F = RNG.uniform(-0.05, 0.05, 2)
            if dim == 1:
                lam[1] = F[1] = 0.0
            u = lam[:2]
            p = rho * lam[2] * T_L
            E = RNG.uniform(0.1, 0.6)
            uh = u + F * dt / (2 * rho)
            H = E + p / rho
            g = core.geq(c, rho, u, lam[2], p, E, uh, F)
            v = vel(dim, lam)
            assert np.sum(g) == pytest.approx(2 * rho * E, rel=1e-13)
            for a in range(dim):
                assert np.sum(g * v[:, a]) == pytest.approx(2 * rho * uh[a] * H, rel=1e-11, abs=1e-13)
                for b in range(dim):
                    expect = 2 * rho * uh[a] * uh[b] * (H + p / rho) + (2 * p * H if a == b else 0.0)
                    assert np.sum(g * v[:, a] * v[:, b]) == pytest.approx(expect, rel=1e-11, abs=1e-13)
            # without force it is eq. 8: rho W [2 e - D p/rho + v^2]
            g0 = core.geq(c, rho, u, lam[2], p, E, u, np.zeros(2))
            e = E - 0.5 * np.dot(u, u)
            eq8 = rho * core.weights(c) * (2 * e - dim * p / rho + np.sum(v * v, axis=1))
            assert np.allclose(g0, eq8, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("dim", [1, 2])
def test_heat_flux_kernel_moments(dim):
    c = cfg(dim)
    for _ in range(20):
        lam, rho = rand_gauge(), RNG.uniform(0.5, 6.0)
        if dim == 1:
            lam[1] = 0.0
        p = rho * lam[2] * T_L
        psi = core.psi(c, rho, lam[:2], lam[2], p)
        v = vel(dim, lam)
        assert np.sum(psi) == pytest.approx(1.0, rel=1e-13)
        for a in range(dim):
            assert abs(np.sum(psi * v[:, a])) < 1e-13
            for b in range(dim):
                assert abs(np.sum(psi * v[:, a] * v[:, b])) < 1e-13


@pytest.mark.parametrize("dim", [1, 2])
def test_collision_local_conservation(dim):
    """The collision changes (rho, rho u, 2 rho E) by exactly (0, F dt, (M0 + 2 u_hat.F) dt)
    and conserves them exactly without force and correction (eqs. 16, 19)."""
    c = core.Config(dim=dim, nx=4, ny=4 if dim == 2 else 1, omega=1.5, dt=0.2)
    for _ in range(20):
        lam = rand_gauge()
        lam[2] = RNG.uniform(0.05, 0.25)
        if dim == 1:
            lam[1] = 0.0
        rho = RNG.uniform(1.0, 3.0)
        W = core.weights(c)
        fstr = rho * W * (1 + 0.05 * RNG.normal(size=c.Q))
        gstr = rho * W * (0.8 + 0.05 * RNG.normal(size=c.Q))
        F = RNG.uniform(-0.02, 0.02, 2)
        M0 = RNG.uniform(-0.01, 0.01)
        if dim == 1:
            F[1] = 0.0
        fo, go, lo = core.collide(c, lam, fstr, gstr, F, M0)
        vs, vo = vel(dim, lam), vel(dim, lo)
        rho_s = np.sum(fstr)
        assert np.sum(fo) == pytest.approx(rho_s, rel=1e-14)
        j_s = fstr @ vs
        j_o = fo @ vo
        assert np.allclose(j_o, j_s + F[:dim] * c.dt, rtol=1e-12, atol=1e-14)
        u_col = j_s / rho_s
        uh = u_col + F[:dim] * c.dt / (2 * rho_s)
        assert np.sum(go) == pytest.approx(np.sum(gstr) + (M0 + 2 * np.dot(uh, F[:dim])) * c.dt, rel=1e-13)
        # the new gauge velocity is the streamed velocity u = j/rho (eq. 2 and App. F)
        assert np.allclose(lo[:dim], u_col, rtol=1e-13, atol=1e-15)

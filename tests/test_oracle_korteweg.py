"""Pins of the oracle's Korteweg force against the continuum, in 2D and 3D.

The Korteweg stress of eq. 18, K = -kappa (rho lap rho + |grad rho|^2 / 2) I +
kappa grad rho (x) grad rho, has the divergence -div K = kappa rho grad(lap rho) (vector
calculus: div(grad rho (x) grad rho) = lap rho grad rho + grad |grad rho|^2 / 2), and the
force of App. F is F = -div K.  On smooth periodic fields made of oblique Fourier modes,
every component of grad rho is nonzero, so the off-diagonal stress enters the force.  The
oracle's lattice stencils must converge to the continuum force at second order in the grid
spacing: a wrong sign or factor in any stress component (diagonal or off-diagonal), or a
transposed index, leaves an O(1) error that does not shrink under refinement.
"""
import numpy as np
import pytest

from oracle import core

KAPPA = 0.0176


def modes_field(n, modes, dim):
    """rho = 2 + sum a sin(k.x + phase) on an n^dim periodic lattice (x fastest), and the
    continuum force kappa rho grad(lap rho) of it, shape (dim, N)."""
    axes = np.meshgrid(*([np.arange(n, dtype=float)] * dim), indexing="ij")[::-1]  # x, y(, z)
    rho = np.full(axes[0].shape, 2.0)
    glap = [np.zeros_like(rho) for _ in range(dim)]
    for m, a, phase in modes:
        k = 2.0 * np.pi * np.asarray(m, dtype=float) / n
        arg = sum(k[d] * axes[d] for d in range(dim)) + phase
        rho += a * np.sin(arg)
        for d in range(dim):
            glap[d] -= a * (k @ k) * k[d] * np.cos(arg)   # grad(lap) of the mode
    force = np.stack([KAPPA * rho * g for g in glap]).reshape(dim, -1)
    return rho.ravel(), force


def rel_err(F, exact):
    return np.max(np.abs(F - exact)) / np.max(np.abs(exact))


MODES2 = [((1, 2), 0.3, 0.4), ((2, -1), 0.2, 1.1), ((0, 1), 0.1, 2.0)]
MODES3 = [((1, 2, 1), 0.3, 0.4), ((2, -1, 1), 0.2, 1.1), ((1, 0, -2), 0.1, 2.0)]


def test_force_2d_converges_to_the_continuum_at_second_order():
    errs = []
    for n in (32, 64, 128):
        c = core.Config(dim=2, nx=n, ny=n, kappa=KAPPA)
        rho, exact = modes_field(n, MODES2, 2)
        Fx, Fy = core.korteweg_force(c, rho)
        errs.append(rel_err(np.stack([Fx, Fy]), exact))
    assert errs[-1] < 4e-3, errs
    for coarse, fine in zip(errs, errs[1:]):
        assert 3.6 < coarse / fine < 4.4, errs


def test_force_3d_converges_to_the_continuum_at_second_order():
    errs = []
    for n in (12, 24, 48):
        c = core.Config3(nx=n, ny=n, nz=n, kappa=KAPPA)
        rho, exact = modes_field(n, MODES3, 3)
        errs.append(rel_err(core.korteweg_force3(c, rho), exact))
    assert errs[-1] < 0.03, errs
    assert 3.2 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4, errs


def test_force_2d_on_a_rectangular_lattice_and_each_axis():
    """Distinct extents (nx != ny) and a field varying along y only: the y force is the
    one-dimensional continuum force, the x force vanishes (catches swapped axes)."""
    nx, ny = 24, 96
    c = core.Config(dim=2, nx=nx, ny=ny, kappa=KAPPA)
    y = np.repeat(np.arange(ny, dtype=float), nx)
    k = 2.0 * np.pi / ny
    rho = 2.0 + 0.3 * np.sin(k * y)
    Fx, Fy = core.korteweg_force(c, rho)
    exact = KAPPA * rho * (-0.3 * k ** 3 * np.cos(k * y))
    assert np.max(np.abs(Fx)) < 1e-15
    assert rel_err(Fy, exact) < 3e-3

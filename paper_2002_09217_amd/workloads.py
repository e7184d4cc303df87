"""Seeded synthetic inputs shaped like the paper's cases (Reyhanian, Dorschner &
Karlin, arXiv:2002.09217): macroscopic fields (rho, u, T) and run parameters.

This module holds geometry and random numbers only, none of the method's arithmetic.
The van der Waals constants it needs (coexistence densities, post-shock state) are
read from data/vdw_constants.json, which oracle/write_constants.py writes from the
oracle's Maxwell and Rankine-Hugoniot routines.  Both the oracle and the HIP path
take their inputs from here.

Shared choices (the paper gives no grid sizes, time step, omega or kappa):
  a = 2/49, b = 2/21, R = 1 (main text), delta = 1/3, two streaming passes,
  dt = 0.2 for the shock cases and 0.1 for the droplets (DT_DROPLET), omega = 1.0 for
  the shock cases and 1.5 for the droplets, kappa = 0.0176 for droplets (a 10-90 %
  interface width of about 4.4 nodes at T/T_cr = 0.9).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

_DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "vdw_constants.json")
with open(_DATA) as _fh:
    CONST = json.load(_fh)

A, B, R = CONST["a"], CONST["b"], CONST["R"]
RHO_CR, T_CR, P_CR = CONST["rho_cr"], CONST["T_cr"], CONST["p_cr"]
DT = 0.2
# Time step of the droplet workloads.  At dt = 0.2 the 256 x 256 droplet at 0.9 T_cr
# grows a slow mode and leaves the EoS domain after ~15000 steps; at dt = 0.1 it holds
# for the full 20000 steps (omega = 1.5 or 1.0).  Below 0.9 T_cr (the serving jobs go
# down to 0.85 T_cr, liquid/vapour density ratio ~7) dt = 0.2 loses positivity of p
# within a few hundred steps, dt = 0.1 holds on single droplets.  Merging droplets at
# T <= 0.86 T_cr can still leave the EoS domain; such jobs end with an error status,
# the same alone and batched.
DT_DROPLET = 0.1
KAPPA_DROPLET = 0.0176
PERIODIC, OUTFLOW, INFLOW = 0, 1, 2


def coexistence(t_over_tcr: float):
    """(rho_vapour, rho_liquid) at a tabulated T/T_cr (0.850, 0.855, ..., 0.995)."""
    tab = CONST["coexistence"]
    i = int(np.argmin(np.abs(np.asarray(tab["T_over_Tcr"]) - t_over_tcr)))
    if abs(tab["T_over_Tcr"][i] - t_over_tcr) > 1e-9:
        raise KeyError(f"T/T_cr = {t_over_tcr} is not tabulated")
    return tab["rho_v"][i], tab["rho_l"][i]


@dataclass
class Case:
    """Run parameters (same fields as the oracle's and the library's configs) plus the
    initial macroscopic fields."""
    name: str
    dim: int
    n: tuple
    params: dict
    rho: np.ndarray
    u: np.ndarray          # (dim, N)
    T: np.ndarray
    steps: int = 100
    bc: tuple = ((PERIODIC, PERIODIC), (PERIODIC, PERIODIC))
    inflow: tuple = ()     # ((axis, side, (rho, ux, uy, T)), ...)
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(np.prod(self.n[: self.dim]))


def base_params(**kw) -> dict:
    p = dict(a=A, b=B, R=R, delta=1.0 / 3.0, omega=1.5, kappa=0.0, k_scale=1.0, dt=DT, n_pass=2,
             eos=0, isothermal=0, T0=0.0, eos_c=(0.0, 0.0, 0.0, 0.0))
    p.update(kw)
    return p


def _grid(nx, ny):
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(ny, dtype=np.float64)
    return np.meshgrid(x, y, indexing="xy")  # shape (ny, nx), x fastest


def droplet_field(nx, ny, rho_v, rho_l, centres, radii, width=4.0, periodic=(True, True)):
    """rho(r) = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh(2 (r - R)/width) for each droplet,
    r the (minimum-image on periodic axes) distance to the centre; several droplets are
    combined by taking the largest density."""
    X, Y = _grid(nx, ny)
    out = np.full((ny, nx), rho_v)
    for (cx, cy), rad in zip(centres, radii):
        dx, dy = X - cx, Y - cy
        if periodic[0]:
            dx = dx - nx * np.round(dx / nx)
        if periodic[1]:
            dy = dy - ny * np.round(dy / ny)
        r = np.sqrt(dx * dx + dy * dy)
        out = np.maximum(out, 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (r - rad) / width))
    return out.ravel()


def static_droplet(n=256, t_over_tcr=0.9, radius=40.0, width=4.0, steps=20000, **kw) -> Case:
    """Subcritical static droplet, D2Q9, periodic (radius 40 on 256 x 256 by default)."""
    rv, rl = coexistence(t_over_tcr)
    rho = droplet_field(n, n, rv, rl, [(n / 2, n / 2)], [radius], width)
    N = n * n
    return Case(name=f"droplet{n}", dim=2, n=(n, n),
                params=base_params(**{"omega": 1.5, "kappa": KAPPA_DROPLET, "dt": DT_DROPLET, **kw}),
                rho=rho, u=np.zeros((2, N)), T=np.full(N, t_over_tcr * T_CR), steps=steps,
                meta=dict(rho_v=rv, rho_l=rl, radius=radius, t_over_tcr=t_over_tcr))


def shock_tube(n=1000, steps=2000, **kw) -> Case:
    """1D van der Waals shock tube, D1Q3: T = 1.05 T_cr, rho = 1.5 rho_cr on the left half
    and 0.5 rho_cr on the right half, u = 0, outflow at both ends, no interface energy."""
    x = np.arange(n)
    rho = np.where(x < n // 2, 1.5 * RHO_CR, 0.5 * RHO_CR).astype(np.float64)
    return Case(name=f"shocktube{n}", dim=1, n=(n,), params=base_params(omega=1.0, **kw),
                rho=rho, u=np.zeros((1, n)), T=np.full(n, 1.05 * T_CR), steps=steps,
                bc=((OUTFLOW, OUTFLOW), (PERIODIC, PERIODIC)))


def reduced_shock_tube(name="anomalous", n=800, steps=None, delta=None, **kw) -> Case:
    """1D van der Waals shock tube between two states the paper prints in reduced units:
    "anomalous" (main text, Fig. 4, delta = 0.0125), "case_I" and "case_II" (App. E).
    The diaphragm sits at the middle, u = 0, outflow at both ends, no interface energy;
    the temperatures are those of the stored table.  delta overrides the table's value
    (with the same rho and T on each side).  The default step count reaches the
    paper's snapshot time t* = (t/L) sqrt(p_cr/rho_cr) = 0.45."""
    tube = CONST["shock_tubes"][name]
    x = np.arange(n)
    left = x < n // 2
    rho = np.where(left, tube["left"]["rho"], tube["right"]["rho"]).astype(np.float64)
    T = np.where(left, tube["left"]["T"], tube["right"]["T"]).astype(np.float64)
    d = tube["delta"] if delta is None else delta
    p = base_params(omega=1.0, delta=d, **kw)
    if steps is None:
        steps = int(round(0.45 * n / np.sqrt(P_CR / RHO_CR) / p["dt"]))
    return Case(name=f"shocktube_{name}{n}", dim=1, n=(n,), params=p, rho=rho, u=np.zeros((1, n)), T=T,
                steps=steps, bc=((OUTFLOW, OUTFLOW), (PERIODIC, PERIODIC)), meta=dict(tube=tube))


def droplet_shock(nx=1024, ny=512, steps=1500, radius=50.0, x_drop=300.0, x_shock=150.0, **kw) -> Case:
    """Planar shock (pressure ratio 3, post-shock state from the Rankine-Hugoniot relations)
    running into saturated vapour at 0.95 T_cr that holds a liquid droplet; inflow at x = 0
    (post-shock state), outflow at x = nx - 1, periodic in y."""
    sh = CONST["shock"]
    X, Y = _grid(nx, ny)
    rho = droplet_field(nx, ny, sh["rho0"], sh["rho_liquid"], [(x_drop, ny / 2)], [radius], 4.0,
                        periodic=(False, True)).reshape(ny, nx)
    post = X < x_shock
    rho = np.where(post, sh["rho1"], rho)
    T = np.where(post, sh["T1"], 0.95 * T_CR)
    ux = np.where(post, sh["u1"], 0.0)
    N = nx * ny
    return Case(name=f"dropshock{nx}x{ny}", dim=2, n=(nx, ny),
                params=base_params(omega=1.0, kappa=KAPPA_DROPLET, **kw),
                rho=rho.ravel(), u=np.stack([ux.ravel(), np.zeros(N)]), T=T.ravel(), steps=steps,
                bc=((INFLOW, OUTFLOW), (PERIODIC, PERIODIC)),
                inflow=((0, 0, (sh["rho1"], sh["u1"], 0.0, sh["T1"])),), meta=dict(shock=sh))


def perturbed(nx, ny, seed, dim=2, rho0=2.0, t_over_tcr=1.05, u0=(0.0, 0.0), amp=0.05, modes=3,
              **kw) -> Case:
    """Smooth seeded single-phase state: a few random Fourier modes (periodic on the
    lattice) on rho, u and T.  numpy PCG64 with the given seed."""
    rng = np.random.default_rng(seed)
    if dim == 1:
        ny = 1
    X, Y = _grid(nx, ny)

    def field_(scale):
        f = np.zeros_like(X)
        for _ in range(modes):
            kx = rng.integers(1, 4)
            ky = rng.integers(0, 4) if dim == 2 else 0
            ph = rng.uniform(0.0, 2.0 * np.pi)
            f += rng.uniform(-1.0, 1.0) * np.sin(2 * np.pi * (kx * X / nx + ky * Y / ny) + ph)
        return scale * f / modes

    rho = rho0 * (1.0 + field_(amp))
    T = t_over_tcr * T_CR * (1.0 + field_(0.2 * amp))
    ux = u0[0] + field_(0.4 * amp)
    N = nx * ny
    u = np.stack([ux.ravel(), (u0[1] + field_(0.4 * amp)).ravel()]) if dim == 2 else ux.reshape(1, N)
    n = (nx, ny) if dim == 2 else (nx,)
    return Case(name=f"perturbed{nx}x{ny}s{seed}", dim=dim, n=n, params=base_params(**kw),
                rho=rho.ravel(), u=u, T=T.ravel(), meta=dict(seed=seed))


def perturbed3(nx, ny, nz, seed, rho0=2.0, t_over_tcr=1.05, u0=(0.0, 0.0, 0.0), amp=0.05, modes=3,
               **kw) -> Case:
    """Smooth seeded single-phase state on a periodic nx x ny x nz box (D3Q27): a few
    random Fourier modes on rho, u and T.  numpy PCG64 with the given seed."""
    rng = np.random.default_rng(seed)
    Z, Y, X = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float), np.arange(nx, dtype=float),
                          indexing="ij")  # x fastest

    def field_(scale):
        f = np.zeros_like(X)
        for _ in range(modes):
            k = rng.integers(1, 4), rng.integers(0, 4), rng.integers(0, 4)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            f += rng.uniform(-1.0, 1.0) * np.sin(2 * np.pi * (k[0] * X / nx + k[1] * Y / ny + k[2] * Z / nz) + ph)
        return scale * f / modes

    rho = rho0 * (1.0 + field_(amp))
    T = t_over_tcr * T_CR * (1.0 + field_(0.2 * amp))
    u = np.stack([(u0[a] + field_(0.4 * amp)).ravel() for a in range(3)])
    return Case(name=f"perturbed3_{nx}x{ny}x{nz}s{seed}", dim=3, n=(nx, ny, nz),
                bc=((PERIODIC, PERIODIC), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)),
                params=base_params(**kw), rho=rho.ravel(), u=u, T=T.ravel(), meta=dict(seed=seed))


def static_droplet3(n=256, t_over_tcr=0.9, radius=48.0, width=4.0, steps=2000, **kw) -> Case:
    """Subcritical static droplet on a periodic n^3 box (D3Q27), centred, tanh profile
    of the given width between the Maxwell densities (radius 48 on 256^3 by default)."""
    rv, rl = coexistence(t_over_tcr)
    c = n / 2.0
    z, y, x = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), np.arange(n, dtype=float),
                          indexing="ij")
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    rho = (0.5 * (rl + rv) - 0.5 * (rl - rv) * np.tanh(2.0 * (r - radius) / width)).ravel()
    N = n ** 3
    return Case(name=f"droplet3d{n}", dim=3, n=(n, n, n),
                bc=((PERIODIC, PERIODIC), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)),
                params=base_params(**{"omega": 1.5, "kappa": KAPPA_DROPLET, "dt": DT_DROPLET, **kw}),
                rho=rho, u=np.zeros((3, N)), T=np.full(N, t_over_tcr * T_CR), steps=steps,
                meta=dict(rho_v=rv, rho_l=rl, radius=radius, t_over_tcr=t_over_tcr))


def serving_jobs(count=64, seed=0, steps=5000, rate=20.0, sides=(64, 128, 256, 512)):
    """Batched-serving workload: seeded D2Q9 droplet jobs with sides drawn from `sides`,
    T/T_cr uniform in [0.85, 1.10] (snapped to the 0.005 grid of the coexistence table),
    1-4 droplets with radii uniform in [0.05, 0.2] x side, Poisson arrivals at `rate`
    jobs/s.  Supercritical jobs use 1.5 and 0.5 rho_cr inside and outside the droplets.
    Returns a list of (arrival_time_s, Case)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for j in range(count):
        t += rng.exponential(1.0 / rate)
        side = int(rng.choice(sides))
        tr = round(round(rng.uniform(0.85, 1.10) / 0.005) * 0.005, 3)
        nd = int(rng.integers(1, 5))
        radii = rng.uniform(0.05, 0.2, nd) * side
        centres = rng.uniform(0, side, (nd, 2))
        if tr < 1.0:
            rv, rl = coexistence(min(tr, 0.995))
        else:
            rv, rl = 0.5 * RHO_CR, 1.5 * RHO_CR
        rho = droplet_field(side, side, rv, rl, [tuple(c) for c in centres], list(radii), 4.0)
        N = side * side
        case = Case(name=f"job{j}", dim=2, n=(side, side),
                    params=base_params(omega=1.5, kappa=KAPPA_DROPLET, dt=DT_DROPLET),
                    rho=rho, u=np.zeros((2, N)), T=np.full(N, tr * T_CR), steps=steps,
                    meta=dict(job=j, t_over_tcr=tr, droplets=nd))
        jobs.append((t, case))
    return jobs

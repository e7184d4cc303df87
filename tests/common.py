"""Helpers shared by the tests: run one workload Case on the oracle and on the HIP
path through the C ABI, and compare fields."""
from __future__ import annotations

import numpy as np

from oracle import core
from oracle.thermo import VdW
from paper_2002_09217_amd import pond

# relative velocity errors are taken against max(|u|, U_ch), U_ch = sqrt(p_cr/rho_cr)
U_CH = float(np.sqrt((1.0 / 6.0) / 3.5))


def _eos_kw(p) -> dict:
    return dict(eos=p.get("eos", 0), isothermal=p.get("isothermal", 0), T0=p.get("T0", 0.0),
                eos_c=tuple(p.get("eos_c", (0.0,) * 4)))


def oracle_config(case) -> core.Config:
    p = case.params
    inflow = [[(0.0,) * 4, (0.0,) * 4], [(0.0,) * 4, (0.0,) * 4]]
    for a, s, st in case.inflow:
        inflow[a][s] = tuple(st)
    return core.Config(dim=case.dim, nx=case.n[0], ny=case.n[1] if case.dim == 2 else 1,
                       bc=case.bc, inflow=tuple(tuple(x) for x in inflow), a=p["a"], b=p["b"],
                       R=p["R"], delta=p["delta"], omega=p["omega"], kappa=p["kappa"],
                       k_scale=p["k_scale"], dt=p["dt"], n_pass=p["n_pass"], **_eos_kw(p))


def pond_config(case, precision=pond.FP64, stream=None, tile=-1, two_kernel=0) -> pond.Config:
    p = case.params
    return pond.Config(dim=case.dim, n=tuple(case.n), bc=case.bc, inflow=case.inflow,
                       a=p["a"], b=p["b"], R=p["R"], delta=p["delta"], omega=p["omega"],
                       kappa=p["kappa"], k_scale=p["k_scale"], dt=p["dt"], n_pass=p["n_pass"],
                       precision=precision, tile=tile, stream=stream, two_kernel=two_kernel, **_eos_kw(p))


def run_oracle(case, steps):
    sim = core.Sim(oracle_config(case))
    uy = case.u[1] if case.dim == 2 else None
    sim.init(case.rho, case.u[0], case.T, uy=uy)
    if steps:
        sim.step(steps)
    return sim.moments()


def oracle_config3(case) -> core.Config3:
    p = case.params
    return core.Config3(nx=case.n[0], ny=case.n[1], nz=case.n[2], a=p["a"], b=p["b"], R=p["R"],
                        delta=p["delta"], omega=p["omega"], kappa=p["kappa"], k_scale=p["k_scale"],
                        dt=p["dt"], n_pass=p["n_pass"], **_eos_kw(p))


def run_oracle3(case, steps):
    sim = core.Sim3(oracle_config3(case)).init(case.rho, case.u, case.T)
    if steps:
        sim.step(steps)
    return sim.moments()


def run_gpu(case, steps, precision=pond.FP64, tile=-1, two_kernel=0):
    lat = pond.Lattice(pond_config(case, precision, tile=tile, two_kernel=two_kernel))
    try:
        lat.init_fields(case.rho, case.u, case.T)
        if steps:
            lat.step(steps)
        return lat.moments()
    finally:
        lat.close()


def rel_err(a, b, field):
    """Relative L-infinity error; velocities against max(max|b|, U_ch)."""
    den = np.max(np.abs(b))
    if field in ("ux", "uy", "uz"):
        den = max(den, U_CH)
    return float(np.max(np.abs(a - b)) / den)


def compare(gpu, ref, fields=("rho", "ux", "uy", "E", "T", "p")):
    return {f: rel_err(gpu[f], ref[f], f) for f in fields}


def pulse_speed(sim_factory, rho0, Tr, n=800, sigma=8.0, amp=1e-3, dt=0.2, times=(150.0, 300.0), isentrope=None):
    """Speed of the right-moving half of a Gaussian isentropic density pulse: the
    displacement of its centroid (a window of +-3 sigma around its peak) between two
    times.  sim_factory(rho, T, dt) returns an object with step(n) and moments().
    isentrope(rho) gives T along the pulse (default: the van der Waals isentrope through
    rho0 at Tr T_cr)."""
    x = np.arange(n, dtype=float)
    x0 = n / 2
    rho = rho0 * (1.0 + amp * np.exp(-0.5 * ((x - x0) / sigma) ** 2))
    T = VdW().T_isentrope(rho, rho0, Tr * VdW().T_cr) if isentrope is None else isentrope(rho)
    sim = sim_factory(rho, T, dt)
    pos, done = [], 0
    for t in times:
        nsteps = int(round(t / dt))
        sim.step(nsteps - done)
        done = nsteps
        d = sim.moments()["rho"] - rho0
        right = x > x0 + 2 * sigma
        xp = x[right][np.argmax(d[right])]
        win = np.abs(x - xp) < 3 * sigma
        pos.append(np.sum(x[win] * d[win]) / np.sum(d[win]))
    return (pos[1] - pos[0]) / (times[1] - times[0])

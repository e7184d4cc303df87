"""Physics of the HIP path through the C ABI: a small isentropic pressure pulse travels
at the adiabatic van der Waals sound speed (App. A; main text, Fig. 1) along the
saturation curve and in the single-phase region, in every precision; the anomalous
shock tube (main text, Fig. 4) shows a rarefaction shock and a compression fan where
the classical states (App. E) show the opposite pair."""
import numpy as np
import pytest

from oracle.thermo import VdW
from paper_2002_09217_amd import pond, workloads as W
from tests.common import compare, pond_config, pulse_speed, run_gpu, run_oracle

pytestmark = pytest.mark.gpu
VDW = VdW()


def _states():
    out = [(1.75, 1.05), (3.5, 1.2)]
    for tr in (0.85, 0.9, 0.95):
        rv, rl = W.coexistence(tr)
        out += [(rv, tr), (rl, tr)]
    return out


@pytest.mark.parametrize("precision", [pond.FP64, pond.FP32_STORE, pond.FP32_STORE_FP64_MATH])
def test_pulse_travels_at_the_vdw_sound_speed(precision):
    def factory(rho, T, dt):
        cfg = pond.Config(dim=1, n=(rho.size,), bc=((0, 0),), omega=1.5, kappa=0.0, dt=dt, n_pass=2,
                          precision=precision, tile=0)
        lat = pond.Lattice(cfg)
        lat.init_fields(rho, np.zeros(rho.size), T)
        return lat

    for rho0, tr in _states():
        c = pulse_speed(factory, rho0, tr)
        ref = VDW.sound_vdw(rho0, tr * VDW.T_cr)
        print(f"rho {rho0:.4f} T/Tcr {tr}: pulse {c:.5f} vdW {ref:.5f} ({c / ref - 1:+.2e})", flush=True)
        assert c == pytest.approx(ref, rel=3e-3)


def _gpu_steepening(case, t1_steps, precision=pond.FP64):
    lat = pond.Lattice(pond_config(case, precision=precision, tile=0))
    lat.init_fields(case.rho, case.u, case.T)
    out, n = [], case.n[0]
    for _ in range(2):
        lat.step(t1_steps)
        dp = np.abs(np.diff(lat.moments()["p"]))
        out.append((dp[: n // 2].max(), dp[n // 2:].max(), int(np.argmax(dp[: n // 2])),
                    n // 2 + int(np.argmax(dp[n // 2:]))))
    lat.close()
    return out


def test_anomalous_shock_tube_parity_with_the_oracle():
    case = W.reduced_shock_tube("anomalous", n=400, dt=0.2)
    ref, got = run_oracle(case, 500), run_gpu(case, 500)
    errs = compare(got, ref, ("rho", "ux", "E", "T", "p"))
    print(errs, flush=True)
    assert max(errs.values()) <= 1e-12


@pytest.mark.parametrize("precision", [pond.FP64, pond.FP32_STORE])
def test_anomalous_rarefaction_shock_and_classical_control(precision):
    """Main text, Fig. 4 (delta = 0.0125) on 2000 nodes: the expansion toward the
    high-pressure side stays a shock and the compression spreads as a fan; App. E case I
    (delta = 0.329) and the anomalous states at delta = 1/3 give the classical pair."""
    n = 2000
    case = W.reduced_shock_tube("anomalous", n=n, dt=0.2)
    (l1, r1, xl1, xr1), (l2, r2, xl2, xr2) = _gpu_steepening(case, case.steps // 2, precision)
    print(f"anomalous: rarefaction {l2 / l1:.3f} compression {r2 / r1:.3f}", flush=True)
    assert l2 / l1 > 0.85 and r2 / r1 < 0.75
    assert xl2 < xl1 < n // 2 < xr1 < xr2
    for name, d, frac in (("anomalous", 1.0 / 3.0, 6), ("case_I", None, 6)):
        c = W.reduced_shock_tube(name, n=n, dt=0.2, delta=d)
        (l1, r1, *_), (l2, r2, *_) = _gpu_steepening(c, c.steps // frac, precision)
        print(f"{name} delta {c.params['delta']:.4f}: rarefaction {l2 / l1:.3f} compression {r2 / r1:.3f}",
              flush=True)
        assert l2 / l1 < 0.75 and r2 / r1 > 0.85


def _laplace_ratio(s, R, relax, samples=200):
    """Delta p R_e / sigma of a static droplet with kappa = 0.0176 s^2 and a profile of width
    4 s at 0.9 T_cr (energy equation on): relaxed by restarting from rest whenever the
    kinetic energy peaks, then Delta p = p_in - p_out averaged over samples x 20 steps, with
    p_in and p_out the mean pressures more than 8 s nodes inside and outside the nominal
    radius (closer in, the pressure dip of the interface and the stiff liquid bias them)."""
    import math
    kappa = 0.0176 * s * s
    n = 2 * R + 24 * s
    n += (-n) % 16
    case = W.static_droplet(n=n, radius=float(R), width=4.0 * s, kappa=kappa, dt=0.1, omega=1.0)
    print(f"laplace: s={s} R={R} n={n}", flush=True)
    lat = pond.Lattice(pond_config(case, tile=0))
    try:
        lat.init_fields(case.rho, case.u, case.T)
        prev, done = 0.0, 0
        while done < relax:
            lat.step(10)
            done += 10
            m = lat.moments()
            ke = float(np.sum(m["rho"] * (m["ux"] ** 2 + m["uy"] ** 2)))
            if ke < prev:
                lat.init_fields(m["rho"], np.zeros((2, n * n)), m["T"])
                prev = 0.0
            else:
                prev = ke
        X, Y = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
        r = np.hypot(X - n / 2, Y - n / 2).ravel()
        dps, Ts = [], []
        for _ in range(samples):
            lat.step(20)
            m = lat.moments()
            dps.append(m["p"][r < R - 8 * s].mean() - m["p"][r > R + 8 * s].mean())
            Ts.append(m["T"].mean())
    finally:
        lat.close()
    rho = m["rho"]
    lo, hi = np.percentile(rho, 1), np.percentile(rho, 99)
    Re = math.sqrt(np.sum((rho - lo) / (hi - lo)) / math.pi)
    return np.mean(dps) * Re / VDW.surface_tension(np.mean(Ts), kappa)


def test_laplace_law_on_droplets():
    """Supplement, surface tension: the pressure jump of static droplets falls like 1/R.
    With the interface resolved by 8.8 nodes (kappa = 4 x 0.0176), Delta p R is the same
    for R = 40, 60, 80 within 3 % and close to the square-gradient tension (measured 0.88 of
    it: with the energy equation the interface keeps evolving slowly).  At the workloads'
    4.4-node interface the jump is still positive and of Laplace size."""
    fine = [_laplace_ratio(2, R, 12000) for R in (40, 60, 80)]
    print("laplace kappa x4, R = 40, 60, 80: Delta p R / sigma =", fine, flush=True)
    assert max(fine) / min(fine) < 1.03, fine
    assert all(0.8 < x < 1.0 for x in fine), fine
    coarse = [_laplace_ratio(1, R, 6000) for R in (20, 30, 40)]
    print("laplace kappa x1, R = 20, 30, 40: Delta p R / sigma =", coarse, flush=True)
    assert all(0.65 < x < 1.0 for x in coarse), coarse
    assert max(coarse) / min(coarse) < 1.2, coarse

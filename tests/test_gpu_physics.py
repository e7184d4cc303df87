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
        # FP32 streaming rounds the 1e-3 pulse at the 1e-3 level of its own amplitude
        assert c == pytest.approx(ref, rel=5e-3 if precision == pond.FP32_STORE else 3e-3)


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

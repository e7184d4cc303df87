"""Physics of the HIP path through the C ABI: a small isentropic pressure pulse travels
at the adiabatic van der Waals sound speed (App. A; main text, Fig. 1) along the
saturation curve and in the single-phase region, in every precision."""
import numpy as np
import pytest

from oracle.thermo import VdW
from paper_2002_09217_amd import pond, workloads as W
from tests.common import pulse_speed

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

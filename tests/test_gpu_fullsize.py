"""Configs 2 and 3 at their full sizes and full lengths, beyond the oracle: properties that
hold at any size.  Both initial states are mirror symmetric (the 256^2 droplet about its
centre lines and diagonal, the droplet-shock case about the droplet's y line, its shock being
planar), the scheme's stencils respect the mirrors, so the computed state must keep them:
FP64 to round-off accumulated over the run.  In the FP32 storage forms mirror nodes round
their stored FP32 values apart (tile references are not mirror images of each other), by
about one FP32 ulp of a deviation per step, which accumulates like a random walk: 2^-24
sqrt(20000) ~ 1e-5 over config 2 with FP32 streaming (bound 3e-5), rare single-ulp tips of
the stored deviations with FP64 arithmetic (bound 1e-8)."""
import numpy as np
import pytest

from paper_2002_09217_amd import pond, workloads as W
from tests.common import U_CH, pond_config

pytestmark = pytest.mark.gpu

TOL = {pond.FP64: 1e-12, pond.FP32_STORE_FP64_MATH: 1e-8, pond.FP32_STORE: 3e-5}


def _run(case, precision, steps):
    lat = pond.Lattice(pond_config(case, precision))
    try:
        lat.init_fields(case.rho, case.u, case.T)
        lat.step(steps)
        assert lat.steps_done() == steps
        return lat.moments()
    finally:
        lat.close()


@pytest.mark.parametrize("precision", [pond.FP64, pond.FP32_STORE_FP64_MATH, pond.FP32_STORE])
def test_config2_droplet_keeps_its_symmetry_over_20000_steps(precision):
    case = W.static_droplet(n=256)
    n = 256
    m = _run(case, precision, 20000)
    rho, ux, uy = (m[k].reshape(n, n) for k in ("rho", "ux", "uy"))   # [y][x]
    refl = (n - np.arange(n)) % n                                      # about the centre n/2
    sc = np.max(rho)
    errs = {"swap xy": np.max(np.abs(rho - rho.T)) / sc,
            "reflect x": np.max(np.abs(rho - rho[:, refl])) / sc,
            "reflect y": np.max(np.abs(rho - rho[refl, :])) / sc,
            "u swap xy": np.max(np.abs(ux - uy.T)) / U_CH,
            "u reflect x": np.max(np.abs(ux + ux[:, refl])) / U_CH}
    print(precision, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= TOL[precision], errs
    # still a droplet in its vapour: liquid core and vapour at their coexistence densities
    assert rho[n // 2, n // 2] == pytest.approx(case.meta["rho_l"], rel=5e-3)
    assert rho[0, 0] == pytest.approx(case.meta["rho_v"], rel=5e-3)


@pytest.mark.parametrize("precision", [pond.FP64, pond.FP32_STORE_FP64_MATH, pond.FP32_STORE])
def test_config3_droplet_shock_keeps_its_mirror_over_1500_steps(precision):
    case = W.droplet_shock()
    nx, ny = case.n
    m = _run(case, precision, case.steps)
    rho, ux, uy = (m[k].reshape(ny, nx) for k in ("rho", "ux", "uy"))
    refl = (ny - np.arange(ny)) % ny                                   # y -> ny - y about ny/2
    errs = {"rho": np.max(np.abs(rho - rho[refl])) / np.max(rho),
            "u_x": np.max(np.abs(ux - ux[refl])) / max(np.max(np.abs(ux)), U_CH),
            "u_y": np.max(np.abs(uy + uy[refl])) / max(np.max(np.abs(uy)), U_CH)}
    print(precision, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= TOL[precision], errs
    assert np.all(np.isfinite(rho)) and np.min(rho) > 0.0

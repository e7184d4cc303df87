"""Parity of the HIP path (through the C ABI) with the FP64 oracle on identical seeded
inputs.  Bar: 1e-12 relative L-infinity on rho, u, E (and T, p) for the FP64 form;
1e-5 for the FP32-storage form over 100 steps (FP32 rounding, 6e-8 of the deviations from
the tile reference per step, accumulating like a random walk over 100 steps and amplified
a few times at droplet interfaces: 1e-7 to 3e-6 observed) and 1e-6 for FP32 storage with
FP64 arithmetic.  Both forms of the 1D/2D step run: the
fused one-kernel step (the default) and the two-kernel step with stored populations.

Sizes span several 32 x 8 streaming tiles with ragged tails; the full 256 x 256
droplet of the benchmark is compared after 3 and 45 steps (the oracle takes about half a
second per step there on 16 threads)."""
import numpy as np
import pytest

from paper_2002_09217_amd import pond, workloads as W
from tests.common import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _check(case, steps, tol=TOL64, precision=pond.FP64, fields=("rho", "ux", "uy", "E", "T", "p"), tile=-1,
           two_kernel=0):
    ref = run_oracle(case, steps)
    print(f"parity: {case.name} n={case.n} steps={steps} precision={precision} tile={tile} two_kernel={two_kernel}",
          flush=True)
    got = run_gpu(case, steps, precision, tile=tile, two_kernel=two_kernel)
    errs = compare(got, ref, fields)
    print(case.name, steps, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{case.name}: {bad}"
    return errs


@pytest.mark.parametrize("two_kernel", [0, 1])
@pytest.mark.parametrize("n_pass", [1, 2, 3])
@pytest.mark.parametrize("kappa", [0.0, 0.0176])
def test_perturbed_2d_100_steps(n_pass, kappa, two_kernel):
    case = W.perturbed(40, 36, seed=11 + n_pass, rho0=2.0, t_over_tcr=1.05, u0=(0.05, -0.03),
                       n_pass=n_pass, kappa=kappa)
    _check(case, 100, two_kernel=two_kernel)


def test_perturbed_2d_one_step_large_velocity():
    case = W.perturbed(33, 17, seed=5, rho0=1.0, t_over_tcr=1.4, u0=(1.0911, 0.3))
    _check(case, 1)
    _check(case, 20)


@pytest.mark.parametrize("tile", [0, 3, 5])
def test_shear_flow_both_fp64_window_variants(tile):
    """A shear flow faster than sqrt(theta) in some rows and slower in others, on the
    512-lane tile shapes: waves whose stencils all allow it take the FP64 window without
    zero taps, the others the general window."""
    case = W.perturbed(48, 40, seed=12 + tile, rho0=1.0, t_over_tcr=1.4)
    y = np.arange(40, dtype=float).repeat(48)
    case.u[0] = case.u[0] - case.u[0].mean() + 1.2 * np.sin(2.0 * np.pi * y / 40.0)
    _check(case, 20, tile=tile)


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_droplet_64_100_steps(two_kernel):
    case = W.static_droplet(n=64, radius=14.0, steps=100)
    _check(case, 100, two_kernel=two_kernel)


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_droplet_near_the_spinodal_085(two_kernel):
    """The coldest serving temperature, 0.85 T_cr (0.7 % above the temperature where the
    van der Waals loop reaches p < 0): a 64^2 droplet for 100 steps."""
    case = W.static_droplet(n=64, t_over_tcr=0.85, radius=14.0, steps=100)
    _check(case, 100, two_kernel=two_kernel)


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_shock_tube_1d_100_steps(two_kernel):
    case = W.shock_tube(n=1000)
    _check(case, 100, fields=("rho", "ux", "E", "T", "p"), two_kernel=two_kernel)


def test_perturbed_1d_ragged():
    case = W.perturbed(300, 1, seed=3, dim=1, kappa=0.0176)
    _check(case, 100, fields=("rho", "ux", "E", "T", "p"))


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_inflow_outflow_2d(two_kernel):
    case = W.droplet_shock(nx=96, ny=40, radius=8.0, x_drop=50.0, x_shock=20.0)
    _check(case, 50, two_kernel=two_kernel)


@pytest.mark.parametrize("tile", [0, 2, 5])
def test_outflow_on_every_face_2d(tile):
    """Outflow faces on all four sides (corners clamp in both axes), a lattice narrower
    than some halos: the copy stages of the fused step's closure and donor regions."""
    case = W.perturbed(37, 21, seed=71 + tile, kappa=0.0176, u0=(0.2, -0.1))
    case.bc = ((W.OUTFLOW, W.OUTFLOW), (W.OUTFLOW, W.OUTFLOW))
    _check(case, 30, tile=tile)


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_inflow_outflow_1d(two_kernel):
    """D1Q3 with an inflow face at x = 0 (the fused step's ghost donors and closure cells in
    1D) and an outflow face at the other end."""
    case = W.perturbed(150, 1, seed=81, dim=1, kappa=0.0176, u0=(0.08, 0.0))
    case.bc = ((W.INFLOW, W.OUTFLOW), (W.PERIODIC, W.PERIODIC))
    case.inflow = ((0, 0, (2.0, 0.08, 0.0, 1.05 * W.T_CR)),)
    _check(case, 50, fields=("rho", "ux", "E", "T", "p"), two_kernel=two_kernel)


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_inflow_on_a_y_face(two_kernel):
    """Inflow through the low y face, outflow through the high one, periodic in x."""
    case = W.perturbed(30, 41, seed=82, kappa=0.0176, u0=(0.0, 0.06))
    case.bc = ((W.PERIODIC, W.PERIODIC), (W.INFLOW, W.OUTFLOW))
    case.inflow = ((1, 0, (2.0, 0.0, 0.06, 1.05 * W.T_CR)),)
    _check(case, 40, two_kernel=two_kernel)


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_tiny_lattices_with_outflow_faces(two_kernel):
    """Lattices smaller than every halo, outflow on all faces: the copy rules clamp across
    the whole lattice."""
    for nx, ny, dim in ((3, 5, 2), (2, 2, 2), (4, 1, 1)):
        case = W.perturbed(nx, ny, seed=90 + nx * 10 + ny, dim=dim, kappa=0.0176, u0=(0.05, 0.02))
        case.bc = ((W.OUTFLOW, W.OUTFLOW), (W.OUTFLOW, W.OUTFLOW) if dim == 2 else (W.PERIODIC, W.PERIODIC))
        fields = ("rho", "ux", "uy", "E", "T", "p") if dim == 2 else ("rho", "ux", "E", "T", "p")
        print(f"tiny outflow lattice {nx}x{ny} dim {dim}", flush=True)
        _check(case, 10, fields=fields, two_kernel=two_kernel)


def test_tiny_periodic_lattices():
    for nx, ny in ((3, 5), (1, 9), (7, 1)):
        case = W.perturbed(nx, ny, seed=nx * 10 + ny, kappa=0.0176)
        _check(case, 10)


def test_full_size_droplet_256_few_steps():
    case = W.static_droplet(n=256)
    _check(case, 3)


@pytest.fixture(scope="module")
def droplet256_oracle_45():
    case = W.static_droplet(n=256)
    return case, run_oracle(case, 45)


@pytest.mark.parametrize("precision,tol", [(pond.FP64, TOL64), (pond.FP32_STORE, 1e-5)])
def test_full_size_droplet_256_three_long_runs(droplet256_oracle_45, precision, tol):
    """The benchmark's workload (the 256^2 droplet, autotuned tile) for 45 steps: one
    replay of the 45-step graph the benchmark times, fifteen times through the ring."""
    case, ref = droplet256_oracle_45
    print(f"parity: {case.name} n={case.n} steps=45 precision={precision}", flush=True)
    got = run_gpu(case, 45, precision)
    errs = compare(got, ref)
    print(case.name, 45, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= tol, errs


def test_full_size_droplet_shock_1024x512_few_steps():
    """Config 3 at its full size (inflow, outflow, periodic y, the shock and the droplet)
    in the launch configuration the benchmark uses (autotuned tile shape)."""
    case = W.droplet_shock()
    _check(case, 2)


@pytest.mark.parametrize("two_kernel", [0, 1])
@pytest.mark.parametrize("which", ["perturbed", "droplet"])
def test_fp32_storage_within_1e5(which, two_kernel):
    if which == "perturbed":
        case = W.perturbed(40, 36, seed=21, kappa=0.0176)
    else:
        case = W.static_droplet(n=64, radius=14.0)
    _check(case, 100, tol=1e-5, precision=pond.FP32_STORE, two_kernel=two_kernel)


@pytest.mark.parametrize("two_kernel", [0, 1])
@pytest.mark.parametrize("which", ["perturbed", "droplet", "shock_tube"])
def test_fp32_storage_with_fp64_arithmetic_within_1e6(which, two_kernel):
    if which == "perturbed":
        case = W.perturbed(40, 36, seed=22, kappa=0.0176, u0=(0.1, -0.05))
    elif which == "droplet":
        case = W.static_droplet(n=64, radius=14.0)
    else:
        case = W.shock_tube(n=1000)
    fields = ("rho", "ux", "E", "T", "p") if case.dim == 1 else ("rho", "ux", "uy", "E", "T", "p")
    _check(case, 100, tol=1e-6, precision=pond.FP32_STORE_FP64_MATH, fields=fields, two_kernel=two_kernel)


@pytest.mark.parametrize("two_kernel", [0, 1])
@pytest.mark.parametrize("tile", range(6))
def test_every_stream_tile_shape_2d(tile, two_kernel):
    case = W.perturbed(70, 45, seed=30 + tile, kappa=0.0176, u0=(0.1, -0.2))
    _check(case, 30, tile=tile, two_kernel=two_kernel)


@pytest.mark.parametrize("precision,tol", [(pond.FP32_STORE, 1e-5), (pond.FP32_STORE_FP64_MATH, 1e-6)])
@pytest.mark.parametrize("tile", range(6))
def test_every_stream_tile_shape_2d_fp32_storage(tile, precision, tol):
    """Each tile shape's FP32-storage windows (FP32 rows summed in FP32, or FP64 rows added
    straight into the accumulators), including the 256-lane shapes compiled for three
    waves per SIMD."""
    case = W.perturbed(70, 45, seed=50 + tile, kappa=0.0176, u0=(0.1, -0.2))
    _check(case, 30, tol=tol, precision=precision, tile=tile)


@pytest.mark.parametrize("two_kernel", [0, 1])
@pytest.mark.parametrize("tile", range(2))
def test_every_stream_tile_shape_1d(tile, two_kernel):
    case = W.perturbed(333, 1, seed=40 + tile, dim=1, kappa=0.0176, u0=(0.2, 0.0))
    _check(case, 30, tile=tile, fields=("rho", "ux", "E", "T", "p"), two_kernel=two_kernel)

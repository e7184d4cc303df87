"""Parity of the D3Q27 HIP path (through the C ABI) with the three-dimensional FP64
oracle on identical seeded inputs: 1e-12 relative L-infinity for FP64, 1e-6 for FP32
storage with FP64 arithmetic, 1e-4 for FP32 storage and streaming.  Boxes span several
x-y tiles with ragged edges and wrap in every direction."""
import numpy as np
import pytest

from paper_2002_09217_amd import pond, workloads as W
from tests.common import compare, run_gpu, run_oracle3

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "uz", "E", "T", "p")


def _check(case, steps, tol=1e-12, precision=pond.FP64):
    ref = run_oracle3(case, steps)
    got = run_gpu(case, steps, precision)
    errs = compare(got, ref, FIELDS)
    print(case.name, steps, precision, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{case.name}: {bad}"


@pytest.mark.parametrize("n_pass", [1, 2])
@pytest.mark.parametrize("kappa", [0.0, 0.0176])
def test_perturbed_box(n_pass, kappa):
    case = W.perturbed3(19, 11, 6, seed=3 + n_pass, u0=(0.05, -0.03, 0.02), n_pass=n_pass, kappa=kappa, dt=0.2)
    _check(case, 10)


def test_droplet_box():
    case = W.static_droplet3(n=16, radius=5.0)
    _check(case, 10)


def test_tiny_and_flat_boxes():
    for n in ((3, 4, 5), (7, 1, 1), (1, 6, 2)):
        case = W.perturbed3(*n, seed=sum(n), kappa=0.0176, dt=0.2)
        _check(case, 5)


def test_large_velocity():
    case = W.perturbed3(10, 9, 8, seed=9, t_over_tcr=1.4, u0=(0.6, -0.3, 0.25), dt=0.2)
    _check(case, 5)


@pytest.mark.parametrize("precision,tol", [(pond.FP32_STORE, 1e-4), (pond.FP32_STORE_FP64_MATH, 1e-6)])
def test_fp32_storage_forms(precision, tol):
    case = W.perturbed3(17, 12, 7, seed=11, kappa=0.0176, dt=0.2)
    _check(case, 10, tol=tol, precision=precision)

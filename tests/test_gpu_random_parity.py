"""Seeded sweep of small random configurations on the HIP path through the C ABI against
the FP64 oracle: dimension, ragged sizes (down to one node per axis), every combination
of periodic, outflow and inflow faces, n_pass 1-3, the Korteweg force on or off, the
equation of state (van der Waals or Dieterici with the energy equation), tile shape and
step form (fused or two kernels), after a few steps.  Bar: 1e-12 relative L-infinity.
The case list is fixed by numpy PCG64(2024): rerunning a case number reruns that case."""
import numpy as np
import pytest

from oracle.thermo import Dieterici
from paper_2002_09217_amd import pond, workloads as W
from tests.common import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

DIET = Dieterici()
NCASES = 64


def _case(k):
    rng = np.random.default_rng([2024, k])
    dim = int(rng.integers(1, 3))
    nx = int(rng.integers(1, 41))
    ny = int(rng.integers(1, 29)) if dim == 2 else 1
    kw = dict(kappa=float(rng.choice([0.0, 0.0176])), n_pass=int(rng.integers(1, 4)), dt=0.2,
              omega=float(rng.choice([1.0, 1.5])))
    law = rng.random()
    if law < 0.25:
        kw.update(eos=pond.EOS_DIETERICI, isothermal=0, a=DIET.a, b=DIET.b, R=DIET.R)
    elif law < 0.35:
        kw.update(eos=pond.EOS_VDW, isothermal=1, T0=1.05 * W.T_CR)
    u0 = (float(rng.uniform(-0.1, 0.1)), float(rng.uniform(-0.1, 0.1)))
    case = W.perturbed(nx, ny, seed=1000 + k, dim=dim, rho0=2.0, t_over_tcr=1.05, u0=u0, **kw)
    faces = [[W.PERIODIC, W.PERIODIC], [W.PERIODIC, W.PERIODIC]]
    inflow = []
    for a in range(dim):
        kind = int(rng.integers(0, 3))          # 0 periodic, 1 outflow on both, 2 inflow/outflow
        if kind == 1:
            faces[a] = [W.OUTFLOW, W.OUTFLOW]
        elif kind == 2:
            side = int(rng.integers(0, 2))
            faces[a] = [W.OUTFLOW, W.OUTFLOW]
            faces[a][side] = W.INFLOW
            ust = [0.0, 0.0]
            ust[a] = 0.05 if side == 0 else -0.05
            inflow.append((a, side, (2.0, ust[0], ust[1], 1.05 * W.T_CR)))
    case.bc = (tuple(faces[0]), tuple(faces[1]))
    case.inflow = tuple(inflow)
    tiles = 6 if dim == 2 else 2
    return case, int(rng.integers(0, tiles)), int(rng.integers(0, 2)), int(rng.integers(3, 9))


@pytest.mark.parametrize("k", range(NCASES))
def test_random_configuration(k):
    case, tile, two_kernel, steps = _case(k)
    p = case.params
    print(f"case {k}: dim {case.dim} n {case.n} bc {case.bc} inflow {len(case.inflow)} n_pass {p['n_pass']} "
          f"kappa {p['kappa']} eos {p.get('eos', 0)} tile {tile} two_kernel {two_kernel} steps {steps}", flush=True)
    ref = run_oracle(case, steps)
    got = run_gpu(case, steps, tile=tile, two_kernel=two_kernel)
    fields = ("rho", "ux", "uy", "E", "T", "p") if case.dim == 2 else ("rho", "ux", "E", "T", "p")
    errs = compare(got, ref, fields)
    print("   ", {f: f"{v:.2e}" for f, v in errs.items()}, flush=True)
    assert max(errs.values()) <= 1e-12, errs


@pytest.mark.parametrize("k", range(0, NCASES, 2))
def test_random_configuration_fp32_storage(k):
    """The same cases in the two FP32-storage precisions (bars 1e-5 and 1e-6, as for the
    fixed FP32 parity cases)."""
    case, tile, two_kernel, steps = _case(k)
    precision = pond.FP32_STORE if k % 4 == 0 else pond.FP32_STORE_FP64_MATH
    tol = 1e-5 if precision == pond.FP32_STORE else 1e-6
    print(f"case {k}: precision {precision} dim {case.dim} n {case.n} bc {case.bc} tile {tile} "
          f"two_kernel {two_kernel} steps {steps}", flush=True)
    ref = run_oracle(case, steps)
    got = run_gpu(case, steps, precision, tile=tile, two_kernel=two_kernel)
    fields = ("rho", "ux", "uy", "E", "T", "p") if case.dim == 2 else ("rho", "ux", "E", "T", "p")
    errs = compare(got, ref, fields)
    print("   ", {f: f"{v:.2e}" for f, v in errs.items()}, flush=True)
    assert max(errs.values()) <= tol, errs

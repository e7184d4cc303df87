"""Batches through the C ABI, in both step forms: a lattice advanced inside a batch of
other lattices (several groups, mixed sizes, dimensions and precisions, members joining
and leaving) gives bitwise the same state as the same lattice advanced alone; a member
that fails leaves the batch without disturbing the others; a batch holds one step form;
admission footprints."""
import numpy as np
import pytest

from oracle.thermo import Dieterici
from paper_2002_09217_amd import pond, workloads as W
from tests.common import pond_config

DIET = Dieterici()

pytestmark = pytest.mark.gpu


def _fields(m):
    return np.concatenate([m[k] for k in ("rho", "ux", "uy", "T", "p", "E")])


def _lat(case, tile, precision=pond.FP64, two_kernel=0):
    lat = pond.Lattice(pond_config(case, precision=precision, tile=tile, two_kernel=two_kernel))
    lat.init_fields(case.rho, case.u, case.T)
    return lat


def _mix():
    """(case, tile, precision) of the batch members: sizes spanning one to many tiles
    with ragged tails, both dimensions, all three precisions, two tile shapes, and
    isothermal lattices (the streaming kernels' general equation-of-state variant)."""
    return [
        (W.perturbed(40, 36, seed=1, kappa=0.0176, u0=(0.05, -0.03)), 0, pond.FP64),
        (W.static_droplet(n=64, radius=14.0), 0, pond.FP64),
        (W.perturbed(33, 17, seed=2, t_over_tcr=1.4, u0=(0.3, 0.1)), 2, pond.FP64),
        (W.perturbed(70, 45, seed=3, kappa=0.0176), 2, pond.FP32_STORE),
        (W.perturbed(300, 1, seed=4, dim=1, kappa=0.0176), 0, pond.FP64),
        (W.perturbed(7, 1, seed=5, kappa=0.0176), 0, pond.FP64),
        (W.perturbed(129, 1, seed=6, dim=1), 1, pond.FP32_STORE),
        (W.perturbed(50, 30, seed=8, kappa=0.0176), 0, pond.FP32_STORE_FP64_MATH),
        (W.perturbed(45, 20, seed=9, rho0=1.5, kappa=0.0176, eos=pond.EOS_DIETERICI, isothermal=1,
                     T0=0.9 * DIET.T_cr, a=DIET.a, b=DIET.b), 0, pond.FP64),
        (W.perturbed(90, 1, seed=10, dim=1, rho0=5.0, eos=pond.EOS_DOUBLE_WELL, isothermal=1, T0=0.1,
                     eos_c=(8e-4, 5.0, 0.5, 0.1)), 0, pond.FP32_STORE),
    ]


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_batch_members_bitwise_equal_to_alone(two_kernel):
    mix = _mix()
    # chunks of every remainder and one past the long graph run (45 fused steps, 16 for
    # two kernels): every ring slot or state buffer and both graph lengths
    schedule = (1, 6, 50, 2)
    total = sum(schedule)
    alone = []
    for case, tile, prec in mix:
        lat = _lat(case, tile, prec, two_kernel)
        lat.step(total)
        alone.append(_fields(lat.moments()))
        lat.close()

    batch = pond.Batch()
    lats = [_lat(case, tile, prec, two_kernel) for case, tile, prec in mix]
    # the last member joins after the first chunk, and is stepped alone before it
    for lat in lats[:-1]:
        batch.add(lat)
    assert batch.size() == len(mix) - 1
    assert batch.step(schedule[0]) == []
    lats[-1].step(schedule[0])
    batch.add(lats[-1])
    with pytest.raises(pond.PondError) as err:     # members are stepped by the batch only
        lats[0].step(1)
    assert err.value.code == -7
    for n in schedule[1:]:
        assert batch.step(n) == []
    for lat, ref in zip(lats, alone):
        assert lat.steps_done() == total
        assert np.array_equal(_fields(lat.moments()), ref)
    # a member that leaves continues alone from where the batch left it
    batch.remove(lats[1])
    lats[1].step(3)
    assert batch.step(3) == []
    assert lats[1].steps_done() == lats[0].steps_done() == total + 3
    batch.close()
    for lat in lats:
        lat.close()


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_failed_member_leaves_batch_others_unaffected(two_kernel):
    good = W.perturbed(48, 40, seed=7, kappa=0.0176)
    # |u| + sqrt(theta) > 1/dt: the departure stencil would leave the +-2 window
    bad = W.perturbed(24, 24, seed=2, rho0=1.0, t_over_tcr=1.5, u0=(0.7, 0.0), dt=1.0, amp=0.0)
    ref_lat = _lat(good, 0, two_kernel=two_kernel)
    ref_lat.step(10)
    ref = _fields(ref_lat.moments())
    ref_lat.close()

    g = _lat(good, 0, two_kernel=two_kernel)
    b = _lat(bad, 0, two_kernel=two_kernel)
    before = _fields(b.moments())
    batch = pond.Batch()
    batch.add(b)
    batch.add(g)
    failed = batch.step(4)
    assert failed == [b] and batch.size() == 1
    assert b.steps_done() == 0 and np.array_equal(_fields(b.moments()), before)
    with pytest.raises(pond.PondError) as err:
        b.step(1)
    assert err.value.code == -7
    assert batch.step(6) == []
    assert g.steps_done() == 10 and np.array_equal(_fields(g.moments()), ref)
    batch.close()
    g.close()
    b.close()


def test_batch_refuses_a_member_of_the_other_step_form():
    case = W.perturbed(20, 12, seed=11, kappa=0.0176)
    fused, split = _lat(case, 0), _lat(case, 0, two_kernel=1)
    batch = pond.Batch()
    batch.add(fused)
    with pytest.raises(pond.PondError) as err:
        batch.add(split)
    assert err.value.code == -1 and batch.size() == 1
    split.step(2)                     # the refused lattice is still stepped on its own
    assert split.steps_done() == 2
    batch.close()
    fused.close()
    split.close()


def test_footprint_matches_device_allocation():
    import torch
    case = W.static_droplet(n=256)
    for prec in (pond.FP64, pond.FP32_STORE):
        cfg = pond_config(case, precision=prec, tile=0)
        fp = pond.footprint(cfg)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        lat = pond.Lattice(cfg)
        free1 = torch.cuda.mem_get_info()[0]
        lat.close()
        used = free0 - free1
        print("footprint", prec, fp, "allocated", used, flush=True)
        assert fp - (1 << 20) <= used <= fp + (64 << 20)
    assert pond.footprint(pond_config(case, precision=pond.FP32_STORE)) < pond.footprint(pond_config(case))

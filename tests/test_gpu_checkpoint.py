"""Checkpoint / resume through the C ABI: a lattice saved mid-run and loaded into a fresh
handle (or back into the same one after it moved on) continues bitwise as the
uninterrupted run, in every precision; checkpoints of another configuration are refused."""
import numpy as np
import pytest

from paper_2002_09217_amd import pond, workloads as W
from tests.common import pond_config

pytestmark = pytest.mark.gpu


def _fields(m):
    return np.concatenate([m[k] for k in ("rho", "ux", "uy", "T", "p", "E")])


@pytest.mark.parametrize("two_kernel", [0, 1])
@pytest.mark.parametrize("precision", [pond.FP64, pond.FP32_STORE, pond.FP32_STORE_FP64_MATH])
def test_resume_is_bitwise(precision, two_kernel):
    case = W.perturbed(50, 34, seed=4, kappa=0.0176, u0=(0.1, 0.05))
    a = pond.Lattice(pond_config(case, precision=precision, tile=-1, two_kernel=two_kernel))
    a.init_fields(case.rho, case.u, case.T)
    # 13 steps, then 50 after the checkpoint: a long graph run, short runs and single
    # launches after the resume
    a.step(13)
    ck = a.save()
    a.step(50)
    ref = _fields(a.moments())
    # a fresh handle with another tile shape adopts the saved one
    info = a.tile_info()
    b = pond.Lattice(pond_config(case, precision=precision, tile=(info["variant"] + 1) % info["variants"],
                                 two_kernel=two_kernel))
    b.load(ck)
    assert b.steps_done() == 13 and b.tile_info()["variant"] == info["variant"]
    b.step(50)
    assert b.steps_done() == 63
    assert np.array_equal(_fields(b.moments()), ref)
    # rewinding the original handle
    a.load(ck)
    assert a.steps_done() == 13
    a.step(50)
    assert np.array_equal(_fields(a.moments()), ref)
    a.close()
    b.close()


def test_mismatched_checkpoints_refused_and_fresh_handle_resumes():
    case = W.shock_tube(n=300)
    a = pond.Lattice(pond_config(case, tile=0))
    a.init_fields(case.rho, case.u, case.T)
    a.step(5)
    ck = a.save()
    other = W.shock_tube(n=301)
    b = pond.Lattice(pond_config(other, tile=0))
    with pytest.raises(pond.PondError) as err:
        b.load(ck)
    assert err.value.code == -1
    c = pond.Lattice(pond_config(case, precision=pond.FP32_STORE, tile=0))
    with pytest.raises(pond.PondError) as err:
        c.load(ck)
    assert err.value.code == -1
    with pytest.raises(pond.PondError) as err:
        a.load(ck[: len(ck) // 2])
    assert err.value.code == -1
    # a handle that never ran can resume from a checkpoint directly
    d = pond.Lattice(pond_config(case, tile=0))
    d.load(ck)
    d.step(7)
    a.step(7)
    assert np.array_equal(_fields(d.moments()), _fields(a.moments()))
    for x in (a, b, c, d):
        x.close()


def test_isothermal_checkpoint_resumes_and_is_refused_by_another_equation_of_state():
    from oracle.thermo import Dieterici
    g = Dieterici()
    iso = dict(eos=pond.EOS_DIETERICI, isothermal=1, T0=0.9 * g.T_cr, a=g.a, b=g.b)
    case = W.perturbed(36, 28, seed=6, rho0=1.5, kappa=0.0176, **iso)
    a = pond.Lattice(pond_config(case, tile=0))
    a.init_fields(case.rho, case.u, case.T)
    a.step(9)
    ck = a.save()
    a.step(8)
    ref = _fields(a.moments())
    b = pond.Lattice(pond_config(case, tile=0))
    b.load(ck)
    b.step(8)
    assert np.array_equal(_fields(b.moments()), ref)
    other = W.perturbed(36, 28, seed=6, rho0=1.5, kappa=0.0176, eos=pond.EOS_DIETERICI, isothermal=1,
                        T0=0.85 * g.T_cr, a=g.a, b=g.b)   # another T0
    c = pond.Lattice(pond_config(other, tile=0))
    with pytest.raises(pond.PondError) as err:
        c.load(ck)
    assert err.value.code == -1
    for x in (a, b, c):
        x.close()


def test_checkpoint_of_the_other_step_form_is_refused():
    """A fused handle's checkpoint holds the streamed state, a two-kernel handle's the
    collided populations: each form refuses the other's."""
    case = W.perturbed(30, 22, seed=8, kappa=0.0176)
    a = pond.Lattice(pond_config(case, tile=0, two_kernel=0))
    b = pond.Lattice(pond_config(case, tile=0, two_kernel=1))
    try:
        for x in (a, b):
            x.init_fields(case.rho, case.u, case.T)
            x.step(4)
        ca, cb = a.save(), b.save()
        for dst, ck in ((b, ca), (a, cb)):
            with pytest.raises(pond.PondError) as err:
                dst.load(ck)
            assert err.value.code == -1
        # both forms hold the same state to round-off
        ma, mb = a.moments(), b.moments()
        assert np.allclose(_fields(ma), _fields(mb), rtol=1e-12, atol=1e-13)
    finally:
        a.close()
        b.close()


def test_dieterici_energy_equation_checkpoint_resumes_bitwise():
    from oracle.thermo import Dieterici
    g = Dieterici()
    case = W.perturbed(28, 24, seed=9, rho0=2.5, kappa=0.0176, eos=pond.EOS_DIETERICI, isothermal=0, a=g.a, b=g.b)
    a = pond.Lattice(pond_config(case, tile=0))
    a.init_fields(case.rho, case.u, case.T)
    a.step(7)
    ck = a.save()
    a.step(11)
    ref = _fields(a.moments())
    b = pond.Lattice(pond_config(case, tile=0))
    b.load(ck)
    b.step(11)
    assert np.array_equal(_fields(b.moments()), ref)
    a.close()
    b.close()

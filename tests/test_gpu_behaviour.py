"""Behaviour of the HIP path through the C ABI: determinism, equivalence of the
step schedules (graph pairs, single launches, instrumented launches), monitors,
and the error paths (forced from the host through the inputs, kernels exit normally)."""
import numpy as np
import pytest

from paper_2002_09217_amd import pond, workloads as W
from tests.common import pond_config, run_oracle

pytestmark = pytest.mark.gpu


def _lattice(case, tile=0, **kw):
    lat = pond.Lattice(pond_config(case, tile=tile, **kw))
    lat.init_fields(case.rho, case.u, case.T)
    return lat


def _fields(m):
    return np.concatenate([m[k] for k in ("rho", "ux", "uy", "T", "p", "E")])


@pytest.mark.parametrize("precision", [pond.FP64, pond.FP32_STORE])
def test_runs_are_bitwise_deterministic(precision):
    case = W.static_droplet(n=64, radius=14.0)
    out = []
    for _ in range(2):
        lat = _lattice(case, precision=precision)
        lat.step(37)
        out.append(_fields(lat.moments()))
        lat.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_step_schedules_agree_bitwise(two_kernel):
    """One call, many short calls, and timed steps give the same state: replays of the 45-
    and 3-step graphs and single launches from every ring slot, with the closure checks that
    end each run (fused step), or of the 16- and 2-step graphs and single steps from either
    state buffer (two kernels)."""
    case = W.perturbed(45, 19, seed=9, kappa=0.0176)
    a = _lattice(case, two_kernel=two_kernel)
    a.step(100)
    b = _lattice(case, two_kernel=two_kernel)
    for n in (1, 2, 3, 1, 5, 17, 11, 60):
        b.step(n)
    c = _lattice(case, two_kernel=two_kernel)
    c.step_timed(5)
    c.step(95)
    assert a.steps_done() == b.steps_done() == c.steps_done() == 100
    fa, fb, fc = (_fields(x.moments()) for x in (a, b, c))
    assert np.array_equal(fa, fb) and np.array_equal(fa, fc)
    for x in (a, b, c):
        x.close()


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_timing_calls_leave_the_state_alone(two_kernel):
    """pond_time_kernel on both kernels and pond_step_timed: positive durations, and the
    state and step count afterwards are those of plain pond_step."""
    case = W.perturbed(40, 24, seed=12, kappa=0.0176)
    a = _lattice(case, two_kernel=two_kernel)
    a.step(12)
    b = _lattice(case, two_kernel=two_kernel)
    assert b.time_kernel(0, 3) > 0.0 and b.time_kernel(1, 3) > 0.0
    b.step(5)
    assert b.time_kernel(0, 2) > 0.0 and b.time_kernel(1, 2) > 0.0
    t = b.step_timed(7)
    assert all(v > 0.0 for v in t.values())
    assert a.steps_done() == b.steps_done() == 12
    assert np.array_equal(_fields(a.moments()), _fields(b.moments()))
    a.close()
    b.close()


def test_lattice_and_batch_close_at_the_end_of_a_with_block():
    case = W.perturbed(16, 12, seed=13)
    with pond.Lattice(pond_config(case)) as lat, pond.Batch() as batch:
        lat.init_fields(case.rho, case.u, case.T)
        batch.add(lat)
        assert batch.step(4) == [] and lat.steps_done() == 4
    assert lat._h is None and batch._h is None


def test_monitors_match_oracle_sums():
    case = W.static_droplet(n=48, radius=10.0)
    lat = _lattice(case)
    lat.step(10)
    mon = lat.monitors()
    lat.close()
    ref = run_oracle(case, 10)
    rho, E = ref["rho"], ref["E"]
    assert mon["mass"] == pytest.approx(np.sum(rho), rel=1e-13)
    assert mon["momentum"][0] == pytest.approx(np.sum(rho * ref["ux"]), abs=1e-12 * np.sum(rho))
    assert mon["energy"] == pytest.approx(np.sum(rho * E), rel=1e-13)
    assert mon["min_p"] == pytest.approx(np.min(ref["p"]), rel=1e-12)
    assert mon["energy_total"] > mon["energy"]
    assert 0.0 < mon["max_v_dt"] < 1.0


def test_init_outside_eos_domain_is_rejected():
    case = W.perturbed(16, 16, seed=1, rho0=3.5, t_over_tcr=0.5)   # p < 0 on the vdW loop
    lat = pond.Lattice(pond_config(case))
    with pytest.raises(pond.PondError) as err:
        lat.init_fields(case.rho, case.u, case.T)
    assert err.value.code == -4
    with pytest.raises(pond.PondError) as err:
        lat.step(1)
    assert err.value.code == -7
    lat.close()


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("field", ["rho", "ux", "uy", "T"])
def test_init_with_nonfinite_input_is_rejected(field, bad):
    """A NaN or Inf in any input field ends pond_init_fields with POND_E_NONFINITE."""
    case = W.perturbed(20, 18, seed=4)
    rho, u, T = case.rho.copy(), case.u.copy(), case.T.copy()
    target = {"rho": rho, "ux": u[0], "uy": u[1], "T": T}[field]
    target[57] = bad
    print(f"non-finite input: {field}[57] = {bad}", flush=True)
    lat = pond.Lattice(pond_config(case, tile=0))
    with pytest.raises(pond.PondError) as err:
        lat.init_fields(rho, u, T)
    assert err.value.code == -5, err.value
    with pytest.raises(pond.PondError) as err:
        lat.step(1)
    assert err.value.code == -7
    # the same handle accepts a finite state afterwards
    lat.init_fields(case.rho, case.u, case.T)
    lat.step(2)
    assert np.all(np.isfinite(lat.moments()["rho"]))
    lat.close()


def test_halo_violation_keeps_last_state():
    # |u| + sqrt(theta) > 1/dt: the departure stencil would leave the +-2 window
    case = W.perturbed(24, 24, seed=2, rho0=1.0, t_over_tcr=1.5, u0=(0.7, 0.0), dt=1.0, amp=0.0)
    lat = _lattice(case)
    before = _fields(lat.moments())
    with pytest.raises(pond.PondError) as err:
        lat.step(3)
    assert err.value.code == -6
    assert lat.steps_done() == 0
    assert np.array_equal(_fields(lat.moments()), before)
    with pytest.raises(pond.PondError) as err:
        lat.step(1)
    assert err.value.code == -7
    lat.close()


@pytest.mark.parametrize("two_kernel", [0, 1])
def test_failure_mid_run_keeps_the_last_completed_state(two_kernel):
    """A run that leaves the EoS domain in step 310 (serving job 1: 128^2, four droplets at
    0.85 T_cr) ends with POND_E_PRESSURE or POND_E_NONFINITE, whichever the failing state
    shows first, after 309 completed steps, and the handle holds bitwise the state of a run
    of exactly 309 steps.  The fused step finds a closure error in the state it reads, one
    step late, and steps back to the state before."""
    case = W.serving_jobs()[1][1]
    print(f"two_kernel {two_kernel}: serving job 1 {case.meta}", flush=True)
    a = _lattice(case, two_kernel=two_kernel)
    b = _lattice(case, two_kernel=two_kernel)
    try:
        a.step(300)
        with pytest.raises(pond.PondError) as err:
            a.step(40)
        print(f"   {err.value}", flush=True)
        assert err.value.code in (-4, -5), err.value
        assert "step 310" in str(err.value)
        assert a.steps_done() == 309
        b.step(309)
        assert np.array_equal(_fields(a.moments()), _fields(b.moments()))
    finally:
        a.close()
        b.close()


def test_autotuned_tile_is_valid_and_results_agree_to_roundoff():
    case = W.perturbed(64, 48, seed=12, kappa=0.0176)
    auto = _lattice(case, tile=-1)
    info = auto.tile_info()
    assert 0 <= info["variant"] < info["variants"] and info["tx"] * info["ty"] >= 64
    auto.step(20)
    fixed = _lattice(case, tile=(info["variant"] + 1) % info["variants"])
    fixed.step(20)
    a, b = auto.moments(), fixed.moments()
    for k in ("rho", "E"):
        assert np.max(np.abs(a[k] - b[k])) <= 1e-13 * np.max(np.abs(b[k]))
    auto.close()
    fixed.close()

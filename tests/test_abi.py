"""The C-ABI library loads, exports every entry point include/pond.h declares, validates
configurations before touching the device, and the binding fails loudly without it.
No compute call is made (these run without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2002_09217_amd import pond

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pond.h")


def declared_symbols():
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(pond_\w+)\s*\(", text, re.M)))


def test_header_declares_the_entry_points():
    names = declared_symbols()
    for required in ("pond_create", "pond_init_fields", "pond_step", "pond_moments", "pond_destroy"):
        assert required in names
    assert set(names) == set(pond.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = pond.load()
    out = subprocess.run(["nm", "-D", "--defined-only", pond.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(pond_\w+)", out))
    for name in declared_symbols():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_missing_library_raises(monkeypatch):
    monkeypatch.setattr(pond, "_lib", None)
    with pytest.raises(ImportError):
        pond.load("/nonexistent/libpond.so")


@pytest.mark.parametrize("field,value", [
    ("dim", 4), ("delta", 0.9), ("delta", 0.0), ("omega", 2.0), ("omega", 0.0), ("n_pass", 0),
    ("dt", 0.0), ("precision", 7),
])
def test_create_rejects_invalid_config_without_device(field, value):
    lib = pond.load()
    cfg = pond.Config(dim=2, n=(8, 8))
    c = cfg.to_c()
    setattr(c, field, value)
    h = ctypes.c_void_p()
    assert lib.pond_create(ctypes.byref(c), ctypes.byref(h)) == -1
    assert not h.value


def test_create_rejects_bad_sizes_and_boundaries():
    lib = pond.load()
    for n, bc in (((0, 8), 0), ((8, -1), 0), ((8, 8), 5)):
        c = pond.Config(dim=2, n=n).to_c()
        c.bc[0][0] = bc
        h = ctypes.c_void_p()
        assert lib.pond_create(ctypes.byref(c), ctypes.byref(h)) == -1


def test_null_arguments():
    lib = pond.load()
    assert lib.pond_destroy(None) == 0
    assert lib.pond_step(None, 1) == -1
    assert lib.pond_create(None, None) == -1
    assert lib.pond_last_error(None) == b"NULL handle"


@pytest.mark.parametrize("kw", [
    dict(eos=3, isothermal=1, T0=0.1),                                       # unknown law
    dict(eos=pond.EOS_DOUBLE_WELL, T0=0.1),                                  # needs isothermal
    dict(eos=pond.EOS_VDW, isothermal=1, T0=0.0),                            # T0 <= 0
    dict(eos=pond.EOS_DOUBLE_WELL, isothermal=1, T0=0.1, eos_c=(0.0, 5.0, 0.5, 0.1)),   # beta
    dict(eos=pond.EOS_DOUBLE_WELL, isothermal=1, T0=0.1, eos_c=(1e-3, 0.5, 5.0, 0.1)),  # rho_l < rho_v
    dict(eos=pond.EOS_DOUBLE_WELL, isothermal=1, T0=0.1, eos_c=(1e-3, 5.0, 0.5, -1.0)),  # p0
])
def test_create_rejects_invalid_equation_of_state_without_device(kw):
    lib = pond.load()
    c = pond.Config(dim=2, n=(8, 8), **kw).to_c()
    h = ctypes.c_void_p()
    assert lib.pond_create(ctypes.byref(c), ctypes.byref(h)) == -1
    assert not h.value


def test_create_rejects_three_dimensional_limits_without_device():
    lib = pond.load()
    for n, bc in (((1024, 1024, 1024), 0), ((8, 8, 8), 1)):   # > 2^29 nodes; an outflow face
        c = pond.Config(dim=3, n=n).to_c()
        for a in range(3):
            for s in range(2):
                c.bc[a][s] = bc
        h = ctypes.c_void_p()
        assert lib.pond_create(ctypes.byref(c), ctypes.byref(h)) == -1


def test_node_count_limits_without_device():
    """1D and 2D lattices up to 2^30 nodes are accepted (the kernels index planes with
    64-bit offsets), one node more is refused; pond_footprint validates like pond_create."""
    lib = pond.load()
    v = ctypes.c_ulonglong()
    for dim, ok, too_big in ((2, (32768, 32768), (32768, 32769)), (1, (1 << 30,), ((1 << 30) + 1,))):
        c = pond.Config(dim=dim, n=ok).to_c()
        assert lib.pond_footprint(ctypes.byref(c), ctypes.byref(v)) == 0
        assert v.value > (1 << 30) * (2 * 5 * 8)       # at least the side planes of both states
        c = pond.Config(dim=dim, n=too_big).to_c()
        assert lib.pond_footprint(ctypes.byref(c), ctypes.byref(v)) == -1
        h = ctypes.c_void_p()
        assert lib.pond_create(ctypes.byref(c), ctypes.byref(h)) == -1


def test_noalloc_entry_point_validates_without_device():
    """pond_step_noalloc refuses bad arguments and lattices beyond its static scratch before
    it touches a device."""
    lib = pond.load()
    cur, done = ctypes.c_int(0), ctypes.c_int(-1)
    c = pond.Config(dim=2, n=(700, 700), tile=0, two_kernel=1).to_c()  # 4096 + 144 * 490000 B > 64 MiB
    assert lib.pond_step_noalloc(ctypes.byref(c), 64, 64, ctypes.byref(cur), 1, ctypes.byref(done)) == -8
    assert cur.value == 0 and done.value == 0
    c = pond.Config(dim=3, n=(8, 8, 8), tile=0, two_kernel=1).to_c()
    assert lib.pond_step_noalloc(ctypes.byref(c), 64, 64, ctypes.byref(cur), 1, None) == -1
    c = pond.Config(dim=2, n=(16, 16), tile=0).to_c()                 # the fused step: refused
    assert lib.pond_step_noalloc(ctypes.byref(c), 64, 64, ctypes.byref(cur), 1, None) == -1
    c = pond.Config(dim=2, n=(16, 16), tile=0, two_kernel=1).to_c()
    assert lib.pond_step_noalloc(ctypes.byref(c), None, 64, ctypes.byref(cur), 1, None) == -1
    assert lib.pond_step_noalloc(ctypes.byref(c), 64, 64, ctypes.byref(cur), -1, None) == -1
    assert lib.pond_step_noalloc(None, 64, 64, ctypes.byref(cur), 1, None) == -1

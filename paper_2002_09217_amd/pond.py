"""Python binding of libpond (include/pond.h): argument marshalling only.

Every step of the method runs in the HIP kernels of libpond.so; this module only
converts numpy arrays and Python values into the C ABI.  There is no fallback: a
missing or unloadable library raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpond.so")

POND_OK = 0
STATUS = {
    0: "POND_OK", -1: "POND_E_INVALID", -2: "POND_E_NOMEM", -3: "POND_E_DEVICE",
    -4: "POND_E_PRESSURE", -5: "POND_E_NONFINITE", -6: "POND_E_HALO", -7: "POND_E_STATE",
    -8: "POND_E_SCRATCH",
}
BC_PERIODIC, BC_OUTFLOW, BC_INFLOW = 0, 1, 2
FP64, FP32_STORE, FP32_STORE_FP64_MATH = 0, 1, 2
EOS_VDW, EOS_DIETERICI, EOS_DOUBLE_WELL = 0, 1, 2

# kernel ids of pond_time_kernel
K_STREAM, K_FORCE_COLLIDE = 0, 1
KERNEL_NAMES = {K_STREAM: "k_stream", K_FORCE_COLLIDE: "k_force_collide"}

EXPORTED = ["pond_create", "pond_init_fields", "pond_step", "pond_moments", "pond_monitors",
            "pond_steps_done", "pond_last_error", "pond_destroy", "pond_time_kernel",
            "pond_step_timed", "pond_tile_info", "pond_footprint", "pond_batch_create",
            "pond_batch_add", "pond_batch_remove", "pond_batch_step", "pond_batch_size",
            "pond_batch_destroy", "pond_checkpoint_size", "pond_save", "pond_load", "pond_step_noalloc"]


class pond_config(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("bc", (ctypes.c_int * 2) * 3),
        ("inflow", ((ctypes.c_double * 5) * 2) * 3),
        ("a", ctypes.c_double),
        ("b", ctypes.c_double),
        ("R", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("eos", ctypes.c_int),
        ("isothermal", ctypes.c_int),
        ("T0", ctypes.c_double),
        ("eos_c", ctypes.c_double * 4),
        ("omega", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("k_scale", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("n_pass", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("tile", ctypes.c_int),
        ("two_kernel", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


class PondError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str = ""):
        super().__init__(f"{where}: {STATUS.get(code, code)} {msg}".strip())
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libpond.so; raises when it is missing (build it with paper_2002_09217_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2002_09217_amd.build`")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (soname
    # libamdhip64.so.7), which libpond then binds to instead of loading a second copy;
    # PyTorch's streams and memory are then valid handles for libpond.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    hp = ctypes.c_void_p
    L.pond_create.argtypes = [ctypes.POINTER(pond_config), ctypes.POINTER(hp)]
    L.pond_init_fields.argtypes = [hp, dp, dp, dp]
    L.pond_step.argtypes = [hp, ctypes.c_int]
    L.pond_moments.argtypes = [hp, dp, dp, dp, dp, dp]
    L.pond_monitors.argtypes = [hp, dp]
    L.pond_steps_done.argtypes = [hp, ctypes.POINTER(ctypes.c_longlong)]
    L.pond_last_error.argtypes = [hp]
    L.pond_last_error.restype = ctypes.c_char_p
    L.pond_destroy.argtypes = [hp]
    L.pond_time_kernel.argtypes = [hp, ctypes.c_int, ctypes.c_int, dp]
    L.pond_step_timed.argtypes = [hp, ctypes.c_int, dp]
    L.pond_tile_info.argtypes = [hp, ctypes.POINTER(ctypes.c_int)]
    L.pond_footprint.argtypes = [ctypes.POINTER(pond_config), ctypes.POINTER(ctypes.c_ulonglong)]
    L.pond_batch_create.argtypes = [ctypes.c_void_p, ctypes.POINTER(hp)]
    L.pond_batch_add.argtypes = [hp, hp]
    L.pond_batch_remove.argtypes = [hp, hp]
    L.pond_batch_step.argtypes = [hp, ctypes.c_int]
    L.pond_batch_size.argtypes = [hp, ctypes.POINTER(ctypes.c_int)]
    L.pond_batch_destroy.argtypes = [hp]
    L.pond_checkpoint_size.argtypes = [hp, ctypes.POINTER(ctypes.c_ulonglong)]
    L.pond_save.argtypes = [hp, ctypes.c_void_p, ctypes.c_ulonglong]
    L.pond_load.argtypes = [hp, ctypes.c_void_p, ctypes.c_ulonglong]
    L.pond_step_noalloc.argtypes = [ctypes.POINTER(pond_config), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    for name in EXPORTED:
        getattr(L, name).restype = getattr(L, name).restype or ctypes.c_int
    L.pond_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Config:
    """Mirror of pond_config (lattice units: dx = 1)."""
    dim: int = 2
    n: tuple = (64, 64)
    bc: tuple = ((BC_PERIODIC, BC_PERIODIC), (BC_PERIODIC, BC_PERIODIC))
    inflow: tuple = ()          # ((axis, side, (rho, ux, uy, T)), ...)
    a: float = 2.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    delta: float = 1.0 / 3.0
    omega: float = 1.5
    kappa: float = 0.0
    k_scale: float = 1.0
    dt: float = 0.2
    n_pass: int = 2
    eos: int = 0                # EOS_VDW, EOS_DIETERICI, EOS_DOUBLE_WELL
    isothermal: int = 0         # nonzero: T = T0 everywhere (required unless EOS_VDW)
    T0: float = 0.0
    eos_c: tuple = (0.0, 0.0, 0.0, 0.0)   # EOS_DOUBLE_WELL: beta, rho_l, rho_v, p0
    precision: int = FP64
    tile: int = -1              # streaming tile shape; -1: measured at the first init
    two_kernel: int = 0         # 1D/2D: 0 = fused one-kernel step, 1 = two kernels, stored populations
    stream: int | None = None   # hipStream_t as an integer (e.g. torch's cuda_stream)

    def to_c(self) -> pond_config:
        c = pond_config()
        c.dim = self.dim
        n = tuple(self.n) + (1,) * (3 - len(self.n))
        for i in range(3):
            c.n[i] = int(n[i])
        for a in range(min(self.dim, len(self.bc), 3)):
            for s in range(2):
                c.bc[a][s] = int(self.bc[a][s])
        for a, s, st in self.inflow:
            rho, ux, uy, T = st
            vals = (rho, ux, uy, 0.0, T)
            for k in range(5):
                c.inflow[a][s][k] = float(vals[k])
        c.a, c.b, c.R, c.delta = self.a, self.b, self.R, self.delta
        c.eos, c.isothermal, c.T0 = int(self.eos), int(self.isothermal), float(self.T0)
        for i in range(4):
            c.eos_c[i] = float(self.eos_c[i])
        c.omega, c.kappa, c.k_scale, c.dt = self.omega, self.kappa, self.k_scale, self.dt
        c.n_pass, c.precision, c.tile = self.n_pass, self.precision, self.tile
        c.two_kernel = int(self.two_kernel)
        c.stream = self.stream
        return c

    @property
    def N(self) -> int:
        return int(np.prod(self.n[: self.dim]))


def footprint(cfg: Config) -> int:
    """Device bytes pond_create allocates for cfg."""
    c = cfg.to_c()
    v = ctypes.c_ulonglong()
    rc = load().pond_footprint(ctypes.byref(c), ctypes.byref(v))
    if rc != POND_OK:
        raise PondError(rc, "pond_footprint")
    return int(v.value)


def step_noalloc(cfg: Config, state0: int, state1: int, cur: int, nsteps: int):
    """pond_step_noalloc on two caller-owned device state buffers (device addresses as
    integers).  Returns (status, buffer holding the last completed state, steps done)."""
    c = cfg.to_c()
    cc, done = ctypes.c_int(cur), ctypes.c_int()
    rc = load().pond_step_noalloc(ctypes.byref(c), state0, state1, ctypes.byref(cc), int(nsteps),
                                  ctypes.byref(done))
    return rc, cc.value, done.value


@dataclass(eq=False)
class Lattice:
    """One libpond handle (compared and hashed by identity)."""
    cfg: Config
    _h: ctypes.c_void_p = field(default=None, init=False, repr=False)

    def __post_init__(self):
        L = load()
        self._c = self.cfg.to_c()
        h = ctypes.c_void_p()
        rc = L.pond_create(ctypes.byref(self._c), ctypes.byref(h))
        if rc != POND_OK:
            raise PondError(rc, "pond_create")
        self._h = h

    def _check(self, rc: int, where: str):
        if rc != POND_OK:
            raise PondError(rc, where, load().pond_last_error(self._h).decode())

    def init_fields(self, rho, u, T):
        N, dim = self.cfg.N, self.cfg.dim
        rho = np.ascontiguousarray(rho, dtype=np.float64).ravel()
        u = np.ascontiguousarray(u, dtype=np.float64).ravel()
        T = np.ascontiguousarray(T, dtype=np.float64).ravel()
        if rho.size != N or T.size != N or u.size != dim * N:
            raise ValueError("field sizes do not match the lattice")
        self._check(load().pond_init_fields(self._h, _dp(rho), _dp(u), _dp(T)), "pond_init_fields")
        return self

    def step(self, n: int = 1):
        self._check(load().pond_step(self._h, int(n)), "pond_step")
        return self

    def moments(self) -> dict:
        N, dim = self.cfg.N, self.cfg.dim
        rho, u, T, p, E = np.empty(N), np.empty(dim * N), np.empty(N), np.empty(N), np.empty(N)
        self._check(load().pond_moments(self._h, _dp(rho), _dp(u), _dp(T), _dp(p), _dp(E)), "pond_moments")
        out = {"rho": rho, "ux": u[:N], "T": T, "p": p, "E": E}
        out["uy"] = u[N:2 * N] if dim >= 2 else np.zeros(N)
        if dim == 3:
            out["uz"] = u[2 * N:]
        return out

    def monitors(self) -> dict:
        dim = self.cfg.dim
        out = np.empty(dim + 5)
        self._check(load().pond_monitors(self._h, _dp(out)), "pond_monitors")
        return {"mass": out[0], "momentum": out[1:1 + dim].copy(), "energy": out[dim + 1],
                "energy_total": out[dim + 2], "min_p": out[dim + 3], "max_v_dt": out[dim + 4]}

    def steps_done(self) -> int:
        v = ctypes.c_longlong()
        self._check(load().pond_steps_done(self._h, ctypes.byref(v)), "pond_steps_done")
        return v.value

    def time_kernel(self, which: int, reps: int) -> float:
        """Mean duration of one launch of a kernel in microseconds (HIP events)."""
        us = ctypes.c_double()
        self._check(load().pond_time_kernel(self._h, int(which), int(reps), ctypes.byref(us)),
                    "pond_time_kernel")
        return us.value

    @property
    def fused(self) -> bool:
        """One fused kernel per step (1D/2D lattices without two_kernel)."""
        return self.cfg.dim != 3 and not self.cfg.two_kernel

    def step_timed(self, n: int) -> dict:
        """Advance n steps with HIP events around every kernel launch; mean microseconds
        per launch of each kernel inside the step pipeline (k_step for the fused step)."""
        out = np.zeros(2)
        self._check(load().pond_step_timed(self._h, int(n), _dp(out)), "pond_step_timed")
        if self.fused:
            return {"k_step": float(out[0])}
        return {KERNEL_NAMES[K_STREAM]: float(out[0]), KERNEL_NAMES[K_FORCE_COLLIDE]: float(out[1])}

    def tile_info(self) -> dict:
        out = (ctypes.c_int * 4)()
        self._check(load().pond_tile_info(self._h, out), "pond_tile_info")
        return {"variant": out[0], "tx": out[1], "ty": out[2], "variants": out[3]}

    def last_error(self) -> str:
        return load().pond_last_error(self._h).decode()

    def save(self) -> bytes:
        """Checkpoint of the current state (pond_save)."""
        n = ctypes.c_ulonglong()
        self._check(load().pond_checkpoint_size(self._h, ctypes.byref(n)), "pond_checkpoint_size")
        buf = ctypes.create_string_buffer(n.value)
        self._check(load().pond_save(self._h, buf, n.value), "pond_save")
        return buf.raw

    def load(self, data: bytes):
        """Make a checkpoint the current state (pond_load)."""
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        self._check(load().pond_load(self._h, buf, len(data)), "pond_load")
        return self

    def close(self):
        if self._h is not None:
            if getattr(self, "_batch", None) is not None:   # pond_destroy leaves the batch
                self._batch.members.remove(self)
                self._batch = None
            load().pond_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A libpond batch: member lattices advanced together, each bitwise as alone."""

    def __init__(self, stream: int | None = None):
        h = ctypes.c_void_p()
        rc = load().pond_batch_create(stream, ctypes.byref(h))
        if rc != POND_OK:
            raise PondError(rc, "pond_batch_create")
        self._h = h
        self.members: list[Lattice] = []

    def add(self, lat: Lattice):
        rc = load().pond_batch_add(self._h, lat._h)
        if rc != POND_OK:
            raise PondError(rc, "pond_batch_add", lat.last_error() if rc != -1 else "")
        self.members.append(lat)
        lat._batch = self
        return self

    def remove(self, lat: Lattice):
        rc = load().pond_batch_remove(self._h, lat._h)
        if rc != POND_OK:
            raise PondError(rc, "pond_batch_remove")
        self.members.remove(lat)
        lat._batch = None
        return self

    def step(self, n: int = 1) -> list:
        """Advance every member n steps; returns the members that failed (they have left
        the batch and are in the error state, as after a failed Lattice.step)."""
        before = [m.steps_done() for m in self.members]
        rc = load().pond_batch_step(self._h, int(n))
        if rc == POND_OK:
            return []
        if rc in (-1, -2, -3):
            raise PondError(rc, "pond_batch_step")
        failed = [m for m, b in zip(self.members, before) if m.steps_done() - b < n]
        for m in failed:
            m._batch = None
        self.members = [m for m in self.members if m not in failed]
        return failed

    def size(self) -> int:
        v = ctypes.c_int()
        rc = load().pond_batch_size(self._h, ctypes.byref(v))
        if rc != POND_OK:
            raise PondError(rc, "pond_batch_size")
        return v.value

    def close(self):
        if self._h is not None:
            load().pond_batch_destroy(self._h)
            self._h = None
            for m in self.members:
                m._batch = None
            self.members = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

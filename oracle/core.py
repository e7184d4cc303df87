"""TEST INFRASTRUCTURE ONLY -- ctypes front end of the FP64 CPU oracle (pond_oracle.c).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The product path never does.

The oracle integrates the two-population Particles-on-Demand model of
Reyhanian, Dorschner & Karlin (arXiv:2002.09217) in the paper's own order;
see the header of ``pond_oracle.c`` for the equations followed and for the
readings of the points the paper leaves open.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pond_oracle.c")
SRC3 = os.path.join(HERE, "pond_oracle3.c")
LIB = os.path.join(HERE, "liboracle.so")

PERIODIC, OUTFLOW, INFLOW = 0, 1, 2

ERRORS = {0: "ok", -1: "invalid", -2: "nomem", -4: "pressure", -5: "nonfinite"}


def build(force: bool = True) -> str:
    """Compile the oracle with FMA contraction disabled (plain IEEE FP64)."""
    if force or _stale():
        tmp = LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c99",
            "-Wall", "-Wno-unused-function", "-shared", "-fPIC", SRC, SRC3, "-o", tmp, "-lm",
        ])
        os.replace(tmp, LIB)
    return LIB


def _stale() -> bool:
    return not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC), os.path.getmtime(SRC3))


EOS_VDW, EOS_DIETERICI, EOS_WELL = 0, 1, 2


class Eos(ctypes.Structure):
    """Equation of state of a run (orc_eos): kind, isothermal switch with T0, and the
    double-well constants (beta, rho_l, rho_v, p0)."""
    _fields_ = [("kind", ctypes.c_int), ("isothermal", ctypes.c_int), ("T0", ctypes.c_double),
                ("c", ctypes.c_double * 4)]


def _eos(kind, isothermal, T0, c) -> Eos:
    e = Eos()
    e.kind, e.isothermal, e.T0 = int(kind), int(isothermal), float(T0)
    for i in range(4):
        e.c[i] = float(c[i])
    return e


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("bc", (ctypes.c_int * 2) * 2),
        ("inflow", ((ctypes.c_double * 4) * 2) * 2),
        ("a", ctypes.c_double),
        ("b", ctypes.c_double),
        ("R", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("k_scale", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("n_pass", ctypes.c_int),
        ("eos", Eos),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Params)
        L.orc_transfer_1d.argtypes = [ctypes.c_double] * 4 + [dp]
        L.orc_transfer_pop.argtypes = [pp, dp, dp, dp, dp]
        L.orc_lagrange4.argtypes = [ctypes.c_double, dp]
        L.orc_force_source.argtypes = [pp, ctypes.c_double, dp, ctypes.c_double, dp, dp]
        L.orc_geq.argtypes = [pp, ctypes.c_double, dp, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, dp, dp, dp]
        L.orc_psi.argtypes = [pp, ctypes.c_double, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_collide.argtypes = [pp, dp, dp, dp, dp, ctypes.c_double, dp, dp, dp]
        L.orc_collide.restype = ctypes.c_int
        L.orc_init.argtypes = [pp] + [dp] * 11
        L.orc_init.restype = ctypes.c_int
        L.orc_step.argtypes = [pp, ctypes.c_int] + [dp] * 7 + [ctypes.POINTER(ctypes.c_int), dp]
        L.orc_step.restype = ctypes.c_int
        L.orc_moments.argtypes = [pp] + [dp] * 12
        L.orc_korteweg_force.argtypes = [pp, dp, dp, dp]
        L.orc_heat_correction.argtypes = [pp] + [dp] * 5
        p3 = ctypes.POINTER(Params3)
        L.orc3_transfer_pop.argtypes = [dp, dp, dp, dp]
        L.orc3_force_source.argtypes = [ctypes.c_double, dp, ctypes.c_double, dp, dp]
        L.orc3_geq.argtypes = [p3, ctypes.c_double, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               dp, dp, dp]
        L.orc3_psi.argtypes = [ctypes.c_double, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc3_collide.argtypes = [p3, dp, dp, dp, dp, ctypes.c_double, dp, dp, dp]
        L.orc3_collide.restype = ctypes.c_int
        L.orc3_init.argtypes = [p3] + [dp] * 8
        L.orc3_init.restype = ctypes.c_int
        L.orc3_step.argtypes = [p3, ctypes.c_int] + [dp] * 5 + [ctypes.POINTER(ctypes.c_int)]
        L.orc3_step.restype = ctypes.c_int
        L.orc3_moments.argtypes = [p3] + [dp] * 9
        L.orc3_korteweg_force.argtypes = [p3, dp, dp]
        L.orc3_heat_correction.argtypes = [p3] + [dp] * 5
        pe = ctypes.POINTER(Eos)
        d = ctypes.c_double
        for name in ("orc_eos_e", "orc_eos_cv", "orc_eos_T_of_e"):
            getattr(L, name).argtypes = [pe, d, d, d, d, d, d]
            getattr(L, name).restype = d
        L.orc_eos_T_of_p.argtypes = [pe, d, d, d, d, d]
        L.orc_eos_T_of_p.restype = d
        L.orc_eos_p.argtypes = [pe, d, d, d, d, d]
        L.orc_eos_p.restype = d
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


@dataclass
class Config:
    """Physical and numerical parameters of one run (lattice units, dx = dt = 1)."""
    dim: int = 2
    nx: int = 32
    ny: int = 32
    bc: tuple = ((PERIODIC, PERIODIC), (PERIODIC, PERIODIC))
    inflow: tuple = (((0.0,) * 4, (0.0,) * 4), ((0.0,) * 4, (0.0,) * 4))
    a: float = 2.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    delta: float = 1.0 / 3.0
    omega: float = 1.5
    kappa: float = 0.0
    k_scale: float = 1.0
    dt: float = 1.0
    n_pass: int = 2
    eos: int = EOS_VDW          # EOS_VDW, EOS_DIETERICI, EOS_WELL (isothermal)
    isothermal: int = 0         # nonzero: T = T0 everywhere
    T0: float = 0.0
    eos_c: tuple = (0.0, 0.0, 0.0, 0.0)   # EOS_WELL: beta, rho_l, rho_v, p0

    def params(self) -> Params:
        P = Params()
        P.dim, P.nx, P.ny = self.dim, self.nx, (self.ny if self.dim == 2 else 1)
        for ax in range(2):
            for s in range(2):
                P.bc[ax][s] = int(self.bc[ax][s])
                for k in range(4):
                    P.inflow[ax][s][k] = float(self.inflow[ax][s][k])
        P.a, P.b, P.R, P.delta = self.a, self.b, self.R, self.delta
        P.omega, P.kappa, P.k_scale, P.dt = self.omega, self.kappa, self.k_scale, self.dt
        P.n_pass = self.n_pass
        P.eos = _eos(self.eos, self.isothermal, self.T0, self.eos_c)
        return P

    @property
    def Q(self) -> int:
        return 9 if self.dim == 2 else 3

    @property
    def N(self) -> int:
        return self.nx * (self.ny if self.dim == 2 else 1)


class OracleError(RuntimeError):
    pass


def _eos_call(name, cfg: Config, *args) -> float:
    E = _eos(cfg.eos, cfg.isothermal, cfg.T0, cfg.eos_c)
    return getattr(lib(), name)(ctypes.byref(E), *[float(x) for x in args])


def eos_p(cfg: Config, rho, T) -> float:
    """Pressure p(rho, T) of the run's equation of state (orc_eos_p)."""
    return _eos_call("orc_eos_p", cfg, cfg.a, cfg.b, cfg.R, rho, T)


def eos_e(cfg: Config, rho, T) -> float:
    """Internal energy e(rho, T) (orc_eos_e; Dieterici by quadrature)."""
    return _eos_call("orc_eos_e", cfg, cfg.a, cfg.b, cfg.R, cfg.R / cfg.delta, rho, T)


def eos_cv(cfg: Config, rho, T) -> float:
    """(de/dT)_rho of a state (orc_eos_cv)."""
    return _eos_call("orc_eos_cv", cfg, cfg.a, cfg.b, cfg.R, cfg.R / cfg.delta, rho, T)


def eos_T_of_e(cfg: Config, rho, e) -> float:
    """Temperature of a state from its internal energy (orc_eos_T_of_e)."""
    return _eos_call("orc_eos_T_of_e", cfg, cfg.a, cfg.b, cfg.R, cfg.R / cfg.delta, rho, e)


def eos_T_of_p(cfg: Config, rho, p) -> float:
    """Temperature of a state from its pressure (orc_eos_T_of_p)."""
    return _eos_call("orc_eos_T_of_p", cfg, cfg.a, cfg.b, cfg.R, rho, p)


@dataclass
class Sim:
    """State of the oracle: post-collision populations in each node's gauge."""
    cfg: Config
    f: np.ndarray = field(init=False)
    g: np.ndarray = field(init=False)
    ux: np.ndarray = field(init=False)
    uy: np.ndarray = field(init=False)
    th: np.ndarray = field(init=False)
    Fx: np.ndarray = field(init=False)
    Fy: np.ndarray = field(init=False)
    steps: int = 0
    last_resid: float = 0.0

    def __post_init__(self):
        Q, N = self.cfg.Q, self.cfg.N
        self.f = np.zeros((Q, N))
        self.g = np.zeros((Q, N))
        self.ux, self.uy, self.th = np.zeros(N), np.zeros(N), np.zeros(N)
        self.Fx, self.Fy = np.zeros(N), np.zeros(N)
        self._P = self.cfg.params()

    def init(self, rho, ux, T, uy=None):
        N = self.cfg.N
        rho, ux, T = _arr(rho, N), _arr(ux, N), _arr(T, N)
        uy = _arr(np.zeros(N) if uy is None else uy, N)
        rc = lib().orc_init(ctypes.byref(self._P), _p(rho), _p(ux), _p(uy), _p(T), _p(self.f),
                            _p(self.g), _p(self.ux), _p(self.uy), _p(self.th), _p(self.Fx),
                            _p(self.Fy))
        if rc:
            raise OracleError(f"orc_init: {ERRORS.get(rc, rc)}")
        self.steps = 0
        return self

    def step(self, n: int = 1):
        done = ctypes.c_int(0)
        res = ctypes.c_double(0.0)
        rc = lib().orc_step(ctypes.byref(self._P), int(n), _p(self.f), _p(self.g), _p(self.ux),
                            _p(self.uy), _p(self.th), _p(self.Fx), _p(self.Fy),
                            ctypes.byref(done), ctypes.byref(res))
        self.steps += done.value
        self.last_resid = res.value
        if rc:
            raise OracleError(f"orc_step: {ERRORS.get(rc, rc)} after {done.value} steps")
        return self

    def moments(self) -> dict:
        N = self.cfg.N
        out = {k: np.zeros(N) for k in ("rho", "ux", "uy", "T", "p", "E")}
        lib().orc_moments(ctypes.byref(self._P), _p(self.f), _p(self.ux), _p(self.uy),
                          _p(self.th), _p(self.Fx), _p(self.Fy), _p(out["rho"]), _p(out["ux"]),
                          _p(out["uy"]), _p(out["T"]), _p(out["p"]), _p(out["E"]))
        return out


# ---------------------------------------------------------------------------
# single-node helpers exposed for the unit pins
# ---------------------------------------------------------------------------
def transfer_1d(u_from, th_from, u_to, th_to) -> np.ndarray:
    G = np.zeros((3, 3))
    lib().orc_transfer_1d(u_from, th_from, u_to, th_to, _p(G))
    return G


def transfer_pop(cfg: Config, lam_from, lam_to, fin) -> np.ndarray:
    P = cfg.params()
    lf, lt, fi = _arr(lam_from, 3), _arr(lam_to, 3), _arr(fin, cfg.Q)
    out = np.zeros(cfg.Q)
    lib().orc_transfer_pop(ctypes.byref(P), _p(lf), _p(lt), _p(fi), _p(out))
    return out


def lagrange4(t: float) -> np.ndarray:
    w = np.zeros(4)
    lib().orc_lagrange4(float(t), _p(w))
    return w


def force_source(cfg: Config, rho, u, theta, du) -> np.ndarray:
    P = cfg.params()
    S = np.zeros(cfg.Q)
    lib().orc_force_source(ctypes.byref(P), rho, _p(_arr(u, 2)), theta, _p(_arr(du, 2)), _p(S))
    return S


def geq(cfg: Config, rho, u, theta, p, E, uh, F) -> np.ndarray:
    P = cfg.params()
    g = np.zeros(cfg.Q)
    lib().orc_geq(ctypes.byref(P), rho, _p(_arr(u, 2)), theta, p, E, _p(_arr(uh, 2)),
                  _p(_arr(F, 2)), _p(g))
    return g


def psi(cfg: Config, rho, u, theta, p) -> np.ndarray:
    P = cfg.params()
    out = np.zeros(cfg.Q)
    lib().orc_psi(ctypes.byref(P), rho, _p(_arr(u, 2)), theta, p, _p(out))
    return out


def collide(cfg: Config, lam_str, fstr, gstr, F, M0):
    P = cfg.params()
    fo, go, lo = np.zeros(cfg.Q), np.zeros(cfg.Q), np.zeros(3)
    rc = lib().orc_collide(ctypes.byref(P), _p(_arr(lam_str, 3)), _p(_arr(fstr, cfg.Q)),
                           _p(_arr(gstr, cfg.Q)), _p(_arr(F, 2)), float(M0), _p(fo), _p(go),
                           _p(lo))
    if rc:
        raise OracleError(f"orc_collide: {ERRORS.get(rc, rc)}")
    return fo, go, lo


def korteweg_force(cfg: Config, rho):
    """F = -div K of a density field (eq. 18 and App. F), on the config's lattice."""
    P = cfg.params()
    r = _arr(rho, cfg.N)
    Fx, Fy = np.zeros(cfg.N), np.zeros(cfg.N)
    lib().orc_korteweg_force(ctypes.byref(P), _p(r), _p(Fx), _p(Fy))
    return Fx, Fy


def heat_correction(cfg: Config, T, h, mu, kc):
    """M0 = 2 div(-mu grad h + k grad T) in flux form (eq. 9)."""
    P = cfg.params()
    out = np.zeros(cfg.N)
    lib().orc_heat_correction(ctypes.byref(P), _p(_arr(T, cfg.N)), _p(_arr(h, cfg.N)),
                              _p(_arr(mu, cfg.N)), _p(_arr(kc, cfg.N)), _p(out))
    return out


def velocities(cfg: Config, lam) -> np.ndarray:
    """Discrete velocities v_i = sqrt(theta) c_i + u of a gauge (eq. 1), shape (Q, 2)."""
    s = np.sqrt(lam[2])
    if cfg.dim == 1:
        return np.array([[lam[0] + s * c, 0.0] for c in (-1, 0, 1)])
    return np.array([[lam[0] + s * cx, lam[1] + s * cy] for cx in (-1, 0, 1) for cy in (-1, 0, 1)])


def weights(cfg: Config) -> np.ndarray:
    w1 = np.array([1 / 6, 2 / 3, 1 / 6])
    return w1 if cfg.dim == 1 else np.outer(w1, w1).ravel()



# ---------------------------------------------------------------------------
# three dimensions (D3Q27, periodic box; pond_oracle3.c)
# ---------------------------------------------------------------------------
class Params3(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double), ("delta", ctypes.c_double),
        ("omega", ctypes.c_double), ("kappa", ctypes.c_double), ("k_scale", ctypes.c_double),
        ("dt", ctypes.c_double), ("n_pass", ctypes.c_int), ("eos", Eos),
    ]


@dataclass
class Config3:
    """Parameters of a run on a periodic nx x ny x nz box (lattice units)."""
    nx: int = 8
    ny: int = 8
    nz: int = 8
    a: float = 2.0 / 49.0
    b: float = 2.0 / 21.0
    R: float = 1.0
    delta: float = 1.0 / 3.0
    omega: float = 1.5
    kappa: float = 0.0
    k_scale: float = 1.0
    dt: float = 1.0
    n_pass: int = 2
    eos: int = EOS_VDW
    isothermal: int = 0
    T0: float = 0.0
    eos_c: tuple = (0.0, 0.0, 0.0, 0.0)

    def params(self) -> Params3:
        P = Params3()
        P.nx, P.ny, P.nz = self.nx, self.ny, self.nz
        P.a, P.b, P.R, P.delta = self.a, self.b, self.R, self.delta
        P.omega, P.kappa, P.k_scale, P.dt, P.n_pass = self.omega, self.kappa, self.k_scale, self.dt, self.n_pass
        P.eos = _eos(self.eos, self.isothermal, self.T0, self.eos_c)
        return P

    Q = 27

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class Sim3:
    """D3Q27 oracle state: populations (27 planes each), gauge u (3 planes), theta, F (3 planes)."""
    cfg: Config3
    steps: int = 0

    def __post_init__(self):
        N = self.cfg.N
        self.f, self.g = np.zeros((27, N)), np.zeros((27, N))
        self.u, self.th, self.F = np.zeros((3, N)), np.zeros(N), np.zeros((3, N))
        self._P = self.cfg.params()

    def init(self, rho, uh, T):
        N = self.cfg.N
        rc = lib().orc3_init(ctypes.byref(self._P), _p(_arr(rho, N)), _p(_arr(uh, 3 * N)), _p(_arr(T, N)),
                             _p(self.f), _p(self.g), _p(self.u), _p(self.th), _p(self.F))
        if rc:
            raise OracleError(f"orc3_init: {ERRORS.get(rc, rc)}")
        self.steps = 0
        return self

    def step(self, n: int = 1):
        done = ctypes.c_int(0)
        rc = lib().orc3_step(ctypes.byref(self._P), int(n), _p(self.f), _p(self.g), _p(self.u), _p(self.th),
                             _p(self.F), ctypes.byref(done))
        self.steps += done.value
        if rc:
            raise OracleError(f"orc3_step: {ERRORS.get(rc, rc)} after {done.value} steps")
        return self

    def moments(self) -> dict:
        N = self.cfg.N
        rho, uh, T, p, E = np.zeros(N), np.zeros((3, N)), np.zeros(N), np.zeros(N), np.zeros(N)
        lib().orc3_moments(ctypes.byref(self._P), _p(self.f), _p(self.u), _p(self.th), _p(self.F), _p(rho),
                           _p(uh), _p(T), _p(p), _p(E))
        return {"rho": rho, "ux": uh[0], "uy": uh[1], "uz": uh[2], "T": T, "p": p, "E": E}


def transfer3_pop(lam_from, lam_to, fin) -> np.ndarray:
    out = np.zeros(27)
    lib().orc3_transfer_pop(_p(_arr(lam_from, 4)), _p(_arr(lam_to, 4)), _p(_arr(fin, 27)), _p(out))
    return out


def force_source3(rho, u, theta, du) -> np.ndarray:
    S = np.zeros(27)
    lib().orc3_force_source(rho, _p(_arr(u, 3)), theta, _p(_arr(du, 3)), _p(S))
    return S


def geq3(cfg: Config3, rho, u, theta, p, E, uh, F) -> np.ndarray:
    P = cfg.params()
    g = np.zeros(27)
    lib().orc3_geq(ctypes.byref(P), rho, _p(_arr(u, 3)), theta, p, E, _p(_arr(uh, 3)), _p(_arr(F, 3)), _p(g))
    return g


def psi3(rho, u, theta, p) -> np.ndarray:
    out = np.zeros(27)
    lib().orc3_psi(rho, _p(_arr(u, 3)), theta, p, _p(out))
    return out


def collide3(cfg: Config3, lam_str, fstr, gstr, F, M0):
    P = cfg.params()
    fo, go, lo = np.zeros(27), np.zeros(27), np.zeros(4)
    rc = lib().orc3_collide(ctypes.byref(P), _p(_arr(lam_str, 4)), _p(_arr(fstr, 27)), _p(_arr(gstr, 27)),
                            _p(_arr(F, 3)), float(M0), _p(fo), _p(go), _p(lo))
    if rc:
        raise OracleError(f"orc3_collide: {ERRORS.get(rc, rc)}")
    return fo, go, lo


def korteweg_force3(cfg: Config3, rho) -> np.ndarray:
    P = cfg.params()
    F = np.zeros((3, cfg.N))
    lib().orc3_korteweg_force(ctypes.byref(P), _p(_arr(rho, cfg.N)), _p(F))
    return F


def heat_correction3(cfg: Config3, T, h, mu, kc) -> np.ndarray:
    P = cfg.params()
    out = np.zeros(cfg.N)
    lib().orc3_heat_correction(ctypes.byref(P), _p(_arr(T, cfg.N)), _p(_arr(h, cfg.N)), _p(_arr(mu, cfg.N)),
                               _p(_arr(kc, cfg.N)), _p(out))
    return out


def velocities3(lam) -> np.ndarray:
    """v_i = sqrt(theta) c_i + u of a gauge (u_x, u_y, u_z, theta), shape (27, 3)."""
    s = np.sqrt(lam[3])
    return np.array([[lam[0] + s * i, lam[1] + s * j, lam[2] + s * k]
                     for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])


def weights3() -> np.ndarray:
    w1 = np.array([1 / 6, 2 / 3, 1 / 6])
    return np.einsum("i,j,k->ijk", w1, w1, w1).ravel()

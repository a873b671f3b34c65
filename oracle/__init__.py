"""FP64 CPU oracle for the colour-gradient + NCI lattice Boltzmann update.

TEST INFRASTRUCTURE ONLY.  The test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only users; the GPU library never
imports or links it.  It shares no code with the GPU path.

The arithmetic lives in ``lbo.c`` (plain C, FP64, OpenMP over nodes); this
module only loads the shared library with ctypes and marshals numpy arrays.
See ``lbo.h`` for the method summary and section references.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBO_LIB points the tests' mutation checks at a deliberately altered build
_LIB_PATH = os.environ.get("LBO_LIB") or os.path.join(_HERE, "liblbo.so")
_lib = None

D2Q9, D3Q27 = 0, 1


def build(force: bool = True) -> str:
    """Compile liblbo.so with gcc (strict IEEE FP64, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-o", _LIB_PATH, os.path.join(_HERE, "lbo.c"), "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("walls_y", C.c_int32), ("tau", C.c_double), ("A_s", C.c_double),
                ("beta", C.c_double), ("A_nci", C.c_double), ("h_min", C.c_double),
                ("h_max", C.c_double), ("force", C.c_double * 3), ("tau2", C.c_double),
                ("nci_mode", C.c_int32), ("rho_ratio", C.c_double), ("alpha1", C.c_double)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = C.CDLL(_LIB_PATH)
        P = C.POINTER
        dp, ip = P(C.c_double), P(C.c_int32)
        lib.lbo_lattice.argtypes = [C.c_int, ip, dp, ip]
        lib.lbo_lattice.restype = C.c_int
        lib.lbo_create.argtypes = [P(_Params)]
        lib.lbo_create.restype = C.c_void_p
        lib.lbo_destroy.argtypes = [C.c_void_p]
        lib.lbo_nodes.argtypes = [C.c_void_p]
        lib.lbo_nodes.restype = C.c_int64
        lib.lbo_time.argtypes = [C.c_void_p]
        lib.lbo_time.restype = C.c_int64
        lib.lbo_set_geometry.argtypes = [C.c_void_p, C.POINTER(C.c_uint8), dp, dp, dp]
        lib.lbo_set_geometry.restype = C.c_int
        lib.lbo_init_fields.argtypes = [C.c_void_p, dp, dp, dp]
        lib.lbo_init_fields.restype = C.c_int
        lib.lbo_set_populations.argtypes = [C.c_void_p, dp, dp]
        lib.lbo_get_populations.argtypes = [C.c_void_p, dp, dp]
        lib.lbo_step.argtypes = [C.c_void_p, C.c_int64]
        lib.lbo_fields.argtypes = [C.c_void_p, dp, dp, dp]
        lib.lbo_observables.argtypes = [C.c_void_p, dp]
        lib.lbo_diagnostics.argtypes = [C.c_void_p, dp, dp, dp, ip, dp]
        lib.lbo_equilibrium.argtypes = [C.c_int, C.c_double, dp, dp]
        lib.lbo_collide_node.argtypes = [P(_Params), dp, dp, dp, dp, dp, dp]
        lib.lbo_equilibrium_k.argtypes = [C.c_int, C.c_double, C.c_double, dp, dp]
        lib.lbo_A_h.argtypes = [C.c_double] * 4
        lib.lbo_A_h.restype = C.c_double
        lib.lbo_A_h_shifted.argtypes = [C.c_double] * 4
        lib.lbo_A_h_shifted.restype = C.c_double
        lib.lbo_node_nci.argtypes = [P(_Params), dp, C.c_int64, dp, ip, dp]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


@dataclass
class Params:
    """Model parameters; field meanings as in ``lbo.h``."""
    lattice: int = D2Q9
    nx: int = 128
    ny: int = 64
    nz: int = 1
    walls_y: int = 0
    tau: float = 1.0
    A_s: float = 0.05
    beta: float = 0.7
    A_nci: float = 0.005
    h_min: float = 2.0
    h_max: float = 4.0
    force: tuple = field(default_factory=lambda: (0.0, 0.0, 0.0))
    tau2: float = 0.0
    nci_mode: int = 0
    rho_ratio: float = 0.0
    alpha1: float = 0.0

    def to_c(self) -> _Params:
        p = _Params()
        for k in ("lattice", "nx", "ny", "nz", "walls_y", "tau", "A_s", "beta", "A_nci",
                  "h_min", "h_max", "tau2", "nci_mode", "rho_ratio", "alpha1"):
            setattr(p, k, getattr(self, k))
        for a in range(3):
            p.force[a] = float(self.force[a])
        return p

    @property
    def dim(self) -> int:
        return 2 if self.lattice == D2Q9 else 3

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz


FLUID, SOLID, INLET, OUTLET = 0, 1, 2, 3


def lattice(lat: int):
    """Return (c[Q,3] int, w[Q] float64, opp[Q] int) of the oracle's lattice."""
    lib = _load()
    c = np.zeros((27, 3), np.int32)
    w = np.zeros(27)
    opp = np.zeros(27, np.int32)
    Q = lib.lbo_lattice(lat, _ip(c), _dp(w), _ip(opp))
    return c[:Q].copy(), w[:Q].copy(), opp[:Q].copy()


def equilibrium(lat: int, rho: float, u) -> np.ndarray:
    lib = _load()
    uu = np.zeros(3)
    uu[:len(u)] = u
    out = np.zeros(27)
    lib.lbo_equilibrium(lat, float(rho), _dp(uu), _dp(out))
    return out[:27 if lat == D3Q27 else 9].copy()


def equilibrium_k(lat: int, alpha: float, rho: float, u) -> np.ndarray:
    """Density-ratio variant: component equilibrium with rest fraction alpha."""
    lib = _load()
    uu = np.zeros(3)
    uu[:len(u)] = u
    out = np.zeros(27)
    lib.lbo_equilibrium_k(lat, float(alpha), float(rho), _dp(uu), _dp(out))
    return out[:27 if lat == D3Q27 else 9].copy()


def collide_node(p: Params, f1, f2, G, F):
    lib = _load()
    f1 = np.ascontiguousarray(f1, np.float64)
    f2 = np.ascontiguousarray(f2, np.float64)
    G3 = np.zeros(3); G3[:len(G)] = G
    F3 = np.zeros(3); F3[:len(F)] = F
    o1 = np.zeros_like(f1); o2 = np.zeros_like(f2)
    pc = p.to_c()
    lib.lbo_collide_node(C.byref(pc), _dp(f1), _dp(f2), _dp(G3), _dp(F3), _dp(o1), _dp(o2))
    return o1, o2


def A_h(h: float, A: float, h_min: float, h_max: float) -> float:
    return _load().lbo_A_h(float(h), float(A), float(h_min), float(h_max))


def A_h_shifted(h: float, A: float, h_min: float, h_max: float) -> float:
    return _load().lbo_A_h_shifted(float(h), float(A), float(h_min), float(h_max))


def node_nci(p: Params, psi: np.ndarray, node: int):
    """Gradient G, hit distance h (0 = none) and F_rep at one node of psi."""
    lib = _load()
    psi = np.ascontiguousarray(psi, np.float64).ravel()
    G = np.zeros(3); Fr = np.zeros(3); hit = np.zeros(1, np.int32)
    pc = p.to_c()
    lib.lbo_node_nci(C.byref(pc), _dp(psi), int(node), _dp(G), _ip(hit), _dp(Fr))
    return G, int(hit[0]), Fr


class Oracle:
    """Handle around one oracle lattice.  Arrays are numpy float64 with the
    node index x + nx*(y + ny*z) (x fastest)."""

    def __init__(self, p: Params):
        self.p = p
        self._lib = _load()
        self._pc = p.to_c()
        self._h = self._lib.lbo_create(C.byref(self._pc))
        c, w, opp = lattice(p.lattice)
        self.c, self.w, self.opp, self.Q = c, w, opp, len(w)

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.lbo_destroy(self._h)
            self._h = None

    @property
    def N(self) -> int:
        return self.p.N

    @property
    def t(self) -> int:
        return self._lib.lbo_time(self._h)

    def set_geometry(self, node_type, rho1, rho2, u=None):
        """Node types (FLUID/SOLID/INLET/OUTLET, N bytes); inlet nodes take
        rho1, rho2, u at their index.  Call before init_fields."""
        t = np.ascontiguousarray(node_type, np.uint8).ravel()
        r1 = np.ascontiguousarray(rho1, np.float64).ravel()
        r2 = np.ascontiguousarray(rho2, np.float64).ravel()
        uu = None if u is None else np.ascontiguousarray(u, np.float64).ravel()
        assert t.size == self.N and r1.size == self.N and r2.size == self.N
        rc = self._lib.lbo_set_geometry(self._h, t.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(r1),
                                        _dp(r2), None if uu is None else _dp(uu))
        if rc != 0:
            raise ValueError("invalid geometry")

    def init_fields(self, rho1, rho2, u=None):
        r1 = np.ascontiguousarray(rho1, np.float64).ravel()
        r2 = np.ascontiguousarray(rho2, np.float64).ravel()
        up = None
        if u is not None:
            uu = np.ascontiguousarray(u, np.float64).ravel()
            assert uu.size == self.p.dim * self.N
            up = _dp(uu)
        rc = self._lib.lbo_init_fields(self._h, _dp(r1), _dp(r2), up)
        if rc != 0:
            raise ValueError("invalid densities")

    def set_populations(self, f1, f2):
        a = np.ascontiguousarray(f1, np.float64).reshape(self.Q, self.N)
        b = np.ascontiguousarray(f2, np.float64).reshape(self.Q, self.N)
        self._lib.lbo_set_populations(self._h, _dp(a), _dp(b))

    def get_populations(self):
        a = np.zeros((self.Q, self.N)); b = np.zeros((self.Q, self.N))
        self._lib.lbo_get_populations(self._h, _dp(a), _dp(b))
        return a, b

    def step(self, n: int = 1):
        self._lib.lbo_step(self._h, int(n))

    def fields(self):
        r1 = np.zeros(self.N); r2 = np.zeros(self.N); u = np.zeros(self.p.dim * self.N)
        self._lib.lbo_fields(self._h, _dp(r1), _dp(r2), _dp(u))
        return r1, r2, u.reshape(self.p.dim, self.N)

    def observables(self) -> dict:
        o = np.zeros(8)
        self._lib.lbo_observables(self._h, _dp(o))
        return {"mass": o[0:2].copy(), "mom": o[2:5].copy(), "Q": o[5], "Q_d": o[6],
                "umax": o[7]}

    def diagnostics(self):
        psi = np.zeros(self.N); G = np.zeros(3 * self.N); F = np.zeros(3 * self.N)
        hit = np.zeros(self.N, np.int32); mg = np.zeros(self.N)
        self._lib.lbo_diagnostics(self._h, _dp(psi), _dp(G), _dp(F), _ip(hit), _dp(mg))
        return {"psi": psi, "G": G.reshape(3, self.N), "Frep": F.reshape(3, self.N),
                "hit": hit, "margin": mg}

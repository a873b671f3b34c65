"""ctypes binding of the HIP C-ABI library ``liblbnci.so`` (include/lbnci.h).

Argument marshalling only: every step of the lattice Boltzmann update runs in
the library's HIP kernels.  There is no CPU fallback; a missing library or
GPU raises.  Work goes to the default HIP stream unless a stream of the
library's own runtime is given (``Stream``): a Python framework that bundles
its own HIP runtime hands out streams that are not valid in this one.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field, asdict

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBNCI_LIB", os.path.join(_PKG, "liblbnci.so"))

LB_D2Q9, LB_D3Q27 = 0, 1
LB_STORE_FP32, LB_STORE_FP16_DEV, LB_STORE_BF16_DEV, LB_STORE_FP32_F32 = 0, 1, 2, 3
STORAGE = {"fp32": LB_STORE_FP32, "fp16": LB_STORE_FP16_DEV, "bf16": LB_STORE_BF16_DEV,
           "fp32_f32": LB_STORE_FP32_F32}
ERRORS = {-1: "LB_EINVAL", -2: "LB_ENOMEM", -3: "LB_EDEVICE", -4: "LB_ENUMERIC", -5: "LB_ESTATE"}


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class lb_params(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("walls_y", C.c_int32), ("tau", C.c_double), ("A_s", C.c_double),
                ("beta", C.c_double), ("A_nci", C.c_double), ("h_min", C.c_double),
                ("h_max", C.c_double), ("force", C.c_double * 3), ("storage", C.c_int32),
                ("obs_every", C.c_int32), ("conv_window", C.c_int32), ("conv_m", C.c_int32),
                ("conv_eps", C.c_double), ("tau2", C.c_double),
                ("nci_mode", C.c_int32), ("rho_ratio", C.c_double), ("alpha1", C.c_double),
                ("mass_tol", C.c_double)]


class lb_obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double * 2), ("mom", C.c_double * 3),
                ("Q", C.c_double), ("Q_d", C.c_double), ("umax", C.c_double),
                ("Q_window", C.c_double), ("converged", C.c_int32), ("flags", C.c_int32)]


class lb_droplet_stats(C.Structure):
    _fields_ = [("count", C.c_int64), ("dispersed", C.c_int64), ("rows", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads liblbnci.so and declares the C ABI.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = C.CDLL(path)
    P, dp, ip = C.POINTER, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    vp = C.c_void_p
    sig = {
        "lb_create": ([P(lb_params), vp, P(vp)], C.c_int),
        "lb_init_fields": ([vp, dp, dp, dp], C.c_int),
        "lb_set_populations": ([vp, dp, dp], C.c_int),
        "lb_step": ([vp, C.c_int64], C.c_int),
        "lb_prepare": ([vp], C.c_int),
        "lb_step_timed": ([vp, C.c_int64, dp], C.c_int),
        "lb_graphs": ([vp], C.c_int),
        "lb_observables": ([vp, P(lb_obs)], C.c_int),
        "lb_get_fields": ([vp, dp, dp, dp], C.c_int),
        "lb_get_fields_static": ([vp, dp, dp, dp], C.c_int),
        "lb_get_populations": ([vp, dp, dp], C.c_int),
        "lb_get_nci": ([vp, dp, dp, ip], C.c_int),
        "lb_destroy": ([vp], None),
        "lb_lattice_tables": ([C.c_int32, ip, dp], C.c_int),
        "lb_time": ([vp], C.c_int64),
        "lb_device_bytes": ([vp], C.c_int64),
        "lb_last_error": ([], C.c_char_p),
        "lb_profile": ([vp, C.c_int], C.c_int),
        "lb_kernel_times": ([vp, dp, dp, P(C.c_int64)], C.c_int),
        "lb_copy_probe": ([C.c_int64, C.c_int, vp, dp, dp], C.c_int),
        "lb_stream_create": ([P(vp)], C.c_int),
        "lb_stream_destroy": ([vp], C.c_int),
        "lb_droplets": ([vp, P(lb_droplet_stats), ip, C.c_int64, P(C.c_int64), P(C.c_int64), dp],
                        C.c_int),
        "lb_vorticity": ([vp, dp], C.c_int),
        "lb_set_geometry": ([vp, C.POINTER(C.c_uint8), dp, dp, dp], C.c_int),
        "lb_analysis_times": ([vp, dp, dp], C.c_int),
        "lb_batch_create": ([P(lb_params), C.c_int32, vp, P(vp)], C.c_int),
        "lb_batch_init_fields": ([vp, C.c_int32, dp, dp, dp], C.c_int),
        "lb_batch_step": ([vp, C.c_int64, C.c_int32], C.c_int),
        "lb_batch_flags": ([vp, ip], C.c_int),
        "lb_batch_observables": ([vp, C.c_int32, P(lb_obs)], C.c_int),
        "lb_batch_get_fields": ([vp, C.c_int32, dp, dp, dp], C.c_int),
        "lb_batch_info": ([vp, C.c_int32, P(C.c_int64), P(C.c_int32), P(C.c_int32)], C.c_int),
        "lb_batch_graphs": ([vp], C.c_int),
        "lb_batch_destroy": ([vp], None),
        "lb_batch_tune": ([vp, C.c_int32, dp], C.c_int),
        "lb_batch_set_config": ([vp, C.c_int32, C.c_int32, C.c_int32], C.c_int),
        "lb_batch_get_config": ([vp, P(C.c_int32), P(C.c_int32), P(C.c_int32)], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc < 0:
        raise LBError(rc, _lib.lb_last_error().decode())
    return rc


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))


def current_stream_handle():
    """The stream a handle uses when none is given: 0, the default stream."""
    return 0


class Stream:
    """A non-blocking HIP stream of the library's runtime (lb_stream_create),
    default priority.  ``handle`` is the hipStream_t to pass as ``stream=``;
    close() (or leaving a ``with`` block) waits for its work and releases it,
    after the handles that use it are closed."""

    def __init__(self):
        self.lib = load_library()
        h = C.c_void_p()
        _check(self.lib.lb_stream_create(C.byref(h)))
        self.handle = h.value

    def close(self):
        if getattr(self, "handle", None):
            _check(self.lib.lb_stream_destroy(C.c_void_p(self.handle)))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_probe(nbytes: int, iters: int = 20, stream: int | None = None):
    """Achievable streaming bandwidth (read + write) of a plain copy kernel."""
    lib = load_library()
    ms = C.c_double(); gb = C.c_double()
    st = current_stream_handle() if stream is None else stream
    _check(lib.lb_copy_probe(int(nbytes), int(iters), C.c_void_p(st), C.byref(ms), C.byref(gb)))
    return {"ms": ms.value, "GBps": gb.value}


def lattice_tables(lattice: int):
    lib = load_library()
    c = np.zeros((27, 3), np.int32)
    w = np.zeros(27)
    Q = _check(lib.lb_lattice_tables(lattice, _ip(c), _dp(w)))
    return c[:Q].copy(), w[:Q].copy()


@dataclass
class Params:
    """Mirror of ``lb_params``."""
    lattice: int = LB_D2Q9
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
    storage: int = LB_STORE_FP32
    obs_every: int = 0
    conv_window: int = 0
    conv_m: int = 3
    conv_eps: float = 1e-4
    tau2: float = 0.0
    nci_mode: int = 0
    rho_ratio: float = 0.0
    alpha1: float = 0.0
    mass_tol: float = 0.0

    @classmethod
    def from_dict(cls, d: dict, **kw):
        keys = {f for f in cls.__dataclass_fields__}
        v = {k: d[k] for k in d if k in keys}
        v.update(kw)
        return cls(**v)

    def to_c(self) -> lb_params:
        p = lb_params()
        for k, v in asdict(self).items():
            if k == "force":
                for a in range(3):
                    p.force[a] = float(v[a]) if a < len(v) else 0.0
            else:
                setattr(p, k, v)
        return p

    @property
    def dim(self):
        return 2 if self.lattice == LB_D2Q9 else 3

    @property
    def N(self):
        return self.nx * self.ny * self.nz


class Lattice:
    """One lattice handle (lb_create ... lb_destroy)."""

    def __init__(self, p: Params, stream: int | None = None):
        self.lib = load_library()
        self.p = p
        self._pc = p.to_c()
        h = C.c_void_p()
        st = current_stream_handle() if stream is None else stream
        _check(self.lib.lb_create(C.byref(self._pc), C.c_void_p(st), C.byref(h)))
        self.h = h
        self.c, self.w = lattice_tables(p.lattice)
        self.Q = len(self.w)

    def close(self):
        if getattr(self, "h", None):
            self.lib.lb_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @property
    def N(self):
        return self.p.N

    @property
    def t(self) -> int:
        return self.lib.lb_time(self.h)

    @property
    def device_bytes(self) -> int:
        return self.lib.lb_device_bytes(self.h)

    def set_geometry(self, node_type, rho1, rho2, u=None):
        """lb_set_geometry: node types (LB_NODE_*), and the inlet/outlet
        prescriptions carried in rho1, rho2, u at those nodes."""
        t = np.ascontiguousarray(node_type, np.uint8).ravel()
        r1 = np.ascontiguousarray(rho1, np.float64).ravel()
        r2 = np.ascontiguousarray(rho2, np.float64).ravel()
        uu = None if u is None else np.ascontiguousarray(u, np.float64).ravel()
        if t.size != self.N or r1.size != self.N or r2.size != self.N:
            raise ValueError("geometry arrays must have N entries")
        if uu is not None and uu.size != self.p.dim * self.N:
            raise ValueError("u must have dim*N entries")
        _check(self.lib.lb_set_geometry(self.h, t.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(r1), _dp(r2),
                                        _dp(uu)))

    def init_fields(self, rho1, rho2, u=None):
        r1 = np.ascontiguousarray(rho1, np.float64).ravel()
        r2 = np.ascontiguousarray(rho2, np.float64).ravel()
        if r1.size != self.N or r2.size != self.N:
            raise ValueError("density arrays must hold N values")
        uu = None
        if u is not None:
            uu = np.ascontiguousarray(u, np.float64).ravel()
            if uu.size != self.p.dim * self.N:
                raise ValueError("u must hold dim*N values")
        _check(self.lib.lb_init_fields(self.h, _dp(r1), _dp(r2), _dp(uu)))

    def set_populations(self, f1, f2):
        a = np.ascontiguousarray(f1, np.float64).reshape(self.Q, self.N)
        b = np.ascontiguousarray(f2, np.float64).reshape(self.Q, self.N)
        _check(self.lib.lb_set_populations(self.h, _dp(a), _dp(b)))

    def step(self, n: int = 1):
        _check(self.lib.lb_step(self.h, int(n)))

    def step_timed(self, n: int) -> float:
        """lb_step_timed: n steps between HIP events on the handle's stream;
        returns their device time in ms (synchronises)."""
        ms = C.c_double()
        _check(self.lib.lb_step_timed(self.h, int(n), C.byref(ms)))
        return ms.value

    def prepare(self):
        """lb_prepare: capture the step-replay graphs now instead of inside
        the first lb_step that uses them."""
        _check(self.lib.lb_prepare(self.h))

    def observables(self) -> dict:
        o = lb_obs()
        rc = self.lib.lb_observables(self.h, C.byref(o))
        if rc < 0 and rc != -4:
            _check(rc)
        return {"step": o.step, "mass": np.array(o.mass[:]), "mom": np.array(o.mom[:]), "Q": o.Q,
                "Q_d": o.Q_d, "umax": o.umax, "Q_window": o.Q_window,
                "converged": bool(o.converged), "flags": o.flags, "rc": rc}

    def fields(self):
        r1 = np.zeros(self.N); r2 = np.zeros(self.N); u = np.zeros(self.p.dim * self.N)
        _check(self.lib.lb_get_fields(self.h, _dp(r1), _dp(r2), _dp(u)))
        return r1, r2, u.reshape(self.p.dim, self.N)

    def populations(self):
        f1 = np.zeros((self.Q, self.N)); f2 = np.zeros((self.Q, self.N))
        _check(self.lib.lb_get_populations(self.h, _dp(f1), _dp(f2)))
        return f1, f2

    @property
    def graphs(self) -> bool:
        """True while plain steps are replayed from captured hipGraphs."""
        return self.lib.lb_graphs(self.h) == 1

    def profile(self, enable: bool = True):
        _check(self.lib.lb_profile(self.h, int(enable)))

    def kernel_times(self):
        a = C.c_double(); b = C.c_double(); n = C.c_int64()
        _check(self.lib.lb_kernel_times(self.h, C.byref(a), C.byref(b), C.byref(n)))
        return {"ms_phase": a.value, "ms_main": b.value, "launches": n.value}

    def droplets(self, labels: bool = True, cap: int | None = None) -> dict:
        """Droplets of the current state (lb_droplets): count, dispersed node
        count, rows (hex-n), per-node labels and the table in label order."""
        cap = self.N // 2 + 1 if cap is None else cap
        st = lb_droplet_stats()
        lab = np.empty(self.N, np.int32) if labels else None
        root = np.empty(cap, np.int64); vol = np.empty(cap, np.int64); cen = np.empty((cap, 3))
        i64 = C.POINTER(C.c_int64)
        _check(self.lib.lb_droplets(self.h, C.byref(st), _ip(lab), cap, root.ctypes.data_as(i64),
                                    vol.ctypes.data_as(i64), _dp(cen)))
        k = min(st.count, cap)
        return {"count": st.count, "dispersed": st.dispersed, "rows": st.rows, "labels": lab,
                "roots": root[:k].copy(), "volumes": vol[:k].copy(), "centroids": cen[:k].copy()}

    def vorticity(self):
        """curl u of the current state (lb_vorticity): [N] in 2-D, [3, N] in 3-D."""
        w = np.empty((1 if self.p.dim == 2 else 3) * self.N)
        _check(self.lib.lb_vorticity(self.h, _dp(w)))
        return w if self.p.dim == 2 else w.reshape(3, self.N)

    def analysis_times(self):
        a = C.c_double(); b = C.c_double()
        _check(self.lib.lb_analysis_times(self.h, C.byref(a), C.byref(b)))
        return {"ms_droplets": a.value, "ms_vorticity": b.value}

    def nci(self):
        psi = np.zeros(self.N); fr = np.zeros(self.p.dim * self.N); hit = np.zeros(self.N, np.int32)
        _check(self.lib.lb_get_nci(self.h, _dp(psi), _dp(fr), _ip(hit)))
        return psi, fr.reshape(self.p.dim, self.N), hit


LB_BATCH_LAUNCH, LB_BATCH_PERSISTENT, LB_BATCH_AUTO = 0, 1, 2


def _obs_dict(o: lb_obs, rc: int) -> dict:
    return {"step": o.step, "mass": np.array(o.mass[:]), "mom": np.array(o.mom[:]), "Q": o.Q,
            "Q_d": o.Q_d, "umax": o.umax, "Q_window": o.Q_window,
            "converged": bool(o.converged), "flags": o.flags, "rc": rc}


class Batch:
    """Many independent lattices stepped together (lb_batch_* ABI)."""

    def __init__(self, params: list, stream: int | None = None):
        self.lib = load_library()
        self.params = list(params)
        arr = (lb_params * len(self.params))(*[p.to_c() for p in self.params])
        self._arr = arr
        h = C.c_void_p()
        st = current_stream_handle() if stream is None else stream
        _check(self.lib.lb_batch_create(arr, len(self.params), C.c_void_p(st), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.lb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def __len__(self):
        return len(self.params)

    def init_fields(self, c: int, rho1, rho2, u=None):
        p = self.params[c]
        r1 = np.ascontiguousarray(rho1, np.float64).ravel()
        r2 = np.ascontiguousarray(rho2, np.float64).ravel()
        if r1.size != p.N or r2.size != p.N:
            raise ValueError("density arrays must hold N values")
        uu = None if u is None else np.ascontiguousarray(u, np.float64).ravel()
        _check(self.lib.lb_batch_init_fields(self.h, int(c), _dp(r1), _dp(r2), _dp(uu)))

    def step(self, n: int, mode: int = 2, numeric_ok: bool = False) -> list:
        """Advances every active channel by n steps.  A channel flagged with a
        NaN/Inf or a mass drift (LB_ENUMERIC) raises, unless numeric_ok: then
        the flagged channels' indices are returned (the others stepped)."""
        rc = self.lib.lb_batch_step(self.h, int(n), int(mode))
        if rc == -4 and numeric_ok:
            return [c for c, f in enumerate(self.flags()) if f]
        _check(rc)
        return []

    def flags(self) -> np.ndarray:
        """lb_batch_flags: the lb_obs flag bits of every channel."""
        out = np.zeros(len(self.params), np.int32)
        _check(self.lib.lb_batch_flags(self.h, _ip(out)))
        return out

    def observables(self, c: int) -> dict:
        o = lb_obs()
        rc = self.lib.lb_batch_observables(self.h, int(c), C.byref(o))
        if rc < 0 and rc != -4:
            _check(rc)
        return _obs_dict(o, rc)

    def fields(self, c: int):
        p = self.params[c]
        r1 = np.zeros(p.N); r2 = np.zeros(p.N); u = np.zeros(p.dim * p.N)
        _check(self.lib.lb_batch_get_fields(self.h, int(c), _dp(r1), _dp(r2), _dp(u)))
        return r1, r2, u.reshape(p.dim, p.N)

    def info(self, c: int) -> dict:
        st = C.c_int64(); act = C.c_int32(); blk = C.c_int32()
        _check(self.lib.lb_batch_info(self.h, int(c), C.byref(st), C.byref(act), C.byref(blk)))
        return {"steps": st.value, "active": bool(act.value), "blocks": blk.value}

    @property
    def graphs(self) -> bool:
        return self.lib.lb_batch_graphs(self.h) == 1

    def signature(self) -> str:
        """Shape class of the batch for the tuning cache: lattice, storage and
        the sorted channel sizes rounded to tiles."""
        p0 = self.params[0]
        sizes = sorted(((p.nx + 63) // 64, (p.ny + 3) // 4, p.nz) for p in self.params)
        return f"L{p0.lattice}-S{p0.storage}-" + "_".join(f"{a}x{b}x{c}" for a, b, c in sizes)

    def config(self) -> dict:
        m = C.c_int32(); o = C.c_int32(); b = C.c_int32()
        _check(self.lib.lb_batch_get_config(self.h, C.byref(m), C.byref(o), C.byref(b)))
        return {"mode": m.value, "tile_order": o.value, "main_by": b.value}

    def set_config(self, mode: int, tile_order: int, main_by: int):
        _check(self.lib.lb_batch_set_config(self.h, int(mode), int(tile_order), int(main_by)))

    def tune(self, trial_steps: int = 20, cache: str | None = None) -> dict:
        """Picks the fastest configuration (lb_batch_tune), or reuses the one
        cached for this batch's signature in the JSON file `cache`.  Trial steps
        are real steps of the channels."""
        import json
        key = self.signature()
        db = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                db = json.load(f)
        if key in db:
            cfg = db[key]
            self.set_config(cfg["mode"], cfg["tile_order"], cfg["main_by"])
            return dict(cfg, cached=True)
        ms = C.c_double()
        _check(self.lib.lb_batch_tune(self.h, int(trial_steps), C.byref(ms)))
        cfg = dict(self.config(), ms_per_step=ms.value)
        if cache:
            db[key] = cfg
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(db, f, indent=1)
        return dict(cfg, cached=False)

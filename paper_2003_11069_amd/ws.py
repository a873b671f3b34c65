"""ctypes binding of the warm-start U-Net C ABI (include/wsnet.h), which lives
in the same HIP library as the lattice Boltzmann kernels.

Argument marshalling only: convolutions, pooling, loss and Adam all run in the
library's HIP kernels.  Images are NHWC float32; device buffers come from
``DeviceArray`` (the library's own hipMalloc helpers), so no other GPU
framework is needed.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import lb as _lb

ERRORS = {-1: "WS_EINVAL", -2: "WS_ENOMEM", -3: "WS_EDEVICE"}


class WSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class ws_config(C.Structure):
    _fields_ = [("levels", C.c_int32), ("base", C.c_int32), ("cin", C.c_int32), ("cout", C.c_int32),
                ("H", C.c_int32), ("W", C.c_int32), ("max_batch", C.c_int32), ("conv_algo", C.c_int32)]


_declared = None


def _lib():
    global _declared
    lib = _lb.load_library()
    if _declared is lib:
        return lib
    vp, fp, dp = C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_double)
    sig = {
        "ws_create": ([C.POINTER(ws_config), vp, C.POINTER(vp)], C.c_int),
        "ws_destroy": ([vp], None),
        "ws_num_params": ([vp], C.c_int64),
        "ws_device_bytes": ([vp], C.c_int64),
        "ws_set_params": ([vp, fp, C.c_int64], C.c_int),
        "ws_get_params": ([vp, fp, C.c_int64], C.c_int),
        "ws_get_grads": ([vp, fp, C.c_int64], C.c_int),
        "ws_forward": ([vp, vp, C.c_int32, vp], C.c_int),
        "ws_backward": ([vp, vp, vp, C.c_int32, dp], C.c_int),
        "ws_adam": ([vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
        "ws_train_step": ([vp, vp, vp, C.c_int32, C.c_float, dp], C.c_int),
        "ws_flops": ([vp, C.c_int32, dp, dp], C.c_int),
        "ws_malloc": ([C.c_int64, C.POINTER(vp)], C.c_int),
        "ws_free": ([vp], C.c_int),
        "ws_memcpy": ([vp, vp, C.c_int64, C.c_int32], C.c_int),
        "ws_sync": ([], C.c_int),
        "ws_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _declared = lib
    return lib


def _check(rc: int):
    if rc < 0:
        raise WSError(rc, _lib().ws_last_error().decode())
    return rc


class DeviceArray:
    """float32 device buffer of a fixed shape (hipMalloc through the library)."""

    def __init__(self, shape):
        self.shape = tuple(int(s) for s in shape)
        self.size = int(np.prod(self.shape))
        p = C.c_void_p()
        _check(_lib().ws_malloc(4 * self.size, C.byref(p)))
        self._p = p

    @classmethod
    def from_host(cls, a: np.ndarray) -> "DeviceArray":
        d = cls(a.shape)
        d.upload(a)
        return d

    def ptr(self, offset: int = 0) -> int:
        """Device address of element `offset` (flat)."""
        if not 0 <= offset <= self.size:
            raise IndexError(offset)
        return self._p.value + 4 * offset

    def upload(self, a: np.ndarray, offset: int = 0):
        a = np.ascontiguousarray(a, dtype=np.float32)
        if offset + a.size > self.size:
            raise ValueError("upload beyond the buffer")
        _check(_lib().ws_memcpy(self.ptr(offset), a.ctypes.data, 4 * a.size, 0))

    def download(self, count: int | None = None, offset: int = 0) -> np.ndarray:
        count = self.size - offset if count is None else count
        if offset + count > self.size:
            raise ValueError("download beyond the buffer")
        out = np.empty(count, np.float32)
        _check(_lib().ws_memcpy(out.ctypes.data, self.ptr(offset), 4 * count, 1))
        return out

    def numpy(self) -> np.ndarray:
        return self.download().reshape(self.shape)

    def free(self):
        if getattr(self, "_p", None) is not None and self._p.value:
            _lib().ws_free(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


@dataclass
class UNetConfig:
    levels: int = 4
    base: int = 32
    cin: int = 3
    cout: int = 3
    H: int = 128
    W: int = 256
    max_batch: int = 8
    conv_algo: int = 0  # 0: direct 3x3 kernels where the shape allows; 1: implicit GEMM only

    def to_c(self) -> ws_config:
        return ws_config(self.levels, self.base, self.cin, self.cout, self.H, self.W, self.max_batch,
                         self.conv_algo)


class UNet:
    """The warm-start U-Net on the GPU (parameters zero until set_params)."""

    def __init__(self, cfg: UNetConfig, stream: int | None = None):
        self.cfg = cfg
        lib = _lib()
        h = C.c_void_p()
        s = _lb.current_stream_handle() if stream is None else stream
        _check(lib.ws_create(C.byref(cfg.to_c()), C.c_void_p(s), C.byref(h)))
        self._h = h
        self.n_params = int(lib.ws_num_params(h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().ws_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def device_bytes(self) -> int:
        return int(_lib().ws_device_bytes(self._h))

    def _vec(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {a.size}")
        return a

    def set_params(self, p):
        p = self._vec(p)
        _check(_lib().ws_set_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float)), p.size))

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _check(_lib().ws_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float)), out.size))
        return out

    def grads(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _check(_lib().ws_get_grads(self._h, out.ctypes.data_as(C.POINTER(C.c_float)), out.size))
        return out

    def _img(self, n, c):
        return n * self.cfg.H * self.cfg.W * c

    def forward_ptr(self, x_ptr: int, batch: int, y_ptr: int):
        _check(_lib().ws_forward(self._h, C.c_void_p(x_ptr), batch, C.c_void_p(y_ptr)))

    def backward_ptr(self, x_ptr: int, t_ptr: int, batch: int, want_loss: bool = True):
        loss = C.c_double(float("nan"))
        _check(_lib().ws_backward(self._h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), batch,
                                  C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def train_step_ptr(self, x_ptr: int, t_ptr: int, batch: int, lr: float, want_loss: bool = False):
        loss = C.c_double(float("nan"))
        _check(_lib().ws_train_step(self._h, C.c_void_p(x_ptr), C.c_void_p(t_ptr), batch, lr,
                                    C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def forward(self, x: np.ndarray) -> np.ndarray:
        """Host convenience: x [B,H,W,cin] -> y [B,H,W,cout]."""
        B = x.shape[0]
        dx = DeviceArray.from_host(x)
        dy = DeviceArray((B, self.cfg.H, self.cfg.W, self.cfg.cout))
        self.forward_ptr(dx.ptr(), B, dy.ptr())
        return dy.numpy()

    def backward(self, x: np.ndarray, target: np.ndarray) -> float:
        dx = DeviceArray.from_host(x)
        dt = DeviceArray.from_host(target)
        return self.backward_ptr(dx.ptr(), dt.ptr(), x.shape[0])

    def adam(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        _check(_lib().ws_adam(self._h, lr, beta1, beta2, eps, weight_decay))

    def flops(self, batch: int):
        f, b = C.c_double(), C.c_double()
        _check(_lib().ws_flops(self._h, batch, C.byref(f), C.byref(b)))
        return f.value, b.value


def sync():
    _check(_lib().ws_sync())

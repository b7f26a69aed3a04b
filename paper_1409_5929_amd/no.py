"""Python binding of the warm-start network library (``include/lbm_no.h``).

Argument marshalling only: the forward pass, loss, backward pass and Adam
all run in ``liblbm_no.so`` (HIP, gfx950).  Tensors are torch device tensors
(float32, contiguous, [batch][channel][height][width]); torch provides device
memory and streams.  Importing works without a GPU; creating a network needs
the built library and raises if it is missing.

The entry points mirror ``include/lbm_no.h``: lbm_no_create is
WarmStartNet(...), lbm_no_param_count is param_count, and every other
lbm_no_<name> is WarmStartNet.<name> (get(which) also as params() and
grads(), destroy also as close()).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbm_no.so")
_lib = None


class NoError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime torch was built against)

    if not os.path.exists(LIB_PATH):
        raise NoError(f"{LIB_PATH} is missing: build it with python -m paper_1409_5929_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.lbm_no_param_count.argtypes = [P(ctypes.c_int32), P(ctypes.c_int64)]
    lib.lbm_no_create.argtypes = [P(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  P(ctypes.c_float), vp, P(vp)]
    lib.lbm_no_forward.argtypes = [vp, vp, ctypes.c_int32, vp]
    lib.lbm_no_gradients.argtypes = [vp, vp, vp, ctypes.c_int32, P(ctypes.c_double)]
    lib.lbm_no_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
    lib.lbm_no_get.argtypes = [vp, ctypes.c_int32, P(ctypes.c_float)]
    lib.lbm_no_set_params.argtypes = [vp, P(ctypes.c_float)]
    lib.lbm_no_sync.argtypes = [vp]
    lib.lbm_no_destroy.argtypes = [vp]
    lib.lbm_no_destroy.restype = None
    lib.lbm_no_last_error.restype = ctypes.c_char_p
    for f in ("lbm_no_param_count", "lbm_no_create", "lbm_no_forward", "lbm_no_gradients", "lbm_no_adam",
              "lbm_no_get", "lbm_no_set_params", "lbm_no_sync"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise NoError(f"lbm_no error {rc}: {_lib.lbm_no_last_error().decode()}")


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def param_count(widths) -> int:
    lib = _load()
    w = (ctypes.c_int32 * 4)(*widths)
    n = ctypes.c_int64()
    _check(lib.lbm_no_param_count(w, ctypes.byref(n)))
    return n.value


class WarmStartNet:
    """Handle of one network (widths c1..c4) for height x width inputs."""

    def __init__(self, widths, height, width, max_batch, params, stream=None):
        import torch

        lib = _load()
        self._lib = lib
        self.widths = tuple(int(w) for w in widths)
        self.height, self.width, self.max_batch = int(height), int(width), int(max_batch)
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != param_count(self.widths):
            raise NoError("parameter vector has the wrong length")
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.lbm_no_create((ctypes.c_int32 * 4)(*self.widths), self.height, self.width, self.max_batch,
                                 _fptr(p), ctypes.c_void_p(stream), ctypes.byref(h)))
        self._h = h

    def _tensor(self, t, channels):
        import torch

        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise ValueError("expected a float32 contiguous device tensor")
        if t.dim() != 4 or tuple(t.shape[1:]) != (channels, self.height, self.width):
            raise ValueError(f"tensor shape {tuple(t.shape)}, expected (batch, {channels}, "
                             f"{self.height}, {self.width})")
        return ctypes.c_void_p(t.data_ptr())

    def _ordered(self, call):
        """Run call() with the handle's stream ordered after torch's current
        stream (which wrote the inputs) and the current stream after the
        handle's (which writes the outputs) when the two differ."""
        import torch

        cur = torch.cuda.current_stream()
        if (cur.cuda_stream or 0) == (self.stream or 0):
            return call()
        own = torch.cuda.ExternalStream(self.stream)
        own.wait_stream(cur)
        out = call()
        cur.wait_stream(own)
        return out

    def forward(self, x):
        import torch

        y = torch.empty((x.shape[0], 3, self.height, self.width), dtype=torch.float32, device=x.device)
        self._ordered(lambda: _check(self._lib.lbm_no_forward(self._h, self._tensor(x, 6), int(x.shape[0]),
                                                               self._tensor(y, 3))))
        return y

    def gradients(self, x, target) -> float:
        loss = ctypes.c_double()
        self._ordered(lambda: _check(self._lib.lbm_no_gradients(self._h, self._tensor(x, 6),
                                                                 self._tensor(target, 3), int(x.shape[0]),
                                                                 ctypes.byref(loss))))
        return loss.value

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(self._lib.lbm_no_adam(self._h, float(lr), float(beta1), float(beta2), float(eps)))

    def params(self) -> np.ndarray:
        return self.get(0)

    def grads(self) -> np.ndarray:
        return self.get(1)

    def get(self, which: int) -> np.ndarray:
        """Parameters (which = 0) or the last gradients (which = 1), host float32."""
        out = np.empty(param_count(self.widths), dtype=np.float32)
        _check(self._lib.lbm_no_get(self._h, int(which), _fptr(out)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != param_count(self.widths):  # the library copies that many floats
            raise NoError("parameter vector has the wrong length")
        _check(self._lib.lbm_no_set_params(self._h, _fptr(p)))

    def sync(self):
        _check(self._lib.lbm_no_sync(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbm_no_destroy(self._h)
            self._h = None

    destroy = close

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

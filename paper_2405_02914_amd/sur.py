"""ctypes binding of the surrogate C ABI (include/sur.h) in libimpm.so.

Argument marshalling only: every computation runs in the library's HIP
kernels.  Inputs and outputs of infer / train are torch tensors on the HIP
device (float32, contiguous); parameters and gradients come back as numpy.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .impm import lib as _impm_lib

SUR_OK = 0


class sur_params(C.Structure):
    _fields_ = [
        ("H", C.c_int32), ("W", C.c_int32), ("channels", C.c_int32 * 4), ("max_batch", C.c_int32),
        ("_pad0", C.c_int32), ("seed", C.c_uint64), ("lr", C.c_float), ("beta1", C.c_float),
        ("beta2", C.c_float), ("eps", C.c_float),
    ]


EXPORTS = ("sur_params_default", "sur_create", "sur_destroy", "sur_num_params", "sur_infer", "sur_train_step",
           "sur_compute_grads", "sur_get_grads", "sur_get_params", "sur_set_params", "sur_save", "sur_load",
           "sur_debug_read", "sur_set_lr", "sur_contact_area", "sur_last_error")

_bound = False


def lib():
    global _bound
    L = _impm_lib()
    if _bound:
        return L
    vp, i32, fp = C.c_void_p, C.c_int32, C.c_void_p
    L.sur_params_default.argtypes = [C.POINTER(sur_params)]
    L.sur_create.argtypes = [C.POINTER(sur_params), vp, C.POINTER(vp)]
    L.sur_destroy.argtypes = [vp]
    L.sur_destroy.restype = None
    L.sur_num_params.argtypes = [vp, C.POINTER(C.c_int64)]
    L.sur_infer.argtypes = [vp, fp, fp, fp, fp, i32]
    L.sur_train_step.argtypes = [vp, fp, fp, fp, fp, i32, C.POINTER(C.c_float)]
    L.sur_compute_grads.argtypes = [vp, fp, fp, fp, fp, i32, C.POINTER(C.c_float)]
    L.sur_get_grads.argtypes = [vp, fp]
    L.sur_get_params.argtypes = [vp, fp]
    L.sur_set_params.argtypes = [vp, fp]
    L.sur_save.argtypes = [vp, C.c_char_p]
    L.sur_load.argtypes = [vp, C.c_char_p]
    L.sur_debug_read.argtypes = [vp, i32, i32, fp]
    L.sur_set_lr.argtypes = [vp, C.c_float]
    L.sur_contact_area.argtypes = [vp, fp, fp, i32, C.c_float, fp]
    L.sur_last_error.argtypes = [vp]
    L.sur_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("sur_destroy", "sur_last_error"):
            getattr(L, name).restype = C.c_int
    _bound = True
    return L


class SurError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _dev(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError("expected a contiguous float32 tensor on the HIP device")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return None
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Surrogate:
    """One surrogate network (a sur_t handle) with its Adam state."""

    def __init__(self, H=128, W=128, channels=(32, 64, 128, 256), max_batch=64, seed=2405,
                 lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        p = sur_params()
        lib().sur_params_default(C.byref(p))
        p.H, p.W, p.max_batch, p.seed = H, W, max_batch, seed
        p.channels[:] = list(channels)
        p.lr, p.beta1, p.beta2, p.eps = lr, beta1, beta2, eps
        self.params = p
        h = C.c_void_p()
        rc = lib().sur_create(C.byref(p), _stream(stream), C.byref(h))
        if rc != SUR_OK:
            raise SurError(rc, "sur_create rejected the parameters")
        self.h = h
        n = C.c_int64()
        self._chk(lib().sur_num_params(self.h, C.byref(n)))
        self.n_params = n.value
        self.H, self.W, self.channels = H, W, tuple(channels)

    def _chk(self, rc):
        if rc != SUR_OK:
            raise SurError(rc, lib().sur_last_error(self.h).decode() if self.h else "")

    def close(self):
        if getattr(self, "h", None):
            lib().sur_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:       # interpreter shutdown: module globals may be gone
            pass

    def sur_infer(self, depth, pose, prev, out=None):
        import torch
        n = depth.shape[0]
        if out is None:
            out = torch.empty((n, self.H, self.W, 3), device=depth.device, dtype=torch.float32)
        self._chk(lib().sur_infer(self.h, _dev(depth), _dev(pose), _dev(prev), _dev(out), n))
        return out

    def sur_train_step(self, depth, pose, prev, target, want_loss=False):
        loss = C.c_float()
        self._chk(lib().sur_train_step(self.h, _dev(depth), _dev(pose), _dev(prev), _dev(target), depth.shape[0],
                                       C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def sur_compute_grads(self, depth, pose, prev, target):
        loss = C.c_float()
        self._chk(lib().sur_compute_grads(self.h, _dev(depth), _dev(pose), _dev(prev), _dev(target),
                                          depth.shape[0], C.byref(loss)))
        return loss.value

    def sur_contact_area(self, depth, disp, tol=0.02, out=None):
        import torch
        n = depth.shape[0]
        if out is None:
            out = torch.empty(n, device=depth.device, dtype=torch.float32)
        self._chk(lib().sur_contact_area(self.h, _dev(depth), _dev(disp), n, float(tol), _dev(out)))
        return out

    def sur_set_lr(self, lr):
        self._chk(lib().sur_set_lr(self.h, float(lr)))

    def sur_get_grads(self):
        g = np.zeros(self.n_params, np.float32)
        self._chk(lib().sur_get_grads(self.h, g.ctypes.data_as(C.c_void_p)))
        return g

    def sur_get_params(self):
        t = np.zeros(self.n_params, np.float32)
        self._chk(lib().sur_get_params(self.h, t.ctypes.data_as(C.c_void_p)))
        return t

    def sur_set_params(self, theta):
        t = np.ascontiguousarray(theta, np.float32)
        if t.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        self._chk(lib().sur_set_params(self.h, t.ctypes.data_as(C.c_void_p)))

    def sur_debug_read(self, which, layer, shape):
        """BF16 tensor (which 0: activation, 1: pre-activation gradient, 2:
        network input) of the last pass, returned as float64."""
        u = np.zeros(int(np.prod(shape)), np.uint16)
        self._chk(lib().sur_debug_read(self.h, int(which), int(layer), u.ctypes.data_as(C.c_void_p)))
        return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64).reshape(shape)

    def sur_save(self, path):
        self._chk(lib().sur_save(self.h, str(path).encode()))

    def sur_load(self, path):
        self._chk(lib().sur_load(self.h, str(path).encode()))

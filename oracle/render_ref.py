"""ctypes binding of the FP64 renderer oracle (render_oracle.c).

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's CPU baseline
leg, never by the product library."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "render_oracle.c")
LIB = os.path.join(HERE, "librender_oracle.so")


class Light(C.Structure):
    _fields_ = [("c", C.c_double * 3), ("e1", C.c_double * 3), ("e2", C.c_double * 3), ("L", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("out_w", C.c_int32), ("out_h", C.c_int32),
                ("Lx", C.c_double), ("Ly", C.c_double), ("spp", C.c_int32), ("bounces", C.c_int32),
                ("seed", C.c_uint64), ("n_lights", C.c_int32), ("tex_w", C.c_int32), ("tex_h", C.c_int32),
                ("_pad", C.c_int32)]


def build(force=False):
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC,
                               "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.rt_render_oracle.argtypes = [C.POINTER(Params), C.c_void_p, C.POINTER(Light), C.c_void_p, C.c_void_p]
        _lib.rt_render_oracle.restype = None
        _lib.rt_render_oracle_pixels.argtypes = [C.POINTER(Params), C.c_void_p, C.POINTER(Light), C.c_void_p,
                                                 C.c_void_p, C.c_int64, C.c_void_p]
        _lib.rt_render_oracle_pixels.restype = None
    return _lib


def lights_array(lights):
    arr = (Light * len(lights))()
    for k, l in enumerate(lights):
        arr[k].c[:] = list(l["c"]); arr[k].e1[:] = list(l["e1"]); arr[k].e2[:] = list(l["e2"])
        arr[k].L[:] = list(l["L"])
    return arr


def _params(h, t, Lx, Ly, lights, out_w, out_h, spp, seed, bounces):
    return Params(W=h.shape[1], H=h.shape[0], out_w=out_w, out_h=out_h, Lx=Lx, Ly=Ly, spp=spp, bounces=bounces,
                  seed=seed, n_lights=len(lights), tex_w=t.shape[1], tex_h=t.shape[0])


def render(height, Lx, Ly, lights, texture, out_w, out_h, spp, seed=1, bounces=2):
    """height: (H, W) metres; texture: (th, tw, 3); returns (out_h, out_w, 3)."""
    h = np.ascontiguousarray(height, np.float64)
    t = np.ascontiguousarray(texture, np.float64)
    p = _params(h, t, Lx, Ly, lights, out_w, out_h, spp, seed, bounces)
    out = np.zeros((out_h, out_w, 3))
    lib().rt_render_oracle(C.byref(p), h.ctypes.data, lights_array(lights), t.ctypes.data, out.ctypes.data)
    return out


def render_pixels(pixels, height, Lx, Ly, lights, texture, out_w, out_h, spp, seed=1, bounces=2):
    """The listed pixels (flat indices v * out_w + u) of the same image: (n, 3)."""
    h = np.ascontiguousarray(height, np.float64)
    t = np.ascontiguousarray(texture, np.float64)
    pix = np.ascontiguousarray(pixels, np.int64)
    p = _params(h, t, Lx, Ly, lights, out_w, out_h, spp, seed, bounces)
    out = np.zeros((len(pix), 3))
    lib().rt_render_oracle_pixels(C.byref(p), h.ctypes.data, lights_array(lights), t.ctypes.data, pix.ctypes.data,
                                  len(pix), out.ctypes.data)
    return out

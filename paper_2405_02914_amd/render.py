"""Python binding of the tactile image renderer in libimpm.so
(include/render.h): argument marshalling only.

The C names are kept (rt_workspace_bytes, rt_render, rt_render_work).  `Renderer` holds one
scene's lights, texture and workspace on the current HIP device and renders a
device height map (for instance the output of sim_surface_heightmap) into a
device image.  There is no fallback path: the library must have been built.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import impm


class rt_light(C.Structure):
    _fields_ = [("c", C.c_double * 3), ("e1", C.c_double * 3), ("e2", C.c_double * 3), ("L", C.c_double * 3)]


class rt_params(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("out_w", C.c_int32), ("out_h", C.c_int32),
                ("Lx", C.c_double), ("Ly", C.c_double), ("spp", C.c_int32), ("bounces", C.c_int32),
                ("seed", C.c_uint64), ("n_lights", C.c_int32), ("tex_w", C.c_int32), ("tex_h", C.c_int32),
                ("_pad", C.c_int32)]


EXPORTS = ("rt_workspace_bytes", "rt_render", "rt_render_work")

_bound = None


def lib():
    """libimpm.so with the renderer's signatures declared."""
    global _bound
    L = impm.lib()
    if _bound is not L:
        L.rt_workspace_bytes.argtypes = [C.POINTER(rt_params)]
        L.rt_workspace_bytes.restype = C.c_uint64
        L.rt_render.argtypes = [C.POINTER(rt_params), C.c_void_p, C.POINTER(rt_light), C.c_void_p, C.c_void_p,
                                C.c_void_p, C.c_uint64, C.c_void_p]
        L.rt_render.restype = C.c_int
        L.rt_render_work.argtypes = L.rt_render.argtypes + [C.POINTER(C.c_uint64)]
        L.rt_render_work.restype = C.c_int
        _bound = L
    return L


def light_records(lights):
    """ctypes array of rt_light from dicts with keys c, e1, e2, L."""
    arr = (rt_light * len(lights))()
    for k, l in enumerate(lights):
        arr[k].c[:] = [float(v) for v in l["c"]]
        arr[k].e1[:] = [float(v) for v in l["e1"]]
        arr[k].e2[:] = [float(v) for v in l["e2"]]
        arr[k].L[:] = [float(v) for v in l["L"]]
    return arr


def rt_workspace_bytes(params: rt_params) -> int:
    n = int(lib().rt_workspace_bytes(C.byref(params)))
    if n == 0:
        raise ValueError("rt_workspace_bytes: invalid renderer parameters")
    return n


def _device_args(name, params, height, lights, texture, out, workspace, stream):
    import torch
    for what, t in (("height", height), ("texture", texture), ("out", out), ("workspace", workspace)):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError(f"{name}: {what} must be a contiguous device tensor")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    return (C.byref(params), C.c_void_p(height.data_ptr()), light_records(lights), C.c_void_p(texture.data_ptr()),
            C.c_void_p(out.data_ptr()), C.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
            C.c_void_p(stream))


def _check(name, rc):
    if rc != 0:
        raise RuntimeError(f"{name} failed ({'invalid arguments' if rc == -1 else 'HIP error'}, code {rc})")


def rt_render(params: rt_params, height, lights, texture, out, workspace, stream=None) -> None:
    """Enqueue one render on `stream` (default: torch's current stream).
    height, texture, out and workspace are contiguous device tensors."""
    _check("rt_render", lib().rt_render(*_device_args("rt_render", params, height, lights, texture, out, workspace,
                                                      stream)))


def rt_render_work(params: rt_params, height, lights, texture, out, workspace, stream=None) -> dict:
    """rt_render, waited for, with its work counts."""
    work = (C.c_uint64 * 4)()
    _check("rt_render_work", lib().rt_render_work(*_device_args("rt_render_work", params, height, lights, texture,
                                                                out, workspace, stream), work))
    return dict(rays=int(work[0]), tiles=int(work[1]), cells=int(work[2]), triangles=int(work[3]))


class Renderer:
    """One scene (lights, texture, footprint Lx x Ly, samples, bounces, seed)
    rendering H x W height maps into out_h x out_w x 3 FP32 images on the
    current device."""

    def __init__(self, lights, texture, Lx, Ly, spp=128, bounces=2, seed=1):
        import torch
        tex = np.ascontiguousarray(texture, np.float32)
        self.texture = torch.from_numpy(tex).to("cuda")
        self.lights = [dict(l) for l in lights]
        self.Lx, self.Ly, self.spp, self.bounces, self.seed = float(Lx), float(Ly), int(spp), int(bounces), int(seed)
        self._ws = None

    def params(self, H, W, out_h, out_w) -> rt_params:
        return rt_params(W=W, H=H, out_w=out_w, out_h=out_h, Lx=self.Lx, Ly=self.Ly, spp=self.spp,
                         bounces=self.bounces, seed=self.seed, n_lights=len(self.lights),
                         tex_w=self.texture.shape[1], tex_h=self.texture.shape[0])

    def _prepare(self, height, out_h, out_w, out):
        import torch
        H, W = height.shape
        out_h = H if out_h is None else out_h
        out_w = W if out_w is None else out_w
        p = self.params(H, W, out_h, out_w)
        need = rt_workspace_bytes(p)
        if self._ws is None or self._ws.numel() < need:
            # torch's device allocations are aligned far beyond the 256 bytes required
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        if out is None:
            out = torch.empty((out_h, out_w, 3), dtype=torch.float32, device="cuda")
        return p, out

    def render(self, height, out_h=None, out_w=None, out=None, stream=None):
        """height: (H, W) FP32 device tensor (metres).  Returns (out_h, out_w, 3)."""
        p, out = self._prepare(height, out_h, out_w, out)
        rt_render(p, height, self.lights, self.texture, out, self._ws, stream)
        return out

    def render_work(self, height, out_h=None, out_w=None, out=None, stream=None):
        """render, waited for; returns (image, work counts)."""
        p, out = self._prepare(height, out_h, out_w, out)
        return out, rt_render_work(p, height, self.lights, self.texture, out, self._ws, stream)

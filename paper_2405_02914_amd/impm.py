"""Python binding of libimpm.so (include/impm.h): argument marshalling only.

Every function keeps the C name.  The library must have been built
(`python -m paper_2405_02914_amd.build` or `__graft_entry__.build()`); loading
fails loudly when it is missing: there is no fallback path.  PyTorch is used
only for device buffers and the current HIP stream when a caller asks for
device outputs.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libimpm.so")

SIM_OK, SIM_EINVAL, SIM_ENOMEM, SIM_EHIP, SIM_ENUMERIC, SIM_ESTATE = 0, -1, -2, -3, -4, -5
_ERRNAMES = {-1: "SIM_EINVAL", -2: "SIM_ENOMEM", -3: "SIM_EHIP", -4: "SIM_ENUMERIC", -5: "SIM_ESTATE"}


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class sim_params(C.Structure):
    _fields_ = [
        ("cells", C.c_int32 * 3), ("ppc", C.c_int32), ("dx", C.c_double),
        ("seed", C.c_uint64), ("E", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
        ("dt", C.c_double), ("subcycle", C.c_int32), ("pad_lateral", C.c_int32),
        ("pad_top", C.c_int32), ("pad_bottom", C.c_int32), ("band", C.c_int32),
        ("mode", C.c_int32), ("rest_limit", C.c_int32), ("rest_threshold", C.c_double),
        ("fixed_z_fraction", C.c_double), ("shape", C.c_int32), ("_pad0", C.c_int32),
        ("radius", C.c_double), ("half_length", C.c_double), ("half_extent", C.c_double * 3),
        ("fillet", C.c_double), ("pose0", C.c_double * 7), ("stress_each_pass", C.c_int32),
        ("_pad1", C.c_int32), ("hf_n", C.c_int32), ("_pad2", C.c_int32), ("hf_half", C.c_double),
        ("hf", C.POINTER(C.c_double)), ("object_mode", C.c_int32), ("_pad3", C.c_int32),
        ("object_density", C.c_double), ("object_cap", C.c_double), ("columns", C.POINTER(C.c_uint8)),
    ]


class sim_stats(C.Structure):
    _fields_ = [
        ("substeps", C.c_int64), ("steps", C.c_int64), ("passes", C.c_int64),
        ("limit_hits", C.c_int64), ("last_r", C.c_double), ("device_error", C.c_int32),
        ("_pad", C.c_int32), ("pose", C.c_double * 7), ("xo", C.c_double * 3),
        ("calib_particle", C.c_int64),
    ]


EXPORTS = ("sim_params_default", "sim_create", "sim_destroy", "sim_set_indenter_pose", "sim_step",
           "sim_synchronize", "sim_surface_heightmap", "sim_surface_displacement", "sim_get_stats",
           "sim_num_particles", "sim_grid_dims", "sim_read_particles", "sim_write_particles",
           "sim_read_rest", "sim_debug_keep_grid", "sim_read_grid", "sim_debug_force_passes",
           "sim_set_tile", "sim_set_tile_threads", "sim_profile", "sim_profile_read", "sim_last_error",
           "sim_batch_create", "sim_batch_destroy", "sim_batch_size", "sim_batch_get",
           "sim_batch_set_indenter_poses", "sim_batch_step", "sim_batch_synchronize",
           "sim_batch_heightmaps", "sim_batch_displacements", "sim_batch_last_error",
           "sim_autotune_tile", "sim_set_graph", "sim_set_compaction", "sim_batch_set_graph",
           "sim_indenter_depthmap", "sim_batch_depthmaps", "sim_surface_heightmap_noalloc",
           "sim_batch_set_active")

_lib = None


def lib():
    """Load libimpm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -m paper_2405_02914_amd.build)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp, fp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p
    L.sim_params_default.argtypes = [C.POINTER(sim_params)]
    L.sim_create.argtypes = [C.POINTER(sim_params), vp, C.POINTER(vp)]
    L.sim_destroy.argtypes = [vp]
    L.sim_destroy.restype = None
    L.sim_set_indenter_pose.argtypes = [vp, dp, dp]
    L.sim_step.argtypes = [vp, i32]
    L.sim_synchronize.argtypes = [vp]
    L.sim_surface_heightmap.argtypes = [vp, fp, i32, i32, i32]
    L.sim_surface_displacement.argtypes = [vp, fp, i32, i32, i32]
    L.sim_surface_heightmap_noalloc.argtypes = [vp, fp, i32, i32]
    L.sim_get_stats.argtypes = [vp, C.POINTER(sim_stats)]
    L.sim_num_particles.argtypes = [vp, C.POINTER(C.c_int64)]
    L.sim_grid_dims.argtypes = [vp, C.POINTER(C.c_int32)]
    L.sim_read_particles.argtypes = [vp, dp, fp, fp, fp]
    L.sim_write_particles.argtypes = [vp, dp, fp, fp, fp]
    L.sim_read_rest.argtypes = [vp, dp, vp]
    L.sim_debug_keep_grid.argtypes = [vp, i32]
    L.sim_read_grid.argtypes = [vp, fp, fp, fp]
    L.sim_debug_force_passes.argtypes = [vp, vp, i32]
    L.sim_set_tile.argtypes = [vp, i32, i32, i32]
    L.sim_set_tile_threads.argtypes = [vp, i32, i32, i32, i32]
    L.sim_profile.argtypes = [vp, i32]
    L.sim_set_graph.argtypes = [vp, i32]
    L.sim_set_compaction.argtypes = [vp, i32]
    L.sim_indenter_depthmap.argtypes = [vp, fp, i32, i32, C.c_double, i32]
    L.sim_batch_depthmaps.argtypes = [vp, fp, i32, i32, C.c_double, i32]
    L.sim_batch_set_graph.argtypes = [vp, i32]
    L.sim_batch_set_active.argtypes = [vp, C.POINTER(C.c_int32)]
    L.sim_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.sim_last_error.argtypes = [vp]
    L.sim_last_error.restype = C.c_char_p
    L.sim_batch_create.argtypes = [C.POINTER(sim_params), i32, vp, vp, C.POINTER(vp)]
    L.sim_batch_destroy.argtypes = [vp]
    L.sim_batch_destroy.restype = None
    L.sim_batch_size.argtypes = [vp, C.POINTER(C.c_int32)]
    L.sim_batch_get.argtypes = [vp, i32, C.POINTER(vp)]
    L.sim_batch_set_indenter_poses.argtypes = [vp, dp, dp]
    L.sim_batch_step.argtypes = [vp, i32]
    L.sim_batch_synchronize.argtypes = [vp]
    L.sim_batch_heightmaps.argtypes = [vp, fp, i32, i32, i32]
    L.sim_batch_displacements.argtypes = [vp, fp, i32, i32, i32]
    L.sim_batch_last_error.argtypes = [vp]
    L.sim_batch_last_error.restype = C.c_char_p
    L.sim_autotune_tile.argtypes = [C.POINTER(sim_params), i32, vp, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double)]
    for name in EXPORTS:
        if name not in ("sim_destroy", "sim_last_error", "sim_batch_destroy", "sim_batch_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def to_params(p) -> sim_params:
    """sim_params from a workloads.SensorParams-like object."""
    q = sim_params()
    q.cells[:] = list(p.cells)
    q.ppc, q.dx, q.seed = p.ppc, p.dx, p.seed
    q.E, q.nu, q.rho, q.dt, q.subcycle = p.E, p.nu, p.rho, p.dt, p.subcycle
    q.pad_lateral, q.pad_top, q.pad_bottom, q.band = p.pad_lateral, p.pad_top, p.pad_bottom, p.band
    q.mode, q.rest_limit, q.rest_threshold = p.mode, p.rest_limit, p.rest_threshold
    q.fixed_z_fraction, q.shape = p.fixed_z_fraction, p.shape
    q.radius, q.half_length = p.radius, p.half_length
    q.half_extent[:] = list(p.half_extent)
    q.fillet = p.fillet
    q.pose0[:] = list(p.pose0)
    q.stress_each_pass = p.stress_each_pass
    q.object_mode = getattr(p, "object_mode", 0)
    q.object_density = getattr(p, "object_density", p.rho)
    q.object_cap = getattr(p, "object_cap", 2.5e-3)
    if getattr(p, "columns", None) is not None:
        cols = np.ascontiguousarray(p.columns, np.uint8)
        q.columns = cols.ctypes.data_as(C.POINTER(C.c_uint8))
        q._keep_cols = cols              # the library copies the table at creation
    if getattr(p, "hf", None) is not None:
        t = np.ascontiguousarray(p.hf, np.float64)
        q.hf_n, q.hf_half = t.shape[0], p.hf_half
        q.hf = t.ctypes.data_as(C.POINTER(C.c_double))
        q._keep = t                      # the library copies the table at creation
    return q


class Sim:
    """One simulated sensor (a sim_t handle)."""

    def __init__(self, params, stream=None):
        self.params = params
        self._c = to_params(params)
        h = C.c_void_p()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        rc = lib().sim_create(C.byref(self._c), C.c_void_p(stream), C.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, "sim_create rejected the parameters")
        self.h = h
        n = C.c_int64()
        self._chk(lib().sim_num_particles(self.h, C.byref(n)))
        self.n = n.value
        d = (C.c_int32 * 3)()
        self._chk(lib().sim_grid_dims(self.h, d))
        self.nodes = tuple(d)
        self.n_nodes = int(np.prod(self.nodes))

    def _chk(self, rc):
        if rc != SIM_OK:
            msg = lib().sim_last_error(self.h).decode() if getattr(self, "h", None) else ""
            raise SimError(rc, msg)

    def close(self):
        if getattr(self, "h", None):
            lib().sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sim_set_indenter_pose(self, pos, quat):
        self._chk(lib().sim_set_indenter_pose(self.h, _p(np.ascontiguousarray(pos, np.float64)),
                                              _p(np.ascontiguousarray(quat, np.float64))))

    def sim_step(self, n):
        self._chk(lib().sim_step(self.h, int(n)))

    def run_schedule(self, segments):
        for n, pos, q in segments:
            self.sim_set_indenter_pose(pos, q)
            self.sim_step(n)

    def sim_synchronize(self):
        self._chk(lib().sim_synchronize(self.h))

    def sim_indenter_depthmap(self, W, H, scale=1.0, out=None):
        """(H - z_low) * scale per pixel; host numpy (H, W) unless `out` is a
        device tensor of H*W floats."""
        if out is not None:
            self._chk(lib().sim_indenter_depthmap(self.h, C.c_void_p(out.data_ptr()), W, H, float(scale), 1))
            return out
        o = np.zeros((H, W), np.float32)
        self._chk(lib().sim_indenter_depthmap(self.h, _p(o), W, H, float(scale), 0))
        return o

    def sim_surface_heightmap_noalloc(self, W, H, out):
        """Height map into the device tensor `out` (H*W floats) without a device
        allocation (fixed library workspace of 512*512 pixels)."""
        self._chk(lib().sim_surface_heightmap_noalloc(self.h, C.c_void_p(out.data_ptr()), W, H))
        return out

    def sim_surface_heightmap(self, W, H, out=None):
        """Host numpy (H, W) unless `out` is a device tensor of H*W floats."""
        if out is not None:
            self._chk(lib().sim_surface_heightmap(self.h, C.c_void_p(out.data_ptr()), W, H, 1))
            return out
        o = np.zeros((H, W), np.float32)
        self._chk(lib().sim_surface_heightmap(self.h, _p(o), W, H, 0))
        return o

    def sim_surface_displacement(self, W, H, out=None):
        if out is not None:
            self._chk(lib().sim_surface_displacement(self.h, C.c_void_p(out.data_ptr()), W, H, 1))
            return out
        o = np.zeros((H, W, 3), np.float32)
        self._chk(lib().sim_surface_displacement(self.h, _p(o), W, H, 0))
        return o

    def sim_get_stats(self, check=True):
        st = sim_stats()
        rc = lib().sim_get_stats(self.h, C.byref(st))
        if check:
            self._chk(rc)
        return dict(substeps=st.substeps, steps=st.steps, passes=st.passes,
                    limit_hits=st.limit_hits, last_r=st.last_r, device_error=st.device_error,
                    pose=list(st.pose), xo=list(st.xo), calib_particle=st.calib_particle)

    def sim_read_particles(self):
        x = np.zeros((self.n, 3)); v = np.zeros((self.n, 3), np.float32)
        Cm = np.zeros((self.n, 3, 3), np.float32); G = np.zeros((self.n, 3, 3), np.float32)
        self._chk(lib().sim_read_particles(self.h, _p(x), _p(v), _p(Cm), _p(G)))
        return x, v, Cm, G

    def sim_write_particles(self, x=None, v=None, Cm=None, G=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dt)
                for a, dt in ((x, np.float64), (v, np.float32), (Cm, np.float32), (G, np.float32))]
        self._chk(lib().sim_write_particles(self.h, *[_p(a) for a in arrs]))

    def sim_read_rest(self):
        X = np.zeros((self.n, 3)); fl = np.zeros(self.n, np.uint8)
        self._chk(lib().sim_read_rest(self.h, _p(X), _p(fl)))
        return X, fl

    def sim_debug_keep_grid(self, on=True):
        self._chk(lib().sim_debug_keep_grid(self.h, int(on)))

    def sim_read_grid(self):
        M = np.zeros(self.n_nodes, np.float32); MG = np.zeros((self.n_nodes, 3), np.float32)
        V = np.zeros((self.n_nodes, 3), np.float32)
        self._chk(lib().sim_read_grid(self.h, _p(M), _p(MG), _p(V)))
        return M, MG, V

    def sim_debug_force_passes(self, passes):
        a = np.ascontiguousarray(passes, np.int32)
        self._chk(lib().sim_debug_force_passes(self.h, _p(a), a.size))

    def sim_set_graph(self, on=True):
        self._chk(lib().sim_set_graph(self.h, int(on)))

    def sim_set_compaction(self, every_steps):
        self._chk(lib().sim_set_compaction(self.h, int(every_steps)))

    def sim_profile(self, on=True):
        self._chk(lib().sim_profile(self.h, int(on)))

    def sim_profile_read(self):
        ms = C.c_double(); k = C.c_int64()
        self._chk(lib().sim_profile_read(self.h, C.byref(ms), C.byref(k)))
        return ms.value, k.value

    def sim_set_tile(self, tx, ty, tz, threads=256):
        self._chk(lib().sim_set_tile_threads(self.h, tx, ty, tz, threads))


def sim_params_default() -> sim_params:
    p = sim_params()
    rc = lib().sim_params_default(C.byref(p))
    if rc != SIM_OK:
        raise SimError(rc, "sim_params_default")
    return p


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    return C.c_void_p(stream)


class _Borrowed(Sim):
    """A sensor owned by a batch (not destroyed by Python)."""

    def __init__(self, handle, params):
        self.params = params
        self.h = handle
        n = C.c_int64()
        self._chk(lib().sim_num_particles(self.h, C.byref(n)))
        self.n = n.value
        d = (C.c_int32 * 3)()
        self._chk(lib().sim_grid_dims(self.h, d))
        self.nodes = tuple(d)
        self.n_nodes = int(np.prod(self.nodes))

    def close(self):
        self.h = None


class Batch:
    """Many independent sensors stepped together (a sim_batch_t handle)."""

    def __init__(self, params_list, tiles=None, stream=None):
        n = len(params_list)
        recs = [to_params(p) for p in params_list]     # hold the height-field tables
        arr = (sim_params * n)(*recs)
        self._arr = arr
        t = None
        if tiles is not None:
            t = np.ascontiguousarray(np.asarray(tiles, np.int32).reshape(n, 4))
        h = C.c_void_p()
        rc = lib().sim_batch_create(arr, n, _p(t), _stream(stream), C.byref(h))
        if rc != SIM_OK:
            raise SimError(rc, "sim_batch_create rejected the parameters")
        self.h = h
        self.n = n
        self.sensors = []
        for i in range(n):
            sh = C.c_void_p()
            self._chk(lib().sim_batch_get(self.h, i, C.byref(sh)))
            self.sensors.append(_Borrowed(sh, params_list[i]))

    def _chk(self, rc):
        if rc != SIM_OK:
            raise SimError(rc, lib().sim_batch_last_error(self.h).decode() if self.h else "")

    def close(self):
        if getattr(self, "h", None):
            for s in self.sensors:
                s.close()
            lib().sim_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sim_batch_set_indenter_poses(self, pos, quat):
        self._chk(lib().sim_batch_set_indenter_poses(self.h, _p(np.ascontiguousarray(pos, np.float64)),
                                                     _p(np.ascontiguousarray(quat, np.float64))))

    def sim_batch_set_graph(self, on=True):
        self._chk(lib().sim_batch_set_graph(self.h, int(on)))

    def sim_batch_set_active(self, flags):
        """Members the following sim_batch_step calls advance (n booleans)."""
        a = np.ascontiguousarray(np.asarray(flags).reshape(self.n) != 0, np.int32)
        self._chk(lib().sim_batch_set_active(self.h, a.ctypes.data_as(C.POINTER(C.c_int32))))

    def sim_batch_step(self, n):
        self._chk(lib().sim_batch_step(self.h, int(n)))

    def sim_batch_synchronize(self):
        self._chk(lib().sim_batch_synchronize(self.h))

    def sim_batch_heightmaps(self, W, H, out=None):
        if out is not None:
            self._chk(lib().sim_batch_heightmaps(self.h, C.c_void_p(out.data_ptr()), W, H, 1))
            return out
        o = np.zeros((self.n, H, W), np.float32)
        self._chk(lib().sim_batch_heightmaps(self.h, _p(o), W, H, 0))
        return o

    def sim_batch_depthmaps(self, W, H, scale=1.0, out=None):
        if out is not None:
            self._chk(lib().sim_batch_depthmaps(self.h, C.c_void_p(out.data_ptr()), W, H, float(scale), 1))
            return out
        o = np.zeros((self.n, H, W), np.float32)
        self._chk(lib().sim_batch_depthmaps(self.h, _p(o), W, H, float(scale), 0))
        return o

    def sim_batch_displacements(self, W, H, out=None):
        if out is not None:
            self._chk(lib().sim_batch_displacements(self.h, C.c_void_p(out.data_ptr()), W, H, 1))
            return out
        o = np.zeros((self.n, H, W, 3), np.float32)
        self._chk(lib().sim_batch_displacements(self.h, _p(o), W, H, 0))
        return o


def sim_autotune_tile(params, steps=8, stream=None):
    """Fastest compiled tile shape (tx, ty, tz, threads) for these sensor
    parameters and its time per executed step (ms)."""
    q = to_params(params)
    out = (C.c_int32 * 4)()
    ms = C.c_double()
    rc = lib().sim_autotune_tile(C.byref(q), int(steps), _stream(stream), out, C.byref(ms))
    if rc != SIM_OK:
        raise SimError(rc, "sim_autotune_tile")
    return tuple(out), ms.value

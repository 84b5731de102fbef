"""ctypes binding of the FP64 CPU oracle (impm_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this module; the product library never does.  It shares no
code with the HIP path; the only common input is the parameter record of
`paper_2405_02914_amd.workloads`, which holds no arithmetic of the method.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "impm_oracle.c")
LIB = os.path.join(HERE, "libimpm_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fused multiply-add contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [
        ("cells", C.c_int32 * 3), ("ppc", C.c_int32), ("dx", C.c_double),
        ("seed", C.c_uint64), ("E", C.c_double), ("nu", C.c_double),
        ("rho", C.c_double), ("dt", C.c_double), ("subcycle", C.c_int32),
        ("pad_lateral", C.c_int32), ("pad_top", C.c_int32), ("pad_bottom", C.c_int32),
        ("band", C.c_int32), ("mode", C.c_int32), ("rest_limit", C.c_int32),
        ("rest_threshold", C.c_double), ("fixed_z_fraction", C.c_double),
        ("shape", C.c_int32), ("_pad0", C.c_int32), ("radius", C.c_double),
        ("half_length", C.c_double), ("half_extent", C.c_double * 3),
        ("fillet", C.c_double), ("pose0", C.c_double * 7),
        ("stress_each_pass", C.c_int32), ("_pad1", C.c_int32),
        ("hf_n", C.c_int32), ("_pad2", C.c_int32), ("hf_half", C.c_double),
        ("hf", C.POINTER(C.c_double)),
        ("object_mode", C.c_int32), ("_pad3", C.c_int32), ("object_density", C.c_double),
        ("object_cap", C.c_double), ("columns", C.POINTER(C.c_uint8)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        P = C.c_void_p
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
        i32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        i64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Params)]
        L.orc_destroy.argtypes = [P]
        L.orc_step.argtypes = [P, C.c_int32]
        L.orc_set_target_pose.argtypes = [P, dp, dp]
        L.orc_num_particles.restype = C.c_int64
        L.orc_num_particles.argtypes = [P]
        L.orc_error.restype = C.c_int32
        L.orc_error.argtypes = [P]
        L.orc_calib_particle.restype = C.c_int64
        L.orc_calib_particle.argtypes = [P]
        L.orc_grid_dims.argtypes = [P, i32]
        for f in ("orc_get_state", "orc_set_state"):
            getattr(L, f).argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_get_rest.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_get_grid.argtypes = [P, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_set_grid.argtypes = [P, C.c_void_p, C.c_void_p]
        L.orc_min_margin.restype = C.c_double
        L.orc_min_margin.argtypes = [P]
        L.orc_set_pose.argtypes = [P, dp, dp]
        L.orc_set_threads.restype = C.c_int32
        L.orc_set_threads.argtypes = [P, C.c_int32]
        L.orc_num_object.restype = C.c_int64
        L.orc_num_object.argtypes = [P]
        L.orc_get_object.argtypes = [P, C.c_void_p, C.c_void_p]
        L.orc_object_mass.restype = C.c_double
        L.orc_object_mass.argtypes = [P]
        L.orc_phase_p2g_object.argtypes = [P, C.c_double]
        L.orc_get_counters.argtypes = [P, i64, C.POINTER(C.c_double)]
        L.orc_get_pose.argtypes = [P, dp]
        L.orc_get_xo.argtypes = [P, dp]
        L.orc_force_passes.argtypes = [P, i32, C.c_int64]
        L.orc_enable_pass_log.argtypes = [P, C.c_int64]
        L.orc_get_pass_log.restype = C.c_int64
        L.orc_get_pass_log.argtypes = [P, i32, C.c_int64]
        L.orc_phase_p2g.argtypes = [P, C.c_double]
        L.orc_phase_p2g_momentum.argtypes = [P]
        L.orc_phase_grid.argtypes = [P, C.c_int, C.c_int]
        L.orc_phase_g2p.argtypes = [P, C.c_int]
        L.orc_phase_commit.argtypes = [P, C.c_double]
        L.orc_inside_mask.argtypes = [P, u8]
        L.orc_point_phi.argtypes = [P, dp, C.c_int64, dp]
        L.orc_indenter_depthmap.argtypes = [P, C.c_int, C.c_int, C.c_double, dp]
        L.orc_indenter_depthmap.restype = C.c_int
        L.orc_energy.restype = C.c_double
        L.orc_energy.argtypes = [P]
        L.orc_surface_displacement.argtypes = [P, dp, C.c_int, C.c_int]
        L.orc_surface_heightmap.argtypes = [P, dp, C.c_int, C.c_int]
        L.orc_polar.argtypes = [dp, dp]
        L.orc_kirchhoff.argtypes = [dp, C.c_double, C.c_double, dp]
        L.orc_splitmix64_at.restype = C.c_uint64
        L.orc_splitmix64_at.argtypes = [C.c_uint64, C.c_uint64]
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def to_params(p) -> _Params:
    q = _Params()
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
    q.object_mode, q.object_density, q.object_cap = p.object_mode, p.object_density, p.object_cap
    if getattr(p, "columns", None) is not None:
        cols = np.ascontiguousarray(p.columns, np.uint8)
        q.columns = cols.ctypes.data_as(C.POINTER(C.c_uint8))
        q._keep_cols = cols              # the oracle copies the table at creation
    if getattr(p, "hf", None) is not None:
        t = np.ascontiguousarray(p.hf, np.float64)
        q.hf_n, q.hf_half = t.shape[0], p.hf_half
        q.hf = t.ctypes.data_as(C.POINTER(C.c_double))
        q._keep = t                      # the oracle copies the table at creation
    return q


class OracleSim:
    """FP64 reference simulation of one sensor."""

    def __init__(self, params):
        self.params = params
        self._p = to_params(params)
        self.h = lib().orc_create(C.byref(self._p))
        if not self.h:
            raise ValueError("oracle rejected the parameters")
        self.n = lib().orc_num_particles(self.h)
        nn = np.zeros(3, np.int32)
        lib().orc_grid_dims(self.h, nn)
        self.nodes = tuple(int(v) for v in nn)
        self.n_nodes = int(np.prod(self.nodes))

    def close(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def __del__(self):
        self.close()

    # -- driving
    def set_target_pose(self, pos, quat):
        lib().orc_set_target_pose(self.h, np.asarray(pos, np.float64), np.asarray(quat, np.float64))

    def step(self, n):
        rc = lib().orc_step(self.h, int(n))
        if rc == -2:
            raise FloatingPointError(f"oracle state invalid (code {lib().orc_error(self.h)})")
        if rc != 0:
            raise ValueError("bad substep count")

    def run_schedule(self, segments):
        for n, pos, q in segments:
            self.set_target_pose(pos, q)
            self.step(n)

    def force_passes(self, passes):
        a = np.ascontiguousarray(passes, np.int32)
        lib().orc_force_passes(self.h, a, a.size)

    def enable_pass_log(self, cap):
        lib().orc_enable_pass_log(self.h, int(cap))

    def pass_log(self, cap=1 << 20):
        out = np.zeros(cap, np.int32)
        n = lib().orc_get_pass_log(self.h, out, cap)
        return out[:min(n, cap)]

    # -- state
    def state(self):
        x = np.zeros((self.n, 3)); v = np.zeros((self.n, 3))
        Cm = np.zeros((self.n, 3, 3)); F = np.zeros((self.n, 3, 3))
        lib().orc_get_state(self.h, _ptr(x), _ptr(v), _ptr(Cm), _ptr(F))
        return x, v, Cm, F

    def set_state(self, x=None, v=None, Cm=None, F=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (x, v, Cm, F)]
        lib().orc_set_state(self.h, *[_ptr(a) for a in arrs])

    def rest(self):
        X = np.zeros((self.n, 3)); b = np.zeros(self.n, np.uint8); s = np.zeros(self.n, np.uint8)
        lib().orc_get_rest(self.h, _ptr(X), _ptr(b), _ptr(s))
        return X, b.astype(bool), s.astype(bool)

    def grid(self):
        M = np.zeros(self.n_nodes); MG = np.zeros((self.n_nodes, 3)); V = np.zeros((self.n_nodes, 3))
        lib().orc_get_grid(self.h, _ptr(M), _ptr(MG), _ptr(V))
        return M, MG, V

    def set_grid(self, M=None, MG=None):
        arrs = [None if a is None else np.ascontiguousarray(a, np.float64) for a in (M, MG)]
        lib().orc_set_grid(self.h, *[_ptr(a) for a in arrs])

    def counters(self):
        c = np.zeros(4, np.int64); r = C.c_double()
        lib().orc_get_counters(self.h, c, C.byref(r))
        return dict(substeps=int(c[0]), steps=int(c[1]), passes=int(c[2]),
                    limit_hits=int(c[3]), last_r=r.value)

    def set_threads(self, n):
        """OpenMP threads of the timing leg (1: the plain serial loops)."""
        return int(lib().orc_set_threads(self.h, int(n)))

    def objects(self):
        """Object particles: (world positions, body-frame positions), each (n_obj, 3)."""
        n = int(lib().orc_num_object(self.h))
        x = np.zeros((n, 3)); b = np.zeros((n, 3))
        lib().orc_get_object(self.h, _ptr(x), _ptr(b))
        return x, b

    def object_mass(self):
        return float(lib().orc_object_mass(self.h))

    def p2g_with_object(self, h=None):
        lib().orc_phase_p2g_object(self.h, self.params.dt if h is None else h)

    def min_margin(self):
        """min |r - threshold| / threshold over every relative-rest test so far."""
        return float(lib().orc_min_margin(self.h))

    def set_pose(self, pos, quat):
        lib().orc_set_pose(self.h, np.asarray(pos, np.float64), np.asarray(quat, np.float64))

    def pose(self):
        o = np.zeros(7); lib().orc_get_pose(self.h, o); return o

    def xo(self):
        o = np.zeros(3); lib().orc_get_xo(self.h, o); return o

    @property
    def calib_particle(self):
        return int(lib().orc_calib_particle(self.h))

    # -- phases (invariant tests)
    def p2g(self, h=None):
        lib().orc_phase_p2g(self.h, self.params.dt if h is None else h)

    def p2g_momentum(self):
        lib().orc_phase_p2g_momentum(self.h)

    def grid_update(self, contact=True, bc=True):
        lib().orc_phase_grid(self.h, int(contact), int(bc))

    def g2p(self, bottom_rule=False):
        lib().orc_phase_g2p(self.h, int(bottom_rule))

    def commit(self, h=None):
        lib().orc_phase_commit(self.h, self.params.dt if h is None else h)

    def point_phi(self, X):
        X = np.ascontiguousarray(X, np.float64).reshape(-1, 3)
        out = np.zeros(len(X)); lib().orc_point_phi(self.h, X, len(X), out); return out

    def indenter_depthmap(self, W, H, scale=1.0):
        out = np.zeros((H, W))
        if lib().orc_indenter_depthmap(self.h, W, H, scale, out) != 0:
            raise ValueError("the depth map needs an indenter rotated about z only")
        return out

    def inside_mask(self):
        m = np.zeros(self.n_nodes, np.uint8); lib().orc_inside_mask(self.h, m); return m.astype(bool)

    def energy(self):
        return float(lib().orc_energy(self.h))

    def surface_displacement(self, W, H):
        o = np.zeros((H, W, 3)); lib().orc_surface_displacement(self.h, o, W, H); return o

    def surface_heightmap(self, W, H):
        o = np.zeros((H, W)); lib().orc_surface_heightmap(self.h, o, W, H); return o


def polar(F):
    R = np.zeros(9); lib().orc_polar(np.ascontiguousarray(F, np.float64).reshape(9), R)
    return R.reshape(3, 3)


def kirchhoff(F, mu, lam):
    t = np.zeros(9)
    lib().orc_kirchhoff(np.ascontiguousarray(F, np.float64).reshape(9), mu, lam, t)
    return t.reshape(3, 3)


def splitmix64_at(seed, t):
    return int(lib().orc_splitmix64_at(seed, t))

"""Seeded synthetic workloads: sensor parameters, indenter motion schedules and
random particle states.

This module is the only one that the oracle side and the HIP side both use.  It
holds input recipes (sizes, material constants, poses, random numbers) and none
of the method's arithmetic.

Units are SI (m, s, kg, Pa).  Coordinates are slab-local: the origin is the
slab's (-x, -y) bottom corner and z points up.  Quaternions are body->world,
(w, x, y, z).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SHAPE_NONE, SHAPE_SPHERE, SHAPE_CAPSULE, SHAPE_BOX, SHAPE_HEIGHTFIELD = 0, 1, 2, 3, 4
MODE_IMPM, MODE_PLAIN = 0, 1
OBJECT_COLLIDER, OBJECT_PARTICLES = 0, 1


@dataclasses.dataclass
class SensorParams:
    """One elastomer slab, its background grid, material and indenter."""
    cells: tuple = (32, 32, 8)        # slab cells per axis
    dx: float = 0.5e-3                # grid spacing (m)
    ppc: int = 8                      # particles per cell (a cube: 1, 8, 27)
    seed: int = 2405
    E: float = 3.0e5                  # Young's modulus (Pa)
    nu: float = 0.45                  # Poisson's ratio
    rho: float = 1000.0               # density (kg/m^3)
    dt: float = 2.0e-5                # configured substep (s)
    subcycle: int = 1                 # executed steps per configured substep
    pad_lateral: int = 4              # empty cells beside the slab
    pad_top: int = 4                  # empty cells above the slab
    pad_bottom: int = 2               # cells below the slab's bottom face
    band: int = 2                     # boundary band of zero-velocity nodes
    mode: int = MODE_IMPM
    rest_limit: int = 10              # LIMIT of the IMPM loop
    rest_threshold: float = 0.5       # threshold of the relative-rest test
    fixed_z_fraction: float = 0.5     # "lower half layer" whose z velocity is zeroed
    shape: int = SHAPE_SPHERE
    radius: float = 4.0e-3
    half_length: float = 0.0
    half_extent: tuple = (0.0, 0.0, 0.0)
    fillet: float = 0.0
    pose0: tuple = (8.0e-3, 8.0e-3, 8.0e-3, 1.0, 0.0, 0.0, 0.0)
    stress_each_pass: int = 0         # 1: every IMPM pass re-adds the elastic impulse
    # height-field indenter: (n, n) body-frame heights over [-hf_half, hf_half]^2
    hf: object = dataclasses.field(default=None, compare=False, repr=False)
    hf_half: float = 0.0
    # object representation: 0 rigid collider at the grid, 1 object particles
    object_mode: int = 0
    object_density: float = 1000.0    # kg/m^3 of the object particles
    object_cap: float = 2.5e-3        # object particles fill the body this far above its lowest point
    # shaped elastomer: (Ny, Nx) column heights in cells (None: the full cuboid)
    columns: object = dataclasses.field(default=None, compare=False, repr=False)

    @property
    def n_particles(self) -> int:
        if self.columns is not None:
            return int(np.asarray(self.columns, np.int64).sum()) * self.ppc
        return self.cells[0] * self.cells[1] * self.cells[2] * self.ppc

    @property
    def nodes(self) -> tuple:
        return (self.cells[0] + 2 * self.pad_lateral + 1,
                self.cells[1] + 2 * self.pad_lateral + 1,
                self.cells[2] + self.pad_bottom + self.pad_top + 1)

    @property
    def height(self) -> float:
        return self.cells[2] * self.dx

    @property
    def lengths(self) -> tuple:
        return tuple(c * self.dx for c in self.cells)

    def replace(self, **kw) -> "SensorParams":
        return dataclasses.replace(self, **kw)


def padding_for(dx: float) -> int:
    """Lateral and top padding in cells: at least 4 cells and at least 2 mm."""
    return max(4, int(math.ceil(2.0e-3 / dx - 1e-9)))


def perlin2(x, y, seed: int):
    """Perlin's gradient noise in 2-D (improved fade 6t^5 - 15t^4 + 10t^3, eight
    gradient directions picked by a seeded permutation hash); values in about
    [-1, 1], zero at integer lattice points."""
    perm = np.random.default_rng(seed).permutation(256)
    perm = np.concatenate([perm, perm])
    xi, yi = np.floor(x).astype(np.int64), np.floor(y).astype(np.int64)
    fx, fy = x - xi, y - yi
    xi &= 255
    yi &= 255
    g = np.array([(1, 1), (-1, 1), (1, -1), (-1, -1), (1, 0), (-1, 0), (0, 1), (0, -1)], np.float64)

    def corner(dx, dy):
        h = perm[perm[xi + dx] + yi + dy] & 7
        return g[h, 0] * (fx - dx) + g[h, 1] * (fy - dy)

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    u, v = fade(fx), fade(fy)
    a = corner(0, 0) + u * (corner(1, 0) - corner(0, 0))
    b = corner(0, 1) + u * (corner(1, 1) - corner(0, 1))
    return a + v * (b - a)


def heightfield_table(seed: int, footprint: float, amplitude: float, wavelength: float,
                      bowl_radius: float, n: int = 65):
    """Lower surface of a textured indenter: amplitude * perlin(x / wavelength,
    y / wavelength) + r^2 / (2 bowl_radius) sampled on an n x n lattice over
    [-footprint, footprint]^2 (row j = y), shifted so that its lowest sample
    inside the disc r <= footprint is at height 0."""
    t = np.linspace(-footprint, footprint, n)
    X, Y = np.meshgrid(t, t, indexing="xy")
    off = np.random.default_rng(seed + 1).uniform(0.0, 64.0, size=2)
    z = amplitude * perlin2(X / wavelength + off[0], Y / wavelength + off[1], seed) \
        + (X * X + Y * Y) / (2.0 * bowl_radius)
    disc = X * X + Y * Y <= footprint * footprint
    return z - z[disc].min()


def holed_disc_table(r_out: float, r_hole: float, fillet: float, hole_fillet: float,
                     hole_depth: float, n: int = 129, skirt: float = 0.5e-3, skirt_slope: float = 5.0):
    """Lower surface of a flat-faced disc indenter with a central circular hole
    (a stand-in for an indenter with a recessed centre): height 0 on the
    annular face r_hole <= r <= r_out - fillet, the outer edge rounded with
    radius `fillet` up to height `fillet` at r = r_out, then a steep skirt
    (rising skirt_slope per unit radius) out to r_out + skirt, so that the
    solid's vertical side wall stands well above the slab; the hole's edge
    rounded with radius `hole_fillet` down from the face and the hole floor at
    `hole_depth` above the face.  Sampled on an n x n lattice over
    [-R, R]^2 with R = r_out + skirt (row j = y); the footprint disc is r <= R."""
    R = r_out + skirt
    t = np.linspace(-R, R, n)
    X, Y = np.meshgrid(t, t, indexing="xy")
    r = np.hypot(X, Y)
    z = np.zeros_like(r)
    edge = r > r_out - fillet
    q = np.clip(r[edge] - (r_out - fillet), 0.0, fillet)
    z[edge] = fillet - np.sqrt(fillet * fillet - q * q)
    out = r > r_out
    z[out] = fillet + skirt_slope * (r[out] - r_out)
    inner = r < r_hole + hole_fillet
    q = np.clip((r_hole + hole_fillet) - r[inner], 0.0, hole_fillet)
    z[inner] = np.minimum(hole_fillet - np.sqrt(hole_fillet * hole_fillet - q * q), hole_depth)
    z[r <= r_hole] = hole_depth
    return z


def protocol_sensor(dx: float = 0.25e-3, cells=(128, 128, 32), r_out: float = 4.0e-3,
                    r_hole: float = 1.5e-3, mode: int = MODE_IMPM, subcycle: int = 4, **kw) -> SensorParams:
    """The slab of the full-resolution sensor with the holed-disc indenter
    (outer edge rounded 0.75 mm, a steep 0.5 mm skirt beyond it, hole edge
    0.3 mm, hole floor 1.0 mm above the face) centred over it, its face
    touching the top surface."""
    L, H = cells[0] * dx, cells[2] * dx
    pad = padding_for(dx)
    tab = holed_disc_table(r_out, r_hole, 0.75e-3, 0.3e-3, 1.0e-3)
    p = SensorParams(cells=tuple(cells), dx=dx, pad_lateral=pad, pad_top=pad, mode=mode, subcycle=subcycle,
                     shape=SHAPE_HEIGHTFIELD, hf=tab, hf_half=r_out + 0.5e-3,
                     pose0=(L / 2, cells[1] * dx / 2, H, 1.0, 0.0, 0.0, 0.0))
    return p.replace(**kw) if kw else p


def protocol_schedule(pose0, kind: str, sign: float = 1.0, press: float = 0.5e-3, n_press: int = 250,
                      increments: int = 5, step_mm: float = 1.0, step_deg: float = 5.0,
                      n_per_increment: int = 500, n_per_degree_step: int = 250):
    """The slip / rotation protocol of the paper's experiments (Sec. IV-A),
    synthetic: press `press` straight down over n_press substeps, then either
    slip `increments` steps of `step_mm` mm along sign * x ("slip") or rotate
    `increments` steps of `step_deg` degrees about the normal, sign +1 counter-
    clockwise ("rotate").  Returns the segment list (n, target_pos,
    target_quat); a height map is taken after the press and after every
    increment (the caller takes one per segment)."""
    x0, y0, z0 = pose0[:3]
    segs = [(n_press, (x0, y0, z0 - press), (1.0, 0.0, 0.0, 0.0))]
    for k in range(1, increments + 1):
        if kind == "slip":
            segs.append((n_per_increment, (x0 + sign * step_mm * 1e-3 * k, y0, z0 - press), (1.0, 0.0, 0.0, 0.0)))
        elif kind == "rotate":
            segs.append((n_per_degree_step, (x0, y0, z0 - press), quat_about_z(sign * step_deg * k)))
        else:
            raise ValueError(kind)
    return segs


def dome_columns(cells, dx: float, radius: float, base_cells: int, centre=None):
    """Column heights of a shaped elastomer: a flat pad of base_cells layers
    under a spherical cap of the given radius (m), clipped to the slab's
    height and outline (a dome-topped gel).  Returns (Ny, Nx) uint8."""
    Nx, Ny, Nz = cells
    cx, cy = centre if centre is not None else (Nx * dx / 2, Ny * dx / 2)
    x = (np.arange(Nx) + 0.5) * dx - cx
    y = (np.arange(Ny) + 0.5) * dx - cy
    X, Y = np.meshgrid(x, y, indexing="xy")
    r2 = X * X + Y * Y
    top = Nz * dx
    cap = np.where(r2 < radius * radius, np.sqrt(np.maximum(radius * radius - r2, 0.0)) - (radius - (top - base_cells * dx)), 0.0)
    h = base_cells + np.floor(np.maximum(cap, 0.0) / dx + 1e-9)
    return np.clip(h, 0, Nz).astype(np.uint8)


def disc_columns(cells, dx: float, radius: float, centre=None):
    """Column heights of a round pad: full height inside the disc, empty outside."""
    Nx, Ny, Nz = cells
    cx, cy = centre if centre is not None else (Nx * dx / 2, Ny * dx / 2)
    x = (np.arange(Nx) + 0.5) * dx - cx
    y = (np.arange(Ny) + 0.5) * dx - cy
    X, Y = np.meshgrid(x, y, indexing="xy")
    return np.where(X * X + Y * Y <= radius * radius, Nz, 0).astype(np.uint8)


def quat_about_z(deg: float) -> tuple:
    h = math.radians(deg) * 0.5
    return (math.cos(h), 0.0, 0.0, math.sin(h))


def config1(subcycle: int = 1, **kw) -> SensorParams:
    """Single sensor: slab 16x16x4 mm, grid 32x32x8 (dx 0.5 mm), 65,536 particles,
    sphere r = 4 mm whose lowest point starts on the slab's top surface over the centre."""
    dx = 0.5e-3
    pad = padding_for(dx)
    p = SensorParams(cells=(32, 32, 8), dx=dx, pad_lateral=pad, pad_top=pad,
                     shape=SHAPE_SPHERE, radius=4.0e-3,
                     pose0=(8.0e-3, 8.0e-3, 4.0e-3 + 4.0e-3, 1.0, 0.0, 0.0, 0.0),
                     subcycle=subcycle)
    return p.replace(**kw) if kw else p


def config1_schedule(n_substeps: int = 100, depth: float = 1.0e-3):
    """Press the sphere `depth` straight down at constant speed over n substeps.
    Returns a list of (n_substeps, target_pos, target_quat) segments."""
    p = config1()
    x, y, z = p.pose0[:3]
    return [(n_substeps, (x, y, z - depth), (1.0, 0.0, 0.0, 0.0))]


def config2(subcycle: int = 1, **kw) -> SensorParams:
    """Full sensor resolution: slab 32x32x8 mm on a 128x128x32 grid (dx 0.25 mm),
    4,194,304 particles; capsule rod r = 3 mm (straight half-length 6 mm along
    body x) lying over the centre with its lowest line on the top surface."""
    dx = 0.25e-3
    pad = padding_for(dx)
    p = SensorParams(cells=(128, 128, 32), dx=dx, pad_lateral=pad, pad_top=pad,
                     shape=SHAPE_CAPSULE, radius=3.0e-3, half_length=6.0e-3,
                     pose0=(16.0e-3, 16.0e-3, 8.0e-3 + 3.0e-3, 1.0, 0.0, 0.0, 0.0),
                     subcycle=subcycle)
    return p.replace(**kw) if kw else p


def config2_schedule(total: int = 2000, frame: int = 50, press: float = 1.5e-3,
                     slip: float = 2.0e-3, rot_deg: float = 30.0):
    """Press `press` over the first quarter of the substeps, then slip `slip` along
    +x while rotating `rot_deg` about the normal over the rest, one segment per
    output frame.  Returns a list of (n_substeps, target_pos, target_quat)."""
    p = config2()
    x0, y0, z0 = p.pose0[:3]
    n_press = total // 4
    segs = []
    done = 0
    while done < total:
        n = min(frame, total - done)
        end = done + n
        if end <= n_press:
            a = end / n_press
            pos = (x0, y0, z0 - press * a)
            q = (1.0, 0.0, 0.0, 0.0)
        else:
            if done < n_press:          # a frame that straddles the phase change
                n = n_press - done
                end = n_press
                pos, q = (x0, y0, z0 - press), (1.0, 0.0, 0.0, 0.0)
                segs.append((n, pos, q))
                done = end
                continue
            b = (end - n_press) / (total - n_press)
            pos = (x0 + slip * b, y0, z0 - press)
            q = quat_about_z(rot_deg * b)
        segs.append((n, pos, q))
        done = end
    return segs


def small_sensor(cells=(8, 8, 4), dx=0.5e-3, **kw) -> SensorParams:
    """A slab small enough for the oracle to step in well under a second."""
    pad = kw.pop("pad", 4)
    L = [c * dx for c in cells]
    H = cells[2] * dx
    radius = kw.pop("radius", 1.5e-3)
    p = SensorParams(cells=tuple(cells), dx=dx, pad_lateral=pad, pad_top=pad,
                     shape=kw.pop("shape", SHAPE_SPHERE), radius=radius,
                     pose0=(L[0] / 2, L[1] / 2, H + radius, 1.0, 0.0, 0.0, 0.0))
    return p.replace(**kw) if kw else p


def representable_positions(params: SensorParams, x: np.ndarray) -> np.ndarray:
    """Round positions (metres, FP64) to the lattice a device holding each particle
    as an integer cell plus an FP32 offset inside it can store exactly:
    x = (cell + fl32(offset)) dx in slab coordinates."""
    x = np.asarray(x, dtype=np.float64)
    g = x / params.dx
    cell = np.floor(g)
    off = (g - cell).astype(np.float32).astype(np.float64)
    return (cell + off) * params.dx


def random_state(params: SensorParams, x_rest: np.ndarray, seed: int,
                 v_scale: float = 1e-2, c_scale: float = 20.0, g_scale: float = 1e-2,
                 x_scale: float = 0.05):
    """A seeded random particle state around the rest configuration.

    x_rest is (n, 3) in metres.  Returns (x, v, C, G) with x float64 (n,3) on the
    device-representable lattice, and float32 v (n,3), C (n,3,3) and G = F - I
    (n,3,3): positions jittered by up to x_scale*dx, velocities ~ N(0, v_scale)
    m/s, C ~ N(0, c_scale) 1/s, G ~ N(0, g_scale).  Both sides start from exactly
    these values (F = I + G is exact in FP64).
    """
    rng = np.random.default_rng(seed)
    n = x_rest.shape[0]
    x = x_rest + rng.uniform(-x_scale, x_scale, size=(n, 3)) * params.dx
    v = rng.normal(0.0, v_scale, size=(n, 3))
    C = rng.normal(0.0, c_scale, size=(n, 3, 3))
    G = rng.normal(0.0, g_scale, size=(n, 3, 3))
    return (representable_positions(params, x), v.astype(np.float32),
            C.astype(np.float32), G.astype(np.float32))


def _schedule(pose0, n_total, press, slip, slip_dir, rot_deg, frame=50, press_frac=0.25):
    """Press `press` straight down over the first press_frac of the substeps,
    then slip `slip` along direction slip_dir (radians in the x-y plane) while
    rotating rot_deg about the normal over the rest; segments end at frame
    boundaries and at the phase change.  Returns (n, target_pos, target_quat)."""
    x0, y0, z0 = pose0[:3]
    n_press = int(round(n_total * press_frac))
    cuts = sorted(set(list(range(frame, n_total + 1, frame)) + [n_press, n_total]))
    segs, done = [], 0
    for end in cuts:
        if end <= done:
            continue
        if end <= n_press:
            a = end / n_press
            pos, q = (x0, y0, z0 - press * a), (1.0, 0.0, 0.0, 0.0)
        else:
            b = (end - n_press) / (n_total - n_press)
            pos = (x0 + slip * b * math.cos(slip_dir), y0 + slip * b * math.sin(slip_dir), z0 - press)
            q = quat_about_z(rot_deg * b)
        segs.append((end - done, pos, q))
        done = end
    return segs


def config3(n_sensors: int = 64, seed: int = 3, k_range=(4, 12), dx: float = 0.5e-3,
            n_substeps: int = 500, subcycle: int = 2):
    """Batch of independent sensors: cells (8k, 8k, 2k) with k ~ U{k_range}, 8
    particles per cell; indenter ~ U{sphere r 2-6 mm, capsule r 2-4 mm with
    half-length 1-4 mm, rounded box half-sides 1.5-4 mm, Perlin height field
    with amplitude 0.2-0.5 mm, wavelength 1.5-4 mm, footprint radius 3-6 mm and
    a bowl that rises 2.5-3.5 mm at the footprint's edge}; press depth
    U[0.3, 1.5] mm over the first quarter of the substeps, then slip U[0, 3] mm in
    a direction U[0, 2 pi) and rotation U[-45, 45] degrees.  Returns the list of
    SensorParams and the list of schedules."""
    rng = np.random.default_rng(seed)
    params, scheds = [], []
    for i in range(n_sensors):
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        p, sch = _random_trajectory(rng, (8 * k, 8 * k, 2 * k), dx, subcycle, n_substeps, 1000 + i)
        params.append(p)
        scheds.append(sch)
    return params, scheds


def _random_trajectory(rng, cells, dx, subcycle, n_substeps, seed):
    """One sensor with a random indenter (the distribution of config3) whose
    lowest point starts on the slab's top over its centre, and its schedule."""
    L, H = cells[0] * dx, cells[2] * dx
    pad = padding_for(dx)
    kind = int(rng.integers(0, 4))
    if kind == 0:
        r = float(rng.uniform(2e-3, 6e-3))
        shape = dict(shape=SHAPE_SPHERE, radius=r)
        drop = r
    elif kind == 1:
        r = float(rng.uniform(2e-3, 4e-3))
        shape = dict(shape=SHAPE_CAPSULE, radius=r, half_length=float(rng.uniform(1e-3, 4e-3)))
        drop = r
    elif kind == 2:
        hx, hy = float(rng.uniform(1.5e-3, 4e-3)), float(rng.uniform(1.5e-3, 4e-3))
        shape = dict(shape=SHAPE_BOX, half_extent=(hx, hy, 2e-3), fillet=0.5e-3)
        drop = 2e-3
    else:
        # the bowl rises rim = 2.5-3.5 mm at the footprint's edge, so the
        # solid's vertical side wall stays above the slab at every press depth
        foot = float(rng.uniform(3e-3, 6e-3))
        amp, lam = float(rng.uniform(0.2e-3, 0.5e-3)), float(rng.uniform(1.5e-3, 4e-3))
        rim = float(rng.uniform(2.5e-3, 3.5e-3))
        tab = heightfield_table(int(rng.integers(0, 2**31)), foot, amp, lam, foot * foot / (2.0 * rim))
        shape = dict(shape=SHAPE_HEIGHTFIELD, hf=tab, hf_half=foot)
        drop = 0.0
    p = SensorParams(cells=tuple(cells), dx=dx, pad_lateral=pad, pad_top=pad, seed=seed,
                     subcycle=subcycle, pose0=(L / 2, L / 2, H + drop, 1.0, 0.0, 0.0, 0.0), **shape)
    press = float(rng.uniform(0.3e-3, 1.5e-3))
    slip = float(rng.uniform(0.0, 3e-3))
    ang = float(rng.uniform(0.0, 2 * math.pi))
    rot = float(rng.uniform(-45.0, 45.0))
    return p, _schedule(p.pose0, n_substeps, press, slip, ang, rot)


def surrogate_trajectories(n: int, seed: int, cells=(64, 64, 16), dx: float = 0.5e-3, n_substeps: int = 1000,
                           subcycle: int = 2):
    """Training or test trajectories for the surrogate: sensors with the
    32 x 32 x 8 mm footprint of config2 (at dx 0.5 mm by default) and config3's
    random indenters and press / slip / rotate schedules; frames every 50
    substeps.  Returns (params, schedules)."""
    rng = np.random.default_rng(seed)
    out = [_random_trajectory(rng, cells, dx, subcycle, n_substeps, 100000 * seed + i) for i in range(n)]
    return [o[0] for o in out], [o[1] for o in out]


def pose_change(pose_a, pose_b):
    """Surrogate pose input from pose a (pos m, quat wxyz) to pose b:
    translation in mm and the rotation vector (rad) of q_b q_a^-1."""
    pa, qa = np.asarray(pose_a[0], np.float64), np.asarray(pose_a[1], np.float64)
    pb, qb = np.asarray(pose_b[0], np.float64), np.asarray(pose_b[1], np.float64)
    w1, x1, y1, z1 = qb
    w2, x2, y2, z2 = qa[0], -qa[1], -qa[2], -qa[3]
    r = np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                  w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
    if r[0] < 0:
        r = -r
    s = np.linalg.norm(r[1:])
    rv = np.zeros(3) if s == 0 else r[1:] / s * 2.0 * math.atan2(s, r[0])
    return np.concatenate([(pb - pa) * 1000.0, rv]).astype(np.float32)


# ---------------------------------------------------------------- surrogate inputs

def surrogate_layer_shapes(channels=(32, 64, 128, 256), in_ch=10):
    """(cin, cout) of the 14 convolutions of the surrogate in parameter order."""
    c0, c1, c2, c3 = channels
    return [(in_ch, c0), (c0, c0), (c0, c1), (c1, c1), (c1, c2), (c2, c2), (c2, c3), (c3, c3),
            (c3, c2), (c2, c2), (c2, c1), (c1, c1), (c1, c0), (c0, c0)]


def surrogate_weights(channels=(32, 64, 128, 256), seed=0, head_scale=0.05, bias_scale=0.05):
    """Seeded flat parameter vector in the surrogate's layout: He-normal
    convolution weights W[Cout][3][3][Cin], small random biases, a small head."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in surrogate_layer_shapes(channels):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), co * 9 * ci))
        parts.append(rng.normal(0.0, bias_scale, co))
    parts.append(rng.normal(0.0, head_scale, 3 * channels[0]))
    parts.append(rng.normal(0.0, bias_scale, 3))
    return np.concatenate(parts).astype(np.float32)


def surrogate_batch(n, H, W, seed=0):
    """Seeded synthetic surrogate inputs (float32): depth (mm) ~ U[-4, 4], pose
    change ~ N(0, 0.2), previous displacement ~ N(0, 0.3) mm and a target that
    differs from it by ~ N(0, 0.05) mm."""
    rng = np.random.default_rng(seed)
    depth = rng.uniform(-4.0, 4.0, (n, H, W)).astype(np.float32)
    pose = rng.normal(0.0, 0.2, (n, 6)).astype(np.float32)
    prev = rng.normal(0.0, 0.3, (n, H, W, 3)).astype(np.float32)
    tgt = (prev + rng.normal(0.0, 0.05, (n, H, W, 3))).astype(np.float32)
    return depth, pose, prev, tgt


# ---------------------------------------------------------------- rendering inputs

# The four LEDs of the Gelsight-style scene (Sec. IV-B: coloured LEDs whose RGB
# values were fitted to real images; the commented LED table gives green
# (200, 255, 200), blue (25, 75, 255) and red (255, 50, 75) at energy 2e3 and
# white (255, 255, 255) at 1e3).  One LED per side of the footprint.
GELSIGHT_LEDS = (((200, 255, 200), 2.0e3), ((25, 75, 255), 2.0e3), ((255, 50, 75), 2.0e3),
                 ((255, 255, 255), 1.0e3))


def sensor_lights(Lx: float, Ly: float, top: float, colours=GELSIGHT_LEDS, below: float = 3.0e-3,
                  out: float = 1.0e-3, tilt_deg: float = 30.0, strip: float = 1.0e-3,
                  radiance: float = 16.0):
    """Rectangular LED strips along the four sides of an Lx x Ly footprint
    (order -x, +x, -y, +y), each `out` outside its edge and `below` under the
    undeformed surface at height `top`, 0.8 of the side long and `strip` wide,
    emitting toward the footprint's centre line tilted `tilt_deg` up toward the
    surface.  Radiance: RGB / 255 x energy / 1e3 x `radiance`.  Returns dicts
    with keys c, e1, e2, L (the renderer's light records)."""
    s, c = math.sin(math.radians(tilt_deg)), math.cos(math.radians(tilt_deg))
    sides = [((-out, Ly / 2), (1.0, 0.0), Ly), ((Lx + out, Ly / 2), (-1.0, 0.0), Ly),
             ((Lx / 2, -out), (0.0, 1.0), Lx), ((Lx / 2, Ly + out), (0.0, -1.0), Lx)]
    lights = []
    for ((x, y), (ux, uy), side), (rgb, energy) in zip(sides, colours):
        n = np.array([ux * c, uy * c, s])               # emitting normal
        t = np.array([-uy, ux, 0.0])                    # along the side
        e1 = 0.8 * side * t
        e2 = strip * np.cross(n, t)                     # e1 x e2 = |e1| |e2| n
        L = tuple(float(v) / 255.0 * energy / 1e3 * radiance for v in rgb)
        lights.append(dict(c=(x, y, top - below), e1=tuple(e1), e2=tuple(e2), L=L))
    return lights


def sensor_texture(h: int, w: int, seed: int = 0, markers: int = 12):
    """Synthetic base image of the coated elastomer (the real no-contact images
    are absent): a light grey coat with seeded low-frequency mottling and a
    markers x markers grid of dark dots; h x w x 3 albedos in (0, 1)."""
    yy, xx = np.meshgrid(np.arange(h) + 0.5, np.arange(w) + 0.5, indexing="ij")
    base = 0.72 + 0.06 * perlin2(xx / w * 6.0, yy / h * 6.0, seed) + 0.03 * perlin2(xx / w * 23.0, yy / h * 23.0,
                                                                                      seed + 1)
    pitch_x, pitch_y = w / markers, h / markers
    dx = (xx % pitch_x) - pitch_x / 2
    dy = (yy % pitch_y) - pitch_y / 2
    dot = np.hypot(dx / pitch_x, dy / pitch_y) < 0.12
    img = np.repeat(base[:, :, None], 3, axis=2) * np.array([1.0, 0.98, 0.95])
    img[dot] *= 0.25
    return np.clip(img, 0.02, 0.98)


def dented_heightmap(h: int, w: int, Lx: float, Ly: float, top: float, depth: float = 1.0e-3,
                     radius: float = 3.0e-3, centre=None, seed: int = 0, roughness: float = 2.0e-6):
    """A height map of a slab pressed by a sphere: top minus the spherical cap
    of the given depth and contact radius, plus seeded roughness; row v, column
    u at the pixel centres ((u+1/2) Lx/w, (v+1/2) Ly/h)."""
    cx, cy = centre if centre is not None else (Lx / 2, Ly / 2)
    x = (np.arange(w) + 0.5) * Lx / w
    y = (np.arange(h) + 0.5) * Ly / h
    X, Y = np.meshgrid(x, y, indexing="xy")
    R = (radius * radius + depth * depth) / (2.0 * depth)     # sphere radius of that cap
    r2 = (X - cx) ** 2 + (Y - cy) ** 2
    cap = np.where(r2 < radius * radius, np.sqrt(np.maximum(R * R - r2, 0.0)) - (R - depth), 0.0)
    rng = np.random.default_rng(seed)
    return top - cap + roughness * rng.standard_normal((h, w))

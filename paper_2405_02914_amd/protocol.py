"""The slip and rotation protocol of the paper's experiments (Sec. IV-A and
V-B), run on synthetic inputs through the C ABI: the holed-disc indenter is
pressed 0.5 mm into the full-resolution slab, then slid in 1 mm increments up
to 5 mm, or rotated in 5 degree increments up to 45 degrees, once with the
improved method (IMPM, Algorithm 1) and once with the plain single-exchange
MPM the paper compares it against ("normal").  A height map is taken after the
press and after every increment.

The paper's comparison is against photographs, which are absent; what can be
reproduced is its description of the two simulations (Sec. V-B): under slip
the plain method's surface loses the indenter's central hole, and under
rotation the plain method, lacking the fixed bottom layer, lets the unpressed
hole region sink deeper.  `hole_metrics` measures both from a height map.
"""
from __future__ import annotations

import time

import numpy as np

from . import impm, workloads as W


def run(params, segs, hm: int = 256):
    """Step a sensor through `segs`, taking a hm x hm height map (mm of depth
    below the undeformed top, positive into the slab) after every segment.
    and its surface displacement map (mm, hm x hm x 3).  A segment whose state
    the library rejects (SIM_ENUMERIC: the sticking contact has sheared the
    slab past what the elastomer model can carry) ends the run.  Returns
    (depth maps [k, hm, hm] and displacement maps [k, hm, hm, 3] of the
    completed segments, their poses [(pos, quat)], stats, seconds, the failed
    segment's index or None)."""
    import torch
    s = impm.Sim(params)
    try:
        maps, disps, poses, failed = [], [], [], None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = torch.empty(hm * hm, device="cuda", dtype=torch.float32)
        out3 = torch.empty(hm * hm * 3, device="cuda", dtype=torch.float32)
        for k, (n, pos, q) in enumerate(segs):
            s.sim_set_indenter_pose(pos, q)
            s.sim_step(n)
            s.sim_surface_heightmap(hm, hm, out=out)
            s.sim_surface_displacement(hm, hm, out=out3)
            try:
                s.sim_synchronize()
            except impm.SimError as e:
                if e.code != impm.SIM_ENUMERIC:
                    raise
                failed = k
                break
            maps.append(out.clone())
            disps.append(out3.clone())
            poses.append((pos, q))
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        depth = [(params.height - m.cpu().numpy().reshape(hm, hm)) * 1e3 for m in maps]
        disp = [d.cpu().numpy().reshape(hm, hm, 3) * 1e3 for d in disps]
        return (np.stack(depth) if depth else np.zeros((0, hm, hm)),
                np.stack(disp) if disp else np.zeros((0, hm, hm, 3)), poses, s.sim_get_stats(check=False), secs,
                failed)
    finally:
        s.close()


def _pixel_centres(params, hm):
    Lx, Ly = params.lengths[0], params.lengths[1]
    u = (np.arange(hm) + 0.5) * Lx / hm
    v = (np.arange(hm) + 0.5) * Ly / hm
    return np.meshgrid(u, v, indexing="xy")


def hole_metrics(params, depth_mm, pos, r_out, r_hole, fillet=0.75e-3, hole_fillet=0.3e-3,
                 start=None, margin=0.25e-3):
    """From one depth map (mm, rows = y): the mean depth under the indenter's
    flat annular face and inside its hole (both at the indenter's current
    centre `pos`), their difference (how visible the hole is), and, when the
    slide's start position is given, the mean depth of the trace the indenter
    left behind (the swept band outside the current footprint)."""
    hm = depth_mm.shape[0]
    X, Y = _pixel_centres(params, hm)
    r = np.hypot(X - pos[0], Y - pos[1])
    face = (r >= r_hole + hole_fillet + margin) & (r <= r_out - fillet - margin)
    hole = r <= r_hole - margin
    out = {"face_mm": float(depth_mm[face].mean()), "hole_mm": float(depth_mm[hole].mean())}
    out["hole_contrast_mm"] = out["face_mm"] - out["hole_mm"]
    if start is not None and abs(pos[0] - start[0]) > r_out:
        lo, hi = sorted((start[0], pos[0]))
        band = (np.abs(Y - start[1]) <= r_out - fillet) & (X >= lo) & (X <= hi) & (r > r_out + 2 * margin)
        out["trace_mm"] = float(depth_mm[band].mean()) if band.any() else 0.0
    return out


def follow_metric(params, disp_mm, pos, quat, start, r_out, r_hole, fillet=0.75e-3, hole_fillet=0.3e-3,
                  margin=0.25e-3):
    """How far the surface under the indenter's flat face has followed the
    indenter (relative rest: 1 = moved with it, 0 = stayed behind), from one
    displacement map (mm; the surface particles' displacement from their rest
    positions, at their current positions).  Slide: the face's mean x
    displacement over the indenter's x travel.  Rotation: the face's mean angle
    about the indenter's centre (rest position to current position) over the
    indenter's angle about z.  None before the indenter has moved sideways."""
    hm = disp_mm.shape[0]
    X, Y = _pixel_centres(params, hm)
    r = np.hypot(X - pos[0], Y - pos[1])
    face = (r >= r_hole + hole_fillet + margin) & (r <= r_out - fillet - margin)
    u = disp_mm[face] * 1e-3
    slide = pos[0] - start[0]
    angle = 2.0 * np.arctan2(quat[3], quat[0])
    if abs(slide) > 1e-9:
        return float(u[:, 0].mean() / slide)
    if abs(angle) > 1e-9:
        x1, y1 = X[face] - pos[0], Y[face] - pos[1]
        x0, y0 = x1 - u[:, 0], y1 - u[:, 1]
        th = np.arctan2(x0 * y1 - y0 * x1, x0 * x1 + y0 * y1)
        return float(th.mean() / angle)
    return None


def protocol(kind: str, sign: float = -1.0, dx: float = 0.25e-3, cells=(128, 128, 32), hm: int = 256,
             r_out: float = 4.0e-3, r_hole: float = 1.5e-3, object_density: float = None, **sched_kw):
    """Both methods through one protocol ("slip" or "rotate"; sign -1: leftward
    or clockwise), the object a grid collider, or object particles of the given
    density (kg/m^3) when object_density is set.  Returns a dict with the
    per-increment metrics of each method, its stats and its particle-updates
    per second."""
    res = {}
    extra = {} if object_density is None else dict(object_mode=W.OBJECT_PARTICLES, object_density=object_density)
    for name, mode in (("impm", W.MODE_IMPM), ("normal", W.MODE_PLAIN)):
        p = W.protocol_sensor(dx=dx, cells=cells, r_out=r_out, r_hole=r_hole, mode=mode, **extra)
        segs = W.protocol_schedule(p.pose0, kind, sign=sign, **sched_kw)
        maps, disps, poses, st, secs, failed = run(p, segs, hm)
        rows = [hole_metrics(p, d, pz[0], r_out, r_hole, start=p.pose0[:3]) for d, pz in zip(maps, poses)]
        for row, u, pz in zip(rows, disps, poses):
            row["follow"] = follow_metric(p, u, pz[0], pz[1], p.pose0[:3], r_out, r_hole)
        res[name] = {"metrics": rows, "passes_per_step": st["passes"] / max(st["steps"], 1),
                     "limit_hits": st["limit_hits"], "steps": st["steps"], "failed_segment": failed,
                     "particle_updates_per_s": p.n_particles * st["steps"] / secs, "seconds": secs}
    return res

"""Serving many sensors with the surrogate and IMPM fallback.

Every frame (50 substeps of the indenter schedule) each sensor's surface
displacement comes from the surrogate, except on re-solve frames, where the
IMPM simulator advances the sensor's stored state from its last IMPM pose to
the frame's pose within one frame's substeps and its result replaces the
prediction (and re-anchors the surrogate's recurrent input).  A re-solve is
due on every `resolve_every`-th frame and on any frame whose predicted contact
area (pixels with depth + u_z >= -0.02 mm) deviates by more than `area_tol`
from the area of the last IMPM frame (relative to at least `area_floor`
pixels, so that a touch from zero contact counts as a large change).

Sensors are grouped by resolution class (one impm.Batch each, since a batch
shares its sub-cycle count).  A scheduled re-solve runs for the whole group; a
contact-area re-solve runs only for the sensors that triggered it (the other
members sit the batch call out, sim_batch_set_active), except for a group's
first re-solve, which steps every member.  All simulation, network, depth-map
and contact-area work runs in the library's kernels; torch holds the buffers.
"""
from __future__ import annotations

import time

import numpy as np

from . import impm, workloads as W

RES = 128


class Server:
    def __init__(self, params, scheds, net, stream, resolve_every=20, area_tol=0.10, area_floor=16.0,
                 contact_tol_mm=0.02, record=False, log=None):
        import torch
        self.params, self.scheds, self.net, self.st = params, scheds, net, stream
        self.log = log or (lambda *a, **k: None)
        self.N = len(params)
        self.F = len(scheds[0])
        self.resolve_every, self.area_tol, self.area_floor = resolve_every, area_tol, area_floor
        self.tol = contact_tol_mm
        order = sorted(range(self.N), key=lambda i: (params[i].subcycle, params[i].cells))
        if order != list(range(self.N)):
            raise ValueError("sensors must be listed grouped by resolution class")
        self.groups = []                       # (start, end, Batch)
        dev = torch.device("cuda")
        i = 0
        with torch.cuda.stream(stream):
            while i < self.N:
                j = i
                while j < self.N and (params[j].subcycle, params[j].cells) == (params[i].subcycle, params[i].cells):
                    j += 1
                t0 = time.perf_counter()
                tile, _ = impm.sim_autotune_tile(params[i], steps=8, stream=stream.cuda_stream)
                self.groups.append([i, j, impm.Batch(params[i:j], tiles=[tile] * (j - i), stream=stream.cuda_stream)])
                self.log(f"[serve] group of {j - i} sensors of {params[i].cells} cells ready in "
                         f"{time.perf_counter() - t0:.1f} s", flush=True)
                i = j
            self.disp = torch.zeros((self.N, RES, RES, 3), device=dev)
            self.depth = torch.zeros((self.N, RES, RES), device=dev)
            self.pose6 = torch.zeros((self.N, 6), device=dev)
            self.area = torch.zeros(self.N, device=dev)
            self.area_ref = torch.zeros(self.N, device=dev)
            self.tmp3 = torch.empty((self.N, RES, RES, 3), device=dev)
        self.poses = [(p.pose0[:3], p.pose0[3:]) for p in params]
        self.k = 0
        self.record = torch.zeros((self.N, self.F + 1, RES, RES, 3), device=dev) if record else None
        self.latency_ms, self.kind = [], []
        self.resolves = {"scheduled": 0, "contact_area": 0}
        self.stepped = [False] * len(self.groups)
        self.last_solved = np.zeros(self.N, np.int64)   # frame of each sensor's last IMPM state
        self.max_gap = np.zeros(self.N, np.int64)       # longest jump a re-solve has taken, in frames
        self.full_s = [0.0] * len(self.groups)     # wall time of whole-group re-solves (plain batched frames)
        self.full_n = [0] * len(self.groups)

    def _resolve(self, gi, n_substeps, members=None):
        """Advance group gi's IMPM state to the frame's poses (every member, or
        the members flagged in `members`); returns how many were re-solved."""
        import torch
        a, b, batch = self.groups[gi]
        if members is None or not self.stepped[gi]:
            members = np.ones(b - a, bool)
        batch.sim_batch_set_active(members)
        sel = a + np.nonzero(members)[0]
        self.max_gap[sel] = np.maximum(self.max_gap[sel], self.k + 1 - self.last_solved[sel])
        self.last_solved[sel] = self.k + 1
        full = bool(members.all())
        if full:
            self.st.synchronize()
            t0 = time.perf_counter()
        batch.sim_batch_step(n_substeps)
        if full:
            self.st.synchronize()
            self.full_s[gi] += time.perf_counter() - t0
            self.full_n[gi] += 1
        self.stepped[gi] = True
        batch.sim_batch_displacements(RES, RES, out=self.tmp3[a:b])
        area = self.net.sur_contact_area(self.depth[a:b], self.tmp3[a:b] * 1000.0, self.tol)
        if members.all():
            self.disp[a:b] = self.tmp3[a:b] * 1000.0
            self.area_ref[a:b] = area
        else:
            idx = torch.from_numpy(np.nonzero(members)[0]).to(self.disp.device)
            self.disp[a + idx] = self.tmp3[a + idx] * 1000.0
            self.area_ref[a + idx] = area[idx]
        return int(members.sum())

    def step(self):
        """Serve the next frame of every sensor; returns its latency (ms)."""
        import torch
        k = self.k
        t0 = time.perf_counter()
        with torch.cuda.stream(self.st):
            new = [(s[k][1], s[k][2]) for s in self.scheds]
            pose6 = np.stack([W.pose_change(p, q) for p, q in zip(self.poses, new)])
            self.pose6.copy_(torch.from_numpy(pose6))
            for a, b, batch in self.groups:
                batch.sim_batch_set_indenter_poses([q[0] for q in new[a:b]], [q[1] for q in new[a:b]])
                batch.sim_batch_depthmaps(RES, RES, 1000.0, out=self.depth[a:b])
            scheduled = (k + 1) % self.resolve_every == 0
            if not scheduled:
                self.net.sur_infer(self.depth, self.pose6, self.disp, out=self.tmp3)
                self.net.sur_contact_area(self.depth, self.tmp3, self.tol, out=self.area)
                dev = (self.area - self.area_ref).abs() > self.area_tol * torch.clamp(self.area_ref, min=self.area_floor)
                dev = dev.cpu().numpy()
                self.disp.copy_(self.tmp3)
            n_sub = self.scheds[0][k][0]
            kinds = []
            for gi, (a, b, _) in enumerate(self.groups):
                if scheduled:
                    self.resolves["scheduled"] += self._resolve(gi, n_sub)
                    kinds.append("impm")
                elif dev[a:b].any():
                    self.resolves["contact_area"] += self._resolve(gi, n_sub, dev[a:b])
                    kinds.append("impm")
                else:
                    kinds.append("surrogate")
            if self.record is not None:
                self.record[:, k + 1] = self.disp
        self.st.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        self.poses = new
        self.k += 1
        self.latency_ms.append(ms)
        self.kind.append(kinds)
        self.log(f"[serve] frame {k + 1}: {ms:.1f} ms, {kinds}", flush=True)
        return ms

    def run(self, frames=None):
        import torch
        # frame 0: every group's IMPM state at pose0 anchors the surrogate (zero displacement)
        with torch.cuda.stream(self.st):
            for a, b, batch in self.groups:
                batch.sim_batch_depthmaps(RES, RES, 1000.0, out=self.depth[a:b])
            self.net.sur_contact_area(self.depth, self.disp, self.tol, out=self.area_ref)
        self.st.synchronize()
        t0 = time.perf_counter()
        for _ in range(frames or self.F):
            self.step()
        wall = time.perf_counter() - t0
        # a sensor whose IMPM state latched a numerical error (the library's range
        # and finiteness guards) is reported, not served on silently
        failed = []
        for a, b, batch in self.groups:
            try:
                batch.sim_batch_synchronize()
            except impm.SimError:
                pass
            for q, sen in enumerate(batch.sensors):
                try:
                    sen.sim_get_stats()
                except impm.SimError:
                    failed.append(a + q)
        lat = np.array(self.latency_ms)
        out = {"sensors": self.N, "frames": len(lat), "wall_s": wall, "frames_per_s": self.N * len(lat) / wall,
               "latency_p50_ms": float(np.percentile(lat, 50)), "latency_p99_ms": float(np.percentile(lat, 99)),
               "resolved_sensor_frames": dict(self.resolves), "failed_sensors": failed,
               "failed_sensor_details": [{"sensor": i, "cells": self.params[i].cells, "shape": self.params[i].shape,
                                          "longest_jump_frames": int(self.max_gap[i])} for i in failed],
               "longest_jump_frames": int(self.max_gap.max()),
               "groups": [(b - a, self.params[a].cells) for a, b, _ in self.groups]}
        if all(self.full_n):
            # a whole-group re-solve is one plain batched IMPM frame of the group
            frame = [t / n for t, n in zip(self.full_s, self.full_n)]
            out["impm_group_frame_ms"] = [1e3 * f for f in frame]
            out["plain_impm_frames_per_s_est"] = self.N / sum(frame)
        return out

    def close(self):
        for g in self.groups:
            g[2].close()
        self.groups = []


def sensor_mix(n_per_class, frames, seed=5):
    """Config 5's sensors: the 32 x 32 x 8 mm footprint at 64 x 64 x 16,
    96 x 96 x 24 and 128 x 128 x 32 cells (dx 0.5, 1/3 and 0.25 mm; 2, 3 and 4
    executed steps per substep), random indenters and press / slip / rotate
    schedules of `frames` frames.  n_per_class: one count for every class, or
    three counts."""
    counts = [n_per_class] * 3 if np.isscalar(n_per_class) else list(n_per_class)
    params, scheds = [], []
    for c, (cells, sub) in enumerate((((64, 64, 16), 2), ((96, 96, 24), 3), ((128, 128, 32), 4))):
        p, s = W.surrogate_trajectories(counts[c], seed=seed * 10 + c, cells=cells, dx=32e-3 / cells[0],
                                        n_substeps=50 * frames, subcycle=sub)
        params += p
        scheds += s
    return params, scheds

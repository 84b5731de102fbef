"""Surrogate training on IMPM trajectories, evaluation and serving rates.

  python -m paper_2405_02914_amd.surrogate_train --train 512 --test 64 --steps 3000 \\
      --out surrogate.json [--save weights.bin]

1. Data.  Seeded random trajectories (workloads.surrogate_trajectories:
   32 x 32 x 8 mm sensors, random sphere / capsule / box / height-field
   indenters pressed, slipped and rotated) run through the batched IMPM
   simulator (libimpm.so); at every frame (50 substeps) the 128 x 128 indenter
   depth map (mm) and surface displacement (mm) are recorded on the device.
2. Training.  Adam on random minibatches of (frame k-1 -> frame k)
   transitions: input depth_k, pose change k-1 -> k, IMPM displacement k-1;
   target IMPM displacement k.
3. Evaluation on held-out trajectories: RMS error (mm, over pixels, components
   and frames) of the surrogate with the IMPM previous frame (one step), of the
   surrogate fed its own predictions from the rest state (roll-out), and of
   the persistence predictor next = prev (the method without the network).
4. Rates: surrogate inference frames/s at a serving batch, against the IMPM
   frames/s of the data generation (same sensors, batched).

Torch is used for device buffers, streams and minibatch gathering; every
simulation and network step runs in the library's kernels.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import impm, sur, workloads as W

RES = 128


class Dataset:
    """Device tensors of recorded frames: depth (T, F+1, R, R) mm, disp
    (T, F+1, R, R, 3) mm, pose change into each frame (T, F+1, 6)."""

    def __init__(self, depth, disp, pose6, impm_frames_per_s, particles):
        self.depth, self.disp, self.pose6 = depth, disp, pose6
        self.T, self.F = depth.shape[0], depth.shape[1] - 1
        self.impm_frames_per_s = impm_frames_per_s
        self.particles = particles

    def transitions(self, t, k):
        """Inputs and targets of transitions (t[i], k[i]), k >= 1."""
        return (self.depth[t, k].contiguous(), self.pose6[t, k].contiguous(),
                self.disp[t, k - 1].contiguous(), self.disp[t, k].contiguous())


def generate(params, scheds, stream, batch=64, log=print):
    """Run the trajectories through batched IMPM and record every frame."""
    import torch
    T = len(params)
    F = len(scheds[0])
    dev = torch.device("cuda")
    depth = torch.zeros((T, F + 1, RES, RES), device=dev)
    disp = torch.zeros((T, F + 1, RES, RES, 3), device=dev)
    pose6 = torch.zeros((T, F + 1, 6), device=dev)
    for t in range(T):
        poses = [(params[t].pose0[:3], params[t].pose0[3:])] + [(s[1], s[2]) for s in scheds[t]]
        for k in range(1, F + 1):
            pose6[t, k] = torch.from_numpy(W.pose_change(poses[k - 1], poses[k]))
    tile, _ = impm.sim_autotune_tile(params[0], steps=8, stream=stream.cuda_stream)
    step_time, frames = 0.0, 0
    bad = []
    with torch.cuda.stream(stream):
        for i in range(0, T, batch):
            j = min(T, i + batch)
            b = impm.Batch(params[i:j], tiles=[tile] * (j - i), stream=stream.cuda_stream)
            tmp = torch.empty((j - i, RES, RES), device=dev)
            tmp3 = torch.empty((j - i, RES, RES, 3), device=dev)
            b.sim_batch_depthmaps(RES, RES, 1000.0, out=tmp)
            depth[i:j, 0] = tmp
            for k in range(F):
                b.sim_batch_set_indenter_poses([s[k][1] for s in scheds[i:j]], [s[k][2] for s in scheds[i:j]])
                stream.synchronize()
                t0 = time.perf_counter()
                b.sim_batch_step(scheds[i][k][0])
                stream.synchronize()
                step_time += time.perf_counter() - t0
                frames += j - i
                b.sim_batch_depthmaps(RES, RES, 1000.0, out=tmp)
                b.sim_batch_displacements(RES, RES, out=tmp3)
                depth[i:j, k + 1] = tmp
                disp[i:j, k + 1] = tmp3 * 1000.0
            try:
                b.sim_batch_synchronize()
            except impm.SimError:
                pass
            for q, s in enumerate(b.sensors):        # a latched numerical error drops the trajectory
                try:
                    s.sim_get_stats()
                except impm.SimError:
                    bad.append(i + q)
            b.close()
            log(f"[data] trajectories {j}/{T}, IMPM {frames / step_time:.1f} frames/s, dropped {len(bad)}",
                flush=True)
    stream.synchronize()
    keep = torch.tensor([t for t in range(T) if t not in set(bad)], device=dev, dtype=torch.long)
    d = Dataset(depth[keep], disp[keep], pose6[keep], frames / step_time, params[0].n_particles)
    d.dropped = bad
    return d


def train(net, data, steps, batch, stream, lr=1e-3, seed=0, log=print, log_every=250, rollout=0,
          rollout_from=0.25):
    """Adam on random transitions; cosine learning-rate decay to lr / 20.

    rollout = R > 0 (pushforward training): after the first `rollout_from` of
    the steps, the previous displacement of each minibatch is the network's own
    prediction r frames on from the IMPM frame k - 1 - r, with r drawn from
    0..R per step (no gradient through those predictions), so that training
    sees the inputs a served roll-out feeds the network."""
    import torch
    dev = data.depth.device
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    gc = torch.Generator()
    gc.manual_seed(seed + 1)
    losses = []
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for it in range(steps):
            net.sur_set_lr(lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * it / max(1, steps)))))
            t = torch.randint(0, data.T, (batch,), device=dev, generator=g)
            k = torch.randint(1, data.F + 1, (batch,), device=dev, generator=g)
            r = 0
            if rollout and it >= rollout_from * steps:
                r = min(int(torch.randint(0, rollout + 1, (1,), generator=gc)), data.F - 1)
                k = torch.clamp(k, min=r + 1)
            prev = data.disp[t, k - 1 - r].contiguous()
            for j in range(r):
                kk = k - r + j
                prev = net.sur_infer(data.depth[t, kk].contiguous(), data.pose6[t, kk].contiguous(), prev)
            want = (it % log_every == 0) or it == steps - 1
            loss = net.sur_train_step(data.depth[t, k].contiguous(), data.pose6[t, k].contiguous(), prev,
                                      data.disp[t, k].contiguous(), want_loss=want)
            if want:
                losses.append((it, loss))
                log(f"[train] step {it} loss {loss:.4e} ({time.perf_counter() - t0:.1f} s)", flush=True)
    if stream is not None:
        stream.synchronize()
    return losses, time.perf_counter() - t0


def evaluate(net, data, stream, batch=64):
    """RMS errors (mm) on every transition of every trajectory in data."""
    import torch
    se_one = se_roll = se_keep = 0.0
    count = 0
    with torch.cuda.stream(stream):
        for i in range(0, data.T, batch):
            j = min(data.T, i + batch)
            idx = torch.arange(i, j, device="cuda")
            roll = data.disp[i:j, 0].contiguous()
            for k in range(1, data.F + 1):
                kk = torch.full_like(idx, k)
                d, p, prev, tgt = data.transitions(idx, kk)
                one = net.sur_infer(d, p, prev)
                roll = net.sur_infer(d, p, roll)
                se_one += float(((one - tgt) ** 2).sum())
                se_roll += float(((roll - tgt) ** 2).sum())
                se_keep += float(((prev - tgt) ** 2).sum())
                count += tgt.numel()
    stream.synchronize()
    return {"rms_one_step_mm": math.sqrt(se_one / count), "rms_rollout_mm": math.sqrt(se_roll / count),
            "rms_persistence_mm": math.sqrt(se_keep / count), "values": count}


def inference_rate(net, data, stream, batch, reps=20):
    """Surrogate frames/s at a serving batch (inputs resident on the device)."""
    import torch
    with torch.cuda.stream(stream):
        t = torch.arange(batch, device="cuda") % data.T
        k = 1 + torch.arange(batch, device="cuda") % data.F
        d, p, prev, _ = data.transitions(t, k)
        out = torch.empty_like(prev)
        net.sur_infer(d, p, prev, out=out)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            net.sur_infer(d, p, prev, out=out)
        stream.synchronize()
        dt = time.perf_counter() - t0
    return batch * reps / dt, dt / reps


def kernel_timing(batch=64, serve_batch=256, reps=20, stream=None):
    """Training-step and inference times (ms) on seeded synthetic inputs of the
    serving shape, without data generation: the short run that kernel
    profiles of the network time."""
    import torch
    st = stream or torch.cuda.Stream()
    d, p, pv, tg = W.surrogate_batch(batch, RES, RES, seed=0)
    d2, p2, pv2, _ = W.surrogate_batch(serve_batch, RES, RES, seed=1)
    with torch.cuda.stream(st):
        tr = [torch.from_numpy(a).cuda() for a in (d, p, pv, tg)]
        inf = [torch.from_numpy(a).cuda() for a in (d2, p2, pv2)]
        out = torch.empty_like(inf[2])
    net = sur.Surrogate(RES, RES, max_batch=max(batch, serve_batch), stream=st.cuda_stream)
    res = {}
    for name, fn in (("train_ms", lambda: net.sur_train_step(*tr)), ("infer_ms", lambda: net.sur_infer(*inf, out=out))):
        for _ in range(3):
            fn()
        st.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        st.synchronize()
        res[name] = 1e3 * (time.perf_counter() - t0) / reps
    net.close()
    res.update(batch=batch, serve_batch=serve_batch, reps=reps)
    return res


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=512)
    ap.add_argument("--test", type=int, default=64)
    ap.add_argument("--substeps", type=int, default=1000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--serve-batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--rollout", type=int, default=0,
                    help="pushforward training: feed up to this many of the network's own predictions")
    ap.add_argument("--out", default=None)
    ap.add_argument("--save", default=None)
    ap.add_argument("--timing-only", action="store_true",
                    help="time training steps and inference on synthetic inputs, no data generation")
    a = ap.parse_args()
    torch.cuda.set_device(0)
    if a.timing_only:
        print(json.dumps(kernel_timing(a.batch, a.serve_batch)), flush=True)
        return
    st = torch.cuda.Stream()
    ptr, str_ = W.surrogate_trajectories(a.train, seed=1, n_substeps=a.substeps)
    pte, ste = W.surrogate_trajectories(a.test, seed=2, n_substeps=a.substeps)
    t0 = time.perf_counter()
    dtr = generate(ptr, str_, st)
    dte = generate(pte, ste, st)
    gen_s = time.perf_counter() - t0
    net = sur.Surrogate(RES, RES, max_batch=max(a.batch, a.serve_batch), lr=a.lr, stream=st.cuda_stream)
    losses, train_s = train(net, dtr, a.steps, a.batch, st, lr=a.lr, rollout=a.rollout)
    ev = evaluate(net, dte, st)
    ev_train = evaluate(net, dtr, st)
    fps, lat = inference_rate(net, dte, st, a.serve_batch)
    res = {"train_trajectories": dtr.T, "test_trajectories": dte.T,
           "dropped_trajectories": len(dtr.dropped) + len(dte.dropped), "frames_per_trajectory": dtr.F,
           "sensor_particles": dtr.particles, "data_generation_s": gen_s, "train_steps": a.steps,
           "batch": a.batch, "rollout": a.rollout, "train_s": train_s, "train_ms_per_step": 1e3 * train_s / a.steps,
           "losses": losses, "test": ev, "train_set": ev_train,
           "surrogate_frames_per_s": fps, "surrogate_batch_latency_ms": 1e3 * lat, "serve_batch": a.serve_batch,
           "impm_frames_per_s": dtr.impm_frames_per_s, "speedup_vs_impm": fps / dtr.impm_frames_per_s}
    print(json.dumps(res), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    if a.save:
        net.sur_save(a.save)


if __name__ == "__main__":
    main()

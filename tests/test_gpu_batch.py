"""Batched sensors (many independent sensors advanced together) through the C
ABI: every member of a batch computes exactly what the same sensor computes
alone (the kernels are the same code and the node sums are exact fixed-point
sums), a member matches the FP64 oracle, and the tile autotuner returns a
compiled shape."""
import numpy as np
import pytest

from paper_2405_02914_amd import workloads as W

pytestmark = pytest.mark.gpu

TILES = [(8, 4, 4, 256), (4, 4, 4, 256), (8, 8, 2, 256), (8, 4, 4, 256), (4, 8, 4, 256)]


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2405_02914_amd import impm
    impm.lib()
    return impm


def small_batch(n=5, n_substeps=40):
    params, scheds = W.config3(n_sensors=n, seed=7, k_range=(2, 3), n_substeps=n_substeps)
    return params, scheds


def run_batch(b, scheds):
    for k in range(len(scheds[0])):
        pos = np.array([s[k][1] for s in scheds])
        quat = np.array([s[k][2] for s in scheds])
        b.sim_batch_set_indenter_poses(pos, quat)
        b.sim_batch_step(scheds[0][k][0])
    b.sim_batch_synchronize()


def test_batch_members_equal_standalone(gpu):
    params, scheds = small_batch()
    print("[batch] sizes", [p.cells for p in params], "shapes", [p.shape for p in params], flush=True)
    b = gpu.Batch(params, tiles=TILES[:len(params)])
    run_batch(b, scheds)
    hb = b.sim_batch_heightmaps(32, 32)
    for i, p in enumerate(params):
        s = gpu.Sim(p)
        s.sim_set_tile(*TILES[i])
        s.run_schedule(scheds[i])
        s.sim_synchronize()
        for u, w in zip(b.sensors[i].sim_read_particles(), s.sim_read_particles()):
            assert np.array_equal(u, w), f"sensor {i}"
        st_b, st_s = b.sensors[i].sim_get_stats(), s.sim_get_stats()
        assert st_b["passes"] == st_s["passes"] and st_b["steps"] == st_s["steps"]
        assert np.array_equal(hb[i], s.sim_surface_heightmap(32, 32))
        s.close()
    b.close()


def test_batch_member_matches_oracle(gpu, oracle_lib):
    params, scheds = small_batch(n=3, n_substeps=30)
    i = 1
    o = oracle_lib.OracleSim(params[i])
    o.enable_pass_log(100000)
    o.run_schedule(scheds[i])
    b = gpu.Batch(params)
    b.sensors[i].sim_debug_force_passes(o.pass_log())
    run_batch(b, scheds)
    xg = b.sensors[i].sim_read_particles()[0]
    xo = o.state()[0]
    err = np.abs(xg - xo).max() / params[i].dx
    print(f"[batch] member vs oracle: max|x| {err:.3e} dx", flush=True)
    assert err <= 1e-3
    b.close()


def _state_equal(a, b):
    return all(np.array_equal(u, w) for u, w in zip(a.sim_read_particles(), b.sim_read_particles()))


def test_graph_replay_equals_eager(gpu):
    """Graph replays (batch and single sensor) against the eager launches, checked
    after every call, with host reads and height maps between replays; the
    sequences repeat, so most calls replay an already captured graph."""
    params, scheds = small_batch(n=3, n_substeps=60)
    bg = gpu.Batch(params)                  # graph replay (the default)
    be = gpu.Batch(params)
    be.sim_batch_set_graph(False)
    sg, se = gpu.Sim(params[0]), gpu.Sim(params[0])
    sg.sim_set_graph(True)
    # the schedules cut at the press/slip change and every 50 substeps; advance
    # them in chunks of 5 substeps so the same graph is replayed many times
    for k in range(len(scheds[0])):
        n, _, _ = scheds[0][k]
        pos = np.array([s[k][1] for s in scheds])
        quat = np.array([s[k][2] for s in scheds])
        for b in (bg, be):
            b.sim_batch_set_indenter_poses(pos, quat)
        for s in (sg, se):
            s.sim_set_indenter_pose(pos[0], quat[0])
        done = 0
        while done < n:
            m = min(5, n - done)
            for b in (bg, be):
                b.sim_batch_step(m)
            for s in (sg, se):
                s.sim_step(m)
            done += m
            for i in range(len(params)):
                assert _state_equal(bg.sensors[i], be.sensors[i]), (k, done, i)
            assert _state_equal(sg, se), (k, done)
            assert np.array_equal(sg.sim_surface_heightmap(16, 16), se.sim_surface_heightmap(16, 16))
    assert sg.sim_get_stats()["passes"] == se.sim_get_stats()["passes"]
    for x in (bg, be, sg, se):
        x.close()


def test_batch_rejects_mismatched_steps(gpu):
    params, _ = small_batch(n=2)
    with pytest.raises(gpu.SimError):
        gpu.Batch([params[0], params[1].replace(subcycle=3)])


def test_autotune_returns_compiled_shape(gpu):
    params, _ = small_batch(n=1)
    tile, ms = gpu.sim_autotune_tile(params[0], steps=4)
    print("[autotune]", tile, ms, flush=True)
    assert ms > 0
    s = gpu.Sim(params[0])
    s.sim_set_tile(*tile)          # accepted: a compiled shape
    s.close()

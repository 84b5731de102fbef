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


def four_segments(scheds):
    """Press, then the slide of each schedule split into three targets."""
    out = []
    for s in scheds:
        (n0, p0, q0), (_, p1, q1) = s[0], s[1]
        p0, p1 = np.array(p0), np.array(p1)
        out.append([(n0, tuple(p0), q0), (10, tuple(p0 + (p1 - p0) / 3), q1), (10, tuple(p0 + 2 * (p1 - p0) / 3), q1),
                    (10, tuple(p1), q1)])
    return out


@pytest.mark.parametrize("graph", [True, False])
def test_members_sit_out_calls(gpu, graph):
    """sim_batch_set_active: a member that sits a call out keeps its state
    bitwise and its counters; its next call moves it from its last stepped pose
    to the latest target, which is what the same sensor computes alone when it
    skips that call; the members that run compute what they compute alone."""
    params, scheds = small_batch(n=4)
    segs = four_segments(scheds)
    masks = [[1, 1, 1, 1], [1, 0, 1, 1], [1, 0, 1, 0], [1, 1, 1, 1]]
    b = gpu.Batch(params, tiles=TILES[:len(params)])
    b.sim_batch_set_graph(graph)
    before = None
    for k, mask in enumerate(masks):
        b.sim_batch_set_indenter_poses(np.array([s[k][1] for s in segs]), np.array([s[k][2] for s in segs]))
        b.sim_batch_set_active(mask)
        snap = [m.sim_read_particles() for m in b.sensors] if k else None
        stats = [m.sim_get_stats()["steps"] for m in b.sensors]
        b.sim_batch_step(segs[0][k][0])
        b.sim_batch_synchronize()
        for i, a in enumerate(mask):
            if not a:
                for u, w in zip(b.sensors[i].sim_read_particles(), snap[i]):
                    assert np.array_equal(u, w), f"segment {k}: member {i} moved while sitting out"
                assert b.sensors[i].sim_get_stats()["steps"] == stats[i]
    for i, p in enumerate(params):
        s = gpu.Sim(p)
        s.sim_set_tile(*TILES[i])
        for k, mask in enumerate(masks):
            if mask[i]:
                s.sim_set_indenter_pose(segs[i][k][1], segs[i][k][2])
                s.sim_step(segs[i][k][0])
        s.sim_synchronize()
        for u, w in zip(b.sensors[i].sim_read_particles(), s.sim_read_particles()):
            assert np.array_equal(u, w), f"member {i}"
        st_b, st_s = b.sensors[i].sim_get_stats(), s.sim_get_stats()
        assert st_b["passes"] == st_s["passes"] and st_b["steps"] == st_s["steps"]
        s.close()
    b.close()


def test_sitting_out_is_checked(gpu):
    """A member cannot sit out the batch's first call or a call of an odd
    number of executed steps; a call with no active member does nothing."""
    p = W.small_sensor(cells=(8, 8, 3), subcycle=1)
    b = gpu.Batch([p, p])
    b.sim_batch_set_indenter_poses(np.array([p.pose0[:3]] * 2), np.array([p.pose0[3:]] * 2))
    b.sim_batch_set_active([1, 0])
    with pytest.raises(gpu.SimError) as e:
        b.sim_batch_step(2)
    assert e.value.code == gpu.SIM_ESTATE
    b.sim_batch_set_active([1, 1])
    b.sim_batch_step(2)
    b.sim_batch_set_active([0, 1])
    with pytest.raises(gpu.SimError) as e:
        b.sim_batch_step(1)
    assert e.value.code == gpu.SIM_EINVAL
    b.sim_batch_step(2)
    b.sim_batch_set_active([0, 0])
    x = [m.sim_read_particles()[0] for m in b.sensors]
    b.sim_batch_step(2)
    b.sim_batch_synchronize()
    assert all(np.array_equal(m.sim_read_particles()[0], xi) for m, xi in zip(b.sensors, x))
    assert [m.sim_get_stats()["steps"] for m in b.sensors] == [2, 4]
    b.close()

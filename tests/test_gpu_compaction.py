"""Storage compaction (sim_set_compaction) through the C ABI: a sensor whose
particle state is moved into the binned order every few executed steps computes
bitwise what the same sensor computes without it.  The node sums are exact
fixed-point sums, so no result depends on where a particle is stored; what can
go wrong is bookkeeping: the id map, the calibration particle of the
relative-rest test, the surface flags and the host reads and writes."""
import numpy as np
import pytest

from paper_2405_02914_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2405_02914_amd import impm
    impm.lib()
    return impm


def _segments(p):
    # press, then slip with rotation: the relative-rest loop iterates, so the
    # calibration particle's slot matters
    c = np.array(p.pose0[:3])
    return [(20, tuple(c + [0, 0, -0.4e-3]), (1, 0, 0, 0)),
            (30, tuple(c + [0.4e-3, 0, -0.4e-3]), W.quat_about_z(20))]


def _same_state(a, b):
    for u, w in zip(a.sim_read_particles(), b.sim_read_particles()):
        if not np.array_equal(u, w):
            return False
    return True


def _stats_equal(a, b):
    sa, sb = a.sim_get_stats(), b.sim_get_stats()
    return all(sa[k] == sb[k] for k in ("steps", "passes", "limit_hits", "last_r", "calib_particle"))


@pytest.mark.parametrize("graph", [False, True])
def test_compaction_is_bitwise_invisible(gpu, graph):
    p = W.small_sensor(cells=(16, 16, 6), radius=1.5e-3, subcycle=2)
    a, b = gpu.Sim(p), gpu.Sim(p)
    b.sim_set_compaction(3)
    if graph:
        a.sim_set_graph(True)
        b.sim_set_graph(True)
    print(f"compaction test: {p.cells} cells, graph={graph}", flush=True)
    for k, (n, pos, q) in enumerate(_segments(p)):
        for s in (a, b):
            s.sim_set_indenter_pose(pos, q)
        done = 0
        while done < n:
            m = min(5, n - done)
            for s in (a, b):
                s.sim_step(m)
            done += m
            # the first segment is read back after every call (host maps
            # refreshed each time), the second only at its end (several
            # compactions with stale host maps in between)
            if k == 0:
                assert _same_state(a, b), (k, done)
                assert np.array_equal(a.sim_surface_heightmap(32, 32), b.sim_surface_heightmap(32, 32))
    assert np.array_equal(a.sim_surface_heightmap(32, 32), b.sim_surface_heightmap(32, 32))
    assert _same_state(a, b)
    assert _stats_equal(a, b)
    assert np.array_equal(a.sim_read_rest()[1], b.sim_read_rest()[1])
    for s in (a, b):
        s.close()


def test_write_after_compaction(gpu):
    """A state written through the ABI after compactions lands on the right
    particles: both sensors take the same state and continue identically."""
    p = W.small_sensor(cells=(12, 12, 4), radius=1.5e-3, subcycle=2)
    a, b = gpu.Sim(p), gpu.Sim(p)
    b.sim_set_compaction(2)
    segs = _segments(p)
    n, pos, q = segs[0]
    for s in (a, b):
        s.sim_set_indenter_pose(pos, q)
        s.sim_step(n)
    x, v, Cm, G = a.sim_read_particles()
    rng = np.random.default_rng(5)
    v = (v + rng.normal(0, 1e-3, v.shape)).astype(np.float32)
    for s in (a, b):
        s.sim_write_particles(x, v, Cm, G)
    n, pos, q = segs[1]
    for s in (a, b):
        s.sim_set_indenter_pose(pos, q)
        s.sim_step(n)
    assert _same_state(a, b)
    assert _stats_equal(a, b)
    for s in (a, b):
        s.close()


def test_batch_members_with_compaction(gpu):
    """Batch members that compact (on their own streams, after the batch's
    launches) stay bitwise equal to the members of a batch that does not."""
    params, scheds = W.config3(n_sensors=3, seed=7, k_range=(2, 3), n_substeps=60)
    a, b = gpu.Batch(params), gpu.Batch(params)
    for s in b.sensors:
        s.sim_set_compaction(3)
    print(f"batch compaction test: {[p.cells for p in params]}", flush=True)
    for k in range(len(scheds[0])):
        pos = np.array([s[k][1] for s in scheds])
        quat = np.array([s[k][2] for s in scheds])
        n = scheds[0][k][0]
        for x in (a, b):
            x.sim_batch_set_indenter_poses(pos, quat)
        done = 0
        while done < n:
            m = min(5, n - done)
            for x in (a, b):
                x.sim_batch_step(m)
            done += m
    for x in (a, b):
        x.sim_batch_synchronize()
    for i in range(len(params)):
        assert _same_state(a.sensors[i], b.sensors[i]), i
        assert _stats_equal(a.sensors[i], b.sensors[i]), i
    assert np.array_equal(a.sim_batch_heightmaps(16, 16), b.sim_batch_heightmaps(16, 16))
    for x in (a, b):
        x.close()

"""The synthetic slip / rotation protocol of the paper's experiments (Sec. IV-A):
its input recipes and its height-map metrics on the CPU, and the device's
protocol runs against the FP64 oracle on a small sensor (GPU)."""
import numpy as np
import pytest

from paper_2405_02914_amd import protocol as P, workloads as W
from tests.conftest import gpu_available


def test_holed_disc_table_shape():
    t = W.holed_disc_table(4e-3, 1.5e-3, 0.75e-3, 0.3e-3, 1.0e-3, n=129, skirt=0.0)
    step = 8e-3 / 128
    x = np.arange(129) * step - 4e-3
    X, Y = np.meshgrid(x, x, indexing="xy")
    r = np.hypot(X, Y)
    assert np.all(t[(r >= 1.85e-3) & (r <= 3.2e-3)] == 0.0)          # the flat annular face
    assert np.all(t[r <= 1.5e-3] == 1.0e-3)                           # the hole floor
    assert np.all(t[(r > 3.26e-3) & (r <= 4e-3)] > 0.0)               # the rounded outer edge
    assert abs(t[64, 128] - 0.75e-3) < 1e-9                           # edge height at r = r_out
    s = W.holed_disc_table(4e-3, 1.5e-3, 0.75e-3, 0.3e-3, 1.0e-3, n=129)
    assert abs(s[64, 128] - (0.75e-3 + 5.0 * 0.5e-3)) < 1e-9          # the skirt beyond r_out


def test_protocol_schedules():
    p = W.protocol_sensor()
    s = W.protocol_schedule(p.pose0, "slip", sign=-1.0)
    assert [n for n, _, _ in s] == [250] + [500] * 5
    assert s[0][1][2] == pytest.approx(p.pose0[2] - 0.5e-3)
    assert [round((pos[0] - p.pose0[0]) * 1e3, 9) for _, pos, _ in s] == [0, -1, -2, -3, -4, -5]
    r = W.protocol_schedule(p.pose0, "rotate", sign=-1.0, increments=9)
    assert len(r) == 10 and r[-1][2] == W.quat_about_z(-45.0)


def test_hole_metrics_on_a_synthetic_map():
    p = W.protocol_sensor()
    hm = 256
    X, Y = P._pixel_centres(p, hm)
    c = (p.pose0[0] - 5e-3, p.pose0[1])
    r = np.hypot(X - c[0], Y - c[1])
    d = np.zeros((hm, hm))
    d[(r > 1.5e-3) & (r < 3.5e-3)] = 0.5
    d[r <= 1.5e-3] = 0.125
    band = (np.abs(Y - p.pose0[1]) <= 3.25e-3) & (X >= c[0]) & (X <= p.pose0[0]) & (r > 4.5e-3)
    d[band] = 0.0625
    m = P.hole_metrics(p, d, c, 4e-3, 1.5e-3, start=p.pose0[:3])
    assert m["face_mm"] == 0.5 and m["hole_mm"] == 0.125
    assert m["hole_contrast_mm"] == 0.375 and m["trace_mm"] == 0.0625


def test_follow_metric_on_synthetic_displacements():
    """A face that turned rigidly with the indenter follows it fully (1); a
    face displaced half the slide follows it by 0.5; before any sideways
    motion there is nothing to follow."""
    p = W.protocol_sensor()
    hm = 256
    X, Y = P._pixel_centres(p, hm)
    c = p.pose0[:3]
    th = np.radians(-10.0)
    x1, y1 = X - c[0], Y - c[1]
    x0 = np.cos(th) * x1 + np.sin(th) * y1                 # rotated back by -th
    y0 = -np.sin(th) * x1 + np.cos(th) * y1
    d = np.zeros((hm, hm, 3))
    d[..., 0], d[..., 1] = (x1 - x0) * 1e3, (y1 - y0) * 1e3
    assert P.follow_metric(p, d, c, W.quat_about_z(-10.0), c, 4e-3, 1.5e-3) == pytest.approx(1.0, abs=1e-9)
    half = np.zeros((hm, hm, 3))
    half[..., 0] = -0.5
    moved = (c[0] - 1e-3, c[1], c[2])
    assert P.follow_metric(p, half, moved, (1.0, 0.0, 0.0, 0.0), c, 4e-3, 1.5e-3) == pytest.approx(0.5)
    assert P.follow_metric(p, half, c, (1.0, 0.0, 0.0, 0.0), c, 4e-3, 1.5e-3) is None


@pytest.mark.gpu
@pytest.mark.skipif(not gpu_available(), reason="needs a HIP device")
@pytest.mark.parametrize("kind", ["slip", "rotate"])
@pytest.mark.parametrize("mode", [W.MODE_IMPM, W.MODE_PLAIN])
@pytest.mark.parametrize("obj", ["collider", "particles"])
def test_small_protocol_matches_oracle(oracle_lib, kind, mode, obj):
    """The protocol on a 16 x 16 x 6-cell slab (dx 0.5 mm): press 0.5 mm, two
    increments of 0.5 mm slip or 10 degrees, the object a grid collider or
    object particles as dense as the elastomer; the device replays the
    oracle's pass schedule; every height map within 1e-3 dx."""
    from paper_2405_02914_amd import impm
    extra = {} if obj == "collider" else dict(object_mode=W.OBJECT_PARTICLES, object_density=1000.0)
    p = W.protocol_sensor(dx=0.5e-3, cells=(16, 16, 6), r_out=2.5e-3, r_hole=1.0e-3, mode=mode, subcycle=2,
                          **extra)
    segs = W.protocol_schedule(p.pose0, kind, sign=-1.0, n_press=40, increments=2, step_mm=0.5,
                               step_deg=10.0, n_per_increment=40, n_per_degree_step=40)
    print(f"[protocol] {kind} mode {mode} {obj}: {p.n_particles} particles", flush=True)
    o = oracle_lib.OracleSim(p)
    o.enable_pass_log(100000)
    ho = []
    for n, pos, q in segs:
        o.set_target_pose(pos, q)
        o.step(n)
        ho.append(o.surface_heightmap(32, 32))
    g = impm.Sim(p)
    g.sim_debug_force_passes(o.pass_log())
    for k, (n, pos, q) in enumerate(segs):
        g.sim_set_indenter_pose(pos, q)
        g.sim_step(n)
        hg = g.sim_surface_heightmap(32, 32)
        err = np.abs(hg - ho[k]).max()
        print(f"[protocol] segment {k}: max |h| error {err / p.dx:.2e} dx, max depth "
              f"{(p.height - ho[k].min()) * 1e3:.3f} mm", flush=True)
        assert err <= 1e-3 * p.dx
    assert g.sim_get_stats()["passes"] == o.counters()["passes"]
    # the press shows in the map (object particles as dense as the slab are
    # pushed back by it, so their press is shallower)
    assert (p.height - ho[0].min()) > (0.3e-3 if obj == "collider" else 0.1e-3)
    xg, xo = g.sim_read_particles()[0], o.state()[0]
    assert np.abs(xg - xo).max() <= 1e-3 * p.dx

"""Shaped elastomers (column heights over the cuboid's cells, Sec. VI) on the
device against the FP64 oracle."""
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


@pytest.fixture(scope="module")
def ref(oracle_lib):
    return oracle_lib


@pytest.mark.parametrize("kind", ["dome", "disc"])
def test_shaped_elastomer_matches_oracle(gpu, ref, kind):
    cells = (16, 14, 6)
    p = W.small_sensor(cells=cells, radius=1.5e-3, subcycle=2)
    cols = W.dome_columns(cells, p.dx, 4.0e-3, 3) if kind == "dome" else W.disc_columns(cells, p.dx, 3.2e-3)
    top = float(cols.max()) * p.dx
    p = p.replace(columns=cols, pose0=(p.pose0[0], p.pose0[1], top + p.radius, 1, 0, 0, 0))
    g, o = gpu.Sim(p), ref.OracleSim(p)
    print(f"[shape] {kind}: {o.n} particles of {cells[0] * cells[1] * cells[2] * p.ppc}", flush=True)
    assert g.n == o.n == p.n_particles
    # the initial state, rest data and calibration particle: bitwise
    assert np.array_equal(g.sim_read_particles()[0], o.state()[0])
    Xg, fl = g.sim_read_rest()
    Xo, bo, so = o.rest()
    assert np.array_equal(Xg, Xo)
    assert np.array_equal((fl & 1) != 0, bo) and np.array_equal((fl & 2) != 0, so)
    assert g.sim_get_stats()["calib_particle"] == o.calib_particle
    assert np.array_equal(g.sim_surface_heightmap(24, 20), o.surface_heightmap(24, 20).astype(np.float32))
    c = np.array(p.pose0[:3])
    segs = [(15, tuple(c + [0, 0, -0.35e-3]), (1, 0, 0, 0)),
            (15, tuple(c + [0.15e-3, 0.05e-3, -0.35e-3]), W.quat_about_z(8))]
    o.enable_pass_log(10000)
    o.run_schedule(segs)
    g.sim_debug_force_passes(o.pass_log())
    g.run_schedule(segs)
    err = np.abs(g.sim_read_particles()[0] - o.state()[0]).max() / p.dx
    hg, ho = g.sim_surface_heightmap(32, 28), o.surface_heightmap(32, 28)
    herr = np.abs(hg - ho).max() / p.dx
    dg, do = g.sim_surface_displacement(32, 28), o.surface_displacement(32, 28)
    print(f"[shape] {kind}: max|dx| {err:.2e} dx, height map {herr:.2e} dx, indentation "
          f"{(top - ho.min()) * 1e3:.3f} mm", flush=True)
    assert err <= 1e-3 and herr <= 1e-3
    assert np.abs(dg - do).max() <= 1e-3 * p.dx
    assert top - ho.min() > 0.15e-3

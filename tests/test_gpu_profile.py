"""Kernel timing through the C ABI (sim_profile): every first-pass launch, or a
uniform sample of every k-th executed step, and the rejection of a negative
setting."""
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


def test_profile_counts_every_or_every_kth_step(gpu):
    p = W.small_sensor(cells=(8, 8, 4), subcycle=2)
    s = gpu.Sim(p)
    print(f"profile test: {p.cells} cells, subcycle {p.subcycle}", flush=True)
    pos = tuple(p.pose0[:3])
    s.sim_set_indenter_pose(pos, (1.0, 0.0, 0.0, 0.0))
    s.sim_profile(1)
    s.sim_step(6)                        # 12 executed steps
    ms, k = s.sim_profile_read()
    assert k == 12 and ms > 0.0
    s.sim_profile(4)
    s.sim_step(6)                        # executed steps 12..23: 12, 16, 20 are timed
    ms, k = s.sim_profile_read()
    assert k == 3 and ms > 0.0
    s.sim_profile(0)
    s.sim_step(2)
    assert s.sim_profile_read()[1] == 0
    with pytest.raises(gpu.SimError):
        s.sim_profile(-1)
    s.close()

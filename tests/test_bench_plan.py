"""Host logic of bench.py: arguments and the frame plan of the timed region
(CPU only; no GPU call)."""
import pytest

import bench
from paper_2405_02914_amd import workloads as W


def _plan(steps):
    segs = W.config2_schedule()
    return segs, bench.frame_plan(segs, steps)


@pytest.mark.parametrize("steps,warmup", [(20, 5), (40, 1), (7, 3), (1, 0), (45, 2)])
def test_any_step_and_warmup_count_is_accepted(steps, warmup):
    args = bench.parse(["--gpus", "1", "--steps", str(steps), "--warmup", str(warmup)])
    assert (args.steps, args.warmup, args.gpus) == (steps, warmup, 1)
    segs, timed = _plan(args.steps)
    _, warm = _plan(args.warmup)
    assert len(timed) == steps and len(warm) == warmup
    # every frame is one 50-substep height-map frame
    assert all(n == bench.FRAME for n, _, _ in timed + warm)
    # the timed frames start at the beginning of the schedule
    assert timed[:min(steps, len(segs))] == segs[:steps]


def test_schedule_is_40_frames_of_press_then_slip():
    segs, timed = _plan(40)
    assert len(segs) == 40 and sum(n for n, _, _ in segs) == 2000
    assert timed == segs
    p = W.config2()
    # frames 0-9 press straight down, 10-39 slip along +x and rotate about z
    for k in range(10):
        pos, q = segs[k][1], segs[k][2]
        assert pos[0] == p.pose0[0] and pos[1] == p.pose0[1] and q == (1.0, 0.0, 0.0, 0.0)
    assert segs[9][1][2] == pytest.approx(p.pose0[2] - 1.5e-3, abs=1e-12)
    assert segs[39][1][0] == pytest.approx(p.pose0[0] + 2.0e-3, abs=1e-12)


def test_frames_past_the_schedule_hold_the_final_pose():
    segs, timed = _plan(45)
    assert timed[:40] == segs
    for n, pos, q in timed[40:]:
        assert (n, pos, q) == (bench.FRAME, segs[-1][1], segs[-1][2])


def test_driver_default_times_substeps_0_to_999():
    _, timed = _plan(20)
    assert sum(n for n, _, _ in timed) == 1000


def test_negative_frame_count_is_rejected():
    with pytest.raises(ValueError):
        bench.frame_plan(W.config2_schedule(), -1)


def test_kernel_source_hash_is_stable():
    a, b = bench.kernel_source_sha(), bench.kernel_source_sha()
    assert a == b and len(a) == 16


def test_compaction_interval_defaults_per_workload():
    # the single sensor compacts every 50 executed steps, the other workloads
    # every 100, and an explicit value (0 included) is kept
    assert bench.parse([]).compact_every == 50
    assert bench.parse(["--workload", "batch"]).compact_every == 100
    assert bench.parse(["--workload", "object"]).compact_every == 100
    assert bench.parse(["--compact-every", "0"]).compact_every == 0
    assert bench.parse(["--workload", "batch", "--compact-every", "25"]).compact_every == 25

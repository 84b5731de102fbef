"""The surrogate trained on IMPM trajectories (the batched simulator produces
the data; the library's kernels train the network) predicts held-out frames
better than the method without it (persistence: next = prev) and serves
frames far faster than the simulator."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_trained_surrogate_gains_over_persistence_and_is_faster():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2405_02914_amd import sur, surrogate_train as T, workloads as W
    st = torch.cuda.Stream()
    ptr, s_tr = W.surrogate_trajectories(24, seed=11, n_substeps=500)
    pte, s_te = W.surrogate_trajectories(8, seed=12, n_substeps=500)
    print("[train-test] generating", flush=True)
    dtr = T.generate(ptr, s_tr, st, batch=24)
    dte = T.generate(pte, s_te, st, batch=8)
    assert not dtr.disp[:, 0].any()                     # rest state
    assert float(dtr.disp[:, -1].abs().max()) > 0.1     # mm: the indenters deform the surface
    net = sur.Surrogate(T.RES, T.RES, max_batch=64, stream=st.cuda_stream)
    losses, secs = T.train(net, dtr, steps=400, batch=32, stream=st, log_every=100)
    ev = T.evaluate(net, dte, st, batch=8)
    fps, _ = T.inference_rate(net, dte, st, batch=64, reps=10)
    print("[train-test]", ev, f"surrogate {fps:.0f} frames/s, IMPM {dtr.impm_frames_per_s:.1f} frames/s",
          flush=True)
    assert losses[-1][1] < 0.2 * losses[0][1]
    assert ev["rms_one_step_mm"] < ev["rms_persistence_mm"]
    assert fps >= 20 * dtr.impm_frames_per_s
    net.close()

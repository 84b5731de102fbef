"""Parity of the HIP surrogate (BF16 MFMA kernels, through the C ABI) with the
FP64 oracle of oracle/sur_oracle.py, on seeded weights and inputs.

Tolerances.  Both sides round weights, activations and pre-activation
gradients to BF16 at the same points; the device sums in FP32 where the oracle
sums exactly.  An FP32 sum of up to 2304 products lands on the other side of a
BF16 rounding boundary for a small fraction of the elements, moving each by one
BF16 step (at most 2^-7 relative).

  per layer (the tight check): each convolution's output, pre-activation
    gradient and weight gradient is recomputed by the oracle from the device's
    own inputs to that layer; every element must agree within one BF16 step
    (2^-7 |ref| + 2^-10 rms(ref) for sums that cancel), at most 2 % of them
    may differ at all, and weight gradients (FP32 sums, no rounding) agree to
    1e-4 normwise.
  end to end: single-step flips propagate and grow through 14 layers.  An
    FP32-accumulating evaluation of the same network differs from the FP64
    oracle by 1e-3 to 5e-3 normwise on these inputs, so the head output
    (next - prev) is checked at 1e-2 and the gradient blocks at 5e-2.
"""
import numpy as np
import pytest

from paper_2405_02914_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_FWD = 1e-2
TOL_GRAD = 5e-2
CH = (32, 64, 128, 256)


@pytest.fixture(scope="module")
def sur():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2405_02914_amd import sur as S
    S.lib()
    return S


@pytest.fixture(scope="module")
def ora():
    from oracle import sur_oracle
    return sur_oracle


def dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def rel(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def oracle_forward(ora, theta, depth, pose, prev):
    net = ora.SurrogateOracle(CH)
    X = ora.assemble_input(depth, pose, prev)
    pred, _ = net.forward(theta.astype(np.float64), X, prev.astype(np.float64))
    return pred


@pytest.mark.parametrize("H,Wd,n", [(32, 32, 2), (40, 24, 3), (8, 8, 1)])
def test_forward_matches_oracle(sur, ora, H, Wd, n):
    """Several pixel tiles with a ragged last tile, non-square images, the
    smallest image (8 x 8, a 1 x 1 bottom level)."""
    print(f"[sur] forward H={H} W={Wd} n={n}", flush=True)
    theta = W.surrogate_weights(CH, seed=1)
    depth, pose, prev, _ = W.surrogate_batch(n, H, Wd, seed=2)
    s = sur.Surrogate(H, Wd, CH, max_batch=n)
    s.sur_set_params(theta)
    d, p, pv = dev(depth, pose, prev)
    out = s.sur_infer(d, p, pv).cpu().numpy()
    ref = oracle_forward(ora, theta, depth, pose, prev)
    e = rel(out - prev, ref - prev)
    print(f"[sur] head output rel err {e:.2e}", flush=True)
    assert e <= TOL_FWD
    s.close()


def blocks(ora):
    out, k = [], 0
    for li, (ci, co, _, _, _) in enumerate(ora.layer_specs(CH)):
        out.append((f"W{li}", k, k + co * 9 * ci)); k += co * 9 * ci
        out.append((f"b{li}", k, k + co)); k += co
    out.append(("Wh", k, k + 3 * CH[0])); k += 3 * CH[0]
    out.append(("bh", k, k + 3))
    return out


def test_gradients_match_oracle(sur, ora):
    H, Wd, n = 32, 32, 2
    theta = W.surrogate_weights(CH, seed=3)
    depth, pose, prev, tgt = W.surrogate_batch(n, H, Wd, seed=4)
    s = sur.Surrogate(H, Wd, CH, max_batch=n)
    s.sur_set_params(theta)
    loss = s.sur_compute_grads(*dev(depth, pose, prev, tgt))
    g = s.sur_get_grads()
    net = ora.SurrogateOracle(CH)
    X = ora.assemble_input(depth, pose, prev)
    lo, go = net.loss_and_grad(theta.astype(np.float64), X, prev.astype(np.float64), tgt.astype(np.float64))
    print(f"[sur] loss {loss:.6e} oracle {lo:.6e}", flush=True)
    # |d loss| / loss <= 2 |d pred| / |pred - target|, with |d pred| at the
    # end-to-end tolerance of the head output
    assert abs(loss - lo) <= 1e-2 * lo
    worst = 0.0
    for name, a, b in blocks(ora):
        e = rel(g[a:b], go[a:b])
        worst = max(worst, e)
        assert e <= TOL_GRAD, (name, e)
    print(f"[sur] worst gradient block rel err {worst:.2e}", flush=True)
    s.close()


def bf16_close(g, r, label):
    """Element-wise: within one BF16 step; few elements differ at all."""
    g = np.asarray(g); r = np.asarray(r)
    rms = np.sqrt(np.mean(r * r)) if r.size else 0.0
    bad = np.abs(g - r) > 2.0 ** -7 * np.abs(r) + 2.0 ** -10 * rms
    frac = np.mean(g != r)
    print(f"[sur] {label}: differing {frac:.2e}, beyond one step {bad.sum()}", flush=True)
    assert not bad.any(), label
    assert frac <= 0.02, label


def test_per_layer_forward_and_backward(sur, ora):
    """Every convolution (stride 1, stride 2, upsampled with skip), the head,
    the input assembly, every pre-activation gradient and every weight
    gradient, each recomputed by the oracle from the device's own inputs to
    that layer."""
    H, Wd, n = 24, 40, 2
    theta = W.surrogate_weights(CH, seed=13)
    depth, pose, prev, tgt = W.surrogate_batch(n, H, Wd, seed=14)
    s = sur.Surrogate(H, Wd, CH, max_batch=n)
    s.sur_set_params(theta)
    s.sur_compute_grads(*dev(depth, pose, prev, tgt))
    g = s.sur_get_grads().astype(np.float64)
    specs = ora.layer_specs(CH)
    convs, (Wh, bh) = ora.unflatten(theta.astype(np.float64), CH)
    gconvs, (gWh, gbh) = ora.unflatten(g, CH)
    # shapes of every activation
    shapes, h, w = [], H, Wd
    for ci, co, st, up, skip in specs:
        h, w = (h // 2, w // 2) if st == 2 else ((h * 2, w * 2) if up else (h, w))
        shapes.append((n, h, w, co))
    x0 = s.sur_debug_read(2, 0, (n, H, Wd, 32))
    assert np.array_equal(x0[..., :10], ora.assemble_input(depth, pose, prev))
    assert not x0[..., 10:].any()
    acts = [s.sur_debug_read(0, li, shapes[li]) for li in range(14)]
    dzs = [s.sur_debug_read(1, li, shapes[li]) for li in range(14)]
    consumer = {skip: li for li, (_, _, _, _, skip) in enumerate(specs) if skip is not None}
    for li, (ci, co, st, up, skip) in enumerate(specs):
        x = x0[..., :10] if li == 0 else acts[li - 1]
        xin = ora.upsample2(x) if up else x
        Wb = ora.bf16_round(convs[li][0])
        z = ora.conv3x3(xin, Wb, st) + convs[li][1]
        if skip is not None:
            z = z + acts[skip]
        bf16_close(acts[li], ora.bf16_round(np.maximum(z, 0.0)), f"forward conv{li}")
        dW, dX = ora.conv3x3_backward(xin, Wb, st, dzs[li])
        assert rel(gconvs[li][0], dW) <= 1e-4, ("dW", li, rel(gconvs[li][0], dW))
        assert rel(gconvs[li][1], dzs[li].reshape(-1, co).sum(0)) <= 1e-4, ("db", li)
        if li > 0:
            dA = ora.upsample2_backward(dX) if up else dX
            if li - 1 in consumer:
                dA = dA + dzs[consumer[li - 1]]
            bf16_close(dzs[li - 1], ora.bf16_round(dA * (acts[li - 1] > 0)), f"gradient into conv{li - 1}")
    # head and loss gradient
    a13 = acts[13]
    pred = prev + a13 @ ora.bf16_round(Wh).T + bh
    out = s.sur_infer(*dev(depth, pose, prev)).cpu().numpy()
    assert np.abs(out - pred).max() <= 1e-5 * np.abs(pred).max()
    dout = 2.0 * (pred - tgt) / pred.size
    bf16_close(dzs[13], ora.bf16_round((dout @ ora.bf16_round(Wh)) * (a13 > 0)), "gradient into conv13")
    assert rel(gWh, dout.reshape(-1, 3).T @ a13.reshape(-1, CH[0])) <= 1e-4
    assert rel(gbh, dout.reshape(-1, 3).sum(0)) <= 1e-4
    s.close()


def test_adam_step(sur):
    """One training step applies Adam (bias-corrected, step 1 then step 2) to
    the FP32 master weights with the gradients it computed."""
    H, Wd, n = 16, 16, 2
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    theta = W.surrogate_weights(CH, seed=5).astype(np.float64)
    depth, pose, prev, tgt = W.surrogate_batch(n, H, Wd, seed=6)
    s = sur.Surrogate(H, Wd, CH, max_batch=n, lr=lr)
    s.sur_set_params(theta)
    m = np.zeros_like(theta); v = np.zeros_like(theta)
    th = s.sur_get_params().astype(np.float64)
    for t in (1, 2):
        s.sur_train_step(*dev(depth, pose, prev, tgt))
        g = s.sur_get_grads().astype(np.float64)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        th = th - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
        got = s.sur_get_params().astype(np.float64)
        err = np.abs(got - th).max()
        print(f"[sur] adam step {t}: max |theta - ref| {err:.2e}", flush=True)
        assert err <= 2e-3 * lr + 1e-6
        th = got
    s.close()


def test_full_size_forward(sur, ora):
    """The serving shape, 128 x 128, one sample."""
    theta = W.surrogate_weights(CH, seed=7)
    depth, pose, prev, _ = W.surrogate_batch(1, 128, 128, seed=8)
    s = sur.Surrogate(128, 128, CH, max_batch=4)
    s.sur_set_params(theta)
    out = s.sur_infer(*dev(depth, pose, prev)).cpu().numpy()
    ref = oracle_forward(ora, theta, depth, pose, prev)
    e = rel(out - prev, ref - prev)
    print(f"[sur] 128x128 head output rel err {e:.2e}", flush=True)
    assert e <= TOL_FWD
    s.close()


def test_params_roundtrip_and_checkpoint(sur, tmp_path):
    theta = W.surrogate_weights(CH, seed=9)
    depth, pose, prev, tgt = W.surrogate_batch(2, 16, 16, seed=10)
    s = sur.Surrogate(16, 16, CH, max_batch=2)
    s.sur_set_params(theta)
    assert np.array_equal(s.sur_get_params(), theta)
    s.sur_train_step(*dev(depth, pose, prev, tgt))
    f = tmp_path / "sur.bin"
    s.sur_save(f)
    s2 = sur.Surrogate(16, 16, CH, max_batch=2)
    s2.sur_load(f)
    assert np.array_equal(s2.sur_get_params(), s.sur_get_params())
    # identical Adam state: the next step gives identical parameters
    s.sur_train_step(*dev(depth, pose, prev, tgt))
    s2.sur_train_step(*dev(depth, pose, prev, tgt))
    assert np.allclose(s2.sur_get_params(), s.sur_get_params(), rtol=0, atol=1e-6)
    s3 = sur.Surrogate(32, 32, CH, max_batch=1)
    with pytest.raises(sur.SurError):
        s3.sur_load(f)                      # another image size
    for x in (s, s2, s3):
        x.close()


def test_rejects_bad_arguments(sur):
    with pytest.raises(sur.SurError):
        sur.Surrogate(20, 16, CH)           # not a multiple of 8
    with pytest.raises(sur.SurError):
        sur.Surrogate(16, 16, (32, 48, 128, 256))
    s = sur.Surrogate(16, 16, CH, max_batch=2)
    depth, pose, prev, _ = W.surrogate_batch(3, 16, 16, seed=0)
    with pytest.raises(sur.SurError):
        s.sur_infer(*dev(depth, pose, prev))     # n > max_batch
    s.close()


def test_training_fits_a_learnable_map(sur):
    """A target that depends on the inputs (z displacement follows the clipped
    depth): 150 Adam steps on one batch cut the loss at least tenfold."""
    H, Wd, n = 32, 32, 4
    depth, pose, prev, _ = W.surrogate_batch(n, H, Wd, seed=11)
    tgt = prev.copy()
    tgt[..., 2] += 0.1 * np.clip(depth, -3, 3)
    s = sur.Surrogate(H, Wd, CH, max_batch=n, seed=12)
    args = dev(depth, pose, prev, tgt)
    l0 = s.sur_train_step(*args, want_loss=True)
    for _ in range(148):
        s.sur_train_step(*args)
    l1 = s.sur_train_step(*args, want_loss=True)
    print(f"[sur] training loss {l0:.3e} -> {l1:.3e}", flush=True)
    assert l1 <= 0.1 * l0
    s.close()

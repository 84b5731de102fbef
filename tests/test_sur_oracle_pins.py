"""Pins of the surrogate oracle (oracle/sur_oracle.py) against things fixed
outside it: BF16 rounding of a library, convolution by its definition and by an
independent library convolution, gradients by central finite differences, and
Adam's first steps in closed form."""
import numpy as np
import pytest
import torch

from oracle import sur_oracle as S

TINY = (2, 3, 4, 5)


def test_bf16_round_matches_torch():
    """Round-to-nearest-even to 8 significant bits equals torch's float32 ->
    bfloat16 conversion on float32 inputs (ties and negatives included)."""
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 5000), rng.normal(0, 1e-6, 1000),
                        1.0 + np.arange(-300, 300) * 2.0 ** -9]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16_round(x.astype(np.float64)), want)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_matches_loops(stride):
    rng = np.random.default_rng(stride)
    X = rng.normal(size=(2, 7, 6, 3))
    W = rng.normal(size=(4, 3, 3, 3))
    got = S.conv3x3(X, W, stride)
    Ho, Wo = (7 - 1) // stride + 1, (6 - 1) // stride + 1
    want = np.zeros((2, Ho, Wo, 4))
    for n in range(2):
        for y in range(Ho):
            for x in range(Wo):
                for o in range(4):
                    acc = 0.0
                    for ty in range(3):
                        for tx in range(3):
                            yy, xx = stride * y + ty - 1, stride * x + tx - 1
                            if 0 <= yy < 7 and 0 <= xx < 6:
                                acc += float(X[n, yy, xx] @ W[o, ty, tx])
                    want[n, y, x, o] = acc
    assert np.allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_matches_torch_conv2d(stride):
    """Against torch.nn.functional.conv2d (cross-correlation, zero padding 1)."""
    rng = np.random.default_rng(10 + stride)
    X = rng.normal(size=(2, 8, 10, 5))
    W = rng.normal(size=(6, 3, 3, 5))
    want = torch.nn.functional.conv2d(torch.from_numpy(X).permute(0, 3, 1, 2),
                                      torch.from_numpy(W).permute(0, 3, 1, 2), stride=stride, padding=1)
    assert np.allclose(S.conv3x3(X, W, stride), want.permute(0, 2, 3, 1).numpy(), rtol=0, atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_backward_finite_differences(stride):
    rng = np.random.default_rng(20 + stride)
    X = rng.normal(size=(1, 6, 5, 2))
    W = rng.normal(size=(3, 3, 3, 2))
    R = rng.normal(size=S.conv3x3(X, W, stride).shape)       # loss = <R, conv(X, W)>
    dW, dX = S.conv3x3_backward(X, W, stride, R)
    h = 1e-6
    for arr, grad in ((W, dW), (X, dX)):
        for idx in zip(*[rng.integers(0, s, 6) for s in arr.shape]):
            old = arr[idx]
            arr[idx] = old + h; lp = np.sum(R * S.conv3x3(X, W, stride))
            arr[idx] = old - h; lm = np.sum(R * S.conv3x3(X, W, stride))
            arr[idx] = old
            assert abs((lp - lm) / (2 * h) - grad[idx]) <= 1e-7 * max(1.0, abs(grad[idx]))


def tiny_problem(seed=0, N=2, H=16, W=16):
    rng = np.random.default_rng(seed)
    net = S.SurrogateOracle(channels=TINY, bf16=False)
    theta = rng.normal(0, 0.5, net.n_params)
    X = rng.normal(size=(N, H, W, 10))
    prev = rng.normal(size=(N, H, W, 3))
    tgt = rng.normal(size=(N, H, W, 3))
    return net, theta, X, prev, tgt


def test_network_gradient_finite_differences():
    """Every parameter block of the U-shape (each convolution's W and b, the
    head) against central differences of the exact (unrounded) loss."""
    net, theta, X, prev, tgt = tiny_problem()
    loss, g = net.loss_and_grad(theta, X, prev, tgt)
    rng = np.random.default_rng(1)
    blocks, k = [], 0
    for ci, co, _, _, _ in net.specs:
        blocks += [(k, k + co * 9 * ci), (k + co * 9 * ci, k + co * 9 * ci + co)]
        k += co * 9 * ci + co
    blocks += [(k, k + 3 * TINY[0]), (k + 3 * TINY[0], k + 3 * TINY[0] + 3)]
    h = 1e-6
    for a, b in blocks:
        for i in rng.integers(a, b, 3):
            t = theta.copy(); t[i] += h; lp, _ = net.loss_and_grad(t, X, prev, tgt)
            t[i] -= 2 * h; lm, _ = net.loss_and_grad(t, X, prev, tgt)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (a, b, i, fd, g[i])


def test_network_matches_torch_reference():
    """The same architecture written with torch.nn.functional (conv2d, nearest
    interpolation, relu) in FP64 gives the same prediction."""
    import torch.nn.functional as F
    net, theta, X, prev, tgt = tiny_problem(seed=3)
    pred, _ = net.forward(theta, X, prev)
    convs, (Wh, bh) = S.unflatten(theta, TINY)
    x = torch.from_numpy(X).permute(0, 3, 1, 2)
    acts = []
    for (ci, co, s, up, skip), (W, b) in zip(net.specs, convs):
        if up:
            x = F.interpolate(x, scale_factor=2, mode="nearest")
        z = F.conv2d(x, torch.from_numpy(W).permute(0, 3, 1, 2), torch.from_numpy(b), stride=s, padding=1)
        if skip is not None:
            z = z + acts[skip]
        x = torch.relu(z)
        acts.append(x)
    head = torch.einsum("nchw,oc->nhwo", x, torch.from_numpy(Wh)) + torch.from_numpy(bh)
    assert np.allclose(pred, prev + head.numpy(), rtol=0, atol=1e-10)


def test_zero_network_predicts_previous():
    net = S.SurrogateOracle(channels=TINY)
    rng = np.random.default_rng(4)
    prev = rng.normal(size=(1, 8, 8, 3))
    pred, _ = net.forward(np.zeros(net.n_params), rng.normal(size=(1, 8, 8, 10)), prev)
    assert np.array_equal(pred, prev)


def test_adam_first_steps_closed_form():
    """Step 1 from zero moments moves each parameter by lr g / (|g| + eps);
    step 2 with gradients g1, g2 by the bias-corrected moments written out."""
    g1 = np.array([0.3, -2.0, 1e-9, 0.0])
    g2 = np.array([0.1, 1.0, -4e-9, 5.0])
    th0 = np.array([1.0, -1.0, 0.5, 0.0])
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    th1, m, v = S.SurrogateOracle.adam(th0, g1, np.zeros(4), np.zeros(4), 1, lr, b1, b2, eps)
    assert np.allclose(th1, th0 - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    th2, _, _ = S.SurrogateOracle.adam(th1, g2, m, v, 2, lr, b1, b2, eps)
    mh = (0.09 * g1 + 0.1 * g2) / 0.19
    vh = (0.000999 * g1 ** 2 + 0.001 * g2 ** 2) / (1 - 0.999 ** 2)
    assert np.allclose(th2, th1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-15)


def test_bf16_network_rounds_activations():
    """With rounding on, every stored activation is a BF16 value and the
    prediction stays close to the exact network."""
    net_e, theta, X, prev, tgt = tiny_problem(seed=5)
    net_r = S.SurrogateOracle(channels=TINY, bf16=True)
    Xr = S.bf16_round(X)
    pr, (acts, _) = net_r.forward(theta, Xr, prev)
    pe, _ = net_e.forward(theta, Xr, prev)
    for a in acts:
        assert np.array_equal(S.bf16_round(a), a)
    assert np.linalg.norm(pr - pe) <= 0.05 * np.linalg.norm(pe - prev)


def test_assemble_input_channels():
    depth = np.array([[[0.5, -4.0], [4.0, 0.0]]])
    pose = np.array([[0.1, -0.2, 0.0, 0.01, 0.0, -0.03]])
    prev = np.arange(12, dtype=np.float64).reshape(1, 2, 2, 3) * 0.01
    X = S.assemble_input(depth, pose, prev, bf16=False)
    assert np.allclose(X[0, :, :, 0], [[0.5, -3.0], [3.0, 0.0]])
    assert np.allclose(X[0, 1, 0, 1:7], pose[0])
    assert np.allclose(X[..., 7:], prev)

"""Plain FP64 oracle of the learned surrogate: a U-shaped convolutional network
that maps the indenter depth map, the pose change and the previous surface
displacement of a sensor to its next surface displacement.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports or calls this
module; only the test suite, the smoke check and the benchmark's CPU baseline
leg use it.  It shares no code with the HIP path.

The surrogate is not described in arXiv 2405.02914: the paper's simulator
(Sec. III-A) is the slow, exact method, and the surrogate is an added serving
pattern that learns one frame of it.  What this file fixes, so that the device
path can be compared against it:

  network     4 levels of 3x3 convolutions (zero padding 1) with channel widths
              c = (c0, c1, c2, c3); each level has two convolutions; the
              encoder halves the resolution with a stride-2 convolution; the
              decoder doubles it by nearest-neighbour upsampling followed by a
              convolution whose pre-activation adds the encoder activation of
              the same level (skip); ReLU after every convolution; a 1x1 head
              maps c0 channels to 3, and the prediction is prev + head.
  inputs      channel 0: depth of the indenter below the slab top, mm, clipped
              to [-3, 3]; channels 1-6: pose change (translation mm, rotation
              vector rad), the same at every pixel; channels 7-9: previous
              displacement (mm).
  precision   weights and activations are BF16 values (round to nearest even
              of the exact value); every sum is exact here (FP64) and FP32 on
              the device; gradients of pre-activations are rounded to BF16
              where the device stores them; weight and bias gradients, the
              head and the loss are not rounded.
  loss        mean over all pixels and components of (pred - target)^2.
  optimiser   Adam (Kingma and Ba 2015, Algorithm 1) with bias correction on
              the unrounded master parameters.

Flat parameter layout: for each of the 14 convolutions in order, W[Cout][3][3]
[Cin] then b[Cout]; then the head W[3][c0] and b[3].
"""
from __future__ import annotations

import numpy as np


def bf16_round(x):
    """Round to the nearest BF16 value (8 significant bits), ties to even."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)                  # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(np.ldexp(m, 8)), e - 8)


def layer_specs(channels=(32, 64, 128, 256), in_ch=10):
    """(cin, cout, stride, upsample, skip_source) of the 14 convolutions."""
    c0, c1, c2, c3 = channels
    return [
        (in_ch, c0, 1, False, None), (c0, c0, 1, False, None),     # 0, 1: level 0
        (c0, c1, 2, False, None), (c1, c1, 1, False, None),        # 2, 3: level 1
        (c1, c2, 2, False, None), (c2, c2, 1, False, None),        # 4, 5: level 2
        (c2, c3, 2, False, None), (c3, c3, 1, False, None),        # 6, 7: level 3
        (c3, c2, 1, True, 5), (c2, c2, 1, False, None),            # 8, 9: up to level 2
        (c2, c1, 1, True, 3), (c1, c1, 1, False, None),            # 10, 11: up to level 1
        (c1, c0, 1, True, 1), (c0, c0, 1, False, None),            # 12, 13: up to level 0
    ]


def n_params(channels=(32, 64, 128, 256), in_ch=10, out_ch=3):
    n = sum(co * 9 * ci + co for ci, co, _, _, _ in layer_specs(channels, in_ch))
    return n + out_ch * channels[0] + out_ch


def unflatten(theta, channels=(32, 64, 128, 256), in_ch=10, out_ch=3):
    """Views (W, b) per convolution, then (Wh, bh) of the head."""
    out, k = [], 0
    for ci, co, _, _, _ in layer_specs(channels, in_ch):
        W = theta[k:k + co * 9 * ci].reshape(co, 3, 3, ci); k += co * 9 * ci
        b = theta[k:k + co]; k += co
        out.append((W, b))
    Wh = theta[k:k + out_ch * channels[0]].reshape(out_ch, channels[0]); k += out_ch * channels[0]
    bh = theta[k:k + out_ch]; k += out_ch
    assert k == theta.size
    return out, (Wh, bh)


# ---------------------------------------------------------------- convolution

def patches(X, stride):
    """im2col of a 3x3 window with zero padding 1: (N, Ho, Wo, 3, 3, C)."""
    N, H, W, C = X.shape
    Xp = np.zeros((N, H + 2, W + 2, C))
    Xp[:, 1:H + 1, 1:W + 1] = X
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    P = np.empty((N, Ho, Wo, 3, 3, C))
    for ty in range(3):
        for tx in range(3):
            P[:, :, :, ty, tx] = Xp[:, ty:ty + stride * (Ho - 1) + 1:stride, tx:tx + stride * (Wo - 1) + 1:stride]
    return P


def conv3x3(X, W, stride):
    """out[n,y,x,o] = sum_{ty,tx,c} Xpad[n, s y + ty, s x + tx, c] W[o,ty,tx,c]."""
    P = patches(X, stride)
    N, Ho, Wo = P.shape[:3]
    return (P.reshape(N * Ho * Wo, -1) @ W.reshape(W.shape[0], -1).T).reshape(N, Ho, Wo, W.shape[0])


def conv3x3_backward(X, W, stride, dZ):
    """Gradients of conv3x3 with respect to W and X, given dZ = dL/d(out)."""
    P = patches(X, stride)
    N, Ho, Wo = P.shape[:3]
    C = X.shape[3]
    dW = (dZ.reshape(-1, W.shape[0]).T @ P.reshape(N * Ho * Wo, -1)).reshape(W.shape)
    dP = (dZ.reshape(-1, W.shape[0]) @ W.reshape(W.shape[0], -1)).reshape(N, Ho, Wo, 3, 3, C)
    H, Wd = X.shape[1:3]
    dXp = np.zeros((N, H + 2, Wd + 2, C))
    for ty in range(3):
        for tx in range(3):
            dXp[:, ty:ty + stride * (Ho - 1) + 1:stride, tx:tx + stride * (Wo - 1) + 1:stride] += dP[:, :, :, ty, tx]
    return dW, dXp[:, 1:H + 1, 1:Wd + 1]


def upsample2(X):
    return X.repeat(2, axis=1).repeat(2, axis=2)


def upsample2_backward(dXu):
    N, H, W, C = dXu.shape
    return dXu.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# ---------------------------------------------------------------- network

class SurrogateOracle:
    """The network of the module docstring; `bf16=False` turns every rounding
    off (exact FP64 arithmetic, for the finite-difference pins)."""

    def __init__(self, channels=(32, 64, 128, 256), in_ch=10, out_ch=3, bf16=True):
        self.channels, self.in_ch, self.out_ch = tuple(channels), in_ch, out_ch
        self.specs = layer_specs(channels, in_ch)
        self.n_params = n_params(channels, in_ch, out_ch)
        self.rnd = bf16_round if bf16 else (lambda x: np.asarray(x, np.float64))

    def forward(self, theta, X, prev):
        """X: (N, H, W, in_ch) network input (already rounded), prev: (N, H, W, 3)
        previous displacement (mm).  Returns pred and the cache of activations."""
        convs, (Wh, bh) = unflatten(np.asarray(theta, np.float64), self.channels, self.in_ch, self.out_ch)
        acts, ins = [], []
        x = np.asarray(X, np.float64)
        for li, ((ci, co, s, up, skip), (W, b)) in enumerate(zip(self.specs, convs)):
            xin = upsample2(x) if up else x
            z = conv3x3(xin, self.rnd(W), s) + b
            if skip is not None:
                z = z + acts[skip]
            a = self.rnd(np.maximum(z, 0.0))
            ins.append(xin)
            acts.append(a)
            x = a
        head = x @ self.rnd(Wh).T + bh
        pred = np.asarray(prev, np.float64) + head
        return pred, (acts, ins)

    def loss_and_grad(self, theta, X, prev, target):
        theta = np.asarray(theta, np.float64)
        convs, (Wh, bh) = unflatten(theta, self.channels, self.in_ch, self.out_ch)
        pred, (acts, ins) = self.forward(theta, X, prev)
        diff = pred - np.asarray(target, np.float64)
        loss = float(np.mean(diff * diff))
        dout = 2.0 * diff / diff.size
        g = np.zeros_like(theta)
        gconvs, (gWh, gbh) = unflatten(g, self.channels, self.in_ch, self.out_ch)
        a13 = acts[-1]
        gWh[...] = dout.reshape(-1, self.out_ch).T @ a13.reshape(-1, a13.shape[-1])
        gbh[...] = dout.reshape(-1, self.out_ch).sum(0)
        dA = dout @ self.rnd(Wh)                       # d loss / d a13
        skip_grad = {}
        for li in range(len(self.specs) - 1, -1, -1):
            ci, co, s, up, skip = self.specs[li]
            a = acts[li]
            if li in skip_grad:
                dA = dA + skip_grad[li]
            dZ = self.rnd(dA * (a > 0))
            if skip is not None:
                skip_grad[skip] = dZ
            W, _ = convs[li]
            gW, gb = gconvs[li]
            dW, dX = conv3x3_backward(ins[li], self.rnd(W), s, dZ)
            gW[...] = dW
            gb[...] = dZ.reshape(-1, co).sum(0)
            if li == 0:
                break
            dA = upsample2_backward(dX) if up else dX
        return loss, g

    @staticmethod
    def adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam update (step number t >= 1); returns new theta, m, v."""
        m = beta1 * m + (1.0 - beta1) * grad
        v = beta2 * v + (1.0 - beta2) * grad * grad
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def contact_area(depth_mm, disp_mm, tol_mm=0.02):
    """Pixels per sample where the indenter's lower surface (slab top minus
    depth) lies at or below the displaced surface plus tol:
    top - depth <= top + u_z + tol."""
    depth_mm = np.asarray(depth_mm, np.float64)
    uz = np.asarray(disp_mm, np.float64)[..., 2]
    return ((-depth_mm) <= uz + tol_mm).reshape(depth_mm.shape[0], -1).sum(1)


def assemble_input(depth_mm, pose6, prev_mm, bf16=True):
    """Network input (N, H, W, 10): depth (mm, clipped to [-3, 3]), the six
    pose-change values at every pixel, the previous displacement (mm)."""
    depth_mm = np.asarray(depth_mm, np.float64)
    N, H, W = depth_mm.shape
    X = np.empty((N, H, W, 10))
    X[..., 0] = np.clip(depth_mm, -3.0, 3.0)
    X[..., 1:7] = np.asarray(pose6, np.float64)[:, None, None, :]
    X[..., 7:10] = prev_mm
    return bf16_round(X) if bf16 else X

"""Pins of the FP64 renderer oracle (Sec. III-B: the elastomer surface meshed
from the depth image, diffuse, lit by the sensor's LEDs, path traced).

Fixed independently: the irradiance of a flat surface from a rectangle in a
parallel plane (Lambert's closed form of the point-to-rectangle form factor),
a tiny light against the inverse-square cosine law, the shadow that an
indentation casts (found geometrically), linearity in the albedo, the bounce
term vanishing on a flat surface, and determinism of the draws."""
import math

import numpy as np
import pytest

from oracle import render_ref as R

L_MM = 8e-3


@pytest.fixture(scope="module", autouse=True)
def built():
    R.build()


def flat(z=3e-3, n=12):
    return np.full((n, n), z)


def white(v=1.0):
    return np.full((2, 2, 3), v)


def corner_factor(a, b, c):
    """Form factor from a differential area to a parallel a x b rectangle at
    distance c, the area's normal through one corner of the rectangle."""
    X, Y = a / c, b / c
    return (X / math.sqrt(1 + X * X) * math.atan(Y / math.sqrt(1 + X * X)) +
            Y / math.sqrt(1 + Y * Y) * math.atan(X / math.sqrt(1 + Y * Y))) / (2 * math.pi)


def test_parallel_rectangle_closed_form():
    """Flat surface at z = 3 mm seen from below; a 4 x 2 mm light at z = 1 mm
    facing up, centred under the pixel: pixel = rho L F with F four corner form
    factors (Monte Carlo, 4096 samples, within 4 standard errors)."""
    z0, zl, a, b = 3e-3, 1e-3, 2e-3, 1e-3
    light = dict(c=(L_MM / 2, L_MM / 2, zl), e1=(2 * a, 0, 0), e2=(0, 2 * b, 0), L=(2.0, 1.0, 0.5))
    img = R.render(flat(z0), L_MM, L_MM, [light], white(0.8), 1, 1, 4096, seed=3, bounces=1)
    F = 4 * corner_factor(a, b, z0 - zl)
    want = 0.8 * np.array([2.0, 1.0, 0.5]) * F
    # the per-sample estimate's spread, from the same estimator with more samples
    ref = R.render(flat(z0), L_MM, L_MM, [light], white(0.8), 1, 1, 65536, seed=9, bounces=1)
    assert np.allclose(ref[0, 0], want, rtol=4e-3)
    assert np.allclose(img[0, 0], want, rtol=1.5e-2)


def test_tiny_light_inverse_square_cosine():
    """A 10 nm light: the pixel value is rho L A cos(p) cos(l) / (pi d^2)."""
    z0 = 3e-3
    c = np.array([1e-3, 6e-3, 0.5e-3])
    s = 1e-8
    e1, e2 = np.array([s, 0, 0]), np.array([0, 0.6 * s, 0.8 * s])     # tilted light
    light = dict(c=tuple(c), e1=tuple(e1), e2=tuple(e2), L=(1e10, 2e10, 3e10))
    img = R.render(flat(z0), L_MM, L_MM, [light], white(0.5), 4, 4, 2, seed=1, bounces=1)
    for v in range(4):
        for u in range(4):
            p = np.array([(u + 0.5) * 2e-3, (v + 0.5) * 2e-3, z0])
            w = c - p
            d = np.linalg.norm(w)
            w /= d
            nl = np.cross(e1, e2)
            A = np.linalg.norm(nl)
            cos_p = w @ np.array([0, 0, -1.0])
            cos_l = -(nl / A) @ w
            want = 0.5 * np.array([1e10, 2e10, 3e10]) * A * cos_p * cos_l / (math.pi * d * d) if cos_l > 0 else 0 * w
            assert np.allclose(img[v, u], want, rtol=1e-5)


def test_indentation_casts_a_shadow():
    """A 2 mm square pushed 1 mm down toward the camera, lit by a tiny light at
    grazing height on the -x side: surface points whose segment to the light
    passes the dip's block are dark, the others lit (pixels near the dip's
    sloped rims excluded)."""
    n = 33
    h = np.full((n, n), 3e-3)
    px = L_MM / n
    xs = (np.arange(n) + 0.5) * px
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    dip = (np.abs(X - 4e-3) < 1e-3) & (np.abs(Y - 4e-3) < 1e-3)
    h[dip] = 2e-3
    lc = np.array([-20e-3, 4e-3, 1.5e-3])
    light = dict(c=tuple(lc), e1=(0, 1e-7, 0), e2=(0, 0, 1e-7), L=(1e12, 1e12, 1e12))
    img = R.render(h, L_MM, L_MM, [light], white(1.0), n, n, 1, seed=1, bounces=1)
    x_lo, x_hi = X[dip].min(), X[dip].max()
    checked = 0
    for v in range(n):
        for u in range(n):
            x, y = X[v, u], Y[v, u]
            if dip[v, u] or abs(y - 4e-3) > 0.8e-3 or x < x_hi + 2 * px:
                continue                           # rims, off-axis and the dip's own pixels
            # the segment from (x, y, 3 mm) to the light at the dip's far (+x) edge
            t = (x - x_hi) / (x - lc[0])
            z_at = 3e-3 + t * (lc[2] - 3e-3)
            shadow = z_at > 2e-3
            lit = img[v, u, 0] > 0
            assert lit == (not shadow), (u, v)
            checked += 1
    assert checked > 10


def test_albedo_scales_direct_light_and_flat_surface_has_no_bounce():
    light = dict(c=(4e-3, 4e-3, 1e-3), e1=(4e-3, 0, 0), e2=(0, 3e-3, 0), L=(1.0, 1.0, 1.0))
    a = R.render(flat(), L_MM, L_MM, [light], white(1.0), 6, 6, 16, seed=5, bounces=1)
    b = R.render(flat(), L_MM, L_MM, [light], white(0.25), 6, 6, 16, seed=5, bounces=1)
    c = R.render(flat(), L_MM, L_MM, [light], white(1.0), 6, 6, 16, seed=5, bounces=2)
    assert np.array_equal(b, 0.25 * a)
    assert np.array_equal(a, c)


def test_bounce_adds_light_in_a_groove_and_draws_are_deterministic():
    n = 24
    xs = (np.arange(n) + 0.5) * L_MM / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    h = 3e-3 - 1.5e-3 * np.exp(-((X - 4e-3) ** 2) / (2 * 0.6e-3 ** 2))      # a ridge toward the camera
    lights = [dict(c=(4e-3, 4e-3, 0.5e-3), e1=(6e-3, 0, 0), e2=(0, 6e-3, 0), L=(1.0, 0.8, 0.6))]
    one = R.render(h, L_MM, L_MM, lights, white(0.9), 8, 8, 32, seed=7, bounces=1)
    two = R.render(h, L_MM, L_MM, lights, white(0.9), 8, 8, 32, seed=7, bounces=2)
    again = R.render(h, L_MM, L_MM, lights, white(0.9), 8, 8, 32, seed=7, bounces=2)
    other = R.render(h, L_MM, L_MM, lights, white(0.9), 8, 8, 32, seed=8, bounces=2)
    assert np.array_equal(two, again) and not np.array_equal(two, other)
    assert np.all(two >= one) and (two - one).max() > 0

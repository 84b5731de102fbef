"""Pins of the FP64 renderer oracle (Sec. III-B: the elastomer surface meshed
from the depth image, diffuse, lit by the sensor's LEDs, path traced).

Fixed independently: the irradiance of a flat surface from a rectangle in a
parallel plane (Lambert's closed form of the point-to-rectangle form factor),
a tiny light against the inverse-square cosine law (on a flat surface, a tilted
plane and a quadratic surface, whose shading normals are known in closed form), the shadow that an
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


def _tiny_light_value(p, nrm, c, e1, e2, L, rho):
    w = c - p
    d = np.linalg.norm(w)
    w = w / d
    nl = np.cross(e1, e2)
    A = np.linalg.norm(nl)
    cos_p, cos_l = nrm @ w, -(nl / A) @ w
    return rho * L * A * cos_p * cos_l / (math.pi * d * d) if (cos_p > 0 and cos_l > 0) else 0.0 * L


@pytest.mark.parametrize("kind", ["plane", "quadratic"])
def test_shading_normal_on_planes_and_quadratics(kind):
    """Shading normal (reading: the slope field interpolated from central
    differences).  On a tilted plane z = z0 + a x + b y every pixel sees the
    plane's normal; on z = z0 + c (x - x0)^2 + e (y - y0)^2 the central
    difference is the exact derivative, so at the samples (image = map
    resolution) the normal is the analytic one (border samples excluded: there
    the difference is one-sided).  Tiny light: the inverse-square cosine law
    with that normal."""
    nx, ny, Ly = 9, 7, 6e-3          # non-square samples: px != py
    X, Y = np.meshgrid((np.arange(nx) + 0.5) * L_MM / nx, (np.arange(ny) + 0.5) * Ly / ny, indexing="xy")
    if kind == "plane":
        a, b = 0.08, -0.05
        h = 3e-3 + a * X + b * Y
        grad = lambda x, y: (a, b)
    else:
        c, e = 20.0, -12.0
        h = 3e-3 + c * (X - 4e-3) ** 2 + e * (Y - 3.5e-3) ** 2
        grad = lambda x, y: (2 * c * (x - 4e-3), 2 * e * (y - 3.5e-3))
    lc = np.array([3.1e-3, 4.3e-3, 0.5e-3])
    s = 1e-8
    e1, e2 = np.array([s, 0, 0]), np.array([0, s, 0])
    Lrgb = np.array([1e10, 2e10, 3e10])
    light = dict(c=tuple(lc), e1=tuple(e1), e2=tuple(e2), L=tuple(Lrgb))
    img = R.render(h, L_MM, Ly, [light], white(0.5), nx, ny, 2, seed=1, bounces=1)
    for v in (range(ny) if kind == "plane" else range(1, ny - 1)):
        for u in (range(nx) if kind == "plane" else range(1, nx - 1)):
            gx, gy = grad(X[v, u], Y[v, u])
            nrm = np.array([gx, gy, -1.0]) / math.sqrt(gx * gx + gy * gy + 1.0)
            p = np.array([X[v, u], Y[v, u], h[v, u]])
            want = _tiny_light_value(p, nrm, lc, e1, e2, Lrgb, 0.5)
            assert want.max() > 1e-3                        # lit: the test has teeth
            assert np.allclose(img[v, u], want, rtol=2e-5, atol=0.0), (u, v)


def test_pixel_subset_matches_the_whole_image():
    n = 16
    xs = (np.arange(n) + 0.5) * L_MM / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    h = 3e-3 - 1e-3 * np.exp(-((X - 4e-3) ** 2 + (Y - 4e-3) ** 2) / (2 * 1e-3 ** 2))
    lights = [dict(c=(4e-3, -1e-3, 0.5e-3), e1=(6e-3, 0, 0), e2=(0, 0.5e-3, 0.87e-3), L=(1.0, 0.8, 0.6))]
    full = R.render(h, L_MM, L_MM, lights, white(0.9), 12, 10, 8, seed=4, bounces=2)
    pix = [0, 7, 33, 119]
    sub = R.render_pixels(pix, h, L_MM, L_MM, lights, white(0.9), 12, 10, 8, seed=4, bounces=2)
    assert np.array_equal(sub, full.reshape(-1, 3)[pix])


def test_texture_is_bilinear_between_texel_centres():
    """Direct light only, flat surface: the image of a textured surface divided
    by that of a white one is the albedo at the pixel's surface point.  A 3 x 2
    texture (red channel 0.2, 0.8, 0.5 along x; green 0.3 and 0.9 along y) is
    linear between texel centres and constant beyond the outer centres."""
    light = dict(c=(4e-3, 4e-3, 1e-3), e1=(8e-3, 0, 0), e2=(0, 8e-3, 0), L=(1.0, 1.0, 1.0))
    tex = np.zeros((2, 3, 3))
    tex[:, :, 0] = [0.2, 0.8, 0.5]
    tex[0, :, 1], tex[1, :, 1] = 0.3, 0.9
    tex[:, :, 2] = 1.0
    n = 12
    a = R.render(flat(), L_MM, L_MM, [light], tex, n, n, 4, seed=2, bounces=1)
    b = R.render(flat(), L_MM, L_MM, [light], white(1.0), n, n, 4, seed=2, bounces=1)
    rho = a / b
    for u in range(n):
        s = min(max((u + 0.5) / n * 3 - 0.5, 0.0), 2.0)
        i = min(int(s), 1)
        want = (1 - (s - i)) * [0.2, 0.8, 0.5][i] + (s - i) * [0.2, 0.8, 0.5][i + 1]
        assert np.allclose(rho[:, u, 0], want, rtol=1e-12)
    for v in range(n):
        t = min(max((v + 0.5) / n * 2 - 0.5, 0.0), 1.0)
        assert np.allclose(rho[v, :, 1], 0.3 + 0.6 * t, rtol=1e-12)
    assert np.allclose(rho[:, :, 2], 1.0, rtol=1e-12)


def test_one_bounce_matches_the_form_factor_integral():
    """The interreflection term on a V-groove seen from below (two planes of
    slope +-a meeting at a sample column, so the mesh is exact), lit by a tiny
    light under the fold (no shadows anywhere).  The term is the bounces = 2
    image minus the bounces = 1 image (same draws for the direct part).  The
    expectation, computed here as an area integral over the facing plane
    instead of over directions: rho(p) * integral of cos(p) cos(p2) / (pi r^2)
    * D(p2) dA, with D(p2) the direct light at p2 (shading normal of p2, the
    camera-side test with it), against 16 seeds x 65536 samples (4 standard
    errors)."""
    W_, H_, fold = 17, 5, 8
    Lx, Ly = 8e-3, 2e-3
    px, py = Lx / W_, Ly / H_
    a = 0.5
    z0 = 3e-3
    xs = (np.arange(W_) + 0.5) * px
    hx = z0 - a * np.abs(xs - xs[fold])
    h = np.tile(hx, (H_, 1))
    lc = np.array([xs[fold], Ly / 2, 0.5e-3])
    s = 1e-8
    Lrgb = np.array([1e9, 1e9, 1e9])
    light = dict(c=tuple(lc), e1=(s, 0, 0), e2=(0, s, 0), L=tuple(Lrgb))
    rho = 0.6                                    # uniform albedo: the term carries rho^2
    u0, v0 = 4, 2                                # pixel on the left plane, away from the fold
    runs1, runs2 = [], []
    for seed in range(16):
        one = R.render_pixels([v0 * W_ + u0], h, Lx, Ly, [light], white(rho), W_, H_, 65536, seed=100 + seed,
                              bounces=1)[0, 0]
        two = R.render_pixels([v0 * W_ + u0], h, Lx, Ly, [light], white(rho), W_, H_, 65536, seed=100 + seed,
                              bounces=2)[0, 0]
        runs1.append(one)
        runs2.append(two - one)
    mc = np.mean(runs2)
    se = np.std(runs2, ddof=1) / math.sqrt(len(runs2))
    # the integral: p on the left plane; p2 over the right plane's part of the mesh
    p = np.array([xs[u0], (v0 + 0.5) * py, hx[u0]])
    n1 = np.array([a, 0.0, -1.0]) / math.sqrt(1 + a * a)
    nx_, ny_ = 1600, 400
    X2 = xs[fold] + (np.arange(nx_) + 0.5) / nx_ * (xs[-1] - xs[fold])
    Y2 = 0.5 * py + (np.arange(ny_) + 0.5) / ny_ * ((H_ - 1) * py)
    X2, Y2 = np.meshgrid(X2, Y2, indexing="xy")
    Z2 = z0 - a * (X2 - xs[fold])
    dA = (xs[-1] - xs[fold]) / nx_ * ((H_ - 1) * py) / ny_ * math.sqrt(1 + a * a)
    # shading slope on the right plane: vertex slopes 0 at the fold, -a beyond, linear between
    sx = np.where(X2 - xs[fold] < px, -a * (X2 - xs[fold]) / px, -a)
    n2s = np.stack([sx, np.zeros_like(sx), -np.ones_like(sx)], -1) / np.sqrt(sx * sx + 1)[..., None]
    n2g = np.array([-a, 0.0, -1.0]) / math.sqrt(1 + a * a)
    R2 = np.stack([X2, Y2, Z2], -1) - p
    r = np.linalg.norm(R2, axis=-1)
    om = R2 / r[..., None]
    cos1 = om @ n1
    cos2 = -(om @ n2g)
    side = (n2s * om).sum(-1) < 0                # met from the camera side
    wl = lc - np.stack([X2, Y2, Z2], -1)
    dl = np.linalg.norm(wl, axis=-1)
    wl = wl / dl[..., None]
    cp2 = np.maximum((n2s * wl).sum(-1), 0)
    cl = np.maximum(-wl[..., 2], 0)              # the light faces +z: cos = -(n_l . w)
    D = Lrgb[0] * s * s * cp2 * cl / (math.pi * dl * dl)
    integrand = np.where((cos1 > 0) & (cos2 > 0) & side, cos1 * cos2 / (math.pi * r * r) * D, 0.0)
    want = rho * rho * float(integrand.sum() * dA)
    print(f"bounce term: Monte Carlo {mc:.6e} +- {se:.1e}, integral {want:.6e}")
    assert want > 0.01 * np.mean(runs1)           # the bounce is a visible share of the pixel
    assert abs(mc - want) <= 4 * se + 2e-3 * want, (mc, want, se)

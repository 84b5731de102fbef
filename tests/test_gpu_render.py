"""The device renderer (include/render.h) against the FP64 oracle on the same
draws (Sec. III-B: the elastomer surface meshed from the depth image, diffuse,
lit by the sensor's LEDs, path traced).

The estimator is a deterministic function of the draws, so the two agree to
FP32 rounding except where a ray grazes a mesh edge and FP32 and FP64 decide
its hit differently (a shadow flips, or a bounce meets the other triangle of a
cell): that changes one sample of one pixel.  (The shading normal and the
texture lookup are continuous, so pixels that fall on triangle or texel edges
do not flip.)  The bar: 99 % of pixels within 1e-4 of the image's largest
value, the mean absolute difference within 2e-5 of the mean value, and no
pixel off by more than two samples' worth of the brightest pixel (2 / spp)."""
import numpy as np
import pytest

from paper_2405_02914_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2405_02914_amd import render
    render.lib()
    return render


@pytest.fixture(scope="module")
def oracle():
    from oracle import render_ref
    render_ref.build()
    return render_ref


def scene(h, w, Lx, Ly, top, depth, seed):
    hm = W.dented_heightmap(h, w, Lx, Ly, top, depth=depth, radius=0.3 * min(Lx, Ly), seed=seed,
                            roughness=2e-6).astype(np.float32)
    return hm, W.sensor_lights(Lx, Ly, top), W.sensor_texture(24, 32, seed=seed)


def check(img_g, img_o, spp, tag):
    err = np.abs(img_g - img_o)
    scale = img_o.max()
    frac = float((err.max(axis=-1) <= 1e-4 * scale).mean())
    mean_rel = float(err.mean() / img_o.mean())
    print(f"[render] {tag}: {frac * 100:.2f}% of pixels within 1e-4, mean |diff| {mean_rel:.2e} of the mean, "
          f"max |diff| {err.max() / scale:.2e} of the max", flush=True)
    assert frac >= 0.99
    assert mean_rel <= 2e-5
    assert err.max() <= 2.0 / spp * scale


@pytest.mark.parametrize("bounces", [1, 2])
@pytest.mark.parametrize("shape", [(40, 32, 20, 16), (37, 29, 23, 13)])
def test_render_matches_oracle(gpu, oracle, bounces, shape):
    """Height maps spanning several 8 x 8-cell tiles with ragged edges; images
    smaller than, and not a multiple of, the 64-pixel block."""
    import torch
    w, h, ow, oh = shape
    Lx, Ly, top = 8e-3, 6.4e-3, 3e-3
    hm, lights, tex = scene(h, w, Lx, Ly, top, 0.8e-3, seed=w)
    spp = 16
    r = gpu.Renderer(lights, tex, Lx, Ly, spp=spp, bounces=bounces, seed=11)
    img = r.render(torch.from_numpy(hm).cuda(), oh, ow).cpu().numpy()
    torch.cuda.synchronize()
    ref = oracle.render(hm.astype(np.float64), Lx, Ly, lights, tex.astype(np.float32).astype(np.float64), ow, oh,
                        spp, seed=11, bounces=bounces)
    assert img.shape == ref.shape and np.all(np.isfinite(img))
    check(img, ref, spp, f"{w}x{h} -> {ow}x{oh}, {bounces} bounce(s)")


@pytest.mark.parametrize("shape", [(200, 150, 100, 75), (257, 131, 257, 131)])
def test_multi_block_maps_sampled_pixels(gpu, oracle, shape):
    """Maps of several 64 x 64-cell blocks of the height-range grid, ragged at
    both ends, with an off-centre dent: 48 pixels computed one by one."""
    import torch
    w, h, ow, oh = shape
    Lx, Ly, top = 16e-3, 12e-3, 3e-3
    hm = W.dented_heightmap(h, w, Lx, Ly, top, depth=1.0e-3, radius=3e-3, centre=(6e-3, 7e-3), seed=w,
                            roughness=1e-6).astype(np.float32)
    lights = W.sensor_lights(Lx, Ly, top)
    tex = W.sensor_texture(48, 64, seed=w)
    r = gpu.Renderer(lights, tex, Lx, Ly, spp=4, bounces=2, seed=11)
    img = r.render(torch.from_numpy(hm).cuda(), oh, ow).cpu().numpy().reshape(-1, 3)
    pix = np.random.default_rng(1).choice(ow * oh, 48, replace=False)
    ref = oracle.render_pixels(pix, hm.astype(np.float64), Lx, Ly, lights, tex.astype(np.float32).astype(np.float64),
                               ow, oh, 4, seed=11, bounces=2)
    err = np.abs(img[pix] - ref).max(axis=-1)
    scale = ref.max()
    print(f"[render] {w}x{h} -> {ow}x{oh}: sampled max |diff| {err.max() / scale:.2e} of the max", flush=True)
    assert int((err <= 1e-4 * scale).sum()) >= len(pix) - 1
    assert err.max() <= 2.0 / 4 * scale


def test_render_flat_surface_and_degenerate_sizes(gpu, oracle):
    """A flat map (every ray below the map's range at once), the smallest map
    (2 x 2: one cell, one tile) and a one-pixel image."""
    import torch
    Lx = Ly = 4e-3
    lights = W.sensor_lights(Lx, Ly, 2e-3)
    tex = W.sensor_texture(4, 4)
    for hm, ow, oh in ((np.full((9, 9), 2e-3, np.float32), 9, 9), (np.full((2, 2), 2e-3, np.float32), 1, 1)):
        r = gpu.Renderer(lights, tex, Lx, Ly, spp=8, bounces=2, seed=3)
        img = r.render(torch.from_numpy(hm).cuda(), oh, ow).cpu().numpy()
        ref = oracle.render(hm.astype(np.float64), Lx, Ly, lights, tex.astype(np.float32).astype(np.float64), ow,
                            oh, 8, seed=3, bounces=2)
        assert np.allclose(img, ref, rtol=1e-4, atol=1e-6 * ref.max())


def test_full_size_sampled_pixels(gpu, oracle):
    """The benchmark's frame: a 640 x 480 height map of the 32 mm slab pressed
    1 mm, rendered at 640 x 480 with 128 samples and one interreflection, in the
    benchmark's launch configuration; 12 pixels (the dent's centre, its rim and
    the flat field) computed one by one by the oracle."""
    import torch
    Lx = Ly = 32e-3
    top = 8e-3
    hm = W.dented_heightmap(480, 640, Lx, Ly, top, depth=1.0e-3, radius=5e-3, seed=0).astype(np.float32)
    lights = W.sensor_lights(Lx, Ly, top)
    tex = W.sensor_texture(480, 640)
    r = gpu.Renderer(lights, tex, Lx, Ly, spp=128, bounces=2, seed=1)
    img = r.render(torch.from_numpy(hm).cuda()).cpu().numpy().reshape(-1, 3)
    rng = np.random.default_rng(5)
    cu, cv = 320, 240
    pix = [cv * 640 + cu, cv * 640 + cu + 90, (cv + 70) * 640 + cu, (cv - 93) * 640 + cu - 20, 0, 640 * 480 - 1]
    pix += list(rng.integers(0, 640 * 480, 6))
    ref = oracle.render_pixels(pix, hm.astype(np.float64), Lx, Ly, lights, tex.astype(np.float32).astype(np.float64),
                               640, 480, 128, seed=1, bounces=2)
    got = img[pix]
    scale = ref.max()
    err = np.abs(got - ref).max(axis=-1)
    print(f"[render] full size: sampled pixels max |diff| {err.max() / scale:.2e} of the max, "
          f"{int((err <= 1e-4 * scale).sum())} of {len(pix)} within 1e-4", flush=True)
    assert np.all(np.isfinite(img))
    assert int((err <= 1e-4 * scale).sum()) >= len(pix) - 1
    assert err.max() <= 2.0 / 128 * scale

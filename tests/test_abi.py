"""The C ABI library loads and exports every entry point include/impm.h,
include/sur.h and include/render.h declare (no device calls: runs without a
GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "impm.h")
SUR_HEADER = os.path.join(ROOT, "include", "sur.h")
RENDER_HEADER = os.path.join(ROOT, "include", "render.h")


def declared_functions(header=HEADER, prefix="sim"):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sim_create", "sim_set_indenter_pose", "sim_step", "sim_surface_heightmap"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2405_02914_amd import impm
    if not os.path.exists(impm.LIB_PATH):
        pytest.fail("libimpm.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(impm.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(impm.EXPORTS)


def test_library_exports_every_surrogate_symbol():
    from paper_2405_02914_amd import impm, sur
    lib = ctypes.CDLL(impm.LIB_PATH)
    names = declared_functions(SUR_HEADER, "sur")
    for n in ("sur_create", "sur_infer", "sur_train_step", "sur_save", "sur_load", "sur_destroy"):
        assert n in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) <= set(sur.EXPORTS)
    assert ctypes.sizeof(sur.sur_params) == 4 * 8 + 8 + 4 * 4


def test_binding_struct_layouts_match_header():
    """The ctypes records have the sizes the header's field lists imply."""
    from paper_2405_02914_amd import impm
    assert ctypes.sizeof(impm.sim_params) == 12 + 4 + 8 + 8 + 8 * 4 + 4 * 8 + 8 * 2 + 8 + 8 * 2 + 24 + 8 + 56 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(impm.sim_stats) == 8 * 5 + 8 + 56 + 24 + 8


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2405_02914_amd import impm
    monkeypatch.setattr(impm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(impm, "_lib", None)
    with pytest.raises(RuntimeError):
        impm.lib()


def test_library_exports_every_renderer_symbol():
    from paper_2405_02914_amd import impm, render
    lib = ctypes.CDLL(impm.LIB_PATH)
    names = declared_functions(RENDER_HEADER, "rt")
    assert names == ["rt_render", "rt_render_work", "rt_workspace_bytes"]
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) <= set(render.EXPORTS)
    assert ctypes.sizeof(render.rt_light) == 12 * 8
    assert ctypes.sizeof(render.rt_params) == 4 * 4 + 2 * 8 + 2 * 4 + 8 + 4 * 4


def test_renderer_host_validation():
    """Workspace size and argument checks run on the host before any device
    call (pointers here are never dereferenced: invalid calls return -1)."""
    from paper_2405_02914_amd import render as R
    p = R.rt_params(W=640, H=480, out_w=640, out_h=480, Lx=32e-3, Ly=32e-3, spp=128, bounces=2, seed=1,
                    n_lights=4, tex_w=64, tex_h=48)
    tw, th = (640 - 1 + 7) // 8, (480 - 1 + 7) // 8
    blocks = ((tw + 7) // 8) * ((th + 7) // 8)
    assert R.rt_workspace_bytes(p) == 256 + 8 * (tw * th + blocks)
    bad = [dict(W=1), dict(spp=0), dict(bounces=3), dict(n_lights=5), dict(n_lights=0), dict(Lx=0.0),
           dict(tex_w=0), dict(out_h=0)]
    L = R.lib()
    for kw in bad:
        q = R.rt_params(**{**{f: getattr(p, f) for f, _ in R.rt_params._fields_}, **kw})
        assert L.rt_workspace_bytes(ctypes.byref(q)) == 0, kw
        lights = R.light_records([dict(c=(0, 0, 0), e1=(1, 0, 0), e2=(0, 1, 0), L=(1, 1, 1))] * 4)
        fake = ctypes.c_void_p(1 << 20)
        assert L.rt_render(ctypes.byref(q), fake, lights, fake, fake, fake, 1 << 30, None) == -1, kw
    lights = R.light_records([dict(c=(0, 0, 0), e1=(1, 0, 0), e2=(0, 1, 0), L=(1, 1, 1))] * 4)
    fake = ctypes.c_void_p(1 << 20)
    # too small or misaligned workspace, null pointers, a degenerate light
    assert L.rt_render(ctypes.byref(p), fake, lights, fake, fake, fake, 255, None) == -1
    assert L.rt_render(ctypes.byref(p), fake, lights, fake, fake, ctypes.c_void_p((1 << 20) + 4), 1 << 30,
                       None) == -1
    assert L.rt_render(ctypes.byref(p), None, lights, fake, fake, fake, 1 << 30, None) == -1
    flat = R.light_records([dict(c=(0, 0, 0), e1=(1, 0, 0), e2=(2, 0, 0), L=(1, 1, 1))] * 4)
    assert L.rt_render(ctypes.byref(p), fake, flat, fake, fake, fake, 1 << 30, None) == -1


def test_sim_create_host_validation():
    """sim_create checks its parameters on the host before any device call:
    each invalid record returns SIM_EINVAL and no handle (runs without a GPU)."""
    import numpy as np
    from paper_2405_02914_amd import impm, workloads as W
    L = impm.lib()
    base = W.small_sensor(cells=(6, 6, 3))
    hf = W.heightfield_table(5, 2.0e-3, 0.3e-3, 1.5e-3, 4e-3)
    bad_hf = hf.copy()
    bad_hf[2, 2] = np.nan
    cases = [dict(cells=(0, 6, 3)), dict(ppc=5), dict(dx=0.0), dict(dt=-1e-5), dict(E=0.0), dict(rho=0.0),
             dict(nu=0.5), dict(nu=0.0), dict(subcycle=0), dict(rest_limit=0), dict(rest_limit=33),
             dict(rest_threshold=-1.0), dict(mode=7), dict(shape=9),
             dict(shape=W.SHAPE_HEIGHTFIELD, hf=bad_hf, hf_half=2.0e-3),
             dict(shape=W.SHAPE_HEIGHTFIELD, hf=hf, hf_half=0.0),
             dict(cells=(1100, 6, 3)),                         # more than 1023 nodes along x
             dict(cells=(1000, 1000, 300)),                    # 2.4e9 particles
             dict(pose0=(8e-3, 8e-3, 8e-3, 0.0, 0.0, 0.0, 0.0)),
             dict(columns=np.full((6, 6), 4, np.int32)),       # taller than cells[2]
             dict(columns=np.zeros((6, 6), np.int32)),         # no cell at all
             dict(object_mode=5), dict(object_mode=1, shape=W.SHAPE_NONE), dict(object_mode=1, object_density=0.0)]
    for kw in cases:
        rec = impm.to_params(base.replace(**kw))
        h = ctypes.c_void_p()
        rc = L.sim_create(ctypes.byref(rec), None, ctypes.byref(h))
        assert rc == impm.SIM_EINVAL and not h.value, kw
    h = ctypes.c_void_p()
    assert L.sim_create(None, None, ctypes.byref(h)) == impm.SIM_EINVAL

"""Pins of the oracle's object particles (Sec. III-A: the object and the
elastomer are both represented by particles; Algorithm 1 sets the object
particles' velocities to the prescribed motion before every exchange).

Fixed independently of the oracle's code: the lattice sampling by brute force
over a sphere, the rigid motion reproduced exactly by the transfer (the affine
term of a rigid body is [w]x, so the grid velocity of nodes reached by object
particles alone is the rigid velocity in closed form), momentum conservation,
rigid placement (the body's shape is kept), sticking during a slide, and the
heavy-object limit approaching the grid collider."""
import math

import numpy as np
import pytest

from paper_2405_02914_amd import workloads as W


@pytest.fixture(scope="module")
def ref(oracle_lib):
    return oracle_lib


def sphere_sensor(**kw):
    kw.setdefault("radius", 1.5e-3)
    return W.small_sensor(cells=(10, 10, 4), object_mode=1, object_cap=1.0e-3, **kw)


def test_object_particles_are_the_body_lattice(ref):
    """Sphere r: body lattice ((i+1/2)h, (j+1/2)h, -r + (k+1/2)h), h = dx/2,
    inside |p| <= r and at most object_cap above the lowest point."""
    p = sphere_sensor()
    o = ref.OracleSim(p)
    x, b = o.objects()
    h, r, cap = p.dx / 2, p.radius, p.object_cap
    pts = []
    n = int(math.ceil(r / h))
    for k in range(int(math.ceil(cap / h))):
        for j in range(-n, n):
            for i in range(-n, n):
                q = ((i + 0.5) * h, (j + 0.5) * h, -r + (k + 0.5) * h)
                if q[0] ** 2 + q[1] ** 2 + q[2] ** 2 <= r * r:
                    pts.append(q)
    pts = np.array(pts)
    assert b.shape == pts.shape and np.array_equal(b, pts)
    assert np.allclose(x, b + np.array(p.pose0[:3]), rtol=0, atol=1e-15)
    assert o.object_mass() == pytest.approx(p.object_density * p.dx ** 3 / p.ppc, rel=1e-15)
    # x_o: the lowest particle; ties to the farthest from the axis, then the smallest (x, y)
    low = pts[pts[:, 2] == pts[:, 2].min()]
    rr = low[:, 0] ** 2 + low[:, 1] ** 2
    far = low[rr == rr.max()]
    want = far[np.lexsort((far[:, 1], far[:, 0]))][0]
    assert np.allclose(o.xo(), want + np.array(p.pose0[:3]), rtol=0, atol=1e-15)


def test_rigid_motion_is_transferred_exactly(ref):
    """Object particles hovering 3 cells above the slab, moving with v_o and
    spinning about z: every node reached only by object particles gets
    V = v_o + w x (X - c) (the transfer of a rigid field is exact)."""
    p = sphere_sensor(pose0=(2.5e-3, 2.5e-3, 2.0e-3 + 3 * 0.5e-3 + 1.5e-3, 1, 0, 0, 0), pad=6)
    o = ref.OracleSim(p)
    el = ref.OracleSim(p.replace(object_mode=0, shape=W.SHAPE_NONE))
    move = np.array([0.7e-6, -0.4e-6, -0.3e-6])
    ang = 0.02
    tgt = tuple(np.array(p.pose0[:3]) + move)
    o.set_target_pose(tgt, W.quat_about_z(ang))
    o.p2g_with_object()
    o.grid_update(contact=False, bc=False)
    el.p2g()
    M, MG, V = o.grid()
    Mel = el.grid()[0]
    only = (M > 0) & (Mel == 0)
    assert only.sum() > 50
    nx, ny, nz = o.nodes
    idx = np.nonzero(only)[0]
    i, j, k = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    X = np.stack([(i - p.pad_lateral) * p.dx, (j - p.pad_lateral) * p.dx, (k - p.pad_bottom) * p.dx], 1)
    c = np.array(p.pose0[:3])
    vo = move / p.dt
    w = np.array([0.0, 0.0, math.radians(ang) / p.dt])
    want = vo + np.cross(w, X - c)
    assert np.abs(V[idx] - want).max() <= 1e-12 * np.abs(want).max()


def test_transfer_conserves_momentum_with_object_particles(ref):
    """Total grid momentum = elastomer momentum + object particles' momentum."""
    p = sphere_sensor()
    o = ref.OracleSim(p)
    X, _, _ = o.rest()
    x, v, Cm, G = W.random_state(p, X, 5)
    o.set_state(x=x, v=v, Cm=Cm, F=np.eye(3)[None] + G.astype(np.float64))
    tgt = (p.pose0[0] + 0.5e-6, p.pose0[1], p.pose0[2] - 1e-6)
    o.set_target_pose(tgt, W.quat_about_z(0.01))
    o.p2g_with_object()
    M, MG, _ = o.grid()
    xo, _ = o.objects()
    c = np.array(p.pose0[:3])
    vo = (np.array(tgt) - c) / p.dt
    w = np.array([0.0, 0.0, math.radians(0.01) / p.dt])
    vobj = vo + np.cross(w, xo - c)
    mp = p.rho * p.dx ** 3 / p.ppc
    want = mp * v.astype(np.float64).sum(0) + o.object_mass() * vobj.sum(0)
    assert np.abs(MG.sum(0) - want).max() <= 1e-12 * np.abs(want).max()
    assert M.sum() == pytest.approx(mp * len(x) + o.object_mass() * len(xo), rel=1e-13)


def test_object_particles_stay_rigid(ref):
    """After press, slide and rotation the object particles sit exactly at the
    body lattice under the current pose."""
    p = sphere_sensor(subcycle=2)
    o = ref.OracleSim(p)
    _, b = o.objects()
    c = np.array(p.pose0[:3])
    segs = [(20, tuple(c + [0, 0, -0.3e-3]), (1, 0, 0, 0)), (20, tuple(c + [0.2e-3, 0.1e-3, -0.3e-3]), W.quat_about_z(15))]
    o.run_schedule(segs)
    x, _ = o.objects()
    pose = o.pose()
    q = pose[3:]
    wq, xq, yq, zq = q
    R = np.array([[1 - 2 * (yq * yq + zq * zq), 2 * (xq * yq - wq * zq), 2 * (xq * zq + wq * yq)],
                  [2 * (xq * yq + wq * zq), 1 - 2 * (xq * xq + zq * zq), 2 * (yq * zq - wq * xq)],
                  [2 * (xq * zq - wq * yq), 2 * (yq * zq + wq * xq), 1 - 2 * (xq * xq + yq * yq)]])
    assert np.abs(x - (pose[:3] + b @ R.T)).max() <= 1e-15


def test_sticking_slide_with_object_particles(ref):
    """Pressed 0.3 mm, then slid 0.2 mm: the elastomer calibration particle x_e
    follows the object's bottom particle x_o (sticking contact through the
    shared grid), well beyond what the slab does far away."""
    p = W.small_sensor(cells=(12, 12, 4), radius=1.5e-3, subcycle=2, object_mode=1, object_cap=1.0e-3)
    o = ref.OracleSim(p)
    c = np.array(p.pose0[:3])
    X0 = o.rest()[0]
    e = o.calib_particle
    o.run_schedule([(10, tuple(c + [0, 0, -0.3e-3]), (1, 0, 0, 0))])
    xe0, xo0 = o.state()[0][e].copy(), o.xo()
    o.run_schedule([(20, tuple(c + [0.2e-3, 0, -0.3e-3]), (1, 0, 0, 0))])
    x = o.state()[0]
    de = x[e] - xe0
    dxo = o.xo() - xo0
    far = np.argmin(np.abs(X0[:, 0] - 0.5e-3) + np.abs(X0[:, 1] - 0.5e-3) + np.abs(X0[:, 2] - 1.75e-3))
    print("x_e moved", de, "x_o moved", dxo, "far particle", x[far] - X0[far])
    assert dxo[0] == pytest.approx(0.2e-3, rel=1e-9)
    assert de[0] > 0.5 * dxo[0]
    assert abs(x[far, 0] - X0[far, 0]) < 0.3 * de[0]
    assert o.counters()["passes"] > o.counters()["steps"]      # the loop iterates during the slide


def test_heavy_object_approaches_the_collider(ref):
    """With object particles 10^4 times denser than the elastomer, a press gives
    nearly the surface the grid collider gives (the collider is the limit of
    object particles that dominate the node mass)."""
    base = W.small_sensor(cells=(12, 12, 4), radius=1.5e-3, subcycle=2)
    c = np.array(base.pose0[:3])
    seg = [(20, tuple(c + [0, 0, -0.4e-3]), (1, 0, 0, 0))]
    hs = {}
    for name, q in (("collider", base), ("heavy", base.replace(object_mode=1, object_density=1e7)),
                    ("equal", base.replace(object_mode=1, object_density=1e3))):
        o = ref.OracleSim(q)
        o.run_schedule(seg)
        hs[name] = o.surface_heightmap(24, 24)
    top = base.height
    dc, dh, de = top - hs["collider"].min(), top - hs["heavy"].min(), top - hs["equal"].min()
    print("indentation collider", dc, "heavy", dh, "equal density", de)
    assert dc > 0.2e-3 and dh > 0.2e-3
    assert abs(dh - dc) < 0.5 * base.dx
    assert np.abs(hs["heavy"] - hs["collider"]).max() < base.dx

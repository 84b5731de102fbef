"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage of arXiv 2405.02914 (Sec. III-A, Eq. 1-9 and
Algorithm 1) it pins and the independent fact it uses: closed forms, published
test vectors, library routines (SVD), brute force over all node/particle pairs,
and conservation laws of the transfers.
"""
import math
import os

import numpy as np
import pytest

from paper_2405_02914_amd import workloads as W
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ref(oracle_lib):
    return oracle_lib


def tiny(cells=(2, 2, 2), ppc=8, **kw):
    kw.setdefault("shape", W.SHAPE_NONE)
    return W.small_sensor(cells=cells, ppc=ppc, pad=4, **kw)


def random_tiny_state(ref, p, seed=7, g_scale=0.05):
    s = ref.OracleSim(p)
    X, _, _ = s.rest()
    x, v, Cm, G = W.random_state(p, X, seed, g_scale=g_scale, x_scale=0.3)
    F = np.eye(3)[None] + G.astype(np.float64)
    s.set_state(x=x, v=v, Cm=Cm, F=F)
    return s, x, v.astype(np.float64), Cm.astype(np.float64), F


# ---------------------------------------------------------------- generator

def test_splitmix64_published_vectors(ref):
    """SplitMix64 (Steele, Lea, Flood 2014): the first outputs for seed 0 and for
    seed 1234567 as printed with the generator's public reference code."""
    assert [ref.splitmix64_at(0, t) for t in (1, 2, 3, 4)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert ref.splitmix64_at(1234567, 1) == 6457827717110365317
    assert ref.splitmix64_at(1234567, 2) == 3203168211198807973


def test_init_stratified_and_fp32(ref):
    """8 particles per cell, one per 2x2x2 sub-cell, offsets FP32-representable."""
    p = W.small_sensor(cells=(4, 3, 2), shape=W.SHAPE_NONE)
    s = ref.OracleSim(p)
    X, bottom, surface = s.rest()
    assert s.n == 4 * 3 * 2 * 8
    g = X / p.dx
    cell = np.floor(g)
    off = g - cell
    # offsets are FP32 values (up to the FP64 rounding of (cell + r) * dx / dx)
    assert np.allclose(off, off.astype(np.float32), rtol=0, atol=1e-12)
    ids = np.arange(s.n)
    c = ids // 8
    sub = ids % 8
    ci = np.stack([c % 4, (c // 4) % 3, c // 12], 1)
    si = np.stack([sub % 2, (sub // 2) % 2, sub // 4], 1)
    assert np.array_equal(cell.astype(int), ci)
    assert np.all((off >= si * 0.5 - 1e-12) & (off < si * 0.5 + 0.5 + 1e-12))
    # surface = top sub-layer of the top cell layer; bottom = lower half by rest height
    assert surface.sum() == 4 * 3 * 4
    assert np.array_equal(bottom, X[:, 2] < 0.5 * p.height)


# ---------------------------------------------------------------- Eq. (1): weights

def _read_golden():
    rows = []
    for line in open(os.path.join(GOLDEN, "single_particle_masses.txt")):
        if line.startswith("#") or not line.strip():
            continue
        case, kind, count, frac = line.split()
        rows.append((case, kind, int(count), float(frac)))
    return rows


@pytest.mark.parametrize("case", ["on_node", "cell_centre"])
def test_single_particle_node_masses(ref, case):
    """Eq. (1) with one particle: node masses equal the hand-derived products of
    the quadratic B-spline's 1-D weights (golden fixture)."""
    p = tiny(cells=(1, 1, 1), ppc=1)
    s = ref.OracleSim(p)
    mp = p.rho * p.dx ** 3
    x = np.array([[0.0, 0.0, 0.0]]) if case == "on_node" else np.array([[0.5, 0.5, 0.5]]) * p.dx
    if case == "on_node":
        x = x + p.dx            # node (1,1,1) of the slab, still inside the padded grid
    s.set_state(x=x, v=np.zeros((1, 3)), Cm=np.zeros((1, 3, 3)), F=np.eye(3)[None])
    s.p2g()
    M, _, _ = s.grid()
    got = np.sort(M[M > 0] / mp)[::-1]
    want = []
    for c, kind, count, frac in _read_golden():
        if c == case:
            want += [frac] * count
    want = np.sort(np.array(want))[::-1]
    assert got.shape == want.shape
    assert np.allclose(got, want, rtol=1e-14, atol=0)


# ---------------------------------------------------------------- Eq. (4): stress

def _lame(p):
    return p.E / (2 * (1 + p.nu)), p.E * p.nu / ((1 + p.nu) * (1 - 2 * p.nu))


def test_kirchhoff_uniaxial_closed_form(ref):
    """S_p of Eq. (4), fixed-corotated: for F = diag(1+e, 1, 1) the rotation is I
    and tau = 2 mu diag(e(1+e), 0, 0) + lam e (1+e) I."""
    mu, lam = _lame(W.config1())
    for e in (-0.2, -1e-3, 1e-6, 0.05, 0.3):
        F = np.diag([1 + e, 1.0, 1.0])
        want = 2 * mu * np.diag([e * (1 + e), 0, 0]) + lam * e * (1 + e) * np.eye(3)
        got = ref.kirchhoff(F, mu, lam)
        assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * mu)


def test_kirchhoff_rest_zero_and_objective(ref):
    mu, lam = _lame(W.config1())
    assert np.array_equal(ref.kirchhoff(np.eye(3), mu, lam), np.zeros((3, 3)))
    rng = np.random.default_rng(3)
    for _ in range(20):
        F = np.eye(3) + rng.normal(0, 0.2, (3, 3))
        if np.linalg.det(F) <= 0.1:
            continue
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        if np.linalg.det(Q) < 0:
            Q[:, 0] *= -1
        t = ref.kirchhoff(F, mu, lam)
        assert np.allclose(t, t.T, atol=1e-9 * mu)                     # symmetric
        assert np.allclose(ref.kirchhoff(Q @ F, mu, lam), Q @ t @ Q.T, atol=1e-9 * mu)  # objective
        assert np.allclose(t, brute.kirchhoff_svd(F, mu, lam), atol=1e-9 * mu)


def test_polar_matches_svd(ref):
    """Rotation factor of F = R S equals U V^T from the SVD (library routine)."""
    rng = np.random.default_rng(11)
    for _ in range(50):
        F = np.eye(3) + rng.normal(0, 0.4, (3, 3))
        if np.linalg.det(F) <= 0.05:
            continue
        R = ref.polar(F)
        assert np.allclose(R, brute.polar_svd(F), atol=1e-12)
        assert abs(np.linalg.det(R) - 1) < 1e-12


# ---------------------------------------------------------------- transfers vs brute force

def test_p2g_matches_brute_force(ref):
    """Eq. (1)-(4) on a tiny grid against all-pairs brute force."""
    p = tiny()
    s, x, v, Cm, F = random_tiny_state(ref, p)
    s.p2g()
    M, MG, _ = s.grid()
    Mb, MGb = brute.p2g(p, x, v, Cm, F, p.dt)
    assert np.allclose(M, Mb, rtol=0, atol=1e-14 * Mb.max())
    assert np.allclose(MG, MGb, rtol=0, atol=1e-12 * np.abs(MGb).max())


def test_p2g_momentum_only_matches_brute_force(ref):
    p = tiny()
    s, x, v, Cm, F = random_tiny_state(ref, p)
    s.p2g_momentum()
    M, MG, _ = s.grid()
    Mb, MGb = brute.p2g(p, x, v, Cm, F, p.dt, with_stress=False)
    assert np.allclose(MG, MGb, rtol=0, atol=1e-12 * np.abs(MGb).max())


def test_g2p_matches_brute_force(ref):
    """Eq. (6)-(7) on a tiny grid against all-pairs brute force."""
    p = tiny()
    s, x, v, Cm, F = random_tiny_state(ref, p)
    s.p2g()
    s.grid_update(contact=False, bc=False)
    _, _, V = s.grid()
    s.g2p(False)
    _, v1, C1, _ = s.state()
    vb, Cb = brute.g2p(p, x, V)
    assert np.allclose(v1, vb, rtol=0, atol=1e-12 * np.abs(vb).max())
    assert np.allclose(C1, Cb, rtol=0, atol=1e-12 * np.abs(Cb).max())


# ---------------------------------------------------------------- conservation

def _ang(p, x, v, Cm, mp):
    """Angular momentum of APIC particles: sum m (x x v + (W^2/4) eps_kab C_ba)."""
    D = p.dx ** 2 / 4
    skew = np.stack([Cm[:, 2, 1] - Cm[:, 1, 2], Cm[:, 0, 2] - Cm[:, 2, 0], Cm[:, 1, 0] - Cm[:, 0, 1]], 1)
    return mp * (np.cross(x, v) + D * skew).sum(0)


def test_p2g_g2p_conservation(ref):
    """P2G conserves mass, linear and angular momentum (the stress impulse has zero
    sum and zero moment because tau is symmetric and sum_i w (X_i - x_p) = 0);
    G2P conserves the grid's linear and angular momentum."""
    p = tiny(cells=(3, 3, 2))
    s, x, v, Cm, F = random_tiny_state(ref, p, seed=5)
    mp = p.rho * p.dx ** 3 / p.ppc
    X = brute.node_positions(p)
    s.p2g()
    M, MG, _ = s.grid()
    assert math.isclose(M.sum(), mp * s.n, rel_tol=1e-13)
    P0 = mp * v.sum(0)
    scale = mp * s.n * np.abs(v).max()
    assert np.allclose(MG.sum(0), P0, atol=1e-12 * scale)
    L0 = _ang(p, x, v, Cm, mp)
    assert np.allclose(np.cross(X, MG).sum(0), L0, atol=1e-12 * scale * p.dx * 10)
    s.grid_update(contact=False, bc=False)
    _, _, V = s.grid()
    s.g2p(False)
    _, v1, C1, _ = s.state()
    assert np.allclose(mp * v1.sum(0), (M[:, None] * V).sum(0), atol=1e-12 * scale)
    assert np.allclose(_ang(p, x, v1, C1, mp), np.cross(X, M[:, None] * V).sum(0),
                       atol=1e-12 * scale * p.dx * 10)


@pytest.mark.parametrize("kind", ["uniform", "rotation", "affine"])
def test_affine_field_reproduced(ref, kind):
    """APIC reproduces affine velocity fields exactly: v = b + A x with C = A
    survives P2G -> G2P unchanged (F = I, no boundary, no contact)."""
    p = tiny(cells=(3, 3, 3))
    s = ref.OracleSim(p)
    X, _, _ = s.rest()
    b = np.array([0.1, -0.05, 0.02])
    A = {"uniform": np.zeros((3, 3)),
         "rotation": np.array([[0, -30.0, 10.0], [30.0, 0, -5.0], [-10.0, 5.0, 0]]),
         "affine": np.array([[5.0, 2.0, -1.0], [0.5, -3.0, 4.0], [1.0, 1.5, 2.0]])}[kind]
    v = b + X @ A.T
    Cm = np.tile(A, (s.n, 1, 1))
    s.set_state(v=v, Cm=Cm)
    s.p2g()
    s.grid_update(contact=False, bc=False)
    s.g2p(False)
    _, v1, C1, _ = s.state()
    assert np.allclose(v1, v, rtol=0, atol=1e-13)
    assert np.allclose(C1, Cm, rtol=0, atol=1e-10)


def test_uniform_translation_one_substep(ref):
    """Uniform velocity u, C = 0, F = I away from all boundaries and with no
    indenter: after a substep v = u, C = 0, F = I and x += u dt (Eq. 9)."""
    p = tiny(cells=(3, 3, 2), mode=W.MODE_PLAIN)
    s = ref.OracleSim(p)
    X, _, _ = s.rest()
    u = np.array([0.2, -0.1, 0.05])
    s.set_state(v=np.tile(u, (s.n, 1)))
    s.p2g(); s.grid_update(contact=False, bc=False); s.g2p(False); s.commit()
    x1, v1, C1, F1 = s.state()
    assert np.allclose(v1, u, atol=1e-14)
    assert np.abs(C1).max() < 1e-9
    assert np.allclose(F1, np.eye(3), atol=1e-13)
    assert np.allclose(x1, X + u * p.dt, atol=1e-18)


# ---------------------------------------------------------------- whole substeps

def test_rest_is_bitwise_preserved(ref):
    """An unloaded slab (no indenter, v = 0, C = 0, F = I) stays exactly at rest:
    no body force, tau(I) = 0 (Sec. III-A has no gravity)."""
    p = W.small_sensor(cells=(6, 5, 3), shape=W.SHAPE_NONE, subcycle=2)
    s = ref.OracleSim(p)
    x0, v0, C0, F0 = s.state()
    s.step(50)
    x1, v1, C1, F1 = s.state()
    assert np.array_equal(x0, x1) and np.array_equal(F0, F1)
    assert not v1.any() and not C1.any()


def test_integer_cell_translation_invariance(ref):
    """Shifting the slab and the indenter by whole cells (more padding on one
    side) leaves the trajectory unchanged up to rounding."""
    base = W.small_sensor(cells=(6, 6, 3), radius=1.2e-3, subcycle=2)
    a = ref.OracleSim(base)
    a.set_target_pose((base.pose0[0] + 0.2e-3, base.pose0[1], base.pose0[2] - 0.4e-3), (1, 0, 0, 0))
    a.step(10)
    xa, va, Ca, Fa = a.state()
    # the same physical problem on a grid with 2 more lateral padding cells
    shifted = base.replace(pad_lateral=base.pad_lateral + 2)
    b = ref.OracleSim(shifted)
    b.set_target_pose((base.pose0[0] + 0.2e-3, base.pose0[1], base.pose0[2] - 0.4e-3), (1, 0, 0, 0))
    b.step(10)
    xb, vb, Cb, Fb = b.state()
    assert np.allclose(xa, xb, rtol=0, atol=1e-15)
    assert np.allclose(va, vb, rtol=0, atol=1e-12 * np.abs(va).max())
    assert np.allclose(Fa, Fb, rtol=0, atol=1e-12)


def test_subcycle_equals_smaller_dt(ref):
    """One configured substep with subcycle k is k steps of dt/k."""
    p = W.small_sensor(cells=(5, 5, 3), radius=1.2e-3)
    a = ref.OracleSim(p.replace(subcycle=2))
    b = ref.OracleSim(p.replace(subcycle=1, dt=p.dt / 2))
    tgt = (p.pose0[0], p.pose0[1], p.pose0[2] - 0.3e-3)
    for s, n in ((a, 5), (b, 10)):
        s.set_target_pose(tgt, (1, 0, 0, 0))
        s.step(n)
    for u, w in zip(a.state(), b.state()):
        assert np.allclose(u, w, rtol=0, atol=1e-12 * max(1e-30, np.abs(u).max()))


def test_plain_equals_impm_with_limit_one(ref):
    """The paper's "normal" MPM (one exchange, no bottom rule) equals IMPM with
    LIMIT = 1 and an empty bottom layer, under slip so that IMPM would iterate."""
    p = W.small_sensor(cells=(6, 6, 3), radius=1.2e-3, subcycle=2)
    tgt = ((p.pose0[0] + 0.3e-3, p.pose0[1], p.pose0[2] - 0.4e-3), W.quat_about_z(10))
    a = ref.OracleSim(p.replace(mode=W.MODE_PLAIN))
    b = ref.OracleSim(p.replace(rest_limit=1, fixed_z_fraction=0.0))
    for s in (a, b):
        s.set_target_pose(*tgt)
        s.step(8)
    for u, w in zip(a.state(), b.state()):
        assert np.array_equal(u, w)
    assert a.counters()["passes"] == 16


def test_pure_press_is_single_pass(ref):
    """Algorithm 1's test has nothing to align under a pure press (no tangential
    object velocity at x_o): every step does exactly one exchange."""
    p = W.small_sensor(cells=(6, 6, 3), radius=1.2e-3, subcycle=2)
    s = ref.OracleSim(p)
    s.set_target_pose((p.pose0[0], p.pose0[1], p.pose0[2] - 0.4e-3), (1, 0, 0, 0))
    s.step(10)
    c = s.counters()
    assert c["steps"] == 20 and c["passes"] == 20 and c["limit_hits"] == 0


def test_bottom_layer_z_is_fixed(ref):
    """IMPM zeroes the z velocity of the lower half layer (the bottom is glued to
    the sensor), so those particles keep their z exactly, even under slip."""
    p = W.small_sensor(cells=(6, 6, 4), radius=1.2e-3, subcycle=2)
    s = ref.OracleSim(p)
    X, bottom, _ = s.rest()
    s.set_target_pose((p.pose0[0] + 0.3e-3, p.pose0[1], p.pose0[2] - 0.5e-3), W.quat_about_z(10))
    s.step(10)
    x, v, _, _ = s.state()
    assert bottom.any()
    assert np.array_equal(x[bottom, 2], X[bottom, 2])
    assert not v[bottom, 2].any()


def test_forced_pass_schedule(ref):
    p = W.small_sensor(cells=(5, 5, 3), radius=1.2e-3)
    s = ref.OracleSim(p)
    s.enable_pass_log(100)
    s.force_passes([3, 1, 2])
    s.set_target_pose((p.pose0[0] + 0.2e-3, p.pose0[1], p.pose0[2] - 0.2e-3), (1, 0, 0, 0))
    s.step(3)
    assert list(s.pass_log()) == [3, 1, 2]
    assert s.counters()["passes"] == 6


def test_energy_does_not_grow(ref):
    """Explicit stability at the configured sub-cycling (CFL 0.67): a strained,
    moving slab loses energy but never gains it (kinetic + elastic)."""
    for dx, k in ((0.5e-3, 2), (0.25e-3, 4)):
        p = W.small_sensor(cells=(6, 6, 3), dx=dx, shape=W.SHAPE_NONE, subcycle=k)
        s = ref.OracleSim(p)
        X, _, _ = s.rest()
        F = np.tile(np.eye(3), (s.n, 1, 1)); F[:, 2, 2] = 0.99; F[:, 0, 0] = 1.005
        v = np.zeros((s.n, 3)); v[:, 0] = 0.05 * np.sin(np.pi * X[:, 1] / (6 * dx))
        s.set_state(v=v, F=F)
        e = [s.energy()]
        for _ in range(20):
            s.step(10)
            e.append(s.energy())
        assert all(b <= a * (1 + 1e-9) for a, b in zip(e, e[1:])), e


def test_energy_is_the_stress_potential(ref):
    """The energy the stability test watches is the one whose derivative is the
    stress the method uses: for a slab at rest with one uniform F, the central
    difference of the total energy in F_ab equals n V_p P_ab, with the first
    Piola stress P = tau F^-T from the Kirchhoff stress; and with v = 0 and
    F = I it is zero, with F = I and a uniform v it is the kinetic energy."""
    p = W.small_sensor(cells=(3, 3, 2), shape=W.SHAPE_NONE)
    s = ref.OracleSim(p)
    n = s.n
    Vp = p.dx ** 3 / p.ppc
    mp = p.rho * Vp
    mu, lam = p.E / (2 * (1 + p.nu)), p.E * p.nu / ((1 + p.nu) * (1 - 2 * p.nu))
    s.set_state(v=np.zeros((n, 3)), F=np.tile(np.eye(3), (n, 1, 1)))
    assert s.energy() == 0.0
    s.set_state(v=np.tile([0.3, -0.2, 0.1], (n, 1)))
    assert np.isclose(s.energy(), 0.5 * n * mp * 0.14, rtol=1e-14)
    s.set_state(v=np.zeros((n, 3)))
    rng = np.random.default_rng(8)
    F0 = np.eye(3) + 0.08 * rng.normal(size=(3, 3))
    Pk = ref.kirchhoff(F0, mu, lam) @ np.linalg.inv(F0).T
    eps = 1e-6
    for a in range(3):
        for b in range(3):
            E = []
            for sgn in (1, -1):
                F = F0.copy()
                F[a, b] += sgn * eps
                s.set_state(F=np.tile(F, (n, 1, 1)))
                E.append(s.energy())
            dE = (E[0] - E[1]) / (2 * eps)
            assert np.isclose(dE, n * Vp * Pk[a, b], rtol=1e-6, atol=1e-9 * p.E * n * Vp), (a, b)


def test_stability_limit_bites_without_subcycling(ref):
    """The same slab at the configured dt without sub-cycling (CFL 1.35) fails,
    which is why the sub-cycle factor exists."""
    p = W.small_sensor(cells=(6, 6, 3), shape=W.SHAPE_NONE, subcycle=1)
    s = ref.OracleSim(p)
    F = np.tile(np.eye(3), (s.n, 1, 1)); F[:, 2, 2] = 0.99
    s.set_state(F=F)
    with pytest.raises(FloatingPointError):
        s.step(200)


# ---------------------------------------------------------------- contact and pose

def test_inside_mask_sphere_closed_form(ref):
    """Nodes inside the sphere are exactly those within r of its centre."""
    p = W.small_sensor(cells=(8, 8, 4), radius=1.3e-3)
    s = ref.OracleSim(p)
    X = brute.node_positions(p)
    c = np.array(p.pose0[:3])
    want = ((X - c) ** 2).sum(1) <= p.radius ** 2
    assert np.array_equal(s.inside_mask(), want)


def test_inside_mask_capsule_rotated(ref):
    """A capsule rod (axis = body x) rotated 90 degrees about z lies along world y."""
    p = W.small_sensor(cells=(8, 8, 4), shape=W.SHAPE_CAPSULE, radius=0.8e-3)
    p = p.replace(half_length=1.2e-3)
    s = ref.OracleSim(p)
    s.set_target_pose(p.pose0[:3], W.quat_about_z(90))
    s.step(1)
    X = brute.node_positions(p)
    c = np.array(p.pose0[:3])
    d = X - c
    t = np.clip(d[:, 1], -p.half_length, p.half_length)
    want = d[:, 0] ** 2 + (d[:, 1] - t) ** 2 + d[:, 2] ** 2 <= p.radius ** 2
    got = s.inside_mask()
    # nodes within rounding of the surface may go either way
    near = np.abs(np.sqrt(d[:, 0] ** 2 + (d[:, 1] - t) ** 2 + d[:, 2] ** 2) - p.radius) < 1e-12
    assert np.array_equal(got[~near], want[~near])


def _hf_sensor(tab, half, z_lift=0.0):
    p = W.small_sensor(cells=(10, 10, 4))
    L = 10 * p.dx
    return p.replace(shape=W.SHAPE_HEIGHTFIELD, hf=tab, hf_half=half,
                     pose0=(L / 2, L / 2, p.height + z_lift, 1.0, 0.0, 0.0, 0.0))


def test_inside_mask_heightfield_plane_rotated(ref):
    """A height field sampled from a plane is that plane under bilinear
    interpolation: rotated 30 degrees about z, the nodes inside are those over
    the footprint disc and above the tilted plane (body frame)."""
    half, n = 2.1e-3, 9
    a, b, c = 0.31, -0.17, -0.9e-3
    t = np.linspace(-half, half, n)
    X_, Y_ = np.meshgrid(t, t, indexing="xy")
    p = _hf_sensor(a * X_ + b * Y_ + c, half)
    s = ref.OracleSim(p)
    q = W.quat_about_z(30)
    s.set_target_pose(p.pose0[:3], q)
    s.step(1)
    th = np.radians(30)
    Rz = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    d = brute.node_positions(p) - np.array(p.pose0[:3])
    pb = d @ Rz                       # body coordinates: R^T d for each row
    r2 = pb[:, 0] ** 2 + pb[:, 1] ** 2
    phi = a * pb[:, 0] + b * pb[:, 1] + c - pb[:, 2]
    want = (r2 <= half * half) & (phi <= 0)
    near = (np.abs(phi) < 1e-12) | (np.abs(np.sqrt(r2) - half) < 1e-12)
    got = s.inside_mask()
    assert want.sum() > 50
    assert np.array_equal(got[~near], want[~near])


def test_heightfield_calibration_point(ref):
    """x_o of a height field is its lowest sample inside the footprint disc: a
    unique off-centre minimum is found, and for a flat table the tie goes to the
    samples farthest from the axis, then the smallest x, then the smallest y."""
    half, n = 2.0e-3, 9
    t = np.linspace(-half, half, n)
    X_, Y_ = np.meshgrid(t, t, indexing="xy")
    tab = (X_ - t[5]) ** 2 + (Y_ - t[2]) ** 2 + 1e-4
    tab[0, 0] = -1.0                  # outside the disc: ignored
    p = _hf_sensor(tab, half)
    s = ref.OracleSim(p)
    assert np.allclose(s.xo(), np.array(p.pose0[:3]) + [t[5], t[2], 1e-4], atol=1e-15)
    flat = np.full((n, n), 3e-4)
    p = _hf_sensor(flat, half)
    s = ref.OracleSim(p)
    assert np.array_equal(s.xo(), np.array(p.pose0[:3]) + [-half, 0.0, 3e-4])


def test_pose_reaches_target_and_xo_tracks(ref):
    p = W.small_sensor(cells=(6, 6, 3), radius=1.2e-3)
    s = ref.OracleSim(p)
    xo0 = s.xo()
    tgt = (p.pose0[0] + 0.3e-3, p.pose0[1] - 0.1e-3, p.pose0[2] - 0.2e-3)
    s.set_target_pose(tgt, (1, 0, 0, 0))
    s.step(4)
    assert np.allclose(s.pose()[:3], tgt, atol=1e-18)
    assert np.allclose(s.xo() - xo0, np.array(tgt) - np.array(p.pose0[:3]), atol=1e-15)


def test_sticking_contact_drags_surface(ref):
    """Relative rest (Sec. III-A, relative rest check): under slip the elastomer
    point nearest the indenter's lowest point follows it tangentially."""
    p = W.small_sensor(cells=(10, 10, 4), radius=1.5e-3, subcycle=2)
    s = ref.OracleSim(p)
    e = s.calib_particle
    x0, _, _, _ = s.state()
    c = np.array(p.pose0[:3])
    s.set_target_pose(c + [0, 0, -0.4e-3], (1, 0, 0, 0)); s.step(20)
    xa, _, _, _ = s.state()
    s.set_target_pose(c + [0.4e-3, 0, -0.4e-3], (1, 0, 0, 0)); s.step(40)
    xb, _, _, _ = s.state()
    moved = xb[e, 0] - xa[e, 0]
    assert 0.5 * 0.4e-3 < moved < 1.1 * 0.4e-3


def test_hertz_contact_radius_sanity(ref):
    """Loose textbook check: a sphere pressed d into the slab touches it over a
    radius of order sqrt(R d) (Hertz), within a couple of cells."""
    p = W.small_sensor(cells=(16, 16, 6), radius=3.0e-3, subcycle=2)
    s = ref.OracleSim(p)
    d = 0.5e-3
    s.set_target_pose((p.pose0[0], p.pose0[1], p.pose0[2] - d), (1, 0, 0, 0))
    s.step(40)
    s.set_target_pose((p.pose0[0], p.pose0[1], p.pose0[2] - d), (1, 0, 0, 0))
    s.step(40)
    hm = s.surface_heightmap(32, 32)
    L = p.lengths[0]
    u = (np.arange(32) + 0.5) * L / 32
    dep = (p.height - hm) > 0.1 * d
    r_pix = np.sqrt(((u[None, :] - L / 2) ** 2 + (u[:, None] - L / 2) ** 2))[dep]
    a = r_pix.max()
    hertz = math.sqrt(p.radius * d)
    assert abs(a - hertz) < 2.5 * p.dx, (a, hertz)


# ---------------------------------------------------------------- surface maps

def test_heightmap_rest_is_exact(ref):
    p = W.small_sensor(cells=(8, 6, 3), shape=W.SHAPE_NONE)
    s = ref.OracleSim(p)
    hm = s.surface_heightmap(16, 12)
    assert np.array_equal(hm, np.full((12, 16), p.height))


def test_displacement_uniform_shift_reproduced(ref):
    """Shepard-normalised interpolation reproduces a uniform displacement."""
    p = W.small_sensor(cells=(8, 6, 3), shape=W.SHAPE_NONE)
    s = ref.OracleSim(p)
    X, _, _ = s.rest()
    u = np.array([1e-5, -2e-5, -3e-5])
    s.set_state(x=X + u)
    d = s.surface_displacement(16, 12)
    assert np.allclose(d, u, rtol=0, atol=1e-17)


def test_displacement_brute_force_pixels(ref):
    """Surface displacement at pixel centres by brute force over surface
    particles; the pixel pitches differ along x and y (0.5 dx and 5/7 dx)."""
    p = W.small_sensor(cells=(6, 5, 3), shape=W.SHAPE_NONE)
    s = ref.OracleSim(p)
    X, _, surf = s.rest()
    rng = np.random.default_rng(4)
    x = X + rng.normal(0, 0.1 * p.dx, X.shape)
    s.set_state(x=x)
    Wd, Hd = 12, 7
    got = s.surface_displacement(Wd, Hd)
    px, py = p.lengths[0] / Wd, p.lengths[1] / Hd
    assert abs(px - py) > 0.1 * p.dx
    xs, Xs = x[surf], X[surf]
    for (v, u) in [(0, 0), (3, 7), (6, 11), (5, 5), (2, 1)]:
        cx, cy = (u + 0.5) * px, (v + 0.5) * py
        w = brute.N((xs[:, 0] - cx) / px) * brute.N((xs[:, 1] - cy) / py)
        want = (w[:, None] * (xs - Xs)).sum(0) / w.sum()
        assert np.allclose(got[v, u], want, rtol=1e-12, atol=1e-20)


def test_deformation_gradient_maps_line_elements(ref):
    """Eq. (8)-(9) are the kinematics of one body: after two affine velocity
    steps with non-commuting gradients L1, L2 the particles' relative positions
    obey x_p - x_q = F (X_p - X_q), which fixes the order (I + dt C) F."""
    p = tiny(cells=(3, 3, 3))
    s = ref.OracleSim(p)
    X, _, _ = s.rest()
    h = 2e-4
    L1 = np.array([[0.0, 40.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    L2 = np.array([[0.0, 0.0, 0.0], [30.0, 0.0, 0.0], [0.0, 0.0, -20.0]])
    for L in (L1, L2):
        x, _, _, _ = s.state()
        s.set_state(v=x @ L.T, Cm=np.tile(L, (s.n, 1, 1)))
        s.p2g_momentum(); s.grid_update(contact=False, bc=False); s.g2p(False); s.commit(h)
    x, _, _, F = s.state()
    assert not np.allclose(L1 @ L2, L2 @ L1)
    for p_, q_ in ((0, 5), (3, 40), (17, 99)):
        assert np.allclose(x[p_] - x[q_], F[p_] @ (X[p_] - X[q_]), rtol=0, atol=1e-15)


def test_rotation_sense_of_sticking_contact(ref):
    """A positive rotation about the normal (right-handed, z up) drags the
    contact patch counter-clockwise: at +x of the axis the surface moves +y."""
    p = W.small_sensor(cells=(12, 12, 4), shape=W.SHAPE_CAPSULE, radius=0.8e-3, subcycle=2)
    p = p.replace(half_length=1.5e-3, pose0=(p.pose0[0], p.pose0[1], p.height + 0.8e-3, 1, 0, 0, 0))
    s = ref.OracleSim(p)
    c = np.array(p.pose0[:3])
    s.set_target_pose(c + [0, 0, -0.3e-3], (1, 0, 0, 0)); s.step(20)
    xa, _, _, _ = s.state()
    s.set_target_pose(c + [0, 0, -0.3e-3], W.quat_about_z(20)); s.step(40)
    xb, _, _, _ = s.state()
    X, _, surf = s.rest()
    d = xb - xa
    right = surf & (np.abs(X[:, 0] - c[0] - 1.2e-3) < 0.3e-3) & (np.abs(X[:, 1] - c[1]) < 0.3e-3)
    left = surf & (np.abs(X[:, 0] - c[0] + 1.2e-3) < 0.3e-3) & (np.abs(X[:, 1] - c[1]) < 0.3e-3)
    assert right.any() and left.any()
    assert d[right, 1].mean() > 1e-5 and d[left, 1].mean() < -1e-5


def _quat_matrix(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


@pytest.mark.parametrize("tilt", [0.0, 40.0])
def test_contact_velocity_is_the_rigid_motion(ref, tilt):
    """Nodes inside the indenter take the object's velocity (relative rest): it
    equals the displacement of a body-fixed point between the two poses divided
    by the step, up to the second-order term of the rotation.  With the start
    orientation tilted about the capsule's own axis (the same solid), the step's
    rotation is applied in the world frame, q1 = dq q0, and the velocity is that
    of dq's world axis, not of the body-frame axis q0^-1 dq q0."""
    p = W.small_sensor(cells=(8, 8, 4), shape=W.SHAPE_CAPSULE, radius=1.0e-3)
    t = math.radians(tilt)
    q0 = np.array([math.cos(t / 2), math.sin(t / 2), 0.0, 0.0])
    p = p.replace(half_length=1.0e-3, pose0=(p.pose0[0], p.pose0[1], p.height + 0.5e-3, *q0))
    s = ref.OracleSim(p)
    ang = 0.01
    dq = np.array((math.cos(ang / 2), 0.02 * math.sin(ang / 2), -0.03 * math.sin(ang / 2), math.sin(ang / 2)))
    dq /= np.linalg.norm(dq)
    qn = _quat_mul(dq, q0)
    c0 = np.array(p.pose0[:3])
    c1 = c0 + np.array([2e-6, -1e-6, -3e-6])
    s.set_target_pose(c1, qn)
    s.p2g()
    s.grid_update(contact=True, bc=False)
    _, _, V = s.grid()
    inside = s.inside_mask()
    assert inside.sum() > 10
    X = brute.node_positions(p)[inside]
    R = _quat_matrix(qn) @ _quat_matrix(q0).T
    moved = (X - c0) @ R.T + c1
    want = (moved - X) / p.dt
    err = np.abs(V[inside] - want).max()
    assert err < 2 * ang * np.abs(want).max(), err


@pytest.mark.slow
def test_elastic_impulse_once_per_step_is_the_stable_reading(ref):
    """Algorithm 1 repeats the exchange while the relative-rest test fails.  If
    every repetition re-added the elastic momentum ME_i (Eq. 4), a step with
    several passes would apply the elastic impulse several times: under slip and
    rotation the oracle then inverts elements (det F <= 0), while adding it in
    the step's first exchange only stays valid.  This fixes the reading used on
    both sides (the literal variant remains available as stress_each_pass = 1)."""
    res = {}
    for sep in (1, 0):
        p = W.small_sensor(cells=(16, 16, 6), dx=0.25e-3, subcycle=4, radius=1.5e-3, pad=8,
                           stress_each_pass=sep)
        s = ref.OracleSim(p)
        c = np.array(p.pose0[:3])
        try:
            s.set_target_pose(c + [0, 0, -0.5e-3], (1, 0, 0, 0))
            s.step(200)
            for i in range(10):
                s.set_target_pose(c + [0.05e-3 * (i + 1), 0, -0.5e-3], W.quat_about_z(3 * (i + 1)))
                s.step(20)
            res[sep] = "ok"
        except FloatingPointError:
            res[sep] = "invalid"
    assert res == {1: "invalid", 0: "ok"}, res


@pytest.mark.parametrize("shape", [W.SHAPE_SPHERE, W.SHAPE_CAPSULE, W.SHAPE_BOX, W.SHAPE_HEIGHTFIELD])
def test_indenter_depthmap_agrees_with_inside_test(ref, shape):
    """The depth map's lowest point on each pixel's vertical line is the
    indenter's boundary: 1e-9 m above it is inside, 1e-9 m below is outside;
    a line that misses the indenter is outside at every height sampled."""
    p = W.small_sensor(cells=(16, 16, 4))
    L = 16 * p.dx
    if shape == W.SHAPE_SPHERE:
        p = p.replace(radius=2.5e-3, pose0=(L / 2, L / 2, p.height + 2.0e-3, 1, 0, 0, 0))
    elif shape == W.SHAPE_CAPSULE:
        p = p.replace(shape=shape, radius=1.2e-3, half_length=2.0e-3,
                      pose0=(L / 2, L / 2, p.height + 1.0e-3, 1, 0, 0, 0))
    elif shape == W.SHAPE_BOX:
        p = p.replace(shape=shape, half_extent=(2.0e-3, 1.5e-3, 1.0e-3), fillet=0.4e-3,
                      pose0=(L / 2, L / 2, p.height + 0.8e-3, 1, 0, 0, 0))
    else:
        tab = W.heightfield_table(3, 3.0e-3, 0.3e-3, 2.0e-3, 8e-3)
        p = p.replace(shape=shape, hf=tab, hf_half=3.0e-3, pose0=(L / 2, L / 2, p.height - 0.2e-3, 1, 0, 0, 0))
    s = ref.OracleSim(p)
    s.set_target_pose(p.pose0[:3], W.quat_about_z(35))
    s.step(1)                               # rotated 35 degrees about z
    Wd, H = 24, 20
    d = s.indenter_depthmap(Wd, H)
    u, v = np.meshgrid((np.arange(Wd) + 0.5) * L / Wd, (np.arange(H) + 0.5) * L / H)
    hit = d > -1e8
    assert 10 < hit.sum() < hit.size
    zl = p.height - d[hit]
    up = np.stack([u[hit], v[hit], zl + 1e-9], -1)
    dn = np.stack([u[hit], v[hit], zl - 1e-9], -1)
    assert (s.point_phi(up) <= 0).all()
    assert (s.point_phi(dn) > 0).all()
    for z in np.linspace(-0.01, 0.02, 61):
        miss = np.stack([u[~hit], v[~hit], np.full((~hit).sum(), z)], -1)
        assert (s.point_phi(miss) > 0).all()
    # a tilted indenter is rejected
    t = ref.OracleSim(p.replace(pose0=tuple(p.pose0[:3]) + (np.cos(0.1), np.sin(0.1), 0.0, 0.0)))
    with pytest.raises(ValueError):
        t.indenter_depthmap(8, 8)

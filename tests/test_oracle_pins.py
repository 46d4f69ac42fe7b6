"""Pins of the FP64 oracle against what physics and geometry fix.

Every check here is independent of the oracle's own code: closed forms of
semi-implicit Euler, conservation laws, textbook friction results, analytic
contact geometry, brute-force properties and finite differences.  CPU only.
"""
import math

import numpy as np
import pytest

from helpers import DT, G, S, custom_batch, kinetic, momenta, quat_axis_angle, quat_to_R
from oracle import oracle as O


def sim_of(batch, **kw):
    return O.OracleSim(batch, **kw)


# ------------------------------------------------------------ integration
def test_ballistic_closed_form():
    """x_n = x0 + n dt v0 + g dt^2 n(n+1)/2 and v_n = v0 + n g dt (semi-implicit Euler)."""
    bodies = [dict(shape=S.SPHERE, param=[0.1, 0, 0], pos=[0, 0, 50.0], vel=[1.0, -2.0, 3.0, 0, 0, 0]),
              dict(shape=S.BOX, param=[0.1, 0.2, 0.3], pos=[5, 0, 60.0], vel=[0, 0.5, 0, 0, 0, 0])]
    b = custom_batch([bodies])
    sim = sim_of(b)
    x0 = sim.pose.reshape(-1, 7)[:, :3].copy()
    v0 = sim.vel.reshape(-1, 6)[:, :3].copy()
    n = 120
    for _ in range(n):
        r = sim.step(iters=10)
        assert r["n_pairs"][0] == 0
    g = np.array([0, 0, -G])
    xn = x0 + n * DT * v0 + g * DT * DT * n * (n + 1) / 2
    vn = v0 + n * g * DT
    np.testing.assert_allclose(sim.pose.reshape(-1, 7)[:, :3], xn, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sim.vel.reshape(-1, 6)[:, :3], vn, rtol=1e-12, atol=1e-12)


def test_quaternion_constant_omega():
    """Each step rotates by exactly 2*atan(|w| dt / 2) about w (first-order
    update followed by normalisation)."""
    w = np.array([0.3, -1.2, 2.0])
    b = custom_batch([[dict(shape=S.SPHERE, param=[0.1, 0, 0], pos=[0, 0, 100.0],
                            vel=[0, 0, 0, *w])]])
    sim = sim_of(b, gravity=(0.0, 0.0, 0.0))
    q0 = sim.pose.reshape(-1, 7)[0, 3:].copy()
    n = 50
    for _ in range(n):
        sim.step(iters=1)
    q = sim.pose.reshape(-1, 7)[0, 3:]
    step_angle = 2 * math.atan(np.linalg.norm(w) * DT / 2)
    expect = quat_axis_angle(w, n * step_angle)
    # q = dq (x) q0
    w0, x0, y0, z0 = expect
    a0, a1, a2, a3 = q0
    qq = np.array([w0 * a0 - x0 * a1 - y0 * a2 - z0 * a3,
                   w0 * a1 + x0 * a0 + y0 * a3 - z0 * a2,
                   w0 * a2 - x0 * a3 + y0 * a0 + z0 * a1,
                   w0 * a3 + x0 * a2 - y0 * a1 + z0 * a0])
    assert abs(abs(np.dot(qq, q)) - 1.0) < 1e-12


def test_momentum_no_contacts():
    """Without contacts total momentum changes by exactly n dt M g."""
    bodies = [dict(shape=k % 3, param=[0.1, 0.05, 0.07], mass=0.5 + k, pos=[3.0 * k, 0, 30.0],
                   vel=[k, 1, 0, 0.5, k, 1]) for k in range(6)]
    b = custom_batch([bodies])
    sim = sim_of(b)
    P0, _ = momenta(b, sim.pose, sim.vel)
    n = 30
    for _ in range(n):
        sim.step(iters=10)
    P1, _ = momenta(b, sim.pose, sim.vel)
    M = float(np.sum(b.mass.astype(np.float64)))
    np.testing.assert_allclose(P1 - P0, [0, 0, -G * n * DT * M], atol=1e-10)


# ------------------------------------------------------------ solver invariants
def _colliding_cluster(seed):
    rng = np.random.default_rng(seed)
    bodies = []
    for k in range(8):
        shape = k % 3
        param = [0.12, 0.1, 0.08] if shape != S.SPHERE else [0.12, 0, 0]
        if shape == S.CAPSULE:
            param = [0.07, 0.1, 0]
        pos = [0.18 * (k % 4), 0.18 * (k // 4), 10.0]
        q = rng.normal(size=4)
        bodies.append(dict(shape=shape, param=param, mass=0.3 + rng.random(), pos=pos,
                           quat=q / np.linalg.norm(q), vel=np.concatenate([rng.normal(size=3), rng.normal(size=3)])))
    return custom_batch([bodies])


@pytest.mark.parametrize("solver", [O.PGS, O.JACOBI])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_solver_conserves_momentum(seed, solver):
    """Dynamic-only contacts in zero gravity: impulses are equal, opposite and
    share a point, so linear and angular momentum (at the pre-integration
    pose) are unchanged by the solve."""
    b = _colliding_cluster(seed)
    sim = sim_of(b, gravity=(0.0, 0.0, 0.0))
    pose0 = sim.pose.copy()
    P0, L0 = momenta(b, pose0, sim.vel)
    r = sim.step(iters=20, solver=solver)
    assert r["n_contacts"][0] > 3
    P1, L1 = momenta(b, pose0, sim.vel)
    np.testing.assert_allclose(P1, P0, atol=1e-10)
    np.testing.assert_allclose(L1, L0, atol=1e-10)


def test_solver_dissipative():
    """All contacts inside [-slop, 0] (zero bias) and e = 0: kinetic energy does
    not increase through the solve."""
    for seed in range(4):
        rng = np.random.default_rng(10 + seed)
        bodies = [dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=1.0, pos=[0, 0, 5.0],
                       vel=np.concatenate([rng.normal(size=3), rng.normal(size=3)])),
                  dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=2.0, pos=[0.198, 0.0, 5.0],
                       vel=np.concatenate([rng.normal(size=3), rng.normal(size=3)])),
                  dict(shape=S.BOX, param=[0.1, 0.1, 0.1], mass=1.5, pos=[-0.199, 0.0, 5.0],
                       vel=np.concatenate([rng.normal(size=3), rng.normal(size=3)]))]
        b = custom_batch([bodies])
        sim = sim_of(b, gravity=(0.0, 0.0, 0.0))
        pose0 = sim.pose.copy()
        E0 = kinetic(b, pose0, sim.vel)
        r = sim.step(iters=30)
        phi = r["c_phi"][0, :r["n_contacts"][0]]
        assert len(phi) >= 2 and np.all(phi <= 0) and np.all(phi >= -0.005)
        E1 = kinetic(b, pose0, sim.vel)
        assert E1 <= E0 * (1 + 1e-12)


def test_resting_sphere_single_contact():
    """A sphere resting on the plane (phi in [-slop, 0]) receives exactly
    m |g| dt of normal impulse; the second sweep changes nothing."""
    m = 1.7
    b = custom_batch([[dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=m, pos=[0, 0, 0.098])]])
    sim = sim_of(b)
    r = sim.step(iters=50, tol=1e-13)
    assert r["n_contacts"][0] == 1
    assert r["sweeps"][0] == 2
    m = float(b.mass[0])
    assert abs(r["c_lambda"][0, 0, 0] - m * G * DT) < 1e-12
    assert np.allclose(sim.vel.reshape(-1, 6)[0], 0, atol=1e-12)


def test_box_on_plane_sum_of_normals():
    """Statically indeterminate: only the sum of the 4 corner impulses is fixed."""
    m = 2.3
    q = quat_axis_angle([0, 0, 1], 0.4)
    b = custom_batch([[dict(shape=S.BOX, param=[0.2, 0.1, 0.05], mass=m, pos=[0, 0, 0.049], quat=q)]])
    sim = sim_of(b)
    r = sim.step(iters=500, tol=1e-12)
    nc = r["n_contacts"][0]
    assert nc == 4
    m = float(b.mass[0])
    assert abs(r["c_lambda"][0, :nc, 0].sum() - m * G * DT) < 1e-9
    assert np.max(np.abs(sim.vel.reshape(-1, 6)[0])) < 1e-9


def test_stack_interface_loads():
    """Stack of boxes: each interface carries (mass above) |g| dt."""
    masses = [1.0, 2.0, 0.5, 1.5]
    h = 0.1
    bodies = [dict(shape=S.BOX, param=[h, h, h], mass=m_, pos=[0, 0, h + 2 * h * k - 0.001 * (k + 1)])
              for k, m_ in enumerate(masses)]
    b = custom_batch([bodies])
    sim = sim_of(b)
    r = sim.step(iters=3000, tol=1e-12)
    nc = r["n_contacts"][0]
    keys = r["c_key"][0, :nc]
    lam = r["c_lambda"][0, :nc, 0]
    A = keys >> 20
    Bk = (keys >> 8) & 0xFFF
    for k in range(len(masses)):
        above = sum(masses[k:])
        # interface below box k: ground for k == 0, else box k-1
        sel = (A == k) & (Bk == 0xFFF) if k == 0 else (A == k - 1) & (Bk == k)
        assert sel.sum() == 4
        assert abs(lam[sel].sum() - above * G * DT) < 1e-8, (k, lam[sel].sum(), above * G * DT)


def test_sliding_box_friction():
    """A sliding box loses mu |g| dt of speed per step, then stays at rest."""
    mu = 0.5
    v0 = 0.6
    b = custom_batch([[dict(shape=S.BOX, param=[0.1, 0.1, 0.1], mass=1.0, mu=mu, pos=[0, 0, 0.0995],
                            vel=[v0, 0, 0, 0, 0, 0])]])
    sim = sim_of(b)  # ground friction 0.5 -> combined sqrt(0.5*0.5) = 0.5
    v0 = float(b.vel[0, 0])
    speeds = []
    for _ in range(30):
        sim.step(iters=200, tol=1e-13)
        speeds.append(sim.vel.reshape(-1, 6)[0, 0])
    k_stop = int(math.floor(v0 / (mu * G * DT)))
    for k in range(k_stop):
        assert abs(speeds[k] - (v0 - (k + 1) * mu * G * DT)) < 1e-9
    assert all(abs(s) < 1e-9 for s in speeds[k_stop + 1:])


def test_rolling_sphere_five_sevenths():
    """A sphere launched sliding with v0 and no spin ends up rolling at 5/7 v0."""
    v0 = 2.0
    r_ = 0.1
    b = custom_batch([[dict(shape=S.SPHERE, param=[r_, 0, 0], mass=1.0, mu=0.5, pos=[0, 0, r_],
                            vel=[v0, 0, 0, 0, 0, 0])]])
    sim = sim_of(b)
    v0 = float(b.vel[0, 0])
    for _ in range(200):
        sim.step(iters=100, tol=1e-13)
    v = sim.vel.reshape(-1, 6)[0]
    assert abs(v[0] - 5.0 / 7.0 * v0) < 1e-6
    assert abs(v[4] - v[0] / r_) < 1e-5        # rolling: w_y = v_x / r


def test_inelastic_head_on():
    """Two touching spheres, zero gravity, e = 0: one sweep gives the common velocity."""
    m1, m2, v1, v2 = 1.0, 3.0, 2.0, -1.0
    b = custom_batch([[dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=m1, pos=[-0.1, 0, 5.0], vel=[v1, 0, 0, 0, 0, 0]),
                       dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=m2, pos=[0.1, 0, 5.0], vel=[v2, 0, 0, 0, 0, 0])]])
    sim = sim_of(b, gravity=(0.0, 0.0, 0.0))
    sim.step(iters=1)
    vc = (m1 * v1 + m2 * v2) / (m1 + m2)
    v = sim.vel.reshape(-1, 6)
    assert abs(v[0, 0] - vc) < 1e-12 and abs(v[1, 0] - vc) < 1e-12


def test_resting_stack_stable():
    """5 boxes (h = 0.1 m, 1 kg) over 600 steps, 20 sweeps, previous-step warm
    start: little drift, little sink, at rest at the end."""
    h = 0.1
    bodies = [dict(shape=S.BOX, param=[h, h, h], mass=1.0, pos=[0, 0, h + 2 * h * k]) for k in range(5)]
    b = custom_batch([bodies])
    sim = sim_of(b)
    x0 = sim.pose.reshape(-1, 7)[:, :3].copy()
    for _ in range(600):
        sim.step(iters=20, warm=O.PREV)
    x = sim.pose.reshape(-1, 7)[:, :3]
    assert np.linalg.norm(x[4, :2] - x0[4, :2]) < 1e-3
    assert np.all(x0[:, 2] - x[:, 2] <= 0.005 + 0.001 + 1e-9)
    assert np.abs(sim.vel).max() < 1e-3


def test_prev_warm_start_converges_immediately():
    """Resting sphere, second step warm-started from the first: residual ~0 after one sweep."""
    b = custom_batch([[dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=1.0, pos=[0, 0, 0.098])]])
    sim = sim_of(b)
    sim.step(iters=50, tol=1e-13, warm=O.PREV)
    r = sim.step(iters=50, tol=1e-12, warm=O.PREV)
    assert r["sweeps"][0] == 1


def test_jacobi_single_contact():
    b = custom_batch([[dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=1.3, pos=[0, 0, 0.098])]])
    sim = sim_of(b)
    r = sim.step(iters=50, tol=1e-13, solver=O.JACOBI)
    assert abs(r["c_lambda"][0, 0, 0] - float(b.mass[0]) * G * DT) < 1e-12


# ------------------------------------------------------------ narrowphase analytic cases
def test_sphere_sphere_and_ground():
    c, amb = O.collide(S.SPHERE, [0.1, 0, 0], [0, 0, 1, 1, 0, 0, 0], S.SPHERE, [0.2, 0, 0], [0.3, 0, 1, 1, 0, 0, 0])
    assert len(c) == 1
    f, n, p, phi = c[0]
    assert abs(phi - 0.0) < 1e-15 and np.allclose(n, [-1, 0, 0]) and np.allclose(p, [0.1, 0, 1])
    c, _ = O.collide(S.SPHERE, [0.1, 0, 0], [1, 2, 0.09, 1, 0, 0, 0])
    assert len(c) == 1 and abs(c[0][3] + 0.01) < 1e-15 and np.allclose(c[0][1], [0, 0, 1])
    assert np.allclose(c[0][2], [1, 2, -0.005])
    c, _ = O.collide(S.SPHERE, [0.1, 0, 0], [0, 0, 0.2, 1, 0, 0, 0])
    assert len(c) == 0          # phi = 0.1 > margin


def test_box_on_plane_corners():
    h = [0.3, 0.2, 0.1]
    c, amb = O.collide(S.BOX, h, [0.5, 0.5, 0.095, 1, 0, 0, 0])
    assert [x[0] for x in c] == [0, 1, 2, 3]
    for f, n, p, phi in c:
        assert abs(phi - (-0.005)) < 1e-15 and np.allclose(n, [0, 0, 1])
        sx = h[0] if f & 1 else -h[0]
        sy = h[1] if f & 2 else -h[1]
        assert np.allclose(p, [0.5 + sx, 0.5 + sy, -0.0025])


def test_box_on_box_face_rectangle():
    """Small box resting on a big box: 4 contacts at the small box's corners."""
    big = [1.0, 1.0, 0.5]
    small = [0.1, 0.2, 0.1]
    q = quat_axis_angle([0, 0, 1], 0.3)
    c, amb = O.collide(S.BOX, small, [0.1, -0.2, 0.5 + 0.1 - 0.002, *q], S.BOX, big, [0, 0, 0, 1, 0, 0, 0])
    assert amb == 0 and len(c) == 4
    R = quat_to_R(q)
    corners = [np.array([0.1, -0.2, 0.598]) + R @ np.array([sx * 0.1, sy * 0.2, -0.1])
               for sx in (1, -1) for sy in (1, -1)]
    for f, n, p, phi in c:
        assert np.allclose(n, [0, 0, 1]) and abs(phi + 0.002) < 1e-12
        assert min(np.linalg.norm(p[:2] - cc[:2]) for cc in corners) < 1e-12
        assert abs(p[2] - 0.499) < 1e-12


def test_box_on_box_overlap_octagon_reduced():
    """Two equal squares rotated 45 deg: the overlap is an octagon, reduced to 4."""
    q = quat_axis_angle([0, 0, 1], math.pi / 4)
    c, amb = O.collide(S.BOX, [0.2, 0.2, 0.1], [0, 0, 0.199, *q], S.BOX, [0.2, 0.2, 0.1], [0, 0, 0, 1, 0, 0, 0])
    assert len(c) == 4
    for f, n, p, phi in c:
        assert np.allclose(n, [0, 0, 1])
        # octagon vertices lie on the boundary of both squares
        assert max(abs(p[0]), abs(p[1])) <= 0.2 + 1e-9


def test_capsule_parallel_to_plane_two_contacts():
    q = quat_axis_angle([0, 1, 0], math.pi / 2)   # core along x
    c, amb = O.collide(S.CAPSULE, [0.05, 0.2, 0], [0, 0, 0.049, *q])
    assert [x[0] for x in c] == [0, 1]
    xs = sorted(x[2][0] for x in c)
    assert np.allclose(xs, [-0.2, 0.2]) and all(abs(x[3] + 0.001) < 1e-12 for x in c)


def test_crossed_capsules_one_contact():
    qa = quat_axis_angle([0, 1, 0], math.pi / 2)   # along x
    qb = quat_axis_angle([1, 0, 0], math.pi / 2)   # along y
    c, amb = O.collide(S.CAPSULE, [0.05, 0.3, 0], [0.1, 0.05, 0.2, *qa], S.CAPSULE, [0.04, 0.3, 0], [0, 0, 0.1, *qb])
    assert len(c) == 1
    f, n, p, phi = c[0]
    assert abs(phi - (0.1 - 0.05 - 0.04)) < 1e-12 and np.allclose(n, [0, 0, 1])
    assert np.allclose(p, [0, 0.05, 0.1 + 0.04 + 0.005])


def test_parallel_capsules_two_contacts():
    qa = quat_axis_angle([0, 1, 0], math.pi / 2)
    c, amb = O.collide(S.CAPSULE, [0.05, 0.3, 0], [0.2, 0, 0.1, *qa], S.CAPSULE, [0.05, 0.3, 0], [0, 0, 0.0, *qa])
    assert [x[0] for x in c] == [0, 1]
    assert sorted(np.round([x[2][0] for x in c], 12)) == [-0.1, 0.3]
    assert all(abs(x[3] - 0.0) < 1e-12 for x in c)


def test_capsule_on_box_face_two_contacts():
    q = quat_axis_angle([0, 1, 0], math.pi / 2)
    c, amb = O.collide(S.CAPSULE, [0.05, 0.2, 0], [0, 0.1, 0.5 + 0.049, *q], S.BOX, [1, 1, 0.5], [0, 0, 0, 1, 0, 0, 0])
    assert [x[0] for x in c] == [0, 1]
    for f, n, p, phi in c:
        assert np.allclose(n, [0, 0, 1]) and abs(phi + 0.001) < 1e-12
    # overhanging the edge: the clipped end sits on the box edge
    c, amb = O.collide(S.CAPSULE, [0.05, 0.2, 0], [0.9, 0.1, 0.5 + 0.049, *q], S.BOX, [1, 1, 0.5], [0, 0, 0, 1, 0, 0, 0])
    assert len(c) == 2 and np.isclose(max(x[2][0] for x in c), 1.0)


def test_capsule_across_box_edge_one_contact():
    qb = quat_axis_angle([1, 0, 0], math.pi / 2)   # core along y, above the x = 1 top edge, tilted
    qt = quat_axis_angle([0, 1, 0], 0.5)
    w0, x0, y0, z0 = qt
    a0, a1, a2, a3 = qb
    q = [w0 * a0 - x0 * a1 - y0 * a2 - z0 * a3, w0 * a1 + x0 * a0 + y0 * a3 - z0 * a2,
         w0 * a2 - x0 * a3 + y0 * a0 + z0 * a1, w0 * a3 + x0 * a2 - y0 * a1 + z0 * a0]
    d = 0.06
    pos = [1.0 + d / math.sqrt(2), 0.0, 0.5 + d / math.sqrt(2)]
    c, amb = O.collide(S.CAPSULE, [0.05, 0.2, 0], [*pos, *q], S.BOX, [1, 1, 0.5], [0, 0, 0, 1, 0, 0, 0])
    assert len(c) == 1 and c[0][0] == 2
    assert abs(c[0][3] - (d - 0.05)) < 1e-12
    assert np.allclose(c[0][1], [1 / math.sqrt(2), 0, 1 / math.sqrt(2)])


def test_sphere_box_outside_edge_and_inside():
    c, _ = O.collide(S.SPHERE, [0.1, 0, 0], [1.05, 0, 0.55, 1, 0, 0, 0], S.BOX, [1, 1, 0.5], [0, 0, 0, 1, 0, 0, 0])
    assert len(c) == 1 and abs(c[0][3] - (math.hypot(0.05, 0.05) - 0.1)) < 1e-12
    c, _ = O.collide(S.SPHERE, [0.1, 0, 0], [0.2, 0.1, 0.45, 1, 0, 0, 0], S.BOX, [1, 1, 0.5], [0, 0, 0, 1, 0, 0, 0])
    assert len(c) == 1 and np.allclose(c[0][1], [0, 0, 1]) and abs(c[0][3] - (-0.05 - 0.1)) < 1e-12


def test_box_box_edge_edge():
    """Two boxes touching edge to edge: crossed edges, one contact, f = 0x80 | axis."""
    qa = quat_axis_angle([1, 0, 0], math.pi / 4)   # edge along x at the bottom
    qb = quat_axis_angle([0, 1, 0], math.pi / 4)   # edge along y at the top
    ha = hb = 0.1
    e = ha * math.sqrt(2)
    gap = 0.004
    c, amb = O.collide(S.BOX, [ha, ha, ha], [0, 0, e + gap / 2, *qa], S.BOX, [hb, hb, hb], [0, 0, -e - gap / 2, *qb])
    assert len(c) == 1 and c[0][0] & 0x80
    assert abs(c[0][3] - gap) < 1e-12 and np.allclose(c[0][1], [0, 0, 1]) and np.allclose(c[0][2], 0, atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_narrowphase_metamorphic(seed):
    """Same phi under a global rigid motion; swapping A and B flips the normal
    (and keeps phi) for every pair type."""
    rng = np.random.default_rng(seed)
    params = {S.SPHERE: [0.1, 0, 0], S.BOX: [0.12, 0.08, 0.1], S.CAPSULE: [0.06, 0.12, 0]}
    Rq = rng.normal(size=4)
    Rq /= np.linalg.norm(Rq)
    R = quat_to_R(Rq)
    t = rng.normal(size=3)
    for sa in (0, 1, 2):
        for sb in (0, 1, 2):
            for _ in range(20):
                qa = rng.normal(size=4); qa /= np.linalg.norm(qa)
                qb = rng.normal(size=4); qb /= np.linalg.norm(qb)
                pa = rng.normal(size=3) * 0.12
                pb = rng.normal(size=3) * 0.12
                c1, amb1 = O.collide(sa, params[sa], [*pa, *qa], sb, params[sb], [*pb, *qb])
                c2, amb2 = O.collide(sb, params[sb], [*pb, *qb], sa, params[sa], [*pa, *qa])
                if amb1 or amb2:
                    continue
                if sa != sb:
                    assert len(c1) == len(c2)
                    for x, y in zip(c1, c2):
                        assert x[0] == y[0]
                        assert np.allclose(x[1], -y[1], atol=1e-12) and abs(x[3] - y[3]) < 1e-12
                # rigid motion
                def mv(p, q):
                    w0, x0, y0, z0 = Rq
                    a0, a1, a2, a3 = q
                    qq = [w0 * a0 - x0 * a1 - y0 * a2 - z0 * a3, w0 * a1 + x0 * a0 + y0 * a3 - z0 * a2,
                          w0 * a2 - x0 * a3 + y0 * a0 + z0 * a1, w0 * a3 + x0 * a2 - y0 * a1 + z0 * a0]
                    return [*(R @ p + t), *qq]
                c3, amb3 = O.collide(sa, params[sa], mv(pa, qa), sb, params[sb], mv(pb, qb))
                if amb3:
                    continue
                assert [x[0] for x in c1] == [x[0] for x in c3]
                for x, y in zip(c1, c3):
                    assert abs(x[3] - y[3]) < 1e-9
                    assert np.allclose(R @ x[1], y[1], atol=1e-9)
                    assert np.allclose(R @ x[2] + t, y[2], atol=1e-9)


def test_contact_phi_matches_distance_sampling():
    """Separated convex pairs: phi of a single contact equals the true distance
    between the shapes (sampled surfaces give an upper bound close to it)."""
    rng = np.random.default_rng(5)
    for _ in range(30):
        pa = np.array([0, 0, 0.0])
        pb = rng.normal(size=3)
        pb = pb / np.linalg.norm(pb) * (0.1 + 0.12 + 0.01 + 0.005 * rng.random())
        c, amb = O.collide(S.SPHERE, [0.1, 0, 0], [*pa, 1, 0, 0, 0], S.SPHERE, [0.12, 0, 0], [*pb, 1, 0, 0, 0])
        d = np.linalg.norm(pb - pa) - 0.22
        assert len(c) == 1 and abs(c[0][3] - d) < 1e-12


# ------------------------------------------------------------ broadphase / colouring
def test_pairs_contain_contacts_and_respect_bounds():
    """Every pair with a contact is in the pair set; every pair is within the
    bounding-sphere reach (AABB overlap implies |xi - xj| <= sqrt(3)(Ri + Rj + 2 margin))."""
    b = S.batch_drop(3)
    sim = sim_of(b)
    for _ in range(60):
        sim.step(iters=5, warm=O.PREV)
    pose = sim.pose.reshape(-1, 7)
    r = sim.step(iters=5, warm=O.PREV)
    for s in range(3):
        off = b.body_offset[s]
        pk = set(r["pair_key"][s, :r["n_pairs"][s]].tolist())
        ck = r["c_key"][s, :r["n_contacts"][s]]
        for k in ck:
            a, bb = int(k >> 20), int((k >> 8) & 0xFFF)
            assert ((a << 16) | (0xFFFF if bb == 0xFFF else bb)) in pk
        keys = sorted(pk)
        assert keys == sorted(keys)
        for k in pk:
            a, bb = k >> 16, k & 0xFFFF
            if bb == 0xFFFF:
                continue
            Ra = S.bounding_radius(int(b.shape[off + a]), b.param[off + a])
            Rb = S.bounding_radius(int(b.shape[off + bb]), b.param[off + bb])
            # note: pose here is after this step; use the pre-step reach plus motion slack
            assert np.linalg.norm(pose[off + a, :3] - pose[off + bb, :3]) <= math.sqrt(3) * (Ra + Rb + 0.04) + 0.1


def test_pairs_closed_interval_touching():
    """AABBs that touch exactly (closed intervals) form a pair; a hair apart do not."""
    m = 0.25
    r1 = 0.25
    x = 2 * (r1 + m)             # sphere AABBs touch exactly (exact binary values)
    b = custom_batch([[dict(shape=S.SPHERE, param=[r1, 0, 0], pos=[0, 0, 5]),
                       dict(shape=S.SPHERE, param=[r1, 0, 0], pos=[x, 0, 5]),
                       dict(shape=S.SPHERE, param=[r1, 0, 0], pos=[-x - 0.001, 0, 5])]])
    sim = sim_of(b, margin=m)
    keys = np.zeros(16, np.uint32)
    import ctypes
    n = O.lib().ora_pairs(ctypes.byref(sim.m), sim.pose.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0,
                          keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), 16)
    assert n == 1 and keys[0] == (0 << 16) | 1


def test_colouring_first_fit_property():
    """Colours: no dynamic body twice in one colour, and every contact of colour
    c has, for each c' < c, an earlier contact of colour c' on one of its
    dynamic bodies (the defining property of first fit in canonical order)."""
    b = S.batch_drop(2, seed0=7)
    sim = sim_of(b)
    for _ in range(90):
        r = sim.step(iters=10, warm=O.PREV)
    for s in range(2):
        nc = r["n_contacts"][s]
        keys = r["c_key"][s, :nc]
        col = r["c_colour"][s, :nc]
        dyn = lambda i: i != 0xFFF and b.motion[b.body_offset[s] + i] == S.DYNAMIC
        bodies = [[i for i in (int(k >> 20), int((k >> 8) & 0xFFF)) if dyn(i)] for k in keys]
        for c in range(col.max() + 1):
            seen = set()
            for q in np.nonzero(col == c)[0]:
                for i in bodies[q]:
                    assert i not in seen
                    seen.add(i)
        for q in range(nc):
            for c in range(col[q]):
                assert any(col[p] == c and set(bodies[p]) & set(bodies[q]) for p in range(q))
        assert r["n_colours"][s] == col.max() + 1


# ------------------------------------------------------------ arm
def test_arm_straight_up_and_velocity_by_finite_difference():
    """theta = 0: links stacked along +z from the base.  Link velocities equal
    the finite difference of the link poses under the joint velocities."""
    b = custom_batch([[dict(shape=S.SPHERE, param=[0.1, 0, 0], pos=[3, 3, 5])]], arm=True)
    sim = sim_of(b)
    pose = sim.pose.reshape(-1, 7)
    z = 0.8
    for k, L in enumerate(S.ARM_LINK_LENGTH):
        assert np.allclose(pose[1 + k, :3], [0, 0, z + L / 2], atol=1e-15)
        z += L
    th = np.array([0.3, -0.4, 0.2, 0.5, -0.1, 0.25, 0.7])
    thd = np.array([0.5, -0.3, 0.8, 0.2, -0.6, 0.4, 0.1])
    b2 = custom_batch([[dict(shape=S.SPHERE, param=[0.1, 0, 0], pos=[3, 3, 5])]], arm=True, theta=th)
    eps = 1e-6
    sims = []
    th = b2.arm_theta[0].astype(np.float64)
    for sgn in (-1, 1):
        ss = sim_of(b2)
        ss.set_theta(th + sgn * eps * thd)
        sims.append(ss.pose.reshape(-1, 7)[1:, :3].copy())
    vfd = (sims[1] - sims[0]) / (2 * eps)
    s2 = sim_of(b2)
    s2.step(actions=thd[None, :], iters=1)
    v = s2.vel.reshape(-1, 6)[1:, :3]
    np.testing.assert_allclose(v, vfd, atol=1e-6)
    # joint angles advanced by dt * thd
    np.testing.assert_allclose(s2.theta, th + DT * thd, atol=1e-15)


def test_arm_holds_sphere_contact_force():
    """A sphere resting on a horizontal arm link is held: C_t -> m |g|."""
    th = np.zeros(7)
    th[1] = math.pi / 2        # joint 1 (about y) lays the arm along +x
    b0 = custom_batch([[dict(shape=S.SPHERE, param=[0.05, 0, 0], pos=[5, 5, 5])]], arm=True, theta=th)
    link_pose = sim_of(b0).pose.reshape(-1, 7)[1:]
    # sphere on top of link 3 (the long 0.3 m link after the bend)
    c = link_pose[3, :3]
    m = 0.7
    b = custom_batch([[dict(shape=S.SPHERE, param=[0.05, 0, 0], mass=m, mu=0.8, pos=[c[0], c[1], c[2] + 0.1 - 0.001])]],
                     arm=True, theta=th)
    sim = sim_of(b)
    for _ in range(5):
        r = sim.step(actions=np.zeros((1, 7)), iters=100, tol=1e-12, warm=O.PREV)
    assert abs(r["arm_force"][0] - float(b.mass[0]) * G) < 1e-6


# ------------------------------------------------------------ flags
def test_capacity_flag_on_small_cache():
    b = S.batch_drop(1)
    sim = O.OracleSim(b, cache_cap=4)
    for _ in range(100):
        r = sim.step(iters=5)
    assert r["flags"][0] & O.F_CAPACITY


def test_not_converged_flag():
    b = S.batch_drop(1)
    sim = sim_of(b)
    for _ in range(100):
        r = sim.step(iters=2, tol=1e-12)
    assert r["flags"][0] & O.F_NOT_CONVERGED and r["sweeps"][0] == 2


# ------------------------------------------------------------ MLP
def _net(seed, positive=False):
    rng = np.random.default_rng(seed)
    p = dict(w1=rng.normal(size=(64, 16)) * 0.3, b1=rng.normal(size=64) * 0.1,
             w2=rng.normal(size=(64, 64)) * 0.15, b2=rng.normal(size=64) * 0.1,
             w3=rng.normal(size=(3, 64)) * 0.2, b3=rng.normal(size=3) * 0.1,
             mean=rng.normal(size=16), std=0.5 + rng.random(16))
    if positive:
        for k in ("w1", "w2", "b1", "b2"):
            p[k] = np.abs(p[k])
    return p


def test_mlp_reduces_to_affine_chain_when_relu_inactive():
    """With every pre-activation positive the net is the product of its affine maps."""
    p = _net(0, positive=True)
    x = p["mean"] + np.abs(np.random.default_rng(1).normal(size=(20, 16))) * p["std"]
    y = O.mlp_forward(p, x)
    z = (x - p["mean"]) / p["std"]
    ref = ((z @ p["w1"].T + p["b1"]) @ p["w2"].T + p["b2"]) @ p["w3"].T + p["b3"]
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_mlp_gradient_central_differences():
    p = _net(2)
    rng = np.random.default_rng(3)
    x = rng.normal(size=(7, 16)) + p["mean"]
    t = rng.normal(size=(7, 3))
    loss, g = O.mlp_loss_grad(p, x, t)
    eps = 1e-6
    for k in ("w1", "b1", "w2", "b2", "w3", "b3"):
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            lp, _ = O.mlp_loss_grad(p, x, t)
            flat[i] = old - eps
            lm, _ = O.mlp_loss_grad(p, x, t)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, an)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    xs = np.concatenate([rng.normal(size=2000) * 10 ** rng.uniform(-8, 8, size=2000),
                         [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 3.0e38]])
    ref = torch.tensor(xs, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([O.bf16(v) for v in xs])
    np.testing.assert_array_equal(got, ref)


# ------------------------------------------------------------ Adam
def test_adam_first_step_is_lr_times_sign():
    """Bias correction makes the first update exactly lr * g / (|g| + eps)."""
    rng = np.random.default_rng(5)
    g = rng.normal(size=50) * 10 ** rng.uniform(-3, 3, size=50)
    p0 = rng.normal(size=50)
    p, m, v, _, _ = O.adam_step(p0, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    np.testing.assert_allclose(p0 - p, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)


def test_adam_constant_gradient_constant_step():
    """With a constant gradient the corrected moments equal g and g^2 at
    every step, so each update is lr * sign(g) (up to eps)."""
    g = np.array([0.3, -2.0, 5e-3])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for k in range(1, 40):
        q, m, v, _, _ = O.adam_step(p, m, v, g, k, 1e-2)
        np.testing.assert_allclose(p - q, 1e-2 * np.sign(g), rtol=1e-5)
        p = q


def test_adam_scale_invariant_and_clip_norm():
    """Rescaling every gradient by one constant leaves the trajectory
    unchanged (eps aside); clipping yields norm min(|g|, clip) along g."""
    rng = np.random.default_rng(6)
    gs = [rng.normal(size=20) for _ in range(5)]
    pa = pb = rng.normal(size=20)
    ma = va = mb = vb = np.zeros(20)
    for k, g in enumerate(gs, 1):
        pa, ma, va, _, _ = O.adam_step(pa, ma, va, g, k, 1e-3)
        pb, mb, vb, _, _ = O.adam_step(pb, mb, vb, 1e3 * g, k, 1e-3)
    np.testing.assert_allclose(pa, pb, rtol=0, atol=1e-9)
    g = gs[0]
    n = np.linalg.norm(g)
    _, _, _, gc, norm = O.adam_step(np.zeros(20), np.zeros(20), np.zeros(20), g, 1, 1e-3, clip=0.5 * n)
    assert abs(norm - n) <= 1e-12 * n
    assert abs(np.linalg.norm(gc) - 0.5 * n) <= 1e-12 * n
    assert abs(gc @ g / (np.linalg.norm(gc) * n) - 1) <= 1e-12
    _, _, _, gc, _ = O.adam_step(np.zeros(20), np.zeros(20), np.zeros(20), g, 1, 1e-3, clip=2 * n)
    np.testing.assert_array_equal(gc, g)


# ------------------------------------------------------------ learned warm start in the step
def _const_net(y=(0.0, 0.0, 0.0), scale=0.0, seed=0):
    """Network with output y everywhere (scale 0), or random weights times scale."""
    rng = np.random.default_rng(seed)
    p = dict(w1=rng.normal(size=(64, 16)) * scale, b1=np.zeros(64), w2=rng.normal(size=(64, 64)) * scale,
             b2=np.zeros(64), w3=rng.normal(size=(3, 64)) * scale, b3=np.asarray(y, float),
             mean=np.zeros(16), std=np.ones(16))
    if scale:
        p["b1"] = np.ones(64) * scale
        p["b2"] = np.ones(64) * scale
    return p


def test_learned_new_contact_unit_is_gravity_impulse():
    """A new resting sphere contact started from network output (1, 0, 0)
    starts at exactly m g dt (k_n = 1/m at the centre), which is the
    converged impulse: one sweep reaches the tolerance."""
    b = custom_batch([[dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=1.3, pos=[0, 0, 0.1])]])
    sim = sim_of(b)
    sim.set_mlp(_const_net((1.0, 0.0, 0.0)))
    r = sim.step(iters=50, tol=1e-10, warm=O.LEARNED)
    assert r["c_feat"][0, 0, 15] == 1.0
    assert abs(r["c_lambda"][0, 0, 0] - float(b.mass[0]) * G * DT) < 1e-12
    assert r["sweeps"][0] == 1 and not (r["flags"][0] & O.F_FELLBACK)


def _stack_state():
    h = 0.1
    bodies = [dict(shape=S.BOX, param=[h, h, h], mass=1.0 + 0.5 * k, pos=[0.01 * k, 0, h + 2 * h * k])
              for k in range(3)]
    b = custom_batch([bodies])
    sim = sim_of(b)
    for _ in range(60):
        sim.step(iters=100, tol=1e-8, warm=O.PREV)
    return b, sim


def test_learned_zero_net_is_classic_warm_start():
    """Persisting contacts keep their previous impulses: with a zero network
    (new contacts start at zero, as in PREV) the learned step is the PREV
    step, bit for bit, and the start is not rejected."""
    b, sim = _stack_state()
    pose, vel, theta = sim.pose.copy(), sim.vel.copy(), sim.theta.copy()
    cache = sim.cache_arrays()
    ra = sim.step(iters=100, tol=1e-4, warm=O.PREV)
    pa, va = sim.pose.copy(), sim.vel.copy()
    sim.set_state(pose, vel, theta, cache)
    sim.set_mlp(_const_net())
    rb = sim.step(iters=100, tol=1e-4, warm=O.LEARNED)
    assert not (rb["flags"][0] & O.F_FELLBACK)
    assert ra["sweeps"][0] == rb["sweeps"][0]
    np.testing.assert_array_equal(sim.pose, pa)
    np.testing.assert_array_equal(sim.vel, va)
    np.testing.assert_array_equal(ra["c_lambda"], rb["c_lambda"])


def test_learned_bad_start_rejected_for_cold():
    """Huge impulses on new contacts raise the solver's objective: the
    network's part is dropped (FELLBACK); with every contact new, the step
    is the COLD step."""
    b = custom_batch([[dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=1.0, pos=[0, 0, 0.11], vel=[0, 0, -0.5, 0, 0, 0]),
                       dict(shape=S.BOX, param=[0.1, 0.1, 0.1], mass=2.0, pos=[1, 0, 0.105])]])
    sim = sim_of(b)
    pose, vel, theta = sim.pose.copy(), sim.vel.copy(), sim.theta.copy()
    cache = sim.cache_arrays()
    ra = sim.step(iters=100, tol=1e-6, warm=O.COLD)
    pa, va = sim.pose.copy(), sim.vel.copy()
    sim.set_state(pose, vel, theta, cache)
    sim.set_mlp(_const_net((500.0, 300.0, -200.0)))
    rb = sim.step(iters=100, tol=1e-6, warm=O.LEARNED)
    assert ra["n_contacts"][0] >= 2
    assert rb["flags"][0] & O.F_FELLBACK
    assert ra["sweeps"][0] == rb["sweeps"][0]
    np.testing.assert_array_equal(sim.pose, pa)
    np.testing.assert_array_equal(sim.vel, va)

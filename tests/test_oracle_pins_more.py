"""More pins of the FP64 oracle: each one fixes a part of the step that a
plausible slip would otherwise leave unnoticed (a wrong inertia formula, a
missing Jacobi scale, friction carried over without re-projection, a wrong
speculative or restitution bias, the wrong box corners or box-box points,
a feature computed from the wrong quantity).  Expected values come from
closed forms, numerical quadrature and hand-derived geometry written out
below; none calls the oracle's arithmetic.  CPU only.
"""
import math

import numpy as np

from helpers import DT, G, S, custom_batch, inertia, quat_axis_angle, quat_to_R
from oracle import oracle as O

ZERO_G = (0.0, 0.0, 0.0)


def _pose(b, i):
    p = b.pose.astype(np.float64)[i]
    return p[:3].copy(), p[3:].copy()


def _world_inv_inertia(b, i):
    """R diag(1/I) R^T with the principal moments I from quadrature and R
    from the stored (float32, so not exactly unit) quaternion, as the step
    uses it."""
    x, q = _pose(b, i)
    R = quat_to_R(q)
    I = inertia(int(b.shape[i]), b.param[i].astype(np.float64), float(b.mass[i]))
    return R @ np.diag(1.0 / I) @ R.T


def _lowest_corner_at(half, q, depth):
    """Centre height that puts the lowest corner of a box (half-extents,
    orientation q) at z = -depth; also returns the sorted corner heights
    relative to the centre."""
    R = quat_to_R(q)
    zs = sorted((R @ (np.array([(k & 1) * 2 - 1, (k >> 1 & 1) * 2 - 1, (k >> 2 & 1) * 2 - 1]) * half))[2]
                for k in range(8))
    return -depth - zs[0], zs


# ------------------------------------------------------------ inertia
def _check_angular_response(shape, param, q, mass):
    """One frictionless corner (or cap) contact in zero gravity: the solve
    applies the impulse P at the contact point, so the final angular
    velocity is w = I_w^-1 (r x P) with the inertia from quadrature."""
    half = np.asarray(param, np.float64)
    if shape == S.BOX:
        zc, zs = _lowest_corner_at(half, q, 0.001)
        assert zs[1] - zs[0] > 0.05            # a single corner within the margin
    else:
        R = quat_to_R(q)
        ends = [(R @ np.array([0, 0, s * half[1]]))[2] for s in (-1, 1)]
        zc = -0.001 + half[0] - min(ends)
        assert abs(ends[0] - ends[1]) > 0.05
    b = custom_batch([[dict(shape=shape, param=param, mass=mass, mu=0.0, pos=[0.2, -0.1, zc], quat=q,
                            vel=[0.0, 0.0, -1.0, 0.0, 0.0, 0.0])]])
    sim = O.OracleSim(b, gravity=ZERO_G, ground_friction=0.0)
    x0, _ = _pose(b, 0)
    Iinv = _world_inv_inertia(b, 0)
    r = sim.step(iters=20)
    assert r["n_contacts"][0] == 1
    n = r["c_normal"][0, 0]
    P = r["c_lambda"][0, 0, 0] * n
    assert r["c_lambda"][0, 0, 0] > 0.05
    arm = r["c_point"][0, 0] - x0
    v = sim.vel.reshape(-1, 6)[0]
    np.testing.assert_allclose(v[:3] - np.array([0.0, 0.0, float(b.vel[0, 2])]), P / float(b.mass[0]),
                               rtol=0, atol=1e-12)
    expect = Iinv @ np.cross(arm, P)
    assert np.linalg.norm(v[3:] - expect) <= 1e-11 * np.linalg.norm(expect), (v[3:], expect)


def test_box_inertia_against_quadrature():
    q = quat_axis_angle([1.0, 2.0, 0.5], 0.7)
    _check_angular_response(S.BOX, [0.1, 0.2, 0.3], q, 2.0)


def test_capsule_inertia_against_quadrature():
    q = quat_axis_angle([1.0, 0.3, 0.0], 0.9)
    _check_angular_response(S.CAPSULE, [0.07, 0.15, 0.0], q, 1.3)


# ------------------------------------------------------------ Jacobi scale
def test_jacobi_first_sweep_flat_box_quarter_scale():
    """A flat box on 4 corner contacts, falling at 1 m/s in zero gravity, no
    bias (all depths inside the slop), no tangential motion.  One Jacobi
    sweep reads the sweep-start velocity for every contact, so each normal
    impulse is (1/4) m_n (0 - u) with u = -1 and m_n = 1 / (1/m + r_y^2/I_x +
    r_x^2/I_y) (the corner lever arms of an axis-aligned box); the 4 equal
    impulses leave the box at v_z = -1 + m_n / m and no spin."""
    hx, hy, hz, m = 0.2, 0.1, 0.05, 1.5
    b = custom_batch([[dict(shape=S.BOX, param=[hx, hy, hz], mass=m, pos=[0.0, 0.0, hz - 0.002],
                            vel=[0.0, 0.0, -1.0, 0.0, 0.0, 0.0])]])
    sim = O.OracleSim(b, gravity=ZERO_G)
    r = sim.step(iters=1, solver=O.JACOBI)
    assert r["n_contacts"][0] == 4
    m = float(b.mass[0])
    I = inertia(S.BOX, b.param[0].astype(np.float64), m)
    x0, _ = _pose(b, 0)
    for k in range(4):
        arm = r["c_point"][0, k] - x0
        kn = 1.0 / m + arm[1] ** 2 / I[0] + arm[0] ** 2 / I[1]
        assert abs(r["c_lambda"][0, k, 0] - 0.25 / kn * 1.0) < 1e-12
    arm = r["c_point"][0, 0] - x0
    mn = 1.0 / (1.0 / m + arm[1] ** 2 / I[0] + arm[0] ** 2 / I[1])
    v = sim.vel.reshape(-1, 6)[0]
    assert abs(v[2] - (-1.0 + mn / m)) < 1e-12
    assert np.abs(v[3:]).max() < 1e-12 and np.abs(v[:2]).max() < 1e-12


# ------------------------------------------------------------ PREV friction re-projection
def test_prev_friction_reprojected_on_new_normal():
    """The cache keeps a contact's friction impulse as a world vector F.  A
    contact whose normal n differs from the one F was stored under starts
    from the normal impulse plus the part of F in the new tangent plane,
    F - (F.n) n: with no sweeps the sphere's velocity changes by exactly
    (lambda_n n + F - (F.n) n) / m."""
    tilt = quat_axis_angle([1.0, 0.0, 0.0], 0.3)
    R = quat_to_R(tilt)
    nf = R @ np.array([0.0, 0.0, 1.0])
    rs, m = 0.1, 2.0
    centre = R @ np.array([0.0, 0.05, 0.1]) + nf * (rs - 0.001)
    bodies = [dict(shape=S.SPHERE, param=[rs, 0, 0], mass=m, mu=0.8, pos=centre),
              dict(shape=S.BOX, motion=S.STATIC, param=[1.0, 1.0, 0.1], mass=0.0, mu=0.8, pos=[0, 0, 0], quat=tilt)]
    b = custom_batch([bodies])
    sim = O.OracleSim(b, gravity=ZERO_G)
    pose0, vel0 = sim.pose.copy(), sim.vel.copy()
    r = sim.step(iters=0)
    assert r["n_contacts"][0] == 1
    key = int(r["c_key"][0, 0])
    assert key == (0 << 20) | (1 << 8) | 0
    n = r["c_normal"][0, 0]
    _, qs = _pose(b, 1)
    np.testing.assert_allclose(n, quat_to_R(qs) @ np.array([0.0, 0.0, 1.0]), atol=1e-12)
    lam_n, F = 0.5, np.array([0.1, -0.2, 0.15])
    cache = (np.array([1], np.int32), np.array([[key]], np.uint32), np.array([[[lam_n, *F]]]))
    sim.set_state(pose0.reshape(-1, 7), vel0.reshape(-1, 6), cache=cache)
    r = sim.step(iters=0, warm=O.PREV)
    Ft = F - np.dot(F, n) * n
    assert np.linalg.norm(Ft) < 0.8 * lam_n            # inside the friction cone: no projection
    dv = sim.vel.reshape(-1, 6)[0, :3] - vel0.reshape(-1, 6)[0, :3]
    # the box's stored quaternion is float32, so n is unit only to ~1e-8:
    # the tangent basis built from it projects F to that level
    np.testing.assert_allclose(dv, (lam_n * n + Ft) / float(b.mass[0]), rtol=0, atol=1e-9)
    assert abs(r["c_lambda"][0, 0, 0] - lam_n) < 1e-15
    assert abs(math.hypot(r["c_lambda"][0, 0, 1], r["c_lambda"][0, 0, 2]) - np.linalg.norm(Ft)) < 1e-9


# ------------------------------------------------------------ speculative contact
def test_speculative_contact_lands_at_zero_separation():
    """A sphere phi = 1.5 cm above the plane (inside the 2 cm margin) falling
    at 3 m/s: the speculative bias -phi/dt lets it approach exactly until it
    touches, v_z = -phi/dt and the next separation is 0.  Falling at 1 m/s it
    does not reach the plane within the step and no impulse acts."""
    r0, phi = 0.1, 0.015
    for vz, hits in ((-3.0, True), (-1.0, False)):
        b = custom_batch([[dict(shape=S.SPHERE, param=[r0, 0, 0], mass=1.0, pos=[0, 0, r0 + phi],
                                vel=[0, 0, vz, 0, 0, 0])]])
        sim = O.OracleSim(b, gravity=ZERO_G)
        z0 = float(b.pose[0, 2])
        ph = z0 - float(b.param[0, 0])
        res = sim.step(iters=10)
        assert res["n_contacts"][0] == 1
        v = sim.vel.reshape(-1, 6)[0, 2]
        z = sim.pose.reshape(-1, 7)[0, 2]
        if hits:
            assert abs(v - (-ph / DT)) < 1e-12
            assert abs((z - float(b.param[0, 0]))) < 1e-12
        else:
            assert res["c_lambda"][0, 0, 0] == 0.0
            assert v == float(b.vel[0, 2])


# ------------------------------------------------------------ restitution
def test_restitution_bounce_and_threshold():
    """e = 0.5 against the plane (restitution 0, combined by the maximum):
    approaching at 2 m/s with the depth inside the slop the sphere leaves at
    e |u0| = 1 m/s; at 0.4 m/s (below the 0.5 m/s threshold) it stops.  With
    10 mm beyond the slop the target is max(Baumgarte, e |u0|)."""
    beta, slop = 0.2, 0.005
    cases = [(-2.0, 0.002, 1.0), (-0.4, 0.002, 0.0), (-2.0, 0.025, None), (-0.6, 0.025, None)]
    for vz, depth, expect in cases:
        b = custom_batch([[dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=1.0, e=0.5, pos=[0, 0, 0.1 - depth],
                                vel=[0, 0, vz, 0, 0, 0])]])
        sim = O.OracleSim(b, gravity=ZERO_G)
        ph = float(b.pose[0, 2]) - float(b.param[0, 0])
        u0 = float(b.vel[0, 2])
        if expect is None:
            e_part = -0.5 * u0 if u0 < -0.5 else 0.0
            expect = max(beta / DT * max(0.0, -ph - slop), e_part)
        sim.step(iters=10)
        assert abs(sim.vel.reshape(-1, 6)[0, 2] - expect) < 1e-12, (vz, depth)


# ------------------------------------------------------------ box on the plane, > 4 corners
def test_thin_box_keeps_four_deepest_corners():
    """A 1 cm thick box tilted 0.05 rad about x with all 8 corners inside the
    margin: the corners on the -y side are the deepest (their height is
    zc - hy sin(t) -+ hz cos(t), and hy sin(t) > hz cos(t)), so corners 0, 1,
    4 and 5 (bit 1 clear) are kept, each at its own height, the contact point
    halfway between the corner and the plane."""
    half = np.array([0.3, 0.2, 0.005])
    q = quat_axis_angle([1.0, 0.0, 0.0], 0.05)
    zc = 0.003
    cs, amb = O.collide(S.BOX, half, [0.0, 0.0, zc, *q])
    assert amb == 0
    R = quat_to_R(q)
    corner = {k: np.array([0, 0, zc]) + R @ (np.array([(k & 1) * 2 - 1, (k >> 1 & 1) * 2 - 1, (k >> 2 & 1) * 2 - 1]) * half)
              for k in range(8)}
    assert all(c[2] <= 0.02 for c in corner.values())
    assert sorted(f for f, _, _, _ in cs) == [0, 1, 4, 5]
    for f, n, p, phi in cs:
        np.testing.assert_allclose(n, [0, 0, 1], atol=0)
        assert abs(phi - corner[f][2]) < 1e-15
        np.testing.assert_allclose(p, [corner[f][0], corner[f][1], 0.5 * corner[f][2]], atol=1e-15)


# ------------------------------------------------------------ capsule core inside a box
def test_capsule_core_inside_box_leaves_through_nearest_face():
    """A horizontal capsule (r 5 cm, core half-length 10 cm along x) whose
    core lies 2 cm under the top face of a 1 x 1 x 0.2 m box: the least
    translation is through the top face (2 cm, against 18 cm for the bottom
    and 48 cm or more for the sides), so the contacts are the core's ends
    clipped to that face, normal +z, depth 2 cm + r.  In the second case the
    core pokes out of the +x side and the clipped end lies on the face edge."""
    qx = quat_axis_angle([0.0, 1.0, 0.0], math.pi / 2)   # capsule axis along x
    r, h = 0.05, 0.1
    for cx, ends in ((0.05, (-0.05, 0.15)), (0.45, (0.35, 0.5))):
        cs, amb = O.collide(S.CAPSULE, [r, h, 0.0], [cx, 0.02, 0.08, *qx],
                            S.BOX, [0.5, 0.5, 0.1], [0, 0, 0, 1, 0, 0, 0])
        assert amb == 0
        assert [f for f, _, _, _ in cs] == [0, 1]
        for (f, n, p, phi), xe in zip(cs, ends):
            np.testing.assert_allclose(n, [0, 0, 1], atol=1e-15)
            assert abs(phi - (0.08 - 0.1 - r)) < 1e-15
            # midpoint of the core end's surface point (z 0.08 - r) and its projection on the face (z 0.1)
            np.testing.assert_allclose(p, [xe, 0.02, 0.5 * ((0.08 - r) + 0.1)], atol=1e-12)


# ------------------------------------------------------------ box-box 4-point reduction
def test_box_box_reduction_hand_derived():
    """Box b (half 0.2, yawed 30 deg, centre (0.3, 0, 0.199)) rests on box a
    (half 0.5 x 0.5 x 0.1, at the origin) 1 mm deep.  a's top face is the
    reference (face index 4 = axis z, + side); b's bottom face is incident
    with corners, in the face's order, P0 = c + e1 + e2, P1 = c - e1 + e2,
    P2 = c - e1 - e2, P3 = c + e1 - e2 (e1, e2 = b's x and y half-axes).  Only
    P3 crosses a side plane (x = 0.5), so clipping gives, in order,
    [I30, P0, P1, P2, I23] (I = where an edge meets x = 0.5).  Reduction:
    the first point I30; the farthest from it, P1; the largest triangle with
    those two, P2; of the last two, P0 adds more area (0.051 against 0.023
    for I23).  Kept: clip indices 0-3, feature (4 << 1) | (index << 4)."""
    yaw = quat_axis_angle([0.0, 0.0, 1.0], math.radians(30.0))
    cb = np.array([0.3, 0.0, 0.199])
    cs, amb = O.collide(S.BOX, [0.5, 0.5, 0.1], [0, 0, 0, 1, 0, 0, 0], S.BOX, [0.2, 0.2, 0.1], [*cb, *yaw])
    assert amb == 0
    R = quat_to_R(yaw)
    c = cb - np.array([0.0, 0.0, 0.1])
    e1, e2 = R[:, 0] * 0.2, R[:, 1] * 0.2
    P = [c + e1 + e2, c - e1 + e2, c - e1 - e2, c + e1 - e2]

    def cut(p, q):   # point of segment pq at x = 0.5
        t = (0.5 - p[0]) / (q[0] - p[0])
        return p + t * (q - p)

    clip = [cut(P[3], P[0]), P[0], P[1], P[2], cut(P[2], P[3])]
    # the derivation's distinctions are clear-cut
    d = [np.linalg.norm(x - clip[0]) for x in clip]
    assert int(np.argmax(d)) == 2 and sorted(d)[-1] - sorted(d)[-2] > 0.04
    assert [f for f, _, _, _ in cs] == [(4 << 1) | (k << 4) for k in range(4)]
    for (f, n, p, phi), x in zip(cs, clip[:4]):
        np.testing.assert_allclose(n, [0, 0, -1], atol=1e-15)     # from b to a
        assert abs(phi - (-0.001)) < 1e-12
        np.testing.assert_allclose(p, [x[0], x[1], 0.099 + 0.0005], atol=1e-12)


# ------------------------------------------------------------ features 0-14
def test_features_hand_computed():
    """The 16 features of two contacts, computed here from their definitions.
    Scene 0: a spinning box on one corner with a cached impulse (a persisting
    contact).  Scene 1: a sphere resting off-centre on a box that rests on
    the plane (a new contact between two dynamic bodies).  For the normal
    +z the tangent basis of Duff et al. 2017 is t1 = +x, t2 = +y."""
    q = quat_axis_angle([1.0, 2.0, 0.5], 0.7)
    half = np.array([0.1, 0.2, 0.3])
    zc, _ = _lowest_corner_at(half, q, 0.001)
    v0 = np.array([0.3, -0.2, -0.5, 0.4, 0.1, -0.3])
    scene0 = [dict(shape=S.BOX, param=half, mass=2.0, mu=0.6, pos=[0.1, 0.2, zc], quat=q, vel=v0)]
    scene1 = [dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=0.7, mu=0.3, pos=[0.15, -0.05, 0.298],
                   vel=[0.05, 0.0, -0.1, 0.0, 0.2, 0.0]),
              dict(shape=S.BOX, param=[0.3, 0.2, 0.1], mass=1.9, mu=0.9, pos=[0.0, 0.0, 0.099],
                   vel=[0.0, 0.02, 0.0, 0.1, 0.0, 0.05])]
    b = custom_batch([scene0, scene1])
    sim = O.OracleSim(b)
    # cached impulse for scene 0's corner: find the corner index first
    R = quat_to_R(b.pose[0, 3:].astype(np.float64))
    x0 = b.pose[0, :3].astype(np.float64)
    corners = [x0 + R @ (np.array([(k & 1) * 2 - 1, (k >> 1 & 1) * 2 - 1, (k >> 2 & 1) * 2 - 1]) * b.param[0].astype(np.float64))
               for k in range(8)]
    kc = int(np.argmin([c_[2] for c_ in corners]))
    key0 = (0 << 20) | (0xFFF << 8) | kc
    lam_prev = np.array([0.3, 0.05, 0.02, 0.01])
    cnt = np.array([1, 0], np.int32)
    keys = np.zeros((2, 1), np.uint32)
    keys[0, 0] = key0
    lams = np.zeros((2, 1, 4))
    lams[0, 0] = lam_prev
    sim.set_state(sim.pose.copy().reshape(-1, 7), sim.vel.copy().reshape(-1, 6), cache=(cnt, keys, lams))
    res = sim.step(iters=10, warm=O.PREV)
    gdt = G * DT

    # scene 0
    assert res["n_contacts"][0] == 1 and int(res["c_key"][0, 0]) == key0
    f = res["c_feat"][0, 0]
    c = corners[kc]
    p = np.array([c[0], c[1], 0.5 * c[2]])
    arm = p - x0
    v = b.vel[0].astype(np.float64)
    lin = v[:3] + np.array([0.0, 0.0, -gdt])
    vr = lin + np.cross(v[3:], arm)
    m = float(b.mass[0])
    Iinv = _world_inv_inertia(b, 0)
    can = np.cross(arm, [0.0, 0.0, 1.0])
    kn = 1.0 / m + can @ Iinv @ can
    unit = gdt / kn
    expect = [vr[2], vr[0], vr[1], -c[2], 1.0 / m, 0.0, can @ Iinv @ can, 0.0,
              lam_prev[0] / unit, lam_prev[1] / unit, lam_prev[2] / unit, 0.0, 0.0, 1.0,
              math.sqrt(float(b.friction[0]) * 0.5), 0.0]
    np.testing.assert_allclose(f, expect, rtol=1e-12, atol=1e-13)

    # scene 1: the sphere-box contact (sphere a = 0, box b = 1, feature 0)
    nc = res["n_contacts"][1]
    ks = [int(k) for k in res["c_key"][1, :nc]]
    i = ks.index((0 << 20) | (1 << 8) | 0)
    assert nc == 5                                     # 4 box corners on the plane + the sphere
    f = res["c_feat"][1, i]
    xs, xb = b.pose[1, :3].astype(np.float64), b.pose[2, :3].astype(np.float64)
    rs = float(b.param[1, 0])
    top = xb[2] + float(b.param[2, 2])
    p = np.array([xs[0], xs[1], 0.5 * ((xs[2] - rs) + top)])
    ra, rb = p - xs, p - xb
    va, vb = b.vel[1].astype(np.float64), b.vel[2].astype(np.float64)
    vr = (va[:3] + [0, 0, -gdt] + np.cross(va[3:], ra)) - (vb[:3] + [0, 0, -gdt] + np.cross(vb[3:], rb))
    ma, mb = float(b.mass[1]), float(b.mass[2])
    Ia, Ib = _world_inv_inertia(b, 1), _world_inv_inertia(b, 2)
    z = np.array([0.0, 0.0, 1.0])
    ca, cb = np.cross(ra, z), np.cross(rb, z)
    expect = [vr[2], vr[0], vr[1], -((xs[2] - rs) - top), 1.0 / ma, 1.0 / mb, ca @ Ia @ ca, cb @ Ib @ cb,
              0.0, 0.0, 0.0, 0.0, 0.0, 1.0, math.sqrt(float(b.friction[1]) * float(b.friction[2])), 1.0 / 5.0]
    np.testing.assert_allclose(f, expect, rtol=1e-12, atol=1e-13)

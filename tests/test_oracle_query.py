"""Pins of the oracle's arm collision queries (motion planning, Sec. 4.5 and
App. C: a sampling planner checks the arm against the scene at each visited
configuration).  Each check is independent of the oracle's formulas:
closed-form separations of a straight or folded arm from a sphere, a shelf
and the ground, the arm's own links left out, and a brute-force distance
(the link's core segment sampled densely, point-to-shape distances of the
test's own) on random configurations among random obstacles."""
import math

import numpy as np
import pytest

from helpers import S, custom_batch
from oracle import oracle as O

R_LINK = S.ARM_RADIUS
BASE_Z = float(np.float32(S.ARM_BASE[2]))
LEN = [float(L) for L in S.ARM_LINK_LENGTH]


def arm_scene(bodies):
    b = custom_batch([bodies], arm=True)
    return O.OracleSim(b)


def one(ora, theta, clearance):
    h, p, a = ora.arm_query(np.asarray(theta, np.float64).reshape(1, -1, 7), clearance)
    return h[0], p[0], a[0]


def test_sphere_beside_straight_arm_closed_form():
    # straight-up arm: link 1 spans z in [0.9, 1.2] on the z axis; a sphere of
    # radius r at (x0, 0, 1.05) is x0 - R_LINK - r from it
    r = 0.1
    for x0 in (0.16, 0.15 + 1e-3, 0.2, 0.3, 0.149):
        ora = arm_scene([dict(shape=S.SPHERE, motion=S.STATIC, param=[r, 0, 0], pos=[x0, 0.0, 1.05])])
        x0f, rf = float(np.float32(x0)), float(np.float32(r))
        phi = x0f - R_LINK - rf
        for c in (0.0, 0.02, 0.1):
            h, p, a = one(ora, np.zeros(7), c)
            assert h[0] == (phi <= c)
            if phi <= c:
                assert abs(p[0] - phi) < 1e-9
            else:
                assert p[0] == np.inf or p[0] > c


def test_shelf_above_and_ground_below_closed_form():
    # straight-up arm top at z = BASE_Z + sum(LEN) + R_LINK; a shelf (static
    # box, half height 0.05) whose bottom face is `gap` above it
    top = BASE_Z + sum(LEN) + R_LINK
    for gap in (-0.01, 0.005, 0.03):
        cz = top + gap + 0.05
        ora = arm_scene([dict(shape=S.BOX, motion=S.STATIC, param=[0.5, 0.5, 0.05], pos=[0.0, 0.0, cz])])
        h, p, _ = one(ora, np.zeros(7), 0.02)
        czf = float(np.float32(cz))
        phi = (czf - float(np.float32(0.05))) - top
        assert h[0] == (phi <= 0.02)
        if phi <= 0.02:
            assert abs(p[0] - phi) < 1e-6
    # folded straight down by joint 1: the tip is at BASE_Z + LEN[0] - sum(LEN[1:])
    ora = arm_scene([])
    th = np.zeros((3, 7))
    th[1, 1] = math.pi
    th[2, 1] = math.pi / 2           # horizontal at z = BASE_Z + LEN[0]
    h, p, _ = one(ora, th, 0.0)
    tip = BASE_Z + LEN[0] - sum(LEN[1:])
    assert list(h) == [0, 1, 0]
    assert abs(p[1] - (tip - R_LINK)) < 1e-7      # float32 capsule half-lengths
    # at a wide clearance the lowest point of a horizontal arm is link 0's
    # lower end at the base, BASE_Z - R_LINK above the floor
    h, p, _ = one(ora, th, 0.9)
    assert h[2] == 1 and abs(p[2] - (BASE_Z - R_LINK)) < 1e-7


def test_arm_links_are_not_obstacles_and_empty_queries():
    ora = arm_scene([])
    h, p, a = one(ora, np.zeros((4, 7)), 0.0)
    assert not h.any() and np.all(p == np.inf) and not a.any()
    h, p, a = ora.arm_query(np.zeros((1, 0, 7)), 0.0)
    assert h.shape == (1, 0)
    with pytest.raises(ValueError):
        ora.arm_query(np.zeros((1, 2, 7)), -1.0)


def test_tie_band_reported():
    r = 0.1
    ora = arm_scene([dict(shape=S.SPHERE, motion=S.STATIC, param=[r, 0, 0], pos=[0.2, 0.0, 1.05])])
    phi = float(np.float32(0.2)) - R_LINK - float(np.float32(r))
    _, _, a = one(ora, np.zeros(7), phi + 3e-6)
    assert a[0] == 1
    _, _, a = one(ora, np.zeros(7), phi + 1e-3)
    assert a[0] == 0


# ---- brute force: sampled link cores against the test's own distances ----
def quat_R(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def point_seg_dist(p, a, b):
    d = b - a
    t = np.clip(((p - a) @ d) / max(d @ d, 1e-300), 0.0, 1.0)
    return np.linalg.norm(p - (a + t[..., None] * d), axis=-1)


def dist_to_obstacle(pts, shape, prm, pose):
    c = pose[:3]
    R = quat_R(pose[3:])
    if shape == S.SPHERE:
        return np.linalg.norm(pts - c, axis=1) - prm[0]
    if shape == S.CAPSULE:
        ax = R[:, 2] * prm[1]
        return point_seg_dist(pts, c - ax, c + ax) - prm[0]
    loc = (pts - c) @ R                       # box frame
    h = np.asarray(prm[:3])
    q = np.abs(loc) - h
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=1)
    inside = np.minimum(q.max(axis=1), 0.0)
    return outside + inside


def link_segments(ora, theta):
    """Link core segments from the pose the oracle itself writes for theta
    (the forward kinematics is pinned by the arm tests of the step)."""
    ora.set_theta(theta)
    pose = ora.pose.reshape(-1, 7)[-7:]
    segs = []
    for k in range(7):
        R = quat_R(pose[k, 3:])
        ax = R[:, 2] * (0.5 * LEN[k])
        segs.append((pose[k, :3] - ax, pose[k, :3] + ax))
    return segs


def test_brute_force_sampled_distances():
    rng = np.random.default_rng(7)
    checked = 0
    for trial in range(6):
        bodies = []
        for i in range(10):
            shape = int(rng.integers(0, 3))
            ang = rng.uniform(0, 2 * math.pi)
            rad = rng.uniform(0.2, 1.0)
            pos = [rad * math.cos(ang), rad * math.sin(ang), rng.uniform(0.2, 2.0)]
            q = rng.normal(size=4)
            q /= np.linalg.norm(q)
            prm = [rng.uniform(0.05, 0.2), rng.uniform(0.05, 0.2), rng.uniform(0.05, 0.2)]
            bodies.append(dict(shape=shape, motion=S.STATIC, param=prm, pos=pos, quat=q))
        b = custom_batch([bodies], arm=True)
        ora = O.OracleSim(b)
        pose0 = ora.pose.copy()
        obs = [(int(b.shape[i]), b.param[i].astype(np.float64), pose0.reshape(-1, 7)[i].copy())
               for i in range(10)]
        thetas = rng.uniform(-math.pi, math.pi, size=(12, 7))
        c = 0.3
        h, p, _ = ora.arm_query(thetas[None], c)
        for j, th in enumerate(thetas):
            segs = link_segments(O.OracleSim(b), th)
            best = math.inf
            penetrating = False
            t = np.linspace(0.0, 1.0, 4001)[:, None]
            for a, bb in segs:
                pts = a + t * (bb - a)
                best = min(best, float(pts[:, 2].min()) - R_LINK)       # ground
                for shape, prm, pose in obs:
                    d = dist_to_obstacle(pts, shape, prm, pose)
                    penetrating |= bool((d < R_LINK).any() and d.min() <= 0)
                    best = min(best, float(d.min()) - R_LINK)
            if penetrating:
                continue                     # the core inside an obstacle: a different reading of depth
            if abs(best - c) > 1e-3:
                assert h[0, j] == (best <= c), (trial, j, best, p[0, j])
            if best <= c - 1e-3:
                assert abs(p[0, j] - best) < 2e-4, (trial, j, best, p[0, j])
                checked += 1
    assert checked >= 10

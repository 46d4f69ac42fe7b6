"""Pins of the oracle's articulated container parts (Sec. 3: doors and
drawers that turn about an axis or slide): one rigid body with one joint
to the world, revolute or prismatic, its coordinate within limits.

Each check is fixed by mechanics, not by the oracle's formulas:
- a flap hanging from a horizontal hinge swings with the period of a
  physical pendulum, 2 pi sqrt(I_o / (m g d)) (I_o from the box's own
  moments and the parallel-axis theorem, in the test);
- a ball striking a door on a vertical hinge: the angular momentum of ball
  and door about the hinge line is the same before and after (neither the
  hinge nor gravity has a moment about it);
- a ball striking a drawer along its slide: the momentum along the slide is
  conserved;
- a joint stops at its limit and never passes it;
- a part and the base it is joined to never collide; the joint coordinate
  stays on the joint (the part's pose is the joint motion of its start)."""
import math

import numpy as np
import pytest

from helpers import DT, G, S
from oracle import oracle as O


def part_batch(bodies, joints):
    """bodies: list of dicts (shape, motion, param, mass, mu, pos, quat, vel);
    joints: {body index: (kind, axis, anchor, (lo, hi), parent)}."""
    sc = S.Scene()
    vels = []
    for b in bodies:
        sc.add(b.get("shape", S.BOX), b.get("motion", S.DYNAMIC), b["param"], b.get("mass", 1.0), b.get("mu", 0.5),
               0.0, b["pos"], b.get("quat", (1.0, 0.0, 0.0, 0.0)))
        vels.append(np.asarray(b.get("vel", np.zeros(6)), np.float64))
    sc.joints = dict(joints)
    bt = S.pack([sc])
    bt.vel = np.asarray(vels, np.float32)
    return bt


def box_inertia(h, m):
    """Principal moments of a solid box of half-extents h."""
    x2, y2, z2 = h[0] ** 2, h[1] ** 2, h[2] ** 2
    return np.array([m / 3 * (y2 + z2), m / 3 * (x2 + z2), m / 3 * (x2 + y2)])


def test_flap_swings_with_the_pendulum_period():
    """A 2 kg flap (half-extents 0.3 x 0.02 x 0.2 m) hanging from a hinge
    along x at its top edge, started at 0.05 rad/s: its small-oscillation
    period matches the physical pendulum to 0.5%."""
    h, m = np.array([0.3, 0.02, 0.2]), 2.0
    top = np.array([0.0, 0.0, 1.5])
    flap = dict(param=h, mass=m, pos=top - [0.0, 0.0, h[2]])
    bt = part_batch([flap], {0: (1, (1.0, 0.0, 0.0), top, (-3.0, 3.0), -1)})
    ora = O.OracleSim(bt)
    ora.q_rate[0] = 0.05
    qs = []
    for t in range(1200):
        ora.step(iters=20, warm=O.PREV, outputs=False)
        qs.append(ora.q[0])
    qs = np.array(qs)
    up = np.nonzero((qs[:-1] < 0) & (qs[1:] >= 0))[0]          # upward zero crossings
    frac = up + (-qs[up]) / (qs[up + 1] - qs[up])
    period = np.mean(np.diff(frac)) * DT
    # the batch holds float32 inputs: the flap's own half-extents, mass and
    # hinge offset as stored
    h, m = bt.param[0].astype(np.float64), float(bt.mass[0])
    top = bt.joint_anchor[0].astype(np.float64)
    d = top[2] - float(bt.pose[0, 2])
    I_o = box_inertia(h, m)[0] + m * d * d
    want = 2 * math.pi * math.sqrt(I_o / (m * G * d))
    assert len(up) >= 3
    assert abs(period / want - 1) < 5e-3, (period, want)
    # and the flap stays on its hinge: the centre keeps its distance d from the hinge line
    c = ora.pose.reshape(-1, 7)[0, :3]
    assert abs(np.hypot(c[1] - top[1], c[2] - top[2]) - d) < 1e-9


def door_and_ball(vball, door_mass=5.0):
    """A door (half-extents 0.02 x 0.4 x 0.9 m) on a vertical hinge at its
    edge x = 0, y = 0; a ball flying at it from +x below its middle; no
    gravity, so that the ball never meets the floor (whose friction would
    have a moment about the hinge line)."""
    hd = np.array([0.02, 0.4, 0.9])
    door = dict(param=hd, mass=door_mass, pos=[0.0, hd[1], 1.0])
    ball = dict(shape=S.SPHERE, param=[0.08, 0, 0], mass=0.6, mu=0.3, pos=[0.3, 0.6, 0.9], vel=[vball, 0, 0, 0, 0, 0])
    bt = part_batch([door, ball], {0: (1, (0.0, 0.0, 1.0), (0.0, 0.0, 1.0), (-2.0, 2.0), -1)})
    return bt, O.OracleSim(bt, gravity=(0.0, 0.0, 0.0)), hd, door_mass


def hinge_momentum(bt, ora):
    """Angular momentum about the vertical hinge line through (0, 0): the
    door's I_o qd plus the ball's (r x m v) . z and its spin (the batch's
    float32 sizes and masses)."""
    hd, md = bt.param[0].astype(np.float64), float(bt.mass[0])
    off = float(bt.pose[0, 1]) - float(bt.joint_anchor[0, 1])
    I_o = box_inertia(hd, md)[2] + md * off ** 2
    mb, rb = float(bt.mass[1]), float(bt.param[1, 0])
    p = ora.pose.reshape(-1, 7)
    v = ora.vel.reshape(-1, 6)
    r = p[1, :3]
    Lb = mb * (r[0] * v[1, 1] - r[1] * v[1, 0])
    Ib = 0.4 * mb * rb ** 2
    return I_o * ora.q_rate[0] + Lb + Ib * v[1, 5]


def test_ball_on_door_conserves_hinge_momentum():
    bt, ora, hd, md = door_and_ball(-3.0)
    L0 = hinge_momentum(bt, ora)
    hit = False
    for t in range(60):
        r = ora.step(iters=200, tol=1e-12, warm=O.PREV)
        hit |= int(r["n_contacts"][0]) > 0 and np.any((r["c_key"][0, :int(r["n_contacts"][0])] >> 8 & 0xFFF) == 1)
        np.testing.assert_allclose(hinge_momentum(bt, ora), L0, rtol=1e-9, atol=1e-12)
    assert hit and ora.q_rate[0] > 0.05   # the door swung away from the ball (positive about +z)


def test_ball_on_drawer_conserves_slide_momentum():
    """A drawer (half-extents 0.25 x 0.3 x 0.1 m, 3 kg) sliding along x, struck
    along -x by a ball: m_ball v_x + m_drawer qd is conserved."""
    drawer = dict(param=[0.25, 0.3, 0.1], mass=3.0, pos=[0.0, 0.0, 0.8])
    ball = dict(shape=S.SPHERE, param=[0.06, 0, 0], mass=0.4, mu=0.3, pos=[0.5, 0.02, 0.82], vel=[-2.5, 0, 0, 0, 0, 0])
    bt = part_batch([drawer, ball], {0: (2, (1.0, 0.0, 0.0), (0.0, 0.0, 0.8), (-0.5, 0.5), -1)})
    ora = O.OracleSim(bt, gravity=(0.0, 0.0, 0.0))
    mb, md = float(bt.mass[1]), float(bt.mass[0])
    P0 = mb * ora.vel.reshape(-1, 6)[1, 0] + md * ora.q_rate[0]
    for t in range(40):
        ora.step(iters=200, tol=1e-12, warm=O.PREV, outputs=False)
        P = mb * ora.vel.reshape(-1, 6)[1, 0] + md * ora.q_rate[0]
        np.testing.assert_allclose(P, P0, rtol=1e-9, atol=1e-12)
    assert ora.q_rate[0] < -0.1
    # the drawer only slides: its orientation and its y, z stay put
    p = ora.pose.reshape(-1, 7)[0]
    np.testing.assert_allclose(p[1:3], bt.pose[0, 1:3], atol=1e-12)
    np.testing.assert_allclose(p[3:], [1.0, 0.0, 0.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(p[0], float(bt.pose[0, 0]) + ora.q[0], atol=1e-12)


@pytest.mark.parametrize("kind", [1, 2])
def test_joint_stops_at_its_limit(kind):
    """Started towards its upper limit (0.3 rad or 0.1 m), the part stops
    there: the coordinate never passes it and rests on it."""
    body = dict(param=[0.02, 0.3, 0.5], mass=2.0, pos=[0.0, 0.3, 1.0])
    axis = (0.0, 0.0, 1.0) if kind == 1 else (0.0, 1.0, 0.0)
    bt = part_batch([body], {0: (kind, axis, (0.0, 0.0, 1.0), (-0.2, 0.3 if kind == 1 else 0.1), -1)})
    ora = O.OracleSim(bt, gravity=(0.0, 0.0, 0.0))
    ora.q_rate[0] = 1.5
    hi = float(bt.joint_limits[0, 1])
    for t in range(60):
        ora.step(iters=50, tol=1e-12, warm=O.PREV, outputs=False)
        assert ora.q[0] <= hi + 1e-12
    assert abs(ora.q[0] - hi) < 1e-12 and abs(ora.q_rate[0]) < 1e-9


def test_part_and_its_base_never_collide():
    """A door hinged at the edge of a static cabinet it touches: no contact
    between them; with the parent index unset they would collide."""
    cab = dict(motion=S.STATIC, param=[0.3, 0.3, 0.5], pos=[0.3, -0.3, 0.5], mass=0.0)
    door = dict(param=[0.02, 0.3, 0.5], mass=2.0, pos=[0.0, 0.3, 0.5])
    for parent, want_contacts in ((0, False), (-1, True)):
        bt = part_batch([cab, door], {1: (1, (0.0, 0.0, 1.0), (0.0, 0.0, 0.5), (-1.5, 1.5), parent)})
        ora = O.OracleSim(bt, gravity=(0.0, 0.0, 0.0))
        ora.q_rate[1] = -0.5   # swing it into the cabinet's side
        seen = False
        for t in range(30):
            r = ora.step(iters=50, warm=O.PREV)
            keys = r["c_key"][0, :int(r["n_contacts"][0])]
            seen |= bool(np.any(((keys >> 20) == 0) & ((keys >> 8 & 0xFFF) == 1)))
        assert seen == want_contacts


def test_parts_refuse_jacobi_and_learned():
    door = dict(param=[0.02, 0.3, 0.5], mass=2.0, pos=[0.0, 0.3, 1.0])
    bt = part_batch([door], {0: (1, (0.0, 0.0, 1.0), (0.0, 0.0, 1.0), (-1.0, 1.0), -1)})
    ora = O.OracleSim(bt)
    with pytest.raises(ValueError):
        ora.step(iters=10, solver=O.JACOBI)


def test_parts_keep_their_islands_awake():
    """Sleeping on: a box resting on a closed drawer never sleeps (the part
    keeps its island awake), a box on the floor far away does."""
    drawer = dict(param=[0.25, 0.3, 0.1], mass=3.0, pos=[0.0, 0.0, 0.5])
    on_drawer = dict(param=[0.05, 0.05, 0.05], mass=0.5, pos=[0.0, 0.0, 0.6 + 0.05 - 0.001])
    far = dict(param=[0.05, 0.05, 0.05], mass=0.5, pos=[1.5, 1.5, 0.049])
    bt = part_batch([drawer, on_drawer, far], {0: (2, (1.0, 0.0, 0.0), (0.0, 0.0, 0.5), (-0.2, 0.2), -1)})
    ora = O.OracleSim(bt)
    ora.set_sleep(0.02, 30)
    for t in range(150):
        ora.step(iters=100, tol=1e-9, warm=O.PREV, outputs=False)
    assert ora.rest[1] >= 30 and ora.rest[2] >= 30      # both at rest long enough
    r = ora.step(iters=100, tol=1e-9, warm=O.PREV)
    n = int(r["n_contacts"][0])
    col = r["c_colour"][0, :n]
    keys = r["c_key"][0, :n]
    a, b = keys >> 20, (keys >> 8) & 0xFFF
    far_c, top_c = (a == 2) | (b == 2), (a == 1) | (b == 1)
    assert far_c.any() and top_c.any()
    assert np.all(col[far_c] == -1), "the far box should sleep"
    assert np.all(col[top_c] >= 0), "the box on the drawer must stay awake"

"""Pins of the oracle's dynamic arm: one articulated body in reduced
coordinates driven by PD position motors (Sec. 1: articulated robots;
Sec. 5: joint motors, Kp 0.3, at most 10 N s of motor impulse per step).

Each check is fixed by mechanics, not by the oracle's formulas:
- held at rest under gravity, every motor carries the gravity moment of the
  links beyond its joint about its axis (statics of the sub-chain), and with
  a ball resting on the arm the ball's weight as well, and the arm's contact
  force is the ball's weight;
- an unloaded motor closes the fraction Kp of its angle error per step;
- a motor never exceeds its largest impulse, and a weak one saturates;
- swept at up to 1 rad/s with 20 sweeps a step, the arm follows its targets;
- links of one arm never collide with each other, and islands the arm
  touches never sleep."""
import numpy as np
import pytest

from helpers import DT, G, S, custom_batch
from oracle import oracle as O

TH0 = np.array([0.3, -0.4, 0.2, 0.5, -0.3, 0.4, 0.1])
L = np.array(S.ARM_LINK_LENGTH)
M = np.array(S.ARM_LINK_MASS)
HORIZONTAL = np.array([0.0, np.pi / 2, 0.0, 0.0, 0.0, 0.0, 0.0])  # links 1..6 along +x


def arm_only(theta=TH0, bodies=(), **consts):
    b = custom_batch([list(bodies)], arm=2, theta=theta)
    return b, O.OracleSim(b, **consts)


def chain(theta, base=None):
    """Independent forward kinematics: joint origins o_k, axes a_k (world)
    and link centres c_k for joint angles theta (rotation about the parent's
    z for even k, y for odd k; link k runs from o_k along its z) from the
    arm base (the batch's float32 base by default)."""
    def rot(axis, ang):
        c, s = np.cos(ang), np.sin(ang)
        if axis == 2:
            return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])
        return np.array([[c, 0, s], [0, 1.0, 0], [-s, 0, c]])
    R = np.eye(3)
    p = np.array(np.float32(S.ARM_BASE) if base is None else base, np.float64)
    o, a, c = [], [], []
    for k in range(7):
        ax = 2 if k % 2 == 0 else 1
        a.append(R[:, ax].copy())
        R = R @ rot(ax, theta[k])
        o.append(p.copy())
        c.append(p + 0.5 * L[k] * R[:, 2])
        p = p + L[k] * R[:, 2]
    return np.array(o), np.array(a), np.array(c)


def gravity_moments(theta, extra=()):
    """Motor impulses that hold the arm at rest over one step: minus dt times
    the gravity moment about joint k's axis of the links beyond it (and of
    extra point weights (point, mass, last joint that carries it))."""
    o, a, c = chain(theta)
    g = np.array([0.0, 0.0, -G])
    lam = np.zeros(7)
    for k in range(7):
        t = sum(np.cross(c[j] - o[k], M[j] * g) for j in range(k, 7))
        for (p, m, j) in extra:
            if k <= j:
                t = t + np.cross(np.asarray(p) - o[k], m * g)
        lam[k] = -DT * np.dot(a[k], t)
    return lam


def test_link_poses_follow_the_joint_angles():
    """The oracle places the links where the independent chain puts them."""
    b, ora = arm_only()
    _, _, c = chain(b.arm_theta[0].astype(np.float64))   # the batch holds float32 angles
    np.testing.assert_allclose(ora.pose.reshape(-1, 7)[-7:, :3], c, atol=1e-12)


def test_static_equilibrium_motor_impulses():
    _, ora = arm_only()
    for t in range(240):
        ora.step(iters=2000, tol=1e-12, warm=O.PREV, outputs=False)
    th = ora.theta.copy()
    r = ora.step(iters=2000, tol=1e-12, warm=O.PREV)
    assert r["residual"][0] <= 1e-12
    want = gravity_moments(th)
    np.testing.assert_allclose(ora.motor_impulse[0], want, rtol=0, atol=1e-9 * np.abs(want).max())
    np.testing.assert_allclose(ora.theta, TH0, atol=1e-6)
    assert np.abs(ora.qd).max() < 1e-6


def test_unloaded_motor_closes_kp_of_the_error():
    """Zero gravity: joint 3's target moved by 0.01 rad; the error falls by
    the factor 1 - Kp every step, the other joints do not move."""
    _, ora = arm_only(gravity=(0.0, 0.0, 0.0))
    ora.target[0, 3] += 0.01
    err = [ora.target[0, 3] - ora.theta[3]]
    for t in range(6):
        ora.step(iters=500, tol=1e-14, warm=O.PREV, outputs=False)
        err.append(ora.target[0, 3] - ora.theta[3])
        others = np.delete(np.arange(7), 3)
        np.testing.assert_allclose(ora.theta[others], TH0[others], atol=1e-12)
    ratio = np.array(err[1:]) / np.array(err[:-1])
    np.testing.assert_allclose(ratio, 1.0 - 0.3, atol=1e-9)


def test_weak_motors_saturate():
    """Motors of 0.02 N s cannot hold the shoulder (it carries 7.5 kg at up
    to half a metre): its motor impulse sits at the bound, none exceeds it,
    and the arm sags away from its targets."""
    _, ora = arm_only(motor_max=0.02)
    for t in range(30):
        ora.step(iters=200, tol=1e-11, warm=O.PREV, outputs=False)
        lam = ora.motor_impulse[0]
        assert np.all(np.abs(lam) <= 0.02 * (1 + 1e-12))
        assert abs(abs(lam[1]) - 0.02) < 1e-12
    assert np.abs(ora.theta - TH0).max() > 0.05


def test_arm_follows_swept_targets():
    """Targets swept at up to 1 rad/s under gravity with 20 sweeps a step:
    the joints lag their targets by about rate * dt / Kp and stay stable."""
    _, ora = arm_only()
    rates = np.array([1.0, -0.8, 0.6, 0.9, -0.7, 0.5, 1.0])
    worst = 0.0
    for t in range(240):
        a = (rates * np.sin(2 * np.pi * t / 240.0))[None]
        ora.step(actions=a, iters=20, warm=O.PREV, outputs=False)
        worst = max(worst, np.abs(ora.target[0] - ora.theta).max())
    assert worst < 1.5 * np.abs(rates).max() * DT / 0.3 + 1e-3, worst
    assert np.abs(ora.qd).max() < 2.0


def balls_on_arm(dx=(0.0,), **consts):
    """The arm held horizontal, 0.5 kg balls resting on top of link 1 (the
    long upper link, along x), offset dx from its centre; the arm's plane
    is a plane of symmetry, so the balls stay on top."""
    o, a, c = chain(HORIZONTAL)
    balls = [dict(shape=S.SPHERE, param=[0.05, 0.0, 0.0], mass=0.5, mu=0.8,
                  pos=c[1] + np.array([d, 0.0, S.ARM_RADIUS + 0.05 - 0.001])) for d in dx]
    return arm_only(theta=HORIZONTAL, bodies=balls, **consts)


def test_ball_on_arm_reaction():
    """The ball settles on the arm: contacts only between the ball and the
    arm, never between links; the arm's contact force C_t is the ball's
    weight, and the motors carry the ball's moment too."""
    _, ora = balls_on_arm()
    for t in range(240):
        r = ora.step(iters=2000, tol=1e-12, warm=O.PREV)
        n = int(r["n_contacts"][0])
        keys = r["c_key"][0, :n]
        a, bb = keys >> 20, (keys >> 8) & 0xFFF
        assert not np.any((a >= 1) & (bb >= 1) & (bb != 0xFFF)), "contact between two arm links"
    assert np.any((a == 0) & (bb >= 1) & (bb != 0xFFF))
    np.testing.assert_allclose(r["arm_force"][0], 0.5 * G, rtol=1e-6)
    ball = ora.pose.reshape(-1, 7)[0, :3]
    want = gravity_moments(ora.theta, extra=[(ball, 0.5, 1)])
    np.testing.assert_allclose(ora.motor_impulse[0], want, rtol=0, atol=1e-6 * np.abs(want).max())


def test_arm_keeps_touching_islands_awake():
    """Sleeping on: the ball resting on the held arm never sleeps, a box on
    the floor far away does."""
    o, a, c = chain(HORIZONTAL)
    on_arm = dict(shape=S.SPHERE, param=[0.05, 0.0, 0.0], mass=0.5, mu=0.8,
                  pos=c[1] + np.array([0.0, 0.0, S.ARM_RADIUS + 0.05 - 0.001]))
    far = dict(shape=S.BOX, param=[0.05, 0.05, 0.05], mass=0.5, pos=[1.5, 1.5, 0.049])
    _, ora = arm_only(theta=HORIZONTAL, bodies=[on_arm, far])
    ora.set_sleep(0.02, 30)
    for t in range(150):
        ora.step(iters=100, tol=1e-9, warm=O.PREV, outputs=False)
    assert ora.rest[1] >= 30
    r = ora.step(iters=100, tol=1e-9, warm=O.PREV)
    n = int(r["n_contacts"][0])
    col = r["c_colour"][0, :n]
    a = r["c_key"][0, :n] >> 20
    assert np.all(col[a == 1] == -1), "the far box should sleep"
    assert np.all(col[a == 0] >= 0), "the ball on the arm must stay awake"


def test_arm_contacts_take_distinct_colours():
    """Every contact on the arm moves the same joint rates: no two share a colour."""
    _, ora = balls_on_arm(dx=(-0.08, 0.08))
    r = ora.step(iters=20, warm=O.PREV)
    n = int(r["n_contacts"][0])
    keys = r["c_key"][0, :n]
    bb = (keys >> 8) & 0xFFF
    on_arm = (bb >= 1) & (bb != 0xFFF)
    cols = r["c_colour"][0, :n][on_arm]
    assert len(cols) >= 2 and len(set(cols.tolist())) == len(cols)


def test_refused_modes():
    b, ora = arm_only()
    with pytest.raises(ValueError):
        ora.step(iters=10, solver=O.JACOBI)

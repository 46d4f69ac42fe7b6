"""Pins of the oracle's sleeping islands (localized physics, Sec. 4.1: the
robot is the only source of forces besides gravity, settled objects are not
recomputed, and the engine's sleeping state is used).  Each check follows
from the rule itself, not from the oracle's arithmetic: a resting body falls
asleep after exactly the stated number of steps at rest and then keeps its
pose bit for bit; a sleeping contact is not solved and carries its impulse;
with sleeping off nothing changes; a disturbance or the arm wakes the whole
island and only that island."""
import numpy as np

from helpers import DT, G, S, custom_batch
from oracle import oracle as O

V_S, T_S = 0.02, 10


def resting_box(z_extra=0.0, x=0.0):
    """A box resting on the ground (its face 1 mm inside the plane)."""
    return dict(shape=S.BOX, param=[0.1, 0.15, 0.05], mass=1.0, mu=0.6, pos=[x, 0.0, 0.049 + z_extra])


def run(sim, n, **kw):
    return [sim.step(iters=20, **kw) for _ in range(n)]


def test_sleeping_off_changes_nothing():
    b = S.batch_drop(2, seed0=5)
    a, c = O.OracleSim(b), O.OracleSim(b)
    c.set_sleep(0.0, T_S)
    for _ in range(40):
        ra = a.step(iters=10, warm=O.PREV)
        rc = c.step(iters=10, warm=O.PREV)
    assert np.array_equal(a.pose, c.pose) and np.array_equal(a.vel, c.vel)
    assert np.array_equal(ra["c_lambda"], rc["c_lambda"]) and np.array_equal(ra["c_colour"], rc["c_colour"])
    assert not c.rest.any()


def test_resting_box_falls_asleep_after_the_stated_steps():
    b = custom_batch([[resting_box()]])
    sim = O.OracleSim(b)
    sim.set_sleep(V_S, T_S)
    # settle: the box comes to rest within a few steps
    for _ in range(30):
        sim.step(iters=20, warm=O.PREV)
    assert sim.rest[0] >= T_S
    pose = sim.pose.copy()
    r_prev = sim.step(iters=20, warm=O.PREV)   # asleep from this step on: nothing moves
    for _ in range(100):
        r = sim.step(iters=20, warm=O.PREV)
        assert np.array_equal(sim.pose, pose), "a sleeping body moved"
        assert not sim.vel.any()
        n = int(r["n_contacts"][0])
        assert n == 4
        assert np.all(r["c_colour"][0, :n] == -1)          # not coloured, not solved
        assert r["n_colours"][0] == 0
        # the contacts carry their impulses unchanged into the cache
        np.testing.assert_array_equal(r["c_lambda"][0, :n], r_prev["c_lambda"][0, :n])
        r_prev = r


def test_rest_counter_counts_steps_at_rest():
    # a body at rest counts up by one per step; moving faster than the
    # threshold resets the count; a free flight is never at rest
    b = custom_batch([[resting_box()], [dict(shape=S.SPHERE, param=[0.1, 0, 0], mass=1.0, pos=[0, 0, 5.0])]])
    sim = O.OracleSim(b, gravity=(0.0, 0.0, 0.0))
    sim.set_sleep(V_S, 1000)
    for k in range(1, 6):
        sim.step(iters=20, warm=O.PREV)
        assert sim.rest[0] == k
    v = sim.vel.reshape(-1, 6)
    v[0, 0] = 2 * V_S                                 # sliding: not at rest (friction decelerates it)
    sim.step(iters=20, warm=O.PREV)
    assert sim.rest[0] == 0
    g = O.OracleSim(b)
    g.set_sleep(V_S, 1000)
    for _ in range(5):
        g.step(iters=20, warm=O.PREV)
        assert g.rest[1] == 0                          # falling: g dt = 0.08 m/s > V_S after one step


def test_disturbance_wakes_the_whole_island_only():
    # two stacks of two boxes, far apart; both fall asleep; a sphere dropped
    # onto stack A wakes both of A's boxes the step it touches and leaves
    # stack B asleep
    def stack(x):
        return [resting_box(x=x), dict(shape=S.BOX, param=[0.08, 0.08, 0.05], mass=0.5, mu=0.6,
                                       pos=[x, 0.0, 0.1 + 0.049])]
    sphere = dict(shape=S.SPHERE, param=[0.05, 0, 0], mass=0.2, pos=[0.0, 0.0, 5.0])
    b = custom_batch([stack(0.0) + stack(2.0) + [sphere]])
    sim = O.OracleSim(b)
    sim.set_sleep(V_S, T_S)
    woke_at = None
    for t in range(200):
        r = sim.step(iters=20, warm=O.PREV)
        n = int(r["n_contacts"][0])
        keys = r["c_key"][0, :n]
        a_, b_ = keys >> 20, (keys >> 8) & 0xFFF
        cols = r["c_colour"][0, :n]
        stack_a = (a_ <= 1) | ((b_ <= 1) & (b_ != 0xFFF))
        stack_b = ((a_ >= 2) & (a_ <= 3)) | ((b_ >= 2) & (b_ <= 3))
        touch = np.any(((a_ == 4) | (b_ == 4)) & stack_a)
        if touch and woke_at is None:
            woke_at = t
            # the sphere is awake (still moving), so its island, A's stack, is solved
            assert np.all(cols[stack_a] >= 0)
            assert np.all(cols[stack_b] == -1)          # B stays asleep
            break
        if t > 60 and woke_at is None and not touch:
            # before the impact both stacks sleep
            assert np.all(cols[stack_a | stack_b] == -1), t
    assert woke_at is not None


def test_arm_contact_wakes_its_island():
    # a box asleep on the floor next to the arm's base; the arm swings down
    # into it: the step its link touches the box, the box is awake and the
    # contact is solved
    box = dict(shape=S.BOX, param=[0.1, 0.1, 0.1], mass=0.5, mu=0.6, pos=[0.55, 0.0, 0.099])
    b = custom_batch([[box]], arm=True)
    sim = O.OracleSim(b)
    sim.set_sleep(V_S, T_S)
    for _ in range(40):
        sim.step(iters=20, warm=O.PREV, actions=np.zeros((1, 7)))
    assert sim.rest[0] >= T_S
    act = np.zeros((1, 7))
    act[0, 1] = 2.0                                    # joint 1 tips the arm over towards +x
    woke = False
    for t in range(200):
        r = sim.step(iters=20, warm=O.PREV, actions=act)
        n = int(r["n_contacts"][0])
        keys = r["c_key"][0, :n]
        a_, b_ = keys >> 20, (keys >> 8) & 0xFFF
        arm = (a_ >= 1) | ((b_ >= 1) & (b_ != 0xFFF))
        if arm.any():
            assert np.all(r["c_colour"][0, :n] >= 0)     # the box's island is awake
            woke = True
            break
        assert np.all(r["c_colour"][0, :n] == -1)
    assert woke

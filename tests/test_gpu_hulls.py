"""Convex hulls on the GPU (Sec. 3 and Sec. 4.3: objects collide as convex
hulls) against the oracle: one step from the same float32 state.

Drop scenes of prisms, bipyramids and chamfered boxes among spheres, boxes
and capsules, settled in the oracle, so that hulls rest on the ground, on
each other and on the other shapes: every pair class with a hull occurs.
Pairs, contact keys (features included), colours, contact geometry and
impulses, and body states as in every parity test (`compare`).  The
persistent launch, the global-memory working set and 256-thread teams give
the same bits as one 64-thread workgroup per scene; modes and libraries
the step does not support are refused."""
import numpy as np
import pytest

from gpu_util import compare, gpu_results, gpu_sim, oracle_warmup, report, snapshot32
from helpers import DT, S
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def hull_batch(n, seed0=500):
    return S.pack([S.drop_scene(seed0 + s, n_spheres=8, n_boxes=8, n_capsules=8, n_hulls=24) for s in range(n)])


def pair_classes(b, r):
    """Counts of contacts by the shapes of their bodies (with a hull)."""
    out = {}
    names = {S.SPHERE: "sphere", S.BOX: "box", S.CAPSULE: "capsule", S.HULL: "hull"}
    for s in range(b.n_scenes):
        b0 = int(b.body_offset[s])
        k = r["c_key"][s, :int(r["n_contacts"][s])]
        for key in k:
            a, bb = int(key) >> 20, (int(key) >> 8) & 0xFFF
            sa = int(b.shape[b0 + a])
            sb = "ground" if bb == 0xFFF else names[int(b.shape[b0 + bb])]
            if S.HULL not in (sa, -1 if bb == 0xFFF else int(b.shape[b0 + bb])):
                continue
            name = "-".join(sorted([names[sa], sb]))
            out[name] = out.get(name, 0) + 1
    return out


@pytest.mark.parametrize("warm,tol,iters,steps", [(O.PREV, 0.0, 20, 120), (O.COLD, 0.0, 20, 60),
                                                  (O.PREV, 1e-4, 1000, 200)])
def test_hull_drop_parity(torch_cuda, warm, tol, iters, steps):
    b = hull_batch(8)
    ora = oracle_warmup(b, steps, iters=20, warm=O.PREV)
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, warm=warm, tol=tol)
    sim.step(None, DT, iters)
    r = ora.step(iters=iters, tol=tol, warm=warm, max_pairs=sim.max_pairs, max_contacts=sim.max_contacts)
    g = gpu_results(sim)
    rep = compare(b, g, r, ora, contact_values=True, tol_band=0.02 if tol > 0 else None)
    report(f"hull drop, step {steps}, warm={warm} tol={tol:g}", rep)
    cls = pair_classes(b, r)
    print(f"contacts with a hull by class: {cls}", flush=True)
    for name in ("ground-hull", "hull-hull", "box-hull", "hull-sphere", "capsule-hull"):
        assert cls.get(name, 0) >= 3, (name, cls)
    assert rep["contacts_solved"] >= 300


def state(sim):
    import torch
    torch.cuda.synchronize()
    cnt, key, lam = sim.cache()
    return dict(pose=sim.pose.cpu().numpy().copy(), vel=sim.vel.cpu().numpy().copy(),
                count=cnt.cpu().numpy().copy(), key=key.cpu().numpy().copy(), lam=lam.cpu().numpy().copy(),
                **{k: v.cpu().numpy().copy() for k, v in sim.stats.items()})


@pytest.mark.parametrize("variant", ["persistent", "hbm", "threads"])
def test_hull_launches_bit_identical(torch_cuda, variant):
    """80 steps of a hull drop: every launch gives the same bits as one
    64-thread workgroup per scene in LDS."""
    from paper_2106_14405_amd.sim import Sim
    b = hull_batch(12, seed0=700)
    sims = []
    for alt in (False, True):
        kw = dict(warm=O.PREV, tol=1e-4, threads=64)
        if alt and variant == "hbm":
            kw["hbm_min_bodies"] = 1
        if alt and variant == "threads":
            kw["threads"] = 256
        sm = Sim(b, **kw)
        if alt and variant == "persistent":
            sm.set_persistent(True, 64)
        sims.append(sm)
    for t in range(80):
        for sm in sims:
            sm.step(None, DT, 200)
        if t % 20 == 19:
            x, y = state(sims[0]), state(sims[1])
            for k in x:
                assert np.array_equal(x[k], y[k]), f"step {t}: {k} differs"


def hull_arm_scene(seed):
    """Hulls among spheres, boxes and capsules dropped round the arm base
    (x, y within 0.8 m, z 0.2 to 1.8 m), and the kinematic arm."""
    sc = S.drop_scene(seed, n_spheres=4, n_boxes=4, n_capsules=4, n_hulls=16, edge=1.6)
    for L in S.ARM_LINK_LENGTH:
        sc.add(S.CAPSULE, S.KINEMATIC, [S.ARM_RADIUS, 0.5 * L, 0.0], 0.0, 0.5, 0.0, S.ARM_BASE, (1.0, 0.0, 0.0, 0.0))
    sc.arm = True
    sc.arm_theta0 = np.zeros(7)
    return sc


@pytest.mark.parametrize("clearance", [0.0, 0.05])
def test_hull_query_parity(torch_cuda, clearance):
    """Arm collision queries (motion planning) against scenes with hulls:
    hit flags bit-exact outside the tie band, separations within 1e-5 m."""
    from test_gpu_query import compare as qcompare, run_both
    b = S.pack([hull_arm_scene(900 + k) for k in range(8)])
    ora = oracle_warmup(b, 40, iters=20)
    for hg, pg, ho, po, ao, c in run_both(torch_cuda, b, ora, 96, [clearance]):
        frac = qcompare(hg, pg, ho, po, ao, c, f"hull scenes, clearance {c}")
        assert 0.05 < frac < 0.95


def test_hull_refusals(torch_cuda):
    from paper_2106_14405_amd import _lib as L
    from paper_2106_14405_amd.sim import Sim
    b = hull_batch(2)
    with pytest.raises(L.SimError):
        Sim(b, warm=O.LEARNED)
    sim = Sim(b, warm=O.PREV)
    with pytest.raises(L.SimError, match="hulls"):
        sim.set_solver(L.PGS, L.LEARNED, 0.0)

    def bad(match, fn):
        bb = S.Batch(**{**b.__dict__})
        bb.hull_vert = b.hull_vert.copy()
        bb.hull_face = b.hull_face.copy()
        bb.param = b.param.copy()
        fn(bb)
        with pytest.raises(L.SimError, match=match):
            Sim(bb, warm=O.PREV)
    v0, nv, f0, nf = b.hull_index[0]
    bad("centre of mass", lambda bb: bb.hull_vert.__setitem__(slice(v0, v0 + nv), b.hull_vert[v0:v0 + nv] + 0.01))
    bad("close the surface", lambda bb: bb.hull_face.__setitem__(f0, np.r_[b.hull_face[f0][:3][::-1], b.hull_face[f0][3:]]))

    def dent(bb):   # one vertex pulled in towards the centre: a face through it bends inwards
        bb.hull_vert[v0] = 0.5 * b.hull_vert[v0]
    bad("convex|centre of mass", dent)
    hb = np.nonzero(b.shape == S.HULL)[0][0]
    bad("index", lambda bb: bb.param.__setitem__((hb, 0), 1e6))


def hull_part_scene(seed):
    """A chamfered-box door on a vertical hinge beside a static post and a
    prism drawer on a slide, with hulls, spheres and boxes dropped on and
    around them (the kernel level with parts and hulls together)."""
    rng = np.random.default_rng(seed)
    sc = S.Scene()
    sc.add(S.BOX, S.STATIC, [0.05, 0.05, 0.5], 0.0, 0.6, 0.0, [0.0, -0.05, 0.5], (1.0, 0.0, 0.0, 0.0))
    Vd, Fd = S.hull_chamfered_box(0.3, 0.02, 0.4, 0.015)
    sc.add_hull(Vd, Fd, S.DYNAMIC, 3.0, 0.6, 0.0, [0.3, 0.03, 0.5], (1.0, 0.0, 0.0, 0.0))
    sc.joints[1] = (1, (0.0, 0.0, 1.0), (0.0, 0.03, 0.5), (-1.5, 1.5), 0)
    Vw, Fw = S.hull_prism(6, 0.2, 0.05)
    sc.add_hull(Vw, Fw, S.DYNAMIC, 2.0, 0.6, 0.0, [-0.6, 0.6, 0.3], (1.0, 0.0, 0.0, 0.0))
    sc.joints[2] = (2, (1.0, 0.0, 0.0), (-0.6, 0.6, 0.3), (-0.3, 0.3), -1)
    for k in range(12):
        p = [rng.uniform(-0.8, 0.8), rng.uniform(-0.3, 0.9), rng.uniform(0.9, 2.0)]
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        if k % 3 == 0:
            sc.add(S.SPHERE, S.DYNAMIC, [rng.uniform(0.04, 0.08), 0, 0], 0.5, 0.5, 0.0, p, q)
        elif k % 3 == 1:
            V, F = S.random_hull(S._Stream(S.stream_key(seed, 11, k)), (0.04, 0.08))
            sc.add_hull(V, F, S.DYNAMIC, 0.6, 0.5, 0.0, p, q)
        else:
            sc.add(S.BOX, S.DYNAMIC, list(rng.uniform(0.03, 0.07, 3)), 0.7, 0.5, 0.0, p, q)
    return sc


def test_hull_parts_parity(torch_cuda):
    """Container parts that are hulls, struck by falling hulls and other
    shapes: one step against the oracle after 120 steps with the parts
    started at 1 rad/s and 0.3 m/s."""
    from gpu_util import joint_snapshot32
    torch = torch_cuda
    b = S.pack([hull_part_scene(70 + k) for k in range(8)])
    ora = O.OracleSim(b)
    for g in np.nonzero(b.joint)[0]:
        ora.q_rate[g] = 1.0 if b.joint[g] == 1 else 0.3
    for t in range(120):
        ora.step(iters=20, warm=O.PREV, outputs=False)
    pose, vel, theta, cache = snapshot32(ora)
    js = joint_snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, warm=O.PREV)
    sim.joint_state.copy_(torch.as_tensor(js))
    sim.step(None, DT, 20)
    r = ora.step(iters=20, warm=O.PREV, max_pairs=sim.max_pairs, max_contacts=sim.max_contacts)
    g = gpu_results(sim)
    rep = compare(b, g, r, ora, contact_values=True)
    report("hull parts", rep)
    jo = ora.joint_state.reshape(-1, 2)
    for gi in np.nonzero(b.joint)[0]:
        s = int(np.searchsorted(b.body_offset, gi, side="right") - 1)
        if r["ambiguous"][s]:
            continue
        assert abs(float(g["joint_state"][0, gi]) - jo[gi, 0]) <= 1e-5
        assert abs(float(g["joint_state"][1, gi]) - jo[gi, 1]) <= 1e-4 * max(abs(jo[gi, 1]), 1.0)
    assert rep["contacts_solved"] >= 100


def test_hull_sleeping_parity(torch_cuda):
    """Sleeping on (0.02 m/s, 30 steps): hulls at rest fall asleep by their
    bounding box's radius; one step against the oracle, rest counters equal."""
    from gpu_util import gpu_set_rest
    sleep = (0.02, 30)
    b = hull_batch(8, seed0=560)
    ora = O.OracleSim(b)
    ora.set_sleep(*sleep)
    for t in range(200):
        ora.step(iters=20, warm=O.PREV, outputs=False)
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, warm=O.PREV)
    sim.set_sleep(*sleep)
    gpu_set_rest(sim, ora.rest)
    sim.step(None, DT, 20)
    r = ora.step(iters=20, warm=O.PREV, max_pairs=sim.max_pairs, max_contacts=sim.max_contacts)
    g = gpu_results(sim)
    rep = compare(b, g, r, ora, contact_values=True, check_rest=True)
    report("hull drop, sleeping", rep)
    hull_rows = b.shape == S.HULL
    assert np.sum(ora.rest[hull_rows] >= sleep[1]) >= 20   # hulls asleep


def _qmul(a, b):
    return np.r_[a[0] * b[0] - a[1:] @ b[1:], a[0] * b[1:] + b[0] * a[1:] + np.cross(a[1:], b[1:])]


def level_capsule_scene(k):
    """A capsule lying level, a few mm above the top face of a static
    hexagonal prism, short enough to lie inside the face or long enough to
    hang over its edges, at a yaw of its own; from k = 8 on the prism is
    turned about a tilted axis and the capsule with it."""
    sc = S.Scene()
    V, F = S.hull_prism(6, 0.2, 0.05)
    ang = 0.0 if k < 8 else 0.25 * (k - 7)
    ax = np.array([1.0, 0.5 * (k % 3), 0.3])
    qh = np.r_[np.cos(ang / 2), np.sin(ang / 2) * ax / np.linalg.norm(ax)]
    ch = np.array([0.0, 0.0, 0.5])
    sc.add_hull(V, F, S.STATIC, 0.0, 0.6, 0.0, list(ch), tuple(qh))
    r, hl = 0.03, (0.05, 0.12, 0.3, 0.45)[k % 4]
    gap = (0.002, 0.004)[k // 4 % 2]
    yaw = 0.37 * k
    qc = _qmul(np.array([np.cos(yaw / 2), 0.0, 0.0, np.sin(yaw / 2)]),
               np.array([np.cos(np.pi / 4), 0.0, np.sin(np.pi / 4), 0.0]))
    loc = np.array([0.01 * (k % 8), 0.02, 0.05 + r + gap])
    pc = ch + _qmul(_qmul(qh, np.r_[0.0, loc]), qh * np.r_[1, -1, -1, -1])[1:]
    sc.add(S.CAPSULE, S.DYNAMIC, [r, hl, 0.0], 0.5, 0.5, 0.0, list(pc), _qmul(qh, qc))
    return sc


def test_capsule_level_on_a_hull_face_parity(torch_cuda):
    """A capsule level with a hull's face touches it at the two ends of its
    core clipped to the face (features 0 and 1), also where it hangs over
    the face's edges: one step against the oracle, the capsule approaching
    the face."""
    b = S.pack([level_capsule_scene(k) for k in range(16)])
    assert b.n_scenes == 16
    ora = O.OracleSim(b)
    # each capsule approaches its face at 0.6 m/s, so that the patch is solved
    pose, vel = ora.pose.reshape(-1, 7), ora.vel.reshape(-1, 6)
    for s in range(b.n_scenes):
        h, c = int(b.body_offset[s]), int(b.body_offset[s]) + 1
        q = pose[h, 3:7]
        up = _qmul(_qmul(q, np.r_[0.0, 0.0, 0.0, 1.0]), q * np.r_[1, -1, -1, -1])[1:]
        vel[c, :3] = -0.6 * up
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, cache, warm=O.COLD)
    sim.step(None, DT, 20)
    r = ora.step(iters=20, warm=O.COLD, max_pairs=sim.max_pairs, max_contacts=sim.max_contacts)
    g = gpu_results(sim)
    rep = compare(b, g, r, ora, contact_values=True)
    report("capsule level on a hull face", rep)
    assert (r["c_lambda"][:, :2, 0] > 0).all()
    for s in range(b.n_scenes):
        assert not r["ambiguous"][s]
        for key, n in ((g["key"], g["count"]), (r["c_key"], r["n_contacts"])):
            assert sorted(int(k) & 0xFF for k in key[s, :int(n[s])]) == [0, 1], s

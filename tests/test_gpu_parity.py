"""GPU parity: the HIP step through the C ABI against the FP64 oracle.

Both sides start every compared step from the identical float32 state (an
oracle run rounded to float32, never a GPU output).  In scenes without a
tie-band decision, pair keys, contact keys and colours are bit-exact;
positions, velocities and orientations agree within 1e-4 relative (floors
1 m, 1 m/s, 1 rad/s; 1e-4 rad for orientation).  In scenes with one, the
same holds outside the tied bodies' contact islands.  Every check prints
how many scenes the tie band flagged and how many bodies it excluded.
"""
import numpy as np
import pytest

from gpu_util import compare, gpu_results, gpu_sim, oracle_warmup, report, snapshot32
from helpers import DT, G, S, custom_batch
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def step_both(batch, ora, warm, iters, tol=0.0, solver=O.PGS, threads=128, max_contacts=None, actions_seed=7,
              step_index=0, use_cache=True):
    import torch
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(batch, pose, vel, theta, cache if use_cache else None, max_contacts=max_contacts,
                  max_pairs=max_contacts, warm=warm, tol=tol, solver=solver, threads=threads)
    act = S.arm_actions(actions_seed, batch.n_scenes, step_index) if batch.arm else None
    if act is not None:
        sim.step(torch.as_tensor(act, device=sim.device), DT, iters)
    else:
        sim.step(None, DT, iters)
    r = ora.step(actions=act, iters=iters, tol=tol, warm=warm, solver=solver, max_pairs=sim.max_pairs,
                 max_contacts=sim.max_contacts)
    g = gpu_results(sim)
    return sim, g, r


def test_ballistic_on_device(torch_cuda):
    """Semi-implicit Euler closed form after 120 steps in float32."""
    torch = torch_cuda
    bodies = [dict(shape=S.SPHERE, param=[0.1, 0, 0], pos=[0, 0, 80.0], vel=[1.0, -2.0, 3.0, 0.4, -0.2, 0.1]),
              dict(shape=S.BOX, param=[0.1, 0.2, 0.3], pos=[5, 0, 90.0], vel=[0, 0.5, 0, 0, 0, 0])]
    b = custom_batch([bodies, bodies])
    from paper_2106_14405_amd.sim import Sim
    sim = Sim(b)
    x0 = b.pose[:, :3].astype(np.float64)
    v0 = b.vel[:, :3].astype(np.float64)
    n = 120
    for _ in range(n):
        sim.step(None, DT, 4)
    torch.cuda.synchronize()
    x = sim.pose.cpu().numpy().T[:, :3].astype(np.float64)
    v = sim.vel.cpu().numpy().T[:, :3].astype(np.float64)
    g = np.array([0, 0, -G])
    xn = x0 + n * DT * v0 + g * DT * DT * n * (n + 1) / 2
    vn = v0 + n * g * DT
    assert np.max(np.abs(x - xn) / np.maximum(np.abs(xn), 1.0)) < 1e-4
    assert np.max(np.abs(v - vn) / np.maximum(np.abs(vn), 1.0)) < 1e-4
    assert int(sim.stats["pairs"].sum()) == 0


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_drop_first_step_initial_state(torch_cuda, seed):
    """Step 0 of the drop case (bodies in the air): pairs exactly as brute force."""
    b = S.batch_drop(1, seed0=seed)
    ora = O.OracleSim(b)
    sim, g, r = step_both(b, ora, O.COLD, 10)
    rep = compare(b, g, r, ora, contact_values=True)
    report(f"drop step 0 seed {seed}", rep)
    assert rep["scenes"] == 1


@pytest.mark.parametrize("warm", [O.COLD, O.PREV])
def test_drop_settled_parity(torch_cuda, warm):
    """Drop case, 64 bodies, one step from 8 oracle-settled states each."""
    tot = None
    for seed in range(8):
        b = S.batch_drop(1, seed0=100 + seed)
        ora = oracle_warmup(b, 60 + 10 * seed, iters=10, warm=O.PREV)
        sim, g, r = step_both(b, ora, warm, 10)
        rep = compare(b, g, r, ora, contact_values=True)
        tot = rep if tot is None else {k: (max(tot[k], v) if k.startswith("max") else tot[k] + v)
                                       for k, v in rep.items()}
    tot["flagged_frac"] = tot["flagged"] / tot["scenes"]
    tot["excluded_frac"] = tot["bodies_excluded"] / max(tot["bodies"], 1)
    report(f"drop settled warm={warm}", tot)
    assert tot["excluded_frac"] <= 0.5 and tot["contacts"] >= 100


def test_drop_batch_many_scenes(torch_cuda):
    """16 drop scenes in one launch, settled by the oracle; ragged contact counts."""
    b = S.batch_drop(16, seed0=300)
    ora = oracle_warmup(b, 90, iters=10, warm=O.PREV)
    sim, g, r = step_both(b, ora, O.PREV, 10)
    rep = compare(b, g, r, ora, contact_values=True)
    report("drop 16 scenes", rep)
    assert rep["excluded_frac"] <= 0.5


def test_large_scene_parity(torch_cuda):
    """Scenes above 512 bodies sort their bodies by LSD radix passes (smaller
    ones rank by counting): two 520-body drop scenes, one 256-thread
    workgroup each, one step from oracle-settled states."""
    b = S.batch_drop(2, seed0=900, n_spheres=260, n_boxes=260)
    assert b.counts().min() > 512
    ora = oracle_warmup(b, 60, iters=10, warm=O.PREV)
    sim, g, r = step_both(b, ora, O.PREV, 10, threads=256, max_contacts=1536)
    rep = compare(b, g, r, ora, contact_values=True)
    report("drop 520 bodies", rep)
    assert rep["contacts"] > 50


@pytest.mark.parametrize("threads", [64, 192, 256])
def test_block_size_bit_identical(torch_cuda, threads):
    """Results are bit-identical for any workgroup size."""
    b = S.batch_drop(4, seed0=500)
    ora = oracle_warmup(b, 80, iters=10, warm=O.PREV)
    pose, vel, theta, cache = snapshot32(ora)
    outs = []
    for T in (128, threads):
        sim = gpu_sim(b, pose, vel, theta, cache, warm=O.PREV, threads=T)
        sim.step(None, DT, 10)
        outs.append(gpu_results(sim))
    a, c = outs
    assert np.array_equal(a["pose"], c["pose"]) and np.array_equal(a["vel"], c["vel"])
    assert np.array_equal(a["key"], c["key"]) and np.array_equal(a["lam"], c["lam"])


def test_two_runs_bit_identical(torch_cuda):
    b = S.batch_drop(4, seed0=600)
    ora = oracle_warmup(b, 70, iters=10, warm=O.PREV)
    pose, vel, theta, cache = snapshot32(ora)
    outs = []
    for _ in range(2):
        sim = gpu_sim(b, pose, vel, theta, cache, warm=O.PREV)
        for _ in range(5):
            sim.step(None, DT, 10)
        outs.append(gpu_results(sim))
    assert np.array_equal(outs[0]["pose"], outs[1]["pose"])
    assert np.array_equal(outs[0]["vel"], outs[1]["vel"])


def test_clutter_arm_parity(torch_cuda):
    """Clutter scenes with statics, capsules and the kinematic arm."""
    b = S.batch_clutter(6, seed0=10000)
    ora = oracle_warmup(b, 100, iters=20, warm=O.PREV)
    sim, g, r = step_both(b, ora, O.PREV, 20, step_index=100)
    rep = compare(b, g, r, ora, contact_values=True)
    report("clutter PREV 20 sweeps, 128 threads", rep)
    assert rep["excluded_frac"] <= 0.5
    # arm joint angles and contact force
    np.testing.assert_allclose(g["theta"], ora.theta.reshape(-1, 7), rtol=0, atol=1e-6)
    unflagged = r["ambiguous"] == 0
    np.testing.assert_allclose(g["stats"]["arm_force"][unflagged], r["arm_force"][unflagged], rtol=1e-3, atol=1e-2)


def test_jacobi_parity(torch_cuda):
    b = S.batch_drop(4, seed0=700)
    ora = oracle_warmup(b, 80, iters=10, warm=O.PREV)
    sim, g, r = step_both(b, ora, O.PREV, 10, solver=O.JACOBI)
    rep = compare(b, g, r, ora, contact_values=True)
    report("drop Jacobi", rep)
    assert rep["excluded_frac"] <= 0.5


def test_tolerance_mode_sweeps(torch_cuda):
    """Tolerance mode: sweep counts equal unless the oracle's residual came
    within 2% of the tolerance at a stopping test; states and impulses
    compared wherever the counts are equal."""
    b = S.batch_drop(8, seed0=800)
    ora = oracle_warmup(b, 80, iters=10, warm=O.PREV)
    sim, g, r = step_both(b, ora, O.PREV, 200, tol=1e-4)
    rep = compare(b, g, r, ora, contact_values=True, tol_band=0.02)
    report("drop tolerance 1e-4 PREV", rep)
    assert rep["sweeps_equal"] >= 6
    assert np.all(g["stats"]["residual"][g["stats"]["flags"] & 4 == 0] <= 1e-4)


@pytest.mark.parametrize("warm", [O.COLD, O.PREV])
def test_clutter_timed_configuration(torch_cuda, warm):
    """The configuration the benchmark times: clutter scenes (statics,
    spheres, boxes, capsules, the arm) settled by the oracle, one wave per
    scene (64 threads), residual tolerance 1e-4 m/s with a 1,000-sweep cap,
    cold and classic warm starts; keys, colours, contact geometry, impulses
    and states compared."""
    b = S.batch_clutter(8, seed0=10000)
    ora = oracle_warmup(b, 150, iters=20, warm=O.PREV)
    sim, g, r = step_both(b, ora, warm, 1000, tol=1e-4, threads=64, step_index=150)
    rep = compare(b, g, r, ora, contact_values=True, tol_band=0.02)
    report(f"clutter timed configuration warm={warm}", rep)
    assert rep["contacts"] >= 500
    assert rep["excluded_frac"] <= 0.5
    np.testing.assert_allclose(g["theta"], ora.theta.reshape(-1, 7), rtol=0, atol=1e-6)
    conv = (g["stats"]["flags"] & 4) == 0
    assert np.all(g["stats"]["residual"][conv] <= 1e-4)


def test_contact_values_clutter(torch_cuda):
    """Normals, points, depths and impulses on clutter scenes (capsules,
    static boxes and arm links among the pairs), fixed 20 sweeps."""
    b = S.batch_clutter(4, seed0=10100)
    ora = oracle_warmup(b, 120, iters=20, warm=O.PREV)
    sim, g, r = step_both(b, ora, O.PREV, 20, threads=64, step_index=120)
    rep = compare(b, g, r, ora, contact_values=True)
    report("clutter contact values", rep)
    # the compared contacts cover every kind of body
    shapes, motion = b.shape, b.motion
    kinds = set()
    for s in range(b.n_scenes):
        b0 = int(b.body_offset[s])
        for k in g["key"][s, :int(g["count"][s])].astype(np.int64):
            a, bb = int(k >> 20), int((k >> 8) & 0xFFF)
            kinds.add(("shape", int(shapes[b0 + a])))
            kinds.add(("motion", int(motion[b0 + a])))
            if bb != 0xFFF:
                kinds.add(("shape", int(shapes[b0 + bb])))
                kinds.add(("motion", int(motion[b0 + bb])))
    assert {("shape", S.SPHERE), ("shape", S.BOX), ("shape", S.CAPSULE), ("motion", S.STATIC)} <= kinds, kinds


def _tie_scene(reverse=False):
    """Bodies whose AABBs touch exactly in float32 and float64 alike: margin
    2^-6 m, sphere radius 7/64 m (AABB half-size 1/8), box half-extents 7/64
    and 15/64 m, capsule radius 7/64 and half-length 1/8 m, identity
    orientations, positions on a 1/4 m lattice: every AABB bound is a short
    dyadic number, computed exactly on both sides."""
    r, h = 7.0 / 64.0, 15.0 / 64.0
    z0 = 1.0
    bodies = []
    # a row along x: consecutive spheres touch exactly (closed intervals)
    for i in range(6):
        bodies.append(dict(shape=S.SPHERE, param=[r, 0, 0], pos=[0.25 * i, 0.0, z0]))
    # equal minima: a column along y at x = 0 (each touches its neighbour in y)
    for j in range(1, 4):
        bodies.append(dict(shape=S.SPHERE, param=[r, 0, 0], pos=[0.0, 0.25 * j, z0]))
    # diagonal corner contact of AABBs
    bodies.append(dict(shape=S.BOX, param=[r, r, r], pos=[0.25, 0.25, z0 + 0.25]))
    # coincident bodies
    bodies.append(dict(shape=S.SPHERE, param=[r, 0, 0], pos=[2.0, 2.0, z0]))
    bodies.append(dict(shape=S.BOX, param=[r, r, r], pos=[2.0, 2.0, z0]))
    # a long box spanning several spheres, touching on its end faces
    bodies.append(dict(shape=S.BOX, param=[h, r, r], pos=[0.375, -0.25, z0]))
    # just separated: a gap of 2^-20 m along x
    bodies.append(dict(shape=S.SPHERE, param=[r, 0, 0], pos=[-0.25 - 2.0 ** -20, 0.0, z0]))
    # capsule along z touching the row from above
    bodies.append(dict(shape=S.CAPSULE, param=[r, 0.125, 0], pos=[0.5, 0.0, z0 + 0.375]))
    # resting exactly on the ground (AABB minimum z = 0) and just above it
    bodies.append(dict(shape=S.SPHERE, param=[r, 0, 0], pos=[-1.0, -1.0, 0.125]))
    bodies.append(dict(shape=S.SPHERE, param=[r, 0, 0], pos=[-1.5, -1.0, 0.125 + 2.0 ** -20]))
    # static boxes touching each other (no pair) and a dynamic sphere (a pair)
    bodies.append(dict(shape=S.BOX, motion=S.STATIC, param=[r, r, r], pos=[-1.0, 1.0, z0]))
    bodies.append(dict(shape=S.BOX, motion=S.STATIC, param=[r, r, r], pos=[-0.75, 1.0, z0]))
    bodies.append(dict(shape=S.SPHERE, param=[r, 0, 0], pos=[-1.0, 1.25, z0]))
    if reverse:
        bodies = bodies[::-1]
    return bodies


@pytest.mark.parametrize("reverse", [False, True])
def test_broadphase_exact_ties(torch_cuda, reverse):
    """Sort-and-sweep against brute force on boxes that touch exactly: the
    GPU's pair set equals the oracle's O(n^2) enumeration bit for bit with
    no tie band (closed intervals: touching boxes pair; static-only pairs
    never), for input in and against x order."""
    bodies = _tie_scene(reverse)
    b = custom_batch([bodies, bodies[::-1]])
    consts = dict(margin=2.0 ** -6)
    ora = O.OracleSim(b, **consts)
    pose, vel, theta, cache = snapshot32(ora)
    for threads in (64, 256):
        sim = gpu_sim(b, pose, vel, theta, None, warm=O.COLD, threads=threads, **consts)
        sim.step(None, DT, 1)
        g = gpu_results(sim)
        ora.set_state(pose, vel, theta)
        r = ora.step(iters=1, warm=O.COLD, max_pairs=sim.max_pairs, max_contacts=sim.max_contacts)
        for s in range(b.n_scenes):
            n = int(r["n_pairs"][s])
            assert int(g["stats"]["pairs"][s]) == n
            assert np.array_equal(g["pair_key"][s, :n].astype(np.uint32), r["pair_key"][s, :n]), (s, threads)
            assert n >= 20
        assert r["ambiguous"].min() > 0          # the oracle does see the ties


def test_capacity_flag(torch_cuda):
    """Contact capacity overflow raises the CAPACITY flag and stays in bounds."""
    b = S.batch_drop(2, seed0=1000)
    ora = oracle_warmup(b, 90, iters=10, warm=O.PREV)
    pose, vel, theta, cache = snapshot32(ora)
    sim = gpu_sim(b, pose, vel, theta, None, max_contacts=16, max_pairs=16)
    sim.step(None, DT, 5)
    g = gpu_results(sim)
    assert np.all(g["stats"]["flags"] & 2)
    assert np.all(g["count"] <= 16)

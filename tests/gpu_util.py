"""Helpers of the GPU tests: build the HIP simulation and the oracle from the
same float32 state, step both, and compare element by element."""
from __future__ import annotations

import numpy as np

from helpers import S
from oracle import oracle as O

# parity bar (single step, float32 GPU vs float64 oracle)
REL = 1e-4          # relative, with floors below
X_FLOOR = 1.0       # m
V_FLOOR = 1.0       # m/s and rad/s
Q_ANGLE = 1e-4      # rad


def quat_angle(qa, qb):
    """Rotation angle between unit quaternions (either sign), computed as
    2 atan2(|a - s b|, |a + s b|) after normalising both: stable near 0."""
    qa = qa / np.linalg.norm(qa, axis=1, keepdims=True)
    qb = qb / np.linalg.norm(qb, axis=1, keepdims=True)
    sgn = np.where(np.sum(qa * qb, axis=1) < 0, -1.0, 1.0)[:, None]
    return 2.0 * np.arctan2(np.linalg.norm(qa - sgn * qb, axis=1), np.linalg.norm(qa + sgn * qb, axis=1))


def oracle_warmup(batch, steps, iters=10, warm=O.PREV, arm_seed=1, **kw):
    """Run the oracle `steps` steps from the batch's initial state (the only
    source of non-initial states for parity inputs)."""
    ora = O.OracleSim(batch, **kw)
    for t in range(steps):
        act = S.arm_actions(arm_seed, batch.n_scenes, t) if batch.arm else None
        ora.step(actions=act, iters=iters, warm=warm, outputs=False)
    return ora


def snapshot32(ora):
    """Float32 state and cache of an oracle run, and the oracle reset to exactly it."""
    pose, vel, theta = ora.state32()
    cnt, key, lam = ora.cache_arrays()
    lam32 = lam.astype(np.float32)
    ora.set_state(pose, vel, theta, (cnt, key, lam32.astype(np.float64)))
    return pose, vel, theta, (cnt, key, lam32)


def gpu_sim(batch, pose, vel, theta, cache=None, max_contacts=None, max_pairs=None, **kw):
    import torch

    from paper_2106_14405_amd.sim import Sim
    b = S.Batch(**{**batch.__dict__})
    b.pose = pose.reshape(-1, 7).astype(np.float32)
    b.vel = vel.reshape(-1, 6).astype(np.float32)
    b.arm_theta = theta.reshape(-1, 7).astype(np.float32)
    sim = Sim(b, max_contacts=max_contacts, max_pairs=max_pairs, **kw)
    if cache is not None:
        cnt, key, lam = cache
        ccount, ckey, clam = sim.cache()
        CM = sim.max_contacts
        w = min(CM, key.shape[1])
        assert int(cnt.max(initial=0)) <= CM
        ccount.copy_(torch.as_tensor(cnt, dtype=torch.int32))
        kk = np.zeros((batch.n_scenes, CM), np.int64)
        kk[:, :w] = key[:, :w].astype(np.int64)
        ckey.copy_(torch.as_tensor(kk.astype(np.uint32).view(np.int32)))
        ll = np.zeros((4, batch.n_scenes, CM), np.float32)
        ll[:, :, :w] = np.transpose(lam[:, :w, :], (2, 0, 1))
        clam.copy_(torch.as_tensor(ll))
    sim.set_export(True)
    return sim


def gpu_results(sim):
    import torch
    torch.cuda.synchronize()
    c = sim.contacts()
    out = {k: v.cpu().numpy() for k, v in c.items() if v is not None}
    out["pose"] = sim.pose.cpu().numpy().T.astype(np.float64)
    out["vel"] = sim.vel.cpu().numpy().T.astype(np.float64)
    out["stats"] = {k: v.cpu().numpy() for k, v in sim.stats.items()}
    out["theta"] = sim.theta.cpu().numpy() if sim.theta is not None else None
    return out


def compare(batch, g, r, ora, check_values=True, scenes=None):
    """Element-by-element comparison.  Returns a report dict; raises on a
    mismatch in an unflagged scene."""
    rep = dict(scenes=0, flagged=0, contacts=0, max_x=0.0, max_v=0.0, max_w=0.0, max_q=0.0, max_lam=0.0)
    Sn = batch.n_scenes
    pose_o = ora.pose.reshape(-1, 7)
    vel_o = ora.vel.reshape(-1, 6)
    for s in (range(Sn) if scenes is None else scenes):
        rep["scenes"] += 1
        if r["ambiguous"][s] != 0:
            rep["flagged"] += 1
            continue
        # pair sets
        np_o = int(r["n_pairs"][s])
        np_g = int(g["stats"]["pairs"][s])
        assert np_g == np_o, f"scene {s}: {np_g} pairs on the GPU, {np_o} in the oracle"
        pk_g = g["pair_key"][s, :np_g].astype(np.uint32)
        assert np.array_equal(pk_g, r["pair_key"][s, :np_o]), f"scene {s}: pair keys differ"
        # contact keys, colours
        nc = int(r["n_contacts"][s])
        assert int(g["count"][s]) == nc, f"scene {s}: {int(g['count'][s])} contacts on the GPU, {nc} in the oracle"
        kg = g["key"][s, :nc].astype(np.uint32)
        assert np.array_equal(kg, r["c_key"][s, :nc]), f"scene {s}: contact keys differ"
        assert np.array_equal(g["colour"][s, :nc], r["c_colour"][s, :nc]), f"scene {s}: colours differ"
        assert int(g["stats"]["colours"][s]) == int(r["n_colours"][s])
        rep["contacts"] += nc
        if not check_values:
            continue
        b0, b1 = int(batch.body_offset[s]), int(batch.body_offset[s + 1])
        xo, xg = pose_o[b0:b1, :3], g["pose"][b0:b1, :3]
        ex = np.max(np.abs(xg - xo) / np.maximum(np.abs(xo), X_FLOOR), initial=0.0)
        vo, vg = vel_o[b0:b1], g["vel"][b0:b1]
        ev = np.max(np.abs(vg[:, :3] - vo[:, :3]) / np.maximum(np.abs(vo[:, :3]), V_FLOOR), initial=0.0)
        ew = np.max(np.abs(vg[:, 3:] - vo[:, 3:]) / np.maximum(np.abs(vo[:, 3:]), V_FLOOR), initial=0.0)
        eq = np.max(quat_angle(pose_o[b0:b1, 3:], g["pose"][b0:b1, 3:]), initial=0.0)
        rep["max_x"] = max(rep["max_x"], ex)
        rep["max_v"] = max(rep["max_v"], ev)
        rep["max_w"] = max(rep["max_w"], ew)
        rep["max_q"] = max(rep["max_q"], eq)
        assert ex <= REL, f"scene {s}: position error {ex:.3e}"
        assert ev <= REL, f"scene {s}: velocity error {ev:.3e}"
        assert ew <= REL, f"scene {s}: angular velocity error {ew:.3e}"
        assert eq <= Q_ANGLE, f"scene {s}: orientation error {eq:.3e} rad"
    return rep

"""Helpers of the GPU tests: build the HIP simulation and the oracle from the
same float32 state, step both, and compare element by element."""
from __future__ import annotations

import numpy as np

from helpers import S
from oracle import oracle as O

# parity bar (single step, float32 GPU vs float64 oracle)
REL = 1e-4          # relative, with floors below
# A tolerance-mode scene that ends at the sweep cap above the tolerance (the
# step flags it NOT_CONVERGED) has no converged solution: its state is the
# cap's iterate, and along the directions the sweeps do not contract (the
# split among a sliding box's four corners, whose friction torque follows
# it) float32 and float64 iterates part over 1,000 sweeps (measured 1.2e-4
# on a spinning box sliding on a shelf).  Such scenes are held to this bar.
REL_CAPPED = 1e-3
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


def arm_snapshot32(ora):
    """Float32 articulated-arm state of an oracle run [S, 3, 7] (joint rates,
    motor targets, motor impulses), and the oracle reset to exactly it."""
    ast = ora.arm_state.astype(np.float32)
    ora.arm_state[:] = ast.astype(np.float64)
    return ast.reshape(-1, 3, 7)


def joint_snapshot32(ora):
    """Float32 joint state of the container parts [2, N] (q, qd planes, the
    library's layout), and the oracle reset to exactly it."""
    js = ora.joint_state.reshape(-1, 2).astype(np.float32)
    ora.joint_state[:] = js.astype(np.float64).reshape(-1)
    return np.ascontiguousarray(js.T)


def gpu_set_rest(sim, rest):
    """Copy the oracle's per-body rest counters into the simulation."""
    import torch
    sim.rest.copy_(torch.as_tensor(np.asarray(rest, np.int32)))


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
    out["rest"] = sim.rest.cpu().numpy().copy()
    out["arm_state"] = sim.arm_state.cpu().numpy().copy() if sim.arm_state is not None else None
    out["joint_state"] = sim.joint_state.cpu().numpy().copy() if sim.joint_state is not None else None
    return out


def body_radii(batch, b0, b1):
    """Bounding radii of bodies [b0, b1): a hull's is its bounding box's
    half-diagonal (from its library vertices), the others' from their params."""
    out = []
    for i in range(b0, b1):
        if int(batch.shape[i]) == S.HULL:
            v0, nv = batch.hull_index[int(batch.param[i, 0])][:2]
            ext = np.abs(batch.hull_vert[v0:v0 + nv]).max(axis=0)
            out.append(float(np.linalg.norm(ext)))
        else:
            out.append(S.bounding_radius(int(batch.shape[i]), batch.param[i]))
    return np.array(out)


def _find(par, x):
    while par[x] != x:
        par[x] = par[par[x]]
        x = par[x]
    return x


def affected_bodies(batch, s, g, r):
    """Local indices of the bodies of scene s whose results may differ
    between the two sides: the bodies of a pair with a tie-band decision in
    the oracle, and every dynamic body linked to one of them through the
    contacts of either side (a contact couples its bodies' impulses; static,
    kinematic bodies and the ground do not link).  Outside this set, a
    step's pairs, contacts, colours (first fit only looks at contacts that
    share a dynamic body) and, with a fixed sweep count, the solve are
    independent of the tied decision."""
    b0, b1 = int(batch.body_offset[s]), int(batch.body_offset[s + 1])
    nb = b1 - b0
    tied = np.nonzero(r["tied"][b0:b1])[0]
    if tied.size == 0:
        return np.zeros(nb, bool)
    dyn = batch.motion[b0:b1] == S.DYNAMIC
    par = list(range(nb))
    if int(batch.arm) == 2:  # the articulated arm's links are one body
        for i in range(nb - 6, nb):
            par[i] = nb - 7
    keys = [r["c_key"][s, :int(r["n_contacts"][s])], g["key"][s, :int(g["count"][s])].astype(np.uint32)]
    for kk in keys:
        for k in kk:
            a, b = int(k) >> 20, (int(k) >> 8) & 0xFFF
            if b == 0xFFF or b >= nb or a >= nb or not (dyn[a] and dyn[b]):
                continue
            ra, rb = _find(par, a), _find(par, b)
            if ra != rb:
                par[ra] = rb
    roots = {_find(par, int(t)) for t in tied}
    aff = np.array([_find(par, i) in roots for i in range(nb)])
    aff[tied] = True
    return aff


def _keep_pairs(keys, aff):
    a = keys >> 16
    b = keys & 0xFFFF
    ok = ~aff[a]
    gb = b != 0xFFFF
    ok[gb] &= ~aff[b[gb]]
    return ok


def _keep_contacts(keys, aff):
    a = keys >> 20
    b = (keys >> 8) & 0xFFF
    ok = ~aff[a]
    gb = b != 0xFFF
    ok[gb] &= ~aff[b[gb]]
    return ok


# contact value bars (float32 geometry of lengths up to a few metres)
N_ATOL = 1e-5      # unit normal
P_ATOL = 1e-5      # m
PHI_ATOL = 1e-5    # m
LAM_REL = 2e-4     # per-body resultant impulses, relative to the scene's largest impulse ...
LAM_ABS = 1e-6     # ... plus this (N s)
# The impulses of a statically indeterminate contact set (a box's four
# corners on a face, a body wedged between two supports or pushed by the
# arm while it stands on the floor) are not unique: only their resultant
# on each body is, and that is held to LAM_REL (force, and torque about a
# common point divided by the body's bounding radius).  The split among
# such contacts follows rounding: measured 2.3e-4 of the scene's largest
# impulse after 20 sweeps and 1.3e-2 after 1,000 (tolerance mode, capped),
# so single contacts are held to these looser bars (a wrong sign, row or
# contact still fails them).
LAM_REL_C = 1e-3
LAM_REL_TOL = 3e-2


def tangents(n):
    """Contact tangent basis of unit normals n [k, 3] (Duff et al. 2017,
    branch at n.z = -1/2, as the step uses)."""
    sg = np.where(n[:, 2] >= -0.5, 1.0, -1.0)
    a = -1.0 / (sg + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    t1 = np.stack([1.0 + sg * n[:, 0] ** 2 * a, sg * b, -sg * n[:, 0]], 1)
    t2 = np.stack([b, sg + n[:, 1] ** 2 * a, -n[:, 1]], 1)
    return t1, t2


def resultants(keys, lam, normal, point, xref):
    """Per-body sums of the contact impulses (n, t1, t2 components) as
    world force and torque about the bodies' reference points xref [nb, 3]
    (a contact's impulse acts +P on body a, -P on body b)."""
    n = np.asarray(normal, np.float64)
    t1, t2 = tangents(n)
    lam = np.asarray(lam, np.float64)
    P = lam[:, :1] * n + lam[:, 1:2] * t1 + lam[:, 2:3] * t2
    pt = np.asarray(point, np.float64)
    F = np.zeros((len(xref), 3))
    T = np.zeros((len(xref), 3))
    for i, k in enumerate(np.asarray(keys, np.int64)):
        a, b = int(k >> 20), int((k >> 8) & 0xFFF)
        F[a] += P[i]
        T[a] += np.cross(pt[i] - xref[a], P[i])
        if b != 0xFFF:
            F[b] -= P[i]
            T[b] -= np.cross(pt[i] - xref[b], P[i])
    return F, T


def compare(batch, g, r, ora, check_values=True, contact_values=False, partial=True, tol_band=None, scenes=None,
            check_rest=False):
    """Element-by-element comparison of one step.

    Unflagged scenes (no oracle decision in the tie band): pair keys,
    contact keys, colours and colour counts bit-exact; with check_values,
    positions (1e-4 relative, floor 1 m), velocities (1e-4 relative to the
    speed, floor 1 m/s; angular velocities as the surface speed |w| r of
    the body) and orientations (1e-4 rad); with contact_values, normals,
    points, depths and impulses of every contact (impulses at LAM_REL_C with a
    fixed sweep count, at LAM_REL_TOL in tolerance mode) and every dynamic
    body's resultant contact impulse at LAM_REL.  Flagged scenes
    (partial=True): pairs, contact keys and contact geometry outside the
    tied pairs' bodies, colours, impulses and states outside their islands
    (`affected_bodies`).

    Sweep counts: with a fixed sweep count they are equal by construction.
    In tolerance mode (tol_band set) they must be equal in unflagged scenes
    unless the oracle's residual came within tol_band * tol of the tolerance
    at one of its stopping tests (r["tol_gap"] < tol_band, the stop
    decision's own tie band); where the counts differ, impulses and states
    are not compared (the pre-solve results still are).  Returns a report;
    raises on a mismatch."""
    rep = dict(scenes=0, flagged=0, flagged_compared=0, skipped=0, sweeps_equal=0, sweeps_band=0,
               values_skipped=0, bodies=0, bodies_excluded=0, bodies_tied=0, contacts=0, contacts_solved=0,
               pairs=0, max_x=0.0, max_v=0.0,
               max_w=0.0, max_q=0.0, max_n=0.0, max_p=0.0, max_phi=0.0, max_lam=0.0, max_res=0.0, capped=0)
    Sn = batch.n_scenes
    pose_o = ora.pose.reshape(-1, 7)
    vel_o = ora.vel.reshape(-1, 6)
    for s in (range(Sn) if scenes is None else scenes):
        rep["scenes"] += 1
        b0, b1 = int(batch.body_offset[s]), int(batch.body_offset[s + 1])
        flagged = r["ambiguous"][s] != 0
        same_sweeps = int(g["stats"]["sweeps"][s]) == int(r["sweeps"][s])
        rep["sweeps_equal"] += int(same_sweeps)
        if not same_sweeps and not flagged:
            near = tol_band is not None and r["tol_gap"][s] < tol_band
            assert near, (f"scene {s}: {int(g['stats']['sweeps'][s])} sweeps on the GPU, {int(r['sweeps'][s])} "
                          f"in the oracle (residual gap to the tolerance {r['tol_gap'][s]:.3g})")
            rep["sweeps_band"] += 1
        if flagged:
            rep["flagged"] += 1
            if not partial:
                rep["skipped"] += 1
                continue
            rep["flagged_compared"] += 1
        values = same_sweeps
        rep["values_skipped"] += int(not values)
        # pairs, contact keys and contact geometry are per pair: only the
        # tied pairs' own bodies are left out; colours, impulses and states
        # couple through the contacts: the tied bodies' islands are left out
        tied = r["tied"][b0:b1].astype(bool)
        aff = affected_bodies(batch, s, g, r)
        rep["bodies"] += b1 - b0
        rep["bodies_excluded"] += int(aff.sum())
        rep["bodies_tied"] += int(tied.sum())
        # pair sets
        np_o = int(r["n_pairs"][s])
        np_g = int(g["stats"]["pairs"][s])
        pk_o = r["pair_key"][s, :np_o]
        pk_g = g["pair_key"][s, :np_g].astype(np.uint32)
        if not flagged:
            assert np_g == np_o, f"scene {s}: {np_g} pairs on the GPU, {np_o} in the oracle"
        ko, kg_ = pk_o[_keep_pairs(pk_o, tied)], pk_g[_keep_pairs(pk_g, tied)]
        assert np.array_equal(kg_, ko), f"scene {s}: pair keys differ (flagged={flagged})"
        rep["pairs"] += len(ko)
        # contact keys, colours
        nc = int(r["n_contacts"][s])
        ncg = int(g["count"][s])
        if not flagged:
            assert ncg == nc, f"scene {s}: {ncg} contacts on the GPU, {nc} in the oracle"
            assert int(g["stats"]["colours"][s]) == int(r["n_colours"][s])
        ck_o = r["c_key"][s, :nc]
        ck_g = g["key"][s, :ncg].astype(np.uint32)
        mo, mg = _keep_contacts(ck_o, tied), _keep_contacts(ck_g, tied)
        assert np.array_equal(ck_g[mg], ck_o[mo]), f"scene {s}: contact keys differ (flagged={flagged})"
        rep["contacts"] += int(mo.sum())
        if contact_values and mo.any():
            io, ig = np.nonzero(mo)[0], np.nonzero(mg)[0]
            en = np.max(np.abs(g["normal"][:, s, ig].T - r["c_normal"][s, io]))
            ep = np.max(np.abs(g["point"][:, s, ig].T - r["c_point"][s, io]))
            eph = np.max(np.abs(g["phi"][s, ig] - r["c_phi"][s, io]))
            rep["max_n"] = max(rep["max_n"], en)
            rep["max_p"] = max(rep["max_p"], ep)
            rep["max_phi"] = max(rep["max_phi"], eph)
            assert en <= N_ATOL, f"scene {s}: normal error {en:.3e}"
            assert ep <= P_ATOL, f"scene {s}: point error {ep:.3e}"
            assert eph <= PHI_ATOL, f"scene {s}: depth error {eph:.3e}"
        # colours and impulses: outside the tied islands
        mo, mg = _keep_contacts(ck_o, aff), _keep_contacts(ck_g, aff)
        assert np.array_equal(ck_g[mg], ck_o[mo]), f"scene {s}: contact keys differ (flagged={flagged})"
        assert np.array_equal(g["colour"][s, :ncg][mg], r["c_colour"][s, :nc][mo]), \
            f"scene {s}: colours differ (flagged={flagged})"
        rep["contacts_solved"] += int(mo.sum())
        if contact_values and mo.any():
            io, ig = np.nonzero(mo)[0], np.nonzero(mg)[0]
            if values:
                lam_o = r["c_lambda"][s, io]
                scale = float(np.abs(r["c_lambda"][s, :nc]).max())
                el = np.max(np.abs(g["lam"][:, s, ig].T - lam_o))
                rep["max_lam"] = max(rep["max_lam"], el / max(scale, 1e-12))
                bar = LAM_REL_C if tol_band is None else LAM_REL_TOL
                assert el <= bar * scale + LAM_ABS, f"scene {s}: impulse error {el:.3e} (scale {scale:.3e})"
                # the unique part: every dynamic body's resultant outside the tied islands
                xref = pose_o[b0:b1, :3]
                Fo, To = resultants(ck_o[mo], lam_o, r["c_normal"][s, io], r["c_point"][s, io], xref)
                Fg, Tg = resultants(ck_g[mg], g["lam"][:, s, ig].T, g["normal"][:, s, ig].T,
                                    g["point"][:, s, ig].T, xref)
                dyn = (batch.motion[b0:b1] == S.DYNAMIC) & ~aff
                if int(batch.arm) == 2:  # links of the articulated arm: the arm as a whole is checked by its rates
                    dyn[-7:] = False
                rad = body_radii(batch, b0, b1)
                jk = batch.joint[b0:b1] if getattr(batch, "joint", None) is not None else np.zeros(b1 - b0, np.uint8)
                part = dyn & (jk > 0)
                dyn &= jk == 0
                if dyn.any():
                    eF = np.linalg.norm(Fg - Fo, axis=1)[dyn].max()
                    eT = (np.linalg.norm(Tg - To, axis=1) / rad)[dyn].max()
                    rep["max_res"] = max(rep["max_res"], max(eF, eT) / max(scale, 1e-12))
                    assert max(eF, eT) <= LAM_REL * scale + LAM_ABS, \
                        f"scene {s}: resultant impulse error force {eF:.3e} torque/r {eT:.3e} (scale {scale:.3e})"
                # a container part: its joint takes every impulse but the
                # generalised one (moment about the hinge line over the
                # bounding radius, or force along the slide), which is unique
                for i in np.nonzero(part)[0]:
                    ax = batch.joint_axis[b0 + i].astype(np.float64)
                    if jk[i] == 1:
                        o = batch.joint_anchor[b0 + i].astype(np.float64)
                        # moments about the anchor from those about xref: T_o = T_x + (x - o) x F
                        go = ax @ (To[i] + np.cross(xref[i] - o, Fo[i]))
                        gg = ax @ (Tg[i] + np.cross(xref[i] - o, Fg[i]))
                        eG = abs(gg - go) / rad[i]
                    else:
                        eG = abs(ax @ (Fg[i] - Fo[i]))
                    rep["max_res"] = max(rep["max_res"], eG / max(scale, 1e-12))
                    assert eG <= LAM_REL * scale + LAM_ABS, \
                        f"scene {s}: generalised impulse error {eG:.3e} on part {i} (scale {scale:.3e})"
        if not check_values or not values:
            continue
        capped = tol_band is not None and bool(int(r["flags"][s]) & O.F_NOT_CONVERGED)
        rep["capped"] += int(capped)
        bar = REL_CAPPED if capped else REL
        keep = ~aff
        xo, xg = pose_o[b0:b1, :3][keep], g["pose"][b0:b1, :3][keep]
        ex = np.max(np.abs(xg - xo) / np.maximum(np.abs(xo), X_FLOOR), initial=0.0)
        vo, vg = vel_o[b0:b1][keep], g["vel"][b0:b1][keep]
        # velocities as vectors: the error relative to the oracle's speed
        # (floor 1 m/s); an angular velocity by the surface speed |w| r it
        # gives the body (r its bounding radius), with the same floor
        rad = body_radii(batch, b0, b1)[keep]
        nv = np.linalg.norm
        ev = np.max(nv(vg[:, :3] - vo[:, :3], axis=1) / np.maximum(nv(vo[:, :3], axis=1), V_FLOOR), initial=0.0)
        ew = np.max(nv(vg[:, 3:] - vo[:, 3:], axis=1) * rad / np.maximum(nv(vo[:, 3:], axis=1) * rad, V_FLOOR),
                    initial=0.0)
        eq = np.max(quat_angle(pose_o[b0:b1, 3:][keep], g["pose"][b0:b1, 3:][keep]), initial=0.0)
        if check_rest:  # steps at rest: integers, equal outside the tied islands
            ro, rg = ora.rest[b0:b1][keep], g["rest"][b0:b1][keep]
            assert np.array_equal(rg, ro), f"scene {s}: rest counters differ"
        rep["max_x"] = max(rep["max_x"], ex)
        rep["max_v"] = max(rep["max_v"], ev)
        rep["max_w"] = max(rep["max_w"], ew)
        rep["max_q"] = max(rep["max_q"], eq)
        assert ex <= bar, f"scene {s}: position error {ex:.3e}"
        assert ev <= bar, f"scene {s}: velocity error {ev:.3e} (capped {capped})"
        assert ew <= bar, f"scene {s}: angular velocity error {ew:.3e} (capped {capped})"
        assert eq <= (10 * Q_ANGLE if capped else Q_ANGLE), f"scene {s}: orientation error {eq:.3e} rad"
    rep["flagged_frac"] = rep["flagged"] / max(rep["scenes"], 1)
    rep["excluded_frac"] = rep["bodies_excluded"] / max(rep["bodies"], 1)
    return rep


def report(name, rep):
    """One line per parity check: how much was compared and how much the tie band excluded."""
    print(f"[parity] {name}: scenes {rep['scenes']}, flagged {rep['flagged']} "
          f"({100 * rep['flagged_frac']:.0f}%, {rep['flagged_compared']} compared outside the tied islands, "
          f"{rep['skipped']} skipped), sweeps equal in {rep['sweeps_equal']} ({rep['sweeps_band']} differ inside "
          f"the stop band, values skipped in {rep['values_skipped']}, capped {rep['capped']}), bodies tied {rep['bodies_tied']}, "
          f"in tied islands {100 * rep['excluded_frac']:.1f}%, pairs {rep['pairs']}, "
          f"contacts {rep['contacts']} ({rep['contacts_solved']} outside tied islands); max err x {rep['max_x']:.1e} v {rep['max_v']:.1e} w {rep['max_w']:.1e} "
          f"q {rep['max_q']:.1e} n {rep['max_n']:.1e} p {rep['max_p']:.1e} phi {rep['max_phi']:.1e} "
          f"lam/scale {rep['max_lam']:.1e} resultant/scale {rep['max_res']:.1e}", flush=True)

"""Test helpers: hand-built scene batches and state accessors."""
from __future__ import annotations

import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2106_14405_amd import scenes as S  # noqa: E402

DT = 1.0 / 120.0
G = 9.81


def quat_axis_angle(axis, angle):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    return np.concatenate([[math.cos(angle / 2)], math.sin(angle / 2) * a])


def quat_to_R(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def custom_batch(scenes_bodies, arm=False, theta=None):
    """scenes_bodies: list (per scene) of lists of dicts with keys
    shape, motion, param, mass, mu, e, pos, quat, vel (6)."""
    scs = []
    vels = []
    for bodies in scenes_bodies:
        sc = S.Scene()
        for b in bodies:
            sc.add(b.get("shape", S.SPHERE), b.get("motion", S.DYNAMIC), b.get("param", [0.1, 0, 0]),
                   b.get("mass", 1.0), b.get("mu", 0.5), b.get("e", 0.0), b["pos"],
                   b.get("quat", (1.0, 0.0, 0.0, 0.0)))
            vels.append(np.asarray(b.get("vel", np.zeros(6)), np.float64))
        if arm:
            sc.arm = True
            sc.arm_theta0 = np.zeros(7) if theta is None else np.asarray(theta, np.float64)
            for L in S.ARM_LINK_LENGTH:
                sc.add(S.CAPSULE, S.KINEMATIC, [S.ARM_RADIUS, 0.5 * L, 0.0], 0.0, 0.5, 0.0,
                       S.ARM_BASE, (1.0, 0.0, 0.0, 0.0))
                vels.append(np.zeros(6))
        scs.append(sc)
    b = S.pack(scs)
    b.vel = np.asarray(vels, np.float32).reshape(-1, 6)
    return b


def inertia(shape, p, m):
    """Principal moments (textbook solid bodies) for the momentum pins."""
    if shape == S.SPHERE:
        return np.full(3, 0.4 * m * p[0] ** 2)
    if shape == S.BOX:
        x2, y2, z2 = p[0] ** 2, p[1] ** 2, p[2] ** 2
        return np.array([m / 3 * (y2 + z2), m / 3 * (x2 + z2), m / 3 * (x2 + y2)])
    r, h = p[0], p[1]
    vc, vs = 2 * math.pi * r * r * h, 4 / 3 * math.pi * r ** 3
    mc = m * vc / (vc + vs)
    ms = m - mc
    Iz = mc * r * r / 2 + 0.4 * ms * r * r
    Ix = mc * (r * r / 4 + h * h / 3) + ms * (0.4 * r * r + h * h + 0.75 * h * r)
    return np.array([Ix, Ix, Iz])


def momenta(batch, pose, vel):
    """Total linear and angular momentum (about the origin) of dynamic bodies."""
    P = np.zeros(3)
    L = np.zeros(3)
    pose = np.asarray(pose, np.float64).reshape(-1, 7)
    vel = np.asarray(vel, np.float64).reshape(-1, 6)
    for i in range(batch.n_bodies):
        if batch.motion[i] != S.DYNAMIC:
            continue
        m = float(batch.mass[i])
        R = quat_to_R(pose[i, 3:])
        I = R @ np.diag(inertia(int(batch.shape[i]), batch.param[i].astype(np.float64), m)) @ R.T
        P += m * vel[i, :3]
        L += np.cross(pose[i, :3], m * vel[i, :3]) + I @ vel[i, 3:]
    return P, L


def kinetic(batch, pose, vel):
    pose = np.asarray(pose, np.float64).reshape(-1, 7)
    vel = np.asarray(vel, np.float64).reshape(-1, 6)
    E = 0.0
    for i in range(batch.n_bodies):
        if batch.motion[i] != S.DYNAMIC:
            continue
        m = float(batch.mass[i])
        R = quat_to_R(pose[i, 3:])
        I = R @ np.diag(inertia(int(batch.shape[i]), batch.param[i].astype(np.float64), m)) @ R.T
        E += 0.5 * m * vel[i, :3] @ vel[i, :3] + 0.5 * vel[i, 3:] @ I @ vel[i, 3:]
    return E

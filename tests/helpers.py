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
        if arm:  # True / 1: kinematic links; 2: dynamic links with joint motors
            dyn = int(arm) == 2
            sc.arm = 2 if dyn else True
            sc.arm_theta0 = np.zeros(7) if theta is None else np.asarray(theta, np.float64)
            for L, lm in zip(S.ARM_LINK_LENGTH, S.ARM_LINK_MASS):
                sc.add(S.CAPSULE, S.DYNAMIC if dyn else S.KINEMATIC, [S.ARM_RADIUS, 0.5 * L, 0.0],
                       lm if dyn else 0.0, 0.5, 0.0, S.ARM_BASE, (1.0, 0.0, 0.0, 0.0))
                vels.append(np.zeros(6))
        scs.append(sc)
    b = S.pack(scs)
    b.vel = np.asarray(vels, np.float32).reshape(-1, 6)
    return b


def _quad(f, a, b, breaks=()):
    """Integral of f over [a, b] split at the given interior points (scipy's
    adaptive Gauss-Kronrod; every integrand below is a polynomial piece by
    piece, so the result is exact to rounding)."""
    from scipy.integrate import quad
    pts = [a, *sorted(x for x in breaks if a < x < b), b]
    return sum(quad(f, lo, hi, epsabs=0.0, epsrel=1e-13, limit=200)[0] for lo, hi in zip(pts[:-1], pts[1:]))


def _inertia_of_slices(rho2, z0, z1, breaks, m):
    """Principal moments about the centre of mass of a uniform solid of
    revolution about z whose cross-section at height z is a disk of squared
    radius rho2(z), scaled to mass m.  A disk of radius R at height z adds
    pi R^4 / 2 to I_z and pi R^4 / 4 + pi R^2 z^2 to I_x (per unit density
    and height); the volume is the integral of pi R^2."""
    vol = _quad(lambda z: math.pi * rho2(z), z0, z1, breaks)
    iz = _quad(lambda z: 0.5 * math.pi * rho2(z) ** 2, z0, z1, breaks)
    ix = _quad(lambda z: 0.25 * math.pi * rho2(z) ** 2 + math.pi * rho2(z) * z * z, z0, z1, breaks)
    return np.array([ix, ix, iz]) * (m / vol)


def inertia(shape, p, m):
    """Principal moments of a solid body of uniform density and mass m,
    integrated numerically over its volume (not from closed forms): a box
    as the separable integrals of y^2 + z^2 etc. over its extents, a sphere
    and a capsule (cylinder of half-length h with hemispherical caps) as
    stacks of disks along z."""
    p = [float(x) for x in p]
    if shape == S.BOX:
        hx, hy, hz = p
        vol = 8 * hx * hy * hz
        sx = _quad(lambda x: x * x, -hx, hx) * 4 * hy * hz / vol
        sy = _quad(lambda y: y * y, -hy, hy) * 4 * hx * hz / vol
        sz = _quad(lambda z: z * z, -hz, hz) * 4 * hx * hy / vol
        return m * np.array([sy + sz, sx + sz, sx + sy])
    if shape == S.SPHERE:
        r = p[0]
        return _inertia_of_slices(lambda z: r * r - z * z, -r, r, (), m)
    r, h = p[0], p[1]

    def rho2(z):
        u = abs(z) - h
        return r * r if u <= 0.0 else r * r - u * u

    return _inertia_of_slices(rho2, -h - r, h + r, (-h, h), m)


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

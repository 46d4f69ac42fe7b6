"""Seeded synthetic scene batches for the batched rigid-body step.

This module is the single source of inputs for both the HIP path and the
FP64 oracle.  It draws shapes, masses, materials, initial poses, arm joint
angles and per-step arm actions from a counter-based SplitMix64 stream
(Steele, Lea & Flood 2014) and returns plain numpy arrays.  It holds none of
the step's arithmetic: no inertia, no kinematics, no collision geometry, no
solver.  Rejection of initial overlaps uses bounding spheres only.

Workloads (stand-ins for the paper's ReplicaCAD/YCB rearrangement scenes,
Sec. 3 and Sec. 4.3; physics at 1/120 s per step, Sec. 4.4):

* ``drop_scene``   -- spheres and boxes dropped from uniform positions in a
  cube onto the ground plane (64 bodies in a 2 m cube for the small case;
  the cube edge grows as (n/64)^(1/3) for larger scenes).
* ``clutter_scene`` -- 20 static boxes (counters, shelves, walls), 108 dynamic
  spheres/boxes/capsules and a kinematic 7-link capsule arm.
* ``uneven_batch`` -- scenes with log-uniform dynamic body counts.

Conventions: z up, ground plane z = 0, quaternions (w, x, y, z) body->world,
box parameters are half-extents, capsule parameters are (radius, half-length
of the core segment along local z).
"""
from __future__ import annotations

import math
import os
import sys
from dataclasses import dataclass, field

import numpy as np

SPHERE, BOX, CAPSULE, HULL = 0, 1, 2, 3
DYNAMIC, STATIC, KINEMATIC = 0, 1, 2

ARM_LINKS = 7
ARM_LINK_LENGTH = (0.10, 0.30, 0.10, 0.30, 0.10, 0.20, 0.10)
ARM_RADIUS = 0.05
ARM_BASE = (0.0, 0.0, 0.8)
# link masses of the dynamic arm (kg), heavier near the base
ARM_LINK_MASS = (2.0, 2.0, 1.5, 1.5, 1.0, 1.0, 0.5)

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def _mix_np(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = z.astype(np.uint64, copy=True)
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def _mix_int(z: int) -> int:
    z &= _M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & _M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & _M64
    z ^= z >> 31
    return z


def stream_key(*ids: int) -> int:
    """Fold integer ids (seed, scene, purpose, ...) into one 64-bit key."""
    h = 0x243F6A8885A308D3
    for i in ids:
        h = _mix_int((h + _GOLDEN) ^ (int(i) & _M64))
    return h


def uniforms(key: int, count: int, start: int = 0) -> np.ndarray:
    """``count`` doubles in [0, 1) from stream ``key``: the 53 high bits of
    mix(key + (k+1)*golden) for k = start .. start+count-1."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key) + k * np.uint64(_GOLDEN)
    z = _mix_np(z)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


class _Stream:
    """Sequential reader over one counter-based stream (values are drawn in
    blocks; the k-th value depends only on (key, k))."""

    BLOCK = 4096

    def __init__(self, key: int):
        self.key = key
        self.pos = 0
        self._buf = np.empty(0)
        self._buf0 = 0

    def take(self, n: int) -> np.ndarray:
        end = self.pos + n
        if self.pos < self._buf0 or end > self._buf0 + len(self._buf):
            self._buf0 = self.pos
            self._buf = uniforms(self.key, max(n, self.BLOCK), self.pos)
        u = self._buf[self.pos - self._buf0:end - self._buf0]
        self.pos = end
        return u

    def uniform(self, lo, hi, n=None):
        if n is None:
            return float(lo + (hi - lo) * self.take(1)[0])
        return lo + (hi - lo) * self.take(n)


def _random_quat(st: _Stream) -> np.ndarray:
    """Uniform random unit quaternion (Shoemake 1992), (w, x, y, z)."""
    u1, u2, u3 = st.take(3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    t2, t3 = 2.0 * math.pi * u2, 2.0 * math.pi * u3
    return np.array([b * math.cos(t3), a * math.sin(t2), a * math.cos(t2), b * math.sin(t3)])


def _yaw_quat(yaw: float) -> np.ndarray:
    return np.array([math.cos(0.5 * yaw), 0.0, 0.0, math.sin(0.5 * yaw)])


# ---- convex hulls (collision proxies of objects: Sec. 3, Sec. 4.3) -------
# Three families of convex polyhedra, each built in its principal frame by
# symmetry (mirror-symmetric about z = 0 and either mirror-symmetric about
# x = 0 and y = 0 or a regular polygon in the xy-plane): the centre of mass
# is the origin and the coordinate axes are principal axes.  A hull is
# (vertices [V, 3], face loops [F] of vertex indices, counter-clockwise
# seen from outside).

def _loop_ccw(V, idx, n):
    """Vertex indices idx of a planar face, ordered counter-clockwise seen
    from outside (outward direction n)."""
    P = V[idx]
    c = P.mean(axis=0)
    t1 = P[0] - c
    t1 = t1 - n * (t1 @ n)
    t1 = t1 / np.linalg.norm(t1)
    t2 = np.cross(n, t1)
    ang = np.arctan2((P - c) @ t2, (P - c) @ t1)
    return [int(idx[i]) for i in np.argsort(ang, kind="stable")]


def hull_prism(n: int, r: float, h: float):
    """Regular n-gonal prism: circumradius r, half-height h."""
    th = 2.0 * math.pi * np.arange(n) / n
    ring = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    V = np.concatenate([np.c_[ring, np.full(n, -h)], np.c_[ring, np.full(n, h)]])
    F = [list(range(n, 2 * n)), list(range(n - 1, -1, -1))]
    F += [[k, (k + 1) % n, n + (k + 1) % n, n + k] for k in range(n)]
    return V, F


def hull_bipyramid(n: int, r: float, h: float):
    """Regular n-gonal bipyramid: equator circumradius r, apexes at +-h."""
    th = 2.0 * math.pi * np.arange(n) / n
    V = np.concatenate([np.c_[r * np.cos(th), r * np.sin(th), np.zeros(n)], [[0.0, 0.0, h], [0.0, 0.0, -h]]])
    F = [[k, (k + 1) % n, n] for k in range(n)] + [[(k + 1) % n, k, n + 1] for k in range(n)]
    return V, F


def hull_chamfered_box(hx: float, hy: float, hz: float, t: float):
    """Box of half-extents (hx, hy, hz) with its 8 corners cut off t along
    each edge: 24 vertices, 6 octagons and 8 triangles."""
    h = np.array([hx, hy, hz])
    V, corner = [], {}
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                sg = np.array([sx, sy, sz], float)
                ids = []
                for ax in range(3):
                    p = sg * h
                    p[ax] -= sg[ax] * t
                    ids.append(len(V))
                    V.append(p)
                corner[(sx, sy, sz)] = ids
    V = np.array(V)
    F = []
    for ax in range(3):
        for sg in (-1, 1):
            nrm = np.zeros(3)
            nrm[ax] = sg
            idx = np.array([i for i in range(len(V)) if abs(V[i, ax] - sg * h[ax]) < 1e-12])
            F.append(_loop_ccw(V, idx, nrm))
    for key, ids in corner.items():
        F.append(_loop_ccw(V, np.array(ids), np.array(key, float) / math.sqrt(3.0)))
    return V, F


def random_hull(st: "_Stream", size=(0.05, 0.15)):
    """A hull of a random family and size: prisms and bipyramids of 3 to 8
    sides (circumradius and half-height U[size]), chamfered boxes
    (half-extents U[size], cut U[0.2, 0.45] of the smallest)."""
    fam = int(st.take(1)[0] * 3.0)
    if fam == 0:
        return hull_prism(3 + int(st.take(1)[0] * 6.0), st.uniform(*size), st.uniform(*size))
    if fam == 1:
        return hull_bipyramid(3 + int(st.take(1)[0] * 6.0), st.uniform(*size), st.uniform(*size))
    h = st.uniform(size[0], size[1], 3)
    return hull_chamfered_box(h[0], h[1], h[2], st.uniform(0.2, 0.45) * float(np.min(h)))


def hull_radius(V) -> float:
    """Largest vertex distance from the origin."""
    return float(np.max(np.linalg.norm(np.asarray(V, float), axis=1)))


def bounding_radius(shape: int, param) -> float:
    """Radius of a sphere about the centre that encloses the shape (a hull:
    its bounding box's half-diagonal, given as param)."""
    if shape == SPHERE:
        return float(param[0])
    if shape in (BOX, HULL):
        return float(math.sqrt(param[0] ** 2 + param[1] ** 2 + param[2] ** 2))
    return float(param[0] + param[1])


@dataclass
class Scene:
    """One scene: per-body arrays (float64 until packed)."""

    shape: list = field(default_factory=list)
    motion: list = field(default_factory=list)
    param: list = field(default_factory=list)
    mass: list = field(default_factory=list)
    friction: list = field(default_factory=list)
    restitution: list = field(default_factory=list)
    pose: list = field(default_factory=list)
    arm: bool = False
    arm_base: tuple = ARM_BASE
    arm_theta0: np.ndarray | None = None
    # articulated container parts: body index -> (joint 1 revolute / 2
    # prismatic, unit axis, anchor point, (lo, hi) limits, parent body index)
    joints: dict = field(default_factory=dict)
    # convex hulls of the scene's HULL bodies ((vertices, face loops)); a
    # HULL body's param[0] is its index here
    hulls: list = field(default_factory=list)

    def add_hull(self, verts, faces, motion, mass, mu, e, pos, quat):
        self.hulls.append((np.asarray(verts, np.float64), [list(f) for f in faces]))
        self.add(HULL, motion, [float(len(self.hulls) - 1), 0.0, 0.0], mass, mu, e, pos, quat)

    def add(self, shape, motion, param, mass, mu, e, pos, quat):
        self.shape.append(shape)
        self.motion.append(motion)
        self.param.append(np.asarray(param, dtype=np.float64))
        self.mass.append(mass)
        self.friction.append(mu)
        self.restitution.append(e)
        self.pose.append(np.concatenate([np.asarray(pos, np.float64), np.asarray(quat, np.float64)]))

    @property
    def n(self):
        return len(self.shape)


def _static_clear(p, R, statics) -> bool:
    """Bounding sphere (p, R) clear of every static yawed box."""
    for (c, h, yaw) in statics:
        d = p - c
        cs, sn = math.cos(yaw), math.sin(yaw)
        lx = cs * d[0] + sn * d[1]
        ly = -sn * d[0] + cs * d[1]
        lz = d[2]
        qx = min(max(lx, -h[0]), h[0])
        qy = min(max(ly, -h[1]), h[1])
        qz = min(max(lz, -h[2]), h[2])
        if (lx - qx) ** 2 + (ly - qy) ** 2 + (lz - qz) ** 2 < R * R:
            return False
    return True


def _place(st, R, lo, hi, placed, statics=(), keepout=None, tries=4000):
    """Rejection-sample a centre in the box [lo, hi] whose bounding sphere of
    radius R overlaps no placed sphere, no static box and no keep-out sphere."""
    if placed:
        P = np.asarray([q[0] for q in placed])
        Rr = np.asarray([q[1] for q in placed])
    for _ in range(tries):
        p = lo + (hi - lo) * st.take(3)
        ok = True
        if placed:
            if np.any(np.sum((P - p) ** 2, axis=1) < (Rr + R) ** 2):
                ok = False
        if ok and keepout is not None:
            kc, kr = keepout
            if np.sum((p - kc) ** 2) < (kr + R) ** 2:
                ok = False
        if ok and statics and not _static_clear(p, R, statics):
            ok = False
        if ok:
            return p
    raise RuntimeError("scene generator could not place a body without overlap")


def drop_scene(seed: int, n_spheres: int = 32, n_boxes: int = 32, size=(0.05, 0.15),
               mass=(0.1, 2.0), friction=0.5, edge: float | None = None, n_capsules: int = 0,
               n_hulls: int = 0) -> Scene:
    """Spheres and boxes (and capsules: radius U[0.03, 0.1], half-length
    U[size]; and convex hulls: random_hull) dropped from uniform positions
    in a cube onto the ground: x, y in [-L/2, L/2], z in [0.2, 0.2 + L],
    L = 2 m * (n/64)^(1/3) unless given; uniform orientation; zero
    velocity; restitution 0.  Hull shapes come from a stream of their own."""
    st = _Stream(stream_key(seed, 1))
    sth = _Stream(stream_key(seed, 10))
    n = n_spheres + n_boxes + n_capsules + n_hulls
    L = edge if edge is not None else 2.0 * (n / 64.0) ** (1.0 / 3.0)
    kinds = np.array([SPHERE] * n_spheres + [BOX] * n_boxes + [CAPSULE] * n_capsules + [HULL] * n_hulls)
    order = np.argsort(st.take(n), kind="stable")
    kinds = kinds[order]
    sc = Scene()
    placed = []
    lo = np.array([-0.5 * L, -0.5 * L, 0.2])
    hi = np.array([0.5 * L, 0.5 * L, 0.2 + L])
    for k in kinds:
        hv = None
        if k == SPHERE:
            param = [st.uniform(*size), 0.0, 0.0]
        elif k == BOX:
            param = list(st.uniform(size[0], size[1], 3))
        elif k == CAPSULE:
            param = [st.uniform(0.03, 0.1), st.uniform(*size), 0.0]
        else:
            hv, hf = random_hull(sth, size)
        m = st.uniform(*mass)
        R = hull_radius(hv) if hv is not None else bounding_radius(int(k), param)
        p = _place(st, R, lo, hi, placed)
        placed.append((p, R))
        q = _random_quat(st)
        if hv is not None:
            sc.add_hull(hv, hf, DYNAMIC, m, friction, 0.0, p, q)
        else:
            sc.add(int(k), DYNAMIC, param, m, friction, 0.0, p, q)
    return sc


def _yaw_boxes_overlap(c1, h1, yaw1, c2, h2, yaw2) -> bool:
    """Whether two boxes turned about z only overlap: their z intervals and
    their footprints (separating axes: the four edge normals)."""
    if abs(c1[2] - c2[2]) >= h1[2] + h2[2]:
        return False
    d = np.asarray(c2[:2], np.float64) - np.asarray(c1[:2], np.float64)
    u1 = [np.array([math.cos(yaw1), math.sin(yaw1)]), np.array([-math.sin(yaw1), math.cos(yaw1)])]
    u2 = [np.array([math.cos(yaw2), math.sin(yaw2)]), np.array([-math.sin(yaw2), math.cos(yaw2)])]
    for ax in u1 + u2:
        r1 = h1[0] * abs(u1[0] @ ax) + h1[1] * abs(u1[1] @ ax)
        r2 = h2[0] * abs(u2[0] @ ax) + h2[1] * abs(u2[1] @ ax)
        if abs(d @ ax) >= r1 + r2:
            return False
    return True


def _plan_cabinet(st: _Stream, taken: list, ring=(0.75, 1.2)) -> dict:
    """A cabinet facing the arm base (Sec. 3: furniture with articulated
    doors and drawers): a static carcass of half-extents U[0.2, 0.3] x
    U[0.25, 0.4] x U[0.35, 0.5] m on the floor, its front face U[ring] m
    from the base (horizontally), clear of the cabinets in `taken`
    (footprints with the door's swing and the drawer's travel in front);
    the door 2-5 kg, the drawer 1-3 kg.  Placed before the static boxes,
    which then keep clear of it."""
    cx, cy, cz = st.uniform(0.2, 0.3), st.uniform(0.25, 0.4), st.uniform(0.35, 0.5)
    mu_c = st.uniform(0.3, 0.8)
    m_door, m_drawer = st.uniform(2.0, 5.0), st.uniform(1.0, 3.0)
    base = np.array(ARM_BASE[:2])
    hc = np.array([cx, cy, cz])
    hf = np.array([cy, cy + 0.05, cz])        # in front: the door's swing and the drawer's travel
    for _ in range(4000):
        ang, front = st.uniform(0.0, 2.0 * math.pi), st.uniform(*ring)
        f = np.array([math.cos(ang), math.sin(ang)])          # from the base outwards
        c2 = base + f * (front + cx)
        C = np.array([c2[0], c2[1], cz])
        F = np.array([c2[0] - f[0] * (cx + cy), c2[1] - f[1] * (cx + cy), cz])
        if not any(_yaw_boxes_overlap(b, h, ang, c, ho, yo) for (b, h) in ((C, hc), (F, hf))
                   for (c, ho, yo) in taken):
            break
    else:
        raise RuntimeError("could not place a cabinet")
    taken += [(C, hc, ang), (F, hf, ang)]
    return dict(C=C, h=hc, yaw=ang + math.pi, mu=mu_c, m_door=m_door, m_drawer=m_drawer)


def _add_cabinet(sc: Scene, cab: dict, statics: list) -> None:
    """The cabinet's bodies: the carcass; a door over the upper half of the
    front on a vertical hinge at one side edge, opening outwards (q in
    [0, 1.9] rad); a drawer in the lower half, its front 2 cm proud of the
    carcass, sliding out along the front normal (q in [0, 1.2 hx] m).  Both
    parts are joined to the carcass (no contacts with it)."""
    C, (cx, cy, cz), yaw, mu_c = cab["C"], cab["h"], cab["yaw"], cab["mu"]
    fn = np.array([math.cos(yaw), math.sin(yaw), 0.0])         # local +x: the front normal, towards the base
    sd = np.array([-math.sin(yaw), math.cos(yaw), 0.0])
    q = _yaw_quat(yaw)
    ic = sc.n
    sc.add(BOX, STATIC, [cx, cy, cz], 0.0, mu_c, 0.0, C, q)
    statics.append((C, np.array([cx, cy, cz]), yaw))
    # door: half-extents (0.015, cy - 0.005, cz / 2 - 0.005) over the upper half,
    # hinge at the +side edge (turning by +q about z swings it outwards)
    hd = np.array([0.015, cy - 0.005, 0.5 * cz - 0.005])
    pd = C + fn * (cx + hd[0] + 0.002) + np.array([0.0, 0.0, 0.5 * cz])
    sc.add(BOX, DYNAMIC, hd, cab["m_door"], mu_c, 0.0, pd, q)
    sc.joints[sc.n - 1] = (1, (0.0, 0.0, 1.0), pd + sd * cy, (0.0, 1.9), ic)
    statics.append((pd, hd, yaw))
    # drawer: in the lower half, its front 2 cm proud of the carcass
    hw = np.array([0.8 * cx, 0.85 * cy, 0.3 * cz])
    pw = C + fn * (cx + 0.02 - hw[0]) - np.array([0.0, 0.0, 0.5 * cz])
    sc.add(BOX, DYNAMIC, hw, cab["m_drawer"], mu_c, 0.0, pw, q)
    sc.joints[sc.n - 1] = (2, tuple(fn), pw, (0.0, 1.2 * cx), ic)
    statics.append((pw, hw, yaw))


def clutter_scene(seed: int, n_static: int = 20, n_each: int = 36, size=(0.03, 0.30),
                  cap_radius=(0.03, 0.15), mass=(0.05, 3.0), friction=(0.3, 0.8),
                  arm: int = True, n_dynamic: int | None = None, cabinets: int = 0) -> Scene:
    """Rearrangement clutter: static boxes on a 4 m x 4 m floor (a quarter of
    them floating shelves), dynamic spheres/boxes/capsules dropped above, and
    a 7-link capsule arm based at (0, 0, 0.8) m: kinematic (arm True or 1) or
    dynamic links of ARM_LINK_MASS joined by motorised joints (arm 2), the
    same scene otherwise.  With n_dynamic
    given, that many dynamic bodies (a third of each shape, the remainder to
    spheres then boxes) dropped from a region scaled by (n_dynamic/108)^(1/3)
    (x, y within +-2 m times the scale, z from 0.2 m up to 4 m times it).
    cabinets > 0 adds that many cabinets with a door and a drawer each
    (_plan_cabinet, _add_cabinet: drawn from a stream of their own and
    placed first; the static boxes keep clear of them; their bodies follow
    the static boxes)."""
    st = _Stream(stream_key(seed, 2) if n_dynamic is None else stream_key(seed, 6, n_dynamic))
    sc = Scene()
    statics = []
    cabs, taken = [], []
    if cabinets:  # placed first, from a stream of their own
        stc = _Stream(stream_key(seed, 9, cabinets))
        cabs = [_plan_cabinet(stc, taken) for _ in range(cabinets)]
    for i in range(n_static):
        hx, hy = st.uniform(0.15, 1.0), st.uniform(0.15, 1.0)
        shelf = st.take(1)[0] < 0.25
        if shelf:
            hz = st.uniform(0.01, 0.05)
            z = st.uniform(0.5, 1.5)
        else:
            hz = st.uniform(0.15, 1.0)
            z = hz
        yaw = st.uniform(0.0, 2.0 * math.pi)
        rad = math.hypot(hx, hy)
        for _ in range(4000):
            x, y = st.uniform(-2.0, 2.0), st.uniform(-2.0, 2.0)
            if math.hypot(x, y) - rad >= 0.8 and not any(
                    _yaw_boxes_overlap((x, y, z), (hx, hy, hz), yaw, c, h, y2) for (c, h, y2) in taken):
                break
        else:
            raise RuntimeError("could not place static box")
        c = np.array([x, y, z])
        statics.append((c, np.array([hx, hy, hz]), yaw))
        sc.add(BOX, STATIC, [hx, hy, hz], 0.0, st.uniform(*friction), 0.0, c, _yaw_quat(yaw))
    for cab in cabs:
        _add_cabinet(sc, cab, statics)
    reach = sum(ARM_LINK_LENGTH) + ARM_RADIUS
    keepout = (np.array(ARM_BASE), reach) if arm else None
    if n_dynamic is None:
        counts, scale = (n_each, n_each, n_each), 1.0
    else:
        third = n_dynamic // 3
        rem = n_dynamic - 3 * third
        counts = (third + (rem > 0), third + (rem > 1), third)
        scale = (n_dynamic / 108.0) ** (1.0 / 3.0)
    kinds = np.array([SPHERE] * counts[0] + [BOX] * counts[1] + [CAPSULE] * counts[2])
    kinds = kinds[np.argsort(st.take(len(kinds)), kind="stable")]
    placed = []
    lo = np.array([-2.0 * scale, -2.0 * scale, 0.2])
    hi = np.array([2.0 * scale, 2.0 * scale, 0.2 + 4.0 * scale])
    for k in kinds:
        if k == SPHERE:
            param = [st.uniform(*size), 0.0, 0.0]
        elif k == BOX:
            param = list(st.uniform(size[0], size[1], 3))
        else:
            param = [st.uniform(*cap_radius), st.uniform(*size), 0.0]
        m = st.uniform(*mass)
        mu = st.uniform(*friction)
        R = bounding_radius(int(k), param)
        p = _place(st, R, lo, hi, placed, statics, keepout)
        placed.append((p, R))
        sc.add(int(k), DYNAMIC, param, m, mu, 0.0, p, _random_quat(st))
    if arm:
        dyn = int(arm) == 2
        sc.arm = 2 if dyn else True
        sc.arm_theta0 = st.uniform(-0.5, 0.5, ARM_LINKS)
        for L, lm in zip(ARM_LINK_LENGTH, ARM_LINK_MASS):
            # pose is a placeholder: arm link poses follow from joint angles
            sc.add(CAPSULE, DYNAMIC if dyn else KINEMATIC, [ARM_RADIUS, 0.5 * L, 0.0], lm if dyn else 0.0,
                   0.5, 0.0, ARM_BASE, (1.0, 0.0, 0.0, 0.0))
    return sc


def _scale_one(args):
    seed, n, arm = args
    return clutter_scene(seed, arm=arm, n_dynamic=n)


def batch_scale(n_scenes: int = 16384, seed0: int = 30000, lo: int = 64, hi: int = 1024, arm: bool = True,
                workers=None) -> Batch:
    """Large clutter: per scene round(exp(U[ln lo, ln hi])) dynamic
    spheres/boxes/capsules with the clutter distributions in a scaled drop
    region, the 20 static boxes and the arm."""
    counts = log_uniform_counts(seed0, n_scenes, lo, hi)
    return pack(_map(_scale_one, [(seed0 + 1 + s, int(n), arm) for s, n in enumerate(counts)], workers))


def log_uniform_counts(seed: int, n_scenes: int, lo: int, hi: int) -> np.ndarray:
    u = uniforms(stream_key(seed, 3), n_scenes)
    return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


@dataclass
class Batch:
    """Packed batch of scenes (structure of arrays, bodies concatenated)."""

    body_offset: np.ndarray   # int32 [S+1]
    shape: np.ndarray         # uint8 [N]
    motion: np.ndarray        # uint8 [N]
    param: np.ndarray         # float32 [N,3]
    mass: np.ndarray          # float32 [N]
    friction: np.ndarray      # float32 [N]
    restitution: np.ndarray   # float32 [N]
    pose: np.ndarray          # float32 [N,7]  x y z qw qx qy qz
    vel: np.ndarray           # float32 [N,6]  v, omega (world)
    arm: int                  # 0 none, 1 (True) kinematic, 2 dynamic with joint motors
    arm_base: np.ndarray      # float32 [S,3]
    arm_theta: np.ndarray     # float32 [S,7]
    # articulated container parts (None: the batch has none): per body the
    # joint kind (0 none, 1 revolute, 2 prismatic), unit axis and anchor
    # (world, at the initial pose, where the joint coordinate is 0), limits
    # (lo, hi) of the coordinate, and the local index of the static body it
    # is joined to (-1: none)
    joint: np.ndarray | None = None          # uint8 [N]
    joint_axis: np.ndarray | None = None     # float32 [N,3]
    joint_anchor: np.ndarray | None = None   # float32 [N,3]
    joint_limits: np.ndarray | None = None   # float32 [N,2]
    joint_parent: np.ndarray | None = None   # int32 [N]
    # convex hulls (None: none): per hull (first vertex, vertex count, first
    # face, face count); vertices in the body frame; face loops padded with -1
    hull_index: np.ndarray | None = None     # int32 [H,4]
    hull_vert: np.ndarray | None = None      # float32 [V,3]
    hull_face: np.ndarray | None = None      # int32 [F,8]

    @property
    def n_scenes(self):
        return len(self.body_offset) - 1

    @property
    def n_bodies(self):
        return int(self.body_offset[-1])

    def counts(self):
        return np.diff(self.body_offset)


def pack(scenes: list[Scene]) -> Batch:
    if not scenes:
        raise ValueError("empty batch")
    arm = scenes[0].arm
    if any(s.arm != arm for s in scenes):
        raise ValueError("all scenes of a batch must agree on the arm")
    off = np.zeros(len(scenes) + 1, dtype=np.int32)
    off[1:] = np.cumsum([s.n for s in scenes])
    cat = lambda a, dt: np.concatenate([np.asarray(getattr(s, a), dtype=dt).reshape(s.n, -1)
                                        for s in scenes]).astype(dt)
    pose = cat("pose", np.float64)
    q = pose[:, 3:7]
    pose[:, 3:7] = q / np.linalg.norm(q, axis=1, keepdims=True)
    S = len(scenes)
    joint = axis = anchor = limits = parent = None
    if any(sc.joints for sc in scenes):
        N = int(off[-1])
        joint = np.zeros(N, np.uint8)
        axis = np.zeros((N, 3), np.float32)
        anchor = np.zeros((N, 3), np.float32)
        limits = np.zeros((N, 2), np.float32)
        parent = np.full(N, -1, np.int32)
        for si, sc in enumerate(scenes):
            for bi, (kind, ax, an, lim, par) in sc.joints.items():
                g = int(off[si]) + bi
                a = np.asarray(ax, np.float64)
                joint[g] = kind
                axis[g] = a / np.linalg.norm(a)
                anchor[g] = an
                limits[g] = lim
                parent[g] = par
    hull_index = hull_vert = hull_face = None
    param_all = cat("param", np.float64)
    if any(sc.hulls for sc in scenes):
        hi_, hv_, hf_ = [], [], []
        nv = nf = 0
        for si, sc in enumerate(scenes):
            base = len(hi_)
            for (V, F) in sc.hulls:
                hi_.append((nv, len(V), nf, len(F)))
                hv_.append(np.asarray(V, np.float64))
                for f in F:
                    row = np.full(8, -1, np.int32)
                    row[:len(f)] = f
                    hf_.append(row)
                nv += len(V)
                nf += len(F)
            for bi in range(sc.n):
                if sc.shape[bi] == HULL:
                    param_all[int(off[si]) + bi, 0] += base
        hull_index = np.asarray(hi_, np.int32).reshape(-1, 4)
        hull_vert = np.concatenate(hv_).astype(np.float32)
        hull_face = np.asarray(hf_, np.int32).reshape(-1, 8)
    return Batch(
        body_offset=off,
        shape=cat("shape", np.uint8).reshape(-1),
        motion=cat("motion", np.uint8).reshape(-1),
        param=param_all.astype(np.float32),
        mass=cat("mass", np.float64).reshape(-1).astype(np.float32),
        friction=cat("friction", np.float64).reshape(-1).astype(np.float32),
        restitution=cat("restitution", np.float64).reshape(-1).astype(np.float32),
        pose=pose.astype(np.float32),
        vel=np.zeros((off[-1], 6), np.float32),
        arm=arm,
        arm_base=np.tile(np.asarray(ARM_BASE, np.float32), (S, 1)),
        arm_theta=(np.stack([s.arm_theta0 for s in scenes]).astype(np.float32) if arm
                   else np.zeros((S, ARM_LINKS), np.float32)),
        joint=joint, joint_axis=axis, joint_anchor=anchor, joint_limits=limits, joint_parent=parent,
        hull_index=hull_index, hull_vert=hull_vert, hull_face=hull_face,
    )


def batch_drop(n_scenes: int = 1, seed0: int = 0, **kw) -> Batch:
    """Small drop case: per scene 32 spheres + 32 boxes, sizes U[0.05, 0.15] m,
    mass U[0.1, 2] kg, friction 0.5, restitution 0, 2 m cube."""
    return pack([drop_scene(seed0 + s, **kw) for s in range(n_scenes)])


def _clutter_one(args):
    seed, arm, kw = args
    return clutter_scene(seed, arm=arm, **kw)


def _drop_one(args):
    seed, ns, nb = args
    return drop_scene(seed, n_spheres=ns, n_boxes=nb)


def _gpu_initialised() -> bool:
    """True once this process has initialised the GPU runtime (torch imported
    and its CUDA/HIP state set up); a fork after that point is not allowed."""
    torch = sys.modules.get("torch")
    if torch is None:
        return False
    try:
        return bool(torch.cuda.is_initialized())
    except Exception:
        return True


def _map(fn, items, workers):
    """Map over scene seeds, in forked worker processes for large batches
    while the GPU runtime is not initialised in this process; serially after
    that (a process that has initialised the GPU must not fork)."""
    if workers is None:
        workers = min(16, os.cpu_count() or 1) if len(items) >= 64 else 1
    if workers > 1 and _gpu_initialised():
        workers = 1
    if workers <= 1:
        return [fn(a) for a in items]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(fn, items, chunksize=max(1, len(items) // (4 * workers)))


def batch_clutter(n_scenes: int = 1024, seed0: int = 10000, arm: bool = True, workers=None, **kw) -> Batch:
    """Clutter case: per scene 20 static boxes + 108 dynamic + 7 arm links."""
    return pack(_map(_clutter_one, [(seed0 + s, arm, kw) for s in range(n_scenes)], workers))


def batch_uneven(n_scenes: int = 4096, seed0: int = 20000, lo: int = 16, hi: int = 512, workers=None) -> Batch:
    """Uneven batch: dynamic counts log-uniform in [lo, hi], drop-case shapes."""
    counts = log_uniform_counts(seed0, n_scenes, lo, hi)
    items = [(seed0 + 1 + s, int(n) // 2, int(n) - int(n) // 2) for s, n in enumerate(counts)]
    return pack(_map(_drop_one, items, workers))


def _fresh_one(args):
    """Pool entry k of scene s: the scene's dynamic bodies re-placed (same
    shapes, masses and materials) at new rejection-sampled positions and
    uniform orientations in the scene's drop region, at rest; static bodies
    and the arm base stay; new joint angles for the arm."""
    key, kind, shape, motion, param, pose, arm = args
    st = _Stream(key)
    out = pose.astype(np.float64).copy()
    dyn = np.nonzero(motion == DYNAMIC)[0]
    statics = []
    for i in np.nonzero(motion == STATIC)[0]:
        q = pose[i, 3:7].astype(np.float64)
        statics.append((pose[i, :3].astype(np.float64), param[i].astype(np.float64),
                        2.0 * math.atan2(q[3], q[0])))
    if kind == "clutter":
        lo, hi = np.array([-2.0, -2.0, 0.2]), np.array([2.0, 2.0, 4.2])
        keepout = (np.array(ARM_BASE), sum(ARM_LINK_LENGTH) + ARM_RADIUS) if arm else None
    else:
        L = 2.0 * (len(dyn) / 64.0) ** (1.0 / 3.0)
        lo, hi = np.array([-0.5 * L, -0.5 * L, 0.2]), np.array([0.5 * L, 0.5 * L, 0.2 + L])
        keepout = None
    placed = []
    for i in dyn:
        R = bounding_radius(int(shape[i]), param[i])
        p = _place(st, R, lo, hi, placed, statics, keepout)
        placed.append((p, R))
        q = _random_quat(st)
        out[i, :3] = p
        out[i, 3:7] = q / np.linalg.norm(q)
    theta = st.uniform(-0.5, 0.5, ARM_LINKS) if arm else np.zeros(ARM_LINKS)
    return out.astype(np.float32), theta.astype(np.float32)


def reset_pool(batch: Batch, size: int, seed: int, kind: str = "drop", workers=None):
    """A pool of `size` fresh states of every scene of the batch, for masked
    episode resets: pose [K, N, 7] float32, velocity zeros [K, N, 6] and arm
    joint angles [K, S, 7].  Entry k of scene s comes from stream
    (seed, 5, s, k); kind "drop" re-drops the dynamic bodies in the scene's
    cube (edge 2 m (n/64)^(1/3)), "clutter" in the clutter region, clear of
    the statics and the arm's reach."""
    S_, N = batch.n_scenes, batch.n_bodies
    items = []
    for k in range(size):
        for s in range(S_):
            b0, b1 = int(batch.body_offset[s]), int(batch.body_offset[s + 1])
            items.append((stream_key(seed, 5, s, k), kind, batch.shape[b0:b1], batch.motion[b0:b1],
                          batch.param[b0:b1], batch.pose[b0:b1], bool(batch.arm)))
    res = _map(_fresh_one, items, workers)
    pose = np.empty((size, N, 7), np.float32)
    theta = np.zeros((size, S_, ARM_LINKS), np.float32)
    for k in range(size):
        for s in range(S_):
            b0, b1 = int(batch.body_offset[s]), int(batch.body_offset[s + 1])
            p, th = res[k * S_ + s]
            pose[k, b0:b1] = p
            theta[k, s] = th
    return pose, np.zeros((size, N, 6), np.float32), theta


def _stream_keys(ids) -> np.ndarray:
    """stream_key over arrays: ids is a sequence of ints or uint64 arrays
    (broadcast together); same folding as stream_key."""
    with np.errstate(over="ignore"):
        h = np.uint64(0x243F6A8885A308D3)
        for i in ids:
            h = _mix_np((np.asarray(h, np.uint64) + np.uint64(_GOLDEN)) ^ np.asarray(i, np.uint64))
    return h


def arm_actions(seed: int, n_scenes: int, step: int) -> np.ndarray:
    """Joint velocities U[-1, 1] rad/s for one step, keyed (seed, scene, step, joint):
    joint k of scene s is value k of stream_key(seed, 4, s, step)."""
    keys = _stream_keys([seed, 4, np.arange(n_scenes, dtype=np.uint64), step])
    k = np.arange(1, ARM_LINKS + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = keys[:, None] + k[None, :] * np.uint64(_GOLDEN)
    u = (_mix_np(z) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (2.0 * u - 1.0).astype(np.float32)


def arm_actions_block(seed: int, n_scenes: int, step0: int, n_steps: int) -> np.ndarray:
    """[n_steps, S, 7] joint velocities; same values as ``arm_actions``."""
    return np.stack([arm_actions(seed, n_scenes, step0 + t) for t in range(n_steps)])


def arm_configurations(seed: int, n_scenes: int, M: int) -> np.ndarray:
    """[S, M, 7] candidate arm configurations (rad) as a sampling planner
    draws them, keyed (seed, 7, scene, configuration, joint): even-numbered
    configurations uniform in [-pi, pi] per joint, odd-numbered ones with
    joint 1 in [0.6, 2.4] rad (the arm leaning out and down over the floor and
    the furniture) and the rest uniform in [-pi, pi]."""
    s_ids = np.arange(n_scenes, dtype=np.uint64)[:, None]
    j_ids = np.arange(M, dtype=np.uint64)[None, :]
    keys = _stream_keys([seed, 7, s_ids, j_ids])                      # [S, M]
    k = np.arange(1, ARM_LINKS + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = keys[..., None] + k * np.uint64(_GOLDEN)
    u = (_mix_np(z) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    th = (2.0 * u - 1.0) * np.pi
    lean = np.arange(M) % 2 == 1
    th[:, lean, 1] = 0.6 + 1.8 * u[:, lean, 1]
    return th.astype(np.float32)

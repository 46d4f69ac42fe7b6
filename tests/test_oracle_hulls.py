"""Pins of the oracle's convex hulls (Sec. 3 and Sec. 4.3: objects collide
as convex hulls), each fixed by something other than the oracle's own
formulas:
- mass properties: a box-shaped hull has the box's closed-form inertia;
  every family's volume equals scipy's convex hull volume, its centre of
  mass is the origin and its inertia matches Monte Carlo quadrature over
  points the test itself classifies with scipy's half-spaces;
- a box entered as a hull gives the box routines' contacts (ground, sphere,
  capsule, box; the box routines are pinned elsewhere);
- sphere-hull and capsule-hull separations equal the distance a
  constrained minimisation finds (scipy SLSQP over convex combinations of
  the vertices); separated hull-hull contacts have their witness points on
  both surfaces (so none is closer than the true distance), and a hull
  resting face to face above another reports the gap exactly;
- a regular octagon of contact (two square prisms turned 45 degrees) is
  reduced to four of its corners spanning the largest quadrilateral;
- a hull dropped on the ground comes to rest on a face with its weight
  carried (normal impulses sum to m g dt)."""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial import ConvexHull

from helpers import DT, G, S
from oracle import oracle as O

FAMILIES = [S.hull_prism(5, 0.12, 0.08), S.hull_bipyramid(6, 0.1, 0.14), S.hull_chamfered_box(0.1, 0.13, 0.07, 0.03),
            S.hull_prism(3, 0.15, 0.05)]


def rquat(rng):
    q = rng.normal(size=4)
    return q / np.linalg.norm(q)


def rot(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def world(V, pose):
    return np.asarray(V) @ rot(pose[3:]).T + pose[:3]


BOX_V = np.array([[sx * 0.1, sy * 0.2, sz * 0.3] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)])
BOX_F = [[0, 4, 6, 2], [1, 3, 7, 5], [0, 1, 5, 4], [2, 6, 7, 3], [0, 2, 3, 1], [4, 5, 7, 6]]


def test_box_hull_inertia_closed_form():
    I, c, v = O.hull_mass([(BOX_V, BOX_F)], 0, 2.0)
    np.testing.assert_allclose(v, 0.2 * 0.4 * 0.6, rtol=1e-12)
    np.testing.assert_allclose(c, 0.0, atol=1e-15)
    want = np.diag([2.0 / 3.0 * (0.04 + 0.09), 2.0 / 3.0 * (0.01 + 0.09), 2.0 / 3.0 * (0.01 + 0.04)])
    np.testing.assert_allclose(I, want, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("k", range(len(FAMILIES)))
def test_hull_mass_properties_against_quadrature(k):
    V, F = FAMILIES[k]
    m = 1.7
    I, c, v = O.hull_mass([(V, F)], 0, m)
    ch = ConvexHull(V)
    np.testing.assert_allclose(v, ch.volume, rtol=1e-10)
    np.testing.assert_allclose(c, 0.0, atol=1e-12)          # built symmetric: centroid at the origin
    rng = np.random.default_rng(k)
    lo, hi = V.min(0), V.max(0)
    pts = rng.uniform(lo, hi, size=(1_000_000, 3))
    inside = np.all(pts @ ch.equations[:, :3].T + ch.equations[:, 3] <= 0, axis=1)
    q = pts[inside]
    cov = q.T @ q / len(q)
    want = m * (np.trace(cov) * np.eye(3) - cov)
    np.testing.assert_allclose(I, want, rtol=0, atol=1e-2 * np.abs(want).max())
    # principal frame: products of inertia vanish
    assert np.abs(I - np.diag(np.diag(I))).max() <= 1e-12 * np.abs(I).max()


def as_set(cs):
    return sorted([(round(p[3], 9), tuple(np.round(p[2], 9)), tuple(np.round(p[1], 9))) for p in cs])


@pytest.mark.parametrize("other", ["ground", "sphere", "capsule", "box"])
def test_box_as_hull_equals_box(other):
    """A box entered as the hull of its corners gives the same contacts as
    the box routines (configurations where the oracle reports no tie)."""
    rng = np.random.default_rng(11)
    hulls = [(BOX_V, BOX_F)]
    hb = [0.1, 0.2, 0.3]
    compared = 0
    for t in range(400):
        pa = np.r_[rng.normal(size=3) * 0.05 + [0, 0, 0.28], rquat(rng)]
        if other == "ground":
            ra, a1 = O.collide(S.BOX, hb, pa, margin=0.02)
            rh, a2 = O.collide(S.HULL, [0, 0, 0], pa, margin=0.02, hulls=hulls)
        else:
            shape = {"sphere": S.SPHERE, "capsule": S.CAPSULE, "box": S.BOX}[other]
            prm = {"sphere": [0.12, 0, 0], "capsule": [0.06, 0.15, 0], "box": [0.15, 0.1, 0.2]}[other]
            pb = np.r_[rng.normal(size=3) * 0.05 + [0, 0, -0.1 - rng.uniform(0, 0.25)], rquat(rng)]
            ra, a1 = O.collide(shape, prm, pb, S.BOX, hb, pa, margin=0.02)
            rh, a2 = O.collide(shape, prm, pb, S.HULL, [0, 0, 0], pa, margin=0.02, hulls=hulls)
        if a1 or a2 or not ra:
            continue
        assert len(ra) == len(rh)
        if len(ra) == 4 and as_set(ra) != as_set(rh):
            # a clipped face of more than 4 points: box_box anchors its
            # reduction at the first clipped point, the hull routine at the
            # smallest id; the normal is the same, the subsets may differ
            for x, y in zip(ra, rh):
                np.testing.assert_allclose(x[1], y[1], atol=1e-9)
            continue
        compared += 1
        np.testing.assert_allclose([c[3] for c in sorted(ra, key=lambda c: tuple(c[2]))],
                                   [c[3] for c in sorted(rh, key=lambda c: tuple(c[2]))], atol=1e-12)
        for x, y in zip(sorted(ra, key=lambda c: tuple(np.round(c[2], 9))), sorted(rh, key=lambda c: tuple(np.round(c[2], 9)))):
            np.testing.assert_allclose(x[1], y[1], atol=1e-9)
            np.testing.assert_allclose(x[2], y[2], atol=1e-9)
    assert compared >= 30


def dist_point_hull(p, W):
    """Least distance from p to the convex hull of the points W (SLSQP over
    convex weights)."""
    n = len(W)
    res = minimize(lambda lam: np.sum((lam @ W - p) ** 2), np.full(n, 1.0 / n), method="SLSQP",
                   bounds=[(0, 1)] * n, constraints=[{"type": "eq", "fun": lambda lam: np.sum(lam) - 1}],
                   options=dict(ftol=1e-16, maxiter=500))
    return math.sqrt(max(res.fun, 0.0))


def dist_seg_hull(a, b, W):
    n = len(W)

    def f(x):
        lam, t = x[:n], x[n]
        return np.sum((lam @ W - (a + t * (b - a))) ** 2)
    best = np.inf
    for t0 in (0.0, 0.5, 1.0):
        res = minimize(f, np.r_[np.full(n, 1.0 / n), t0], method="SLSQP", bounds=[(0, 1)] * (n + 1),
                       constraints=[{"type": "eq", "fun": lambda x: np.sum(x[:n]) - 1}],
                       options=dict(ftol=1e-16, maxiter=500))
        best = min(best, res.fun)
    return math.sqrt(max(best, 0.0))


def dist_hull_hull(WA, WB):
    na, nb = len(WA), len(WB)
    res = minimize(lambda x: np.sum((x[:na] @ WA - x[na:] @ WB) ** 2), np.r_[np.full(na, 1 / na), np.full(nb, 1 / nb)],
                   method="SLSQP", bounds=[(0, 1)] * (na + nb),
                   constraints=[{"type": "eq", "fun": lambda x: np.sum(x[:na]) - 1},
                                {"type": "eq", "fun": lambda x: np.sum(x[na:]) - 1}],
                   options=dict(ftol=1e-16, maxiter=1000))
    return math.sqrt(max(res.fun, 0.0))


@pytest.mark.parametrize("k", range(len(FAMILIES)))
def test_sphere_hull_distance(k):
    V, F = FAMILIES[k]
    rng = np.random.default_rng(20 + k)
    pose = np.r_[0.0, 0.0, 0.5, rquat(rng)]
    W = world(V, pose)
    r = 0.04
    n = 0
    for t in range(30):
        d = rng.normal(size=3)
        c = pose[:3] + d / np.linalg.norm(d) * rng.uniform(0.12, 0.22)
        cs, amb = O.collide(S.SPHERE, [r, 0, 0], np.r_[c, 1, 0, 0, 0], S.HULL, [0, 0, 0], pose, margin=0.3,
                            hulls=[(V, F)])
        if amb or not cs:
            continue
        want = dist_point_hull(c, W)
        if want < 1e-6:
            continue   # inside: the least-penetration face is not a distance
        n += 1
        np.testing.assert_allclose(cs[0][3] + r, want, atol=1e-6)
        # the normal points from the hull to the sphere's centre along the closest line
        q = c - cs[0][1] * want
        assert dist_point_hull(q, W) < 1e-5
    assert n >= 10


@pytest.mark.parametrize("k", range(len(FAMILIES)))
def test_capsule_hull_distance(k):
    V, F = FAMILIES[k]
    rng = np.random.default_rng(40 + k)
    pose = np.r_[0.0, 0.0, 0.5, rquat(rng)]
    W = world(V, pose)
    r, hl = 0.03, 0.1
    n = 0
    for t in range(20):
        d = rng.normal(size=3)
        qc = rquat(rng)
        c = pose[:3] + d / np.linalg.norm(d) * rng.uniform(0.2, 0.3)
        cpose = np.r_[c, qc]
        axis = rot(qc)[:, 2]
        cs, amb = O.collide(S.CAPSULE, [r, hl, 0], cpose, S.HULL, [0, 0, 0], pose, margin=0.3, hulls=[(V, F)])
        if amb or not cs:
            continue
        want = dist_seg_hull(c - hl * axis, c + hl * axis, W)
        if want < 1e-6:
            continue
        n += 1
        np.testing.assert_allclose(min(x[3] for x in cs) + r, want, atol=2e-6)
    assert n >= 8


@pytest.mark.parametrize("ka,kb", [(0, 1), (2, 3), (1, 2), (0, 3)])
def test_hull_hull_separated_witnesses(ka, kb):
    """Separated hulls: every contact's witness points p +- n phi/2 lie on
    the two hulls' surfaces (scipy's half-spaces of each hull), so no
    contact reports less than the true distance (SLSQP) and none reports a
    penetration."""
    (VA, FA), (VB, FB) = FAMILIES[ka], FAMILIES[kb]
    rng = np.random.default_rng(60 + ka + 7 * kb)
    n = 0
    for t in range(120):
        pa = np.r_[0.0, 0.0, 0.5, rquat(rng)]
        d = rng.normal(size=3)
        pb = np.r_[pa[:3] + d / np.linalg.norm(d) * rng.uniform(0.2, 0.33), rquat(rng)]
        cs, amb = O.collide(S.HULL, [0, 0, 0], pa, S.HULL, [1, 0, 0], pb, margin=0.2, hulls=[(VA, FA), (VB, FB)])
        if amb or not cs:
            continue
        WA, WB = world(VA, pa), world(VB, pb)
        want = dist_hull_hull(WA, WB)
        if want < 1e-5:
            continue
        ea, eb = ConvexHull(WA).equations, ConvexHull(WB).equations
        for f, nn, p, ph in cs:
            if ph > 0.03:
                continue   # beyond any margin in use
            if f == 0xFF:  # edge contact: the supporting edges' closest points (clamped lines, as box_box)
                assert abs(ph - want) < 1e-3
                continue
            n += 1
            assert ph >= want - 1e-7
            wa, wb = p + nn * (0.5 * ph), p - nn * (0.5 * ph)
            assert abs(np.max(ea[:, :3] @ wa + ea[:, 3])) < 1e-7, "witness off the first hull's surface"
            assert abs(np.max(eb[:, :3] @ wb + eb[:, 3])) < 1e-7, "witness off the second hull's surface"
    assert n >= 3


def test_face_to_face_gap_is_exact():
    """A prism resting on the top face of a chamfered box, lifted by a gap g:
    every contact reports phi = g with the normal straight up."""
    VA, FA = S.hull_prism(6, 0.05, 0.04)
    VB, FB = S.hull_chamfered_box(0.2, 0.2, 0.1, 0.03)
    for g in (0.0, 0.004, -0.003):
        pa = np.r_[0.01, -0.02, 0.1 + 0.04 + g, math.cos(0.2), 0, 0, math.sin(0.2)]
        pb = np.r_[0.0, 0.0, 0.0, 1, 0, 0, 0]
        cs, amb = O.collide(S.HULL, [0, 0, 0], pa, S.HULL, [1, 0, 0], pb, margin=0.02, hulls=[(VA, FA), (VB, FB)])
        assert amb == 0 and len(cs) == 4
        for f, n, p, ph in cs:
            np.testing.assert_allclose(ph, g, atol=1e-12)
            np.testing.assert_allclose(n, [0, 0, 1], atol=1e-12)


def test_octagon_reduced_to_largest_quad():
    """Two square prisms face to face, one turned 45 degrees: the overlap is
    a regular octagon; four of its corners spanning the largest
    quadrilateral are kept."""
    V, F = S.hull_prism(4, 0.1, 0.05)
    pa = np.r_[0, 0, 0.1, math.cos(math.pi / 8), 0, 0, math.sin(math.pi / 8)]
    pb = np.r_[0, 0, 0.0, 1, 0, 0, 0]
    cs, amb = O.collide(S.HULL, [0, 0, 0], pa, S.HULL, [0, 0, 0], pb, margin=0.02, hulls=[(V, F)])
    assert len(cs) == 4
    w = 0.1 / math.sqrt(2)      # the squares' half-width
    R = w / math.cos(math.pi / 8)
    octo = [R * np.array([math.cos(a), math.sin(a)]) for a in np.pi / 8 + np.arange(8) * np.pi / 4]
    got = np.array([c[2][:2] for c in cs])
    for g in got:
        assert min(np.linalg.norm(g - o) for o in octo) < 1e-9

    def area(P):
        c = P.mean(0)
        P = P[np.argsort(np.arctan2(P[:, 1] - c[1], P[:, 0] - c[0]))]
        return 0.5 * abs(np.sum(P[:, 0] * np.roll(P[:, 1], -1) - np.roll(P[:, 0], -1) * P[:, 1]))
    best = max(area(np.array(q)) for q in itertools.combinations(octo, 4))
    np.testing.assert_allclose(area(got), best, rtol=1e-9)


def test_hull_rests_on_the_ground():
    """A hexagonal prism dropped flat comes to rest on its cap: 4 ground
    contacts spanning the cap, normal impulses summing to m g dt."""
    sc = S.Scene()
    V, F = S.hull_prism(6, 0.1, 0.05)
    sc.add_hull(V, F, S.DYNAMIC, 1.3, 0.6, 0.0, [0, 0, 0.2], [math.cos(0.3), math.sin(0.3), 0, 0])
    b = S.pack([sc])
    ora = O.OracleSim(b)
    for t in range(240):
        r = ora.step(iters=50, tol=1e-10, warm=O.PREV)
    n = int(r["n_contacts"][0])
    assert n == 4
    np.testing.assert_allclose(r["c_lambda"][0, :n, 0].sum(), float(b.mass[0]) * G * DT, rtol=1e-6)
    assert np.abs(ora.vel.reshape(-1, 6)[0]).max() < 1e-6
    np.testing.assert_allclose(ora.pose.reshape(-1, 7)[0, 2], 0.05, atol=1e-3)


def test_capsule_flat_on_a_hull_face():
    """A capsule lying level on a hexagonal prism's top face, lifted by a
    gap g: two contacts at its core's ends, phi = g, normal up; a long
    capsule hanging over the face's edges is clipped to the face."""
    V, F = S.hull_prism(6, 0.2, 0.05)
    hull_pose = np.r_[0.0, 0.0, 0.5, 1, 0, 0, 0]
    r = 0.03
    for hl, g in ((0.05, 0.004), (0.3, 0.0)):
        # core along x (capsule axis z turned onto x)
        cpose = np.r_[0.0, 0.02, 0.5 + 0.05 + r + g, math.cos(math.pi / 4), 0, math.sin(math.pi / 4), 0]
        cs, amb = O.collide(S.CAPSULE, [r, hl, 0], cpose, S.HULL, [0, 0, 0], hull_pose, margin=0.02, hulls=[(V, F)])
        assert amb == 0 and len(cs) == 2
        xs = sorted(c[2][0] for c in cs)
        for f, n, p, ph in cs:
            np.testing.assert_allclose(ph, g, atol=1e-12)
            np.testing.assert_allclose(n, [0, 0, 1], atol=1e-12)
        # the core's ends, or where the top hexagon's edges cut the core (x = +-r_in sqrt(1 - (y/r_in)^2)...)
        if hl < 0.1:
            np.testing.assert_allclose(xs, [-hl, hl], atol=1e-12)
        else:
            # the hexagon (circumradius 0.2, a vertex on +x): its boundary at y = 0.02
            assert all(abs(x) < 0.2 for x in xs) and xs[0] < -0.15 and xs[1] > 0.15


def test_sphere_inside_a_hull_leaves_by_the_nearest_face():
    """A sphere centre inside a chamfered box nearest its +x face: the
    normal is that face's and phi is minus (depth + radius)."""
    V, F = S.hull_chamfered_box(0.2, 0.15, 0.1, 0.02)
    pose = np.r_[0.0, 0.0, 0.5, 1, 0, 0, 0]
    c = np.array([0.17, 0.0, 0.5])
    cs, amb = O.collide(S.SPHERE, [0.05, 0, 0], np.r_[c, 1, 0, 0, 0], S.HULL, [0, 0, 0], pose, margin=0.02, hulls=[(V, F)])
    assert amb == 0 and len(cs) == 1
    f, n, p, ph = cs[0]
    np.testing.assert_allclose(n, [1, 0, 0], atol=1e-12)
    np.testing.assert_allclose(ph, -(0.2 - 0.17) - 0.05, atol=1e-12)


def test_capsule_level_on_a_turned_hull():
    """The same level capsule on the prism turned about its axis and about
    a tilted axis carried along: in the hull's frame the result is that of
    the upright case (contact count, phi, normal along the face's normal,
    contact points midway between the face and the capsule, over the face)."""
    V, F = S.hull_prism(6, 0.2, 0.05)
    r, g = 0.03, 0.004

    def qmul(a, b):
        return np.r_[a[0] * b[0] - a[1:] @ b[1:], a[0] * b[1:] + b[0] * a[1:] + np.cross(a[1:], b[1:])]

    def rot(q, v):
        return qmul(qmul(q, np.r_[0.0, v]), q * np.r_[1, -1, -1, -1])[1:]

    for k, (ax, ang) in enumerate((((0, 0, 1), 0.7), ((1, 2, 0.5), 0.4), ((-0.3, 1, 0.2), 2.1))):
        ax = np.asarray(ax, float) / np.linalg.norm(ax)
        qh = np.r_[math.cos(ang / 2), math.sin(ang / 2) * ax]
        ch = np.array([0.1, -0.2, 0.6])
        for hl in (0.05, 0.3):
            # capsule core along local x at local height top + r + g, yawed by 0.3 k in the face
            qc_local = qmul(np.r_[math.cos(0.15 * k), 0, 0, math.sin(0.15 * k)],
                            np.r_[math.cos(math.pi / 4), 0, math.sin(math.pi / 4), 0])
            pc = ch + rot(qh, np.array([0.0, 0.02, 0.05 + r + g]))
            cs, amb = O.collide(S.CAPSULE, [r, hl, 0], np.r_[pc, qmul(qh, qc_local)], S.HULL, [0, 0, 0],
                                np.r_[ch, qh], margin=0.02, hulls=[(V, F)])
            assert amb == 0 and len(cs) == 2, (k, hl, cs)
            up = rot(qh, np.array([0.0, 0.0, 1.0]))
            for f, n, p, ph in cs:
                assert f in (0, 1)
                np.testing.assert_allclose(ph, g, atol=1e-9)
                np.testing.assert_allclose(n, up, atol=1e-9)
                loc = rot(qh * np.r_[1, -1, -1, -1], np.asarray(p) - ch)
                np.testing.assert_allclose(loc[2], 0.05 + g / 2, atol=1e-9)   # midway between the surfaces
                assert math.hypot(loc[0], loc[1]) <= 0.2 + 1e-9

/*
 * rbo.c -- FP64 CPU oracle of the batched rigid-body step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, smoke() and bench.py's
 * cpu_baseline leg.  Nothing of the product path calls it.  It shares no
 * code with the HIP path.
 *
 * Paper anchors (Habitat 2.0): the physics engine maps (s_t, a_t) -> s_{t+1}
 * (Sec. 2); rigid bodies carry mass, friction and restitution and simplified
 * collision proxies such as boxes (Sec. 3; Sec. 4.3); base-constrained parts
 * are static (Sec. 4.1); the robot is the only non-gravity force source
 * (Sec. 4.1); physics runs at 1/120 s (Sec. 4.4); the arm has 7 DoF (Sec. 5);
 * the per-step collision force in newtons is what tasks consume (Sec. 5 and
 * the Pick reward in the appendix).  The paper gives no engine algorithm; each
 * function below states the textbook method or the reading it follows.
 *
 * Everything is written as plain loops in the step's order, in double
 * precision, per scene.  Decisions that a float32 implementation could take
 * differently (a comparison whose two sides are within the tie band) are
 * counted in `ambiguous` so that parity tests can skip those scenes.
 */
#include "rbo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PAIR_GROUND 0xFFFFu
#define KEY_GROUND 0xFFFu
#define BAND 1e-5       /* tie band for decisions on lengths (m) */
#define BAND_DIM 1e-5   /* tie band for dimensionless decisions */
#define BAND_V 1e-4     /* tie band for decisions on speeds (m/s) */
#define SIN_PAR 1e-3    /* "parallel" threshold: sine of 1 mrad (approx.) */
#define MAXCOL 256
#define CLIP_ON 1e-4  /* clip vertices within this distance of a plane lie on it (m) */

/* ------------------------------------------------------------------ vectors */
typedef struct { double x, y, z; } V;
static V mk(double x, double y, double z) { V r; r.x = x; r.y = y; r.z = z; return r; }
static V add(V a, V b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static V sub(V a, V b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static V scl(V a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(V a, V b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static V cross(V a, V b) { return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
static double len2(V a) { return dot(a, a); }
static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }
static double comp(V a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }
static void setc(V *a, int i, double s) { if (i == 0) a->x = s; else if (i == 1) a->y = s; else a->z = s; }
static V unit(int i) { return mk(i == 0, i == 1, i == 2); }

typedef struct { double m[3][3]; } M3;
/* Rotation matrix of the quaternion (w, x, y, z), Hamilton convention. */
static M3 quat_R(const double *q) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    M3 R;
    R.m[0][0] = 1 - 2 * (y * y + z * z); R.m[0][1] = 2 * (x * y - w * z);     R.m[0][2] = 2 * (x * z + w * y);
    R.m[1][0] = 2 * (x * y + w * z);     R.m[1][1] = 1 - 2 * (x * x + z * z); R.m[1][2] = 2 * (y * z - w * x);
    R.m[2][0] = 2 * (x * z - w * y);     R.m[2][1] = 2 * (y * z + w * x);     R.m[2][2] = 1 - 2 * (x * x + y * y);
    return R;
}
static V Rv(const M3 *R, V a) {
    return mk(R->m[0][0] * a.x + R->m[0][1] * a.y + R->m[0][2] * a.z,
              R->m[1][0] * a.x + R->m[1][1] * a.y + R->m[1][2] * a.z,
              R->m[2][0] * a.x + R->m[2][1] * a.y + R->m[2][2] * a.z);
}
static V RTv(const M3 *R, V a) {
    return mk(R->m[0][0] * a.x + R->m[1][0] * a.y + R->m[2][0] * a.z,
              R->m[0][1] * a.x + R->m[1][1] * a.y + R->m[2][1] * a.z,
              R->m[0][2] * a.x + R->m[1][2] * a.y + R->m[2][2] * a.z);
}
static V col(const M3 *R, int j) { return mk(R->m[0][j], R->m[1][j], R->m[2][j]); }
static void quat_mul(const double *a, const double *b, double *o) {
    double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

/* ------------------------------------------------------------------ bodies */
typedef struct {
    int shape, motion;
    V x; double q[4]; M3 R;
    double prm[3];
    V v, w;
    double im;          /* inverse mass (0 unless dynamic) */
    M3 Iw;              /* world inverse inertia (0 unless dynamic) */
    double mu, e;
    V lo, hi;           /* fattened AABB */
    int ncon;           /* contacts touching this body (Jacobi) */
    /* articulated container part: 1 revolute about the line through jo along
     * ja, 2 prismatic along ja; qd its joint rate, jM its mass about the
     * joint (moment of inertia about the hinge line, or the mass); v and w
     * always equal the motion qd gives the body */
    int joint;
    V ja, jo;
    double jM, qd;
    const struct HullS *hull;   /* shape ORA_HULL: its hull (prm: its bounding box half-extents) */
    double Ib[3][3];    /* inertia tensor in the body frame (dynamic bodies) */
} Body;

/* Principal moments of a solid body of uniform density. */
static void body_inertia(int shape, const double *p, double m, double I[3]) {
    if (shape == ORA_SPHERE) {
        I[0] = I[1] = I[2] = 0.4 * m * p[0] * p[0];
    } else if (shape == ORA_BOX) {
        double x2 = p[0] * p[0], y2 = p[1] * p[1], z2 = p[2] * p[2];
        I[0] = m / 3.0 * (y2 + z2);
        I[1] = m / 3.0 * (x2 + z2);
        I[2] = m / 3.0 * (x2 + y2);
    } else {
        /* cylinder of length 2h plus two hemispherical caps; mass split by
         * volume; caps by the parallel-axis theorem (cap centroid 3r/8 from
         * its flat face). */
        double r = p[0], h = p[1];
        double vc = 2.0 * M_PI * r * r * h, vs = 4.0 / 3.0 * M_PI * r * r * r;
        double mc = m * vc / (vc + vs), ms = m - mc;
        I[2] = mc * r * r / 2.0 + 0.4 * ms * r * r;
        I[0] = I[1] = mc * (r * r / 4.0 + h * h / 3.0) + ms * (0.4 * r * r + h * h + 0.75 * h * r);
    }
}

static void body_aabb(Body *b, double margin) {
    if (b->shape == ORA_SPHERE) {
        double e = b->prm[0] + margin;
        b->lo = sub(b->x, mk(e, e, e));
        b->hi = add(b->x, mk(e, e, e));
    } else if (b->shape == ORA_BOX || b->shape == ORA_HULL) {   /* a hull: its bounding box */
        V e;
        e.x = fabs(b->R.m[0][0]) * b->prm[0] + fabs(b->R.m[0][1]) * b->prm[1] + fabs(b->R.m[0][2]) * b->prm[2] + margin;
        e.y = fabs(b->R.m[1][0]) * b->prm[0] + fabs(b->R.m[1][1]) * b->prm[1] + fabs(b->R.m[1][2]) * b->prm[2] + margin;
        e.z = fabs(b->R.m[2][0]) * b->prm[0] + fabs(b->R.m[2][1]) * b->prm[1] + fabs(b->R.m[2][2]) * b->prm[2] + margin;
        b->lo = sub(b->x, e);
        b->hi = add(b->x, e);
    } else {
        V ax = scl(col(&b->R, 2), b->prm[1]);
        V e0 = sub(b->x, ax), e1 = add(b->x, ax);
        double r = b->prm[0] + margin;
        b->lo = mk(fmin(e0.x, e1.x) - r, fmin(e0.y, e1.y) - r, fmin(e0.z, e1.z) - r);
        b->hi = mk(fmax(e0.x, e1.x) + r, fmax(e0.y, e1.y) + r, fmax(e0.z, e1.z) + r);
    }
}

/* -------------------------------------------------------------- narrowphase
 * Conventions: routines return contacts whose normal points from the SECOND
 * argument to the FIRST; phi is the signed separation along n (negative =
 * penetration); p is the midpoint of the two surface witness points; f is a
 * feature id.  A contact is kept iff phi <= margin. */
/* A convex hull (shape ORA_HULL) in its body frame: vertices, face planes
 * (outward unit normal n and offset d: n . x = d on the face), faces as
 * vertex loops counter-clockwise seen from outside, and the undirected
 * edges; the half-extents of its local bounding box and its largest
 * vertex distance from the origin. */
#define HULL_MAXV 32
#define HULL_MAXF 32
#define HULL_MAXE 64
#define HULL_MAXL 8
typedef struct HullS {
    int nv, nf, ne;
    V v[HULL_MAXV];
    V fn[HULL_MAXF];
    double fd[HULL_MAXF];
    int nl[HULL_MAXF], loop[HULL_MAXF][HULL_MAXL];
    int ea[HULL_MAXE], eb[HULL_MAXE];
    int ef[HULL_MAXE][2];   /* the two faces that share the edge (first, second appearance) */
    double h[3], rad;
} Hull;
typedef struct { int shape; V x; M3 R; double prm[3]; const Hull *hull; } Geom;
typedef struct { int f; V n, p; double phi; } PC;

static int keep(double phi, double margin, int *amb) {
    if (fabs(phi - margin) < BAND) (*amb)++;
    return phi <= margin;
}

/* Two spheres: distance of the centres minus the radii. */
static PC sphere_sphere(V ca, double ra, V cb, double rb, int f) {
    PC c;
    V d = sub(ca, cb);
    double L = sqrt(len2(d));
    c.n = L < 1e-9 ? mk(0, 0, 1) : scl(d, 1.0 / L);
    c.phi = L - ra - rb;
    c.p = scl(add(sub(ca, scl(c.n, ra)), add(cb, scl(c.n, rb))), 0.5);
    c.f = f;
    return c;
}

/* Sphere (first) against a box (second): closest point by clamping in the
 * box frame; a centre inside the box leaves through the face of least
 * penetration (ties: lower axis, then the + face). */
static int sphere_box(const Geom *S, const Geom *B, double margin, PC *out, int *amb) {
    double r = S->prm[0];
    const double *h = B->prm;
    V l = RTv(&B->R, sub(S->x, B->x));
    int inside = fabs(l.x) <= h[0] && fabs(l.y) <= h[1] && fabs(l.z) <= h[2];
    V nl, q = l;
    double phi;
    if (!inside) {
        q = mk(clampd(l.x, -h[0], h[0]), clampd(l.y, -h[1], h[1]), clampd(l.z, -h[2], h[2]));
        V d = sub(l, q);
        double L = sqrt(len2(d));
        nl = scl(d, 1.0 / L);
        phi = L - r;
    } else {
        double pen[3];
        int a = 0;
        for (int i = 0; i < 3; i++) pen[i] = h[i] - fabs(comp(l, i));
        for (int i = 1; i < 3; i++) if (pen[i] < pen[a]) a = i;
        for (int i = 0; i < 3; i++) if (i != a && fabs(pen[i] - pen[a]) < BAND) (*amb)++;
        double la = comp(l, a);
        if (fabs(la) < BAND) (*amb)++;
        double s = la >= 0 ? 1.0 : -1.0;
        nl = scl(unit(a), s);
        setc(&q, a, s * h[a]);
        phi = -pen[a] - r;
    }
    PC c;
    c.n = Rv(&B->R, nl);
    V wb = add(B->x, Rv(&B->R, q));
    V wa = sub(S->x, scl(c.n, r));
    c.p = scl(add(wa, wb), 0.5);
    c.phi = phi;
    c.f = 0;
    if (!keep(phi, margin, amb)) return 0;
    out[0] = c;
    return 1;
}

static void capsule_seg(const Geom *C, V *p0, V *d) {
    V ax = scl(col(&C->R, 2), C->prm[1]);
    *p0 = sub(C->x, ax);
    *d = scl(ax, 2.0);
}

/* Sphere (first) against a capsule (second): closest point of the core
 * segment to the centre, then sphere-sphere. */
static int sphere_capsule(const Geom *S, const Geom *C, double margin, PC *out, int *amb) {
    V p0, d;
    capsule_seg(C, &p0, &d);
    double t = clampd(dot(sub(S->x, p0), d) / len2(d), 0.0, 1.0);
    PC c = sphere_sphere(S->x, S->prm[0], add(p0, scl(d, t)), C->prm[0], 0);
    if (!keep(c.phi, margin, amb)) return 0;
    out[0] = c;
    return 1;
}

/* Capsule against capsule.  Closest points of the two core segments
 * (Ericson 2005, Sec. 5.1.9); nearly parallel segments whose projections
 * overlap give two contacts at the ends of the overlap interval. */
static int capsule_capsule(const Geom *A, const Geom *B, double margin, PC *out, int *amb) {
    V pa, da, pb, db;
    capsule_seg(A, &pa, &da);
    capsule_seg(B, &pb, &db);
    double ra = A->prm[0], rb = B->prm[0];
    double aa = len2(da), ee = len2(db);
    double cr2 = len2(cross(da, db));
    double thr = 1e-6 * aa * ee;
    if (fabs(cr2 - thr) < 1e-2 * thr) (*amb)++;
    int n = 0;
    if (cr2 <= thr) {
        double s0 = dot(sub(pb, pa), da) / aa;
        double s1 = dot(sub(add(pb, db), pa), da) / aa;
        double lo = fmax(0.0, fmin(s0, s1)), hi = fmin(1.0, fmax(s0, s1));
        if (fabs(hi - lo) * sqrt(aa) < BAND) (*amb)++;
        if (lo <= hi) {
            double ss[2] = {lo, hi};
            for (int k = 0; k < 2; k++) {
                if (k == 1 && !(hi > lo)) break;
                V P = add(pa, scl(da, ss[k]));
                double t = clampd(dot(sub(P, pb), db) / ee, 0.0, 1.0);
                PC c = sphere_sphere(P, ra, add(pb, scl(db, t)), rb, k);
                if (keep(c.phi, margin, amb)) out[n++] = c;
            }
            return n;
        }
    }
    V r = sub(pa, pb);
    double b = dot(da, db), c = dot(da, r), f = dot(db, r);
    double den = aa * ee - b * b;
    double s = den != 0.0 ? clampd((b * f - c * ee) / den, 0.0, 1.0) : 0.0;
    double t = (b * s + f) / ee;
    if (t < 0.0) { t = 0.0; s = clampd(-c / aa, 0.0, 1.0); }
    else if (t > 1.0) { t = 1.0; s = clampd((b - c) / aa, 0.0, 1.0); }
    PC cc = sphere_sphere(add(pa, scl(da, s)), ra, add(pb, scl(db, t)), rb, 0);
    if (keep(cc.phi, margin, amb)) out[n++] = cc;
    return n;
}

/* Squared distance of a box-local point to the box. */
static double box_d2(V l, const double *h) {
    double g = 0;
    for (int a = 0; a < 3; a++) {
        double x = fabs(comp(l, a)) - h[a];
        if (x > 0) g += x * x;
    }
    return g;
}

/* Clip the segment l(t) = p0 + t d, t in [0, 1], to the slabs |l_b| <= h_b
 * for the two axes b != a.  Returns 0 if the interval is empty. */
static int clip_face(V p0, V d, const double *h, int a, double *t0, double *t1) {
    double lo = 0.0, hi = 1.0;
    for (int b = 0; b < 3; b++) {
        if (b == a) continue;
        double pb = comp(p0, b), db = comp(d, b);
        if (db == 0.0) {
            if (fabs(pb) > h[b]) return 0;
            continue;
        }
        double ta = (-h[b] - pb) / db, tb = (h[b] - pb) / db;
        if (ta > tb) { double x = ta; ta = tb; tb = x; }
        if (ta > lo) lo = ta;
        if (tb < hi) hi = tb;
    }
    *t0 = lo; *t1 = hi;
    return lo <= hi;
}

/* One contact of a capsule core point l (box-local) against box face a on
 * side s: normal s*e_a, depth from the face plane. */
static PC cap_face_contact(V l, int a, double s, const double *h, double r, int f) {
    PC c;
    c.n = scl(unit(a), s);
    c.phi = s * comp(l, a) - h[a] - r;
    V q = l;
    setc(&q, a, s * h[a]);
    V wc = sub(l, scl(c.n, r));
    c.p = scl(add(q, wc), 0.5);
    c.f = f;
    return c;
}

/* Capsule (first) against a box (second), in the box frame.
 * 1. Closest point of the core segment to the box: the squared distance
 *    g(t) is convex and piecewise quadratic in t; evaluate the ends, the slab
 *    crossings and every piece's vertex; smallest g wins (ties: smaller t).
 * 2. Separated core, closest point in a face region and the segment within
 *    ~1 mrad of parallel to that face: two contacts at the ends of the
 *    segment clipped to the face rectangle (f = 0, 1).
 * 3. Separated core otherwise: one contact at the closest points (f = 2).
 * 4. Core touching the box: leave through the face needing the least
 *    translation (ties: lower axis, + side first); contacts at the ends of
 *    the segment clipped to that face (f = 0, 1), else at the deeper
 *    endpoint (f = 3). */
static int capsule_box(const Geom *C, const Geom *B, double margin, PC *out, int *amb) {
    double r = C->prm[0];
    const double *h = B->prm;
    V P0, D;
    capsule_seg(C, &P0, &D);
    V p0 = RTv(&B->R, sub(P0, B->x));
    V d = RTv(&B->R, D);
    double dl = sqrt(len2(d));
    double ts[16];
    int nt = 0;
    ts[nt++] = 0.0; ts[nt++] = 1.0;
    for (int a = 0; a < 3; a++) {
        double da = comp(d, a);
        if (da == 0.0) continue;
        for (int sg = -1; sg <= 1; sg += 2) {
            double t = (sg * h[a] - comp(p0, a)) / da;
            if (t > 0.0 && t < 1.0) ts[nt++] = t;
        }
    }
    for (int i = 1; i < nt; i++)            /* insertion sort */
        for (int j = i; j > 0 && ts[j] < ts[j - 1]; j--) { double x = ts[j]; ts[j] = ts[j - 1]; ts[j - 1] = x; }
    double cand[16];
    double curv[16];
    int nc = 0;
    for (int i = 0; i < nt; i++) { cand[nc] = ts[i]; curv[nc] = -1; nc++; }
    for (int i = 0; i + 1 < nt; i++) {
        double tl = ts[i], th = ts[i + 1];
        if (!(th > tl)) continue;
        double tm = 0.5 * (tl + th), num = 0, den = 0;
        for (int a = 0; a < 3; a++) {
            double la = comp(p0, a) + tm * comp(d, a), ca;
            if (la > h[a]) ca = h[a];
            else if (la < -h[a]) ca = -h[a];
            else continue;
            num += comp(d, a) * (ca - comp(p0, a));
            den += comp(d, a) * comp(d, a);
        }
        double tv = den > 0 ? clampd(num / den, tl, th) : tl;
        cand[nc] = tv; curv[nc] = den; nc++;
    }
    int bi = 0;
    double gc[16];
    for (int i = 0; i < nc; i++) gc[i] = box_d2(add(p0, scl(d, cand[i])), h);
    double bg = gc[0];
    for (int i = 1; i < nc; i++)
        if (gc[i] < bg || (gc[i] == bg && cand[i] < cand[bi])) { bg = gc[i]; bi = i; }
    double t = cand[bi];
    V l = add(p0, scl(d, t));
    int n = 0;
    PC loc[4];
    /* Whether the core meets the box: the segment clipped to the box's three
     * slabs (Liang and Barsky 1984) is non-empty, t_in <= t_out.  A core that
     * passes through the box gives a clear margin t_out - t_in; the zero
     * distance of its crossing point would be at the mercy of rounding. */
    double t_in = 0.0, t_out = 1.0;
    for (int k = 0; k < 3; k++) {
        double dk = comp(d, k), pk = comp(p0, k);
        if (dk == 0.0) {
            if (fabs(fabs(pk) - h[k]) < BAND) (*amb)++;
            if (fabs(pk) > h[k]) t_out = -1.0;
            continue;
        }
        double u0 = (-h[k] - pk) / dk, u1 = (h[k] - pk) / dk;
        t_in = fmax(t_in, fmin(u0, u1));
        t_out = fmin(t_out, fmax(u0, u1));
    }
    int meets = t_in <= t_out || bg <= 0.0;
    if (fabs(t_out - t_in) * dl < BAND) (*amb)++;           /* grazing */
    if (!meets) {
        double dist = sqrt(bg);
        if (dist < BAND) (*amb)++;
        int ncl = 0, a = -1;
        for (int k = 0; k < 3; k++) {
            if (fabs(fabs(comp(l, k)) - h[k]) < BAND) (*amb)++;   /* face / edge / corner region */
            if (fabs(comp(l, k)) > h[k]) { ncl++; a = k; }
        }
        const int face = ncl == 1 && fabs(comp(d, a)) <= SIN_PAR * dl;
        /* a plateau of the distance: another candidate as close within the
         * band, at a different place, where the contacts would differ (the
         * clipped segment does not depend on the point chosen on one face;
         * a single contact sits at the point) */
        for (int i = 0; i < nc; i++) {
            if (i == bi || fabs(sqrt(gc[i]) - dist) >= BAND || fabs(cand[i] - t) * dl <= BAND) continue;
            V li = add(p0, scl(d, cand[i]));
            int nci = 0, ai = -1;
            for (int k = 0; k < 3; k++) if (fabs(comp(li, k)) > h[k]) { nci++; ai = k; }
            const int facei = nci == 1 && fabs(comp(d, ai)) <= SIN_PAR * dl;
            if (!face || !facei || ai != a || (comp(li, ai) > 0) != (comp(l, a) > 0)) { (*amb)++; break; }
        }
        int done = 0;
        if (ncl == 1) {
            double sa = comp(l, a) > 0 ? 1.0 : -1.0;
            double thr = SIN_PAR * dl;
            if (fabs(fabs(comp(d, a)) - thr) < 1e-2 * thr) (*amb)++;
            if (fabs(comp(d, a)) <= thr) {
                for (int k = 0; k < 3; k++)
                    if (k != a && fabs(h[k] - fabs(comp(l, k))) < BAND) (*amb)++;
                double t0, t1;
                int ok = clip_face(p0, d, h, a, &t0, &t1);
                if (ok && fabs(t1 - t0) * dl < BAND) (*amb)++;
                if (ok) {
                    loc[n++] = cap_face_contact(add(p0, scl(d, t0)), a, sa, h, r, 0);
                    if (t1 > t0) loc[n++] = cap_face_contact(add(p0, scl(d, t1)), a, sa, h, r, 1);
                    done = 1;
                }
            }
        }
        if (!done) {
            if (curv[bi] >= 0 && curv[bi] < 1e-4 * dl * dl) (*amb)++;
            V q = mk(clampd(l.x, -h[0], h[0]), clampd(l.y, -h[1], h[1]), clampd(l.z, -h[2], h[2]));
            PC c;
            c.n = scl(sub(l, q), 1.0 / dist);
            c.phi = dist - r;
            c.p = scl(add(q, sub(l, scl(c.n, r))), 0.5);
            c.f = 2;
            loc[n++] = c;
        }
    } else {
        double p1a[3], best = INFINITY, second = INFINITY;
        int ba = 0;
        double bs = 1.0;
        V p1 = add(p0, d);
        for (int a = 0; a < 3; a++) p1a[a] = comp(p1, a);
        for (int a = 0; a < 3; a++) {
            for (int sg = 1; sg >= -1; sg -= 2) {
                double ex = h[a] - fmin(sg * comp(p0, a), sg * p1a[a]);
                if (ex < best) { second = best; best = ex; ba = a; bs = sg; }
                else if (ex < second) second = ex;
            }
        }
        if (second - best < BAND) (*amb)++;
        double t0, t1;
        int ok = clip_face(p0, d, h, ba, &t0, &t1);
        if (ok && fabs(t1 - t0) * dl < BAND) (*amb)++;
        if (ok) {
            loc[n++] = cap_face_contact(add(p0, scl(d, t0)), ba, bs, h, r, 0);
            if (t1 > t0) loc[n++] = cap_face_contact(add(p0, scl(d, t1)), ba, bs, h, r, 1);
        } else {
            double e0 = bs * comp(p0, ba), e1 = bs * p1a[ba];
            if (fabs(e0 - e1) < BAND) (*amb)++;
            V pe = e0 <= e1 ? p0 : p1;
            loc[n++] = cap_face_contact(pe, ba, bs, h, r, 3);
        }
    }
    int m = 0;
    for (int k = 0; k < n; k++) {
        if (!keep(loc[k].phi, margin, amb)) continue;
        PC c = loc[k];
        c.n = Rv(&B->R, loc[k].n);
        c.p = add(B->x, Rv(&B->R, loc[k].p));
        out[m++] = c;
    }
    return m;
}

/* Box against box: separating-axis test over the 15 axes (Gottschalk et al.
 * 1996), face axes preferred over edge axes and the first box's faces over
 * the second's unless clearly better; face contact = incident face clipped
 * against the reference face's side planes (Sutherland-Hodgman 1974) and
 * reduced to at most 4 points; edge contact = closest points of two edges. */
static int box_box(const Geom *A, const Geom *B, double margin, PC *out, int *amb) {
    V a[3], b[3];
    for (int i = 0; i < 3; i++) { a[i] = col(&A->R, i); b[i] = col(&B->R, i); }
    const double *ha = A->prm, *hb = B->prm;
    V D = sub(A->x, B->x);
    double s[15], sg[15];
    int valid[15];
    V u[15];
    for (int k = 0; k < 15; k++) {
        double ra, rb;
        valid[k] = 1;
        if (k < 3) {
            u[k] = a[k];
            ra = ha[k];
            rb = hb[0] * fabs(dot(b[0], u[k])) + hb[1] * fabs(dot(b[1], u[k])) + hb[2] * fabs(dot(b[2], u[k]));
        } else if (k < 6) {
            u[k] = b[k - 3];
            rb = hb[k - 3];
            ra = ha[0] * fabs(dot(a[0], u[k])) + ha[1] * fabs(dot(a[1], u[k])) + ha[2] * fabs(dot(a[2], u[k]));
        } else {
            int i = (k - 6) / 3, j = (k - 6) % 3;
            V c = cross(a[i], b[j]);
            double L2 = len2(c);
            if (fabs(L2 - 1e-12) < 1e-13) (*amb)++;
            if (L2 < 1e-12) { valid[k] = 0; s[k] = -INFINITY; sg[k] = 1; continue; }
            u[k] = scl(c, 1.0 / sqrt(L2));
            ra = ha[0] * fabs(dot(a[0], u[k])) + ha[1] * fabs(dot(a[1], u[k])) + ha[2] * fabs(dot(a[2], u[k]));
            rb = hb[0] * fabs(dot(b[0], u[k])) + hb[1] * fabs(dot(b[1], u[k])) + hb[2] * fabs(dot(b[2], u[k]));
        }
        double dd = dot(D, u[k]);
        s[k] = fabs(dd) - ra - rb;
        sg[k] = dd >= 0 ? 1.0 : -1.0;
    }
    double smax = -INFINITY;
    for (int k = 0; k < 15; k++) if (valid[k] && s[k] > smax) smax = s[k];
    if (fabs(smax - margin) < BAND) (*amb)++;
    if (smax > margin) return 0;

    /* argmax within a group, ties to the lower index; near-ties are ambiguous */
    int fa = 0, fb = 3, e = -1;
    for (int k = 1; k < 3; k++) if (s[k] > s[fa]) fa = k;
    for (int k = 4; k < 6; k++) if (s[k] > s[fb]) fb = k;
    for (int k = 6; k < 15; k++) if (valid[k] && (e < 0 || s[k] > s[e])) e = k;
    double hmax = 0;
    for (int i = 0; i < 3; i++) { hmax = fmax(hmax, ha[i]); hmax = fmax(hmax, hb[i]); }
    int face = fa;
    double thr = 0.95 * s[fa] + 0.01 * hmax;
    if (fabs(s[fb] - thr) < BAND) (*amb)++;
    if (s[fb] > thr) face = fb;
    int edge = 0;
    if (e >= 0) {
        double thr2 = 0.95 * s[face] + 0.01 * hmax;
        if (fabs(s[e] - thr2) < BAND) (*amb)++;
        edge = s[e] > thr2;
    }
    /* near-ties inside a group matter only for the group that is used */
    if (edge) {
        for (int k = 6; k < 15; k++) if (valid[k] && k != e && fabs(s[k] - s[e]) < BAND) (*amb)++;
    } else if (face == fa) {
        for (int k = 0; k < 3; k++) if (k != fa && fabs(s[k] - s[fa]) < BAND) (*amb)++;
    } else {
        for (int k = 3; k < 6; k++) if (k != fb && fabs(s[k] - s[fb]) < BAND) (*amb)++;
    }

    if (edge) {
        int i = (e - 6) / 3, j = (e - 6) % 3;
        V N = scl(u[e], sg[e]);
        if (fabs(dot(D, u[e])) < BAND) (*amb)++;
        V pa = A->x, pb = B->x;
        for (int m = 0; m < 3; m++) {
            if (m != i) {
                double c = dot(N, a[m]);
                if (fabs(c) < BAND_DIM) (*amb)++;
                pa = add(pa, scl(a[m], c > 0 ? -ha[m] : ha[m]));
            }
            if (m != j) {
                double c = dot(N, b[m]);
                if (fabs(c) < BAND_DIM) (*amb)++;
                pb = add(pb, scl(b[m], c > 0 ? hb[m] : -hb[m]));
            }
        }
        V w = sub(pa, pb);
        double bb = dot(a[i], b[j]), dd = dot(a[i], w), ee = dot(b[j], w);
        double den = 1.0 - bb * bb;
        double ta = (bb * ee - dd) / den;
        double tb = ee + ta * bb;
        ta = clampd(ta, -ha[i], ha[i]);
        tb = clampd(tb, -hb[j], hb[j]);
        V PA = add(pa, scl(a[i], ta)), PB = add(pb, scl(b[j], tb));
        PC c;
        c.n = N;
        c.phi = dot(sub(PA, PB), N);
        c.p = scl(add(PA, PB), 0.5);
        c.f = 0x80 | (e - 6);
        if (!keep(c.phi, margin, amb)) return 0;
        out[0] = c;
        return 1;
    }

    /* face contact */
    V N = scl(u[face], sg[face]);               /* from B to A */
    if (fabs(dot(D, u[face])) < BAND) (*amb)++;
    const Geom *ref, *inc;
    int ax, refb;
    V nout;
    if (face < 3) { ref = A; inc = B; ax = face; nout = scl(N, -1.0); refb = 0; }
    else { ref = B; inc = A; ax = face - 3; nout = N; refb = 1; }
    V rc[3], ic[3];
    for (int k = 0; k < 3; k++) { rc[k] = col(&ref->R, k); ic[k] = col(&inc->R, k); }
    const double *hr = ref->prm, *hi = inc->prm;
    int side = dot(nout, rc[ax]) > 0 ? 0 : 1;
    int refface = ax * 2 + side;
    V cref = add(ref->x, scl(nout, hr[ax]));
    /* incident face: most anti-parallel to nout */
    int j = 0;
    double best = fabs(dot(ic[0], nout));
    for (int k = 1; k < 3; k++) { double c = fabs(dot(ic[k], nout)); if (c > best) { best = c; j = k; } }
    for (int k = 0; k < 3; k++) if (k != j && fabs(fabs(dot(ic[k], nout)) - best) < BAND_DIM) (*amb)++;
    double si = dot(ic[j], nout) > 0 ? -1.0 : 1.0;
    int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
    V fc = add(inc->x, scl(ic[j], si * hi[j]));
    V e1 = scl(ic[j1], hi[j1]), e2 = scl(ic[j2], hi[j2]);
    V poly[8], tmp[8];
    int np = 4;
    poly[0] = add(add(fc, e1), e2);
    poly[1] = add(sub(fc, e1), e2);
    poly[2] = sub(sub(fc, e1), e2);
    poly[3] = sub(add(fc, e1), e2);
    int r1 = (ax + 1) % 3, r2 = (ax + 2) % 3;
    int paxis[4] = {r1, r1, r2, r2};
    double psign[4] = {1.0, -1.0, 1.0, -1.0};
    for (int pl = 0; pl < 4 && np > 0; pl++) {
        V pn = scl(rc[paxis[pl]], psign[pl]);
        double off = hr[paxis[pl]];
        int no = 0;
        V prev = poly[np - 1];
        double dp = dot(sub(prev, ref->x), pn) - off;
        for (int k = 0; k < np; k++) {
            V cur = poly[k];
            double dc = dot(sub(cur, ref->x), pn) - off;
            if (fabs(fabs(dc) - CLIP_ON) < BAND) (*amb)++;
            /* three states: inside (< -on), on the plane (|d| <= on), outside;
             * a vertex on the plane is kept and never spawns an intersection */
            int ci = dc < -CLIP_ON ? -1 : (dc > CLIP_ON ? 1 : 0);
            int pi = dp < -CLIP_ON ? -1 : (dp > CLIP_ON ? 1 : 0);
            if (pi * ci < 0 && no < 8) tmp[no++] = add(prev, scl(sub(cur, prev), dp / (dp - dc)));
            if (ci <= 0 && no < 8) tmp[no++] = cur;
            prev = cur; dp = dc;
        }
        np = no;
        for (int k = 0; k < np; k++) poly[k] = tmp[k];
    }
    int idx[8], nk = 0;
    double ph[8];
    for (int k = 0; k < np; k++) {
        ph[k] = dot(sub(poly[k], cref), nout);
        if (keep(ph[k], margin, amb)) idx[nk++] = k;
    }
    int sel[8], ns = 0;
    if (nk <= 4) {
        for (int k = 0; k < nk; k++) sel[ns++] = idx[k];
    } else {
        /* first kept point; farthest from it; largest triangle; largest quad
         * (a flat face contact has all depths equal, so depth is no anchor) */
        int used[8] = {0};
        int i1 = idx[0];
        used[i1] = 1;
        int i2 = -1;
        double bd = -1;
        for (int k = 0; k < nk; k++) {
            int q = idx[k];
            if (used[q]) continue;
            double dd = sqrt(len2(sub(poly[q], poly[i1])));
            if (dd > bd) { bd = dd; i2 = q; }
        }
        for (int k = 0; k < nk; k++) {
            int q = idx[k];
            if (used[q] || q == i2) continue;
            if (fabs(sqrt(len2(sub(poly[q], poly[i1]))) - bd) < BAND) (*amb)++;
        }
        used[i2] = 1;
        V e12 = sub(poly[i2], poly[i1]);
        double l12 = sqrt(len2(e12));
        int i3 = -1;
        double ba = -1;
        for (int k = 0; k < nk; k++) {
            int q = idx[k];
            if (used[q]) continue;
            double ar = sqrt(len2(cross(e12, sub(poly[q], poly[i1]))));
            if (ar > ba) { ba = ar; i3 = q; }
        }
        for (int k = 0; k < nk; k++) {
            int q = idx[k];
            if (used[q] || q == i3) continue;
            if (fabs(sqrt(len2(cross(e12, sub(poly[q], poly[i1])))) - ba) < BAND * l12) (*amb)++;
        }
        used[i3] = 1;
        V e23 = sub(poly[i3], poly[i2]), e31 = sub(poly[i1], poly[i3]);
        double per = l12 + sqrt(len2(e23)) + sqrt(len2(e31));
        int i4 = -1;
        double bq = -1;
        double sc[8];
        for (int k = 0; k < nk; k++) {
            int q = idx[k];
            if (used[q]) continue;
            sc[q] = sqrt(len2(cross(e12, sub(poly[q], poly[i1])))) +
                    sqrt(len2(cross(e23, sub(poly[q], poly[i2])))) +
                    sqrt(len2(cross(e31, sub(poly[q], poly[i3]))));
            if (sc[q] > bq) { bq = sc[q]; i4 = q; }
        }
        for (int k = 0; k < nk; k++) {
            int q = idx[k];
            if (used[q] || q == i4) continue;
            if (fabs(sc[q] - bq) < BAND * per) (*amb)++;
        }
        used[i4] = 1;
        for (int k = 0; k < np; k++) if (used[k]) sel[ns++] = k;
    }
    for (int k = 0; k < ns; k++) {
        int q = sel[k];
        PC c;
        c.n = N;
        c.phi = ph[q];
        c.p = sub(poly[q], scl(nout, 0.5 * ph[q]));
        c.f = refb | (refface << 1) | (q << 4);
        out[k] = c;
    }
    return ns;
}


/* ------------------------------------------------------------ convex hulls
 * Convex collision proxies (Sec. 3: objects and furniture collide as convex
 * hulls of their parts; Sec. 4.3: simplified collision geometry).  From the
 * library's vertices and face loops: a face's plane is Newell's normal of
 * its loop (Newell 1972, as in Sutherland, Sproull and Schumacker 1974)
 * through the mean of its vertices; the edges are the loops' consecutive
 * vertex pairs, each once, in order of first appearance (faces in order,
 * each loop from its first vertex).  A box is the hull of its 8 corners
 * (corner k at (+-hx, +-hy, +-hz), + where bit 0, 1, 2 of k is set) with
 * faces -x, +x, -y, +y, -z, +z, loops {0 4 6 2} {1 3 7 5} {0 1 5 4}
 * {2 6 7 3} {0 2 3 1} {4 5 7 6}. */
static int hull_finish(Hull *H) {
    H->ne = 0;
    H->h[0] = H->h[1] = H->h[2] = 0.0;
    H->rad = 0.0;
    for (int k = 0; k < H->nv; k++) {
        H->h[0] = fmax(H->h[0], fabs(H->v[k].x));
        H->h[1] = fmax(H->h[1], fabs(H->v[k].y));
        H->h[2] = fmax(H->h[2], fabs(H->v[k].z));
        H->rad = fmax(H->rad, sqrt(len2(H->v[k])));
    }
    for (int f = 0; f < H->nf; f++) {
        const int n = H->nl[f];
        if (n < 3) return -1;
        V nn = mk(0, 0, 0), c = mk(0, 0, 0);
        for (int k = 0; k < n; k++) {
            V a = H->v[H->loop[f][k]], b = H->v[H->loop[f][(k + 1) % n]];
            nn.x += (a.y - b.y) * (a.z + b.z);
            nn.y += (a.z - b.z) * (a.x + b.x);
            nn.z += (a.x - b.x) * (a.y + b.y);
            c = add(c, a);
        }
        double L = sqrt(len2(nn));
        if (!(L > 0)) return -1;
        H->fn[f] = scl(nn, 1.0 / L);
        H->fd[f] = dot(H->fn[f], scl(c, 1.0 / n));
    }
    for (int f = 0; f < H->nf; f++) {
        const int n = H->nl[f];
        for (int k = 0; k < n; k++) {
            int a = H->loop[f][k], b = H->loop[f][(k + 1) % n];
            int lo = a < b ? a : b, hi = a < b ? b : a, seen = -1;
            for (int e = 0; e < H->ne; e++) if (H->ea[e] == lo && H->eb[e] == hi) seen = e;
            if (seen < 0) {
                if (H->ne >= HULL_MAXE) return -1;
                H->ea[H->ne] = lo;
                H->eb[H->ne] = hi;
                H->ef[H->ne][0] = f;
                H->ef[H->ne][1] = -1;
                H->ne++;
            } else {
                H->ef[seen][1] = f;
            }
        }
    }
    for (int e = 0; e < H->ne; e++) if (H->ef[e][1] < 0) return -1;   /* not a closed surface */
    return 0;
}

static int hull_from_lib(const ora_model *m, int h, Hull *H) {
    if (!m || h < 0 || h >= m->n_hulls) return -1;
    const int32_t *ix = m->hull_index + 4 * h;
    int v0 = ix[0], nv = ix[1], f0 = ix[2], nf = ix[3];
    if (nv < 4 || nv > HULL_MAXV || nf < 4 || nf > HULL_MAXF) return -1;
    H->nv = nv;
    H->nf = nf;
    for (int k = 0; k < nv; k++)
        H->v[k] = mk(m->hull_vert[3 * (v0 + k)], m->hull_vert[3 * (v0 + k) + 1], m->hull_vert[3 * (v0 + k) + 2]);
    for (int f = 0; f < nf; f++) {
        int n = 0;
        for (int k = 0; k < HULL_MAXL; k++) {
            int vi = m->hull_face[HULL_MAXL * (f0 + f) + k];
            if (vi < 0) break;
            if (vi >= nv) return -1;
            H->loop[f][n++] = vi;
        }
        H->nl[f] = n;
    }
    return hull_finish(H);
}

static void hull_box(const double *hb, Hull *H) {
    static const int loops[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};
    H->nv = 8;
    H->nf = 6;
    for (int k = 0; k < 8; k++)
        H->v[k] = mk((k & 1) ? hb[0] : -hb[0], (k & 2) ? hb[1] : -hb[1], (k & 4) ? hb[2] : -hb[2]);
    for (int f = 0; f < 6; f++) {
        H->nl[f] = 4;
        for (int k = 0; k < 4; k++) H->loop[f][k] = loops[f][k];
    }
    hull_finish(H);
}

/* Every hull of the library (NULL when there are none or one is unusable). */
static Hull *hulls_of(const ora_model *m) {
    if (!m || m->n_hulls <= 0 || !m->hull_index || !m->hull_vert || !m->hull_face) return NULL;
    Hull *HL = malloc(sizeof(Hull) * m->n_hulls);
    for (int h = 0; h < m->n_hulls; h++)
        if (hull_from_lib(m, h, &HL[h]) != 0) { free(HL); return NULL; }
    return HL;
}

/* Mass properties of a solid hull of uniform density: the solid is the
 * union of the tetrahedra (origin, a, b, c) over a fan triangulation of
 * every face loop (signed volumes, so any interior origin works); a
 * tetrahedron (0, a, b, c) of volume v has second moment
 * v/20 (a a^T + b b^T + c c^T + s s^T), s = a + b + c, and centroid s/4. */
static int hull_mass_props(const Hull *H, double mass, double I[3][3], V *com, double *vol) {
    double C[3][3] = {{0}};
    double V0 = 0;
    V cm = mk(0, 0, 0);
    for (int f = 0; f < H->nf; f++)
        for (int k = 1; k + 1 < H->nl[f]; k++) {
            V a = H->v[H->loop[f][0]], b = H->v[H->loop[f][k]], c = H->v[H->loop[f][k + 1]];
            double v = dot(a, cross(b, c)) / 6.0;
            V sm = add(add(a, b), c);
            V P[4] = {a, b, c, sm};
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    double t = 0;
                    for (int q = 0; q < 4; q++) t += comp(P[q], i) * comp(P[q], j);
                    C[i][j] += v / 20.0 * t;
                }
            V0 += v;
            cm = add(cm, scl(sm, v / 4.0));
        }
    if (!(V0 > 0)) return -1;
    double rho = mass / V0, tr = (C[0][0] + C[1][1] + C[2][2]) * rho;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) I[i][j] = (i == j ? tr : 0.0) - rho * C[i][j];
    *com = scl(cm, 1.0 / V0);
    *vol = V0;
    return 0;
}

int ora_hull_mass(const ora_model *m, int h, double mass, double *I, double *com, double *volume) {
    Hull H;
    if (hull_from_lib(m, h, &H) != 0) return -1;
    double T[3][3];
    V c;
    if (hull_mass_props(&H, mass, T, &c, volume) != 0) return -1;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) I[3 * i + j] = T[i][j];
    com[0] = c.x; com[1] = c.y; com[2] = c.z;
    return 0;
}

/* Whether p (in the face's plane) lies inside face f's loop (strictly or on
 * an edge: the side of every loop edge's in-plane outward normal). */
static int inside_loop(const Hull *H, int f, V p) {
    const int n = H->nl[f];
    for (int k = 0; k < n; k++) {
        V a = H->v[H->loop[f][k]], b = H->v[H->loop[f][(k + 1) % n]];
        if (dot(cross(sub(b, a), H->fn[f]), sub(p, a)) > 0) return 0;
    }
    return 1;
}

/* Closest point of the hull to p, for p outside it: the projections onto
 * faces that p lies above and that fall inside their loops, and the closest
 * point of every edge; the nearest wins (ties: faces first, lower index).
 * Returns the distance; *q the point, *face the face (-1 for an edge). */
static double hull_closest(const Hull *H, V p, V *q, int *face) {
    double best = INFINITY;
    *face = -1;
    for (int f = 0; f < H->nf; f++) {
        double s = dot(H->fn[f], p) - H->fd[f];
        if (s <= 0) continue;
        V pr = sub(p, scl(H->fn[f], s));
        if (inside_loop(H, f, pr) && s < best) { best = s; *q = pr; *face = f; }
    }
    for (int e = 0; e < H->ne; e++) {
        V a = H->v[H->ea[e]], d = sub(H->v[H->eb[e]], a);
        double t = clampd(dot(sub(p, a), d) / len2(d), 0.0, 1.0);
        V c = add(a, scl(d, t));
        double L = sqrt(len2(sub(p, c)));
        if (L < best) { best = L; *q = c; *face = -1; }
    }
    return best;
}

/* Choice among scores v[idx[0..n)] (candidates in index order) with a
 * tolerance: the first candidate whose score is within tol of the largest
 * (so scores equal up to rounding, as on a symmetric face, go to the lower
 * index); a score within band of the cut is ambiguous.  Skips used[].  Returns the
 * candidate, -1 if none. */
static int argmax_tol(const double *v, const int *idx, int n, const int *used, double tol, double band, int *amb) {
    double vmax = -INFINITY;
    for (int k = 0; k < n; k++) if (!used[idx[k]]) vmax = fmax(vmax, v[idx[k]]);
    int best = -1;
    for (int k = 0; k < n; k++) {
        int q = idx[k];
        if (used[q]) continue;
        if (fabs(v[q] - (vmax - tol)) < band) (*amb)++;
        if (best < 0 && v[q] >= vmax - tol) best = q;
    }
    return best;
}

/* At most 4 of n candidate points p[idx[k]] (in index order; n > 4): the
 * first, the farthest from it, the one spanning the largest triangle with
 * those, the one adding most to the three triangles' areas; each by
 * argmax_tol with CLIP_ON (areas scaled by the first edge's length, the
 * last by the triangle's perimeter). */
static void reduce4(const V *p, const int *idx, int n, int first, int *used, int *amb) {
    double sc[96];
    used[first] = 1;
    for (int k = 0; k < n; k++) sc[idx[k]] = sqrt(len2(sub(p[idx[k]], p[first])));
    int i2 = argmax_tol(sc, idx, n, used, CLIP_ON, BAND, amb);
    used[i2] = 1;
    V e12 = sub(p[i2], p[first]);
    double l12 = sqrt(len2(e12));
    for (int k = 0; k < n; k++) sc[idx[k]] = sqrt(len2(cross(e12, sub(p[idx[k]], p[first]))));
    int i3 = argmax_tol(sc, idx, n, used, CLIP_ON * l12, BAND * l12, amb);
    used[i3] = 1;
    V e23 = sub(p[i3], p[i2]), e31 = sub(p[first], p[i3]);
    double per = l12 + sqrt(len2(e23)) + sqrt(len2(e31));
    for (int k = 0; k < n; k++) {
        int q = idx[k];
        sc[q] = sqrt(len2(cross(e12, sub(p[q], p[first])))) + sqrt(len2(cross(e23, sub(p[q], p[i2])))) +
                sqrt(len2(cross(e31, sub(p[q], p[i3]))));
    }
    int i4 = argmax_tol(sc, idx, n, used, CLIP_ON * per, BAND * per, amb);
    used[i4] = 1;
}

/* Hull (first) on the ground plane: vertices with depth <= margin; above
 * 4, reduce4 from the first vertex within CLIP_ON of the deepest (a flat
 * face resting on the ground keeps a spread of its corners); reported in
 * vertex order, the feature the vertex index. */
static int hull_ground(const Geom *A, double margin, PC *out, int *amb) {
    const Hull *H = A->hull;
    V w[HULL_MAXV];
    double z[HULL_MAXV];
    int id[HULL_MAXV], m = 0;
    for (int k = 0; k < H->nv; k++) {
        w[k] = add(A->x, Rv(&A->R, H->v[k]));
        z[k] = w[k].z;
        if (keep(z[k], margin, amb)) id[m++] = k;
    }
    if (m > 4) {
        double nz[HULL_MAXV];
        int used[96] = {0};
        for (int k = 0; k < H->nv; k++) nz[k] = -z[k];
        int first = argmax_tol(nz, id, m, used, CLIP_ON, BAND, amb);
        reduce4(w, id, m, first, used, amb);
        m = 0;
        for (int k = 0; k < H->nv; k++) if (used[k]) id[m++] = k;
    }
    for (int k = 0; k < m; k++) {
        PC c;
        c.n = mk(0, 0, 1);
        c.phi = z[id[k]];
        c.p = mk(w[id[k]].x, w[id[k]].y, 0.5 * w[id[k]].z);
        c.f = id[k];
        out[k] = c;
    }
    return m;
}

/* Sphere (first) against a hull (second), in the hull frame: a centre
 * outside leaves along the line to the hull's closest point; a centre
 * inside through the face of least penetration (ties: lower face). */
static int sphere_hull(const Geom *S, const Geom *G, double margin, PC *out, int *amb) {
    const Hull *H = G->hull;
    double r = S->prm[0];
    V l = RTv(&G->R, sub(S->x, G->x));
    double smax = -INFINITY, sf[HULL_MAXF];
    int fm = 0;
    for (int f = 0; f < H->nf; f++) {
        sf[f] = dot(H->fn[f], l) - H->fd[f];
        if (sf[f] > smax) { smax = sf[f]; fm = f; }
    }
    if (fabs(smax) < BAND) (*amb)++;
    V nl, q;
    double phi;
    if (smax <= 0) {
        for (int f = 0; f < H->nf; f++) if (f != fm && fabs(sf[f] - smax) < BAND) (*amb)++;
        nl = H->fn[fm];
        q = sub(l, scl(nl, smax));
        phi = smax - r;
    } else {
        int face;
        double dist = hull_closest(H, l, &q, &face);
        if (dist < BAND) (*amb)++;
        nl = scl(sub(l, q), 1.0 / dist);
        phi = dist - r;
    }
    PC c;
    c.n = Rv(&G->R, nl);
    V wb = add(G->x, Rv(&G->R, q));
    V wa = sub(S->x, scl(c.n, r));
    c.p = scl(add(wa, wb), 0.5);
    c.phi = phi;
    c.f = 0;
    if (!keep(phi, margin, amb)) return 0;
    out[0] = c;
    return 1;
}

/* The core segment p0 + t d clipped to face f's prism (the in-plane
 * outward normals of its loop edges); ok iff t0 <= t1. */
static int clip_prism(const Hull *H, int f, V p0, V d, double *t0, double *t1) {
    double a = 0.0, b = 1.0;
    const int n = H->nl[f];
    for (int k = 0; k < n; k++) {
        V va = H->v[H->loop[f][k]], vb = H->v[H->loop[f][(k + 1) % n]];
        V mm = cross(sub(vb, va), H->fn[f]);
        double g0 = dot(mm, sub(p0, va)), gd = dot(mm, d);
        if (gd == 0.0) {
            if (g0 > 0) return 0;
            continue;
        }
        double t = -g0 / gd;
        if (gd > 0) b = fmin(b, t);
        else a = fmax(a, t);
    }
    *t0 = a;
    *t1 = b;
    return a <= b;
}

/* One contact of the core point l against face f (hull frame). */
static PC hull_face_contact(const Hull *H, int f, V l, double r, int ft) {
    PC c;
    c.n = H->fn[f];
    double s = dot(c.n, l) - H->fd[f];
    c.phi = s - r;
    V q = sub(l, scl(c.n, s));
    c.p = scl(add(q, sub(l, scl(c.n, r))), 0.5);
    c.f = ft;
    return c;
}

/* Face region of a core point l outside the hull: the face whose plane it
 * is above and whose loop holds its projection (-1: edge or vertex region). */
static int face_region(const Hull *H, V l) {
    int best = -1;
    double bs = 0;
    for (int f = 0; f < H->nf; f++) {
        double s = dot(H->fn[f], l) - H->fd[f];
        if (s > 0 && inside_loop(H, f, sub(l, scl(H->fn[f], s))) && (best < 0 || s > bs)) { best = f; bs = s; }
    }
    return best;
}

/* Capsule (first) against a hull (second), in the hull frame, after
 * capsule_box:
 * 1. Core separated from the hull (the segment clipped to every face's
 *    half-space (Cyrus and Beck 1978) is empty): closest points among the
 *    ends against the hull and the core against every edge (Ericson 2005,
 *    5.1.9, clamped); nearest wins (ties: the order tried).
 * 2. Closest core point in a face's region with the core within ~1 mrad
 *    of parallel to that face, or the core that parallel to a face whose
 *    plane lies at the closest distance (within CLIP_ON) and whose prism it
 *    crosses (a plateau of the distance over the face): two contacts at the
 *    ends of the core clipped to the face's prism (f 0, 1); otherwise one at
 *    the closest points (f 2).
 * 3. Core touching the hull: leave through the face whose plane the deeper
 *    core end lies least below (ties: lower face); contacts at the ends of
 *    the core clipped to that face's prism (f 0, 1), else at the deeper end
 *    (f 3). */
static int capsule_hull(const Geom *C, const Geom *G, double margin, PC *out, int *amb) {
    const Hull *H = G->hull;
    double r = C->prm[0];
    V P0, D;
    capsule_seg(C, &P0, &D);
    V p0 = RTv(&G->R, sub(P0, G->x));
    V d = RTv(&G->R, D);
    double dl = sqrt(len2(d));
    double tin = 0.0, tout = 1.0;
    for (int f = 0; f < H->nf; f++) {
        double dn = dot(H->fn[f], d), s0 = dot(H->fn[f], p0) - H->fd[f];
        if (dn == 0.0) {
            if (fabs(s0) < BAND) (*amb)++;
            if (s0 > 0) tout = -1.0;
            continue;
        }
        double t = -s0 / dn;
        if (dn < 0) tin = fmax(tin, t);
        else tout = fmin(tout, t);
    }
    int meets = tin <= tout;
    if (fabs(tout - tin) * dl < BAND) (*amb)++;
    PC loc[2];
    int n = 0;
    if (!meets) {
        /* candidates: (distance, core parameter, hull point) */
        double cd[2 + HULL_MAXE], ct[2 + HULL_MAXE];
        V cq[2 + HULL_MAXE];
        int nc = 0;
        for (int e2 = 0; e2 < 2; e2++) {
            int face;
            V q;
            cd[nc] = hull_closest(H, add(p0, scl(d, (double)e2)), &q, &face);
            ct[nc] = (double)e2;
            cq[nc] = q;
            nc++;
        }
        for (int e = 0; e < H->ne; e++) {
            V a = H->v[H->ea[e]], u = sub(H->v[H->eb[e]], a);
            /* closest points of p0 + t d and a + s u, t, s in [0, 1] */
            V w = sub(p0, a);
            double A2 = len2(d), B2 = dot(d, u), C2 = len2(u), D2 = dot(d, w), E2 = dot(u, w);
            double den = A2 * C2 - B2 * B2, t = 0.0, sv;
            if (den > 1e-18 * A2 * C2) t = clampd((B2 * E2 - C2 * D2) / den, 0.0, 1.0);
            sv = (B2 * t + E2) / C2;
            if (sv < 0.0) { sv = 0.0; t = clampd(-D2 / A2, 0.0, 1.0); }
            else if (sv > 1.0) { sv = 1.0; t = clampd((B2 - D2) / A2, 0.0, 1.0); }
            V pc = add(p0, scl(d, t)), qc = add(a, scl(u, sv));
            cd[nc] = sqrt(len2(sub(pc, qc)));
            ct[nc] = t;
            cq[nc] = qc;
            nc++;
        }
        int bi = 0;
        for (int i = 1; i < nc; i++) if (cd[i] < cd[bi]) bi = i;
        double dist = cd[bi], t = ct[bi];
        V l = add(p0, scl(d, t)), q = cq[bi];
        if (dist < BAND) (*amb)++;
        int fr = face_region(H, l);
        int facecase = fr >= 0 && fabs(dot(d, H->fn[fr])) <= SIN_PAR * dl;
        if (fr >= 0) {
            double thr = SIN_PAR * dl;
            if (fabs(fabs(dot(d, H->fn[fr])) - thr) < 1e-2 * thr) (*amb)++;
        }
        /* a core level with a face at the distance found lies on that face's
         * plateau, which may end on the face's boundary (where the region of
         * the closest point is ill-defined): the first such face whose prism
         * the core crosses */
        int plateau = 0;
        if (!facecase) {
            for (int f = 0; f < H->nf && !facecase; f++) {
                double thr = SIN_PAR * dl, dn = fabs(dot(d, H->fn[f]));
                if (dn > thr) continue;
                double gap = fabs(dot(H->fn[f], l) - H->fd[f] - dist);
                if (fabs(gap - CLIP_ON) < BAND) (*amb)++;
                double t0, t1;
                if (gap <= CLIP_ON && clip_prism(H, f, p0, d, &t0, &t1)) {
                    if (fabs(dn - thr) < 1e-2 * thr) (*amb)++;
                    fr = f;
                    facecase = plateau = 1;
                }
            }
        }
        /* a plateau of the distance at another place decides differently */
        for (int i = 0; i < nc && !plateau; i++) {
            if (i == bi || fabs(cd[i] - dist) >= BAND || fabs(ct[i] - t) * dl <= BAND) continue;
            V li = add(p0, scl(d, ct[i]));
            int fi = face_region(H, li);
            int fci = fi >= 0 && fabs(dot(d, H->fn[fi])) <= SIN_PAR * dl;
            if (!facecase || !fci || fi != fr) { (*amb)++; break; }
        }
        int done = 0;
        if (facecase) {
            double t0, t1;
            if (clip_prism(H, fr, p0, d, &t0, &t1)) {
                if (fabs(t1 - t0) * dl < BAND) (*amb)++;
                loc[n++] = hull_face_contact(H, fr, add(p0, scl(d, t0)), r, 0);
                if (t1 > t0) loc[n++] = hull_face_contact(H, fr, add(p0, scl(d, t1)), r, 1);
                done = 1;
            }
        }
        if (!done) {
            PC c;
            c.n = scl(sub(l, q), 1.0 / dist);
            c.phi = dist - r;
            c.p = scl(add(q, sub(l, scl(c.n, r))), 0.5);
            c.f = 2;
            loc[n++] = c;
        }
    } else {
        double best = INFINITY, second = INFINITY;
        int bf = 0;
        V p1 = add(p0, d);
        for (int f = 0; f < H->nf; f++) {
            double ex = H->fd[f] - fmin(dot(H->fn[f], p0), dot(H->fn[f], p1));
            if (ex < best) { second = best; best = ex; bf = f; }
            else if (ex < second) second = ex;
        }
        if (second - best < BAND) (*amb)++;
        double t0, t1;
        int ok = clip_prism(H, bf, p0, d, &t0, &t1);
        if (ok && fabs(t1 - t0) * dl < BAND) (*amb)++;
        if (ok) {
            loc[n++] = hull_face_contact(H, bf, add(p0, scl(d, t0)), r, 0);
            if (t1 > t0) loc[n++] = hull_face_contact(H, bf, add(p0, scl(d, t1)), r, 1);
        } else {
            double e0 = dot(H->fn[bf], p0), e1 = dot(H->fn[bf], p1);
            if (fabs(e0 - e1) < BAND) (*amb)++;
            loc[n++] = hull_face_contact(H, bf, e0 <= e1 ? p0 : p1, r, 3);
        }
    }
    int m = 0;
    for (int k = 0; k < n; k++) {
        if (!keep(loc[k].phi, margin, amb)) continue;
        PC c = loc[k];
        c.n = Rv(&G->R, loc[k].n);
        c.p = add(G->x, Rv(&G->R, loc[k].p));
        out[m++] = c;
    }
    return m;
}

/* Hull against hull (a box enters as the hull of its corners): separating
 * axes (Gottschalk et al. 1996) over both hulls' face normals and the
 * cross products of every edge pair, a separation being the gap between
 * the two vertex sets' projections; the first hull's face wins near ties,
 * edges only when clearly better (the thresholds of box_box, the largest
 * half-extent of the two local bounding boxes for the boxes').
 * Edge axes from the pairs of edges that build faces of the Minkowski
 * difference (Gregorius 2013); edge contact: closest points of the two
 * edges (f 0xFF).
 * Face contact: the incident face is the other hull's face most opposed to
 * the reference face; the contact points are the vertices of the two
 * faces' overlap seen along the reference normal (the polygon that
 * clipping the incident face by the reference face's side planes leaves,
 * Sutherland and Hodgman 1974), taken point by point with an index each:
 * incident vertices inside every side plane (id k), incident edges crossing
 * a side plane inside the others (id 8 + 8 k + j), reference corners inside
 * the incident face (id 72 + j; the point on the incident face's plane
 * along the reference normal); three-state sides as in box_box.  Kept
 * points (depth <= margin) above 4 are reduced by reduce4 from the
 * smallest id; the feature is (reference is the second hull) | id << 1,
 * points in id order. */
static int hull_hull(const Geom *A, const Geom *B, double margin, PC *out, int *amb) {
    Hull ba, bb;
    const Hull *HA = A->hull, *HB = B->hull;
    if (A->shape == ORA_BOX) { hull_box(A->prm, &ba); HA = &ba; }
    if (B->shape == ORA_BOX) { hull_box(B->prm, &bb); HB = &bb; }
    V VA[HULL_MAXV], VB[HULL_MAXV], NA[HULL_MAXF], NB[HULL_MAXF];
    double DA[HULL_MAXF], DB[HULL_MAXF];
    for (int k = 0; k < HA->nv; k++) VA[k] = add(A->x, Rv(&A->R, HA->v[k]));
    for (int k = 0; k < HB->nv; k++) VB[k] = add(B->x, Rv(&B->R, HB->v[k]));
    for (int f = 0; f < HA->nf; f++) { NA[f] = Rv(&A->R, HA->fn[f]); DA[f] = dot(NA[f], A->x) + HA->fd[f]; }
    for (int f = 0; f < HB->nf; f++) { NB[f] = Rv(&B->R, HB->fn[f]); DB[f] = dot(NB[f], B->x) + HB->fd[f]; }
    double sA[HULL_MAXF], sB[HULL_MAXF];
    int fa = 0, fb = 0;
    for (int f = 0; f < HA->nf; f++) {
        double s = INFINITY;
        for (int k = 0; k < HB->nv; k++) s = fmin(s, dot(NA[f], VB[k]) - DA[f]);
        sA[f] = s;
        if (s > sA[fa]) fa = f;
    }
    for (int f = 0; f < HB->nf; f++) {
        double s = INFINITY;
        for (int k = 0; k < HA->nv; k++) s = fmin(s, dot(NB[f], VA[k]) - DB[f]);
        sB[f] = s;
        if (s > sB[fb]) fb = f;
    }
    /* edge axes: only pairs whose edges build a face of the Minkowski
     * difference (their arcs on the Gauss map cross: Gregorius 2013); the
     * axis u = e_A x e_B points away from A's centre and the separation is
     * u . (b - a), a and b the edges' first vertices */
    double se = -INFINITY;
    int ei = -1, ej = -1;
    V ue = mk(0, 0, 1);
    for (int i = 0; i < HA->ne; i++) {
        V a = NA[HA->ef[i][0]], b = NA[HA->ef[i][1]], bxa = cross(b, a);
        V da = sub(VA[HA->eb[i]], VA[HA->ea[i]]);
        for (int j = 0; j < HB->ne; j++) {
            V c = scl(NB[HB->ef[j][0]], -1.0), d = scl(NB[HB->ef[j][1]], -1.0), dxc = cross(d, c);
            double cba = dot(c, bxa), dba = dot(d, bxa), adc = dot(a, dxc), bdc = dot(b, dxc);
            /* (arcs that only touch give an axis equal to a face normal, whose
             * separation the face axes already hold: no tie to flag) */
            if (!(cba * dba < 0 && adc * bdc < 0 && cba * bdc > 0)) continue;
            V db = sub(VB[HB->eb[j]], VB[HB->ea[j]]);
            V u = cross(da, db);
            double L2 = len2(u), ref = len2(da) * len2(db);
            if (fabs(L2 - 1e-12 * ref) < 1e-13 * ref) (*amb)++;
            if (L2 < 1e-12 * ref) continue;
            u = scl(u, 1.0 / sqrt(L2));
            if (dot(u, sub(VA[HA->ea[i]], A->x)) < 0) u = scl(u, -1.0);
            double sv = dot(u, sub(VB[HB->ea[j]], VA[HA->ea[i]]));
            if (sv > se) { se = sv; ei = i; ej = j; ue = u; }
        }
    }
    double smax = fmax(fmax(sA[fa], sB[fb]), se);
    if (fabs(smax - margin) < BAND) (*amb)++;
    if (smax > margin) return 0;
    double hmax = 0;
    for (int i = 0; i < 3; i++) hmax = fmax(hmax, fmax(HA->h[i], HB->h[i]));
    int refB = 0;
    double sface = sA[fa];
    double thr = 0.95 * sA[fa] + 0.01 * hmax;
    if (fabs(sB[fb] - thr) < BAND) (*amb)++;
    if (sB[fb] > thr) { refB = 1; sface = sB[fb]; }
    int edge = 0;
    if (ei >= 0) {
        double thr2 = 0.95 * sface + 0.01 * hmax;
        if (fabs(se - thr2) < BAND) (*amb)++;
        edge = se > thr2;
    }
    if (edge) {
        /* near ties with another Minkowski pair of another axis direction */
        for (int i = 0; i < HA->ne; i++) {
            V a = NA[HA->ef[i][0]], b = NA[HA->ef[i][1]], bxa = cross(b, a);
            V da = sub(VA[HA->eb[i]], VA[HA->ea[i]]);
            for (int j = 0; j < HB->ne; j++) {
                V c = scl(NB[HB->ef[j][0]], -1.0), d = scl(NB[HB->ef[j][1]], -1.0), dxc = cross(d, c);
                double cba = dot(c, bxa), dba = dot(d, bxa), adc = dot(a, dxc), bdc = dot(b, dxc);
                if (!(cba * dba < 0 && adc * bdc < 0 && cba * bdc > 0)) continue;
                V db = sub(VB[HB->eb[j]], VB[HB->ea[j]]);
                V u = cross(da, db);
                double L2 = len2(u), ref = len2(da) * len2(db);
                if (L2 < 1e-12 * ref) continue;
                u = scl(u, 1.0 / sqrt(L2));
                if (len2(cross(u, ue)) < 1e-10) continue;
                if (dot(u, sub(VA[HA->ea[i]], A->x)) < 0) u = scl(u, -1.0);
                if (fabs(dot(u, sub(VB[HB->ea[j]], VA[HA->ea[i]])) - se) < BAND) (*amb)++;
            }
        }
        V N = scl(ue, -1.0);   /* from B to A */
        int ia = ei, jb = ej;
        V a0 = VA[HA->ea[ia]], a1 = VA[HA->eb[ia]], b0 = VB[HB->ea[jb]], b1 = VB[HB->eb[jb]];
        V pa = scl(add(a0, a1), 0.5), pb = scl(add(b0, b1), 0.5);
        V ai = sub(a1, a0), bj = sub(b1, b0);
        double la = 0.5 * sqrt(len2(ai)), lb = 0.5 * sqrt(len2(bj));
        ai = scl(ai, 0.5 / la);
        bj = scl(bj, 0.5 / lb);
        V w = sub(pa, pb);
        double bbd = dot(ai, bj), dd = dot(ai, w), ee = dot(bj, w);
        double den = 1.0 - bbd * bbd;
        double ta = (bbd * ee - dd) / den;
        double tb = ee + ta * bbd;
        ta = clampd(ta, -la, la);
        tb = clampd(tb, -lb, lb);
        V PA = add(pa, scl(ai, ta)), PB = add(pb, scl(bj, tb));
        PC c;
        c.n = N;
        c.phi = dot(sub(PA, PB), N);
        c.p = scl(add(PA, PB), 0.5);
        c.f = 0xFF;
        if (!keep(c.phi, margin, amb)) return 0;
        out[0] = c;
        return 1;
    }
    /* near ties inside the face group used */
    if (!refB) { for (int f = 0; f < HA->nf; f++) if (f != fa && fabs(sA[f] - sA[fa]) < BAND) (*amb)++; }
    else { for (int f = 0; f < HB->nf; f++) if (f != fb && fabs(sB[f] - sB[fb]) < BAND) (*amb)++; }
    const Hull *HR = refB ? HB : HA, *HI = refB ? HA : HB;
    const V *VR = refB ? VB : VA, *VI = refB ? VA : VB;
    const V *NI = refB ? NA : NB;
    const double *DI = refB ? DA : DB;
    int rf = refB ? fb : fa;
    V nout = refB ? NB[fb] : NA[fa];
    double Dref = refB ? DB[fb] : DA[fa];
    V N = refB ? nout : scl(nout, -1.0);
    /* incident face: most opposed to nout (ties: lower face) */
    int inf = 0;
    for (int f = 1; f < HI->nf; f++) if (dot(NI[f], nout) < dot(NI[inf], nout)) inf = f;
    for (int f = 0; f < HI->nf; f++)
        if (f != inf && fabs(dot(NI[f], nout) - dot(NI[inf], nout)) < BAND_DIM) (*amb)++;
    const int nR = HR->nl[rf], nI = HI->nl[inf];
    V R[HULL_MAXL], X[HULL_MAXL], mR[HULL_MAXL], mI[HULL_MAXL];
    for (int j = 0; j < nR; j++) R[j] = VR[HR->loop[rf][j]];
    for (int k = 0; k < nI; k++) X[k] = VI[HI->loop[inf][k]];
    for (int j = 0; j < nR; j++) {
        V m = cross(sub(R[(j + 1) % nR], R[j]), nout);
        mR[j] = scl(m, 1.0 / sqrt(len2(m)));
    }
    V ninc = NI[inf];
    for (int k = 0; k < nI; k++) {
        V m = cross(sub(X[(k + 1) % nI], X[k]), ninc);
        mI[k] = scl(m, 1.0 / sqrt(len2(m)));
    }
    /* candidate points in id order */
    V cp[96];
    double cph[96];
    int cid[96], nk = 0;
#define SIDE(dv) ((dv) < -CLIP_ON ? -1 : ((dv) > CLIP_ON ? 1 : 0))
    for (int k = 0; k < nI; k++) {
        int in = 1;
        for (int j = 0; j < nR; j++) {
            double dv = dot(mR[j], sub(X[k], R[j]));
            if (fabs(fabs(dv) - CLIP_ON) < BAND) (*amb)++;
            if (dv > CLIP_ON) in = 0;
        }
        if (in) { cp[nk] = X[k]; cid[nk] = k; nk++; }
    }
    for (int k = 0; k < nI; k++)
        for (int j = 0; j < nR; j++) {
            V x0 = X[k], x1 = X[(k + 1) % nI];
            double d0 = dot(mR[j], sub(x0, R[j])), d1 = dot(mR[j], sub(x1, R[j]));
            if (SIDE(d0) * SIDE(d1) >= 0) continue;
            V y = add(x0, scl(sub(x1, x0), d0 / (d0 - d1)));
            int in = 1;
            for (int i = 0; i < nR; i++) {
                if (i == j) continue;
                double dv = dot(mR[i], sub(y, R[i]));
                if (fabs(fabs(dv) - CLIP_ON) < BAND) (*amb)++;
                if (dv > CLIP_ON) in = 0;
            }
            if (in) { cp[nk] = y; cid[nk] = 8 + 8 * k + j; nk++; }
        }
    double Dinc = DI[inf];
    for (int j = 0; j < nR; j++) {
        double t = (Dinc - dot(ninc, R[j])) / dot(ninc, nout);
        V z = add(R[j], scl(nout, t));
        int in = 1;
        for (int k = 0; k < nI; k++) {
            double dv = dot(mI[k], sub(z, X[k]));
            if (fabs(fabs(dv) - CLIP_ON) < BAND) (*amb)++;
            if (!(dv < -CLIP_ON)) in = 0;
        }
        if (in) { cp[nk] = z; cid[nk] = 72 + j; nk++; }
    }
#undef SIDE
    int idx[96], nkeep = 0;
    for (int k = 0; k < nk; k++) {
        cph[k] = dot(nout, cp[k]) - Dref;
        if (keep(cph[k], margin, amb)) idx[nkeep++] = k;
    }
    int used[96] = {0};
    if (nkeep <= 4) {
        for (int k = 0; k < nkeep; k++) used[idx[k]] = 1;
    } else {
        reduce4(cp, idx, nkeep, idx[0], used, amb);   /* from the smallest id */
    }
    int m = 0;
    for (int k = 0; k < nk; k++) {
        if (!used[k]) continue;
        PC c;
        c.n = N;
        c.phi = cph[k];
        c.p = sub(cp[k], scl(nout, 0.5 * cph[k]));
        c.f = refB | (cid[k] << 1);
        out[m++] = c;
    }
    return m;
}

/* Ground plane z = 0 (second) against a body (first). */
static int ground_contacts(const Geom *A, double margin, PC *out, int *amb) {
    int n = 0;
    V up = mk(0, 0, 1);
    if (A->shape == ORA_HULL) return hull_ground(A, margin, out, amb);
    if (A->shape == ORA_SPHERE) {
        PC c;
        c.n = up;
        c.phi = A->x.z - A->prm[0];
        c.p = mk(A->x.x, A->x.y, 0.5 * (A->x.z - A->prm[0]));
        c.f = 0;
        if (keep(c.phi, margin, amb)) out[n++] = c;
    } else if (A->shape == ORA_CAPSULE) {
        V p0, d;
        capsule_seg(A, &p0, &d);
        for (int k = 0; k < 2; k++) {
            V e = k == 0 ? p0 : add(p0, d);
            PC c;
            c.n = up;
            c.phi = e.z - A->prm[0];
            c.p = mk(e.x, e.y, 0.5 * (e.z - A->prm[0]));
            c.f = k;
            if (keep(c.phi, margin, amb)) out[n++] = c;
        }
    } else {
        /* corners with depth <= margin; at most the 4 deepest (ties: lower
         * corner index); reported in corner order */
        V cn[8];
        double ph[8];
        int id[8], m = 0;
        for (int k = 0; k < 8; k++) {
            V off = mk((k & 1) ? A->prm[0] : -A->prm[0], (k & 2) ? A->prm[1] : -A->prm[1],
                       (k & 4) ? A->prm[2] : -A->prm[2]);
            cn[k] = add(A->x, Rv(&A->R, off));
            ph[k] = cn[k].z;
            if (keep(ph[k], margin, amb)) id[m++] = k;
        }
        if (m > 4) {
            int ord[8];
            for (int k = 0; k < m; k++) ord[k] = id[k];
            for (int i = 1; i < m; i++)
                for (int j = i; j > 0 && (ph[ord[j]] < ph[ord[j - 1]] ||
                                          (ph[ord[j]] == ph[ord[j - 1]] && ord[j] < ord[j - 1])); j--) {
                    int x = ord[j]; ord[j] = ord[j - 1]; ord[j - 1] = x;
                }
            if (fabs(ph[ord[3]] - ph[ord[4]]) < BAND) (*amb)++;
            int keepk[8] = {0};
            for (int k = 0; k < 4; k++) keepk[ord[k]] = 1;
            m = 0;
            for (int k = 0; k < 8; k++) if (keepk[k]) id[m++] = k;
        }
        for (int k = 0; k < m; k++) {
            V c0 = cn[id[k]];
            PC c;
            c.n = up;
            c.phi = ph[id[k]];
            c.p = mk(c0.x, c0.y, 0.5 * c0.z);
            c.f = id[k];
            out[n++] = c;
        }
    }
    return n;
}

/* Contacts of the pair (A, B) with the normal from B to A. */
static int collide(const Geom *A, const Geom *B, double margin, PC *out, int *amb) {
    int ta = A->shape, tb = B->shape, n = 0, flip = 0;
    if (ta == ORA_HULL || tb == ORA_HULL) {
        if (ta == ORA_SPHERE) n = sphere_hull(A, B, margin, out, amb);
        else if (tb == ORA_SPHERE) { n = sphere_hull(B, A, margin, out, amb); flip = 1; }
        else if (ta == ORA_CAPSULE) n = capsule_hull(A, B, margin, out, amb);
        else if (tb == ORA_CAPSULE) { n = capsule_hull(B, A, margin, out, amb); flip = 1; }
        else n = hull_hull(A, B, margin, out, amb);
        if (flip)
            for (int k = 0; k < n; k++) out[k].n = scl(out[k].n, -1.0);
        return n;
    }
    if (ta == ORA_SPHERE && tb == ORA_SPHERE) {
        PC c = sphere_sphere(A->x, A->prm[0], B->x, B->prm[0], 0);
        if (keep(c.phi, margin, amb)) out[n++] = c;
    } else if (ta == ORA_SPHERE && tb == ORA_BOX) n = sphere_box(A, B, margin, out, amb);
    else if (ta == ORA_BOX && tb == ORA_SPHERE) { n = sphere_box(B, A, margin, out, amb); flip = 1; }
    else if (ta == ORA_SPHERE && tb == ORA_CAPSULE) n = sphere_capsule(A, B, margin, out, amb);
    else if (ta == ORA_CAPSULE && tb == ORA_SPHERE) { n = sphere_capsule(B, A, margin, out, amb); flip = 1; }
    else if (ta == ORA_CAPSULE && tb == ORA_BOX) n = capsule_box(A, B, margin, out, amb);
    else if (ta == ORA_BOX && tb == ORA_CAPSULE) { n = capsule_box(B, A, margin, out, amb); flip = 1; }
    else if (ta == ORA_BOX && tb == ORA_BOX) n = box_box(A, B, margin, out, amb);
    else n = capsule_capsule(A, B, margin, out, amb);
    if (flip)
        for (int k = 0; k < n; k++) out[k].n = scl(out[k].n, -1.0);
    return n;
}

static Geom geom_of(int shape, const double *prm, const double *pose, const Hull *HL) {
    Geom g;
    g.shape = shape;
    g.x = mk(pose[0], pose[1], pose[2]);
    g.R = quat_R(pose + 3);
    for (int i = 0; i < 3; i++) g.prm[i] = prm[i];
    g.hull = NULL;
    if (shape == ORA_HULL) {
        g.hull = &HL[(int)prm[0]];
        for (int i = 0; i < 3; i++) g.prm[i] = g.hull->h[i];
    }
    return g;
}

int ora_collide(int shape_a, const double *param_a, const double *pose_a,
                int shape_b, const double *param_b, const double *pose_b,
                int ground, double margin, int *feature, double *normal,
                double *point, double *phi, int *ambiguous) {
    if (shape_a == ORA_HULL || (!ground && shape_b == ORA_HULL)) return -1;
    return ora_collide_hulls(NULL, shape_a, param_a, pose_a, shape_b, param_b, pose_b, ground, margin, feature,
                             normal, point, phi, ambiguous);
}

int ora_collide_hulls(const ora_model *m, int shape_a, const double *param_a, const double *pose_a,
                      int shape_b, const double *param_b, const double *pose_b,
                      int ground, double margin, int *feature, double *normal,
                      double *point, double *phi, int *ambiguous) {
    Hull *HL = hulls_of(m);
    if ((shape_a == ORA_HULL && (!HL || !(param_a[0] >= 0 && param_a[0] < m->n_hulls))) ||
        (!ground && shape_b == ORA_HULL && (!HL || !(param_b[0] >= 0 && param_b[0] < m->n_hulls)))) {
        free(HL);
        return -1;
    }
    Geom A = geom_of(shape_a, param_a, pose_a, HL);
    PC c[4];
    int amb = 0, n;
    if (ground) n = ground_contacts(&A, margin, c, &amb);
    else {
        Geom B = geom_of(shape_b, param_b, pose_b, HL);
        n = collide(&A, &B, margin, c, &amb);
    }
    free(HL);
    for (int k = 0; k < n; k++) {
        feature[k] = c[k].f;
        normal[3 * k] = c[k].n.x; normal[3 * k + 1] = c[k].n.y; normal[3 * k + 2] = c[k].n.z;
        point[3 * k] = c[k].p.x; point[3 * k + 1] = c[k].p.y; point[3 * k + 2] = c[k].p.z;
        phi[k] = c[k].phi;
    }
    if (ambiguous) *ambiguous = amb;
    return n;
}

/* ---------------------------------------------------------------- arm */
/* Forward kinematics of the 7-joint chain: joint axes z, y, z, y, z, y, z in
 * each parent frame; link k is a capsule whose core runs from joint k to
 * joint k+1 along its local z.  Writes link centres/orientations, and the
 * world joint origins and axes. */
static void arm_fk(const ora_model *m, const double *base, const double *th,
                   double lpose[7][7], V o[7], V ax[7]) {
    double q[4] = {1, 0, 0, 0};
    V p = mk(base[0], base[1], base[2]);
    for (int k = 0; k < 7; k++) {
        double hq[4] = {cos(0.5 * th[k]), 0, 0, 0};
        if (k % 2 == 0) hq[3] = sin(0.5 * th[k]); else hq[2] = sin(0.5 * th[k]);
        double qk[4];
        quat_mul(q, hq, qk);
        M3 R = quat_R(qk);
        V zl = col(&R, 2);
        ax[k] = k % 2 == 0 ? zl : col(&R, 1);
        o[k] = p;
        V c = add(p, scl(zl, 0.5 * m->link_len[k]));
        lpose[k][0] = c.x; lpose[k][1] = c.y; lpose[k][2] = c.z;
        for (int i = 0; i < 4; i++) { lpose[k][3 + i] = qk[i]; q[i] = qk[i]; }
        p = add(p, scl(zl, m->link_len[k]));
    }
}

int ora_arm_pose(const ora_model *m, double *pose, const double *theta) {
    if (!m->arm) return 0;
    for (int s = 0; s < m->n_scenes; s++) {
        int b1 = m->body_offset[s + 1];
        double lp[7][7];
        V o[7], ax[7];
        arm_fk(m, m->arm_base + 3 * s, theta + 7 * s, lp, o, ax);
        for (int k = 0; k < 7; k++) memcpy(pose + 7 * (b1 - 7 + k), lp[k], 7 * sizeof(double));
    }
    return 0;
}

/* ---------------------------------------------------------------- pairs */

/* Links of the dynamic arm (arm 2) move with the arm's joint rates, not as
 * free bodies: within a step they carry no velocity or mass of their own
 * (the arm holds both), and they collide with everything but each other. */
#define ORA_ARMLINK 3
static int movable(const Body *b) { return b->motion == ORA_DYNAMIC || b->motion == ORA_ARMLINK; }

/* Brute-force pair set: every i < j with at least one dynamic body whose
 * closed AABBs overlap on x, y and z, then (i, ground) for dynamic i whose
 * AABB reaches z <= 0; lexicographic order. */
static int brute_pairs(const Body *B, int n, int arm0, const int32_t *parent, uint32_t *keys, int cap, int *amb,
                       uint8_t *tied) {
    int np = 0;
    for (int i = 0; i < n; i++) {
        for (int j = i + 1; j < n; j++) {
            if (!movable(&B[i]) && !movable(&B[j])) continue;
            if (i >= arm0) continue;     /* two links of the dynamic arm: joined, not in contact */
            /* a part and the base it is joined to */
            if (parent && ((B[i].joint && parent[i] == j) || (B[j].joint && parent[j] == i))) continue;
            double sl = INFINITY;
            for (int a = 0; a < 3; a++) {
                double s1 = comp(B[i].hi, a) - comp(B[j].lo, a);
                double s2 = comp(B[j].hi, a) - comp(B[i].lo, a);
                sl = fmin(sl, fmin(s1, s2));
            }
            if (fabs(sl) < BAND) {
                (*amb)++;
                if (tied) tied[i] = tied[j] = 1;
            }
            if (sl >= 0) {
                if (np < cap) keys[np] = ((uint32_t)i << 16) | (uint32_t)j;
                np++;
            }
        }
        if (movable(&B[i])) {
            if (fabs(B[i].lo.z) < BAND) {
                (*amb)++;
                if (tied) tied[i] = 1;
            }
            if (B[i].lo.z <= 0) {
                if (np < cap) keys[np] = ((uint32_t)i << 16) | PAIR_GROUND;
                np++;
            }
        }
    }
    return np;
}

/* ---------------------------------------------------------------- scene setup */
/* Inertia tensor of a dynamic body in its frame: the principal moments of
 * body_inertia, or a hull's solid (hull_mass_props). */
static void body_tensor(const Body *b, double mass, double T[3][3]) {
    if (b->shape == ORA_HULL) {
        V c;
        double v;
        hull_mass_props(b->hull, mass, T, &c, &v);
        return;
    }
    double I[3];
    body_inertia(b->shape, b->prm, mass, I);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) T[i][j] = i == j ? I[i] : 0.0;
}

static void inv3(const double A[3][3], double Ai[3][3]) {
    double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                 A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    Ai[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
    Ai[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    Ai[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    Ai[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
    Ai[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    Ai[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    Ai[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
    Ai[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    Ai[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
}

static void load_bodies(const ora_model *m, const double *pose, const double *vel, int s, Body *B, const Hull *HL) {
    int b0 = m->body_offset[s], n = m->body_offset[s + 1] - b0;
    for (int k = 0; k < n; k++) {
        int g = b0 + k;
        Body *b = &B[k];
        b->shape = m->shape[g];
        b->motion = m->motion[g];
        b->x = mk(pose[7 * g], pose[7 * g + 1], pose[7 * g + 2]);
        for (int i = 0; i < 4; i++) b->q[i] = pose[7 * g + 3 + i];
        b->R = quat_R(b->q);
        for (int i = 0; i < 3; i++) b->prm[i] = m->param[3 * g + i];
        b->hull = NULL;
        if (b->shape == ORA_HULL) {
            b->hull = &HL[(int)m->param[3 * g]];
            for (int i = 0; i < 3; i++) b->prm[i] = b->hull->h[i];
        }
        b->v = mk(vel[6 * g], vel[6 * g + 1], vel[6 * g + 2]);
        b->w = mk(vel[6 * g + 3], vel[6 * g + 4], vel[6 * g + 5]);
        b->mu = m->friction[g];
        b->e = m->restitution[g];
        memset(&b->Iw, 0, sizeof(M3));
        b->im = 0;
        b->ncon = 0;
        if (b->motion == ORA_DYNAMIC) {
            double Ii[3][3];
            body_tensor(b, m->mass[g], b->Ib);
            inv3(b->Ib, Ii);
            b->im = 1.0 / m->mass[g];
            /* world inverse inertia R I^-1 R^T */
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    double sum = 0;
                    for (int k2 = 0; k2 < 3; k2++)
                        for (int k3 = 0; k3 < 3; k3++) sum += b->R.m[i][k2] * Ii[k2][k3] * b->R.m[j][k3];
                    b->Iw.m[i][j] = sum;
                }
        } else if (b->motion == ORA_STATIC) {
            b->v = mk(0, 0, 0);
            b->w = mk(0, 0, 0);
        }
    }
}

/* ------------------------------------------------------ container parts
 * Articulated furniture (Sec. 3: doors and drawers that turn about an axis
 * or slide): a part is one rigid body with one degree of freedom relative
 * to the world, a revolute joint about a fixed hinge line or a prismatic
 * one along a fixed axis, its coordinate q held within limits.  Its state is
 * q and the rate qd; the body's velocity is the one qd gives it (w = qd a,
 * v = w x (c - o) for a hinge; v = qd a for a slide).  An impulse P at p
 * changes qd by (a . ((p - o) x P)) / I_o (hinge; I_o its moment of inertia
 * about the hinge line) or (a . P) / m (slide). */
static void part_sync(Body *b) {   /* v, w from qd */
    if (b->joint == 1) {
        b->w = scl(b->ja, b->qd);
        b->v = cross(b->w, sub(b->x, b->jo));
    } else {
        b->v = scl(b->ja, b->qd);
        b->w = mk(0, 0, 0);
    }
}

/* Generalised impulse of an impulse P at point p on a part. */
static double part_gen(const Body *b, V p, V P) {
    return b->joint == 1 ? dot(b->ja, cross(sub(p, b->jo), P)) : dot(b->ja, P);
}

static void load_parts(const ora_model *m, const double *joint_state, int s, Body *B) {
    int b0 = m->body_offset[s], n = m->body_offset[s + 1] - b0;
    for (int k = 0; k < n; k++) {
        Body *b = &B[k];
        int g = b0 + k;
        b->joint = m->joint && b->motion == ORA_DYNAMIC ? m->joint[g] : 0;
        if (!b->joint) continue;
        b->ja = mk(m->joint_axis[3 * g], m->joint_axis[3 * g + 1], m->joint_axis[3 * g + 2]);
        b->jo = mk(m->joint_anchor[3 * g], m->joint_anchor[3 * g + 1], m->joint_anchor[3 * g + 2]);
        double mass = m->mass[g];
        if (b->joint == 1) {
            /* a^T I a about the centre (the axis in the body frame) plus the parallel-axis term */
            V al = mk(dot(col(&b->R, 0), b->ja), dot(col(&b->R, 1), b->ja), dot(col(&b->R, 2), b->ja));
            V d = cross(b->ja, sub(b->x, b->jo));
            double Ia = 0;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) Ia += comp(al, i) * b->Ib[i][j] * comp(al, j);
            b->jM = Ia + mass * len2(d);
        } else {
            b->jM = mass;
        }
        b->qd = joint_state[2 * g + 1];
        part_sync(b);
    }
}

/* ---------------------------------------------------------------- solver */
typedef struct {
    int a, b;               /* local body indices, b = -1 for the ground */
    uint32_t key;
    V n, t1, t2, p, ra, rb;
    double phi, mu, e, bias;
    double m[3], k[3];      /* effective mass and its inverse per row n, t1, t2 */
    double lam[3];
    double feat[16];
    int colour, matched;
    int active;             /* 0: every dynamic body of the contact sleeps (not solved) */
    int arm;                /* dynamic arm: +1 body a is a link, -1 body b is, 0 neither */
    double g[3][7], w[3][7];/* arm side of rows n, t1, t2: joint-space row g and M^-1 g */
} Con;

/* Orthonormal tangents from a unit normal (Duff et al. 2017, "Building an
 * Orthonormal Basis, Revisited").  Their construction has two branches, for
 * the upper and the lower hemisphere of normals; the branch is taken at
 * n.z = TAN_SPLIT instead of n.z = 0, so that the horizontal normals of
 * side-by-side contacts (frequent under gravity along z) lie far from the
 * switch.  Either branch is a valid basis wherever its denominator
 * sgn + n.z stays away from 0 (|sgn + n.z| >= 1/2 here). */
#define TAN_SPLIT (-0.5)
static void tangents(V n, V *t1, V *t2) {
    double sgn = n.z >= TAN_SPLIT ? 1.0 : -1.0;
    double a = -1.0 / (sgn + n.z);
    double b = n.x * n.y * a;
    *t1 = mk(1.0 + sgn * n.x * n.x * a, sgn * b, -sgn * n.x);
    *t2 = mk(b, sgn + n.y * n.y * a, -n.y);
}

static V bvel(const Body *B, int i, V r) {
    if (i < 0) return mk(0, 0, 0);
    return add(B[i].v, cross(B[i].w, r));
}

static V Mv(const M3 *M, V a) { return Rv(M, a); }

static double row_k(const Body *B, const Con *c, V d) {
    double k = 0;
    const Body *A = &B[c->a];
    if (A->joint) {   /* a part: the row's generalised direction over its joint mass */
        double gq = part_gen(A, c->p, d);
        k += gq * gq / A->jM;
    } else {
        V ca = cross(c->ra, d);
        k += A->im + dot(ca, Mv(&A->Iw, ca));
    }
    if (c->b >= 0) {
        const Body *Bb = &B[c->b];
        if (Bb->joint) {
            double gq = part_gen(Bb, c->p, d);
            k += gq * gq / Bb->jM;
        } else {
            V cb = cross(c->rb, d);
            k += Bb->im + dot(cb, Mv(&Bb->Iw, cb));
        }
    }
    return k;
}

/* Apply the impulse P (from B onto A; -P onto B) at the contact. */
static void apply(Body *B, const Con *c, V P) {
    Body *A = &B[c->a];
    if (A->joint) {
        A->qd += part_gen(A, c->p, P) / A->jM;
        part_sync(A);
    } else if (A->motion == ORA_DYNAMIC) {
        A->v = add(A->v, scl(P, A->im));
        A->w = add(A->w, Mv(&A->Iw, cross(c->ra, P)));
    }
    if (c->b >= 0) {
        Body *Bb = &B[c->b];
        if (Bb->joint) {
            Bb->qd -= part_gen(Bb, c->p, P) / Bb->jM;
            part_sync(Bb);
        } else if (Bb->motion == ORA_DYNAMIC) {
            Bb->v = sub(Bb->v, scl(P, Bb->im));
            Bb->w = sub(Bb->w, Mv(&Bb->Iw, cross(c->rb, P)));
        }
    }
}

/* Joint limits of the parts: per part a lower and an upper row on the rate
 * (direction +1, -1), with the contacts' speculative rule: a gap g > 0 to
 * the limit lets the rate close it within the step (target -g/dt), a
 * violation is pushed back at baumgarte/dt of it; impulses >= 0, started
 * from zero every step.  One Gauss-Seidel pass over the parts in body order;
 * returns max |dlambda| * (1/M). */
typedef struct { int body; double q, bias[2], lam[2]; } Limit;

static double limit_sweep(Body *B, Limit *Lm, int nl) {
    double R = 0;
    for (int k = 0; k < nl; k++) {
        Body *b = &B[Lm[k].body];
        for (int r = 0; r < 2; r++) {
            double sgn = r == 0 ? 1.0 : -1.0;
            double l = fmax(0.0, Lm[k].lam[r] + b->jM * (Lm[k].bias[r] - sgn * b->qd));
            double dl = l - Lm[k].lam[r];
            Lm[k].lam[r] = l;
            b->qd += sgn * dl / b->jM;
            part_sync(b);
            R = fmax(R, fabs(dl) / b->jM);
        }
    }
    return R;
}

static V vrel(const Body *B, const Con *c) {
    return sub(bvel(B, c->a, c->ra), bvel(B, c->b, c->rb));
}


/* ------------------------------------------------------------ dynamic arm
 * The dynamic arm (arm 2) is one articulated body in reduced coordinates
 * (Sec. 1: articulated robots; Sec. 5: joint motors with PD position
 * control).  Its state is the joint angles q (theta) and rates qd: the link
 * poses follow q by the forward kinematics and the link velocities follow
 * qd through the link Jacobians, so the joints hold exactly.  M(q), the
 * joint-space mass matrix, is the sum over links of Jv^T m Jv + Jw^T I Jw
 * (column i of link j's Jacobians: a_i x (c_j - o_i) and a_i for i <= j);
 * velocity-product (Coriolis) terms are left out, as the free bodies'
 * gyroscopic term is.  Gravity adds dt M^-1 tau_g to qd.  A contact row d
 * at point p on link j acts on the arm through g_i = d . (a_i x (p - o_i))
 * (i <= j): the arm adds g . qd to the row's velocity and an impulse l
 * changes qd by l M^-1 g.  Motor k is the row e_k: velocity qd_k, target
 * Kp (target_k - q_k) / dt (the error wrapped into [-pi, pi]), effective
 * mass 1 / (M^-1)_kk, impulse bounded by the motor's largest impulse per
 * step.  Motors are solved after the contacts in every sweep, joints 0..6
 * in order, and warm-start from their last impulses. */
typedef struct {
    double q[7], qd[7];
    V o[7], ax[7], c[7];          /* joint origins and axes, link centres (world) */
    double Mi[7][7];              /* M^-1 */
    double lam[7], bias[7], lim;  /* motor rows */
    int l0;                       /* local index of link 0 */
} Arm;

/* M^-1 of the arm at its current links: M from the link Jacobians, then
 * its Cholesky factor, then the inverse column by column. */
static void arm_mass(const ora_model *m, const Body *B, int g0, Arm *A) {
    double M[7][7] = {{0}};
    for (int j = 0; j < 7; j++) {
        const Body *L = &B[A->l0 + j];
        double mass = m->mass[g0 + A->l0 + j], Ip[3];
        body_inertia(ORA_CAPSULE, L->prm, mass, Ip);
        M3 Iw;   /* world inertia R diag(Ip) R^T */
        for (int r = 0; r < 3; r++)
            for (int q = 0; q < 3; q++) {
                double sum = 0;
                for (int k = 0; k < 3; k++) sum += L->R.m[r][k] * Ip[k] * L->R.m[q][k];
                Iw.m[r][q] = sum;
            }
        V jv[7], jw[7];
        for (int i = 0; i <= j; i++) { jw[i] = A->ax[i]; jv[i] = cross(A->ax[i], sub(A->c[j], A->o[i])); }
        for (int i = 0; i <= j; i++)
            for (int k = 0; k <= j; k++) M[i][k] += mass * dot(jv[i], jv[k]) + dot(jw[i], Mv(&Iw, jw[k]));
    }
    double Lc[7][7] = {{0}};
    for (int i = 0; i < 7; i++)
        for (int k = 0; k <= i; k++) {
            double sum = M[i][k];
            for (int t = 0; t < k; t++) sum -= Lc[i][t] * Lc[k][t];
            Lc[i][k] = i == k ? sqrt(sum) : sum / Lc[k][k];
        }
    for (int col_ = 0; col_ < 7; col_++) {
        double y[7], x[7];
        for (int i = 0; i < 7; i++) {
            double sum = i == col_ ? 1.0 : 0.0;
            for (int t = 0; t < i; t++) sum -= Lc[i][t] * y[t];
            y[i] = sum / Lc[i][i];
        }
        for (int i = 6; i >= 0; i--) {
            double sum = y[i];
            for (int t = i + 1; t < 7; t++) sum -= Lc[t][i] * x[t];
            x[i] = sum / Lc[i][i];
        }
        for (int i = 0; i < 7; i++) A->Mi[i][col_] = x[i];
    }
}

static void arm_add(Arm *A, const double *w, double l) {
    for (int i = 0; i < 7; i++) A->qd[i] += l * w[i];
}

static double dot7(const double *a, const double *b) {
    double s = 0;
    for (int i = 0; i < 7; i++) s += a[i] * b[i];
    return s;
}

/* Joint-space rows of contact c's directions on its arm link, and M^-1 of them. */
static void arm_contact_rows(const Arm *A, Con *c) {
    int j = (c->arm > 0 ? c->a : c->b) - A->l0;
    V d[3] = {c->n, c->t1, c->t2};
    for (int r = 0; r < 3; r++) {
        for (int i = 0; i < 7; i++) c->g[r][i] = i <= j ? dot(d[r], cross(A->ax[i], sub(c->p, A->o[i]))) : 0.0;
        for (int i = 0; i < 7; i++) c->w[r][i] = dot7(A->Mi[i], c->g[r]);
    }
}

/* Velocity of row r of contact c, the arm's part included. */
static double row_u(const Body *B, const Arm *A, const Con *c, int r) {
    V d = r == 0 ? c->n : (r == 1 ? c->t1 : c->t2);
    double u = dot(d, vrel(B, c));
    if (c->arm) u += c->arm * dot7(c->g[r], A->qd);
    return u;
}

/* Impulse l along row r of contact c (the bodies' part by apply). */
static void row_apply(Body *B, Arm *A, const Con *c, int r, double l) {
    V d = r == 0 ? c->n : (r == 1 ? c->t1 : c->t2);
    apply(B, c, scl(d, l));
    if (c->arm) arm_add(A, c->w[r], c->arm * l);
}

/* One Gauss-Seidel pass over the motor rows; returns max |dlambda| * k. */
static double motor_sweep(Arm *A) {
    double R = 0;
    for (int k = 0; k < 7; k++) {
        double kk = A->Mi[k][k];
        double l = A->lam[k] + (A->bias[k] - A->qd[k]) / kk;
        l = fmin(fmax(l, -A->lim), A->lim);
        double dl = l - A->lam[k];
        A->lam[k] = l;
        for (int i = 0; i < 7; i++) A->qd[i] += dl * A->Mi[i][k];
        R = fmax(R, fabs(dl) * kk);
    }
    return R;
}

/* Projection of the friction impulse onto the disk of radius mu*lambda_n. */
static void proj_disk(double *l1, double *l2, double lim) {
    double L = sqrt(*l1 * *l1 + *l2 * *l2);
    if (L > lim) {
        if (L > 0) { double f = lim / L; *l1 *= f; *l2 *= f; }
        else { *l1 = 0; *l2 = 0; }
    }
}

static void project(Con *c) {
    if (c->lam[0] < 0) c->lam[0] = 0;
    proj_disk(&c->lam[1], &c->lam[2], c->mu * c->lam[0]);
}

/* One projected Gauss-Seidel sweep in colour-major order.  Rows of one
 * contact: the normal row, then both friction rows from the velocities that
 * follow the normal update.  Returns the sweep residual max |dlambda|*k. */
static double pgs_sweep(Body *B, Arm *A, Con *C, const int *order, int nc) {
    double R = 0;
    for (int q = 0; q < nc; q++) {
        Con *c = &C[order[q]];
        double u = row_u(B, A, c, 0);
        double ln = fmax(0.0, c->lam[0] + c->m[0] * (c->bias - u));
        double dn = ln - c->lam[0];
        c->lam[0] = ln;
        row_apply(B, A, c, 0, dn);
        double l1 = c->lam[1] - c->m[1] * row_u(B, A, c, 1);
        double l2 = c->lam[2] - c->m[2] * row_u(B, A, c, 2);
        proj_disk(&l1, &l2, c->mu * ln);
        double d1 = l1 - c->lam[1], d2 = l2 - c->lam[2];
        c->lam[1] = l1; c->lam[2] = l2;
        apply(B, c, add(scl(c->t1, d1), scl(c->t2, d2)));
        if (c->arm) {
            arm_add(A, c->w[1], c->arm * d1);
            arm_add(A, c->w[2], c->arm * d2);
        }
        R = fmax(R, fabs(dn) * c->k[0]);
        R = fmax(R, fabs(d1) * c->k[1]);
        R = fmax(R, fabs(d2) * c->k[2]);
    }
    return R;
}

/* One Jacobi sweep: every row reads the velocities of the start of the
 * sweep; each increment is divided by max(n_A, n_B) (contacts per dynamic
 * body), projected, then all impulses are applied. */
static double jacobi_sweep(Body *B, int nb, Con *C, const int *order, int nc) {
    V *v0 = malloc(sizeof(V) * nb * 2);
    for (int i = 0; i < nb; i++) { v0[2 * i] = B[i].v; v0[2 * i + 1] = B[i].w; }
    double R = 0;
    double *dl = malloc(sizeof(double) * 3 * (nc ? nc : 1));
    for (int q = 0; q < nc; q++) {
        Con *c = &C[order[q]];
        V va = add(v0[2 * c->a], cross(v0[2 * c->a + 1], c->ra));
        V vb = c->b >= 0 ? add(v0[2 * c->b], cross(v0[2 * c->b + 1], c->rb)) : mk(0, 0, 0);
        V vr = sub(va, vb);
        int na = B[c->a].motion == ORA_DYNAMIC ? B[c->a].ncon : 0;
        int nbb = (c->b >= 0 && B[c->b].motion == ORA_DYNAMIC) ? B[c->b].ncon : 0;
        double sc = 1.0 / (double)(na > nbb ? na : nbb);
        double ln = fmax(0.0, c->lam[0] + sc * c->m[0] * (c->bias - dot(c->n, vr)));
        double l1 = c->lam[1] - sc * c->m[1] * dot(c->t1, vr);
        double l2 = c->lam[2] - sc * c->m[2] * dot(c->t2, vr);
        proj_disk(&l1, &l2, c->mu * ln);
        dl[3 * q] = ln - c->lam[0];
        dl[3 * q + 1] = l1 - c->lam[1];
        dl[3 * q + 2] = l2 - c->lam[2];
        c->lam[0] = ln; c->lam[1] = l1; c->lam[2] = l2;
    }
    for (int q = 0; q < nc; q++) {
        Con *c = &C[order[q]];
        apply(B, c, scl(c->n, dl[3 * q]));
        apply(B, c, add(scl(c->t1, dl[3 * q + 1]), scl(c->t2, dl[3 * q + 2])));
        R = fmax(R, fabs(dl[3 * q]) * c->k[0]);
        R = fmax(R, fabs(dl[3 * q + 1]) * c->k[1]);
        R = fmax(R, fabs(dl[3 * q + 2]) * c->k[2]);
    }
    free(dl);
    free(v0);
    return R;
}

/* ---------------------------------------------------------------- MLP */
double ora_bf16(double x) {
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;      /* inf / nan unchanged */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double qz(const ora_mlp *net, double x) { return net->bf16 ? ora_bf16(x) : x; }

/* Forward pass of one row; keeps the layer activations for backward. */
static void mlp_row(const ora_mlp *net, const double *x, double *z0, double *a1, double *a2, double *y) {
    for (int i = 0; i < 16; i++) {
        double sd = net->std[i] > 1e-6 ? net->std[i] : 1e-6;
        z0[i] = qz(net, (x[i] - net->mean[i]) / sd);
    }
    for (int o = 0; o < 64; o++) {
        double s = 0;
        for (int i = 0; i < 16; i++) s += qz(net, net->w1[16 * o + i]) * z0[i];
        s += net->b1[o];
        a1[o] = s > 0 ? s : 0;
    }
    for (int o = 0; o < 64; o++) a1[o] = qz(net, a1[o]);
    for (int o = 0; o < 64; o++) {
        double s = 0;
        for (int i = 0; i < 64; i++) s += qz(net, net->w2[64 * o + i]) * a1[i];
        s += net->b2[o];
        a2[o] = s > 0 ? s : 0;
    }
    for (int o = 0; o < 64; o++) a2[o] = qz(net, a2[o]);
    for (int o = 0; o < 3; o++) {
        double s = 0;
        for (int i = 0; i < 64; i++) s += qz(net, net->w3[64 * o + i]) * a2[i];
        y[o] = s + net->b3[o];
    }
}

void ora_mlp_forward(const ora_mlp *net, const double *x, int n, double *y) {
    double z0[16], a1[64], a2[64];
    for (int r = 0; r < n; r++) mlp_row(net, x + 16 * r, z0, a1, a2, y + 3 * r);
}

double ora_mlp_loss_grad(const ora_mlp *net, const double *x, const double *t, int n,
                         double *gw1, double *gb1, double *gw2, double *gb2,
                         double *gw3, double *gb3) {
    memset(gw1, 0, sizeof(double) * 64 * 16); memset(gb1, 0, sizeof(double) * 64);
    memset(gw2, 0, sizeof(double) * 64 * 64); memset(gb2, 0, sizeof(double) * 64);
    memset(gw3, 0, sizeof(double) * 3 * 64);  memset(gb3, 0, sizeof(double) * 3);
    double loss = 0, z0[16], a1[64], a2[64], y[3], dy[3], d2[64], d1[64];
    double inv = 1.0 / (3.0 * n);
    for (int r = 0; r < n; r++) {
        mlp_row(net, x + 16 * r, z0, a1, a2, y);
        for (int o = 0; o < 3; o++) {
            double e = y[o] - t[3 * r + o];
            loss += e * e * inv;
            dy[o] = 2.0 * e * inv;
            gb3[o] += dy[o];
            for (int i = 0; i < 64; i++) gw3[64 * o + i] += dy[o] * a2[i];
        }
        for (int i = 0; i < 64; i++) {
            double s = 0;
            for (int o = 0; o < 3; o++) s += qz(net, net->w3[64 * o + i]) * dy[o];
            d2[i] = a2[i] > 0 ? s : 0;
        }
        for (int o = 0; o < 64; o++) {
            gb2[o] += d2[o];
            for (int i = 0; i < 64; i++) gw2[64 * o + i] += d2[o] * a1[i];
        }
        for (int i = 0; i < 64; i++) {
            double s = 0;
            for (int o = 0; o < 64; o++) s += qz(net, net->w2[64 * o + i]) * d2[o];
            d1[i] = a1[i] > 0 ? s : 0;
        }
        for (int o = 0; o < 64; o++) {
            gb1[o] += d1[o];
            for (int i = 0; i < 16; i++) gw1[16 * o + i] += d1[o] * z0[i];
        }
    }
    return loss;
}

/* ---------------------------------------------------------------- step */

static int lookup(const ora_cache *cache, int s, uint32_t key) {
    if (!cache) return -1;
    const uint32_t *k = cache->key + (size_t)s * cache->cap;
    int lo = 0, hi = cache->count[s] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (k[mid] == key) return mid;
        if (k[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static int finite3(V a) { return isfinite(a.x) && isfinite(a.y) && isfinite(a.z); }


/* Sweeps until the residual reaches tol (tol > 0) or iters sweeps ran.
 * *gap receives the smallest |R - tol| / tol over the sweeps whose residual
 * was tested against the tolerance (infinity when none was): how close the
 * stopping decision came to going the other way. */
static int solve(Body *B, int nb, Arm *A, Limit *Lm, int nl, Con *C, const int *order, int nc, int iters,
                 double tol, int solver, double *res, double *gap) {
    int sw = 0;
    double R = 0;
    *gap = INFINITY;
    for (int it = 0; it < iters; it++) {
        R = solver == ORA_JACOBI ? jacobi_sweep(B, nb, C, order, nc) : pgs_sweep(B, A, C, order, nc);
        if (A) R = fmax(R, motor_sweep(A));
        if (nl) R = fmax(R, limit_sweep(B, Lm, nl));
        sw++;
        if (tol > 0) *gap = fmin(*gap, fabs(R - tol) / tol);
        if (tol > 0 && R <= tol) break;
    }
    *res = R;
    return sw;
}

/* Change of the solver's quadratic objective f(l) = 1/2 l^T A l +
 * l^T (u_free - b) when the network's start impulses of the new contacts,
 * l_n, are added to the persisting contacts' previous impulses l_p:
 * f(l_p + l_n) - f(l_p) = sum over the new contacts' rows of the impulse
 * times (the mean of the row velocity before and after l_n was applied)
 * minus the row's target velocity (the bias for the normal row, zero for
 * the friction rows); vs holds the velocities before l_n was applied. */
static double start_objective(const Body *B, const Con *C, int nc, const V *vs) {
    double f = 0;
    for (int q = 0; q < nc; q++) {
        const Con *c = &C[q];
        if (c->matched || !c->active) continue;
        V va = add(vs[2 * c->a], cross(vs[2 * c->a + 1], c->ra));
        V vb = c->b >= 0 ? add(vs[2 * c->b], cross(vs[2 * c->b + 1], c->rb)) : mk(0, 0, 0);
        V v0 = sub(va, vb), v1 = vrel(B, c);
        f += c->lam[0] * (0.5 * (dot(c->n, v0) + dot(c->n, v1)) - c->bias);
        f += c->lam[1] * 0.5 * (dot(c->t1, v0) + dot(c->t1, v1));
        f += c->lam[2] * 0.5 * (dot(c->t2, v0) + dot(c->t2, v1));
    }
    return f;
}

/* Applies the start impulses in solver order (sel < 0), or only those of
 * the persisting (sel 0) or new (sel 1) contacts. */
static void warm_apply(Body *B, Arm *A, Con *C, const int *order, int nc, int sel) {
    for (int q = 0; q < nc; q++) {
        Con *c = &C[order[q]];
        if (sel >= 0 && (c->matched ? 0 : 1) != sel) continue;
        project(c);
        apply(B, c, add(scl(c->n, c->lam[0]), add(scl(c->t1, c->lam[1]), scl(c->t2, c->lam[2]))));
        if (c->arm)
            for (int r = 0; r < 3; r++) arm_add(A, c->w[r], c->arm * c->lam[r]);
    }
}

/* Bounding radius of a body about its centre: the lever arm that turns an
 * angular speed into the largest surface speed. */
static double bound_radius(const Body *b) {
    if (b->shape == ORA_SPHERE) return b->prm[0];
    if (b->shape == ORA_BOX || b->shape == ORA_HULL)   /* a hull: its bounding box's half-diagonal */
        return sqrt(b->prm[0] * b->prm[0] + b->prm[1] * b->prm[1] + b->prm[2] * b->prm[2]);
    return b->prm[0] + b->prm[1];
}

static int uf_find(int *par, int x) {
    while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
    return x;
}

static void step_scene(const ora_model *m, double *pose, double *vel, double *theta, int32_t *rest,
                       double *arm_state, double *joint_state, ora_cache *cache, const double *actions, double dt, int iters,
                       double tol, int warm, int solver, const ora_mlp *mlp, ora_out *out, int s) {
    int b0 = m->body_offset[s], nb = m->body_offset[s + 1] - b0;
    int flags = 0, amb = 0;
    double margin = m->margin;
    V g = mk(m->gravity[0], m->gravity[1], m->gravity[2]);
    double gmag = sqrt(len2(g));

    /* 1. arm: poses at theta_t, link velocities from the joint velocities */
    double thd[7] = {0};
    V ao[7], aax[7];
    if (m->arm && actions) for (int k = 0; k < 7; k++) thd[k] = actions[7 * s + k];
    if (m->arm == 1) {
        double lp[7][7];
        arm_fk(m, m->arm_base + 3 * s, theta + 7 * s, lp, ao, aax);
        for (int k = 0; k < 7; k++) {
            int gi = b0 + nb - 7 + k;
            memcpy(pose + 7 * gi, lp[k], 7 * sizeof(double));
            V c = mk(lp[k][0], lp[k][1], lp[k][2]);
            V w = mk(0, 0, 0), v = mk(0, 0, 0);
            for (int j = 0; j <= k; j++) {
                w = add(w, scl(aax[j], thd[j]));
                v = add(v, scl(cross(aax[j], sub(c, ao[j])), thd[j]));
            }
            vel[6 * gi] = v.x; vel[6 * gi + 1] = v.y; vel[6 * gi + 2] = v.z;
            vel[6 * gi + 3] = w.x; vel[6 * gi + 4] = w.y; vel[6 * gi + 5] = w.z;
        }
    }
    double *ast = m->arm == 2 ? arm_state + 21 * s : NULL;   /* qd, target, motor impulses */
    if (m->arm == 2) {
        /* the motor targets move at the commanded rates; links at q_t */
        for (int k = 0; k < 7; k++) ast[7 + k] += dt * thd[k];
        double lp[7][7];
        arm_fk(m, m->arm_base + 3 * s, theta + 7 * s, lp, ao, aax);
        for (int k = 0; k < 7; k++) memcpy(pose + 7 * (b0 + nb - 7 + k), lp[k], 7 * sizeof(double));
    }
    Body *B = malloc(sizeof(Body) * (nb ? nb : 1));
    Hull *HL = hulls_of(m);
    load_bodies(m, pose, vel, s, B, HL);
    for (int i = 0; i < nb; i++) B[i].joint = 0;
    if (m->joint) load_parts(m, joint_state, s, B);
    Arm AR;
    if (m->arm == 2) {
        AR.l0 = nb - 7;
        for (int k = 0; k < 7; k++) {
            Body *L = &B[AR.l0 + k];
            L->motion = ORA_ARMLINK;
            L->im = 0;
            memset(&L->Iw, 0, sizeof(M3));
            L->v = mk(0, 0, 0);
            L->w = mk(0, 0, 0);
            AR.q[k] = theta[7 * s + k];
            AR.qd[k] = ast[k];
            AR.o[k] = ao[k];
            AR.ax[k] = aax[k];
            AR.c[k] = L->x;
        }
        arm_mass(m, B, b0, &AR);
    }

    /* 2. velocity integration (no gyroscopic term; the arm: dt M^-1 tau_g) */
    for (int i = 0; i < nb; i++) {
        if (B[i].joint) {   /* a part: the gravity moment (force) about its joint over its joint mass */
            B[i].qd += dt * part_gen(&B[i], B[i].x, scl(g, m->mass[b0 + i])) / B[i].jM;
            part_sync(&B[i]);
        } else if (B[i].motion == ORA_DYNAMIC) {
            B[i].v = add(B[i].v, scl(g, dt));
        }
    }
    if (m->arm == 2) {
        double tg[7];
        for (int i = 0; i < 7; i++) {
            V t = mk(0, 0, 0);
            for (int j = i; j < 7; j++) t = add(t, cross(sub(AR.c[j], AR.o[i]), scl(g, m->mass[b0 + AR.l0 + j])));
            tg[i] = dot(AR.ax[i], t);
        }
        for (int i = 0; i < 7; i++) AR.qd[i] += dt * dot7(AR.Mi[i], tg);
    }

    /* 3. AABBs; 4. pairs */
    for (int i = 0; i < nb; i++) body_aabb(&B[i], margin);
    int maxp = nb * (nb + 1) / 2 + 1;
    uint32_t *pk = malloc(sizeof(uint32_t) * maxp);
    uint8_t *tied = calloc((size_t)(nb ? nb : 1), 1);
    const int arm0 = m->arm == 2 ? nb - 7 : nb;   /* first link of the dynamic arm */
    int np = brute_pairs(B, nb, arm0, m->joint_parent ? m->joint_parent + b0 : NULL, pk, maxp, &amb, tied);

    /* 5. narrowphase in canonical pair order; 6. contact list */
    int capc = 4 * np + 1;
    Con *C = calloc(capc, sizeof(Con));
    int nc = 0;
    for (int q = 0; q < np; q++) {
        int a = pk[q] >> 16, b = pk[q] & 0xFFFF;
        int ground = b == PAIR_GROUND;
        Geom GA, GB;
        GA.shape = B[a].shape; GA.x = B[a].x; GA.R = B[a].R; GA.hull = B[a].hull;
        memcpy(GA.prm, B[a].prm, sizeof GA.prm);
        PC pc[4];
        int k, amb0 = amb;
        if (ground) k = ground_contacts(&GA, margin, pc, &amb);
        else {
            GB.shape = B[b].shape; GB.x = B[b].x; GB.R = B[b].R; GB.hull = B[b].hull;
            memcpy(GB.prm, B[b].prm, sizeof GB.prm);
            k = collide(&GA, &GB, margin, pc, &amb);
        }
        if (amb != amb0) {
            tied[a] = 1;
            if (!ground) tied[b] = 1;
        }
        for (int i = 0; i < k; i++) {
            Con *c = &C[nc++];
            c->a = a;
            c->b = ground ? -1 : b;
            c->key = ((uint32_t)a << 20) | ((uint32_t)(ground ? KEY_GROUND : b) << 8) | (uint32_t)pc[i].f;
            c->n = pc[i].n; c->p = pc[i].p; c->phi = pc[i].phi;
        }
    }

    /* Sleeping (localized physics, Sec. 4.1): an island is a set of dynamic
     * bodies joined by this step's contacts between two dynamic bodies.  It
     * sleeps when every body in it has been at rest for sleep_steps steps
     * and none of them touches a kinematic body (the arm: the robot is the
     * only source of forces other than gravity).  A sleeping body keeps its
     * pose, has zero velocity and counts as not dynamic for the solver: its
     * contacts are neither coloured nor solved and carry their previous
     * impulses into the cache. */
    const int sleeping = m->sleep_speed > 0 && m->sleep_steps > 0 && rest != NULL;
    uint8_t *asleep = calloc((size_t)(nb ? nb : 1), 1);
    for (int q = 0; q < nc; q++) C[q].active = 1;
    if (sleeping) {
        int *par = malloc(sizeof(int) * (nb ? nb : 1));
        uint8_t *wake = calloc((size_t)(nb ? nb : 1), 1);
        for (int i = 0; i < nb; i++) par[i] = i;
        for (int q = 0; q < nc; q++) {
            int a = C[q].a, b = C[q].b;
            if (b < 0 || B[a].motion != ORA_DYNAMIC || B[b].motion != ORA_DYNAMIC) continue;
            int ra = uf_find(par, a), rb = uf_find(par, b);
            if (ra != rb) par[ra < rb ? rb : ra] = ra < rb ? ra : rb;
        }
        for (int i = 0; i < nb; i++)
            if (B[i].motion == ORA_DYNAMIC && (rest[b0 + i] < m->sleep_steps || B[i].joint)) wake[uf_find(par, i)] = 1;
        for (int q = 0; q < nc; q++) {
            int a = C[q].a, b = C[q].b;
            if (b < 0) continue;
            int ka = B[a].motion == ORA_KINEMATIC || B[a].motion == ORA_ARMLINK;
            int kb = B[b].motion == ORA_KINEMATIC || B[b].motion == ORA_ARMLINK;
            if (ka && B[b].motion == ORA_DYNAMIC) wake[uf_find(par, b)] = 1;
            if (kb && B[a].motion == ORA_DYNAMIC) wake[uf_find(par, a)] = 1;
        }
        for (int i = 0; i < nb; i++) {
            if (B[i].motion != ORA_DYNAMIC || wake[uf_find(par, i)]) continue;
            asleep[i] = 1;
            B[i].v = mk(0, 0, 0);
            B[i].w = mk(0, 0, 0);
        }
        for (int q = 0; q < nc; q++) {
            int a = C[q].a, b = C[q].b;
            int awake_a = B[a].motion == ORA_DYNAMIC && !asleep[a];
            int awake_b = b >= 0 && B[b].motion == ORA_DYNAMIC && !asleep[b];
            int on_arm = B[a].motion == ORA_ARMLINK || (b >= 0 && B[b].motion == ORA_ARMLINK);
            C[q].active = awake_a || awake_b || on_arm;
        }
        free(wake);
        free(par);
    }
#define AWAKE(i) ((i) >= 0 && B[i].motion == ORA_DYNAMIC && !asleep[i])

    /* 7. setup; contacts per awake dynamic body first (a feature of new contacts) */
    int *ndyn = calloc((size_t)(nb ? nb : 1), sizeof(int));
    for (int q = 0; q < nc; q++) {
        if (AWAKE(C[q].a)) ndyn[C[q].a]++;
        if (AWAKE(C[q].b)) ndyn[C[q].b]++;
    }
    for (int q = 0; q < nc; q++) {
        Con *c = &C[q];
        Body *A = &B[c->a];
        double mub = c->b >= 0 ? B[c->b].mu : m->ground_friction;
        double eb = c->b >= 0 ? B[c->b].e : m->ground_restitution;
        c->mu = sqrt(A->mu * mub);
        c->e = fmax(A->e, eb);
        c->ra = sub(c->p, A->x);
        c->rb = c->b >= 0 ? sub(c->p, B[c->b].x) : mk(0, 0, 0);
        tangents(c->n, &c->t1, &c->t2);
        if (fabs(c->n.z - TAN_SPLIT) < BAND_DIM) {     /* the basis branch is a decision */
            amb++;
            tied[c->a] = 1;
            if (c->b >= 0) tied[c->b] = 1;
        }
        c->arm = m->arm == 2 ? (c->a >= arm0 ? 1 : (c->b >= arm0 ? -1 : 0)) : 0;
        if (c->arm) arm_contact_rows(&AR, c);
        c->k[0] = row_k(B, c, c->n);
        c->k[1] = row_k(B, c, c->t1);
        c->k[2] = row_k(B, c, c->t2);
        if (c->arm)
            for (int r = 0; r < 3; r++) c->k[r] += dot7(c->g[r], c->w[r]);
        for (int r = 0; r < 3; r++) c->m[r] = 1.0 / c->k[r];
        V vr = vrel(B, c);
        if (c->arm)   /* the arm link's point velocity, in the contact frame */
            vr = add(vr, add(scl(c->n, c->arm * dot7(c->g[0], AR.qd)),
                             add(scl(c->t1, c->arm * dot7(c->g[1], AR.qd)), scl(c->t2, c->arm * dot7(c->g[2], AR.qd)))));
        double u0 = dot(c->n, vr);
        if (c->phi > 0) c->bias = -c->phi / dt;
        else c->bias = m->baumgarte / dt * fmax(0.0, -c->phi - m->slop);
        if (c->e > 0 && u0 < -m->rest_thresh) c->bias = fmax(c->bias, -c->e * u0);
        /* previous impulse (friction re-projected on the new tangents) */
        int hit = lookup(cache, s, c->key);
        double lp[3] = {0, 0, 0};
        if (hit >= 0) {
            const double *L = cache->lam + 4 * ((size_t)s * cache->cap + hit);
            V F = mk(L[1], L[2], L[3]);
            lp[0] = L[0]; lp[1] = dot(F, c->t1); lp[2] = dot(F, c->t2);
        }
        c->matched = hit >= 0;
        double *f = c->feat;
        f[0] = u0; f[1] = dot(c->t1, vr); f[2] = dot(c->t2, vr);
        f[3] = -c->phi;
        f[4] = A->im; f[5] = c->b >= 0 ? B[c->b].im : 0;
        V can = cross(c->ra, c->n);
        f[6] = dot(can, Mv(&A->Iw, can));
        if (c->b >= 0) { V cbn = cross(c->rb, c->n); f[7] = dot(cbn, Mv(&B[c->b].Iw, cbn)); }
        else f[7] = 0;
        /* previous impulses in units of |g| dt / k_n (the impulse that
         * cancels one step of gravity along the normal; 1 m/s^2 stands in for
         * |g| when gravity is off), the units of the network's outputs */
        double unit = (gmag > 0 ? gmag : 1.0) * dt * c->m[0];
        f[8] = lp[0] / unit; f[9] = lp[1] / unit; f[10] = lp[2] / unit;
        f[11] = c->n.x; f[12] = c->n.y; f[13] = c->n.z;
        f[14] = c->mu;
        /* new contact: its share 1 / max(n_A, n_B) of the busier body's
         * contacts (the impulse that stops a body splits over them); a
         * persisting contact: 0 */
        {
            int na = ndyn[c->a], nbc = c->b >= 0 ? ndyn[c->b] : 0;
            int mx = na > nbc ? na : nbc;
            f[15] = c->matched ? 0.0 : 1.0 / (double)(mx > 1 ? mx : 1);
        }
        c->lam[0] = c->lam[1] = c->lam[2] = 0;
        if (warm == ORA_PREV) { c->lam[0] = lp[0]; c->lam[1] = lp[1]; c->lam[2] = lp[2]; }
        else if (warm == ORA_LEARNED && mlp) {
            double y[3];
            ora_mlp_forward(mlp, f, 1, y);
            /* a persisting contact keeps its previous impulse (the classic
             * warm start); the network predicts the impulse of a new contact,
             * in units of |g| dt / k_n */
            double sc = gmag * dt * c->m[0];
            for (int r = 0; r < 3; r++) c->lam[r] = c->matched ? lp[r] : y[r] * sc;
        }
        if (!c->active) { c->lam[0] = lp[0]; c->lam[1] = lp[1]; c->lam[2] = lp[2]; }
    }

    free(ndyn);

    /* 9. colouring: first fit in canonical order; only dynamic bodies
     * conflict, and the dynamic arm as one body (slot nb: its contacts all
     * move the same joint rates) */
    uint64_t *used = calloc((size_t)(nb + 1) * (MAXCOL / 64), sizeof(uint64_t));
    int ncol = 0;
    for (int q = 0; q < nc; q++) {
        Con *c = &C[q];
        if (!c->active) { c->colour = -1; continue; }
        int ids[3] = {AWAKE(c->a) ? c->a : -1, AWAKE(c->b) ? c->b : -1, c->arm ? nb : -1};
        uint64_t mask[MAXCOL / 64] = {0};
        for (int t = 0; t < 3; t++) {
            int i = ids[t];
            if (i < 0) continue;
            for (int w = 0; w < MAXCOL / 64; w++) mask[w] |= used[(size_t)i * (MAXCOL / 64) + w];
        }
        int col_ = -1;
        for (int k = 0; k < MAXCOL; k++) if (!((mask[k / 64] >> (k % 64)) & 1)) { col_ = k; break; }
        if (col_ < 0) { flags |= ORA_F_CAPACITY; col_ = MAXCOL - 1; }
        c->colour = col_;
        if (col_ + 1 > ncol) ncol = col_ + 1;
        for (int t = 0; t < 3; t++) {
            int i = ids[t];
            if (i < 0) continue;
            used[(size_t)i * (MAXCOL / 64) + col_ / 64] |= 1ull << (col_ % 64);
            if (i < nb) B[i].ncon++;
        }
    }
    free(used);
    int *order = malloc(sizeof(int) * (nc ? nc : 1));
    int nact = 0;
    for (int k = 0; k < ncol; k++)
        for (int q = 0; q < nc; q++) if (C[q].colour == k) order[nact++] = q;

    /* 8. initial impulses, 10. sweeps */
    V *vsave = malloc(sizeof(V) * 2 * (nb ? nb : 1));
    /* Learned start: the persisting contacts' previous impulses first, then
     * the network's impulses of the new contacts.  The plain solver judges
     * the network's part before any sweep: if it raises the solver's
     * objective it is dropped (new contacts start from zero, the classic
     * warm start) and the step is flagged. */
    Arm *AP = m->arm == 2 ? &AR : NULL;
    if (warm == ORA_LEARNED) {
        warm_apply(B, AP, C, order, nact, 0);
        for (int i = 0; i < nb; i++) { vsave[2 * i] = B[i].v; vsave[2 * i + 1] = B[i].w; }
        warm_apply(B, AP, C, order, nact, 1);
        if (start_objective(B, C, nc, vsave) > 0) {
            flags |= ORA_F_FELLBACK;
            for (int i = 0; i < nb; i++) { B[i].v = vsave[2 * i]; B[i].w = vsave[2 * i + 1]; }
            for (int q = 0; q < nc; q++)
                if (!C[q].matched && C[q].active) C[q].lam[0] = C[q].lam[1] = C[q].lam[2] = 0;
        }
    } else {
        warm_apply(B, AP, C, order, nact, -1);
    }
    if (AP) {   /* motor rows: targets, bound, warm start from the last impulses */
        AR.lim = m->motor_max;
        for (int k = 0; k < 7; k++) {
            double err = remainder(ast[7 + k] - AR.q[k], 2.0 * M_PI);
            if (fabs(fabs(err) - M_PI) < BAND_DIM) { amb++; tied[AR.l0 + k] = 1; }
            AR.bias[k] = m->motor_kp * err / dt;
            AR.lam[k] = warm == ORA_COLD ? 0.0 : fmin(fmax(ast[14 + k], -AR.lim), AR.lim);
            for (int i = 0; i < 7; i++) AR.qd[i] += AR.lam[k] * AR.Mi[i][k];
        }
    }
    /* joint limits of the parts (the gap to each limit at the step's q) */
    Limit *Lm = malloc(sizeof(Limit) * (nb ? nb : 1));
    int nl = 0;
    for (int i = 0; i < nb; i++) {
        if (!B[i].joint) continue;
        Limit *l = &Lm[nl++];
        int gi = b0 + i;
        l->body = i;
        l->q = joint_state[2 * gi];
        double gaps[2] = {l->q - m->joint_limits[2 * gi], m->joint_limits[2 * gi + 1] - l->q};
        for (int r = 0; r < 2; r++) {
            l->bias[r] = gaps[r] > 0 ? -gaps[r] / dt : m->baumgarte / dt * (-gaps[r]);
            l->lam[r] = 0;
        }
    }
    double R = 0, gap = INFINITY;
    int sweeps = solve(B, nb, AP, Lm, nl, C, order, nact, iters, tol, solver, &R, &gap);
    /* a step counts as solved only once its residual reached the tolerance */
    if (tol > 0 && R > tol) flags |= ORA_F_NOT_CONVERGED;
    free(vsave);

    /* 11. position integration; arm joint update */
    for (int i = 0; i < nb; i++) {
        Body *b = &B[i];
        if (b->motion != ORA_DYNAMIC) continue;
        int gi0 = b0 + i;
        if (asleep[i]) {             /* pose kept, velocity zero, counter kept */
            for (int k = 0; k < 6; k++) vel[6 * gi0 + k] = 0.0;
            continue;
        }
        if (sleeping) {              /* at rest: speed and surface speed at most sleep_speed */
            double sp = sqrt(len2(b->v)), sw = sqrt(len2(b->w)) * bound_radius(b);
            if (fabs(sp - m->sleep_speed) < BAND_V || fabs(sw - m->sleep_speed) < BAND_V) {
                amb++;
                tied[i] = 1;
            }
            int at_rest = sp <= m->sleep_speed && sw <= m->sleep_speed;
            rest[gi0] = at_rest ? (rest[gi0] < (1 << 30) ? rest[gi0] + 1 : rest[gi0]) : 0;
        }
        if (b->joint) {
            /* a part moves exactly along its joint: q += dt qd; a hinge turns
             * the body about its line by dt qd, a slide shifts it by dt qd a */
            double dq = dt * b->qd;
            joint_state[2 * gi0] += dq;
            joint_state[2 * gi0 + 1] = b->qd;
            if (b->joint == 1) {
                double c = cos(dq), sn = sin(dq);
                V r = sub(b->x, b->jo), a = b->ja;
                V rr = add(add(scl(r, c), scl(cross(a, r), sn)), scl(a, dot(a, r) * (1.0 - c)));
                b->x = add(b->jo, rr);
                double hq[4] = {cos(0.5 * dq), a.x * sin(0.5 * dq), a.y * sin(0.5 * dq), a.z * sin(0.5 * dq)}, q2[4];
                quat_mul(hq, b->q, q2);
                double L = sqrt(q2[0] * q2[0] + q2[1] * q2[1] + q2[2] * q2[2] + q2[3] * q2[3]);
                for (int k = 0; k < 4; k++) b->q[k] = q2[k] / L;
            } else {
                b->x = add(b->x, scl(b->ja, dq));
            }
            part_sync(b);   /* velocity at the new pose */
        } else {
            b->x = add(b->x, scl(b->v, dt));
            double wq[4] = {0, b->w.x, b->w.y, b->w.z}, dq[4];
            quat_mul(wq, b->q, dq);
            double q2[4], L = 0;
            for (int k = 0; k < 4; k++) { q2[k] = b->q[k] + 0.5 * dt * dq[k]; L += q2[k] * q2[k]; }
            L = sqrt(L);
            for (int k = 0; k < 4; k++) b->q[k] = q2[k] / L;
        }
        int gi = b0 + i;
        pose[7 * gi] = b->x.x; pose[7 * gi + 1] = b->x.y; pose[7 * gi + 2] = b->x.z;
        for (int k = 0; k < 4; k++) pose[7 * gi + 3 + k] = b->q[k];
        vel[6 * gi] = b->v.x; vel[6 * gi + 1] = b->v.y; vel[6 * gi + 2] = b->v.z;
        vel[6 * gi + 3] = b->w.x; vel[6 * gi + 4] = b->w.y; vel[6 * gi + 5] = b->w.z;
        if (!finite3(b->x) || !finite3(b->v) || !finite3(b->w)) flags |= ORA_F_NONFINITE;
    }
    if (m->arm == 1) {
        for (int k = 0; k < 7; k++) theta[7 * s + k] += dt * thd[k];
        double lp[7][7];
        arm_fk(m, m->arm_base + 3 * s, theta + 7 * s, lp, ao, aax);
        for (int k = 0; k < 7; k++) memcpy(pose + 7 * (b0 + nb - 7 + k), lp[k], 7 * sizeof(double));
    } else if (m->arm == 2) {
        /* joint angles advance by their rates; links follow; rates, motor impulses out */
        for (int k = 0; k < 7; k++) {
            theta[7 * s + k] += dt * AR.qd[k];
            ast[k] = AR.qd[k];
            ast[14 + k] = AR.lam[k];
            if (!isfinite(AR.qd[k])) flags |= ORA_F_NONFINITE;
        }
        double lp[7][7];
        arm_fk(m, m->arm_base + 3 * s, theta + 7 * s, lp, ao, aax);
        for (int k = 0; k < 7; k++) {
            int gi = b0 + nb - 7 + k;
            memcpy(pose + 7 * gi, lp[k], 7 * sizeof(double));
            V c = mk(lp[k][0], lp[k][1], lp[k][2]), v = mk(0, 0, 0), w = mk(0, 0, 0);
            for (int j = 0; j <= k; j++) {
                w = add(w, scl(aax[j], AR.qd[j]));
                v = add(v, scl(cross(aax[j], sub(c, ao[j])), AR.qd[j]));
            }
            vel[6 * gi] = v.x; vel[6 * gi + 1] = v.y; vel[6 * gi + 2] = v.z;
            vel[6 * gi + 3] = w.x; vel[6 * gi + 4] = w.y; vel[6 * gi + 5] = w.z;
        }
    }

    /* 12. outputs: arm contact force, cache, contacts, stats */
    double force = 0;
    int arml = m->arm ? nb - 7 : nb;     /* first arm link (either arm) */
    for (int q = 0; q < nc; q++) {
        Con *c = &C[q];
        if (c->a >= arml || (c->b >= arml)) {
            V P = add(scl(c->n, c->lam[0]), add(scl(c->t1, c->lam[1]), scl(c->t2, c->lam[2])));
            force += sqrt(len2(P)) / dt;
        }
    }
    if (cache) {
        int w = nc < cache->cap ? nc : cache->cap;
        if (nc > cache->cap) flags |= ORA_F_CAPACITY;
        for (int q = 0; q < w; q++) {
            Con *c = &C[q];
            size_t o = (size_t)s * cache->cap + q;
            cache->key[o] = c->key;
            V F = add(scl(c->t1, c->lam[1]), scl(c->t2, c->lam[2]));
            cache->lam[4 * o] = c->lam[0];
            cache->lam[4 * o + 1] = F.x; cache->lam[4 * o + 2] = F.y; cache->lam[4 * o + 3] = F.z;
        }
        cache->count[s] = w;
    }
    if (out) {
        if (out->n_pairs) out->n_pairs[s] = np;
        if (out->pair_key) {
            int w = np < out->max_pairs ? np : out->max_pairs;
            memcpy(out->pair_key + (size_t)s * out->max_pairs, pk, sizeof(uint32_t) * w);
        }
        if (out->n_contacts) out->n_contacts[s] = nc;
        int w = nc < out->max_contacts ? nc : out->max_contacts;
        for (int q = 0; q < w; q++) {
            Con *c = &C[q];
            size_t o = (size_t)s * out->max_contacts + q;
            if (out->c_key) out->c_key[o] = c->key;
            if (out->c_normal) { out->c_normal[3 * o] = c->n.x; out->c_normal[3 * o + 1] = c->n.y; out->c_normal[3 * o + 2] = c->n.z; }
            if (out->c_point) { out->c_point[3 * o] = c->p.x; out->c_point[3 * o + 1] = c->p.y; out->c_point[3 * o + 2] = c->p.z; }
            if (out->c_phi) out->c_phi[o] = c->phi;
            if (out->c_lambda) for (int r = 0; r < 3; r++) out->c_lambda[3 * o + r] = c->lam[r];
            if (out->c_colour) out->c_colour[o] = c->colour;
            if (out->c_feat) memcpy(out->c_feat + 16 * o, c->feat, 16 * sizeof(double));
        }
        if (out->n_colours) out->n_colours[s] = ncol;
        if (out->sweeps) out->sweeps[s] = sweeps;
        if (out->residual) out->residual[s] = R;
        if (out->arm_force) out->arm_force[s] = force;
        if (out->flags) out->flags[s] = flags;
        if (out->ambiguous) out->ambiguous[s] = amb;
        if (out->tied) memcpy(out->tied + b0, tied, (size_t)nb);
        if (out->tol_gap) out->tol_gap[s] = gap;
    }
#undef AWAKE
    free(asleep);
    free(tied);
    free(order);
    free(Lm);
    free(C);
    free(pk);
    free(B);
    free(HL);
}

int ora_step(const ora_model *m, double *pose, double *vel, double *theta, int32_t *rest,
             double *arm_state, double *joint_state, ora_cache *cache, const double *actions, double dt, int iters,
             double tol, int warm, int solver, const ora_mlp *mlp,
             ora_out *out, int s0, int s1) {
    if (!m || !pose || !vel || dt <= 0 || iters < 0 || s0 < 0 || s1 > m->n_scenes || s0 > s1) return -1;
    if (m->arm && !theta) return -1;
    if (m->arm < 0 || m->arm > 2) return -1;
    if (m->arm == 2 && (!arm_state || solver != ORA_PGS || warm == ORA_LEARNED)) return -1;
    if (m->joint && (!joint_state || !m->joint_axis || !m->joint_anchor || !m->joint_limits || !m->joint_parent ||
                     solver != ORA_PGS || warm == ORA_LEARNED))
        return -1;
    if (warm == ORA_LEARNED && !mlp) return -1;
    /* hull bodies need a usable library entry */
    Hull *HL = hulls_of(m);
    for (int i = m->body_offset[s0]; i < m->body_offset[s1]; i++)
        if (m->shape[i] == ORA_HULL && (!HL || !(m->param[3 * i] >= 0 && m->param[3 * i] < m->n_hulls))) {
            free(HL);
            return -1;
        }
    free(HL);
    for (int s = s0; s < s1; s++)
        step_scene(m, pose, vel, theta, rest, arm_state, joint_state, cache, actions, dt, iters, tol, warm, solver, mlp,
                   out, s);
    return 0;
}

int ora_pairs(const ora_model *m, const double *pose, int s, uint32_t *keys, int cap) {
    int b0 = m->body_offset[s], nb = m->body_offset[s + 1] - b0;
    Body *B = malloc(sizeof(Body) * (nb ? nb : 1));
    double *vel = calloc((size_t)6 * m->body_offset[m->n_scenes], sizeof(double));
    Hull *HL = hulls_of(m);
    load_bodies(m, pose, vel, s, B, HL);
    for (int i = 0; i < nb; i++) body_aabb(&B[i], m->margin);
    int amb = 0;
    for (int i = 0; i < nb; i++) B[i].joint = m->joint && B[i].motion == ORA_DYNAMIC ? m->joint[m->body_offset[s] + i] : 0;
    int n = brute_pairs(B, nb, m->arm == 2 ? nb - 7 : nb, m->joint_parent ? m->joint_parent + m->body_offset[s] : NULL,
                        keys, cap, &amb, NULL);
    free(vel);
    free(B);
    free(HL);
    return n;
}

/* ---------------------------------------------------------------- arm queries
 * Collision checks of candidate arm configurations, the test a sampling
 * motion planner makes at every configuration it visits (Sec. 4.5 and
 * App. C: the planner checks the arm against the scene at fine joint-space
 * steps).  For scene s and configuration j the arm links are placed by the
 * forward kinematics of theta_q[(s*M + j)*7 ..] and every link (a capsule)
 * is tested against every body of the scene that is not an arm link (its
 * pose as given) and against the ground plane; the arm itself is left out
 * (its neighbouring links overlap at the joints by construction).  The
 * separation of a (link, obstacle) pair is the least signed separation of
 * its contacts (the narrowphase above, run with a margin just wider than the
 * clearance so that its kept set holds every contact that decides); min_phi
 * is the least over all pairs (+INF when no contact is within reach) and the
 * configuration collides, hit = 1, iff min_phi <= clearance.  ambiguous
 * counts configurations whose min_phi lies within BAND of the clearance. */
int ora_arm_query(const ora_model *m, const double *pose, const double *theta_q, int M, double clearance,
                  uint8_t *hit, double *min_phi, int32_t *ambiguous, int s0, int s1) {
    if (!m || !m->arm || !pose || M < 0 || !(clearance >= 0) || s0 < 0 || s1 > m->n_scenes || s0 > s1) return -1;
    if (M > 0 && (!theta_q || !hit)) return -1;
    const double reach = clearance + 2.0 * BAND;
    Hull *HL = hulls_of(m);
    for (int s = s0; s < s1; s++) {
        int b0 = m->body_offset[s], nb = m->body_offset[s + 1] - b0;
        if (nb < 7) { free(HL); return -1; }
        int nobs = nb - 7;
        for (int j = 0; j < M; j++) {
            const size_t q = (size_t)s * (size_t)M + (size_t)j;
            double lp[7][7];
            V o[7], ax[7];
            arm_fk(m, m->arm_base + 3 * s, theta_q + 7 * q, lp, o, ax);
            double best = INFINITY;
            for (int k = 0; k < 7; k++) {
                Geom L = geom_of(ORA_CAPSULE, m->param + 3 * (size_t)(b0 + nobs + k), lp[k], NULL);
                PC c[4];
                int amb = 0;
                int n = ground_contacts(&L, reach, c, &amb);
                for (int i = 0; i < n; i++) best = fmin(best, c[i].phi);
                for (int b = 0; b < nobs; b++) {
                    int g = b0 + b;
                    Geom O = geom_of(m->shape[g], m->param + 3 * (size_t)g, pose + 7 * (size_t)g, HL);
                    n = collide(&L, &O, reach, c, &amb);
                    for (int i = 0; i < n; i++) best = fmin(best, c[i].phi);
                }
            }
            hit[q] = best <= clearance;
            if (min_phi) min_phi[q] = best;
            if (ambiguous) ambiguous[q] = fabs(best - clearance) < BAND;
        }
    }
    free(HL);
    return 0;
}

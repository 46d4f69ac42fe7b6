// hull.h -- convex-hull narrowphase of the step (gfx950, float32).
//
// Convex collision proxies (Sec. 3: objects and furniture collide as convex
// hulls of their parts; Sec. 4.3: simplified collision geometry).  A hull is
// a convex polyhedron of the batch's hull library: body-frame vertices,
// face planes (outward unit normal n, offset d), face loops counter-clockwise
// seen from outside (at most 8 vertices) and undirected edges with their two
// faces; the host derives planes (Newell's normal through the loop's mean
// vertex) and edges (first appearance over the loops) from the vertices and
// loops.  A box enters hull-hull as the hull of its corners, faces -x +x -y
// +y -z +z, from the constant tables below (the order the host's rule gives).
//
// One lane per pair, like the other routines; every array access is to the
// library in global memory (read-only, L1/L2 resident) or is recomputed, so
// no routine needs per-lane arrays.  The contact sets follow the definitions
// below step by step; decisions are taken in the same order and with the
// same tolerances as the double-precision reference, so that they agree
// outside its tie band.
#pragma once

#include <stdint.h>

#include "geom.h"

namespace rbs {

constexpr int kHullMaxV = 32, kHullMaxF = 32, kHullMaxE = 64, kHullMaxL = 8;

// a box as a hull: face loops and edges (vertex a < b, first face, second face)
__constant__ uint8_t kBoxLoop[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};
__constant__ uint8_t kBoxEdge[12][4] = {{0, 4, 0, 2}, {4, 6, 0, 5}, {2, 6, 0, 3}, {0, 2, 0, 4}, {1, 3, 1, 4}, {3, 7, 1, 3},
                                        {5, 7, 1, 5}, {1, 5, 1, 2}, {0, 1, 2, 4}, {4, 5, 2, 5}, {6, 7, 3, 5}, {2, 3, 3, 4}};

// The hull library as the kernel reads it.
struct HullLib {
  const int32_t* info;    // [H][8]: first vertex, vertex count, first face, face count, first edge, edge count
  const float4* vert;     // [V] x y z (body frame), 0
  const float4* plane;    // [F] n, d
  const uint8_t* loop;    // [F][8] vertex indices within the hull, 255 after the last
  const uint8_t* edge;    // [E][4] vertex a, vertex b, face 0, face 1 (within the hull)
};

__device__ __forceinline__ V3 xyz4(float4 a) { return v3(a.x, a.y, a.z); }

// A convex polyhedron in world space: a hull of the library or a box.
struct Poly {
  bool box;
  V3 x, h;                 // centre; box half-extents
  M3 R;
  const float4* v;
  const float4* pl;
  const uint8_t* lp;
  const uint8_t* ed;
  int nv, nf, ne;
  __device__ __forceinline__ V3 local(int k) const {
    if (box) return v3((k & 1) ? h.x : -h.x, (k & 2) ? h.y : -h.y, (k & 4) ? h.z : -h.z);
    return xyz4(v[k]);
  }
  __device__ __forceinline__ V3 vert(int k) const { return x + Rv(R, local(k)); }
  // world plane of face f: normal and offset (n . X = d on the face)
  __device__ __forceinline__ void plane(int f, V3& n, float& d) const {
    V3 nl;
    float dl;
    if (box) {
      const int a = f >> 1;
      const float sg = (f & 1) ? 1.f : -1.f;
      nl = v3(a == 0 ? sg : 0.f, a == 1 ? sg : 0.f, a == 2 ? sg : 0.f);
      dl = comp(h, a);
    } else {
      const float4 p = pl[f];
      nl = v3(p.x, p.y, p.z);
      dl = p.w;
    }
    n = Rv(R, nl);
    d = dot(n, x) + dl;
  }
  __device__ __forceinline__ int nloop(int f) const {
    if (box) return 4;
    int n = 0;
    for (int k = 0; k < kHullMaxL; k++)
      if (lp[kHullMaxL * f + k] != 255u) n = k + 1;
    return n;
  }
  __device__ __forceinline__ int loopv(int f, int k) const { return box ? kBoxLoop[f][k] : lp[kHullMaxL * f + k]; }
  __device__ __forceinline__ void edge(int e, int& a, int& b, int& f0, int& f1) const {
    if (box) { a = kBoxEdge[e][0]; b = kBoxEdge[e][1]; f0 = kBoxEdge[e][2]; f1 = kBoxEdge[e][3]; }
    else { a = ed[4 * e]; b = ed[4 * e + 1]; f0 = ed[4 * e + 2]; f1 = ed[4 * e + 3]; }
  }
};

__device__ __forceinline__ Poly make_poly(const Geom& G, const HullLib& L) {
  Poly p;
  p.x = G.x;
  p.R = G.R;
  p.h = v3(G.p[0], G.p[1], G.p[2]);
  p.box = G.shape != HULL;
  if (p.box) {
    p.nv = 8; p.nf = 6; p.ne = 12;
    p.v = nullptr; p.pl = nullptr; p.lp = nullptr; p.ed = nullptr;
  } else {
    const int32_t* in = L.info + 8 * G.hull;
    p.v = L.vert + in[0];
    p.nv = in[1];
    p.pl = L.plane + in[2];
    p.lp = L.loop + (long)kHullMaxL * in[2];
    p.nf = in[3];
    p.ed = L.edge + 4L * in[4];
    p.ne = in[5];
  }
  return p;
}

// in-plane outward normal of loop edge k of face f (world, not normalised)
__device__ __forceinline__ V3 loop_side(const Poly& P, int f, int n, int k, V3 nf, V3& a) {
  a = P.vert(P.loopv(f, k));
  const V3 b = P.vert(P.loopv(f, k + 1 < n ? k + 1 : 0));
  return cross(b - a, nf);
}

// p (in face f's plane) inside face f's loop
__device__ __forceinline__ bool inside_loop(const Poly& P, int f, V3 nf, V3 p) {
  const int n = P.nloop(f);
  for (int k = 0; k < n; k++) {
    V3 a;
    const V3 m = loop_side(P, f, n, k, nf, a);
    if (dot(m, p - a) > 0.f) return false;
  }
  return true;
}

// Closest point of the polyhedron to p outside it: projections onto faces
// above p that fall inside their loops, then every edge's closest point;
// the nearest wins (ties: faces first, lower index).  Returns the distance.
__device__ inline float poly_closest(const Poly& P, V3 p, V3& q) {
  float best = INFINITY;
  for (int f = 0; f < P.nf; f++) {
    V3 n;
    float d;
    P.plane(f, n, d);
    const float s = dot(n, p) - d;
    if (s <= 0.f) continue;
    const V3 pr = p - n * s;
    if (s < best && inside_loop(P, f, n, pr)) { best = s; q = pr; }
  }
  for (int e = 0; e < P.ne; e++) {
    int a, b, f0, f1;
    P.edge(e, a, b, f0, f1);
    const V3 va = P.vert(a), dv = P.vert(b) - va;
    const float t = clampf(fdiv(dot(p - va, dv), len2(dv)), 0.f, 1.f);
    const V3 c = va + dv * t;
    const float L = fsqrt(len2(p - c));
    if (L < best) { best = L; q = c; }
  }
  return best;
}

// Choice with a tolerance among candidates k < n whose score fn(k, &v)
// reports them present: the first whose score is within tol of the
// largest (ties to the lower index); skips the used mask.
template <class F>
__device__ __forceinline__ int argmax_tol(int n, F fn, uint64_t u0, uint64_t u1, float tol) {
  float vmax = -INFINITY;
  for (int k = 0; k < n; k++) {
    const bool used = k < 64 ? ((u0 >> k) & 1ull) : ((u1 >> (k - 64)) & 1ull);
    float v;
    if (!used && fn(k, v)) vmax = fmaxf(vmax, v);
  }
  for (int k = 0; k < n; k++) {
    const bool used = k < 64 ? ((u0 >> k) & 1ull) : ((u1 >> (k - 64)) & 1ull);
    float v;
    if (!used && fn(k, v) && v >= vmax - tol) return k;
  }
  return -1;
}

__device__ __forceinline__ void mark(uint64_t& u0, uint64_t& u1, int k) {
  if (k < 64) u0 |= 1ull << k;
  else u1 |= 1ull << (k - 64);
}

// At most 4 of the candidates (present(k, &p), k < n, more than 4 present):
// `first`, the farthest from it, the one spanning the largest triangle, the
// one adding most to the three triangles' areas (tolerances CLIP_ON, times
// the first edge's length, times the triangle's perimeter).
template <class F>
__device__ __forceinline__ void reduce4(int n, F present, int first, uint64_t& u0, uint64_t& u1) {
  mark(u0, u1, first);
  V3 p1;
  present(first, p1);
  const int i2 = argmax_tol(n, [&](int k, float& v) {
    V3 p;
    if (!present(k, p)) return false;
    v = fsqrt(len2(p - p1));
    return true;
  }, u0, u1, kClipOn);
  mark(u0, u1, i2);
  V3 p2;
  present(i2, p2);
  const V3 e12 = p2 - p1;
  const float l12 = fsqrt(len2(e12));
  const int i3 = argmax_tol(n, [&](int k, float& v) {
    V3 p;
    if (!present(k, p)) return false;
    v = fsqrt(len2(cross(e12, p - p1)));
    return true;
  }, u0, u1, kClipOn * l12);
  mark(u0, u1, i3);
  V3 p3;
  present(i3, p3);
  const V3 e23 = p3 - p2, e31 = p1 - p3;
  const float per = l12 + fsqrt(len2(e23)) + fsqrt(len2(e31));
  const int i4 = argmax_tol(n, [&](int k, float& v) {
    V3 p;
    if (!present(k, p)) return false;
    v = fsqrt(len2(cross(e12, p - p1))) + fsqrt(len2(cross(e23, p - p2))) + fsqrt(len2(cross(e31, p - p3)));
    return true;
  }, u0, u1, kClipOn * per);
  mark(u0, u1, i4);
}

// Hull on the ground plane: vertices with depth <= margin; above 4,
// reduce4 from the first vertex within CLIP_ON of the deepest; contacts in
// vertex order, feature the vertex index.
__device__ __noinline__ void hull_ground(const Geom& A, const HullLib& HL, float margin, Out4& out) {
  const Poly P = make_poly(A, HL);
  auto kept = [&](int k, V3& w) {
    w = P.vert(k);
    return w.z <= margin;
  };
  int m = 0;
  for (int k = 0; k < P.nv; k++) {
    V3 w;
    m += kept(k, w) ? 1 : 0;
  }
  uint64_t u0 = 0, u1 = 0;
  if (m > 4) {
    const int first = argmax_tol(P.nv, [&](int k, float& v) {
      V3 w;
      if (!kept(k, w)) return false;
      v = -w.z;
      return true;
    }, 0ull, 0ull, kClipOn);
    reduce4(P.nv, kept, first, u0, u1);
  }
  for (int k = 0; k < P.nv; k++) {
    V3 w;
    if (!kept(k, w) || (m > 4 && !((u0 >> k) & 1ull))) continue;
    PC c;
    c.n = v3(0.f, 0.f, 1.f);
    c.phi = w.z;
    c.p = v3(w.x, w.y, 0.5f * w.z);
    c.f = k;
    out.push(c);
  }
}

// Sphere (first) against a hull (second): a centre outside leaves along the
// line to the closest point; inside through the face of least penetration.
__device__ inline void sphere_hull(const Geom& S, const Geom& G, const HullLib& HL, float margin, Out4& out) {
  const Poly P = make_poly(G, HL);
  const float r = S.p[0];
  float smax = -INFINITY;
  V3 nm = v3(0.f, 0.f, 1.f);
  for (int f = 0; f < P.nf; f++) {
    V3 n;
    float d;
    P.plane(f, n, d);
    const float s = dot(n, S.x) - d;
    if (s > smax) { smax = s; nm = n; }
  }
  PC c;
  V3 q;
  if (smax <= 0.f) {
    c.n = nm;
    q = S.x - nm * smax;
    c.phi = smax - r;
  } else {
    const float dist = poly_closest(P, S.x, q);
    c.n = (S.x - q) * frcpg(dist);
    c.phi = dist - r;
  }
  c.p = ((S.x - c.n * r) + q) * 0.5f;
  c.f = 0;
  if (c.phi <= margin) out.push(c);
}

// core segment p0 + t d clipped to face f's prism
__device__ inline bool clip_prism(const Poly& P, int f, V3 nf, V3 p0, V3 d, float& t0, float& t1) {
  float a = 0.f, b = 1.f;
  const int n = P.nloop(f);
  for (int k = 0; k < n; k++) {
    V3 va;
    const V3 m = loop_side(P, f, n, k, nf, va);
    const float g0 = dot(m, p0 - va), gd = dot(m, d);
    if (gd == 0.f) {
      if (g0 > 0.f) return false;
      continue;
    }
    const float t = -fdiv(g0, gd);
    if (gd > 0.f) b = fminf(b, t);
    else a = fmaxf(a, t);
  }
  t0 = a;
  t1 = b;
  return a <= b;
}

__device__ __forceinline__ PC poly_face_contact(V3 n, float d, V3 l, float r, int ft) {
  PC c;
  c.n = n;
  const float s = dot(n, l) - d;
  c.phi = s - r;
  c.p = ((l - n * s) + (l - n * r)) * 0.5f;
  c.f = ft;
  return c;
}

// face region of a core point l outside the polyhedron: the face whose
// plane it is above and whose loop holds its projection, largest height
__device__ inline int face_region(const Poly& P, V3 l, V3& nr, float& dr) {
  int best = -1;
  float bs = 0.f;
  for (int f = 0; f < P.nf; f++) {
    V3 n;
    float d;
    P.plane(f, n, d);
    const float s = dot(n, l) - d;
    if (s > 0.f && (best < 0 || s > bs) && inside_loop(P, f, n, l - n * s)) { best = f; bs = s; nr = n; dr = d; }
  }
  return best;
}

// Capsule (first) against a hull (second), after capsule_box: separated
// core -> closest points among the ends and the core against every edge;
// in a face region within ~1 mrad of parallel, or that parallel to a face
// whose plane lies at the closest distance (within CLIP_ON) and whose
// prism it crosses -> the core clipped to that face's prism (f 0, 1), else
// one contact (f 2); touching core -> the face
// whose plane the deeper end lies least below, clipped (f 0, 1) or the
// deeper end (f 3).
__device__ inline void capsule_hull(const Geom& C, const Geom& G, const HullLib& HL, float margin, Out4& out) {
  const Poly P = make_poly(G, HL);
  const float r = C.p[0];
  V3 p0, d;
  capsule_seg(C, p0, d);
  const float dl = fsqrt(len2(d));
  float tin = 0.f, tout = 1.f;
  for (int f = 0; f < P.nf; f++) {
    V3 n;
    float dd;
    P.plane(f, n, dd);
    const float dn = dot(n, d), s0 = dot(n, p0) - dd;
    if (dn == 0.f) {
      if (s0 > 0.f) tout = -1.f;
      continue;
    }
    const float t = -fdiv(s0, dn);
    if (dn < 0.f) tin = fmaxf(tin, t);
    else tout = fminf(tout, t);
  }
  PC loc0, loc1;
  int n = 0;
  if (!(tin <= tout)) {
    // candidate k: 0, 1 the ends; 2 + e the core against edge e
    auto cand = [&](int k, float& t, V3& q) -> float {
      if (k < 2) {
        t = (float)k;
        return poly_closest(P, p0 + d * t, q);
      }
      int a, b, f0, f1;
      P.edge(k - 2, a, b, f0, f1);
      const V3 va = P.vert(a), u = P.vert(b) - va;
      const V3 w = p0 - va;
      const float A2 = len2(d), B2 = dot(d, u), C2 = len2(u), D2 = dot(d, w), E2 = dot(u, w);
      const float den = A2 * C2 - B2 * B2;
      t = 0.f;
      if (den > 1e-18f * A2 * C2) t = clampf(fdiv(B2 * E2 - C2 * D2, den), 0.f, 1.f);
      float sv = fdiv(B2 * t + E2, C2);
      if (sv < 0.f) { sv = 0.f; t = clampf(fdiv(-D2, A2), 0.f, 1.f); }
      else if (sv > 1.f) { sv = 1.f; t = clampf(fdiv(B2 - D2, A2), 0.f, 1.f); }
      q = va + u * sv;
      return fsqrt(len2((p0 + d * t) - q));
    };
    float dist = INFINITY, t = 0.f;
    V3 q = v3(0.f, 0.f, 0.f);
    for (int k = 0; k < 2 + P.ne; k++) {
      float tk;
      V3 qk;
      const float dk = cand(k, tk, qk);
      if (dk < dist) { dist = dk; t = tk; q = qk; }
    }
    const V3 l = p0 + d * t;
    V3 nr;
    float dr;
    int fr = face_region(P, l, nr, dr);
    bool facecase = fr >= 0 && fabsf(dot(d, nr)) <= kSinParallel * dl;
    // a core level with a face at the distance found: that face's plateau
    for (int f = 0; f < P.nf && !facecase; f++) {
      V3 n;
      float dd;
      P.plane(f, n, dd);
      if (fabsf(dot(d, n)) > kSinParallel * dl) continue;
      float t0, t1;
      if (fabsf(dot(n, l) - dd - dist) <= kClipOn && clip_prism(P, f, n, p0, d, t0, t1)) {
        fr = f;
        nr = n;
        dr = dd;
        facecase = true;
      }
    }
    bool done = false;
    if (facecase) {
      float t0, t1;
      if (clip_prism(P, fr, nr, p0, d, t0, t1)) {
        loc0 = poly_face_contact(nr, dr, p0 + d * t0, r, 0);
        n = 1;
        if (t1 > t0) { loc1 = poly_face_contact(nr, dr, p0 + d * t1, r, 1); n = 2; }
        done = true;
      }
    }
    if (!done) {
      loc0.n = (l - q) * frcpg(dist);
      loc0.phi = dist - r;
      loc0.p = (q + (l - loc0.n * r)) * 0.5f;
      loc0.f = 2;
      n = 1;
    }
  } else {
    float best = INFINITY;
    int bf = 0;
    const V3 p1 = p0 + d;
    for (int f = 0; f < P.nf; f++) {
      V3 nn;
      float dd;
      P.plane(f, nn, dd);
      const float ex = dd - fminf(dot(nn, p0), dot(nn, p1));
      if (ex < best) { best = ex; bf = f; }
    }
    V3 nb;
    float db;
    P.plane(bf, nb, db);
    float t0, t1;
    if (clip_prism(P, bf, nb, p0, d, t0, t1)) {
      loc0 = poly_face_contact(nb, db, p0 + d * t0, r, 0);
      n = 1;
      if (t1 > t0) { loc1 = poly_face_contact(nb, db, p0 + d * t1, r, 1); n = 2; }
    } else {
      const float e0 = dot(nb, p0), e1 = dot(nb, p1);
      loc0 = poly_face_contact(nb, db, e0 <= e1 ? p0 : p1, r, 3);
      n = 1;
    }
  }
  if (n > 0 && loc0.phi <= margin) out.push(loc0);
  if (n > 1 && loc1.phi <= margin) out.push(loc1);
}

// Hull against hull (a box as the hull of its corners): separating axes
// over both face sets (separation: the other's least vertex height above
// the face) and the edge pairs that build faces of the Minkowski
// difference (Gregorius 2013; axis e_A x e_B away from A's centre,
// separation u . (b - a)); A's face unless B's is clearly better, an edge
// only when clearly better.  Edge contact: closest points of the two edges
// (f 0xFF).  Face contact: the incident face most opposed to the reference
// face; candidate points by id (incident vertex k inside every side plane;
// incident edge k crossing side plane j inside the others, 8 + 8k + j;
// reference corner j inside the incident face, on its plane along the
// reference normal, 72 + j); kept if depth <= margin, above 4 reduced by
// reduce4 from the smallest id; feature (reference is B) | id << 1.
__device__ inline void hull_hull(const Geom& GA, const Geom& GB, const HullLib& HL, float margin, Out4& out) {
  const Poly A = make_poly(GA, HL), B = make_poly(GB, HL);
  float sfa = -INFINITY, sfb = -INFINITY;
  int fa = 0, fb = 0;
  // a face axis that already separates the hulls by more than the margin
  // ends the pair (no contact whatever the other axes give)
  for (int f = 0; f < A.nf; f++) {
    V3 n;
    float d;
    A.plane(f, n, d);
    float s = INFINITY;
    for (int k = 0; k < B.nv; k++) s = fminf(s, dot(n, B.vert(k)) - d);
    if (s > margin) return;
    if (s > sfa) { sfa = s; fa = f; }
  }
  for (int f = 0; f < B.nf; f++) {
    V3 n;
    float d;
    B.plane(f, n, d);
    float s = INFINITY;
    for (int k = 0; k < A.nv; k++) s = fminf(s, dot(n, A.vert(k)) - d);
    if (s > margin) return;
    if (s > sfb) { sfb = s; fb = f; }
  }
  float se = -INFINITY;
  int ei = -1, ej = -1;
  V3 ue = v3(0.f, 0.f, 1.f);
  for (int i = 0; i < A.ne; i++) {
    int ia0, ia1, fa0, fa1;
    A.edge(i, ia0, ia1, fa0, fa1);
    V3 a, b;
    float dtmp;
    A.plane(fa0, a, dtmp);
    A.plane(fa1, b, dtmp);
    const V3 bxa = cross(b, a);
    const V3 pa = A.vert(ia0), da = A.vert(ia1) - pa;
    for (int j = 0; j < B.ne; j++) {
      int jb0, jb1, fb0, fb1;
      B.edge(j, jb0, jb1, fb0, fb1);
      V3 c, d;
      B.plane(fb0, c, dtmp);
      B.plane(fb1, d, dtmp);
      c = -c;
      d = -d;
      const V3 dxc = cross(d, c);
      const float cba = dot(c, bxa), dba = dot(d, bxa), adc = dot(a, dxc), bdc = dot(b, dxc);
      if (!(cba * dba < 0.f && adc * bdc < 0.f && cba * bdc > 0.f)) continue;
      const V3 pb = B.vert(jb0), db = B.vert(jb1) - pb;
      V3 u = cross(da, db);
      const float L2 = len2(u), ref = len2(da) * len2(db);
      if (L2 < 1e-12f * ref) continue;
      u = u * frsq(L2);
      if (dot(u, pa - A.x) < 0.f) u = -u;
      const float sv = dot(u, pb - pa);
      if (sv > se) { se = sv; ei = i; ej = j; ue = u; }
    }
  }
  const float smax = fmaxf(fmaxf(sfa, sfb), se);
  if (smax > margin) return;
  const float hmax = fmaxf(fmaxf(fmaxf(GA.p[0], GA.p[1]), fmaxf(GA.p[2], GB.p[0])), fmaxf(GB.p[1], GB.p[2]));
  bool refB = false;
  float sface = sfa;
  if (sfb > 0.95f * sfa + 0.01f * hmax) { refB = true; sface = sfb; }
  if (ei >= 0 && se > 0.95f * sface + 0.01f * hmax) {
    int a0, a1, b0, b1, f0, f1;
    A.edge(ei, a0, a1, f0, f1);
    B.edge(ej, b0, b1, f0, f1);
    const V3 va0 = A.vert(a0), va1 = A.vert(a1), vb0 = B.vert(b0), vb1 = B.vert(b1);
    const V3 pa = (va0 + va1) * 0.5f, pb = (vb0 + vb1) * 0.5f;
    V3 ai = va1 - va0, bj = vb1 - vb0;
    const float la = 0.5f * fsqrt(len2(ai)), lb = 0.5f * fsqrt(len2(bj));
    ai = ai * fdiv(0.5f, la);
    bj = bj * fdiv(0.5f, lb);
    const V3 w = pa - pb;
    const float bb = dot(ai, bj), dd = dot(ai, w), ee = dot(bj, w);
    const float den = 1.0f - bb * bb;
    float ta = fdiv(bb * ee - dd, den);
    float tb = ee + ta * bb;
    ta = clampf(ta, -la, la);
    tb = clampf(tb, -lb, lb);
    const V3 PA = pa + ai * ta, PB = pb + bj * tb;
    PC c;
    c.n = -ue;
    c.phi = dot(PA - PB, c.n);
    c.p = (PA + PB) * 0.5f;
    c.f = 0xFF;
    if (c.phi <= margin) out.push(c);
    return;
  }
  // face contact
  const Poly& Rf = refB ? B : A;
  const Poly& In = refB ? A : B;
  const int rf = refB ? fb : fa;
  V3 nout;
  float Dref;
  Rf.plane(rf, nout, Dref);
  const V3 N = refB ? nout : -nout;
  int inf = 0;
  float best = INFINITY;
  for (int f = 0; f < In.nf; f++) {
    V3 n;
    float d;
    In.plane(f, n, d);
    const float c = dot(n, nout);
    if (c < best) { best = c; inf = f; }
  }
  V3 ninc;
  float Dinc;
  In.plane(inf, ninc, Dinc);
  const int nR = Rf.nloop(rf), nI = In.nloop(inf);
  auto Rv_ = [&](int j) { return Rf.vert(Rf.loopv(rf, j < nR ? j : j - nR)); };
  auto Xv = [&](int k) { return In.vert(In.loopv(inf, k < nI ? k : k - nI)); };
  // side distance of X from reference side plane j (unit in-plane normal)
  auto side = [&](int j, V3 X) {
    const V3 rj = Rv_(j);
    V3 m = cross(Rv_(j + 1) - rj, nout);
    m = m * frsq(len2(m));
    return dot(m, X - rj);
  };
  // candidate id -> point on the incident face (false: absent)
  auto cand = [&](int id, V3& X) -> bool {
    if (id < 8) {
      if (id >= nI) return false;
      X = Xv(id);
      for (int j = 0; j < nR; j++)
        if (side(j, X) > kClipOn) return false;
      return true;
    }
    if (id < 72) {
      const int k = (id - 8) >> 3, j = (id - 8) & 7;
      if (k >= nI || j >= nR) return false;
      const V3 x0 = Xv(k), x1 = Xv(k + 1);
      const float d0 = side(j, x0), d1 = side(j, x1);
      const int s0 = d0 < -kClipOn ? -1 : (d0 > kClipOn ? 1 : 0), s1 = d1 < -kClipOn ? -1 : (d1 > kClipOn ? 1 : 0);
      if (s0 * s1 >= 0) return false;
      X = x0 + (x1 - x0) * fdiv(d0, d0 - d1);
      for (int i = 0; i < nR; i++)
        if (i != j && side(i, X) > kClipOn) return false;
      return true;
    }
    const int j = id - 72;
    if (j >= nR) return false;
    const V3 rj = Rv_(j);
    X = rj + nout * fdiv(Dinc - dot(ninc, rj), dot(ninc, nout));
    for (int k = 0; k < nI; k++) {
      const V3 xk = Xv(k);
      V3 m = cross(Xv(k + 1) - xk, ninc);
      m = m * frsq(len2(m));
      if (!(dot(m, X - xk) < -kClipOn)) return false;
    }
    return true;
  };
  auto kept = [&](int id, V3& X) { return cand(id, X) && dot(nout, X) - Dref <= margin; };
  constexpr int kIds = 80;
  int nk = 0, first = -1;
  for (int id = 0; id < kIds; id++) {
    V3 X;
    if (kept(id, X)) {
      if (first < 0) first = id;
      nk++;
    }
  }
  uint64_t u0 = 0, u1 = 0;
  if (nk > 4) reduce4(kIds, kept, first, u0, u1);
  for (int id = 0; id < kIds; id++) {
    V3 X;
    if (!kept(id, X)) continue;
    if (nk > 4 && !(id < 64 ? ((u0 >> id) & 1ull) : ((u1 >> (id - 64)) & 1ull))) continue;
    PC c;
    c.n = N;
    c.phi = dot(nout, X) - Dref;
    c.p = X - nout * (0.5f * c.phi);
    c.f = (refB ? 1 : 0) | (id << 1);
    out.push(c);
  }
}

// Contacts of a pair with a hull (normal from B to A).  Not inlined: the
// hull routines' registers stay out of the step's own allocation.
__device__ __noinline__ void collide_hull(const Geom& A, const Geom& B, const HullLib& HL, float margin, Out4& out) {
  bool flip = false;
  if (A.shape == SPHERE) sphere_hull(A, B, HL, margin, out);
  else if (B.shape == SPHERE) { sphere_hull(B, A, HL, margin, out); flip = true; }
  else if (A.shape == CAPSULE) capsule_hull(A, B, HL, margin, out);
  else if (B.shape == CAPSULE) { capsule_hull(B, A, HL, margin, out); flip = true; }
  else hull_hull(A, B, HL, margin, out);
  if (flip) out.flip();
}

}  // namespace rbs

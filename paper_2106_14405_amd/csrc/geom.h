// geom.h -- float32 device geometry for the batched rigid-body step (gfx950).
//
// Internal to the HIP library.  Contact conventions: routines return
// contacts whose normal points from the SECOND shape to the FIRST; phi is
// the signed separation along n (negative = penetration); p is the midpoint
// of the two witness points; f is a small feature id.  A contact is kept
// iff phi <= margin.  Standard methods: closest points (Ericson 2005),
// oriented-box separating axes (Gottschalk et al. 1996), polygon clipping
// (Sutherland and Hodgman 1974).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbs {

enum { SPHERE = 0, BOX = 1, CAPSULE = 2, HULL = 3 };
enum { DYNAMIC = 0, STATIC = 1, KINEMATIC = 2 };

constexpr float kSinParallel = 1e-3f;   // segment within ~1 mrad of a face plane
constexpr float kClipOn = 1e-4f;        // clip vertices this close to a plane lie on it (m)
constexpr float kCapParallel = 1e-6f;   // |da x db|^2 <= this * |da|^2 |db|^2
constexpr float kEdgeDegenerate = 1e-12f;

struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return v3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ V3 operator-(V3 a) { return v3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float len2(V3 a) { return dot(a, a); }
__device__ __forceinline__ float clampf(float x, float lo, float hi) { return x < lo ? lo : (x > hi ? hi : x); }
// Hardware reciprocal, square root and reciprocal square root (about 1 ulp):
// contact geometry is continuous in them, and a rounding-level difference is
// far inside the tie band of every discrete decision.
__device__ __forceinline__ float frcpg(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float comp(V3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }
__device__ __forceinline__ void setc(V3& a, int i, float s) {
  if (i == 0) a.x = s; else if (i == 1) a.y = s; else a.z = s;
}
__device__ __forceinline__ V3 unitv(int i) { return v3(i == 0 ? 1.f : 0.f, i == 1 ? 1.f : 0.f, i == 2 ? 1.f : 0.f); }
// Element i of a three-element array, as selects (a runtime index into a
// local array would put the array in scratch memory).
__device__ __forceinline__ float at3(const float* h, int i) { return i == 0 ? h[0] : (i == 1 ? h[1] : h[2]); }
__device__ __forceinline__ V3 sel3(V3 a0, V3 a1, V3 a2, int i) {
  return v3(i == 0 ? a0.x : (i == 1 ? a1.x : a2.x), i == 0 ? a0.y : (i == 1 ? a1.y : a2.y),
            i == 0 ? a0.z : (i == 1 ? a1.z : a2.z));
}
__device__ __forceinline__ V3 selv(bool s, V3 a, V3 b) { return v3(s ? a.x : b.x, s ? a.y : b.y, s ? a.z : b.z); }

// Rotation matrix, row-major m[r][c]; columns are the body axes in world.
struct M3 {
  float m[3][3];
};
__device__ __forceinline__ M3 quat_R(float w, float x, float y, float z) {
  M3 R;
  R.m[0][0] = 1.f - 2.f * (y * y + z * z); R.m[0][1] = 2.f * (x * y - w * z); R.m[0][2] = 2.f * (x * z + w * y);
  R.m[1][0] = 2.f * (x * y + w * z); R.m[1][1] = 1.f - 2.f * (x * x + z * z); R.m[1][2] = 2.f * (y * z - w * x);
  R.m[2][0] = 2.f * (x * z - w * y); R.m[2][1] = 2.f * (y * z + w * x); R.m[2][2] = 1.f - 2.f * (x * x + y * y);
  return R;
}
__device__ __forceinline__ V3 Rv(const M3& R, V3 a) {
  return v3(R.m[0][0] * a.x + R.m[0][1] * a.y + R.m[0][2] * a.z,
            R.m[1][0] * a.x + R.m[1][1] * a.y + R.m[1][2] * a.z,
            R.m[2][0] * a.x + R.m[2][1] * a.y + R.m[2][2] * a.z);
}
__device__ __forceinline__ V3 RTv(const M3& R, V3 a) {
  return v3(R.m[0][0] * a.x + R.m[1][0] * a.y + R.m[2][0] * a.z,
            R.m[0][1] * a.x + R.m[1][1] * a.y + R.m[2][1] * a.z,
            R.m[0][2] * a.x + R.m[1][2] * a.y + R.m[2][2] * a.z);
}
__device__ __forceinline__ V3 col(const M3& R, int j) {
  return v3(at3(R.m[0], j), at3(R.m[1], j), at3(R.m[2], j));
}

struct Geom {
  int shape;
  V3 x;
  M3 R;
  float p[3];   // a hull: the half-extents of its local bounding box
  int hull;     // a hull: its index in the hull library
};
struct PC {
  V3 n, p;
  float phi;
  int f;
};

// Up to eight polygon vertices in registers: indexed access is an unrolled
// select over the slots, so the array never goes to scratch memory.
struct Poly8 {
  V3 v[8];
  __device__ __forceinline__ V3 get(int k) const {
    V3 r = v[0];
#pragma unroll
    for (int j = 1; j < 8; j++) r = selv(j == k, v[j], r);
    return r;
  }
  __device__ __forceinline__ void set(int k, V3 x) {
#pragma unroll
    for (int j = 0; j < 8; j++) v[j] = selv(j == k, x, v[j]);
  }
};

// Up to four contacts held in registers (fixed slots, no indexed array).
__device__ __forceinline__ PC selpc(bool s, const PC& a, const PC& b) {
  PC r;
  r.n = selv(s, a.n, b.n);
  r.p = selv(s, a.p, b.p);
  r.phi = s ? a.phi : b.phi;
  r.f = s ? a.f : b.f;
  return r;
}
struct Out4 {
  PC c0, c1, c2, c3;
  int n;
  __device__ __forceinline__ void push(const PC& c) {
    c0 = selpc(n == 0, c, c0);
    c1 = selpc(n == 1, c, c1);
    c2 = selpc(n == 2, c, c2);
    c3 = selpc(n == 3, c, c3);
    n++;
  }
  __device__ __forceinline__ PC get(int k) const { return selpc(k == 0, c0, selpc(k == 1, c1, selpc(k == 2, c2, c3))); }
  __device__ __forceinline__ void flip() {
    c0.n = -c0.n; c1.n = -c1.n; c2.n = -c2.n; c3.n = -c3.n;
  }
};

__device__ __forceinline__ PC sphere_sphere(V3 ca, float ra, V3 cb, float rb, int f) {
  PC c;
  V3 d = ca - cb;
  float L = fsqrt(len2(d));
  c.n = L < 1e-9f ? v3(0.f, 0.f, 1.f) : d * frcpg(L);
  c.phi = L - ra - rb;
  c.p = ((ca - c.n * ra) + (cb + c.n * rb)) * 0.5f;
  c.f = f;
  return c;
}

// Sphere (first) vs box (second): clamp in the box frame; a centre inside
// leaves through the face of least penetration (ties: lower axis, + face).
__device__ inline void sphere_box(const Geom& S, const Geom& B, float margin, Out4& out) {
  float r = S.p[0];
  const float* h = B.p;
  V3 l = RTv(B.R, S.x - B.x);
  bool inside = fabsf(l.x) <= h[0] && fabsf(l.y) <= h[1] && fabsf(l.z) <= h[2];
  V3 nl, q = l;
  float phi;
  if (!inside) {
    q = v3(clampf(l.x, -h[0], h[0]), clampf(l.y, -h[1], h[1]), clampf(l.z, -h[2], h[2]));
    V3 d = l - q;
    float L = fsqrt(len2(d));
    nl = d * frcpg(L);
    phi = L - r;
  } else {
    float pen0 = h[0] - fabsf(l.x), pen1 = h[1] - fabsf(l.y), pen2 = h[2] - fabsf(l.z);
    int a = 0;
    float pa = pen0;
    if (pen1 < pa) { a = 1; pa = pen1; }
    if (pen2 < pa) { a = 2; pa = pen2; }
    float la = comp(l, a);
    float s = la >= 0.f ? 1.f : -1.f;
    nl = unitv(a) * s;
    setc(q, a, s * at3(h, a));
    phi = -pa - r;
  }
  PC c;
  c.n = Rv(B.R, nl);
  V3 wb = B.x + Rv(B.R, q);
  V3 wa = S.x - c.n * r;
  c.p = (wa + wb) * 0.5f;
  c.phi = phi;
  c.f = 0;
  if (phi <= margin) out.push(c);
}

__device__ __forceinline__ void capsule_seg(const Geom& C, V3& p0, V3& d) {
  V3 ax = col(C.R, 2) * C.p[1];
  p0 = C.x - ax;
  d = ax * 2.0f;
}

__device__ inline void sphere_capsule(const Geom& S, const Geom& C, float margin, Out4& out) {
  V3 p0, d;
  capsule_seg(C, p0, d);
  float t = clampf(fdiv(dot(S.x - p0, d), len2(d)), 0.f, 1.f);
  PC c = sphere_sphere(S.x, S.p[0], p0 + d * t, C.p[0], 0);
  if (c.phi <= margin) out.push(c);
}

// Capsule vs capsule: closest points of the core segments; nearly parallel
// cores whose projections overlap give contacts at both overlap ends.
__device__ inline void capsule_capsule(const Geom& A, const Geom& B, float margin, Out4& out) {
  V3 pa, da, pb, db;
  capsule_seg(A, pa, da);
  capsule_seg(B, pb, db);
  float ra = A.p[0], rb = B.p[0];
  float aa = len2(da), ee = len2(db);
  float cr2 = len2(cross(da, db));
  if (cr2 <= kCapParallel * aa * ee) {
    float s0 = fdiv(dot(pb - pa, da), aa);
    float s1 = fdiv(dot((pb + db) - pa, da), aa);
    float lo = fmaxf(0.f, fminf(s0, s1)), hi = fminf(1.f, fmaxf(s0, s1));
    if (lo <= hi) {
      for (int k = 0; k < 2; k++) {
        if (k == 1 && !(hi > lo)) break;
        float s = k == 0 ? lo : hi;
        V3 P = pa + da * s;
        float t = clampf(fdiv(dot(P - pb, db), ee), 0.f, 1.f);
        PC c = sphere_sphere(P, ra, pb + db * t, rb, k);
        if (c.phi <= margin) out.push(c);
      }
      return;
    }
  }
  V3 r = pa - pb;
  float b = dot(da, db), c = dot(da, r), f = dot(db, r);
  float den = aa * ee - b * b;
  float s = den != 0.f ? clampf(fdiv(b * f - c * ee, den), 0.f, 1.f) : 0.f;
  float t = fdiv(b * s + f, ee);
  if (t < 0.f) { t = 0.f; s = clampf(fdiv(-c, aa), 0.f, 1.f); }
  else if (t > 1.f) { t = 1.f; s = clampf(fdiv(b - c, aa), 0.f, 1.f); }
  PC cc = sphere_sphere(pa + da * s, ra, pb + db * t, rb, 0);
  if (cc.phi <= margin) out.push(cc);
}

__device__ __forceinline__ float box_d2(V3 l, const float* h) {
  float g = 0.f;
  float x = fabsf(l.x) - h[0]; if (x > 0.f) g += x * x;
  x = fabsf(l.y) - h[1]; if (x > 0.f) g += x * x;
  x = fabsf(l.z) - h[2]; if (x > 0.f) g += x * x;
  return g;
}

// Segment l(t) = p0 + t d, t in [0,1], clipped to the slabs |l_b| <= h_b of
// the two axes b != a.  False when empty.
__device__ inline bool clip_face(V3 p0, V3 d, const float* h, int a, float& t0, float& t1) {
  float lo = 0.f, hi = 1.f;
#pragma unroll
  for (int b = 0; b < 3; b++) {
    if (b == a) continue;
    float pb = comp(p0, b), db = comp(d, b);
    if (db == 0.f) {
      if (fabsf(pb) > h[b]) return false;
      continue;
    }
    const float idb = frcpg(db);
    float ta = (-h[b] - pb) * idb, tb = (h[b] - pb) * idb;
    if (ta > tb) { float x = ta; ta = tb; tb = x; }
    if (ta > lo) lo = ta;
    if (tb < hi) hi = tb;
  }
  t0 = lo;
  t1 = hi;
  return lo <= hi;
}

__device__ __forceinline__ PC cap_face_contact(V3 l, int a, float s, const float* h, float r, int f) {
  PC c;
  c.n = unitv(a) * s;
  const float ha = at3(h, a);
  c.phi = s * comp(l, a) - ha - r;
  V3 q = l;
  setc(q, a, s * ha);
  V3 wc = l - c.n * r;
  c.p = (q + wc) * 0.5f;
  c.f = f;
  return c;
}

// Capsule (first) vs box (second), in the box frame: exact minimum of the
// convex piecewise-quadratic squared distance of the core segment to the
// box; face-parallel cores give the clipped segment ends (f 0, 1); other
// separated cores one contact at the closest points (f 2); cores touching
// the box leave through the face of least translation (f 0, 1, or 3).
__device__ inline void capsule_box(const Geom& C, const Geom& B, float margin, Out4& out) {
  float r = C.p[0];
  const float* h = B.p;
  V3 P0, D;
  capsule_seg(C, P0, D);
  V3 p0 = RTv(B.R, P0 - B.x);
  V3 d = RTv(B.R, D);
  // breakpoints 0, 1 and the slab crossings inside (0, 1), in register
  // slots (unused slots hold +inf), sorted by a fixed network
  float ts[8];
#pragma unroll
  for (int k = 0; k < 8; k++) ts[k] = INFINITY;
  ts[0] = 0.f;
  ts[1] = 1.f;
  int nt = 2;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    float da = comp(d, a);
    if (da == 0.f) continue;
#pragma unroll
    for (int sg = -1; sg <= 1; sg += 2) {
      float t = fdiv((float)sg * h[a] - comp(p0, a), da);
      if (t > 0.f && t < 1.f) {
#pragma unroll
        for (int k = 2; k < 8; k++) ts[k] = k == nt ? t : ts[k];
        nt++;
      }
    }
  }
  {
    // Batcher's odd-even merge sort of 8 values: 19 compare-exchanges
    constexpr int kNet[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6}, {5, 7}, {1, 2}, {5, 6},
                                 {0, 4}, {1, 5}, {2, 6}, {3, 7}, {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
    for (int k = 0; k < 19; k++) {
      const float x = ts[kNet[k][0]], y = ts[kNet[k][1]];
      ts[kNet[k][0]] = fminf(x, y);
      ts[kNet[k][1]] = fmaxf(x, y);
    }
  }
  // candidates: breakpoints first, then each piece's vertex
  float bt = ts[0];
  float bg = box_d2(p0 + d * bt, h);
#pragma unroll
  for (int i = 1; i < 8; i++) {
    if (i >= nt) break;
    float g = box_d2(p0 + d * ts[i], h);
    if (g < bg || (g == bg && ts[i] < bt)) { bg = g; bt = ts[i]; }
  }
#pragma unroll
  for (int i = 0; i + 1 < 8; i++) {
    if (i + 1 >= nt) break;
    float tl = ts[i], th = ts[i + 1];
    if (!(th > tl)) continue;
    float tm = 0.5f * (tl + th), num = 0.f, den = 0.f;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      float la = comp(p0, a) + tm * comp(d, a), ca;
      if (la > h[a]) ca = h[a];
      else if (la < -h[a]) ca = -h[a];
      else continue;
      num += comp(d, a) * (ca - comp(p0, a));
      den += comp(d, a) * comp(d, a);
    }
    float tv = den > 0.f ? clampf(fdiv(num, den), tl, th) : tl;
    float g = box_d2(p0 + d * tv, h);
    if (g < bg || (g == bg && tv < bt)) { bg = g; bt = tv; }
  }
  V3 l = p0 + d * bt;
  Out4 loc;
  loc.n = 0;
  // the core meets the box iff the segment clipped to the three slabs
  // (Liang and Barsky 1984) is non-empty: a core passing through the box
  // is told apart by the clipped length, not by a crossing point's zero
  // distance, which rounding can leave slightly positive
  float t_in = 0.f, t_out = 1.f;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const float dk = comp(d, k), pk = comp(p0, k);
    if (dk == 0.f) {
      if (fabsf(pk) > h[k]) t_out = -1.f;
      continue;
    }
    const float u0 = fdiv(-h[k] - pk, dk), u1 = fdiv(h[k] - pk, dk);
    t_in = fmaxf(t_in, fminf(u0, u1));
    t_out = fminf(t_out, fmaxf(u0, u1));
  }
  const bool meets = t_in <= t_out || !(bg > 0.f);
  if (!meets) {
    float dist = fsqrt(bg);
    float dl = fsqrt(len2(d));
    int ncl = 0, a = -1;
#pragma unroll
    for (int k = 0; k < 3; k++)
      if (fabsf(comp(l, k)) > h[k]) { ncl++; a = k; }
    bool done = false;
    if (ncl == 1 && fabsf(comp(d, a)) <= kSinParallel * dl) {
      float sa = comp(l, a) > 0.f ? 1.f : -1.f;
      float t0, t1;
      if (clip_face(p0, d, h, a, t0, t1)) {
        loc.push(cap_face_contact(p0 + d * t0, a, sa, h, r, 0));
        if (t1 > t0) loc.push(cap_face_contact(p0 + d * t1, a, sa, h, r, 1));
        done = true;
      }
    }
    if (!done) {
      V3 q = v3(clampf(l.x, -h[0], h[0]), clampf(l.y, -h[1], h[1]), clampf(l.z, -h[2], h[2]));
      PC c;
      c.n = (l - q) * frcpg(dist);
      c.phi = dist - r;
      c.p = (q + (l - c.n * r)) * 0.5f;
      c.f = 2;
      loc.push(c);
    }
  } else {
    V3 p1 = p0 + d;
    float best = INFINITY;
    int ba = 0;
    float bs = 1.f;
#pragma unroll
    for (int a = 0; a < 3; a++) {
#pragma unroll
      for (int sg = 1; sg >= -1; sg -= 2) {
        float ex = h[a] - fminf((float)sg * comp(p0, a), (float)sg * comp(p1, a));
        if (ex < best) { best = ex; ba = a; bs = (float)sg; }
      }
    }
    float t0, t1;
    if (clip_face(p0, d, h, ba, t0, t1)) {
      loc.push(cap_face_contact(p0 + d * t0, ba, bs, h, r, 0));
      if (t1 > t0) loc.push(cap_face_contact(p0 + d * t1, ba, bs, h, r, 1));
    } else {
      float e0 = bs * comp(p0, ba), e1 = bs * comp(p1, ba);
      loc.push(cap_face_contact(e0 <= e1 ? p0 : p1, ba, bs, h, r, 3));
    }
  }
#pragma unroll
  for (int k = 0; k < 2; k++) {
    if (k >= loc.n) break;
    PC c = loc.get(k);
    if (!(c.phi <= margin)) continue;
    c.n = Rv(B.R, c.n);
    c.p = B.x + Rv(B.R, c.p);
    out.push(c);
  }
}

// Box vs box: 15-axis separating-axis test; the first box's faces win near
// ties, edges only when clearly better; face contacts clip the incident face
// against the reference side planes (three-state: inside / on / outside)
// and keep at most 4 points; edge contacts use the closest edge points.
__device__ inline void box_box(const Geom& A, const Geom& B, float margin, Out4& out) {
  V3 a[3], b[3];
#pragma unroll
  for (int i = 0; i < 3; i++) { a[i] = col(A.R, i); b[i] = col(B.R, i); }
  const float* ha = A.p;
  const float* hb = B.p;
  V3 D = A.x - B.x;
  float smax = -INFINITY;
  int fa = 0, fb = 3, e = -1;
  float sfa = -INFINITY, sfb = -INFINITY, se = -INFINITY;
  float sgfa = 1.f, sgfb = 1.f, sge = 1.f;
  V3 ue = v3(0.f, 0.f, 1.f);
#pragma unroll
  for (int k = 0; k < 15; k++) {
    V3 u;
    float ra, rb;
    if (k < 3) {
      u = a[k];
      ra = ha[k];
      rb = hb[0] * fabsf(dot(b[0], u)) + hb[1] * fabsf(dot(b[1], u)) + hb[2] * fabsf(dot(b[2], u));
    } else if (k < 6) {
      u = b[k - 3];
      rb = hb[k - 3];
      ra = ha[0] * fabsf(dot(a[0], u)) + ha[1] * fabsf(dot(a[1], u)) + ha[2] * fabsf(dot(a[2], u));
    } else {
      V3 c = cross(a[(k - 6) / 3], b[(k - 6) % 3]);
      float L2 = len2(c);
      if (L2 < kEdgeDegenerate) continue;
      u = c * frsq(L2);
      ra = ha[0] * fabsf(dot(a[0], u)) + ha[1] * fabsf(dot(a[1], u)) + ha[2] * fabsf(dot(a[2], u));
      rb = hb[0] * fabsf(dot(b[0], u)) + hb[1] * fabsf(dot(b[1], u)) + hb[2] * fabsf(dot(b[2], u));
    }
    float dd = dot(D, u);
    float s = fabsf(dd) - ra - rb;
    float sg = dd >= 0.f ? 1.f : -1.f;
    smax = fmaxf(smax, s);
    if (k < 3) { if (s > sfa) { sfa = s; fa = k; sgfa = sg; } }
    else if (k < 6) { if (s > sfb) { sfb = s; fb = k; sgfb = sg; } }
    else if (s > se) { se = s; e = k; sge = sg; ue = u; }
  }
  if (smax > margin) return;
  float hmax = fmaxf(fmaxf(fmaxf(ha[0], ha[1]), fmaxf(ha[2], hb[0])), fmaxf(hb[1], hb[2]));
  int face = fa;
  float sface = sfa, sgf = sgfa;
  if (sfb > 0.95f * sfa + 0.01f * hmax) { face = fb; sface = sfb; sgf = sgfb; }
  if (e >= 0 && se > 0.95f * sface + 0.01f * hmax) {
    int i = (e - 6) / 3, j = (e - 6) % 3;
    V3 N = ue * sge;
    V3 pa = A.x, pb = B.x;
#pragma unroll
    for (int m = 0; m < 3; m++) {
      if (m != i) { float c = dot(N, a[m]); pa = pa + a[m] * (c > 0.f ? -ha[m] : ha[m]); }
      if (m != j) { float c = dot(N, b[m]); pb = pb + b[m] * (c > 0.f ? hb[m] : -hb[m]); }
    }
    V3 w = pa - pb;
    const V3 ai = sel3(a[0], a[1], a[2], i), bj = sel3(b[0], b[1], b[2], j);
    const float hai = at3(ha, i), hbj = at3(hb, j);
    float bb = dot(ai, bj), dd = dot(ai, w), ee = dot(bj, w);
    float den = 1.0f - bb * bb;
    float ta = fdiv(bb * ee - dd, den);
    float tb = ee + ta * bb;
    ta = clampf(ta, -hai, hai);
    tb = clampf(tb, -hbj, hbj);
    V3 PA = pa + ai * ta, PB = pb + bj * tb;
    PC c;
    c.n = N;
    c.phi = dot(PA - PB, N);
    c.p = (PA + PB) * 0.5f;
    c.f = 0x80 | (e - 6);
    if (c.phi <= margin) out.push(c);
    return;
  }
  // face contact
  const bool refA = face < 3;
  const int ax = refA ? face : face - 3;
  // reference and incident boxes' axes and half-extents, selected slot by
  // slot and read with runtime indices through selects (no scratch)
  V3 rc[3], ic[3];
  float hr[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    rc[k] = selv(refA, a[k], b[k]);
    ic[k] = selv(refA, b[k], a[k]);
    hr[k] = refA ? ha[k] : hb[k];
    hi[k] = refA ? hb[k] : ha[k];
  }
  const V3 refx = selv(refA, A.x, B.x), incx = selv(refA, B.x, A.x);
  const V3 rax = sel3(rc[0], rc[1], rc[2], ax);
  V3 N = rax * sgf;                        // from B to A
  V3 nout = refA ? -N : N;                 // reference face normal, towards the incident box
  int side = dot(nout, rax) > 0.f ? 0 : 1;
  int refface = ax * 2 + side;
  V3 cref = refx + nout * at3(hr, ax);
  int j = 0;
  float best = fabsf(dot(ic[0], nout));
  float c1 = fabsf(dot(ic[1], nout)), c2 = fabsf(dot(ic[2], nout));
  if (c1 > best) { best = c1; j = 1; }
  if (c2 > best) { best = c2; j = 2; }
  const V3 icj = sel3(ic[0], ic[1], ic[2], j);
  float si = dot(icj, nout) > 0.f ? -1.f : 1.f;
  int j1 = j == 2 ? 0 : j + 1, j2 = j == 0 ? 2 : j - 1;
  V3 fc = incx + icj * (si * at3(hi, j));
  V3 e1 = sel3(ic[0], ic[1], ic[2], j1) * at3(hi, j1), e2 = sel3(ic[0], ic[1], ic[2], j2) * at3(hi, j2);
  // polygons in fixed register slots: every access is an unrolled select
  Poly8 poly, tmp;
  int np = 4;
  poly.v[0] = (fc + e1) + e2;
  poly.v[1] = (fc - e1) + e2;
  poly.v[2] = (fc - e1) - e2;
  poly.v[3] = (fc + e1) - e2;
  const int r1 = ax == 2 ? 0 : ax + 1, r2 = ax == 0 ? 2 : ax - 1;
#pragma unroll
  for (int pl = 0; pl < 4; pl++) {
    if (np == 0) break;
    int pa = pl < 2 ? r1 : r2;
    const V3 rpa = sel3(rc[0], rc[1], rc[2], pa);
    V3 pn = (pl & 1) ? -rpa : rpa;
    float off = at3(hr, pa);
    int no = 0;
    V3 prev = poly.get(np - 1);
    float dp = dot(prev - refx, pn) - off;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (k < np) {
        V3 cur = poly.v[k];
        float dc = dot(cur - refx, pn) - off;
        int cs = dc < -kClipOn ? -1 : (dc > kClipOn ? 1 : 0);
        int ps = dp < -kClipOn ? -1 : (dp > kClipOn ? 1 : 0);
        if (ps * cs < 0 && no < 8) tmp.set(no++, prev + (cur - prev) * fdiv(dp, dp - dc));
        if (cs <= 0 && no < 8) tmp.set(no++, cur);
        prev = cur;
        dp = dc;
      }
    }
    np = no;
    poly = tmp;
  }
  float ph[8];
  int nk = 0;
  unsigned keepm = 0u;
#pragma unroll
  for (int k = 0; k < 8; k++) {
    ph[k] = 0.f;
    if (k < np) {
      ph[k] = dot(poly.v[k] - cref, nout);
      if (ph[k] <= margin) { keepm |= 1u << k; nk++; }
    }
  }
  unsigned sel = keepm;
  if (nk > 4) {
    // first kept point; farthest from it; largest triangle; largest quad
    int i1 = __builtin_ctz(keepm);
    unsigned used = 1u << i1;
    const V3 p1 = poly.get(i1);
    int i2 = -1;
    float bd = -1.f;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (k >= np || !((keepm >> k) & 1u) || ((used >> k) & 1u)) continue;
      float dd = fsqrt(len2(poly.v[k] - p1));
      if (dd > bd) { bd = dd; i2 = k; }
    }
    used |= 1u << i2;
    const V3 p2 = poly.get(i2);
    V3 e12 = p2 - p1;
    int i3 = -1;
    float ba = -1.f;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (k >= np || !((keepm >> k) & 1u) || ((used >> k) & 1u)) continue;
      float ar = fsqrt(len2(cross(e12, poly.v[k] - p1)));
      if (ar > ba) { ba = ar; i3 = k; }
    }
    used |= 1u << i3;
    const V3 p3 = poly.get(i3);
    V3 e23 = p3 - p2, e31 = p1 - p3;
    int i4 = -1;
    float bq = -1.f;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (k >= np || !((keepm >> k) & 1u) || ((used >> k) & 1u)) continue;
      float sc = fsqrt(len2(cross(e12, poly.v[k] - p1))) + fsqrt(len2(cross(e23, poly.v[k] - p2))) +
                 fsqrt(len2(cross(e31, poly.v[k] - p3)));
      if (sc > bq) { bq = sc; i4 = k; }
    }
    used |= 1u << i4;
    sel = used;
  }
#pragma unroll
  for (int k = 0; k < 8; k++) {
    if (k >= np || !((sel >> k) & 1u)) continue;
    PC c;
    c.n = N;
    c.phi = ph[k];
    c.p = poly.v[k] - nout * (0.5f * ph[k]);
    c.f = (refA ? 0 : 1) | (refface << 1) | (k << 4);
    out.push(c);
  }
}

// Ground plane z = 0 (second) vs a body (first).
__device__ inline void ground_contacts(const Geom& A, float margin, Out4& out) {
  const V3 up = v3(0.f, 0.f, 1.f);
  if (A.shape == SPHERE) {
    PC c;
    c.n = up;
    c.phi = A.x.z - A.p[0];
    c.p = v3(A.x.x, A.x.y, 0.5f * (A.x.z - A.p[0]));
    c.f = 0;
    if (c.phi <= margin) out.push(c);
  } else if (A.shape == CAPSULE) {
    V3 p0, d;
    capsule_seg(A, p0, d);
#pragma unroll
    for (int k = 0; k < 2; k++) {
      V3 e = k == 0 ? p0 : p0 + d;
      PC c;
      c.n = up;
      c.phi = e.z - A.p[0];
      c.p = v3(e.x, e.y, 0.5f * (e.z - A.p[0]));
      c.f = k;
      if (c.phi <= margin) out.push(c);
    }
  } else {
    // corners with depth <= margin; at most the 4 deepest (ties: lower index)
    float zc[8];
    V3 cn[8];
    unsigned keepm = 0u;
    int m = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      V3 off = v3((k & 1) ? A.p[0] : -A.p[0], (k & 2) ? A.p[1] : -A.p[1], (k & 4) ? A.p[2] : -A.p[2]);
      cn[k] = A.x + Rv(A.R, off);
      zc[k] = cn[k].z;
      if (zc[k] <= margin) { keepm |= 1u << k; m++; }
    }
    if (m > 4) {
      unsigned sel = 0u;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        int bi = -1;
        float bz = 0.f;
#pragma unroll
        for (int k = 0; k < 8; k++) {
          if (!((keepm >> k) & 1u) || ((sel >> k) & 1u)) continue;
          if (bi < 0 || zc[k] < bz) { bi = k; bz = zc[k]; }
        }
        sel |= 1u << bi;
      }
      keepm = sel;
    }
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (!((keepm >> k) & 1u)) continue;
      PC c;
      c.n = up;
      c.phi = zc[k];
      c.p = v3(cn[k].x, cn[k].y, 0.5f * cn[k].z);
      c.f = k;
      out.push(c);
    }
  }
}

// Contacts of the pair (A, B), normal from B to A.
__device__ inline void collide(const Geom& A, const Geom& B, float margin, Out4& out) {
  int ta = A.shape, tb = B.shape;
  bool flip = false;
  if (ta == SPHERE && tb == SPHERE) {
    PC c = sphere_sphere(A.x, A.p[0], B.x, B.p[0], 0);
    if (c.phi <= margin) out.push(c);
  } else if (ta == SPHERE && tb == BOX) sphere_box(A, B, margin, out);
  else if (ta == BOX && tb == SPHERE) { sphere_box(B, A, margin, out); flip = true; }
  else if (ta == SPHERE && tb == CAPSULE) sphere_capsule(A, B, margin, out);
  else if (ta == CAPSULE && tb == SPHERE) { sphere_capsule(B, A, margin, out); flip = true; }
  else if (ta == CAPSULE && tb == BOX) capsule_box(A, B, margin, out);
  else if (ta == BOX && tb == CAPSULE) { capsule_box(B, A, margin, out); flip = true; }
  else if (ta == BOX && tb == BOX) box_box(A, B, margin, out);
  else capsule_capsule(A, B, margin, out);
  if (flip) out.flip();
}

}  // namespace rbs

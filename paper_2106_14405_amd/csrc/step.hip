// step.hip -- one physics step (s_t, a_t) -> s_{t+1} for a batch of
// independent scenes, one workgroup per scene, the scene's working set
// resident in LDS (gfx950: 160 KB per CU).
//
// Phases of one scene (barrier between phases):
//  a1 arm forward kinematics at theta_t and link velocities from actions
//  a2 v += g dt for dynamic bodies; world inverse inertia R diag(I^-1) R^T
//  a3 fattened AABBs and orderable sort keys of the AABB minimum along x
//  a4 stable LSD radix sort of (key, body) in LDS, 8-bit digits, wave ballots
//  a5 sweep along x -> candidate pairs (y/z overlap, at least one dynamic),
//     ground pairs; radix sort of pair keys -> canonical (i, j) order
//  a6 narrowphase, one lane per pair, wave ballot/mbcnt compaction of the
//     0..4 contacts per pair into the canonical contact list
//  a7 previous-step impulses by binary search of the sorted cache keys
//  a9 first-fit colouring as the parallel fixed point of
//     c_q = mex{ c_p : p < q shares a dynamic body with q }, then a stable
//     one-digit radix sort into colour-major order
//  a10 constraint setup; a11 projected Gauss-Seidel (or Jacobi) sweeps,
//     one barrier per colour, max-residual reduction per sweep
//  a12 semi-implicit position/orientation update; arm theta update + FK
//  a13 cache, contact export, arm contact force, per-scene stats
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "geom.h"
#include "mlp_infer.h"
#include "sim_internal.h"

namespace rbs {

typedef unsigned long long u64;

// misc word slots
enum {
  M_NPAIRS = 0, M_NCONT = 1, M_FLAGS = 2, M_NCOL = 3, M_RES = 4, M_CHANGED = 5, M_SWEEPS = 6,
  M_NPREV = 7, M_STOP = 8, M_WAVE = 16,  // per-wave partials from here (<= 4 waves * 4)
  M_COLSTART = 32                        // unused by kernels with > 31 colours; see cstart
};

__device__ __forceinline__ unsigned lanes_below(u64 m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ uint32_t orderable(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Stable LSD radix sort of n (key, value) pairs held in LDS, `passes`
// 8-bit digits from bit `shift0`.  Ranks within a wave come from eight
// ballots that isolate the lanes holding the same digit.  Returns 1 if the
// sorted data ended in (k1, v1), 0 if in (k0, v0).
__device__ int lds_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int n, int shift0, int passes,
                              uint32_t* hist, uint32_t* base) {
  const int T = blockDim.x, tid = threadIdx.x, W = T >> 6, w = tid >> 6;
  int swapped = 0;
  for (int ps = 0; ps < passes; ps++) {
    const int sh = shift0 + 8 * ps;
    for (int i = tid; i < 256; i += T) base[i] = 0u;
    for (int i = tid; i < 256 * W; i += T) hist[i] = 0u;
    __syncthreads();
    for (int i = tid; i < n; i += T) atomicAdd(&base[(k0[i] >> sh) & 255u], 1u);
    __syncthreads();
    if (tid == 0) {
      uint32_t run = 0;
      for (int d = 0; d < 256; d++) { uint32_t c = base[d]; base[d] = run; run += c; }
    }
    __syncthreads();
    for (int t0 = 0; t0 < n; t0 += T) {
      const int i = t0 + tid;
      const bool valid = i < n;
      uint32_t key = valid ? k0[i] : 0u, val = valid ? v0[i] : 0u;
      uint32_t d = (key >> sh) & 255u;
      u64 peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; b++) {
        u64 bb = __ballot(valid && ((d >> b) & 1u));
        peers &= ((d >> b) & 1u) ? bb : ~bb;
      }
      unsigned rank = lanes_below(peers);
      if (valid && rank == 0) hist[w * 256 + d] = (uint32_t)__popcll(peers);
      __syncthreads();
      if (valid) {
        uint32_t off = base[d] + rank;
        for (int ww = 0; ww < w; ww++) off += hist[ww * 256 + d];
        k1[off] = key;
        v1[off] = val;
      }
      __syncthreads();
      for (int dd = tid; dd < 256; dd += T) {
        uint32_t s = 0;
        for (int ww = 0; ww < W; ww++) { s += hist[ww * 256 + dd]; hist[ww * 256 + dd] = 0u; }
        base[dd] += s;
      }
      __syncthreads();
    }
    uint32_t* t;
    t = k0; k0 = k1; k1 = t;
    t = v0; v0 = v1; v1 = t;
    swapped ^= 1;
  }
  return swapped;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

struct Smem {
  float* f;
  uint32_t* u;
};

__device__ __forceinline__ V3 ld3(const float* a, int stride, int i) { return v3(a[i], a[stride + i], a[2 * stride + i]); }
__device__ __forceinline__ void st3(float* a, int stride, int i, V3 v) {
  a[i] = v.x;
  a[stride + i] = v.y;
  a[2 * stride + i] = v.z;
}

// world inverse inertia (symmetric: xx yy zz xy xz yz) times a vector
__device__ __forceinline__ V3 Iw_mul(const float* I, int NB, int i, V3 a) {
  float xx = I[i], yy = I[NB + i], zz = I[2 * NB + i], xy = I[3 * NB + i], xz = I[4 * NB + i], yz = I[5 * NB + i];
  return v3(xx * a.x + xy * a.y + xz * a.z, xy * a.x + yy * a.y + yz * a.z, xz * a.x + yz * a.y + zz * a.z);
}

// Arm forward kinematics: joint axes z, y, z, y, z, y, z in each parent frame,
// link k spans joint k to joint k+1 along its local z.  Produces link centres
// c, orientations q (w x y z), world joint origins o and axes ax.
__device__ void arm_chain(const float* base, const float* th, const float* len, V3* c, float (*q)[4], V3* o, V3* ax) {
  float q0 = 1.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
  V3 p = v3(base[0], base[1], base[2]);
  for (int k = 0; k < 7; k++) {
    float sn, cs;
    sincosf(0.5f * th[k], &sn, &cs);
    // q (x) (cs, 0, 0, sn) for z joints; q (x) (cs, 0, sn, 0) for y joints
    float w, x, y, z;
    if ((k & 1) == 0) {
      w = q0 * cs - q3 * sn; x = q1 * cs + q2 * sn; y = q2 * cs - q1 * sn; z = q3 * cs + q0 * sn;
    } else {
      w = q0 * cs - q2 * sn; x = q1 * cs - q3 * sn; y = q2 * cs + q0 * sn; z = q3 * cs + q1 * sn;
    }
    q0 = w; q1 = x; q2 = y; q3 = z;
    M3 R = quat_R(w, x, y, z);
    V3 zl = col(R, 2);
    ax[k] = (k & 1) ? col(R, 1) : zl;
    o[k] = p;
    c[k] = p + zl * (0.5f * len[k]);
    q[k][0] = w; q[k][1] = x; q[k][2] = y; q[k][3] = z;
    p = p + zl * len[k];
  }
}

// Arm link poses (and, if thd, link velocities from joint velocities) into
// the LDS body slots b0..b0+6.
__device__ void arm_fk(const StepParams& P, const LdsLayout& L, Smem S, int NB, int b0, const float* base,
                       const float* th, const float* thd) {
  V3 c[7], o[7], ax[7];
  float q[7][4];
  arm_chain(base, th, P.link_len, c, q, o, ax);
  for (int k = 0; k < 7; k++) {
    int bi = b0 + k;
    st3(S.f + L.bx, NB, bi, c[k]);
    for (int j = 0; j < 4; j++) S.f[L.bq + j * NB + bi] = q[k][j];
    M3 R = quat_R(q[k][0], q[k][1], q[k][2], q[k][3]);
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
      for (int cc = 0; cc < 3; cc++) S.f[L.bR + (3 * r + cc) * NB + bi] = R.m[r][cc];
  }
  if (thd) {
    for (int k = 0; k < 7; k++) {
      V3 wv = v3(0.f, 0.f, 0.f), vv = v3(0.f, 0.f, 0.f);
      for (int j = 0; j <= k; j++) {
        wv = wv + ax[j] * thd[j];
        vv = vv + cross(ax[j], c[k] - o[j]) * thd[j];
      }
      st3(S.f + L.bv, NB, b0 + k, vv);
      st3(S.f + L.bw, NB, b0 + k, wv);
    }
  }
}

__device__ __forceinline__ Geom load_geom(const LdsLayout& L, Smem S, int NB, int i) {
  Geom g;
  g.shape = (int)(S.u[L.bmeta + i] & 255u);
  g.x = ld3(S.f + L.bx, NB, i);
#pragma unroll
  for (int r = 0; r < 3; r++)
#pragma unroll
    for (int c = 0; c < 3; c++) g.R.m[r][c] = S.f[L.bR + (3 * r + c) * NB + i];
  g.p[0] = S.f[L.bprm + i];
  g.p[1] = S.f[L.bprm + NB + i];
  g.p[2] = S.f[L.bprm + 2 * NB + i];
  return g;
}

// Velocity of body i at offset r (ground: zero).
__device__ __forceinline__ V3 point_vel(const LdsLayout& L, Smem S, int NB, int i, V3 r) {
  if (i == 0xFFFF) return v3(0.f, 0.f, 0.f);
  return ld3(S.f + L.bv, NB, i) + cross(ld3(S.f + L.bw, NB, i), r);
}

__device__ __forceinline__ bool is_dyn(const LdsLayout& L, Smem S, int i) {
  return i != 0xFFFF && ((S.u[L.bmeta + i] >> 8) & 255u) == DYNAMIC;
}

// Apply impulse P at the contact (onto a; -P onto b), dynamic bodies only.
__device__ __forceinline__ void apply_impulse(const LdsLayout& L, Smem S, int NB, int a, int b, V3 ra, V3 rb, V3 P) {
  if (is_dyn(L, S, a)) {
    float im = S.f[L.bim + a];
    st3(S.f + L.bv, NB, a, ld3(S.f + L.bv, NB, a) + P * im);
    st3(S.f + L.bw, NB, a, ld3(S.f + L.bw, NB, a) + Iw_mul(S.f + L.bI, NB, a, cross(ra, P)));
  }
  if (is_dyn(L, S, b)) {
    float im = S.f[L.bim + b];
    st3(S.f + L.bv, NB, b, ld3(S.f + L.bv, NB, b) - P * im);
    st3(S.f + L.bw, NB, b, ld3(S.f + L.bw, NB, b) - Iw_mul(S.f + L.bI, NB, b, cross(rb, P)));
  }
}

__device__ __forceinline__ void proj_disk(float& l1, float& l2, float lim) {
  float Ls = sqrtf(l1 * l1 + l2 * l2);
  if (Ls > lim) {
    if (Ls > 0.f) { float f = lim / Ls; l1 *= f; l2 *= f; }
    else { l1 = 0.f; l2 = 0.f; }
  }
}

// Contact q: bodies, offsets.
__device__ __forceinline__ void contact_geom(const LdsLayout& L, Smem S, int NB, int CM, int q, int& a, int& b, V3& n,
                                             V3& ra, V3& rb) {
  uint32_t ab = S.u[L.cab + q];
  a = (int)(ab & 0xFFFFu);
  b = (int)(ab >> 16);
  n = ld3(S.f + L.cn, CM, q);
  V3 p = ld3(S.f + L.cp, CM, q);
  ra = p - ld3(S.f + L.bx, NB, a);
  rb = b == 0xFFFF ? v3(0.f, 0.f, 0.f) : p - ld3(S.f + L.bx, NB, b);
}

// One Gauss-Seidel update of contact q: normal row, then both friction rows
// from the velocities after the normal update.  Returns max |dlambda| * k.
__device__ __forceinline__ float pgs_contact(const LdsLayout& L, Smem S, int NB, int CM, int q) {
  int a, b;
  V3 n, ra, rb;
  contact_geom(L, S, NB, CM, q, a, b, n, ra, rb);
  float mn = S.f[L.cm + q], m1 = S.f[L.cm + CM + q], m2 = S.f[L.cm + 2 * CM + q];
  float ln0 = S.f[L.clam + q], l10 = S.f[L.clam + CM + q], l20 = S.f[L.clam + 2 * CM + q];
  V3 vr = point_vel(L, S, NB, a, ra) - point_vel(L, S, NB, b, rb);
  float u = dot(n, vr);
  float ln = fmaxf(0.f, ln0 + mn * (S.f[L.cbias + q] - u));
  float dn = ln - ln0;
  apply_impulse(L, S, NB, a, b, ra, rb, n * dn);
  vr = point_vel(L, S, NB, a, ra) - point_vel(L, S, NB, b, rb);
  V3 t1, t2;
  tangents(n, t1, t2);
  float l1 = l10 - m1 * dot(t1, vr);
  float l2 = l20 - m2 * dot(t2, vr);
  proj_disk(l1, l2, S.f[L.cmu + q] * ln);
  float d1 = l1 - l10, d2 = l2 - l20;
  apply_impulse(L, S, NB, a, b, ra, rb, t1 * d1 + t2 * d2);
  S.f[L.clam + q] = ln;
  S.f[L.clam + CM + q] = l1;
  S.f[L.clam + 2 * CM + q] = l2;
  return fmaxf(fmaxf(fabsf(dn) / mn, fabsf(d1) / m1), fabsf(d2) / m2);
}

// Block-wide maximum of non-negative floats (one value per thread).
__device__ __forceinline__ float block_max(float v, uint32_t* misc) {
  const int tid = threadIdx.x, W = blockDim.x >> 6;
  v = wave_max(v);
  if ((tid & 63) == 0) misc[M_WAVE + (tid >> 6)] = __float_as_uint(v);
  __syncthreads();
  float r = 0.f;
  for (int w = 0; w < W; w++) r = fmaxf(r, __uint_as_float(misc[M_WAVE + w]));
  __syncthreads();
  return r;
}

// Colour-major pass applying the current impulses of every contact (warm start).
__device__ void apply_all(const LdsLayout& L, Smem S, int NB, int CM, int nc, int ncol, const uint32_t* cstart) {
  for (int c = 0; c < ncol; c++) {
    for (int i = (int)cstart[c] + threadIdx.x; i < (int)cstart[c + 1]; i += blockDim.x) {
      int q = (int)S.u[L.cperm + i];
      int a, b;
      V3 n, ra, rb;
      contact_geom(L, S, NB, CM, q, a, b, n, ra, rb);
      V3 t1, t2;
      tangents(n, t1, t2);
      V3 P = n * S.f[L.clam + q] + t1 * S.f[L.clam + CM + q] + t2 * S.f[L.clam + 2 * CM + q];
      apply_impulse(L, S, NB, a, b, ra, rb, P);
    }
    __syncthreads();
  }
}

__device__ float sweeps_pgs(const LdsLayout& L, Smem S, int NB, int CM, int ncol, const uint32_t* cstart) {
  float r = 0.f;
  for (int c = 0; c < ncol; c++) {
    for (int i = (int)cstart[c] + threadIdx.x; i < (int)cstart[c + 1]; i += blockDim.x)
      r = fmaxf(r, pgs_contact(L, S, NB, CM, (int)S.u[L.cperm + i]));
    __syncthreads();
  }
  return r;
}

// One Jacobi sweep: rows read the velocities of the sweep start, increments
// divided by max(n_a, n_b) contacts per dynamic body, applied colour-major.
__device__ float sweep_jacobi(const LdsLayout& L, Smem S, int NB, int CM, int nb, int nc, int ncol,
                              const uint32_t* cstart) {
  const int tid = threadIdx.x, T = blockDim.x;
  float* snap = S.f + L.snap;
  for (int i = tid; i < nb; i += T) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
      snap[k * NB + i] = S.f[L.bv + k * NB + i];
      snap[(3 + k) * NB + i] = S.f[L.bw + k * NB + i];
    }
  }
  __syncthreads();
  float r = 0.f;
  const uint32_t* deg = S.u + L.deg;
  for (int q = tid; q < nc; q += T) {
    int a, b;
    V3 n, ra, rb;
    contact_geom(L, S, NB, CM, q, a, b, n, ra, rb);
    V3 va = v3(snap[a], snap[NB + a], snap[2 * NB + a]) + cross(v3(snap[3 * NB + a], snap[4 * NB + a], snap[5 * NB + a]), ra);
    V3 vb = v3(0.f, 0.f, 0.f);
    if (b != 0xFFFF)
      vb = v3(snap[b], snap[NB + b], snap[2 * NB + b]) + cross(v3(snap[3 * NB + b], snap[4 * NB + b], snap[5 * NB + b]), rb);
    V3 vr = va - vb;
    int na = is_dyn(L, S, a) ? (int)deg[a] : 0;
    int nbb = is_dyn(L, S, b) ? (int)deg[b] : 0;
    float sc = 1.0f / (float)(na > nbb ? na : nbb);
    float mn = S.f[L.cm + q], m1 = S.f[L.cm + CM + q], m2 = S.f[L.cm + 2 * CM + q];
    float ln0 = S.f[L.clam + q], l10 = S.f[L.clam + CM + q], l20 = S.f[L.clam + 2 * CM + q];
    float ln = fmaxf(0.f, ln0 + sc * mn * (S.f[L.cbias + q] - dot(n, vr)));
    V3 t1, t2;
    tangents(n, t1, t2);
    float l1 = l10 - sc * m1 * dot(t1, vr);
    float l2 = l20 - sc * m2 * dot(t2, vr);
    proj_disk(l1, l2, S.f[L.cmu + q] * ln);
    float dn = ln - ln0, d1 = l1 - l10, d2 = l2 - l20;
    S.f[L.dl + q] = dn;
    S.f[L.dl + CM + q] = d1;
    S.f[L.dl + 2 * CM + q] = d2;
    S.f[L.clam + q] = ln;
    S.f[L.clam + CM + q] = l1;
    S.f[L.clam + 2 * CM + q] = l2;
    r = fmaxf(r, fmaxf(fmaxf(fabsf(dn) / mn, fabsf(d1) / m1), fabsf(d2) / m2));
  }
  __syncthreads();
  for (int c = 0; c < ncol; c++) {
    for (int i = (int)cstart[c] + tid; i < (int)cstart[c + 1]; i += T) {
      int q = (int)S.u[L.cperm + i];
      int a, b;
      V3 n, ra, rb;
      contact_geom(L, S, NB, CM, q, a, b, n, ra, rb);
      V3 t1, t2;
      tangents(n, t1, t2);
      apply_impulse(L, S, NB, a, b, ra, rb, n * S.f[L.dl + q]);
      apply_impulse(L, S, NB, a, b, ra, rb, t1 * S.f[L.dl + CM + q] + t2 * S.f[L.dl + 2 * CM + q]);
    }
    __syncthreads();
  }
  return r;
}

__global__ __launch_bounds__(256) void step_kernel(StepParams P, LdsLayout L) {
  extern __shared__ float smem_f[];
  Smem S{smem_f, reinterpret_cast<uint32_t*>(smem_f)};
  const int tid = threadIdx.x, T = blockDim.x;
  const int s = P.scene_list ? P.scene_list[blockIdx.x] : (int)blockIdx.x;
  const int b0 = P.body_offset[s];
  const int nb = P.body_offset[s + 1] - b0;
  const int NB = P.NB, PM = P.PM, CM = P.CM;
  const long N = P.n_bodies;
  uint32_t* misc = S.u + L.misc;
  const float dt = P.dt;
  if (nb > NB) {  // host guarantees otherwise; leave the scene untouched
    if (tid == 0) P.st_flags[s] = FLAG_CAPACITY;
    return;
  }
  if (tid < kMiscWords) misc[tid] = 0u;

  // ---- load bodies (a2) ------------------------------------------------
  const V3 g = v3(P.gx, P.gy, P.gz);
  for (int i = tid; i < nb; i += T) {
    const long gi = b0 + i;
    int shape = P.shape[gi], motion = P.motion[gi];
    S.u[L.bmeta + i] = (uint32_t)shape | ((uint32_t)motion << 8);
    V3 x = v3(P.pose[gi], P.pose[N + gi], P.pose[2 * N + gi]);
    float qw = P.pose[3 * N + gi], qx = P.pose[4 * N + gi], qy = P.pose[5 * N + gi], qz = P.pose[6 * N + gi];
    st3(S.f + L.bx, NB, i, x);
    S.f[L.bq + i] = qw; S.f[L.bq + NB + i] = qx; S.f[L.bq + 2 * NB + i] = qy; S.f[L.bq + 3 * NB + i] = qz;
    M3 R = quat_R(qw, qx, qy, qz);
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
      for (int c = 0; c < 3; c++) S.f[L.bR + (3 * r + c) * NB + i] = R.m[r][c];
    V3 v = v3(P.vel[gi], P.vel[N + gi], P.vel[2 * N + gi]);
    V3 w = v3(P.vel[3 * N + gi], P.vel[4 * N + gi], P.vel[5 * N + gi]);
    float im = 0.f;
    float I[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (motion == DYNAMIC) {
      im = P.inv_mass[gi];
      v = v + g * dt;
      float i0 = P.inv_inertia[gi], i1 = P.inv_inertia[N + gi], i2 = P.inv_inertia[2 * N + gi];
      // R diag(i) R^T
      I[0] = R.m[0][0] * R.m[0][0] * i0 + R.m[0][1] * R.m[0][1] * i1 + R.m[0][2] * R.m[0][2] * i2;
      I[1] = R.m[1][0] * R.m[1][0] * i0 + R.m[1][1] * R.m[1][1] * i1 + R.m[1][2] * R.m[1][2] * i2;
      I[2] = R.m[2][0] * R.m[2][0] * i0 + R.m[2][1] * R.m[2][1] * i1 + R.m[2][2] * R.m[2][2] * i2;
      I[3] = R.m[0][0] * R.m[1][0] * i0 + R.m[0][1] * R.m[1][1] * i1 + R.m[0][2] * R.m[1][2] * i2;
      I[4] = R.m[0][0] * R.m[2][0] * i0 + R.m[0][1] * R.m[2][1] * i1 + R.m[0][2] * R.m[2][2] * i2;
      I[5] = R.m[1][0] * R.m[2][0] * i0 + R.m[1][1] * R.m[2][1] * i1 + R.m[1][2] * R.m[2][2] * i2;
    } else if (motion == STATIC) {
      v = v3(0.f, 0.f, 0.f);
      w = v3(0.f, 0.f, 0.f);
    }
    st3(S.f + L.bv, NB, i, v);
    st3(S.f + L.bw, NB, i, w);
    S.f[L.bim + i] = im;
#pragma unroll
    for (int k = 0; k < 6; k++) S.f[L.bI + k * NB + i] = I[k];
    S.f[L.bprm + i] = P.prm[gi];
    S.f[L.bprm + NB + i] = P.prm[N + gi];
    S.f[L.bprm + 2 * NB + i] = P.prm[2 * N + gi];
    S.f[L.bmu + i] = P.friction[gi];
    S.f[L.be + i] = P.restitution[gi];
  }
  __syncthreads();
  // ---- a1: arm at theta_t, link velocities from the actions -------------
  float thd[7];
  if (P.arm) {
#pragma unroll
    for (int k = 0; k < 7; k++) thd[k] = P.actions ? P.actions[7 * s + k] : 0.f;
    if (tid == 0) arm_fk(P, L, S, NB, nb - 7, P.arm_base + 3 * s, P.theta + 7 * s, thd);
    __syncthreads();
  }

  // ---- a3: AABBs and sort keys ------------------------------------------
  for (int i = tid; i < nb; i += T) {
    Geom G = load_geom(L, S, NB, i);
    V3 lo, hi;
    if (G.shape == SPHERE) {
      float e = G.p[0] + P.margin;
      lo = G.x - v3(e, e, e);
      hi = G.x + v3(e, e, e);
    } else if (G.shape == BOX) {
      V3 e;
      e.x = fabsf(G.R.m[0][0]) * G.p[0] + fabsf(G.R.m[0][1]) * G.p[1] + fabsf(G.R.m[0][2]) * G.p[2] + P.margin;
      e.y = fabsf(G.R.m[1][0]) * G.p[0] + fabsf(G.R.m[1][1]) * G.p[1] + fabsf(G.R.m[1][2]) * G.p[2] + P.margin;
      e.z = fabsf(G.R.m[2][0]) * G.p[0] + fabsf(G.R.m[2][1]) * G.p[1] + fabsf(G.R.m[2][2]) * G.p[2] + P.margin;
      lo = G.x - e;
      hi = G.x + e;
    } else {
      V3 axv = col(G.R, 2) * G.p[1];
      V3 e0 = G.x - axv, e1 = G.x + axv;
      float r = G.p[0] + P.margin;
      lo = v3(fminf(e0.x, e1.x) - r, fminf(e0.y, e1.y) - r, fminf(e0.z, e1.z) - r);
      hi = v3(fmaxf(e0.x, e1.x) + r, fmaxf(e0.y, e1.y) + r, fmaxf(e0.z, e1.z) + r);
    }
    st3(S.f + L.lo, NB, i, lo);
    st3(S.f + L.hi, NB, i, hi);
    S.u[L.skey + i] = orderable(lo.x);
    S.u[L.sval + i] = (uint32_t)i;
  }
  __syncthreads();

  // ---- a4: radix sort bodies by AABB minimum along x --------------------
  int sw = lds_radix_sort(S.u + L.skey, S.u + L.sval, S.u + L.skey2, S.u + L.sval2, nb, 0, 4, S.u + L.hist,
                          S.u + L.hbase);
  const uint32_t* order = S.u + (sw ? L.sval2 : L.sval);

  // ---- a5: sweep and prune -> pairs (unordered), then canonical sort ----
  uint32_t* pk = S.u + L.pk;
  for (int p = tid; p < nb; p += T) {
    int i = (int)order[p];
    float hix = S.f[L.hi + i];
    V3 loi = ld3(S.f + L.lo, NB, i), hii = ld3(S.f + L.hi, NB, i);
    bool di = is_dyn(L, S, i);
    for (int q = p + 1; q < nb; q++) {
      int j = (int)order[q];
      if (S.f[L.lo + j] > hix) break;
      if (!di && !is_dyn(L, S, j)) continue;
      V3 loj = ld3(S.f + L.lo, NB, j), hij = ld3(S.f + L.hi, NB, j);
      if (loj.y <= hii.y && loi.y <= hij.y && loj.z <= hii.z && loi.z <= hij.z) {
        int a = i < j ? i : j, bb = i < j ? j : i;
        uint32_t slot = atomicAdd(&misc[M_NPAIRS], 1u);
        if ((int)slot < PM) pk[slot] = ((uint32_t)a << 11) | (uint32_t)bb;
      }
    }
    if (di && loi.z <= 0.f) {
      uint32_t slot = atomicAdd(&misc[M_NPAIRS], 1u);
      if ((int)slot < PM) pk[slot] = ((uint32_t)i << 11) | 2047u;
    }
  }
  __syncthreads();
  const int npairs_all = (int)misc[M_NPAIRS];
  const int np = npairs_all < PM ? npairs_all : PM;
  if (npairs_all > PM && tid == 0) misc[M_FLAGS] |= FLAG_CAPACITY;
  // keys are unique: sort keys only (values unused -> sort into the same buffer pair)
  int swp = lds_radix_sort(pk, pk, S.u + L.pk2, S.u + L.pk2, np, 0, 3, S.u + L.hist, S.u + L.hbase);
  const uint32_t* pairs = swp ? S.u + L.pk2 : pk;
  if (P.export_on) {
    for (int p = tid; p < np; p += T) {
      uint32_t k = pairs[p];
      uint32_t a = k >> 11, bb = k & 2047u;
      P.x_pair[(long)s * PM + p] = (a << 16) | (bb == 2047u ? kGroundPair : bb);
    }
  }

  // ---- a6: narrowphase, compaction in canonical order --------------------
  {
    const int lane = tid & 63, w = tid >> 6, W = T >> 6;
    uint32_t base = 0;
    for (int t0 = 0; t0 < np; t0 += T) {
      int p = t0 + tid;
      PC pc[4];
      int cnt = 0;
      int a = 0, bb = 0;
      if (p < np) {
        uint32_t k = pairs[p];
        a = (int)(k >> 11);
        bb = (int)(k & 2047u);
        Geom A = load_geom(L, S, NB, a);
        if (bb == 2047) {
          cnt = ground_contacts(A, P.margin, pc);
        } else {
          Geom B = load_geom(L, S, NB, bb);
          cnt = collide(A, B, P.margin, pc);
        }
      }
      // prefix of the counts (0..4) with three ballots per wave
      u64 b0m = __ballot(cnt & 1), b1m = __ballot((cnt >> 1) & 1), b2m = __ballot((cnt >> 2) & 1);
      uint32_t pre = lanes_below(b0m) + 2u * lanes_below(b1m) + 4u * lanes_below(b2m);
      uint32_t wtot = (uint32_t)(__popcll(b0m) + 2 * __popcll(b1m) + 4 * __popcll(b2m));
      if (lane == 0) misc[M_WAVE + w] = wtot;
      __syncthreads();
      uint32_t off = base + pre;
      uint32_t tile = 0;
      for (int ww = 0; ww < W; ww++) {
        uint32_t t = misc[M_WAVE + ww];
        if (ww < w) off += t;
        tile += t;
      }
      for (int k = 0; k < cnt; k++) {
        uint32_t q = off + (uint32_t)k;
        if ((int)q < CM) {
          uint32_t bkey = bb == 2047 ? kGroundKey : (uint32_t)bb;
          S.u[L.ckey + q] = ((uint32_t)a << 20) | (bkey << 8) | (uint32_t)pc[k].f;
          S.u[L.cab + q] = (uint32_t)a | ((uint32_t)(bb == 2047 ? 0xFFFF : bb) << 16);
          st3(S.f + L.cn, CM, q, pc[k].n);
          st3(S.f + L.cp, CM, q, pc[k].p);
          S.f[L.cphi + q] = pc[k].phi;
        }
      }
      base += tile;
      __syncthreads();
    }
    if (tid == 0) {
      misc[M_NCONT] = base;
      if ((int)base > CM) misc[M_FLAGS] |= FLAG_CAPACITY;
    }
  }
  __syncthreads();
  const int nc_all = (int)misc[M_NCONT];
  const int nc = nc_all < CM ? nc_all : CM;

  // ---- a7/a10: previous impulses, constraint setup ----------------------
  const int nprev = P.prev_count ? (P.prev_count[s] < CM ? P.prev_count[s] : CM) : 0;
  for (int i = tid; i < nprev; i += T) S.u[L.prevk + i] = P.prev_key[(long)s * CM + i];
  __syncthreads();
  const float gmag = sqrtf(P.gx * P.gx + P.gy * P.gy + P.gz * P.gz);
  for (int q = tid; q < nc; q += T) {
    int a, b;
    V3 n, ra, rb;
    contact_geom(L, S, NB, CM, q, a, b, n, ra, rb);
    float mub = b == 0xFFFF ? P.ground_mu : S.f[L.bmu + b];
    float eb = b == 0xFFFF ? P.ground_e : S.f[L.be + b];
    float mu = sqrtf(S.f[L.bmu + a] * mub);
    float e = fmaxf(S.f[L.be + a], eb);
    V3 t1, t2;
    tangents(n, t1, t2);
    float k3[3];
    V3 dirs[3] = {n, t1, t2};
#pragma unroll
    for (int r = 0; r < 3; r++) {
      V3 ca = cross(ra, dirs[r]);
      float k = S.f[L.bim + a] + dot(ca, Iw_mul(S.f + L.bI, NB, a, ca));
      if (b != 0xFFFF) {
        V3 cb = cross(rb, dirs[r]);
        k += S.f[L.bim + b] + dot(cb, Iw_mul(S.f + L.bI, NB, b, cb));
      }
      k3[r] = k;
      S.f[L.cm + r * CM + q] = 1.0f / k;
    }
    V3 vr = point_vel(L, S, NB, a, ra) - point_vel(L, S, NB, b, rb);
    float u0 = dot(n, vr);
    float phi = S.f[L.cphi + q];
    float bias = phi > 0.f ? -phi / dt : P.baumgarte / dt * fmaxf(0.f, -phi - P.slop);
    if (e > 0.f && u0 < -P.rest_thresh) bias = fmaxf(bias, -e * u0);
    S.f[L.cbias + q] = bias;
    S.f[L.cmu + q] = mu;
    // previous impulse by binary search of the sorted previous keys
    uint32_t key = S.u[L.ckey + q];
    int lo = 0, hi = nprev - 1, hit = -1;
    while (lo <= hi) {
      int mid = (lo + hi) >> 1;
      uint32_t km = S.u[L.prevk + mid];
      if (km == key) { hit = mid; break; }
      if (km < key) lo = mid + 1; else hi = mid - 1;
    }
    float lp0 = 0.f, lp1 = 0.f, lp2 = 0.f;
    if (hit >= 0) {
      long o = (long)s * CM + hit;
      V3 F = v3(P.prev_lam[P.scene_cm + o], P.prev_lam[2 * P.scene_cm + o], P.prev_lam[3 * P.scene_cm + o]);
      lp0 = P.prev_lam[o];
      lp1 = dot(F, t1);
      lp2 = dot(F, t2);
    }
    float l0 = 0.f, l1 = 0.f, l2 = 0.f;
    float feat[16];
    const bool need_feat = P.warm == WARM_LEARNED || (P.export_on && P.x_feat);
    if (need_feat) {
      feat[0] = u0;
      feat[1] = dot(t1, vr);
      feat[2] = dot(t2, vr);
      feat[3] = -phi;
      feat[4] = S.f[L.bim + a];
      feat[5] = b == 0xFFFF ? 0.f : S.f[L.bim + b];
      V3 can = cross(ra, n);
      feat[6] = dot(can, Iw_mul(S.f + L.bI, NB, a, can));
      if (b != 0xFFFF) {
        V3 cbn = cross(rb, n);
        feat[7] = dot(cbn, Iw_mul(S.f + L.bI, NB, b, cbn));
      } else {
        feat[7] = 0.f;
      }
      feat[8] = lp0; feat[9] = lp1; feat[10] = lp2;
      feat[11] = n.x; feat[12] = n.y; feat[13] = n.z;
      feat[14] = mu;
      feat[15] = hit >= 0 ? 1.f : 0.f;
      if (P.export_on && P.x_feat)
        for (int k = 0; k < 16; k++) P.x_feat[k * P.scene_cm + (long)s * CM + q] = feat[k];
    }
    if (P.warm == WARM_PREV) {
      l0 = lp0; l1 = lp1; l2 = lp2;
    } else if (P.warm == WARM_LEARNED) {
      float y[3];
      mlp_contact(P.mlp, feat, y);
      float sc = gmag * dt / k3[0];
      l0 = y[0] * sc; l1 = y[1] * sc; l2 = y[2] * sc;
    }
    // projection of the initial impulse
    l0 = fmaxf(l0, 0.f);
    proj_disk(l1, l2, mu * l0);
    S.f[L.clam + q] = l0;
    S.f[L.clam + CM + q] = l1;
    S.f[L.clam + 2 * CM + q] = l2;
  }
  __syncthreads();

  // ---- a9: colouring -----------------------------------------------------
  // per-body lists of contacts (dynamic bodies only), canonical order
  uint32_t* deg = S.u + L.deg;
  uint32_t* lstart = S.u + L.lstart;
  uint32_t* list = S.u + L.list;
  for (int i = tid; i <= nb; i += T) deg[i] = 0u;
  __syncthreads();
  for (int q = tid; q < nc; q += T) {
    uint32_t ab = S.u[L.cab + q];
    int a = (int)(ab & 0xFFFFu), b = (int)(ab >> 16);
    if (is_dyn(L, S, a)) atomicAdd(&deg[a], 1u);
    if (is_dyn(L, S, b)) atomicAdd(&deg[b], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int i = 0; i < nb; i++) { lstart[i] = run; run += deg[i]; }
    lstart[nb] = run;
  }
  __syncthreads();
  // fill: slot of contact q in body a's list = number of earlier contacts of a;
  // lists are built unordered and insertion-sorted per body
  for (int i = tid; i < nb; i += T) deg[i] = 0u;
  __syncthreads();
  for (int q = tid; q < nc; q += T) {
    uint32_t ab = S.u[L.cab + q];
    int a = (int)(ab & 0xFFFFu), b = (int)(ab >> 16);
    if (is_dyn(L, S, a)) list[lstart[a] + atomicAdd(&deg[a], 1u)] = (uint32_t)q;
    if (is_dyn(L, S, b)) list[lstart[b] + atomicAdd(&deg[b], 1u)] = (uint32_t)q;
  }
  __syncthreads();
  for (int i = tid; i < nb; i += T) {
    uint32_t s0 = lstart[i], e0 = lstart[i + 1];
    for (uint32_t x = s0 + 1; x < e0; x++) {
      uint32_t v = list[x];
      uint32_t y = x;
      while (y > s0 && list[y - 1] > v) { list[y] = list[y - 1]; y--; }
      list[y] = v;
    }
  }
  uint32_t* colour = S.u + L.ck0;
  for (int q = tid; q < nc; q += T) colour[q] = 0u;
  __syncthreads();
  // fixed point of c_q = mex{c_p : p < q, p shares a dynamic body with q};
  // its unique solution is sequential first fit in canonical order
  for (int round = 0; round < nc + 2; round++) {
    if (tid == 0) misc[M_CHANGED] = 0u;
    __syncthreads();
    bool changed = false;
    for (int q = tid; q < nc; q += T) {
      uint32_t ab = S.u[L.cab + q];
      int ids[2] = {(int)(ab & 0xFFFFu), (int)(ab >> 16)};
      uint32_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;
      for (int t = 0; t < 2; t++) {
        int i = ids[t];
        if (!is_dyn(L, S, i)) continue;
        for (uint32_t x = lstart[i]; x < lstart[i + 1]; x++) {
          uint32_t p = list[x];
          if ((int)p >= q) break;
          uint32_t c = colour[p];
          if (c < 32) m0 |= 1u << c;
          else if (c < 64) m1 |= 1u << (c - 32);
          else if (c < 96) m2 |= 1u << (c - 64);
          else m3 |= 1u << (c - 96);
        }
      }
      uint32_t c;
      if (~m0) c = __builtin_ctz(~m0);
      else if (~m1) c = 32 + __builtin_ctz(~m1);
      else if (~m2) c = 64 + __builtin_ctz(~m2);
      else if (~m3) c = 96 + __builtin_ctz(~m3);
      else c = kMaxColours - 1;  // overflow: flagged below
      if (c != colour[q]) { colour[q] = c; changed = true; }
    }
    if (changed) misc[M_CHANGED] = 1u;
    __syncthreads();
    if (misc[M_CHANGED] == 0u) break;
    __syncthreads();
  }
  // colour overflow check (a contact whose earlier neighbours use all colours)
  for (int q = tid; q < nc; q += T)
    if (colour[q] == kMaxColours - 1) atomicOr(&misc[M_FLAGS], (uint32_t)FLAG_CAPACITY);
  // stable sort of contact indices by colour -> colour-major order
  uint32_t* cidx = S.u + L.cv0;
  for (int q = tid; q < nc; q += T) cidx[q] = (uint32_t)q;
  __syncthreads();
  int swc = lds_radix_sort(colour, cidx, S.u + L.ck1, S.u + L.cperm, nc, 0, 1, S.u + L.hist, S.u + L.hbase);
  (void)swc;  // one pass: result in (ck1, cperm)
  const uint32_t* scol = S.u + L.ck1;
  uint32_t* cstart = S.u + L.hbase;  // colour starts (hbase is free again)
  for (int i = tid; i <= kMaxColours; i += T) cstart[i] = 0u;
  __syncthreads();
  for (int i = tid; i < nc; i += T) {
    uint32_t c = scol[i];
    if (i == 0 || scol[i - 1] != c) cstart[c] = (uint32_t)i;
    if (i == nc - 1) misc[M_NCOL] = c + 1;
    S.u[L.ccol + S.u[L.cperm + i]] = c;
  }
  __syncthreads();
  const int ncol = nc > 0 ? (int)misc[M_NCOL] : 0;
  // fill starts of empty colours below ncol (cannot happen for first fit) and the end
  if (tid == 0) cstart[ncol] = (uint32_t)nc;
  __syncthreads();

  // ---- a8/a11: warm start and sweeps ------------------------------------
  if (P.warm == WARM_LEARNED) {
    for (int i = tid; i < nb; i += T) {
#pragma unroll
      for (int k = 0; k < 3; k++) {
        S.f[L.vsave + k * NB + i] = S.f[L.bv + k * NB + i];
        S.f[L.vsave + (3 + k) * NB + i] = S.f[L.bw + k * NB + i];
      }
    }
    __syncthreads();
  }
  if (P.warm != WARM_COLD) apply_all(L, S, NB, CM, nc, ncol, cstart);
  int sweeps = 0;
  float res = 0.f;
  for (int attempt = 0; attempt < 2; attempt++) {
    sweeps = 0;
    res = 0.f;
    for (int it = 0; it < P.iters; it++) {
      float r = P.solver == SOLVER_JACOBI ? sweep_jacobi(L, S, NB, CM, nb, nc, ncol, cstart)
                                          : sweeps_pgs(L, S, NB, CM, ncol, cstart);
      sweeps++;
      if (P.tol > 0.f || it == P.iters - 1) {
        res = block_max(r, misc);
        if (P.tol > 0.f && res <= P.tol) break;
      }
    }
    if (!(P.tol > 0.f && res > P.tol)) break;
    if (P.warm != WARM_LEARNED || attempt == 1) {
      if (tid == 0) misc[M_FLAGS] |= FLAG_NOT_CONVERGED;
      break;
    }
    // learned start rejected: restore post-gravity velocities, solve cold
    if (tid == 0) misc[M_FLAGS] |= FLAG_FELLBACK;
    for (int i = tid; i < nb; i += T) {
#pragma unroll
      for (int k = 0; k < 3; k++) {
        S.f[L.bv + k * NB + i] = S.f[L.vsave + k * NB + i];
        S.f[L.bw + k * NB + i] = S.f[L.vsave + (3 + k) * NB + i];
      }
    }
    for (int q = tid; q < nc; q += T) {
      S.f[L.clam + q] = 0.f;
      S.f[L.clam + CM + q] = 0.f;
      S.f[L.clam + 2 * CM + q] = 0.f;
    }
    __syncthreads();
  }
  __syncthreads();

  // ---- a12: integrate positions, write state ----------------------------
  for (int i = tid; i < nb; i += T) {
    const long gi = b0 + i;
    uint32_t mt = (S.u[L.bmeta + i] >> 8) & 255u;
    if (mt == DYNAMIC) {
      V3 x = ld3(S.f + L.bx, NB, i), v = ld3(S.f + L.bv, NB, i), w = ld3(S.f + L.bw, NB, i);
      x = x + v * dt;
      float qw = S.f[L.bq + i], qx = S.f[L.bq + NB + i], qy = S.f[L.bq + 2 * NB + i], qz = S.f[L.bq + 3 * NB + i];
      // q + dt/2 (0, w) (x) q
      float dw = -(w.x * qx + w.y * qy + w.z * qz);
      float dx = qw * w.x + (w.y * qz - w.z * qy);
      float dy = qw * w.y + (w.z * qx - w.x * qz);
      float dz = qw * w.z + (w.x * qy - w.y * qx);
      float h = 0.5f * dt;
      qw += h * dw; qx += h * dx; qy += h * dy; qz += h * dz;
      float inv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
      qw *= inv; qx *= inv; qy *= inv; qz *= inv;
      P.pose[gi] = x.x; P.pose[N + gi] = x.y; P.pose[2 * N + gi] = x.z;
      P.pose[3 * N + gi] = qw; P.pose[4 * N + gi] = qx; P.pose[5 * N + gi] = qy; P.pose[6 * N + gi] = qz;
      P.vel[gi] = v.x; P.vel[N + gi] = v.y; P.vel[2 * N + gi] = v.z;
      P.vel[3 * N + gi] = w.x; P.vel[4 * N + gi] = w.y; P.vel[5 * N + gi] = w.z;
      bool fin = isfinite(x.x) && isfinite(x.y) && isfinite(x.z) && isfinite(v.x) && isfinite(v.y) && isfinite(v.z) &&
                 isfinite(w.x) && isfinite(w.y) && isfinite(w.z);
      if (!fin) atomicOr(&misc[M_FLAGS], (uint32_t)FLAG_NONFINITE);
    }
  }
  __syncthreads();  // all reads of the arm links' LDS pose are done
  if (P.arm && tid == 0) {
    float th[7];
    for (int k = 0; k < 7; k++) {
      th[k] = P.theta[7 * s + k] + dt * thd[k];
      P.theta[7 * s + k] = th[k];
    }
    // link velocities stay those of this step; poses move to theta_{t+1}
    arm_fk(P, L, S, NB, nb - 7, P.arm_base + 3 * s, th, nullptr);
    for (int k = 0; k < 7; k++) {
      int i = nb - 7 + k;
      long gi = b0 + i;
      for (int c = 0; c < 3; c++) P.pose[c * N + gi] = S.f[L.bx + c * NB + i];
      for (int c = 0; c < 4; c++) P.pose[(3 + c) * N + gi] = S.f[L.bq + c * NB + i];
      for (int c = 0; c < 3; c++) {
        P.vel[c * N + gi] = S.f[L.bv + c * NB + i];
        P.vel[(3 + c) * N + gi] = S.f[L.bw + c * NB + i];
      }
    }
  }

  // ---- a13: cache, export, arm force, stats ------------------------------
  const int arm0 = P.arm ? nb - 7 : nb;
  float* force = S.f + L.force;
  for (int q = tid; q < nc; q += T) {
    uint32_t ab = S.u[L.cab + q];
    int a = (int)(ab & 0xFFFFu), b = (int)(ab >> 16);
    V3 n = ld3(S.f + L.cn, CM, q);
    V3 t1, t2;
    tangents(n, t1, t2);
    float l0 = S.f[L.clam + q], l1 = S.f[L.clam + CM + q], l2 = S.f[L.clam + 2 * CM + q];
    V3 F = t1 * l1 + t2 * l2;
    long o = (long)s * CM + q;
    P.cur_key[o] = S.u[L.ckey + q];
    P.cur_lam[o] = l0;
    P.cur_lam[P.scene_cm + o] = F.x;
    P.cur_lam[2 * P.scene_cm + o] = F.y;
    P.cur_lam[3 * P.scene_cm + o] = F.z;
    bool arm_c = a >= arm0 || (b != 0xFFFF && b >= arm0);
    force[q] = arm_c ? sqrtf(len2(n * l0 + F)) / dt : 0.f;
  }
  if (P.export_on) {
    for (int q = tid; q < nc; q += T) {
      long o = (long)s * CM + q;
      const long sc = P.scene_cm;
      P.x_normal[o] = S.f[L.cn + q]; P.x_normal[sc + o] = S.f[L.cn + CM + q]; P.x_normal[2 * sc + o] = S.f[L.cn + 2 * CM + q];
      P.x_point[o] = S.f[L.cp + q]; P.x_point[sc + o] = S.f[L.cp + CM + q]; P.x_point[2 * sc + o] = S.f[L.cp + 2 * CM + q];
      P.x_phi[o] = S.f[L.cphi + q];
      P.x_lambda[o] = S.f[L.clam + q]; P.x_lambda[sc + o] = S.f[L.clam + CM + q]; P.x_lambda[2 * sc + o] = S.f[L.clam + 2 * CM + q];
      P.x_colour[o] = (int32_t)S.u[L.ccol + q];
    }
  }
  __syncthreads();
  // fixed-shape tree sum over the contact slots: same result for any block size
  int width = 1;
  while (width < nc) width <<= 1;
  for (int half = width >> 1; half > 0; half >>= 1) {
    for (int i = tid; i < half; i += T)
      if (i + half < nc) force[i] += force[i + half];
    __syncthreads();
  }
  if (tid == 0) {
    P.cur_count[s] = nc;
    P.st_pairs[s] = npairs_all;
    P.st_contacts[s] = nc_all;
    P.st_colours[s] = ncol;
    P.st_sweeps[s] = sweeps;
    P.st_residual[s] = res;
    P.st_flags[s] = (int32_t)misc[M_FLAGS];
    P.st_arm_force[s] = nc > 0 ? force[0] : 0.f;
  }
}

}  // namespace rbs

extern "C" int rbs_launch_step(const rbs::StepParams* P, const rbs::LdsLayout* L, int threads, int grid,
                               hipStream_t stream) {
  size_t bytes = (size_t)L->total * 4u;
  hipLaunchKernelGGL(rbs::step_kernel, dim3(grid), dim3(threads), bytes, stream, *P, *L);
  return (int)hipGetLastError();
}

extern "C" int rbs_set_step_lds_limit(int bytes) {
  return (int)hipFuncSetAttribute((const void*)rbs::step_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

namespace rbs {

// Arm link poses from the joint angles, one thread per scene (set-up and resets).
__global__ void arm_pose_kernel(int S_, const int32_t* off, float* pose, long N, const float* theta, const float* base,
                                StepParams P, const uint8_t* mask) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S_) return;
  if (mask && !mask[s]) return;
  V3 c[7], o[7], ax[7];
  float q[7][4];
  arm_chain(base + 3 * s, theta + 7 * s, P.link_len, c, q, o, ax);
  int b0 = off[s + 1] - 7;
  for (int k = 0; k < 7; k++) {
    long gi = b0 + k;
    pose[gi] = c[k].x; pose[N + gi] = c[k].y; pose[2 * N + gi] = c[k].z;
    for (int j = 0; j < 4; j++) pose[(3 + j) * N + gi] = q[k][j];
  }
}

// Masked reset: one workgroup per scene copies pose/velocity (and joint
// angles) from the caller's pool arrays and empties the contact cache.
__global__ void reset_kernel(const int32_t* off, const uint8_t* mask, float* pose, float* vel, long N,
                             const float* pool_pose, const float* pool_vel, float* theta, const float* pool_theta,
                             int32_t* cache_count_a, int32_t* cache_count_b) {
  int s = blockIdx.x;
  if (!mask[s]) return;
  int b0 = off[s], b1 = off[s + 1];
  for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
    for (int k = 0; k < 7; k++) pose[k * N + i] = pool_pose[k * N + i];
    for (int k = 0; k < 6; k++) vel[k * N + i] = pool_vel[k * N + i];
  }
  if (threadIdx.x < 7 && theta && pool_theta) theta[7 * s + threadIdx.x] = pool_theta[7 * s + threadIdx.x];
  if (threadIdx.x == 0) {
    cache_count_a[s] = 0;
    cache_count_b[s] = 0;
  }
}

}  // namespace rbs

extern "C" int rbs_launch_arm_pose(const rbs::StepParams* P, const uint8_t* mask, hipStream_t stream) {
  int S_ = P->num_scenes;
  hipLaunchKernelGGL(rbs::arm_pose_kernel, dim3((S_ + 63) / 64), dim3(64), 0, stream, S_, P->body_offset, P->pose,
                     P->n_bodies, P->theta, P->arm_base, *P, mask);
  return (int)hipGetLastError();
}

extern "C" int rbs_launch_reset(const rbs::StepParams* P, const uint8_t* mask, const float* pool_pose,
                                const float* pool_vel, const float* pool_theta, int32_t* count_a, int32_t* count_b,
                                hipStream_t stream) {
  hipLaunchKernelGGL(rbs::reset_kernel, dim3(P->num_scenes), dim3(128), 0, stream, P->body_offset, mask, P->pose,
                     P->vel, P->n_bodies, pool_pose, pool_vel, P->theta, pool_theta, count_a, count_b);
  return (int)hipGetLastError();
}

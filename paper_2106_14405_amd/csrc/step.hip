// step.hip -- one physics step (s_t, a_t) -> s_{t+1} for a batch of
// independent scenes, one workgroup per scene, the scene's working set
// resident in LDS (gfx950: 160 KB per CU) as float4-aligned records.
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
//  a10 constraint setup (offsets, effective masses, bias, initial impulse)
//  a9 first-fit colouring as the parallel fixed point of
//     c_q = mex{ c_p : p < q shares a dynamic body with q }, then a stable
//     one-digit radix sort into colour-major order
//  a11 projected Gauss-Seidel (or Jacobi) sweeps, one barrier per colour,
//     max-residual reduction per sweep
//  a12 semi-implicit position/orientation update; arm theta update + FK
//  a13 cache, contact export, arm contact force, per-scene stats
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "arm.h"
#include "geom.h"
#include "hull.h"
#include "mlp_mfma.h"
#include "sim_internal.h"

namespace rbs {

typedef unsigned long long u64;

// The threads that step one scene: a whole workgroup, or a single wave of a
// larger workgroup (persistent launch).  A team starts on a wave boundary.
template <bool kWave>
struct Team {
  static constexpr bool wave = kWave;  // one wave of a multi-wave workgroup
  int tid, T;                          // index within the team; team size, a multiple of 64
};

// Barrier among a team's threads: a workgroup barrier, or for one wave of a
// larger workgroup the wave's own memory fences (its LDS operations
// complete in issue order; the fence also waits for its global stores).
template <class TM>
__device__ __forceinline__ void team_sync(const TM tm) {
  if constexpr (TM::wave) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  } else {
    __syncthreads();
  }
}

// Phase timestamp (constant-rate wall clock) of scene s, slot k, if tracing.
#define TRACE(k)                                                                    \
  do {                                                                              \
    if (P.trace && tid == 0) P.trace[(long)s * kTraceSlots + (k)] = wall_clock64(); \
  } while (0)

__device__ __forceinline__ unsigned lanes_below(u64 m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ uint32_t orderable(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Cross-lane steps by data-parallel primitives (DPP) instead of LDS
// permutes: shifts right by 1, 2, 4 and 8 lanes inside each row of 16
// (lanes with no source read 0), then the last lane of a row broadcast to
// the next row (rows 1 and 3) and lane 31 to rows 2 and 3.
#define RBS_DPP(v, ctrl, rows) __builtin_amdgcn_update_dpp(0u, (v), (ctrl), (rows), 0xf, false)

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += RBS_DPP(v, 0x111, 0xf);  // row_shr:1
  v += RBS_DPP(v, 0x112, 0xf);  // row_shr:2
  v += RBS_DPP(v, 0x114, 0xf);  // row_shr:4
  v += RBS_DPP(v, 0x118, 0xf);  // row_shr:8
  v += RBS_DPP(v, 0x142, 0xa);  // row_bcast:15
  v += RBS_DPP(v, 0x143, 0xc);  // row_bcast:31
  return v;
}

// In-place exclusive prefix sum of a[0..n) in LDS; every thread takes a
// contiguous chunk; returns the total.  misc supplies per-wave slots.
template <class TM>
__device__ uint32_t block_exclusive_scan(uint32_t* a, int n, uint32_t* misc, const TM tm) {
  const int tid = tm.tid, T = tm.T, W = T >> 6, w = tid >> 6, lane = tid & 63;
  const int chunk = (n + T - 1) / T;
  const int i0 = tid * chunk, i1 = min(n, i0 + chunk);
  uint32_t sum = 0;
  for (int i = i0; i < i1; i++) sum += a[i];
  uint32_t incl = wave_incl_scan(sum);
  if (lane == 63) misc[M_SCAN + w] = incl;
  team_sync(tm);
  uint32_t base = 0, total = 0;
  for (int ww = 0; ww < W; ww++) {
    uint32_t t = misc[M_SCAN + ww];
    if (ww < w) base += t;
    total += t;
  }
  uint32_t run = base + incl - sum;
  for (int i = i0; i < i1; i++) {
    uint32_t v = a[i];
    a[i] = run;
    run += v;
  }
  team_sync(tm);
  return total;
}

// Stable LSD radix sort of n (key, value) pairs held in LDS, `passes`
// 8-bit digits from bit `shift0`.  Ranks within a wave come from eight
// ballots that isolate the lanes holding the same digit.  Returns 1 if the
// sorted data ended in (k1, v1), 0 if in (k0, v0).
template <class TM>
__device__ int lds_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int n, int shift0, int passes,
                              uint32_t* hist, uint32_t* base, uint32_t* misc, const TM tm) {
  const int T = tm.T, tid = tm.tid, W = T >> 6, w = tid >> 6;
  int swapped = 0;
  for (int ps = 0; ps < passes; ps++) {
    const int sh = shift0 + 8 * ps;
    for (int i = tid; i < 256; i += T) base[i] = 0u;
    for (int i = tid; i < 256 * W; i += T) hist[i] = 0u;
    team_sync(tm);
    for (int i = tid; i < n; i += T) atomicAdd(&base[(k0[i] >> sh) & 255u], 1u);
    team_sync(tm);
    block_exclusive_scan(base, 256, misc, tm);
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
      team_sync(tm);
      if (valid) {
        uint32_t off = base[d] + rank;
        for (int ww = 0; ww < w; ww++) off += hist[ww * 256 + d];
        k1[off] = key;
        v1[off] = val;
      }
      team_sync(tm);
      if (t0 + T < n) {
        for (int dd = tid; dd < 256; dd += T) {
          uint32_t s = 0;
          for (int ww = 0; ww < W; ww++) { s += hist[ww * 256 + dd]; hist[ww * 256 + dd] = 0u; }
          base[dd] += s;
        }
        team_sync(tm);
      }
    }
    uint32_t* t;
    t = k0; k0 = k1; k1 = t;
    t = v0; v0 = v1; v1 = t;
    swapped ^= 1;
  }
  return swapped;
}

// Bitonic sort of 64 S unique 32-bit keys held by one wave, S consecutive
// elements per lane in registers (element S lane + s), ascending; padding
// keys are ~0u.  Partners within a lane compare in registers, partners in
// other lanes are exchanged by a lane permute.
template <int S>
__device__ __forceinline__ void wave_bitonic(uint32_t (&v)[8], int lane) {
  constexpr int N = 64 * S;
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= S) {
#pragma unroll
        for (int s = 0; s < S; s++) {
          const uint32_t o = __shfl_xor(v[s], j / S);
          const int e = S * lane + s;
          const bool up = (e & k) == 0, low = (e & j) == 0;
          v[s] = up == low ? min(v[s], o) : max(v[s], o);
        }
      } else {
#pragma unroll
        for (int s = 0; s < S; s++) {
          if (s & j) continue;
          const bool up = ((S * lane + s) & k) == 0;
          const uint32_t a = v[s], b = v[s + j];
          v[s] = up ? min(a, b) : max(a, b);
          v[s + j] = up ? max(a, b) : min(a, b);
        }
      }
    }
  }
}

// Sorts n <= 512 unique keys with one wave: load (key of element e from
// `key(e)`, e < n), sort, and hand each sorted (position, key) to `put`.
template <class KeyF, class PutF>
__device__ __forceinline__ void wave_sort512(int n, int lane, KeyF key, PutF put) {
  uint32_t v[8];
  auto run = [&](auto sz) {
    constexpr int S = decltype(sz)::value;
#pragma unroll
    for (int s = 0; s < 8; s++) {
      const int e = S * lane + s;
      v[s] = s < S && e < n ? key(e) : ~0u;
    }
    wave_bitonic<S>(v, lane);
#pragma unroll
    for (int s = 0; s < S; s++) {
      const int e = S * lane + s;
      if (e < n) put(e, v[s]);
    }
  };
  if (n <= 256) run(std::integral_constant<int, 4>{});
  else run(std::integral_constant<int, 8>{});
}

// Stable sort of n <= kRankSortMax (key, value) pairs in LDS by rank: the
// rank of element i is the number of elements j with (key_j, j) < (key_i, i)
// (the order the radix sort yields).  Each thread holds E <= 8 elements in
// register slots; the keys are read as uniform broadcasts, four at a time,
// and compared with every slot (an instantiation per E, so the loop has no
// branches; unique keys need only a 32-bit compare).  k0 must be 16-byte
// aligned; the result goes to (k1, v1), which must not overlap (k0, v0) (v0
// and v1 may be null for keys only).
constexpr int kRankSortMax = 512;

template <int E, bool kUnique>
__device__ __forceinline__ void rank_count(const uint32_t* k0, int n, const uint32_t* mk, const uint32_t* mi,
                                           uint32_t* rk) {
  auto one = [&](uint32_t kj, uint32_t j) {
#pragma unroll
    for (int e = 0; e < E; e++) {
      if constexpr (kUnique) rk[e] += kj < mk[e] ? 1u : 0u;
      else rk[e] += (((u64)kj << 32) | j) < (((u64)mk[e] << 32) | mi[e]) ? 1u : 0u;
    }
  };
  int j = 0;
  for (; j + 4 <= n; j += 4) {
    const uint4 k4 = reinterpret_cast<const uint4*>(k0)[j >> 2];
    one(k4.x, (uint32_t)j);
    one(k4.y, (uint32_t)j + 1u);
    one(k4.z, (uint32_t)j + 2u);
    one(k4.w, (uint32_t)j + 3u);
  }
  for (; j < n; j++) one(k0[j], (uint32_t)j);
}

template <bool kUnique, class TM>
__device__ void lds_rank_sort(const uint32_t* k0, const uint32_t* v0, uint32_t* k1, uint32_t* v1, int n,
                              const TM tm) {
  const int T = tm.T, tid = tm.tid;
  uint32_t mk[8], mi[8], rk[8];
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int i = e * T + tid;
    mk[e] = i < n ? k0[i] : 0xFFFFFFFFu;
    mi[e] = (uint32_t)i;
    rk[e] = 0u;
  }
  switch ((n + T - 1) / T) {
    case 1: rank_count<1, kUnique>(k0, n, mk, mi, rk); break;
    case 2: rank_count<2, kUnique>(k0, n, mk, mi, rk); break;
    case 3: rank_count<3, kUnique>(k0, n, mk, mi, rk); break;
    case 4: rank_count<4, kUnique>(k0, n, mk, mi, rk); break;
    case 5: rank_count<5, kUnique>(k0, n, mk, mi, rk); break;
    case 6: rank_count<6, kUnique>(k0, n, mk, mi, rk); break;
    case 7: rank_count<7, kUnique>(k0, n, mk, mi, rk); break;
    case 8: rank_count<8, kUnique>(k0, n, mk, mi, rk); break;
    default: break;
  }
#pragma unroll
  for (int e = 0; e < 8; e++) {
    const int i = e * T + tid;
    if (i < n) {
      k1[rk[e]] = mk[e];
      if (v1) v1[rk[e]] = v0[i];
    }
  }
  team_sync(tm);
}

// Maximum over the wave of non-negative floats (their bit patterns order
// like the values; absent lanes read 0), in every lane.
__device__ __forceinline__ float wave_max(float v) {
  uint32_t u = __float_as_uint(v);
  u = max(u, RBS_DPP(u, 0x111, 0xf));
  u = max(u, RBS_DPP(u, 0x112, 0xf));
  u = max(u, RBS_DPP(u, 0x114, 0xf));
  u = max(u, RBS_DPP(u, 0x118, 0xf));
  u = max(u, RBS_DPP(u, 0x142, 0xa));
  u = max(u, RBS_DPP(u, 0x143, 0xc));
  return __uint_as_float(__builtin_amdgcn_readlane(u, 63));
}

// Block-wide maximum of non-negative floats (one value per thread).
template <class TM>
__device__ __forceinline__ float block_max(float v, uint32_t* misc, const TM tm) {
  const int tid = tm.tid, W = tm.T >> 6;
  v = wave_max(v);
  if (W == 1) return v;
  if ((tid & 63) == 0) misc[M_WAVE + (tid >> 6)] = __float_as_uint(v);
  team_sync(tm);
  float r = 0.f;
  for (int w = 0; w < W; w++) r = fmaxf(r, __uint_as_float(misc[M_WAVE + w]));
  team_sync(tm);
  return r;
}

struct Smem {
  float* f;
  uint32_t* u;
};

// Hardware reciprocal (v_rcp_f32, about 1 ulp) for the solver's hot path.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Tangent basis of a unit normal (Duff et al. 2017) with a hardware
// reciprocal; used for every contact row of the step (setup, sweeps, cache).
// The construction's two branches (upper and lower hemisphere) switch at
// n.z = -1/2 rather than at 0, away from the horizontal normals of
// side-by-side contacts; each branch's denominator stays >= 1/2 in size.
constexpr float kTangentSplit = -0.5f;
__device__ __forceinline__ float tangent_sign(V3 n) { return n.z >= kTangentSplit ? 1.0f : -1.0f; }
__device__ __forceinline__ float tangent_coef(V3 n) { return -frcp(tangent_sign(n) + n.z); }
// The basis from its coefficient a = -1 / (sgn + n.z) (kept in the solver
// record so that the sweeps need no reciprocal).
__device__ __forceinline__ void tangents_coef(V3 n, float a, V3& t1, V3& t2) {
  float sgn = tangent_sign(n);
  float b = n.x * n.y * a;
  t1 = v3(1.0f + sgn * n.x * n.x * a, sgn * b, -sgn * n.x);
  t2 = v3(b, sgn + n.y * n.y * a, -n.y);
}
__device__ __forceinline__ void tangents_fast(V3 n, V3& t1, V3& t2) { tangents_coef(n, tangent_coef(n), t1, t2); }

__device__ __forceinline__ float4 ld4(const float* base, int i) { return reinterpret_cast<const float4*>(base)[i]; }
__device__ __forceinline__ void st4(float* base, int i, float4 v) { reinterpret_cast<float4*>(base)[i] = v; }
__device__ __forceinline__ V3 xyz(float4 a) { return v3(a.x, a.y, a.z); }
__device__ __forceinline__ float4 f4(V3 a, float w) { return make_float4(a.x, a.y, a.z, w); }

// body geometry: float4 records 3i (x, meta), 3i+1 (q), 3i+2 (params)
__device__ __forceinline__ Geom load_geom(const LdsLayout& L, Smem S, int i) {
  float4 g0 = ld4(S.f + L.geo, 3 * i), g1 = ld4(S.f + L.geo, 3 * i + 1), g2 = ld4(S.f + L.geo, 3 * i + 2);
  Geom g;
  g.shape = (int)(__float_as_uint(g0.w) & 255u);
  g.x = xyz(g0);
  g.R = quat_R(g1.x, g1.y, g1.z, g1.w);
  g.p[0] = g2.x;
  g.p[1] = g2.y;
  g.p[2] = g2.z;
  g.hull = (int)g2.w;
  return g;
}

__device__ __forceinline__ uint32_t body_meta(const LdsLayout& L, Smem S, int i) {
  return __float_as_uint(S.f[L.geo + 12 * i + 3]);
}
__device__ __forceinline__ bool is_dyn_meta(uint32_t meta) { return ((meta >> 8) & 255u) == DYNAMIC; }
// a dynamic body that is not asleep: the bodies the solver moves
__device__ __forceinline__ bool is_awake_meta(uint32_t meta) { return is_dyn_meta(meta) && !(meta & kAsleepBit); }

// Dynamic state of a body in registers.
struct Dyn {
  V3 v, w;
  float im, mu;
  float I[6];  // xx yy zz xy xz yz
};

__device__ __forceinline__ Dyn load_dyn(const LdsLayout& L, Smem S, int i) {
  Dyn d;
  float4 d0 = ld4(S.f + L.dyn, 3 * i), d1 = ld4(S.f + L.dyn, 3 * i + 1);
  float4 d2 = ld4(S.f + L.dyn, 3 * i + 2), d3 = ld4(S.f + L.dyn2, i);
  d.v = xyz(d0);
  d.im = d0.w;
  d.w = xyz(d1);
  d.mu = d1.w;
  d.I[0] = d2.x; d.I[1] = d2.y; d.I[2] = d2.z; d.I[3] = d2.w; d.I[4] = d3.x; d.I[5] = d3.y;
  return d;
}

__device__ __forceinline__ V3 Imul(const float* I, V3 a) {
  return v3(I[0] * a.x + I[3] * a.y + I[4] * a.z, I[3] * a.x + I[1] * a.y + I[5] * a.z,
            I[4] * a.x + I[5] * a.y + I[2] * a.z);
}

// Projection of the friction impulse onto the disk of radius lim >= 0; the
// scale lim / |l| comes from the hardware reciprocal square root (about 1 ulp).
__device__ __forceinline__ void proj_disk(float& l1, float& l2, float lim) {
  const float s2 = l1 * l1 + l2 * l2;
  if (s2 > lim * lim) {  // then s2 > 0
    // v_rsq_f32 reads a denormal s2 (|l| below 1e-19 N s) as zero and
    // returns +inf, and 0 * inf is NaN when lim = 0; below 1e-30 the scale
    // is taken at 1e-30, which still lands inside the disk (|l| f <= lim)
    const float f = lim * __builtin_amdgcn_rsqf(fmaxf(s2, 1e-30f));
    l1 *= f;
    l2 *= f;
  }
}

// Solver record of one contact, 5 float4 in global memory, colour-major
// order:
//  0 (n, m_n)  1 (r_a, m_t1)  2 (r_b, m_t2)  3 (k_1n, k_2n, bias - u_n, mu)
//  4 (key, Jacobi scale, tangent coefficient, u_t1)
// n the normal (the tangents t1, t2 follow from it and the coefficient
// exactly as in the setup), r_a, r_b the contact point relative to the bodies' centres,
// m_d = 1 / k_d the effective mass of row d, and k_dn the change of row d's
// velocity per unit normal impulse (the normal-friction coupling inside one
// contact).  The angular parts r x d and I^-1 (r x d) of the Jacobian rows
// are not stored: the velocity of a row is d . (v_a + w_a x r_a - v_b -
// w_b x r_b) and an impulse P changes w by I^-1 (r x P), with the world
// inverse inertia I^-1 read from LDS.  80 bytes instead of the 208 of
// explicit rows keep a sweep's records in L2.
//
// During the solve a dynamic body's LDS slot holds its velocity change
// since the setup, not its velocity: a row's velocity is u_d + d . (point
// velocity of the changes), with u_d the row's velocity from the dynamic
// bodies' velocities at the setup (u_n folded into the normal row's bias,
// u_t1 in the record, u_t2 in the fourth word of the contact's impulse).
// A sweep's impulse steps are small against a fast body's velocity: added
// to the velocity itself they would be rounded away in float32 while the
// impulses still took them, and the two would drift apart over hundreds of
// sweeps.  Kinematic bodies keep their (unchanging) velocity in the slot.
static_assert(kRec == 5, "record layout below");

struct Rec {
  float4 r[kRec];
};

// One Jacobian row during the setup (effective masses and couplings).
struct Row {
  V3 d, ca, cb, ia, ib;
  float m;
};

__device__ __forceinline__ Rec load_rec(const float4* rec, int i) {
  Rec R;
#pragma unroll
  for (int k = 0; k < kRec; k++) R.r[k] = rec[kRec * i + k];
  return R;
}

__device__ __forceinline__ int rec_a(const Rec& R) { return (int)(__float_as_uint(R.r[4].x) >> 20); }
__device__ __forceinline__ int rec_b(const Rec& R) {
  uint32_t bk = (__float_as_uint(R.r[4].x) >> 8) & 0xFFFu;
  return bk == kGroundKey ? -1 : (int)bk;
}

__device__ __forceinline__ void store_rec(float4* rec, int i, V3 n, V3 ra, V3 rb, const float* m, float k1n, float k2n,
                                          float bias, float mu, uint32_t key, float jsc, float u1) {
  float4* o = rec + kRec * i;
  o[0] = f4(n, m[0]);
  o[1] = f4(ra, m[1]);
  o[2] = f4(rb, m[2]);
  o[3] = make_float4(k1n, k2n, bias, mu);
  o[4] = make_float4(__uint_as_float(key), jsc, tangent_coef(n), u1);
}

// A body as the solver sees it in LDS: velocities, inverse mass (dynamic
// iff > 0), friction coefficient, world inverse inertia (xx yy zz xy xz yz).
// Index -1 (the ground) reads the zero slots in front of the bodies.
struct Vel {
  V3 v, w;
  float im, mu;
  float I[6];
};

__device__ __forceinline__ Vel load_vel(const LdsLayout& L, Smem S, int i) {
  Vel b;
  const float4 d0 = ld4(S.f + L.dyn, 3 * i), d1 = ld4(S.f + L.dyn, 3 * i + 1);
  const float4 d2 = ld4(S.f + L.dyn, 3 * i + 2), d3 = ld4(S.f + L.dyn2, i);
  b.v = xyz(d0);
  b.im = d0.w;
  b.w = xyz(d1);
  b.mu = d1.w;
  b.I[0] = d2.x; b.I[1] = d2.y; b.I[2] = d2.z; b.I[3] = d2.w; b.I[4] = d3.x; b.I[5] = d3.y;
  return b;
}

__device__ __forceinline__ void store_vel(const LdsLayout& L, Smem S, int i, const Vel& b) {
  st4(S.f + L.dyn, 3 * i, f4(b.v, b.im));
  st4(S.f + L.dyn, 3 * i + 1, f4(b.w, b.mu));
}

// Writes back a body of a contact update: dynamic bodies to their slot, the
// others (ground, static, kinematic) to the sink slot, without a branch.
__device__ __forceinline__ void store_vel_dyn(const LdsLayout& L, Smem S, int i, const Vel& b) {
  store_vel(L, S, b.im != 0.f ? i : -2, b);  // (negative: a container part's flag)
}

// Relative velocity of the contact point: (v_a + w_a x r_a) - (v_b + w_b x r_b).
__device__ __forceinline__ V3 point_vel(V3 va, V3 wa, V3 vb, V3 wb, V3 ra, V3 rb) {
  return (va + cross(wa, ra)) - (vb + cross(wb, rb));
}

// Impulse P at r on one body.  With container parts (parts true): a
// prismatic part's velocity changes by its projector a a^T / m times P, a
// revolute part's (about its hinge point) by a a^T / I_o times r x P.
__device__ __forceinline__ void apply_body(Vel& A, V3 r, V3 P, bool parts) {
  if (parts && A.im == kPrismaticFlag) {
    A.v = A.v + Imul(A.I, P);
  } else {
    A.v = A.v + P * (parts ? fmaxf(A.im, 0.f) : A.im);
    A.w = A.w + Imul(A.I, cross(r, P));
  }
}

// Impulse P at the contact point on body a and -P on body b.
__device__ __forceinline__ void apply_impulse(Vel& A, Vel& B, V3 ra, V3 rb, V3 P, bool parts = false) {
  if (!parts) {
    A.v = A.v + P * A.im;
    A.w = A.w + Imul(A.I, cross(ra, P));
    B.v = B.v - P * B.im;
    B.w = B.w - Imul(B.I, cross(rb, P));
  } else {
    apply_body(A, ra, P, true);
    apply_body(B, rb, -P, true);
  }
}

// Synchronisation between colour batches: a single-wave team needs only a
// compiler fence (its LDS operations complete in issue order), which keeps
// prefetched global loads in flight; wider teams use a barrier.
template <class TM>
__device__ __forceinline__ void colour_sync(const TM tm) {
  if (tm.T == 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    team_sync(tm);
  }
}

// The articulated arm (arm 2) as the solver sees it: the joint-rate changes
// in LDS and this scene's joint-space rows of the arm contacts in global
// memory, one slot per colour (every contact on the arm takes its own
// colour, so a colour batch moves the joint rates from one lane at most).
// A contact's record holds its arm side in word (4, y): +1 when body a is
// an arm link, -1 when body b is, 0 when neither (the Jacobi scale's word:
// the Jacobi solver is not used with this arm).
struct ArmCtx {
  bool on;
  float* dq;           // LDS [7] joint-rate changes since the setup
  const float* rows;   // global [kMaxColours][kArmRowWords]
  bool parts;          // the scene has container parts (flagged bodies, limit rows)
};

// Row velocities g . dq of the arm contact in colour c (n, t1, t2).
__device__ __forceinline__ void arm_row_vel(const ArmCtx& A, int c, float u[3]) {
  const float* g = A.rows + (long)c * kArmRowWords;
  u[0] = 0.f; u[1] = 0.f; u[2] = 0.f;
#pragma unroll
  for (int i = 0; i < 7; i++) {
    const float d = A.dq[i];
    u[0] += g[i] * d;
    u[1] += g[7 + i] * d;
    u[2] += g[14 + i] * d;
  }
}

// Impulses (dn, d1, d2) of the arm contact in colour c on the arm side sg:
// dq += sg (dn M^-1 g_n + d1 M^-1 g_t1 + d2 M^-1 g_t2).
__device__ __forceinline__ void arm_row_apply(const ArmCtx& A, int c, float sg, float dn, float d1, float d2) {
  const float* w = A.rows + (long)c * kArmRowWords + 21;
#pragma unroll
  for (int i = 0; i < 7; i++) A.dq[i] += sg * (dn * w[i] + d1 * w[7 + i] + d2 * w[14 + i]);
}

// One Gauss-Seidel update at colour-major position i: the normal row, then
// both friction rows from the velocities after the normal impulse (through
// the couplings k_1n, k_2n), then the contact's total impulse.  Returns the
// residual max |dlambda| * k.
__device__ __forceinline__ float pgs_update(const LdsLayout& L, Smem S, const Rec& R, int i, const ArmCtx& arm,
                                           int c) {
  const int a = rec_a(R), b = rec_b(R);
  const float4 lam = ld4(S.f + L.lam, i);
  Vel A = load_vel(L, S, a);
  Vel B = load_vel(L, S, b);
  const V3 n = xyz(R.r[0]), ra = xyz(R.r[1]), rb = xyz(R.r[2]);
  const float mn = R.r[0].w, m1 = R.r[1].w, m2 = R.r[2].w;
  const float k1n = R.r[3].x, k2n = R.r[3].y, bias = R.r[3].z, mu = R.r[3].w;
  V3 t1, t2;
  tangents_coef(n, R.r[4].z, t1, t2);
  const V3 dv = point_vel(A.v, A.w, B.v, B.w, ra, rb);
  float un = dot(n, dv), u1 = dot(t1, dv), u2 = dot(t2, dv);
  const float asg = arm.on ? R.r[4].y : 0.f;  // arm side of the contact (0: none)
  if (asg != 0.f) {
    float ua[3];
    arm_row_vel(arm, c, ua);
    un += asg * ua[0];
    u1 += asg * ua[1];
    u2 += asg * ua[2];
  }
  const float ln = fmaxf(0.f, lam.x + mn * (bias - un));
  const float dn = ln - lam.x;
  float l1 = lam.y - m1 * ((u1 + R.r[4].w) + k1n * dn);
  float l2 = lam.z - m2 * ((u2 + lam.w) + k2n * dn);
  proj_disk(l1, l2, mu * ln);
  const float d1 = l1 - lam.y, d2 = l2 - lam.z;
  apply_impulse(A, B, ra, rb, n * dn + t1 * d1 + t2 * d2, arm.parts);
  if (asg != 0.f) arm_row_apply(arm, c, asg, dn, d1, d2);
  store_vel_dyn(L, S, a, A);
  store_vel_dyn(L, S, b, B);
  st4(S.f + L.lam, i, make_float4(ln, l1, l2, lam.w));
  return fmaxf(fmaxf(fabsf(dn) * frcp(mn), fabsf(d1) * frcp(m1)), fabsf(d2) * frcp(m2));
}

// Value of the partner lane in a lane pair (lanes 2k, 2k + 1): a DPP quad
// permutation [1, 0, 3, 2], one VALU operation.
__device__ __forceinline__ float pair_swap(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xf, 0xf, false));
}

// The update of pgs_update on a lane pair: lane `side` 0 holds body a, lane
// 1 body b.  Each lane projects its body's point velocity on the three rows
// (signed: + for a, - for b) and adds its partner's projection, so both
// lanes hold the same row velocities (the addition commutes exactly), take
// the same impulse step and apply it to their own body only.  Halves the
// dependent work of one update; used for colours of at most 32 contacts.
__device__ __forceinline__ float pgs_update_pair(const LdsLayout& L, Smem S, const Rec& R, int i, int side,
                                                const ArmCtx& arm, int c) {
  const int me = side ? rec_b(R) : rec_a(R);
  const float sg = side ? -1.f : 1.f;
  // the lane of the arm link's side also holds the arm's part
  const bool arm_lane = arm.on && R.r[4].y == sg;
  const float4 lam = ld4(S.f + L.lam, i);
  Vel M = load_vel(L, S, me);
  const V3 n = xyz(R.r[0]), r = side ? xyz(R.r[2]) : xyz(R.r[1]);
  const float mn = R.r[0].w, m1 = R.r[1].w, m2 = R.r[2].w;
  const float k1n = R.r[3].x, k2n = R.r[3].y, bias = R.r[3].z, mu = R.r[3].w;
  V3 t1, t2;
  tangents_coef(n, R.r[4].z, t1, t2);
  const V3 pv = M.v + cross(M.w, r);
  float cn = sg * dot(n, pv), c1 = sg * dot(t1, pv), c2 = sg * dot(t2, pv);
  if (arm_lane) {
    float ua[3];
    arm_row_vel(arm, c, ua);
    cn += sg * ua[0];
    c1 += sg * ua[1];
    c2 += sg * ua[2];
  }
  const float un = cn + pair_swap(cn);
  const float u1 = (c1 + pair_swap(c1)) + R.r[4].w, u2 = (c2 + pair_swap(c2)) + lam.w;
  const float ln = fmaxf(0.f, lam.x + mn * (bias - un));
  const float dn = ln - lam.x;
  float l1 = lam.y - m1 * (u1 + k1n * dn);
  float l2 = lam.z - m2 * (u2 + k2n * dn);
  proj_disk(l1, l2, mu * ln);
  const float d1 = l1 - lam.y, d2 = l2 - lam.z;
  const V3 P = (n * dn + t1 * d1 + t2 * d2) * sg;
  if (arm.parts) {
    apply_body(M, r, P, true);
  } else {
    M.v = M.v + P * M.im;
    M.w = M.w + Imul(M.I, cross(r, P));
  }
  store_vel_dyn(L, S, me, M);
  if (arm_lane) arm_row_apply(arm, c, sg, dn, d1, d2);
  if (!side) st4(S.f + L.lam, i, make_float4(ln, l1, l2, lam.w));
  return fmaxf(fmaxf(fabsf(dn) * frcp(mn), fabsf(d1) * frcp(m1)), fabsf(d2) * frcp(m2));
}

// Objective change from adding the network's start impulses of colour-major
// contact i (zero for a persisting contact): the impulse times (the mean of
// the row velocity before and after the new contacts' impulses were
// applied) minus the row's target (bias for the normal row, zero for
// friction).  Summed over the contacts this is f(l_p + l_n) - f(l_p) for the
// solver's quadratic objective f(l) = 1/2 l^T A l + l^T (u_free - b).
__device__ __forceinline__ float start_objective(const LdsLayout& L, Smem S, const float4* rec, int i) {
  if (!((S.u[L.fresh + (i >> 5)] >> (i & 31)) & 1u)) return 0.f;
  Rec R = load_rec(rec, i);
  const int a = rec_a(R), b = rec_b(R);
  const float4 lam = ld4(S.f + L.lam, i);
  const Vel A1 = load_vel(L, S, a), B1 = load_vel(L, S, b);
  // velocities before the new contacts' impulses: saved copy (ground: zero)
  const V3 va0 = xyz(ld4(S.f + L.vsave, 2 * a)), wa0 = xyz(ld4(S.f + L.vsave, 2 * a + 1));
  V3 vb0 = v3(0.f, 0.f, 0.f), wb0 = vb0;
  if (b >= 0) {
    vb0 = xyz(ld4(S.f + L.vsave, 2 * b));
    wb0 = xyz(ld4(S.f + L.vsave, 2 * b + 1));
  }
  const V3 n = xyz(R.r[0]), ra = xyz(R.r[1]), rb = xyz(R.r[2]);
  const float bias = R.r[3].z;
  V3 t1, t2;
  tangents_coef(n, R.r[4].z, t1, t2);
  const V3 dv0 = point_vel(va0, wa0, vb0, wb0, ra, rb), dv1 = point_vel(A1.v, A1.w, B1.v, B1.w, ra, rb);
  float f = lam.x * (0.5f * (dot(n, dv0) + dot(n, dv1)) - bias);
  // (velocity changes since the setup: the friction rows add their setup velocity)
  f += lam.y * (0.5f * (dot(t1, dv0) + dot(t1, dv1)) + R.r[4].w);
  f += lam.z * (0.5f * (dot(t2, dv0) + dot(t2, dv1)) + lam.w);
  return f;
}

// Applies the current impulses of every contact, colour-major (warm start);
// with `select` >= 0 only the contacts whose fresh bit equals it.
template <class TM>
__device__ __forceinline__ void apply_all(const LdsLayout& L, Smem S, const float4* rec, int ncol, const uint32_t* cstart,
                          const TM tm, const ArmCtx& arm, int select = -1) {
  for (int c = 0; c < ncol; c++) {
    for (int i = (int)cstart[c] + tm.tid; i < (int)cstart[c + 1]; i += tm.T) {
      if (select >= 0 && (int)((S.u[L.fresh + (i >> 5)] >> (i & 31)) & 1u) != select) continue;
      Rec R = load_rec(rec, i);
      const int a = rec_a(R), b = rec_b(R);
      const float4 lam = ld4(S.f + L.lam, i);
      Vel A = load_vel(L, S, a);
      Vel B = load_vel(L, S, b);
      const V3 n = xyz(R.r[0]);
      V3 t1, t2;
      tangents_coef(n, R.r[4].z, t1, t2);
      apply_impulse(A, B, xyz(R.r[1]), xyz(R.r[2]), n * lam.x + t1 * lam.y + t2 * lam.z, arm.parts);
      store_vel_dyn(L, S, a, A);
      store_vel_dyn(L, S, b, B);
      if (arm.on && R.r[4].y != 0.f) arm_row_apply(arm, c, R.r[4].y, lam.x, lam.y, lam.z);
    }
    colour_sync(tm);
  }
}

// ---- the articulated arm (arm 2) -----------------------------------------
// The arm is one articulated body in reduced coordinates (an articulated
// robot driven by joint motors under PD position control): its joint angles
// and rates are the state, link poses follow the angles by the forward
// kinematics and link velocities the rates through the link Jacobians, so
// the joints hold exactly.  M(q) = sum over links j of Jv^T m_j Jv + Jw^T
// I_j Jw (column i of link j's Jacobians: a_i x (c_j - o_i) and a_i, i <=
// j); velocity-product terms are left out, like the free bodies' gyroscopic
// term.  Gravity adds dt M^-1 tau_g to the rates.  A contact row d at p on
// link j acts on the rates through g_i = d . (a_i x (p - o_i)), i <= j.
// Motor k is the row on rate k with target Kp (target_k - theta_k) / dt
// (the error wrapped into [-pi, pi]), effective mass 1 / (M^-1)_kk and its
// impulse bounded by motor_max; the motors are swept after the contacts.
// The solve works on the rates' changes since the setup (dq), like the free
// bodies' velocities, so the motor rows' targets are less the setup rates.

// One Gauss-Seidel pass over the 7 motor rows by wave 0 (lane i holds rate
// change i); returns the pass's max |dlambda| (M^-1)_kk on every lane.
template <class TM>
__device__ __forceinline__ float arm_motor_sweep(const LdsLayout& L, Smem S, const TM tm, float lim) {
  float* arm = S.f + L.arm;
  const int lane = tm.tid & 63;
  float dq = lane < 7 ? arm[ARM_DQ + lane] : 0.f;
  float r = 0.f;
#pragma unroll
  for (int k = 0; k < 7; k++) {
    const float u = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(dq), k));
    const float kk = arm[ARM_MI + 8 * k];
    const float l0 = arm[ARM_LAM + k];
    const float l = fminf(fmaxf(l0 + (arm[ARM_BIAS + k] - u) / kk, -lim), lim);
    const float dl = l - l0;
    if (lane == 0) arm[ARM_LAM + k] = l;
    if (lane < 7) dq += dl * arm[ARM_MI + 7 * lane + k];
    r = fmaxf(r, fabsf(dl) * kk);
  }
  if (lane < 7) arm[ARM_DQ + lane] = dq;
  return r;
}

// ---- articulated container parts -----------------------------------------
// A door or drawer (a part) is one rigid body with one degree of freedom
// relative to the world: a revolute joint about a fixed hinge line (anchor
// o, unit axis a) or a prismatic one along a; its coordinate q and rate qd
// are the state, q held within limits.  The body moves with the rate (w =
// qd a, v = w x (c - o) for a hinge; v = qd a for a slide), and an impulse P
// at p changes qd by (a . ((p - o) x P)) / M or (a . P) / M, M the mass
// about the joint (the moment of inertia about the hinge line, or the
// mass).  In the solver's LDS slots a part is a body whose inverse inertia
// is the projector a a^T / M: a hinge's velocity is taken about its hinge
// point (its rows' lever arms run from o), a slide's linear velocity
// changes by a a^T P / M and its angular stays zero.  Parts keep their whole
// velocity in the slot during the solve (their setup velocity is not
// folded into the rows), like the kinematic bodies.

// Parts of the scene: slots in body order (wave 0, a ballot per 64
// bodies), rate plus gravity over the step (its moment about the hinge, or
// its force along the slide, over M), slot velocities and projector, and the
// two limit rows (q - lower >= 0, upper - q >= 0) with the contacts'
// speculative target: a gap g > 0 may close within the step (-g / dt), a
// violation is pushed back at baumgarte / dt of it.
__device__ __forceinline__ void part_setup(const StepParams& P, const LdsLayout& L, Smem S, int b0, int nb, float dt,
                                           V3 g, int lane) {
  const long N = P.n_bodies;
  float* pt = S.f + L.parts;
  int np = 0;
  for (int i0 = 0; i0 < nb; i0 += 64) {
    const int i = i0 + lane;
    const long gi = b0 + i;
    const int kind = (i < nb && is_dyn_meta(body_meta(L, S, i))) ? (int)P.joint[gi] : 0;
    const u64 m = __ballot(kind != 0);
    const int slot = np + (int)lanes_below(m);
    np += __popcll(m);
    if (kind == 0 || slot >= kMaxParts) continue;
    const V3 a = v3(P.joint_axis[gi], P.joint_axis[N + gi], P.joint_axis[2 * N + gi]);
    const V3 o = v3(P.joint_anchor[gi], P.joint_anchor[N + gi], P.joint_anchor[2 * N + gi]);
    const float mass = 1.0f / P.inv_mass[gi];
    const Geom G = load_geom(L, S, i);
    const bool rev = kind == 1;
    float M = mass, gq = dot(a, g * mass);
    if (rev) {
      // principal moments about the body axes, the axis in body coordinates
      const V3 al = v3(dot(col(G.R, 0), a), dot(col(G.R, 1), a), dot(col(G.R, 2), a));
      const V3 d = cross(a, G.x - o);
      M = al.x * al.x / P.inv_inertia[gi] + al.y * al.y / P.inv_inertia[N + gi] +
          al.z * al.z / P.inv_inertia[2 * N + gi] + mass * len2(d);
      gq = dot(a, cross(G.x - o, g * mass));
    }
    const float qd = P.joint_state[N + gi] + dt * gq / M;
    const float iM = 1.0f / M;
    const V3 u = a * qd;
    const float mu = S.f[L.dyn + kDynWords * i + 7];
    st4(S.f + L.dyn, 3 * i, rev ? make_float4(0.f, 0.f, 0.f, kRevoluteFlag) : f4(u, kPrismaticFlag));
    st4(S.f + L.dyn, 3 * i + 1, rev ? f4(u, mu) : make_float4(0.f, 0.f, 0.f, mu));
    st4(S.f + L.dyn, 3 * i + 2, make_float4(a.x * a.x * iM, a.y * a.y * iM, a.z * a.z * iM, a.x * a.y * iM));
    const float e = S.f[L.dyn2 + 4 * i + 2];
    st4(S.f + L.dyn2, i, make_float4(a.x * a.z * iM, a.y * a.z * iM, e, (float)slot));
    const float q = P.joint_state[gi];
    const float gap[2] = {q - P.joint_limits[gi], P.joint_limits[N + gi] - q};
    float* E = pt + 4 + slot * kPartStride;
    E[PART_BODY] = __uint_as_float((uint32_t)i);
    E[PART_KIND] = (float)kind;
    E[PART_M] = M;
    E[PART_IM] = iM;
#pragma unroll
    for (int r = 0; r < 2; r++) {
      E[PART_BIAS + r] = gap[r] > 0.f ? -gap[r] / dt : P.baumgarte / dt * (-gap[r]);
      E[PART_LAM + r] = 0.f;
    }
    E[PART_AX] = a.x;
    E[PART_AX + 1] = a.y;
    E[PART_AX + 2] = a.z;
  }
  if (lane == 0) S.u[L.parts] = (uint32_t)(np < kMaxParts ? np : kMaxParts);
}

// One Gauss-Seidel pass over the parts' limit rows by wave 0, a lane per
// part (the rows of different parts touch different bodies): the lower
// row (+1 on the rate), then the upper (-1), impulses >= 0.  Returns the
// pass's max |dlambda| / M of the lane's part (0 on the other lanes).
__device__ __forceinline__ float part_limit_sweep(const LdsLayout& L, Smem S, int lane) {
  float r = 0.f;
  const int np = (int)S.u[L.parts];
  if (lane < np) {
    float* E = S.f + L.parts + 4 + lane * kPartStride;
    const int i = (int)__float_as_uint(E[PART_BODY]);
    const float M = E[PART_M], iM = E[PART_IM];
    const V3 a = v3(E[PART_AX], E[PART_AX + 1], E[PART_AX + 2]);
    // the slot that carries the rate: angular for a hinge, linear for a slide
    float* u = S.f + L.dyn + kDynWords * i + (E[PART_KIND] == 1.f ? 4 : 0);
    V3 w = v3(u[0], u[1], u[2]);
    float qd = dot(a, w);
#pragma unroll
    for (int k = 0; k < 2; k++) {
      const float sg = k == 0 ? 1.f : -1.f;
      const float l0 = E[PART_LAM + k];
      const float l = fmaxf(0.f, l0 + M * (E[PART_BIAS + k] - sg * qd));
      const float dl = l - l0;
      E[PART_LAM + k] = l;
      qd += sg * dl * iM;
      w = w + a * (sg * dl * iM);
      r = fmaxf(r, fabsf(dl) * iM);
    }
    u[0] = w.x;
    u[1] = w.y;
    u[2] = w.z;
  }
  return r;
}

// Sweeps of projected Gauss-Seidel, colour batch after colour batch; the
// record of a lane's next batch is loaded while the current one is solved.
// Stops after `iters` sweeps or once a sweep's residual is <= tol (tol > 0).
// kPairs: small colours by lane pairs (off where the network's registers
// leave no room for the second update's code).
template <bool kPairs, class TM>
__device__ __forceinline__ void solve_pgs(const LdsLayout& L, Smem S, const float4* rec, int ncol, const uint32_t* cstart, int iters,
                          float tol, uint32_t* misc, int* sweeps_out, float* res_out, const TM tm,
                          const ArmCtx& arm, float motor_max) {
  const int tid = tm.tid, T = tm.T;
  int sweeps = 0;
  float res = 0.f;
  // the arm's motor rows, then the parts' limit rows, after the contacts of
  // every sweep (wave 0)
  auto motors = [&]() __attribute__((always_inline)) -> float {
    float rm = 0.f;
    if (tid < 64) {
      if (arm.on) rm = arm_motor_sweep(L, S, tm, motor_max);
      if (arm.parts) rm = fmaxf(rm, part_limit_sweep(L, S, tid));
    }
    colour_sync(tm);
    return rm;
  };
  if (ncol == 0 && (arm.on || arm.parts)) {  // motor and limit rows only
    for (int it = 0; it < iters; it++) {
      const float r = motors();
      sweeps++;
      if (tol > 0.f || it == iters - 1) {
        res = block_max(r, misc, tm);
        if (tol > 0.f && res <= tol) break;
      }
    }
    *sweeps_out = sweeps;
    *res_out = res;
    return;
  }
  if (ncol == 0) {
    // no rows: every sweep has residual 0, so a tolerance stops after the
    // first one and a fixed count runs all of them (as empty sweeps)
    *sweeps_out = iters > 0 ? (tol > 0.f ? 1 : iters) : 0;
    *res_out = 0.f;
    return;
  }
  // Colour starts in registers, read by a uniform colour index: lane k of
  // every wave holds cstart[k] and cstart[64 + k] (entries past ncol are 0).
  static_assert(kMaxColours == 128, "colour starts held in two lanes' words");
  const int lane = tid & 63;
  const int cs_lo = (int)cstart[lane], cs_hi = (int)cstart[64 + lane];
  const int cs_end = __builtin_amdgcn_readfirstlane((int)cstart[kMaxColours]);
  // The sweeps, instantiated twice: with fewer than 64 colours every colour
  // start is one readlane of cs_lo, without the branches of the general
  // lookup in the loop.
  auto sweep_all = [&](auto small) __attribute__((always_inline)) {
    constexpr bool kSmall = decltype(small)::value;
    auto cst = [&](int c) -> int {
      if constexpr (kSmall) return __builtin_amdgcn_readlane(cs_lo, c);
      else return c < 64 ? __builtin_amdgcn_readlane(cs_lo, c)
                         : (c < 128 ? __builtin_amdgcn_readlane(cs_hi, c - 64) : cs_end);
    };
    const int last = cst(ncol) - 1;  // >= 0: ncol > 0 implies contacts
    // A colour of at most 32 contacts is solved by lane pairs (contact
    // tid / 2, one batch for any team of >= 64 threads), a larger one a
    // contact per lane (contact tid, tid + T, ...).  The choice depends on
    // the colour only, so results do not depend on the team size.
    auto paired = [&](int c) { return kPairs && cst(c + 1) - cst(c) <= 32; };
    bool pair = paired(0);
    int i = cst(0) + (pair ? tid >> 1 : tid);
    bool has = i < cst(1);
    float r = 0.f;
    // One colour batch: load the next batch's records (unconditionally, the
    // index clamped to a valid record, so that the loads stay in flight),
    // solve this batch, synchronise.  Two record buffers alternate between
    // batches so that no registers are copied between them.
    auto batch = [&](int c, const Rec& cur, Rec& nxt) __attribute__((always_inline)) {
      const int e = cst(c + 1);
      // next batch: colour c + 1, or colour 0 of the next sweep
      const int cn = c + 1 < ncol ? c + 1 : 0;
      const bool pnext = paired(cn);
      const int inext = cst(cn) + (pnext ? tid >> 1 : tid);
      const bool hnext = inext < cst(cn + 1);
      nxt = load_rec(rec, min(inext, last));
      if (kPairs && pair) {
        if (has) r = fmaxf(r, pgs_update_pair(L, S, cur, i, tid & 1, arm, c));
      } else {
        if (has) r = fmaxf(r, pgs_update(L, S, cur, i, arm, c));
        for (int i2 = i + T; i2 < e; i2 += T) r = fmaxf(r, pgs_update(L, S, load_rec(rec, i2), i2, arm, c));
      }
      colour_sync(tm);
      has = hnext;
      i = inext;
      pair = pnext;
    };
    Rec ra = load_rec(rec, min(i, last)), rb;
    for (int it = 0; it < iters; it++) {
      r = 0.f;
      int c = 0;
      for (; c + 1 < ncol; c += 2) {
        batch(c, ra, rb);
        batch(c + 1, rb, ra);
      }
      if (c < ncol) {  // odd colour count: colour 0 of the next sweep is in rb
        batch(c, ra, rb);
        ra = rb;
      }
      if (arm.on || arm.parts) r = fmaxf(r, motors());
      sweeps++;
      if (tol > 0.f || it == iters - 1) {
        res = block_max(r, misc, tm);
        if (tol > 0.f && res <= tol) break;
      }
    }
  };
  if (ncol < 64) sweep_all(std::true_type{});
  else sweep_all(std::false_type{});
  *sweeps_out = sweeps;
  *res_out = res;
}

// Sweeps of Jacobi: rows read the velocities of the sweep start, increments
// scaled by 1/max(n_a, n_b) contacts per dynamic body (from the record),
// applied colour-major.
template <class TM>
__device__ __forceinline__ void solve_jacobi(const LdsLayout& L, Smem S, const float4* rec, int nb, int nc, int ncol,
                             const uint32_t* cstart, int iters, float tol, uint32_t* misc, int* sweeps_out,
                             float* res_out, const TM tm) {
  const int tid = tm.tid, T = tm.T;
  float* snap = S.f + L.snap;
  int sweeps = 0;
  float res = 0.f;
  for (int it = 0; it < iters; it++) {
    for (int i = tid; i < nb; i += T) {
      st4(snap, 2 * i, ld4(S.f + L.dyn, 3 * i));
      st4(snap, 2 * i + 1, ld4(S.f + L.dyn, 3 * i + 1));
    }
    team_sync(tm);
    float r = 0.f;
    for (int i = tid; i < nc; i += T) {
      Rec R = load_rec(rec, i);
      const int a = rec_a(R), b = rec_b(R);
      const float4 lam = ld4(S.f + L.lam, i);
      const V3 va = xyz(ld4(snap, 2 * a)), wa = xyz(ld4(snap, 2 * a + 1));
      V3 vb = v3(0.f, 0.f, 0.f), wb = vb;
      if (b >= 0) {
        vb = xyz(ld4(snap, 2 * b));
        wb = xyz(ld4(snap, 2 * b + 1));
      }
      const V3 n = xyz(R.r[0]), ra = xyz(R.r[1]), rb = xyz(R.r[2]);
      const float mn = R.r[0].w, m1 = R.r[1].w, m2 = R.r[2].w;
      const float bias = R.r[3].z, mu = R.r[3].w, sc = R.r[4].y;
      V3 t1, t2;
      tangents_coef(n, R.r[4].z, t1, t2);
      const V3 dv = point_vel(va, wa, vb, wb, ra, rb);
      float ln = fmaxf(0.f, lam.x + sc * mn * (bias - dot(n, dv)));
      float l1 = lam.y - sc * m1 * (dot(t1, dv) + R.r[4].w);
      float l2 = lam.z - sc * m2 * (dot(t2, dv) + lam.w);
      proj_disk(l1, l2, mu * ln);
      float dn = ln - lam.x, d1 = l1 - lam.y, d2 = l2 - lam.z;
      st4(S.f + L.dl, i, make_float4(dn, d1, d2, 0.f));
      st4(S.f + L.lam, i, make_float4(ln, l1, l2, lam.w));
      r = fmaxf(r, fmaxf(fmaxf(fabsf(dn) * frcp(mn), fabsf(d1) * frcp(m1)), fabsf(d2) * frcp(m2)));
    }
    team_sync(tm);
    for (int c = 0; c < ncol; c++) {
      for (int i = (int)cstart[c] + tid; i < (int)cstart[c + 1]; i += T) {
        Rec R = load_rec(rec, i);
        const int a = rec_a(R), b = rec_b(R);
        const float4 dl = ld4(S.f + L.dl, i);
        Vel A = load_vel(L, S, a);
        Vel B = load_vel(L, S, b);
        const V3 n = xyz(R.r[0]);
        V3 t1, t2;
        tangents_coef(n, R.r[4].z, t1, t2);
        apply_impulse(A, B, xyz(R.r[1]), xyz(R.r[2]), n * dl.x + t1 * dl.y + t2 * dl.z);
        store_vel_dyn(L, S, a, A);
        store_vel_dyn(L, S, b, B);
      }
      team_sync(tm);
    }
    sweeps++;
    if (tol > 0.f || it == iters - 1) {
      res = block_max(r, misc, tm);
      if (tol > 0.f && res <= tol) break;
    }
  }
  *sweeps_out = sweeps;
  *res_out = res;
}

// Arm link poses (and, if thd, link velocities) into the LDS records of
// bodies b0..b0+6.
__device__ __forceinline__ void arm_fk(const StepParams& P, const LdsLayout& L, Smem S, int b0, const float* base,
                                       const float* th, const float* thd) {
  V3 c[7], o[7], ax[7];
  float q[7][4];
  arm_chain(base, th, P.link_len, c, q, o, ax);
#pragma unroll
  for (int k = 0; k < 7; k++) {
    int bi = b0 + k;
    float meta = S.f[L.geo + 12 * bi + 3];
    st4(S.f + L.geo, 3 * bi, f4(c[k], meta));
    st4(S.f + L.geo, 3 * bi + 1, make_float4(q[k][0], q[k][1], q[k][2], q[k][3]));
  }
  if (thd) {
#pragma unroll
    for (int k = 0; k < 7; k++) {
      V3 wv = v3(0.f, 0.f, 0.f), vv = v3(0.f, 0.f, 0.f);
#pragma unroll
      for (int j = 0; j <= k; j++) {
        wv = wv + ax[j] * thd[j];
        vv = vv + cross(ax[j], c[k] - o[j]) * thd[j];
      }
      int bi = b0 + k;
      float mu = S.f[L.dyn + kDynWords * bi + 7];
      st4(S.f + L.dyn, 3 * bi, f4(vv, 0.f));
      st4(S.f + L.dyn, 3 * bi + 1, f4(wv, mu));
    }
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Setup of the arm by wave 0: joint origins and axes, M^-1 (M from the link
// Jacobians, then Cholesky), the rates after gravity (the setup rates), the
// motor targets moved by dt times the commanded rates, the motor rows'
// targets and warm start; the rate changes start at zero.  Link poses at
// the step's angles are in LDS; masses and principal inverse inertias of
// the links in global memory.
__device__ __forceinline__ void arm_setup(const StepParams& P, const LdsLayout& L, Smem S, int s, long g0, int l0, float dt, V3 g,
                          int lane) {
  float* arm = S.f + L.arm;
  if (lane == 0) {
    V3 c[7], o[7], ax[7];
    float q[7][4];
    arm_chain(P.arm_base + 3 * s, P.theta + 7 * s, P.link_len, c, q, o, ax);
#pragma unroll
    for (int k = 0; k < 7; k++) {
      arm[ARM_O + 3 * k] = o[k].x; arm[ARM_O + 3 * k + 1] = o[k].y; arm[ARM_O + 3 * k + 2] = o[k].z;
      arm[ARM_AX + 3 * k] = ax[k].x; arm[ARM_AX + 3 * k + 1] = ax[k].y; arm[ARM_AX + 3 * k + 2] = ax[k].z;
    }
  }
  wave_sync();
  auto o_of = [&](int k) { return v3(arm[ARM_O + 3 * k], arm[ARM_O + 3 * k + 1], arm[ARM_O + 3 * k + 2]); };
  auto ax_of = [&](int k) { return v3(arm[ARM_AX + 3 * k], arm[ARM_AX + 3 * k + 1], arm[ARM_AX + 3 * k + 2]); };
  // M, one entry per lane (row-major): links j >= max(i, k) contribute
  // m_j (a_i x (c_j - o_i)) . (a_k x (c_j - o_k)) + a_i . I_j a_k
  if (lane < 49) {
    const int i = lane / 7, k = lane - 7 * (lane / 7);
    const V3 oi = o_of(i), ai = ax_of(i), ok = o_of(k), ak = ax_of(k);
    float m = 0.f;
    for (int j = i > k ? i : k; j < 7; j++) {
      const long gj = g0 + l0 + j;
      const V3 cj = xyz(ld4(S.f + L.geo, 3 * (l0 + j)));
      const float4 qj = ld4(S.f + L.geo, 3 * (l0 + j) + 1);
      const M3 R = quat_R(qj.x, qj.y, qj.z, qj.w);
      const V3 bi = RTv(R, ai), bk = RTv(R, ak);
      const long N = P.n_bodies;
      m += (1.0f / P.inv_mass[gj]) * dot(cross(ai, cj - oi), cross(ak, cj - ok)) +
           bi.x * bk.x / P.inv_inertia[gj] + bi.y * bk.y / P.inv_inertia[N + gj] +
           bi.z * bk.z / P.inv_inertia[2 * N + gj];
    }
    arm[ARM_MI + lane] = m;
  }
  wave_sync();
  if (lane == 0) {  // Cholesky factor and inverse, in registers (indices fixed by unrolling)
    float Lc[7][7];
#pragma unroll
    for (int i = 0; i < 7; i++) {
#pragma unroll
      for (int k = 0; k <= i; k++) {
        float sum = arm[ARM_MI + 7 * i + k];
#pragma unroll
        for (int t = 0; t < k; t++) sum -= Lc[i][t] * Lc[k][t];
        Lc[i][k] = i == k ? sqrtf(sum) : sum / Lc[k][k];
      }
    }
#pragma unroll
    for (int col = 0; col < 7; col++) {
      float y[7], x[7];
#pragma unroll
      for (int i = 0; i < 7; i++) {
        float sum = i == col ? 1.f : 0.f;
#pragma unroll
        for (int t = 0; t < i; t++) sum -= Lc[i][t] * y[t];
        y[i] = sum / Lc[i][i];
      }
#pragma unroll
      for (int i = 6; i >= 0; i--) {
        float sum = y[i];
#pragma unroll
        for (int t = i + 1; t < 7; t++) sum -= Lc[t][i] * x[t];
        x[i] = sum / Lc[i][i];
      }
#pragma unroll
      for (int i = 0; i < 7; i++) arm[ARM_MI + 7 * i + col] = x[i];
    }
  }
  wave_sync();
  // gravity moments about the joint axes, then the setup rates
  if (lane < 7) {
    const V3 oi = o_of(lane), ai = ax_of(lane);
    V3 t = v3(0.f, 0.f, 0.f);
    for (int j = lane; j < 7; j++) {
      const V3 cj = xyz(ld4(S.f + L.geo, 3 * (l0 + j)));
      t = t + cross(cj - oi, g * (1.0f / P.inv_mass[g0 + l0 + j]));
    }
    arm[ARM_BIAS + lane] = dot(ai, t);
  }
  wave_sync();
  float* st = P.arm_state + 21 * s;
  float qref = 0.f;
  if (lane < 7) {
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < 7; k++) a += arm[ARM_MI + 7 * lane + k] * arm[ARM_BIAS + k];
    qref = st[lane] + dt * a;
  }
  wave_sync();
  if (lane < 7) {
    arm[ARM_QREF + lane] = qref;
    arm[ARM_DQ + lane] = 0.f;
    const float tgt = st[7 + lane] + dt * (P.actions ? P.actions[7 * s + lane] : 0.f);
    st[7 + lane] = tgt;
    float err = tgt - P.theta[7 * s + lane];
    err -= 6.28318530717958647692f * rintf(err * 0.15915494309189533577f);
    arm[ARM_BIAS + lane] = P.motor_kp * err / dt - qref;
    arm[ARM_LAM + lane] = P.warm == WARM_COLD ? 0.f : fminf(fmaxf(st[14 + lane], -P.motor_max), P.motor_max);
  }
  wave_sync();
}

// Motor warm start (wave 0): dq += sum_k lambda_k M^-1 e_k.
__device__ __forceinline__ void arm_motor_warm(const LdsLayout& L, Smem S, int lane) {
  float* arm = S.f + L.arm;
  if (lane < 7) {
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < 7; k++) a += arm[ARM_MI + 7 * lane + k] * arm[ARM_LAM + k];
    arm[ARM_DQ + lane] += a;
  }
  wave_sync();
}

// Joint-space rows of a contact on arm link j (directions n, t1, t2 at
// point p, arm side sg): g and M^-1 g to the colour's slot in global
// memory; returns g . M^-1 g per row (k_add), the normal-friction couplings
// g_t . M^-1 g_n (c_add) and the rows' velocities sg g . qref (u_add).
__device__ __forceinline__ void arm_contact_rows(const LdsLayout& L, Smem S, float* slot, int j, V3 p, const V3* dirs, float sg,
                                 float* k_add, float* c_add, float* u_add) {
  const float* arm = S.f + L.arm;
  float w0[7];
#pragma unroll
  for (int r = 0; r < 3; r++) {
    float gr[7];
#pragma unroll
    for (int i = 0; i < 7; i++) {
      const V3 oi = v3(arm[ARM_O + 3 * i], arm[ARM_O + 3 * i + 1], arm[ARM_O + 3 * i + 2]);
      const V3 ai = v3(arm[ARM_AX + 3 * i], arm[ARM_AX + 3 * i + 1], arm[ARM_AX + 3 * i + 2]);
      gr[i] = i <= j ? dot(dirs[r], cross(ai, p - oi)) : 0.f;
      slot[7 * r + i] = gr[i];
    }
    float kk = 0.f, uu = 0.f, cc = 0.f;
#pragma unroll
    for (int i = 0; i < 7; i++) {
      float w = 0.f;
#pragma unroll
      for (int k = 0; k < 7; k++) w += arm[ARM_MI + 7 * i + k] * gr[k];
      slot[21 + 7 * r + i] = w;
      kk += gr[i] * w;
      uu += gr[i] * arm[ARM_QREF + i];
      if (r == 0) w0[i] = w;
      else cc += gr[i] * w0[i];
    }
    k_add[r] = kk;
    u_add[r] = sg * uu;
    if (r > 0) c_add[r - 1] = cc;
  }
}

// One step of scene s by team tm, its working set in the LDS at S laid
// out by L.
// kLearned: the learned warm start (P.warm == WARM_LEARNED) is compiled in;
// the other modes use an instantiation without the network's registers.
// Sleeping islands (localized physics): islands are the sets of dynamic
// bodies joined by this step's contacts between two dynamic bodies, found by
// minimum-label propagation with hooking and pointer jumping (a body's label
// ends as the least index in its island, whatever order the updates take; a
// label never exceeds its body's index, so every chain of labels ends).  An
// island sleeps when every body in it has ended sleep_steps steps at rest and
// none of them touches a kinematic body; a sleeping body gets the asleep bit
// in its meta word and zero velocity, and counts as not dynamic for the
// colouring, the solve and the integration.  A container part (parts
// true: flagged in its inverse-mass word) never sleeps and keeps its island
// awake.  Uses the colouring's per-body scratch (deg, lstart), which is free
// until the colouring starts.
template <class TM>
__device__ __forceinline__ void sleep_islands(const StepParams& P, const LdsLayout& L, Smem S, long b0, int nb, int nc,
                              uint32_t* misc, const TM tm, bool parts) {
  const int tid = tm.tid, T = tm.T;
  uint32_t* lab = S.u + L.deg;
  uint32_t* wake = S.u + L.lstart;
  const uint32_t* ckeys = S.u + L.ckey;
  for (int i = tid; i < nb; i += T) {
    lab[i] = (uint32_t)i;
    wake[i] = 0u;
  }
  team_sync(tm);
  for (int round = 0; round <= nb; round++) {
    if (tid == 0) misc[M_CHANGED] = 0u;
    team_sync(tm);
    bool changed = false;
    for (int q = tid; q < nc; q += T) {
      const uint32_t key = ckeys[q];
      const int a = (int)(key >> 20), b = (int)((key >> 8) & 0xFFFu);
      if (b == (int)kGroundKey || !is_dyn_meta(body_meta(L, S, a)) || !is_dyn_meta(body_meta(L, S, b))) continue;
      const uint32_t la = lab[a], lb = lab[b];
      if (la != lb) {
        const uint32_t m = la < lb ? la : lb;
        atomicMin(&lab[a], m);
        atomicMin(&lab[b], m);
        atomicMin(&lab[la], m);
        atomicMin(&lab[lb], m);
        changed = true;
      }
    }
    if (changed) misc[M_CHANGED] = 1u;
    team_sync(tm);
    for (int i = tid; i < nb; i += T) {
      uint32_t x = lab[i];
      while (lab[x] != x) x = lab[x];
      lab[i] = x;
    }
    team_sync(tm);
    if (misc[M_CHANGED] == 0u) break;
    team_sync(tm);
  }
  for (int i = tid; i < nb; i += T)
    if (is_dyn_meta(body_meta(L, S, i)) &&
        (P.rest[b0 + i] < P.sleep_steps || (parts && S.f[L.dyn + kDynWords * i + 3] < 0.f)))
      wake[lab[i]] = 1u;
  for (int q = tid; q < nc; q += T) {
    const uint32_t key = ckeys[q];
    const int a = (int)(key >> 20), b = (int)((key >> 8) & 0xFFFu);
    if (b == (int)kGroundKey) continue;
    const uint32_t ma = body_meta(L, S, a), mb = body_meta(L, S, b);
    // the arm (kinematic or articulated) wakes what it touches
    const uint32_t ka = (ma >> 8) & 255u, kb = (mb >> 8) & 255u;
    if ((ka == KINEMATIC || ka == ARMLINK) && is_dyn_meta(mb)) wake[lab[b]] = 1u;
    if ((kb == KINEMATIC || kb == ARMLINK) && is_dyn_meta(ma)) wake[lab[a]] = 1u;
  }
  team_sync(tm);
  for (int i = tid; i < nb; i += T) {
    const uint32_t meta = body_meta(L, S, i);
    if (!is_dyn_meta(meta) || wake[lab[i]]) continue;
    S.f[L.geo + 12 * i + 3] = __uint_as_float(meta | kAsleepBit);
    const float4 v = ld4(S.f + L.dyn, 3 * i), w = ld4(S.f + L.dyn, 3 * i + 1);
    st4(S.f + L.dyn, 3 * i, make_float4(0.f, 0.f, 0.f, v.w));
    st4(S.f + L.dyn, 3 * i + 1, make_float4(0.f, 0.f, 0.f, w.w));
  }
  team_sync(tm);
}

// A dynamic body's linear velocity at the setup: the state's, plus gravity
// over the step (read again after the solve, which kept only the change).
__device__ __forceinline__ V3 setup_lin_vel(const StepParams& P, long gi, long N, V3 g, float dt) {
  return v3(P.vel[gi], P.vel[N + gi], P.vel[2 * N + gi]) + g * dt;
}

// kExt: 0 the plain step; 1 with the articulated arm; 2 also with
// container parts; 3 also with convex hulls (each level's code, registers
// and stack stay out of the lower levels' kernels).
template <bool kLearned, int kExt, class TM>
__device__ __forceinline__ void scene_step(const StepParams& P, const LdsLayout& L, Smem S, const int s,
                                           const TM tm) {
  constexpr bool kArt = kExt >= 1;
  const int tid = tm.tid, T = tm.T;
  const int b0 = P.body_offset[s];
  const int nb = P.body_offset[s + 1] - b0;
  const int NB = P.NB, PM = P.PM, CM = P.CM;
  const long N = P.n_bodies;
  uint32_t* misc = S.u + L.misc;
  float4* raw = P.raw + (long)s * CM * 2;
  float4* rec = P.crec + (long)s * rec_stride(PM, CM);
  const float dt = P.dt;
  if (nb > NB) {  // host guarantees otherwise; leave the scene untouched
    if (tid == 0) P.st_flags[s] = FLAG_CAPACITY;
    return;
  }
  // this scene's pair and contact capacities (global arrays keep the batch stride)
  const int PMs = scene_cap(nb, PM), CMs = scene_cap(nb, CM);
  if (tid < kMiscWords) misc[tid] = 0u;
  TRACE(0);

  // ---- load bodies; a2: gravity, world inverse inertia -----------------
  const V3 g = v3(P.gx, P.gy, P.gz);
  // the articulated arm and the container parts (their own kernels:
  // compiled out of the others)
  const bool arm2 = kArt && !kLearned && P.arm == 2;
  const bool parts = kExt >= 2 && !kLearned && P.joint != nullptr;
  const int arm0 = arm2 ? nb - 7 : nb;  // its first link
  for (int i = tid; i < nb; i += T) {
    const long gi = b0 + i;
    int shape = P.shape[gi], motion = P.motion[gi];
    if (arm2 && i >= arm0) motion = ARMLINK;  // moved by the arm's joint rates
    uint32_t meta = (uint32_t)shape | ((uint32_t)motion << 8);
    V3 x = v3(P.pose[gi], P.pose[N + gi], P.pose[2 * N + gi]);
    float qw = P.pose[3 * N + gi], qx = P.pose[4 * N + gi], qy = P.pose[5 * N + gi], qz = P.pose[6 * N + gi];
    st4(S.f + L.geo, 3 * i, f4(x, __uint_as_float(meta)));
    st4(S.f + L.geo, 3 * i + 1, make_float4(qw, qx, qy, qz));
    if (shape == HULL) {  // its bounding box's half-extents, its index in the library
      const int h = (int)P.prm[gi];
      st4(S.f + L.geo, 3 * i + 2, make_float4(P.hull_ext[h].x, P.hull_ext[h].y, P.hull_ext[h].z, (float)h));
    } else {
      st4(S.f + L.geo, 3 * i + 2, make_float4(P.prm[gi], P.prm[N + gi], P.prm[2 * N + gi], 0.f));
    }
    V3 v = v3(P.vel[gi], P.vel[N + gi], P.vel[2 * N + gi]);
    V3 w = v3(P.vel[3 * N + gi], P.vel[4 * N + gi], P.vel[5 * N + gi]);
    float im = 0.f;
    float I[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (motion == DYNAMIC) {
      M3 R = quat_R(qw, qx, qy, qz);
      im = P.inv_mass[gi];
      v = setup_lin_vel(P, gi, N, g, dt);
      float i0 = P.inv_inertia[gi], i1 = P.inv_inertia[N + gi], i2 = P.inv_inertia[2 * N + gi];
      // R diag(i) R^T
      I[0] = R.m[0][0] * R.m[0][0] * i0 + R.m[0][1] * R.m[0][1] * i1 + R.m[0][2] * R.m[0][2] * i2;
      I[1] = R.m[1][0] * R.m[1][0] * i0 + R.m[1][1] * R.m[1][1] * i1 + R.m[1][2] * R.m[1][2] * i2;
      I[2] = R.m[2][0] * R.m[2][0] * i0 + R.m[2][1] * R.m[2][1] * i1 + R.m[2][2] * R.m[2][2] * i2;
      I[3] = R.m[0][0] * R.m[1][0] * i0 + R.m[0][1] * R.m[1][1] * i1 + R.m[0][2] * R.m[1][2] * i2;
      I[4] = R.m[0][0] * R.m[2][0] * i0 + R.m[0][1] * R.m[2][1] * i1 + R.m[0][2] * R.m[2][2] * i2;
      I[5] = R.m[1][0] * R.m[2][0] * i0 + R.m[1][1] * R.m[2][1] * i1 + R.m[1][2] * R.m[2][2] * i2;
    } else if (motion == STATIC || motion == ARMLINK) {
      v = v3(0.f, 0.f, 0.f);
      w = v3(0.f, 0.f, 0.f);
    }
    st4(S.f + L.dyn, 3 * i, f4(v, im));
    st4(S.f + L.dyn, 3 * i + 1, f4(w, P.friction[gi]));
    st4(S.f + L.dyn, 3 * i + 2, make_float4(I[0], I[1], I[2], I[3]));
    st4(S.f + L.dyn2, i, make_float4(I[4], I[5], P.restitution[gi], 0.f));
  }
  // ground slot: zero velocity, inverse mass and inverse inertia
  if (tid < kDynWords) S.f[L.dyn - kDynWords + tid] = 0.f;
  if (tid < 4) S.f[L.dyn2 - 4 + tid] = 0.f;
  team_sync(tm);
  if (parts) {  // the parts' rates, projectors and limit rows
    if (tid < 64) part_setup(P, L, S, b0, nb, dt, g, tid);
    team_sync(tm);
  }
  TRACE(1);
  // ---- a1: arm at theta_t, link velocities from the actions -------------
  float thd[7];
  if (P.arm) {
#pragma unroll
    for (int k = 0; k < 7; k++) thd[k] = P.actions ? P.actions[7 * s + k] : 0.f;
    if (tid == 0) {  // (two calls: a selected array pointer would put the array in scratch)
      if (arm2) arm_fk(P, L, S, nb - 7, P.arm_base + 3 * s, P.theta + 7 * s, nullptr);
      else arm_fk(P, L, S, nb - 7, P.arm_base + 3 * s, P.theta + 7 * s, thd);
    }
    team_sync(tm);
    if (arm2) {
      if (tid < 64) arm_setup(P, L, S, s, b0, arm0, dt, g, tid);
      team_sync(tm);
    }
  }

  // ---- a3: AABBs and sort keys ------------------------------------------
  for (int i = tid; i < nb; i += T) {
    Geom G = load_geom(L, S, i);
    V3 lo, hi;
    if (G.shape == SPHERE) {
      float e = G.p[0] + P.margin;
      lo = G.x - v3(e, e, e);
      hi = G.x + v3(e, e, e);
    } else if (G.shape == BOX || G.shape == HULL) {  // a hull: its bounding box
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
    uint32_t meta = body_meta(L, S, i);
    st4(S.f + L.lo, i, f4(lo, is_dyn_meta(meta) ? 1.f : (((meta >> 8) & 255u) == ARMLINK ? 2.f : 0.f)));
    // a part: 1 + the local index of the base it is joined to (never a pair)
    float base = 0.f;
    if (parts && S.f[L.dyn + kDynWords * i + 3] < 0.f) base = (float)(P.joint_parent[b0 + i] + 1);
    st4(S.f + L.hi, i, f4(hi, base));
    S.u[L.skey + i] = orderable(lo.x);
    S.u[L.sval + i] = (uint32_t)i;
  }
  team_sync(tm);
  TRACE(2);

  // ---- a4: radix sort bodies by AABB minimum along x --------------------
  int sw = 1;
  if (nb <= kRankSortMax)
    lds_rank_sort<false>(S.u + L.skey, S.u + L.sval, S.u + L.skey2, S.u + L.sval2, nb, tm);
  else
    sw = lds_radix_sort(S.u + L.skey, S.u + L.sval, S.u + L.skey2, S.u + L.sval2, nb, 0, 4, S.u + L.hist,
                        S.u + L.hbase, misc, tm);
  const uint32_t* order = S.u + (sw ? L.sval2 : L.sval);
  TRACE(3);

  // ---- a5: sweep and prune -> pairs (unordered), then canonical sort ----
  // Sorted position p's candidates are the positions after it whose AABB
  // starts at or before its end along x.  Their counts are found by binary
  // search and scanned, and the candidates are dealt to the lanes in equal
  // contiguous runs (a long body's run no longer holds up the team).
  uint32_t* pk = S.u + L.pk;
  {
    const uint32_t* skeys = S.u + (sw ? L.skey2 : L.skey);  // sorted orderable minimum x
    uint32_t* run = S.u + (sw ? L.skey : L.skey2);          // free sort buffer: [nb] run starts
    for (int p = tid; p < nb; p += T) {
      const uint32_t hx = orderable(ld4(S.f + L.hi, (int)order[p]).x);
      int lo = p + 1, hi = nb;  // first position whose minimum x exceeds hx
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (skeys[mid] > hx) hi = mid;
        else lo = mid + 1;
      }
      run[p] = (uint32_t)(lo - p - 1);
    }
    team_sync(tm);
    const uint32_t total = block_exclusive_scan(run, nb, misc, tm);
    const uint32_t c0 = (uint32_t)(((uint64_t)total * tid) / T), c1 = (uint32_t)(((uint64_t)total * (tid + 1)) / T);
    if (c0 < c1) {
      // the last position whose run starts at or before c0
      int lo = 0, hi = nb;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (run[mid] <= c0) lo = mid;
        else hi = mid;
      }
      int p = lo;
      uint32_t pend = p + 1 < nb ? run[p + 1] : total;
      int q = p + 1 + (int)(c0 - run[p]);
      int i = (int)order[p];
      float4 loi = ld4(S.f + L.lo, i), hii = ld4(S.f + L.hi, i);
      for (uint32_t c = c0; c < c1; c++) {
        while (c >= pend) {  // next position with a non-empty run
          p++;
          pend = p + 1 < nb ? run[p + 1] : total;
          q = p + 1;
          i = (int)order[p];
          loi = ld4(S.f + L.lo, i);
          hii = ld4(S.f + L.hi, i);
        }
        const int j = (int)order[q++];
        const float4 loj = ld4(S.f + L.lo, j);
        if (loi.w == 0.f && loj.w == 0.f) continue;  // neither body moves
        if (loi.w == 2.f && loj.w == 2.f) continue;  // two links of the arm: joined, not in contact
        const float4 hij = ld4(S.f + L.hi, j);
        if (loj.y <= hii.y && loi.y <= hij.y && loj.z <= hii.z && loi.z <= hij.z) {
          if (parts && (hii.w == (float)(j + 1) || hij.w == (float)(i + 1))) continue;  // a part and its base
          int a = i < j ? i : j, bb = i < j ? j : i;
          uint32_t slot = atomicAdd(&misc[M_NPAIRS], 1u);
          if ((int)slot < PMs) pk[slot] = ((uint32_t)a << 11) | (uint32_t)bb;
        }
      }
    }
    // ground pairs of dynamic bodies and arm links reaching z <= 0
    for (int i = tid; i < nb; i += T) {
      const float4 loi = ld4(S.f + L.lo, i);
      if (loi.w != 0.f && loi.z <= 0.f) {
        uint32_t slot = atomicAdd(&misc[M_NPAIRS], 1u);
        if ((int)slot < PMs) pk[slot] = ((uint32_t)i << 11) | 2047u;
      }
    }
  }
  team_sync(tm);
  TRACE(4);
  const int npairs_all = (int)misc[M_NPAIRS];
  const int np = npairs_all < PMs ? npairs_all : PMs;
  if (npairs_all > PMs && tid == 0) misc[M_FLAGS] |= FLAG_CAPACITY;
  // keys are unique: sort keys only (values ride along in the same buffers)
  int swp = 1;
  if (T == 64 && np <= 512) {  // one wave: bitonic sort in registers
    uint32_t* pk2 = S.u + L.pk2;
    wave_sort512(np, tid, [&](int e) { return pk[e]; }, [&](int e, uint32_t k) { pk2[e] = k; });
    team_sync(tm);
  } else if (np <= kRankSortMax) {
    lds_rank_sort<true>(pk, nullptr, S.u + L.pk2, nullptr, np, tm);
  } else {
    swp = lds_radix_sort(pk, pk, S.u + L.pk2, S.u + L.pk2, np, 0, 3, S.u + L.hist, S.u + L.hbase, misc, tm);
  }
  const uint32_t* pairs = swp ? S.u + L.pk2 : pk;
  if (P.export_on) {
    for (int p = tid; p < np; p += T) {
      uint32_t k = pairs[p];
      uint32_t a = k >> 11, bb = k & 2047u;
      P.x_pair[(long)s * PM + p] = (a << 16) | (bb == 2047u ? kGroundPair : bb);
    }
  }
  TRACE(5);

  // ---- a6: narrowphase, compaction in canonical order --------------------
  // Pairs run grouped by shape class, so that a wave executes one contact
  // routine at a time; each pair's contacts (at most 4) are staged in the
  // record buffer (free until setup; 8 PM float4 per scene), then compacted
  // in canonical order.
  {
    const int lane = tid & 63, w = tid >> 6, W = T >> 6;
    uint32_t* nperm = S.u + L.nperm;
    uint8_t* ncnt = reinterpret_cast<uint8_t*>(S.u + L.ncnt);
    uint32_t* cbase = S.u + L.hbase;  // class bases (hbase and hist are free after the pair sort)
    uint32_t* whist = S.u + L.hist;   // [W][16] per-wave class counts of a tile
    float4* stage = rec;              // [PMs][4][2] float4
    auto pair_class = [&](int p) -> uint32_t {
      const uint32_t k = pairs[p];
      const int a = (int)(k >> 11), bb = (int)(k & 2047u);
      const uint32_t sa = body_meta(L, S, a) & 255u;
      if (bb == 2047) return 10u + sa;
      const uint32_t sb = body_meta(L, S, bb) & 255u;
      // the 10 unordered shape pairs of 4 shapes: lo * 4 + hi - lo (lo + 1) / 2
      const uint32_t lo = sa < sb ? sa : sb, hi = sa < sb ? sb : sa;
      return lo * 4u + hi - (lo * (lo + 1u)) / 2u;
    };
    for (int i = tid; i < 16 + 16 * W; i += T) {
      if (i < 16) cbase[i] = 0u;
      else whist[i - 16] = 0u;
    }
    team_sync(tm);
    for (int p = tid; p < np; p += T) atomicAdd(&cbase[pair_class(p)], 1u);
    team_sync(tm);
    if (tid == 0) {
      uint32_t run = 0;
      for (int c = 0; c < 16; c++) {
        const uint32_t v = cbase[c];
        cbase[c] = run;
        run += v;
      }
    }
    team_sync(tm);
    // stable placement by class: rank among the wave's lanes of the same
    // class (four ballots), then the counts of earlier waves and tiles
    for (int t0 = 0; t0 < np; t0 += T) {
      const int p = t0 + tid;
      const bool valid = p < np;
      const uint32_t c = valid ? pair_class(p) : 0u;
      u64 peers = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 4; bit++) {
        const u64 bb = __ballot(valid && ((c >> bit) & 1u));
        peers &= ((c >> bit) & 1u) ? bb : ~bb;
      }
      const unsigned rank = lanes_below(peers);
      if (valid && rank == 0) whist[w * 16 + c] = (uint32_t)__popcll(peers);
      team_sync(tm);
      if (valid) {
        uint32_t off = cbase[c] + rank;
        for (int ww = 0; ww < w; ww++) off += whist[ww * 16 + c];
        nperm[off] = (uint32_t)p;
      }
      team_sync(tm);
      for (int cc = tid; cc < 16; cc += T) {
        uint32_t sum = 0;
        for (int ww = 0; ww < W; ww++) {
          sum += whist[ww * 16 + cc];
          whist[ww * 16 + cc] = 0u;
        }
        cbase[cc] += sum;
      }
      team_sync(tm);
    }
    // contacts of every pair, class by class, staged at the pair's slots
    for (int j = tid; j < np; j += T) {
      const int p = (int)nperm[j];
      const uint32_t k = pairs[p];
      const int a = (int)(k >> 11), bb = (int)(k & 2047u);
      Out4 o;
      o.n = 0;
      Geom A = load_geom(L, S, a);
      if constexpr (kExt == 3) {  // convex hulls: only in their own kernels
        const HullLib HL{P.hull_info, P.hull_vert, P.hull_plane, P.hull_loop, P.hull_edge};
        if (bb == 2047) {
          if (A.shape == HULL) hull_ground(A, HL, P.margin, o);
          else ground_contacts(A, P.margin, o);
        } else {
          Geom B = load_geom(L, S, bb);
          if (A.shape == HULL || B.shape == HULL) collide_hull(A, B, HL, P.margin, o);
          else collide(A, B, P.margin, o);
        }
      } else {
        if (bb == 2047) {
          ground_contacts(A, P.margin, o);
        } else {
          Geom B = load_geom(L, S, bb);
          collide(A, B, P.margin, o);
        }
      }
      ncnt[p] = (uint8_t)o.n;
#pragma unroll
      for (int kk = 0; kk < 4; kk++) {
        if (kk >= o.n) break;
        const PC c = o.get(kk);
        stage[8 * p + 2 * kk] = f4(c.n, c.phi);
        stage[8 * p + 2 * kk + 1] = f4(c.p, __int_as_float(c.f));
      }
    }
    team_sync(tm);
    // compaction in canonical pair order: prefix of the counts by ballots;
    // a tile's staged contacts are read first, so that the loads overlap the
    // prefix and its synchronisation
    uint32_t base = 0;
    for (int t0 = 0; t0 < np; t0 += T) {
      const int p = t0 + tid;
      const int cnt = p < np ? (int)ncnt[p] : 0;
      float4 sv[8];
#pragma unroll
      for (int kk = 0; kk < 4; kk++) {
        if (kk < cnt) {
          sv[2 * kk] = stage[8 * p + 2 * kk];
          sv[2 * kk + 1] = stage[8 * p + 2 * kk + 1];
        }
      }
      u64 b0m = __ballot(cnt & 1), b1m = __ballot((cnt >> 1) & 1), b2m = __ballot((cnt >> 2) & 1);
      uint32_t pre = lanes_below(b0m) + 2u * lanes_below(b1m) + 4u * lanes_below(b2m);
      uint32_t wtot = (uint32_t)(__popcll(b0m) + 2 * __popcll(b1m) + 4 * __popcll(b2m));
      if (lane == 0) misc[M_WAVE + w] = wtot;
      team_sync(tm);
      uint32_t off = base + pre;
      uint32_t tile = 0;
      for (int ww = 0; ww < W; ww++) {
        uint32_t t = misc[M_WAVE + ww];
        if (ww < w) off += t;
        tile += t;
      }
      if (cnt > 0) {
        const uint32_t k = pairs[p];
        const uint32_t a = k >> 11, bb = k & 2047u;
        const uint32_t bkey = bb == 2047u ? kGroundKey : bb;
#pragma unroll
        for (int kk = 0; kk < 4; kk++) {
          const uint32_t q = off + (uint32_t)kk;
          if (kk < cnt && (int)q < CMs) {
            const float4 s0 = sv[2 * kk], s1 = sv[2 * kk + 1];
            S.u[L.ckey + q] = (a << 20) | (bkey << 8) | (uint32_t)__float_as_int(s1.w);
            raw[2 * q] = s0;
            raw[2 * q + 1] = make_float4(s1.x, s1.y, s1.z, 0.f);
          }
        }
      }
      base += tile;
      team_sync(tm);
    }
    if (tid == 0) {
      misc[M_NCONT] = base;
      if ((int)base > CMs) misc[M_FLAGS] |= FLAG_CAPACITY;
    }
  }
  team_sync(tm);
  TRACE(6);
  const int nc_all = (int)misc[M_NCONT];
  const int nc = nc_all < CMs ? nc_all : CMs;
  // sleeping islands (not compiled into the learned kernels, whose registers
  // are at their limit: the library refuses sleeping with the learned start)
  if constexpr (!kLearned) {
    if (P.sleep_speed > 0.f) sleep_islands(P, L, S, b0, nb, nc, misc, tm, parts);
  }

  // ---- a9: colouring -----------------------------------------------------
  uint32_t* deg = S.u + L.deg;
  uint32_t* lstart = S.u + L.lstart;
  uint32_t* list = S.u + L.list;
  uint32_t* rank = S.u + L.rank;
  uint32_t* colour = S.u + L.colour;
  const uint32_t* ckeys = S.u + L.ckey;
  // Starting colours: the colour a contact had in the previous step (found
  // by its key among the sorted previous keys; keys and colours are copied
  // for the search into the scratch that the lists use next), else 0.  The colouring's fixed
  // point does not depend on where the iteration starts; a start close to
  // it only takes fewer rounds.
  {
    const int np0 = P.prev_count ? (P.prev_count[s] < CMs ? P.prev_count[s] : CMs) : 0;
    uint32_t* pkeys = S.u + L.deg;
    uint8_t* pcols = reinterpret_cast<uint8_t*>(S.u + L.deg + CM);  // [CM] bytes after the keys
    for (int i = tid; i < np0; i += T) {
      pkeys[i] = P.prev_key[(long)s * CM + i];
      pcols[i] = P.prev_col[(long)s * CM + i];
    }
    team_sync(tm);
    // both key lists are sorted: each thread takes a contiguous run of
    // contacts, finds the first by binary search and merges the rest
    const int chunk = (nc + T - 1) / T, q0 = tid * chunk, q1 = min(nc, q0 + chunk);
    if (q0 < q1) {
      int pos = 0, hi = np0;  // first previous key >= the run's first key
      const uint32_t k0 = ckeys[q0];
      while (pos < hi) {
        const int mid = (pos + hi) >> 1;
        if (pkeys[mid] < k0) pos = mid + 1;
        else hi = mid;
      }
      for (int q = q0; q < q1; q++) {
        const uint32_t key = ckeys[q];
        while (pos < np0 && pkeys[pos] < key) pos++;
        const int hit = pos < np0 && pkeys[pos] == key ? pos : -1;
        const uint32_t g = hit >= 0 ? (uint32_t)pcols[hit] : 0u;
        colour[q] = g < (uint32_t)kMaxColours ? g : 0u;
        S.u[L.lam + q] = (uint32_t)hit;  // the setup's previous-impulse slot (lam is free until then)
      }
    }
    team_sync(tm);
  }
  // per-body lists of contacts (awake dynamic bodies only, and the
  // articulated arm as one body: its links share the list of its first
  // link, since every contact on the arm moves the same joint rates),
  // canonical order
  auto cbody = [&](int i) { return (arm2 && i >= arm0) ? arm0 : i; };
  auto conflicts = [&](int i) { return (arm2 && i >= arm0) || is_awake_meta(body_meta(L, S, i)); };
  for (int i = tid; i <= nb; i += T) deg[i] = 0u;
  team_sync(tm);
  for (int q = tid; q < nc; q += T) {
    uint32_t key = ckeys[q];
    int a = (int)(key >> 20), b = (int)((key >> 8) & 0xFFFu);
    if (conflicts(a)) atomicAdd(&deg[cbody(a)], 1u);
    if (b != (int)kGroundKey && conflicts(b)) atomicAdd(&deg[cbody(b)], 1u);
  }
  team_sync(tm);
  for (int i = tid; i <= nb; i += T) lstart[i] = i < nb ? deg[i] : 0u;
  team_sync(tm);
  block_exclusive_scan(lstart, nb + 1, misc, tm);
  // fill unordered (deg becomes the per-body count again), then
  // insertion-sort each body's short list
  for (int i = tid; i < nb; i += T) deg[i] = 0u;
  team_sync(tm);
  for (int q = tid; q < nc; q += T) {
    uint32_t key = ckeys[q];
    int a = (int)(key >> 20), b = (int)((key >> 8) & 0xFFFu);
    if (conflicts(a)) list[lstart[cbody(a)] + atomicAdd(&deg[cbody(a)], 1u)] = (uint32_t)q;
    if (b != (int)kGroundKey && conflicts(b)) list[lstart[cbody(b)] + atomicAdd(&deg[cbody(b)], 1u)] = (uint32_t)q;
    rank[q] = 0u;
  }
  team_sync(tm);
  // rank of each contact in its bodies' lists (canonical order): the number
  // of smaller contact indices in the same list, one list entry per lane
  // (its body by binary search of the list starts); low half for a, high
  // half for b.  The lists themselves stay unordered.
  const int ltot = (int)lstart[nb];
  for (int x = tid; x < ltot; x += T) {
    int lo = 0, hi = nb;  // the body i with lstart[i] <= x < lstart[i + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if ((int)lstart[mid] <= x) lo = mid;
      else hi = mid;
    }
    const uint32_t s0 = lstart[lo], e0 = lstart[lo + 1], v = list[x];
    uint32_t r = 0u;
    for (uint32_t y = s0; y < e0; y++) r += list[y] < v ? 1u : 0u;
    // both bodies of a contact write its rank word: combine atomically
    atomicOr(&rank[v], cbody((int)(ckeys[v] >> 20)) == lo ? r : r << 16);
  }
  team_sync(tm);
  TRACE(7);
  // fixed point of c_q = mex{c_p : p < q, p shares a dynamic body with q};
  // its unique solution is sequential first fit in canonical order.  The
  // contacts are taken a team's width at a time in canonical order: earlier
  // chunks are final, so each chunk iterates to its own fixed point, which
  // takes at most as many rounds as its longest dependency chain (one when
  // the starting colours are already the solution).  From here on the
  // per-body lists hold colours: slot lstart[i] + k is the colour of body
  // i's k-th contact, written by that contact, so that a contact reads its
  // predecessors' colours as one contiguous run per body.
  for (int q = tid; q < nc; q += T) {
    const uint32_t key = ckeys[q];
    const int a = (int)(key >> 20), b = (int)((key >> 8) & 0xFFFu);
    const uint32_t rk = rank[q];
    if (conflicts(a)) list[lstart[cbody(a)] + (rk & 0xFFFFu)] = colour[q];
    if (b != (int)kGroundKey && conflicts(b)) list[lstart[cbody(b)] + (rk >> 16)] = colour[q];
  }
  team_sync(tm);
  for (int c0 = 0; c0 < nc; c0 += T) {
    const int q = c0 + tid;
    bool valid = q < nc;
    int la = 0, lb = 0;
    bool da = false, db = false;
    uint32_t sa = 0u, sb = 0u;
    if (valid) {
      const uint32_t key = ckeys[q];
      const int a = (int)(key >> 20), b = (int)((key >> 8) & 0xFFFu);
      const uint32_t rk = rank[q];
      da = conflicts(a);
      db = b != (int)kGroundKey && conflicts(b);
      la = da ? (int)(rk & 0xFFFFu) : 0;
      lb = db ? (int)(rk >> 16) : 0;
      sa = da ? lstart[cbody(a)] : 0u;
      sb = db ? lstart[cbody(b)] : 0u;
      if constexpr (!kLearned) {  // (nothing sleeps in the learned kernels)
        if (!da && !db) {  // every dynamic body of the contact sleeps: not solved
          colour[q] = kSleepColour;
          valid = false;
        }
      }
    }
    for (int round = 0; round <= T + 1; round++) {
      if (tid == 0) misc[M_CHANGED] = 0u;
      team_sync(tm);
      bool changed = false;
      if (valid) {
        // colours below 64 as one 64-bit mask, four independent reads at a time
        u64 m = 0ull;
        uint32_t cmax = 0u;
        auto scan = [&](uint32_t s0, int n) {
          int x = 0;
          for (; x + 4 <= n; x += 4) {
            const uint32_t c0 = list[s0 + x], c1 = list[s0 + x + 1], c2 = list[s0 + x + 2], c3 = list[s0 + x + 3];
            m |= (1ull << (c0 & 63u)) | (1ull << (c1 & 63u)) | (1ull << (c2 & 63u)) | (1ull << (c3 & 63u));
            cmax = max(cmax, max(max(c0, c1), max(c2, c3)));
          }
          for (; x < n; x++) {
            const uint32_t c = list[s0 + x];
            m |= 1ull << (c & 63u);
            cmax = max(cmax, c);
          }
        };
        scan(sa, la);
        scan(sb, lb);
        uint32_t c;
        if (cmax < 64u) {
          c = ~m ? (uint32_t)__builtin_ctzll(~m) : 64u;
        } else {  // colours of 64 and above: the full 128-bit mask
          uint32_t m4[4] = {0u, 0u, 0u, 0u};
          for (int x = 0; x < la + lb; x++) {
            const uint32_t cc = x < la ? list[sa + x] : list[sb + (x - la)];
            m4[cc >> 5] |= 1u << (cc & 31u);
          }
          if (~m4[0]) c = __builtin_ctz(~m4[0]);
          else if (~m4[1]) c = 32 + __builtin_ctz(~m4[1]);
          else if (~m4[2]) c = 64 + __builtin_ctz(~m4[2]);
          else if (~m4[3]) c = 96 + __builtin_ctz(~m4[3]);
          else c = kMaxColours - 1;  // overflow: flagged below
        }
        if (c != colour[q]) {
          colour[q] = c;
          if (da) list[sa + la] = c;
          if (db) list[sb + lb] = c;
          changed = true;
        }
      }
      if (changed) misc[M_CHANGED] = 1u;
      team_sync(tm);
      if (misc[M_CHANGED] == 0u) break;
      team_sync(tm);
    }
  }
  TRACE(8);
  for (int q = tid; q < nc; q += T)
    if (colour[q] == kMaxColours - 1) atomicOr(&misc[M_FLAGS], (uint32_t)FLAG_CAPACITY);
  // stable sort of contact indices by colour -> colour-major order; the sort
  // works on copies so `colour` stays indexed by contact
  if (T == 64 && nc <= 512) {  // one wave: bitonic sort of (colour, contact) keys in registers
    uint32_t* permw = S.u + L.perm;
    wave_sort512(nc, tid, [&](int e) { return (colour[e] << 16) | (uint32_t)e; },
                 [&](int e, uint32_t k) { permw[e] = k & 0xFFFFu; rank[e] = k >> 16; });
    team_sync(tm);
  } else {
    uint32_t* cidx = S.u + L.cv0;
    uint32_t* csk = S.u + L.ck1;
    for (int q = tid; q < nc; q += T) {
      cidx[q] = (uint32_t)q;
      csk[q] = colour[q];
    }
    team_sync(tm);
    lds_radix_sort(csk, cidx, rank, S.u + L.perm, nc, 0, 1, S.u + L.hist, S.u + L.hbase, misc, tm);
  }
  const uint32_t* perm = S.u + L.perm;
  const uint32_t* scol = rank;       // sorted colours (one pass: result in (k1, v1))
  uint32_t* cstart = S.u + L.hbase;  // colour starts (hbase is free again)
  for (int i = tid; i <= kMaxColours; i += T) cstart[i] = 0u;
  team_sync(tm);
  for (int i = tid; i < nc; i += T) {
    uint32_t c = scol[i];
    if (i == 0 || scol[i - 1] != c) cstart[c] = (uint32_t)i;
    // the last solved contact: colour count and solved-contact count
    if (c < kSleepColour && (i == nc - 1 || scol[i + 1] >= kSleepColour)) {
      misc[M_NCOL] = c + 1;
      misc[M_NACT] = (uint32_t)(i + 1);
    }
  }
  team_sync(tm);
  const int ncol = nc > 0 ? (int)misc[M_NCOL] : 0;
  // contacts solved (the rest sleep), colour-major first
  const int nact = kLearned ? nc : (nc > 0 ? (int)misc[M_NACT] : 0);
  if (tid == 0) cstart[ncol] = (uint32_t)nact;
  team_sync(tm);
  TRACE(9);

  // ---- a7/a10: previous impulses, constraint setup (colour-major) ------
  // previous-impulse slot of every contact (found with the starting colours
  // and parked in the impulse array), colour-major, so that the setup loop
  // can load the impulses together with its other inputs (rank is free
  // after the colour sort)
  int32_t* hits = reinterpret_cast<int32_t*>(S.u + L.rank);
  for (int i = tid; i < nc; i += T) hits[i] = (int32_t)S.u[L.lam + perm[i]];
  if (kLearned)
    for (int i = tid; i < (nc + 31) / 32; i += T) S.u[L.fresh + i] = 0u;
  team_sync(tm);
  const float gmag = sqrtf(P.gx * P.gx + P.gy * P.gy + P.gz * P.gz);
  // The global inputs of a contact (narrowphase output, previous impulses)
  // are loaded one tile ahead of its setup.
  struct SetupIn {
    float4 r0, r1, pl;
    int hit;
  };
  auto fetch = [&](int i) {
    SetupIn f;
    const int q = (int)perm[i];
    f.r0 = raw[2 * q];
    f.r1 = raw[2 * q + 1];
    f.hit = hits[i];
    f.pl = make_float4(0.f, 0.f, 0.f, 0.f);
    if (f.hit >= 0) {
      const long o = (long)s * CM + f.hit;
      f.pl = make_float4(P.prev_lam[o], P.prev_lam[P.scene_cm + o], P.prev_lam[2 * P.scene_cm + o],
                         P.prev_lam[3 * P.scene_cm + o]);
    }
    return f;
  };
  // Wave-uniform trip count: the network's matrix-core calls need all 64
  // lanes of a wave; lanes past the end redo the last contact, store nothing.
  const int lane = tid & 63;
  SetupIn nxt;
  if (tid - lane < nc) nxt = fetch(tid < nc ? tid : nc - 1);
  for (int ib = tid - lane; ib < nc; ib += T) {
    const bool live = ib + lane < nc;
    const int i = live ? ib + lane : nc - 1;
    const int q = (int)perm[i];
    const SetupIn in = nxt;
    if (ib + T < nc) nxt = fetch(ib + T + lane < nc ? ib + T + lane : nc - 1);
    float4 r0 = in.r0, r1 = in.r1;
    float phi = r0.w;
    V3 n = xyz(r0), p = xyz(r1);
    uint32_t key = ckeys[q];
    int a = (int)(key >> 20);
    uint32_t bk = (key >> 8) & 0xFFFu;
    int b = bk == kGroundKey ? -1 : (int)bk;
    struct {
      V3 ra, rb;
    } c;
    c.ra = p - xyz(ld4(S.f + L.geo, 3 * a));
    c.rb = b >= 0 ? p - xyz(ld4(S.f + L.geo, 3 * b)) : v3(0.f, 0.f, 0.f);
    Dyn A = load_dyn(L, S, a);
    Dyn B;
    if (b >= 0) {
      B = load_dyn(L, S, b);
    } else {
      B.v = v3(0.f, 0.f, 0.f);
      B.w = v3(0.f, 0.f, 0.f);
      B.im = 0.f;
      B.mu = 0.f;
      for (int k = 0; k < 6; k++) B.I[k] = 0.f;
    }
    float eA = S.f[L.dyn2 + 4 * a + 2];
    float mub = b >= 0 ? B.mu : P.ground_mu;
    float eb = b >= 0 ? S.f[L.dyn2 + 4 * b + 2] : P.ground_e;
    float mu = sqrtf(A.mu * mub);
    float e = fmaxf(eA, eb);
    V3 t1, t2;
    tangents_fast(n, t1, t2);
    Row rw[3];
    V3 dirs[3] = {n, t1, t2};
    float k3[3];
    // a contact on the articulated arm: its joint-space rows (to the colour's slot)
    float asg = 0.f, ka[3] = {0.f, 0.f, 0.f}, kc[2] = {0.f, 0.f}, ua[3] = {0.f, 0.f, 0.f};
    if (arm2) {
      asg = a >= arm0 ? 1.f : (b >= arm0 ? -1.f : 0.f);
      if (asg != 0.f && live)
        arm_contact_rows(L, S, P.arm_rows + ((long)s * kMaxColours + colour[q]) * kArmRowWords,
                         (asg > 0.f ? a : b) - arm0, p, dirs, asg, ka, kc, ua);
    }
    // a container part: a hinge's lever arm runs from its hinge point; a
    // slide's rows act through its linear projector (d . (a a^T / M) d)
    bool slideA = false, slideB = false;
    float imA = A.im, imB = B.im;
    if (parts) {
      if (A.im == kRevoluteFlag) c.ra = p - v3(P.joint_anchor[b0 + a], P.joint_anchor[N + b0 + a],
                                                P.joint_anchor[2 * N + b0 + a]);
      if (b >= 0 && B.im == kRevoluteFlag)
        c.rb = p - v3(P.joint_anchor[b0 + b], P.joint_anchor[N + b0 + b], P.joint_anchor[2 * N + b0 + b]);
      slideA = A.im == kPrismaticFlag;
      slideB = B.im == kPrismaticFlag;
      imA = fmaxf(A.im, 0.f);
      imB = fmaxf(B.im, 0.f);
    }
#pragma unroll
    for (int r = 0; r < 3; r++) {
      rw[r].d = dirs[r];
      rw[r].ca = slideA ? dirs[r] : cross(c.ra, dirs[r]);
      rw[r].ia = Imul(A.I, rw[r].ca);
      float k = imA + dot(rw[r].ca, rw[r].ia) + ka[r];
      if (b >= 0) {
        rw[r].cb = slideB ? dirs[r] : cross(c.rb, dirs[r]);
        rw[r].ib = Imul(B.I, rw[r].cb);
        k += imB + dot(rw[r].cb, rw[r].ib);
      } else {
        rw[r].cb = v3(0.f, 0.f, 0.f);
        rw[r].ib = v3(0.f, 0.f, 0.f);
      }
      k3[r] = k;
      rw[r].m = 1.0f / k;
    }
    const V3 pa = A.v + cross(A.w, c.ra), pb = B.v + cross(B.w, c.rb);
    V3 vr = pa - pb;
    if (asg != 0.f) vr = vr + n * ua[0] + t1 * ua[1] + t2 * ua[2];  // the arm link's point velocity
    float u0 = dot(n, vr);
    // the rows' velocities from the dynamic bodies' velocities at the setup
    // (the solve tracks velocity changes from here; kinematic bodies' and
    // container parts' velocities stay whole)
    const V3 vf = (A.im > 0.f ? pa : v3(0.f, 0.f, 0.f)) - (B.im > 0.f ? pb : v3(0.f, 0.f, 0.f));
    float bias = phi > 0.f ? -phi / dt : P.baumgarte / dt * fmaxf(0.f, -phi - P.slop);
    if (e > 0.f && u0 < -P.rest_thresh) bias = fmaxf(bias, -e * u0);
    // previous impulse (normal, and the friction impulse re-projected on the
    // new tangents)
    const int hit = in.hit;
    float lp0 = 0.f, lp1 = 0.f, lp2 = 0.f;
    if (hit >= 0) {
      const V3 F = v3(in.pl.y, in.pl.z, in.pl.w);
      lp0 = in.pl.x;
      lp1 = dot(F, t1);
      lp2 = dot(F, t2);
    }
    float l0 = 0.f, l1 = 0.f, l2 = 0.f;
    const bool need_feat = kLearned || (P.export_on && P.x_feat);
    if (need_feat) {
      float feat[16];
      feat[0] = u0;
      feat[1] = dot(t1, vr);
      feat[2] = dot(t2, vr);
      feat[3] = -phi;
      feat[4] = A.im;
      feat[5] = B.im;
      V3 can = cross(c.ra, n);
      feat[6] = dot(can, Imul(A.I, can));
      V3 cbn = cross(c.rb, n);
      feat[7] = b >= 0 ? dot(cbn, Imul(B.I, cbn)) : 0.f;
      // previous impulses in units of |g| dt / k_n (1 m/s^2 when gravity is off)
      const float unit = (gmag > 0.f ? gmag : 1.f) * dt / k3[0];
      feat[8] = lp0 / unit; feat[9] = lp1 / unit; feat[10] = lp2 / unit;
      feat[11] = n.x; feat[12] = n.y; feat[13] = n.z;
      feat[14] = mu;
      // new contact: its share 1 / max(n_a, n_b) of the busier body's
      // contacts; a persisting contact: 0
      {
        const int na = A.im > 0.f ? (int)deg[a] : 0;
        const int nbc = (b >= 0 && B.im > 0.f) ? (int)deg[b] : 0;
        const int mx = na > nbc ? na : nbc;
        feat[15] = hit >= 0 ? 0.f : 1.f / (float)(mx > 1 ? mx : 1);
      }
      if (live && P.export_on && P.x_feat)
        for (int k = 0; k < 16; k++) P.x_feat[k * P.scene_cm + (long)s * CM + q] = feat[k];
      if constexpr (kLearned) {
        float y[3];
        mlp_wave(P.mlp, feat, live, y);
        // a persisting contact keeps its previous impulse; the network
        // predicts a new contact's, in units of |g| dt / k_n
        float sc = gmag * dt / k3[0];
        if (hit >= 0) {
          l0 = lp0; l1 = lp1; l2 = lp2;
        } else {
          l0 = y[0] * sc; l1 = y[1] * sc; l2 = y[2] * sc;
        }
      }
    }
    if (P.warm == WARM_PREV || i >= nact) {  // classic warm start, or a sleeping contact
      l0 = lp0; l1 = lp1; l2 = lp2;
    }
    // projection of the initial impulse
    l0 = fmaxf(l0, 0.f);
    proj_disk(l1, l2, mu * l0);
    // Jacobi scale 1/max(n_a, n_b) from the per-body contact counts
    int na = A.im > 0.f ? (int)deg[a] : 0;
    int nbb = (b >= 0 && B.im > 0.f) ? (int)deg[b] : 0;
    float jsc = 1.0f / (float)(na > nbb ? na : nbb);
    if (live) {
      // normal-friction couplings: change of row d's velocity per unit normal impulse
      const float ims = imA + imB;
      const float k1n = dot(t1, n) * ims + dot(rw[1].ca, rw[0].ia) + dot(rw[1].cb, rw[0].ib) + kc[0];
      const float k2n = dot(t2, n) * ims + dot(rw[2].ca, rw[0].ia) + dot(rw[2].cb, rw[0].ib) + kc[1];
      const float m3[3] = {rw[0].m, rw[1].m, rw[2].m};
      // with the arm, the Jacobi scale's word holds the arm side (Jacobi is not used then)
      store_rec(rec, i, n, c.ra, c.rb, m3, k1n, k2n, bias - (dot(n, vf) + ua[0]), mu, key, arm2 ? asg : jsc,
                dot(t1, vf) + ua[1]);
      st4(S.f + L.lam, i, make_float4(l0, l1, l2, dot(t2, vf) + ua[2]));
      if (kLearned && hit < 0 && i < nact) atomicOr(S.u + L.fresh + (i >> 5), 1u << (i & 31));
    }
  }
  team_sync(tm);
  // the solve works on the dynamic bodies' velocity changes from here
  for (int i = tid; i < nb; i += T) {
    const float4 v = ld4(S.f + L.dyn, 3 * i), w = ld4(S.f + L.dyn, 3 * i + 1);
    if (v.w > 0.f) {
      st4(S.f + L.dyn, 3 * i, make_float4(0.f, 0.f, 0.f, v.w));
      st4(S.f + L.dyn, 3 * i + 1, make_float4(0.f, 0.f, 0.f, w.w));
    }
  }
  team_sync(tm);
  TRACE(10);

  // ---- a8/a11: warm start and sweeps ------------------------------------
  const ArmCtx armc{arm2, arm2 ? S.f + L.arm + ARM_DQ : nullptr,
                    arm2 ? P.arm_rows + (long)s * kMaxColours * kArmRowWords : nullptr, parts};
  // Learned start: persisting contacts' previous impulses are applied first,
  // then the network's impulses of the new contacts.  The plain solver
  // judges the network's part before any sweep: if it raises the solver's
  // objective it is dropped (the new contacts start from zero, the classic
  // warm start) and the step is flagged.
  if (kLearned) {
    apply_all(L, S, rec, ncol, cstart, tm, ArmCtx{false, nullptr, nullptr, false}, 0);
    team_sync(tm);
    for (int i = tid; i < nb; i += T) {
      st4(S.f + L.vsave, 2 * i, ld4(S.f + L.dyn, 3 * i));
      st4(S.f + L.vsave, 2 * i + 1, ld4(S.f + L.dyn, 3 * i + 1));
    }
    team_sync(tm);
    apply_all(L, S, rec, ncol, cstart, tm, ArmCtx{false, nullptr, nullptr, false}, 1);
    team_sync(tm);
    float* fval = S.f + L.fval;
    for (int i = tid; i < nact; i += T) fval[i] = start_objective(L, S, rec, i);
    team_sync(tm);
    // fixed-shape tree sum: same result for any block size
    int width = 1;
    while (width < nact) width <<= 1;
    for (int half = width >> 1; half > 0; half >>= 1) {
      for (int i = tid; i < half; i += T)
        if (i + half < nact) fval[i] += fval[i + half];
      team_sync(tm);
    }
    if (nact > 0 && fval[0] > 0.f) {  // uniform across the workgroup
      if (tid == 0) misc[M_FLAGS] |= FLAG_FELLBACK;
      for (int i = tid; i < nb; i += T) {
        st4(S.f + L.dyn, 3 * i, ld4(S.f + L.vsave, 2 * i));
        st4(S.f + L.dyn, 3 * i + 1, ld4(S.f + L.vsave, 2 * i + 1));
      }
      for (int i = tid; i < nact; i += T) {
        if (!((S.u[L.fresh + (i >> 5)] >> (i & 31)) & 1u)) continue;
        const float u2 = S.f[L.lam + 4 * i + 3];
        st4(S.f + L.lam, i, make_float4(0.f, 0.f, 0.f, u2));
      }
    }
    team_sync(tm);
  } else if (P.warm == WARM_PREV) {
    apply_all(L, S, rec, ncol, cstart, tm, armc);
  }
  if (arm2) {  // motor warm start after the contacts'
    if (tid < 64) arm_motor_warm(L, S, tid);
    team_sync(tm);
  }
  TRACE(11);
  int sweeps = 0;
  float res = 0.f;
  const uint64_t clk0 = P.trace ? clock64() : 0;
  if (P.solver == SOLVER_JACOBI)
    solve_jacobi(L, S, rec, nb, nact, ncol, cstart, P.iters, P.tol, misc, &sweeps, &res, tm);
  else
    solve_pgs<!kLearned>(L, S, rec, ncol, cstart, P.iters, P.tol, misc, &sweeps, &res, tm, armc, P.motor_max);
  team_sync(tm);
  // a step counts as solved only once its residual reached the tolerance
  if (P.tol > 0.f && res > P.tol && tid == 0) misc[M_FLAGS] |= FLAG_NOT_CONVERGED;
  team_sync(tm);
  TRACE(12);
  if (P.trace && tid == 0) P.trace[(long)s * kTraceSlots + 15] = clock64() - clk0;  // shader cycles in the solve

  // ---- a12: integrate positions, write state ----------------------------
  for (int i = tid; i < nb; i += T) {
    const long gi = b0 + i;
    uint32_t meta = body_meta(L, S, i);
    // asleep: pose kept, velocity zero, count kept (sleeping is not compiled
    // into the learned kernels)
    bool asleep = false;
    if constexpr (!kLearned) asleep = is_dyn_meta(meta) && !is_awake_meta(meta);
    if (asleep) {
      for (int k = 0; k < 6; k++) P.vel[k * N + gi] = 0.f;
    } else if (is_dyn_meta(meta)) {
      V3 x = xyz(ld4(S.f + L.geo, 3 * i));
      float4 qq = ld4(S.f + L.geo, 3 * i + 1);
      const float4 d0 = ld4(S.f + L.dyn, 3 * i);
      V3 v = xyz(d0), w = xyz(ld4(S.f + L.dyn, 3 * i + 1));
      float qw = qq.x, qx = qq.y, qy = qq.z, qz = qq.w;
      V3 vr, wr;  // the velocity that decides rest (at the step's pose)
      if (parts && d0.w < 0.f) {
        // a container part moves exactly along its joint: q += dt qd; a
        // hinge turns the body about its line by dt qd, a slide shifts it
        // by dt qd a; the velocity out is the rate's at the new pose
        const bool rev = d0.w == kRevoluteFlag;
        const V3 a = v3(P.joint_axis[gi], P.joint_axis[N + gi], P.joint_axis[2 * N + gi]);
        const V3 o = v3(P.joint_anchor[gi], P.joint_anchor[N + gi], P.joint_anchor[2 * N + gi]);
        const float qd = dot(a, rev ? w : v);
        const float dq = dt * qd;
        P.joint_state[gi] += dq;
        P.joint_state[N + gi] = qd;
        if (rev) {
          wr = a * qd;
          vr = cross(wr, x - o);
          float sn, cs, sh, ch;
          sincosf(dq, &sn, &cs);
          sincosf(0.5f * dq, &sh, &ch);
          const V3 r = x - o;
          x = o + (r * cs + cross(a, r) * sn + a * (dot(a, r) * (1.f - cs)));
          // (cos dq/2, a sin dq/2) (x) q
          const V3 hv = a * sh;
          const float nw = ch * qw - (hv.x * qx + hv.y * qy + hv.z * qz);
          const float nx = ch * qx + hv.x * qw + (hv.y * qz - hv.z * qy);
          const float ny = ch * qy + hv.y * qw + (hv.z * qx - hv.x * qz);
          const float nz = ch * qz + hv.z * qw + (hv.x * qy - hv.y * qx);
          const float inv = 1.0f / sqrtf(nw * nw + nx * nx + ny * ny + nz * nz);
          qw = nw * inv; qx = nx * inv; qy = ny * inv; qz = nz * inv;
          w = wr;
          v = cross(wr, x - o);
        } else {
          vr = a * qd;
          wr = v3(0.f, 0.f, 0.f);
          x = x + a * dq;
          v = vr;
          w = wr;
        }
      } else {
        // the solve left the velocity change since the setup in the slot
        v = setup_lin_vel(P, gi, N, g, dt) + v;
        w = v3(P.vel[3 * N + gi], P.vel[4 * N + gi], P.vel[5 * N + gi]) + w;
        vr = v;
        wr = w;
        x = x + v * dt;
        // q + dt/2 (0, w) (x) q
        float dw = -(w.x * qx + w.y * qy + w.z * qz);
        float dx = qw * w.x + (w.y * qz - w.z * qy);
        float dy = qw * w.y + (w.z * qx - w.x * qz);
        float dz = qw * w.z + (w.x * qy - w.y * qx);
        float h = 0.5f * dt;
        qw += h * dw; qx += h * dx; qy += h * dy; qz += h * dz;
        float inv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
        qw *= inv; qx *= inv; qy *= inv; qz *= inv;
      }
      P.pose[gi] = x.x; P.pose[N + gi] = x.y; P.pose[2 * N + gi] = x.z;
      P.pose[3 * N + gi] = qw; P.pose[4 * N + gi] = qx; P.pose[5 * N + gi] = qy; P.pose[6 * N + gi] = qz;
      P.vel[gi] = v.x; P.vel[N + gi] = v.y; P.vel[2 * N + gi] = v.z;
      P.vel[3 * N + gi] = w.x; P.vel[4 * N + gi] = w.y; P.vel[5 * N + gi] = w.z;
      if (!kLearned && P.sleep_speed > 0.f) {  // at rest: speed and surface speed |w| r at most sleep_speed
        const float4 g2 = ld4(S.f + L.geo, 3 * i + 2);
        const uint32_t sh = meta & 255u;
        const float rb = sh == SPHERE ? g2.x
                         : ((sh == BOX || sh == HULL) ? sqrtf(g2.x * g2.x + g2.y * g2.y + g2.z * g2.z) : g2.x + g2.y);
        const bool at_rest = sqrtf(len2(vr)) <= P.sleep_speed && sqrtf(len2(wr)) * rb <= P.sleep_speed;
        const int32_t r0 = P.rest[gi];
        P.rest[gi] = at_rest ? (r0 < (1 << 30) ? r0 + 1 : r0) : 0;
      }
      bool fin = isfinite(x.x) && isfinite(x.y) && isfinite(x.z) && isfinite(v.x) && isfinite(v.y) && isfinite(v.z) &&
                 isfinite(w.x) && isfinite(w.y) && isfinite(w.z);
      if (!fin) atomicOr(&misc[M_FLAGS], (uint32_t)FLAG_NONFINITE);
    }
  }
  team_sync(tm);  // every read of the arm links' LDS records is done
  if (P.arm && tid == 0) {
    float th[7], qd[7];
    if (arm2) {  // the angles advance by the joint rates; links follow, moving at those rates
      float* st = P.arm_state + 21 * s;
      const float* arm = S.f + L.arm;
#pragma unroll
      for (int k = 0; k < 7; k++) {
        qd[k] = arm[ARM_QREF + k] + arm[ARM_DQ + k];
        th[k] = P.theta[7 * s + k] + dt * qd[k];
        P.theta[7 * s + k] = th[k];
        st[k] = qd[k];
        st[14 + k] = arm[ARM_LAM + k];
        if (!isfinite(qd[k])) atomicOr(&misc[M_FLAGS], (uint32_t)FLAG_NONFINITE);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 7; k++) {
        th[k] = P.theta[7 * s + k] + dt * thd[k];
        P.theta[7 * s + k] = th[k];
        qd[k] = 0.f;
      }
    }
    // kinematic arm: link velocities stay those of this step; poses move to theta_{t+1}
    if (arm2) arm_fk(P, L, S, nb - 7, P.arm_base + 3 * s, th, qd);
    else arm_fk(P, L, S, nb - 7, P.arm_base + 3 * s, th, nullptr);
#pragma unroll
    for (int k = 0; k < 7; k++) {
      int i = nb - 7 + k;
      long gi = b0 + i;
      float4 x = ld4(S.f + L.geo, 3 * i), qq = ld4(S.f + L.geo, 3 * i + 1);
      float4 v = ld4(S.f + L.dyn, 3 * i), w = ld4(S.f + L.dyn, 3 * i + 1);
      P.pose[gi] = x.x; P.pose[N + gi] = x.y; P.pose[2 * N + gi] = x.z;
      P.pose[3 * N + gi] = qq.x; P.pose[4 * N + gi] = qq.y; P.pose[5 * N + gi] = qq.z; P.pose[6 * N + gi] = qq.w;
      P.vel[gi] = v.x; P.vel[N + gi] = v.y; P.vel[2 * N + gi] = v.z;
      P.vel[3 * N + gi] = w.x; P.vel[4 * N + gi] = w.y; P.vel[5 * N + gi] = w.z;
    }
  }
  TRACE(13);

  // ---- a13: cache, export, arm force, stats ------------------------------
  const int arml = P.arm ? nb - 7 : nb;
  float* force = S.f + L.force;
  for (int i = tid; i < nc; i += T) {
    const int q = (int)perm[i];
    const float4* R = rec + kRec * i;
    float4 lam = ld4(S.f + L.lam, i);
    const V3 n = xyz(R[0]);
    V3 t1, t2;
    tangents_coef(n, R[4].z, t1, t2);
    uint32_t key = ckeys[q];
    int a = (int)(key >> 20), b = (int)((key >> 8) & 0xFFFu);
    V3 F = t1 * lam.y + t2 * lam.z;
    long o = (long)s * CM + q;
    P.cur_key[o] = key;
    P.cur_col[o] = (uint8_t)colour[q];
    P.cur_lam[o] = lam.x;
    P.cur_lam[P.scene_cm + o] = F.x;
    P.cur_lam[2 * P.scene_cm + o] = F.y;
    P.cur_lam[3 * P.scene_cm + o] = F.z;
    bool arm_c = a >= arml || (b != (int)kGroundKey && b >= arml);
    force[q] = arm_c ? sqrtf(len2(n * lam.x + F)) / dt : 0.f;
    if (P.export_on) {
      const long sc = P.scene_cm;
      V3 pt = xyz(raw[2 * q + 1]);
      P.x_normal[o] = n.x; P.x_normal[sc + o] = n.y; P.x_normal[2 * sc + o] = n.z;
      P.x_point[o] = pt.x; P.x_point[sc + o] = pt.y; P.x_point[2 * sc + o] = pt.z;
      P.x_phi[o] = raw[2 * q].w;
      P.x_lambda[o] = lam.x; P.x_lambda[sc + o] = lam.y; P.x_lambda[2 * sc + o] = lam.z;
      P.x_colour[o] = colour[q] == kSleepColour ? -1 : (int32_t)colour[q];
    }
  }
  team_sync(tm);
  // fixed-shape tree sum over the contact slots: same result for any block size
  int width = 1;
  while (width < nc) width <<= 1;
  for (int half = width >> 1; half > 0; half >>= 1) {
    for (int i = tid; i < half; i += T)
      if (i + half < nc) force[i] += force[i + half];
    team_sync(tm);
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
  TRACE(14);
}

template <bool kLearned, int kExt>
__global__ __launch_bounds__(256) void step_kernel(StepParams P, LdsLayout L) {
  extern __shared__ float4 smem_f4[];
  Smem S{reinterpret_cast<float*>(smem_f4), reinterpret_cast<uint32_t*>(smem_f4)};
  const Team<false> tm{(int)threadIdx.x, (int)blockDim.x};
  const int s = P.scene_list ? P.scene_list[blockIdx.x] : (int)blockIdx.x;
  scene_step<kLearned, kExt>(P, L, S, s, tm);
}

// Scenes whose working set exceeds a workgroup's LDS: the same step with the
// working set in global memory (one region of P.gwords words per scene of
// P.glist, L2 and HBM resident) instead of LDS; one workgroup per scene.
// The team barriers are workgroup-scope fences, which order global memory
// as they order LDS, so the step computes exactly what it computes in LDS.
template <bool kLearned, int kExt>
__global__ __launch_bounds__(256) void step_kernel_hbm(StepParams P, LdsLayout L) {
  const int k = (int)blockIdx.x;
  float* ws = P.gscr + (size_t)k * (size_t)P.gwords;
  const Team<false> tm{(int)threadIdx.x, (int)blockDim.x};
  scene_step<kLearned, kExt>(P, L, Smem{ws, reinterpret_cast<uint32_t*>(ws)}, P.glist[k], tm);
}

// Persistent launch over scenes of uneven size: every workgroup first takes
// scenes from the `team` queue and steps each with all its threads and all
// its LDS, then each of its waves takes scenes from the `wave` queue and
// steps each alone in its quarter of the LDS.  Queues are in descending
// body count, so the largest scenes start first; a workgroup leaves once
// both queues are drained.
template <bool kLearned, int kExt>
__global__ __launch_bounds__(256) void step_persistent(StepParams P, QueueParams Q) {
  extern __shared__ float4 smem_f4[];
  __shared__ int next_scene;
  float* lds = reinterpret_cast<float*>(smem_f4);
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) next_scene = (int)atomicAdd(&Q.head[0], 1u);
    __syncthreads();
    const int k = next_scene;
    __syncthreads();
    if (k >= Q.n_team) break;
    const int s = Q.team[k];
    const int nb = P.body_offset[s + 1] - P.body_offset[s];
    const LdsLayout L = lds_layout(nb, scene_cap(nb, P.PM), scene_cap(nb, P.CM), (int)blockDim.x >> 6, P.solver,
                                   P.warm, P.art);
    scene_step<kLearned, kExt>(P, L, Smem{lds, reinterpret_cast<uint32_t*>(lds)}, s, Team<false>{tid, (int)blockDim.x});
    __syncthreads();
  }
  const int w = tid >> 6, lane = tid & 63;
  float* mine = lds + w * (Q.lds_words / ((int)blockDim.x >> 6));
  for (;;) {
    int k = 0;
    if (lane == 0) k = (int)atomicAdd(&Q.head[1], 1u);
    k = __shfl(k, 0);
    if (k >= Q.n_wave) break;
    const int s = Q.wave[k];
    const int nb = P.body_offset[s + 1] - P.body_offset[s];
    const LdsLayout L = lds_layout(nb, scene_cap(nb, P.PM), scene_cap(nb, P.CM), 1, P.solver, P.warm, P.art);
    scene_step<kLearned, kExt>(P, L, Smem{mine, reinterpret_cast<uint32_t*>(mine)}, s, Team<true>{lane, 64});
  }
}

__global__ void queue_reset_kernel(uint32_t* head) {
  if (threadIdx.x < 2) head[threadIdx.x] = 0u;
}

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

// Masked reset from a pool of K states: one workgroup per flagged scene
// copies pool entry index[s] (pose [K][7][N], velocity [K][6][N], joint
// angles [K][S][7], container parts' q and qd [K][2][N]) into the scene and
// empties its contact cache; the articulated arm's state (arm_state, may be
// null) restarts at rest with its motor targets at the new angles; an entry
// outside [0, K) leaves the scene as it is and flags it.
__global__ void reset_kernel(const int32_t* off, const uint8_t* mask, float* pose, float* vel, int32_t* rest, long N,
                             int S_, int K, const int32_t* index, const float* pool_pose, const float* pool_vel,
                             float* theta, const float* pool_theta, float* joint_state, const float* pool_joint,
                             int32_t* cache_count_a, int32_t* cache_count_b, int32_t* flags, float* arm_state) {
  const int s = blockIdx.x;
  if (!mask[s]) return;
  const int k = index ? index[s] : 0;
  if (k < 0 || k >= K) {
    if (threadIdx.x == 0) flags[s] |= FLAG_BAD_RESET;
    return;
  }
  const float* pp = pool_pose + (size_t)k * 7 * N;
  const float* pv = pool_vel + (size_t)k * 6 * N;
  const int b0 = off[s], b1 = off[s + 1];
  for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
    for (int c = 0; c < 7; c++) pose[c * N + i] = pp[c * N + i];
    for (int c = 0; c < 6; c++) vel[c * N + i] = pv[c * N + i];
    rest[i] = 0;
    if (joint_state && pool_joint)
      for (int c = 0; c < 2; c++) joint_state[c * N + i] = pool_joint[(size_t)k * 2 * N + c * N + i];
  }
  if (threadIdx.x < 7 && theta && pool_theta) {
    const float th = pool_theta[(size_t)k * 7 * S_ + 7 * s + threadIdx.x];
    theta[7 * s + threadIdx.x] = th;
    if (arm_state) {
      arm_state[21 * s + threadIdx.x] = 0.f;
      arm_state[21 * s + 7 + threadIdx.x] = th;
      arm_state[21 * s + 14 + threadIdx.x] = 0.f;
    }
  }
  if (threadIdx.x == 0) {
    cache_count_a[s] = 0;
    cache_count_b[s] = 0;
  }
}

}  // namespace rbs

extern "C" int rbs_launch_step(const rbs::StepParams* P, const rbs::LdsLayout* L, int threads, int grid,
                               hipStream_t stream) {
  size_t bytes = (size_t)L->total * 4u;
  if (P->warm == rbs::WARM_LEARNED)
    hipLaunchKernelGGL((rbs::step_kernel<true, 0>), dim3(grid), dim3(threads), bytes, stream, *P, *L);
  else if (P->hull_info)
    hipLaunchKernelGGL((rbs::step_kernel<false, 3>), dim3(grid), dim3(threads), bytes, stream, *P, *L);
  else if (P->joint)
    hipLaunchKernelGGL((rbs::step_kernel<false, 2>), dim3(grid), dim3(threads), bytes, stream, *P, *L);
  else if (P->arm == 2)
    hipLaunchKernelGGL((rbs::step_kernel<false, 1>), dim3(grid), dim3(threads), bytes, stream, *P, *L);
  else
    hipLaunchKernelGGL((rbs::step_kernel<false, 0>), dim3(grid), dim3(threads), bytes, stream, *P, *L);
  return (int)hipGetLastError();
}

extern "C" int rbs_launch_step_hbm(const rbs::StepParams* P, const rbs::LdsLayout* L, int n, hipStream_t stream) {
  if (n <= 0) return 0;
  if (P->warm == rbs::WARM_LEARNED)
    hipLaunchKernelGGL((rbs::step_kernel_hbm<true, 0>), dim3(n), dim3(256), 0, stream, *P, *L);
  else if (P->hull_info)
    hipLaunchKernelGGL((rbs::step_kernel_hbm<false, 3>), dim3(n), dim3(256), 0, stream, *P, *L);
  else if (P->joint)
    hipLaunchKernelGGL((rbs::step_kernel_hbm<false, 2>), dim3(n), dim3(256), 0, stream, *P, *L);
  else if (P->arm == 2)
    hipLaunchKernelGGL((rbs::step_kernel_hbm<false, 1>), dim3(n), dim3(256), 0, stream, *P, *L);
  else
    hipLaunchKernelGGL((rbs::step_kernel_hbm<false, 0>), dim3(n), dim3(256), 0, stream, *P, *L);
  return (int)hipGetLastError();
}

// Dynamic LDS limits: the whole budget for the per-scene kernels; the
// persistent kernel keeps 256 bytes for its static words.
extern "C" int rbs_set_step_lds_limit(int bytes) {
  const void* k[10] = {(const void*)rbs::step_kernel<false, 0>,     (const void*)rbs::step_kernel<true, 0>,
                       (const void*)rbs::step_kernel<false, 1>,     (const void*)rbs::step_kernel<false, 2>,
                       (const void*)rbs::step_kernel<false, 3>,     (const void*)rbs::step_persistent<false, 0>,
                       (const void*)rbs::step_persistent<true, 0>,  (const void*)rbs::step_persistent<false, 1>,
                       (const void*)rbs::step_persistent<false, 2>, (const void*)rbs::step_persistent<false, 3>};
  for (int i = 0; i < 10; i++) {
    int e = (int)hipFuncSetAttribute(k[i], hipFuncAttributeMaxDynamicSharedMemorySize, i < 5 ? bytes : bytes - 256);
    if (e) {
      (void)hipGetLastError();  // leave no sticky error behind
      return e;
    }
  }
  return 0;
}

// Queue heads reset, then the persistent step; grid = workgroups resident at once.
extern "C" int rbs_launch_persistent(const rbs::StepParams* P, const rbs::QueueParams* Q, int grid,
                                     hipStream_t stream) {
  hipLaunchKernelGGL(rbs::queue_reset_kernel, dim3(1), dim3(64), 0, stream, Q->head);
  const size_t bytes = (size_t)Q->lds_words * 4u;
  if (P->warm == rbs::WARM_LEARNED)
    hipLaunchKernelGGL((rbs::step_persistent<true, 0>), dim3(grid), dim3(256), bytes, stream, *P, *Q);
  else if (P->hull_info)
    hipLaunchKernelGGL((rbs::step_persistent<false, 3>), dim3(grid), dim3(256), bytes, stream, *P, *Q);
  else if (P->joint)
    hipLaunchKernelGGL((rbs::step_persistent<false, 2>), dim3(grid), dim3(256), bytes, stream, *P, *Q);
  else if (P->arm == 2)
    hipLaunchKernelGGL((rbs::step_persistent<false, 1>), dim3(grid), dim3(256), bytes, stream, *P, *Q);
  else
    hipLaunchKernelGGL((rbs::step_persistent<false, 0>), dim3(grid), dim3(256), bytes, stream, *P, *Q);
  return (int)hipGetLastError();
}

extern "C" int rbs_launch_arm_pose(const rbs::StepParams* P, const uint8_t* mask, hipStream_t stream) {
  int S_ = P->num_scenes;
  hipLaunchKernelGGL(rbs::arm_pose_kernel, dim3((S_ + 63) / 64), dim3(64), 0, stream, S_, P->body_offset, P->pose,
                     P->n_bodies, P->theta, P->arm_base, *P, mask);
  return (int)hipGetLastError();
}

extern "C" int rbs_launch_reset(const rbs::StepParams* P, const uint8_t* mask, int K, const int32_t* index,
                                const float* pool_pose, const float* pool_vel, const float* pool_theta,
                                const float* pool_joint, int32_t* count_a, int32_t* count_b, hipStream_t stream) {
  hipLaunchKernelGGL(rbs::reset_kernel, dim3(P->num_scenes), dim3(128), 0, stream, P->body_offset, mask, P->pose,
                     P->vel, P->rest, P->n_bodies, P->num_scenes, K, index, pool_pose, pool_vel, P->theta, pool_theta,
                     P->joint_state, pool_joint, count_a, count_b, P->st_flags,
                     P->arm == 2 ? P->arm_state : nullptr);
  return (int)hipGetLastError();
}

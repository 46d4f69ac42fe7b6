// query.hip -- batched collision checks of arm configurations against the
// scenes as they stand: the test a sampling motion planner makes at every
// configuration it visits (Sec. 4.5 and App. C: the planner checks the arm
// against the scene at fine joint-space steps), for M candidate
// configurations per scene at once, without the solver.
//
// For configuration j of scene s the arm links are placed by the forward
// kinematics of theta[s][j][7]; a configuration collides iff some link (a
// capsule) has a contact with phi <= clearance against a body of the scene
// that is not an arm link, or against the ground plane.  The arm itself is
// left out: its neighbouring links overlap at the joints by construction.
//
// One workgroup of four waves per (scene, block of 64 configurations):
//  - the scene's obstacle boxes (AABBs, no margin) go to LDS once;
//  - each wave takes 16 configurations in turn: all lanes run the chain's
//    forward kinematics (uniform), lanes 0..6 publish their link's capsule
//    and its box widened by the clearance, and test the ground;
//  - each lane tests 64-obstacle chunks against the 7 link boxes; the
//    (link, obstacle) candidates are compacted by wave ballots into an LDS
//    queue in (obstacle chunk, link, lane) order and the wave runs the
//    contact routines on the queue one entry per lane;
//  - the least separation is reduced over the wave; lane 0 writes the flag.
// The box test only prunes: a link box widened by the clearance and a small
// pad meets every obstacle box that the contact test could keep, so the flag
// is decided by the contact routines alone.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "arm.h"
#include "geom.h"
#include "hull.h"

namespace rbs {

struct QueryParams {
  long n_bodies;             // plane stride of the body arrays
  const int32_t* body_offset;
  const uint8_t* shape;
  const float* prm;          // [3][N]
  const float* pose;         // [7][N]
  const float* arm_base;     // [S][3]
  float link_len[7];
  const float* theta;        // [S][M][7]
  int M;
  int cfg_blocks;            // workgroups per scene
  int max_obstacles;         // LDS box slots (largest scene less its 7 links)
  float clearance;
  uint8_t* hit;              // [S][M]
  float* min_phi;            // [S][M] or null
  HullLib hl;                // convex hulls (hl.info null: none)
  const float4* hull_ext;    // [H] their local bounding-box half-extents
};

constexpr int kQueryWaves = 4;
constexpr int kQueryCfgPerWave = 16;
constexpr int kQueryCfgPerBlock = kQueryWaves * kQueryCfgPerWave;
constexpr int kQueryQueue = 7 * 64;   // candidates of one 64-obstacle chunk
constexpr int kLinkWords = 16;        // c xyz, q wxyz, r, half length, box lo xyz... hi in the next slots
constexpr float kQueryPad = 1e-5f;    // m: box test never prunes a pair the contact test keeps

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ Geom body_geom(const QueryParams& Q, long g) {
  const long N = Q.n_bodies;
  Geom G;
  G.shape = Q.shape[g];
  G.x = v3(Q.pose[g], Q.pose[N + g], Q.pose[2 * N + g]);
  G.R = quat_R(Q.pose[3 * N + g], Q.pose[4 * N + g], Q.pose[5 * N + g], Q.pose[6 * N + g]);
  G.p[0] = Q.prm[g];
  G.p[1] = Q.prm[N + g];
  G.p[2] = Q.prm[2 * N + g];
  G.hull = -1;
  if (G.shape == HULL) {  // a hull: its index in the library, its bounding box's half-extents
    G.hull = (int)G.p[0];
    const float4 e = Q.hull_ext[G.hull];
    G.p[0] = e.x;
    G.p[1] = e.y;
    G.p[2] = e.z;
  }
  return G;
}

// Axis-aligned box of a shape widened by w.
__device__ __forceinline__ void shape_box(const Geom& G, float w, V3& lo, V3& hi) {
  V3 e;
  V3 c = G.x;
  if (G.shape == BOX || G.shape == HULL) {  // a hull: its bounding box
    e.x = fabsf(G.R.m[0][0]) * G.p[0] + fabsf(G.R.m[0][1]) * G.p[1] + fabsf(G.R.m[0][2]) * G.p[2];
    e.y = fabsf(G.R.m[1][0]) * G.p[0] + fabsf(G.R.m[1][1]) * G.p[1] + fabsf(G.R.m[1][2]) * G.p[2];
    e.z = fabsf(G.R.m[2][0]) * G.p[0] + fabsf(G.R.m[2][1]) * G.p[1] + fabsf(G.R.m[2][2]) * G.p[2];
  } else if (G.shape == CAPSULE) {
    V3 ax = col(G.R, 2) * G.p[1];
    e = v3(fabsf(ax.x) + G.p[0], fabsf(ax.y) + G.p[0], fabsf(ax.z) + G.p[0]);
  } else {
    e = v3(G.p[0], G.p[0], G.p[0]);
  }
  e = e + v3(w, w, w);
  lo = c - e;
  hi = c + e;
}

extern __shared__ float q_lds[];

__global__ __launch_bounds__(256) void query_kernel(QueryParams Q) {
  const int s = (int)(blockIdx.x / (unsigned)Q.cfg_blocks);
  const int cb = (int)(blockIdx.x % (unsigned)Q.cfg_blocks);
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long b0 = Q.body_offset[s];
  const int nb = Q.body_offset[s + 1] - (int)b0;
  const int nobs = nb - 7;
  const int MO = Q.max_obstacles;
  float* box = q_lds;                                                      // [6][MO]
  uint32_t* queue = reinterpret_cast<uint32_t*>(q_lds + 6 * MO) + wave * kQueryQueue;
  float* lk = q_lds + 6 * MO + kQueryWaves * kQueryQueue + wave * 7 * kLinkWords;

  for (int i = tid; i < nobs; i += (int)blockDim.x) {
    V3 lo, hi;
    shape_box(body_geom(Q, b0 + i), 0.f, lo, hi);
    box[i] = lo.x; box[MO + i] = lo.y; box[2 * MO + i] = lo.z;
    box[3 * MO + i] = hi.x; box[4 * MO + i] = hi.y; box[5 * MO + i] = hi.z;
  }
  __syncthreads();

  const float clear = Q.clearance;
  const long lb = b0 + nobs;  // first arm link
  for (int u = 0; u < kQueryCfgPerWave; u++) {
    const int j = cb * kQueryCfgPerBlock + wave * kQueryCfgPerWave + u;
    if (j >= Q.M) break;  // uniform over the wave
    const size_t qi = (size_t)s * (size_t)Q.M + (size_t)j;
    float th[7];
#pragma unroll
    for (int k = 0; k < 7; k++) th[k] = Q.theta[qi * 7 + k];
    V3 c[7], o[7], ax[7];
    float q[7][4];
    arm_chain(Q.arm_base + 3 * s, th, Q.link_len, c, q, o, ax);
    float best = __builtin_inff();
#pragma unroll
    for (int k = 0; k < 7; k++) {
      if (lane == k) {
        Geom Lg;
        Lg.shape = CAPSULE;
        Lg.x = c[k];
        Lg.R = quat_R(q[k][0], q[k][1], q[k][2], q[k][3]);
        Lg.p[0] = Q.prm[lb + k];
        Lg.p[1] = Q.prm[Q.n_bodies + lb + k];
        Lg.p[2] = 0.f;
        V3 lo, hi;
        shape_box(Lg, clear + kQueryPad, lo, hi);
        float* w = lk + k * kLinkWords;
        w[0] = c[k].x; w[1] = c[k].y; w[2] = c[k].z;
        w[3] = q[k][0]; w[4] = q[k][1]; w[5] = q[k][2]; w[6] = q[k][3];
        w[7] = Lg.p[0]; w[8] = Lg.p[1];
        w[9] = lo.x; w[10] = lo.y; w[11] = lo.z; w[12] = hi.x; w[13] = hi.y; w[14] = hi.z;
        Out4 out;
        out.n = 0;
        ground_contacts(Lg, clear, out);
        for (int t = 0; t < out.n; t++) best = fminf(best, out.get(t).phi);
      }
    }
    wave_sync();
    // link boxes, uniform over the wave
    float blo[7][3], bhi[7][3];
#pragma unroll
    for (int k = 0; k < 7; k++) {
#pragma unroll
      for (int a = 0; a < 3; a++) {
        blo[k][a] = lk[k * kLinkWords + 9 + a];
        bhi[k][a] = lk[k * kLinkWords + 12 + a];
      }
    }
    for (int base = 0; base < nobs; base += 64) {
      const int i = base + lane;
      float ol[3], oh[3];
      const bool in = i < nobs;
#pragma unroll
      for (int a = 0; a < 3; a++) {
        ol[a] = in ? box[a * MO + i] : 1.f;
        oh[a] = in ? box[(3 + a) * MO + i] : -1.f;  // an empty box meets nothing
      }
      uint32_t total = 0;
#pragma unroll
      for (int k = 0; k < 7; k++) {
        const bool meet = ol[0] <= bhi[k][0] && blo[k][0] <= oh[0] && ol[1] <= bhi[k][1] && blo[k][1] <= oh[1] &&
                          ol[2] <= bhi[k][2] && blo[k][2] <= oh[2];
        const uint64_t m = __ballot(meet);
        const uint32_t before = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (meet) queue[total + before] = ((uint32_t)k << 16) | (uint32_t)i;
        total += (uint32_t)__popcll(m);
      }
      wave_sync();
      for (uint32_t e = lane; e < total; e += 64) {
        const uint32_t ent = queue[e];
        const int k = (int)(ent >> 16), oi = (int)(ent & 0xFFFFu);
        const float* w = lk + k * kLinkWords;
        Geom Lg;
        Lg.shape = CAPSULE;
        Lg.x = v3(w[0], w[1], w[2]);
        Lg.R = quat_R(w[3], w[4], w[5], w[6]);
        Lg.p[0] = w[7];
        Lg.p[1] = w[8];
        Lg.p[2] = 0.f;
        Lg.hull = -1;
        const Geom Og = body_geom(Q, b0 + oi);
        Out4 out;
        out.n = 0;
        if (Og.shape == HULL) collide_hull(Lg, Og, Q.hl, clear, out);
        else collide(Lg, Og, clear, out);
        for (int t = 0; t < out.n; t++) best = fminf(best, out.get(t).phi);
      }
      wave_sync();  // the queue is rewritten by the next chunk
    }
    best = wave_min(best);
    if (lane == 0) {
      Q.hit[qi] = best <= clear ? 1 : 0;
      if (Q.min_phi) Q.min_phi[qi] = best;
    }
    wave_sync();  // the link slots are rewritten by the next configuration
  }
}

}  // namespace rbs

using namespace rbs;

extern "C" size_t rbs_query_lds_bytes(int max_obstacles) {
  return sizeof(float) * ((size_t)6 * (size_t)max_obstacles + (size_t)kQueryWaves * kQueryQueue +
                          (size_t)kQueryWaves * 7 * kLinkWords);
}

// n_scenes scenes, the largest with max_bodies bodies (its last 7 the arm).
extern "C" int rbs_launch_query(int n_scenes, int max_bodies, long n_bodies, const int32_t* body_offset,
                                const uint8_t* shape, const float* prm, const float* pose, const float* arm_base,
                                const float* link_len, const float* theta, int M, float clearance, uint8_t* hit,
                                float* min_phi, const int32_t* hull_info, const float4* hull_vert,
                                const float4* hull_plane, const uint8_t* hull_loop, const uint8_t* hull_edge,
                                const float4* hull_ext, hipStream_t stream) {
  if (M <= 0 || n_scenes <= 0) return 0;
  QueryParams Q;
  Q.n_bodies = n_bodies;
  Q.body_offset = body_offset;
  Q.shape = shape;
  Q.prm = prm;
  Q.pose = pose;
  Q.arm_base = arm_base;
  for (int k = 0; k < 7; k++) Q.link_len[k] = link_len[k];
  Q.theta = theta;
  Q.M = M;
  Q.cfg_blocks = (M + kQueryCfgPerBlock - 1) / kQueryCfgPerBlock;
  Q.max_obstacles = max_bodies - 7 > 1 ? max_bodies - 7 : 1;
  Q.clearance = clearance;
  Q.hit = hit;
  Q.min_phi = min_phi;
  Q.hl = HullLib{hull_info, hull_vert, hull_plane, hull_loop, hull_edge};
  Q.hull_ext = hull_ext;
  const size_t grid = (size_t)n_scenes * (size_t)Q.cfg_blocks;
  if (grid > 0x7FFFFFFFu) return -2;
  const size_t lds = rbs_query_lds_bytes(Q.max_obstacles);
  hipLaunchKernelGGL(query_kernel, dim3((unsigned)grid), dim3(kQueryWaves * 64), lds, stream, Q);
  return (int)hipGetLastError();
}

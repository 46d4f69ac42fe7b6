// sim_internal.h -- parameters and LDS layout shared by the host API and the
// step kernel of the HIP library.  Internal; not part of the C ABI.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace rbs {

constexpr int kMaxThreads = 256;
constexpr int kMaxColours = 128;
constexpr int kMaxBodiesPerScene = 1024;
constexpr uint32_t kGroundPair = 0xFFFFu;
constexpr uint32_t kGroundKey = 0xFFFu;

enum { WARM_COLD = 0, WARM_PREV = 1, WARM_LEARNED = 2 };
enum { SOLVER_PGS = 0, SOLVER_JACOBI = 1 };
enum { FLAG_NONFINITE = 1, FLAG_CAPACITY = 2, FLAG_NOT_CONVERGED = 4, FLAG_FELLBACK = 8 };

struct MlpParams {
  const uint16_t* w1;  // bf16 [64][16]  (out, in)
  const uint16_t* w2;  // bf16 [64][64]
  const uint16_t* w3;  // bf16 [3][64]
  const float* b1;     // [64]
  const float* b2;     // [64]
  const float* b3;     // [3]
  const float* mean;   // [16]
  const float* stdv;   // [16]
};

struct StepParams {
  int num_scenes;
  long n_bodies;            // plane stride of body arrays
  long scene_cm;            // plane stride of per-contact arrays (num_scenes * CM)
  long scene_pm;            // num_scenes * PM
  int NB, PM, CM;           // per-scene capacities (bodies, pairs, contacts)
  const int32_t* body_offset;
  const uint8_t* shape;
  const uint8_t* motion;
  const float* prm;         // [3][N]
  const float* inv_mass;    // [N]
  const float* inv_inertia; // [3][N] body-frame principal
  const float* friction;    // [N]
  const float* restitution; // [N]
  float* pose;              // [7][N]  x y z qw qx qy qz
  float* vel;               // [6][N]  vx vy vz wx wy wz
  int arm;
  float* theta;             // [S][7]
  const float* arm_base;    // [S][3]
  float link_len[7];
  float arm_radius;
  const float* actions;     // [S][7] or null
  const uint32_t* prev_key; // [S*CM]
  const float* prev_lam;    // [4][S*CM]
  const int32_t* prev_count;// [S]
  uint32_t* cur_key;
  float* cur_lam;
  int32_t* cur_count;
  int export_on;
  uint32_t* x_pair;         // [S*PM]
  float* x_normal;          // [3][S*CM]
  float* x_point;           // [3][S*CM]
  float* x_phi;             // [S*CM]
  float* x_lambda;          // [3][S*CM]
  int32_t* x_colour;        // [S*CM]
  float* x_feat;            // [16][S*CM] (export and learned only)
  int32_t* st_pairs;
  int32_t* st_contacts;
  int32_t* st_colours;
  int32_t* st_sweeps;
  int32_t* st_flags;
  float* st_residual;
  float* st_arm_force;
  float gx, gy, gz, dt, margin, baumgarte, slop, rest_thresh, ground_mu, ground_e;
  int iters;
  float tol;
  int warm;
  int solver;
  MlpParams mlp;
  const int32_t* scene_list;  // optional scene order (null: identity)
};

// LDS word offsets of one scene's working set.
struct LdsLayout {
  int bx, bq, bR, bv, bw, bim, bI, bprm, bmeta, bmu, be;
  int ckey, cab, cn, cp, cphi, cm, cbias, cmu, clam, ccol, cperm;
  int scr;
  int lo, hi, skey, sval, skey2, sval2, pk, pk2, hist, hbase;
  int prevk, deg, lstart, list, ck0, cv0, ck1, dl, vsave, snap, force;
  int misc;
  int total;  // words
};

constexpr int kMiscWords = 64;

inline __host__ __device__ LdsLayout lds_layout(int NB, int PM, int CM, int waves, int solver, int warm) {
  LdsLayout L;
  int o = 0;
  auto take = [&](int words) { int r = o; o += (words + 3) & ~3; return r; };
  L.bx = take(3 * NB);
  L.bq = take(4 * NB);
  L.bR = take(9 * NB);
  L.bv = take(3 * NB);
  L.bw = take(3 * NB);
  L.bim = take(NB);
  L.bI = take(6 * NB);
  L.bprm = take(3 * NB);
  L.bmeta = take(NB);
  L.bmu = take(NB);
  L.be = take(NB);
  L.ckey = take(CM);
  L.cab = take(CM);
  L.cn = take(3 * CM);
  L.cp = take(3 * CM);
  L.cphi = take(CM);
  L.cm = take(3 * CM);
  L.cbias = take(CM);
  L.cmu = take(CM);
  L.clam = take(3 * CM);
  L.ccol = take(CM);
  L.cperm = take(CM);
  L.misc = take(kMiscWords);
  L.hist = take(256 * waves);
  L.hbase = take(256);
  L.scr = o;
  // broadphase scratch
  int b = L.scr;
  auto tb = [&](int words) { int r = b; b += (words + 3) & ~3; return r; };
  L.lo = tb(3 * NB);
  L.hi = tb(3 * NB);
  L.skey = tb(NB);
  L.sval = tb(NB);
  L.skey2 = tb(NB);
  L.sval2 = tb(NB);
  L.pk = tb(PM);
  L.pk2 = tb(PM);
  int bend = b;
  // post-narrowphase scratch (reuses the broadphase region)
  int p = L.scr;
  auto tp = [&](int words) { int r = p; p += (words + 3) & ~3; return r; };
  L.prevk = tp(CM);
  L.deg = tp(NB + 1);
  L.lstart = tp(NB + 1);
  L.list = tp(2 * CM);
  L.ck0 = tp(CM);
  L.cv0 = tp(CM);
  L.ck1 = tp(CM);
  L.force = L.prevk;   // per-contact arm force, after the solve (prevk is dead)
  L.dl = (solver == SOLVER_JACOBI) ? tp(3 * CM) : -1;
  L.snap = (solver == SOLVER_JACOBI) ? tp(6 * NB) : -1;
  L.vsave = (warm == WARM_LEARNED) ? tp(6 * NB) : -1;
  int pend = p;
  L.total = (bend > pend ? bend : pend);
  return L;
}

}  // namespace rbs

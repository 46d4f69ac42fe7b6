// sim_internal.h -- parameters and LDS layout shared by the host API and the
// step kernel of the HIP library.  Internal; not part of the C ABI.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace rbs {

constexpr int kMaxThreads = 256;
constexpr int kMaxColours = 128;
constexpr int kMaxBodiesPerScene = 2046;  // local body index field: 11 bits, 2047 = ground
constexpr uint32_t kGroundPair = 0xFFFFu;
constexpr uint32_t kGroundKey = 0xFFFu;
constexpr int kTraceSlots = 16;
constexpr int kCapPerBody = 6;   // per-scene pair and contact capacity: kCapPerBody * bodies,
constexpr int kCapFloor = 64;    // at least kCapFloor, at most the batch-wide capacity

// Pair or contact capacity of a scene of nb bodies under batch capacity cap.
inline __host__ __device__ int scene_cap(int nb, int cap) {
  int c = kCapPerBody * nb;
  if (c < kCapFloor) c = kCapFloor;
  return c < cap ? c : cap;
}

enum { WARM_COLD = 0, WARM_PREV = 1, WARM_LEARNED = 2 };
enum { SOLVER_PGS = 0, SOLVER_JACOBI = 1 };
enum { FLAG_NONFINITE = 1, FLAG_CAPACITY = 2, FLAG_NOT_CONVERGED = 4, FLAG_FELLBACK = 8, FLAG_BAD_RESET = 16 };

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
  int32_t* rest;            // [N] steps each body has ended at rest
  float sleep_speed;        // sleeping islands when > 0 (m/s, speed and surface speed)
  int sleep_steps;          // steps at rest before an island may sleep
  int arm;                  // 0 none, 1 kinematic links, 2 articulated body driven by joint motors
  float* theta;             // [S][7] joint angles
  float* arm_state;         // arm 2: [S][21] joint rates, motor targets, motor impulses
  float* arm_rows;          // arm 2: [S][kMaxColours][kArmRowWords] joint-space rows of the arm's contacts
  float motor_kp;           // arm 2: motor position gain
  float motor_max;          // arm 2: largest motor impulse per step (N s)
  // articulated container parts (null: none): per body the joint kind (0
  // none, 1 revolute, 2 prismatic), unit axis and anchor (world), limits of
  // the coordinate, local index of the static base it is joined to (-1 none)
  const uint8_t* joint;     // [N]
  const float* joint_axis;  // [3][N]
  const float* joint_anchor;// [3][N]
  const float* joint_limits;// [2][N]
  const int32_t* joint_parent;  // [N]
  float* joint_state;       // [2][N] joint coordinate and its rate
  int art;                  // articulation code of the layouts: arm | (kArtParts when joint is set)
  // convex hulls (null hull_info: none): the hull library (HullLib's
  // arrays) and each hull's local bounding-box half-extents
  const int32_t* hull_info; // [H][8]
  const float4* hull_vert;  // [V]
  const float4* hull_plane; // [F]
  const uint8_t* hull_loop; // [F][8]
  const uint8_t* hull_edge; // [E][4]
  const float4* hull_ext;   // [H]
  const float* arm_base;    // [S][3]
  float link_len[7];
  float arm_radius;
  const float* actions;     // [S][7] or null
  const uint32_t* prev_key; // [S*CM]
  const float* prev_lam;    // [4][S*CM]
  const int32_t* prev_count;// [S]
  const uint8_t* prev_col;  // [S*CM] colours of the previous step's contacts (a hint only)
  uint8_t* cur_col;
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
  float* x_feat;            // [16][S*CM] (export only)
  float4* raw;              // [S*CM][2] narrowphase output, canonical order: (n, phi), (p, -)
  float4* crec;             // [S][rec_stride(PM, CM)] solver records, colour-major order
  float* gscr;              // working sets of the scenes stepped out of HBM: [n][gwords] words
  long gwords;
  const int32_t* glist;     // those scenes, largest first
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
  uint64_t* trace;            // optional [S][kTraceSlots] phase timestamps (null: off)
};

// Work queues of the persistent launch: scenes stepped by a whole workgroup
// (`team`) and scenes stepped by one wave each (`wave`), largest first, and
// the two queue heads (zeroed before every launch).
struct QueueParams {
  const int32_t* team;
  const int32_t* wave;
  int n_team, n_wave;
  uint32_t* head;        // [2]: team queue, wave queue
  int lds_words;         // dynamic LDS of a workgroup; a wave owns a quarter
};

// LDS word offsets of one scene's working set.  Records are float4-aligned:
//  geo  [NB][12]: (x, y, z, meta) (qw, qx, qy, qz) (p0, p1, p2, -)
//  dyn  [NB][12]: (vx, vy, vz, inv_mass) (wx, wy, wz, mu) (Ixx, Iyy, Izz, Ixy),
//       preceded by two body slots: index -1 the ground (zero velocity and
//       inverse mass, read by contacts with the ground), index -2 a sink for
//       the solver's writes of bodies that are not dynamic (never read).  The
//       48-byte stride spreads the solver's velocity gathers over all LDS banks
//  dyn2 [NB][4]: (Ixz, Iyz, e, -), preceded by the same two slots
//  ckey [CM]: contact keys, canonical order
//  lam  [CM][4]: (lambda_n, lambda_t1, lambda_t2, phi), colour-major order
//  perm [CM]: colour-major position -> canonical contact index
//  fresh [CM/32] (learned warm start only): bit i set when colour-major
//       contact i is new, i.e. started from the network
// The per-contact solver constants live in global memory (StepParams::crec).
// The scratch region is reused phase by phase: broadphase (pairs, AABBs,
// body sort); colouring (previous keys for the starting colours, colours,
// per-body lists); setup (previous-impulse slots); solver (saved
// velocities and start objective terms of a learned start, Jacobi snapshot
// and increments); outputs (arm force partial sums).  Until the setup
// writes it, lam holds each contact's previous-impulse slot.
struct LdsLayout {
  int geo, dyn, dyn2, ckey, lam, perm, fresh, misc, arm, parts, hist, hbase;
  int scr;
  int pk, pk2, lo, hi, skey, sval, skey2, sval2, nperm, ncnt;
  int colour, deg, lstart, list, rank, cv0, ck1;
  int vsave, fval, snap, dl, force;
  int total;  // words
};

constexpr int kMiscWords = 64;
// word slots of the misc region: counters, flags, per-wave partials (one
// word per wave of a 256-thread team from M_WAVE and from M_SCAN)
enum { M_NPAIRS = 0, M_NCONT = 1, M_FLAGS = 2, M_NCOL = 3, M_CHANGED = 5, M_NACT = 6, M_WAVE = 16, M_SCAN = 32 };
// colour of a contact whose dynamic bodies all sleep: sorted after every
// solved colour and never swept
constexpr uint32_t kSleepColour = 128;
// meta-word bit of a sleeping dynamic body (shape in bits 0-7, motion 8-15)
constexpr uint32_t kAsleepBit = 1u << 16;
static_assert(M_SCAN + kMaxThreads / 64 <= kMiscWords && M_WAVE + kMaxThreads / 64 <= M_SCAN, "misc slots");
constexpr int kDynWords = 12;  // words per body in the dyn region (three float4)

// Links of the articulated arm (arm 2): a motion code of the meta word only;
// they carry no velocity or mass of their own in LDS (the arm holds both).
constexpr int ARMLINK = 3;
// LDS words of the articulated arm (arm 2): M^-1 (row-major 7 x 7), the
// joint-rate changes of the solve, the joint rates at the setup, the motor
// impulses and targets, joint origins and axes (x y z each)
enum { ARM_MI = 0, ARM_DQ = 52, ARM_QREF = 60, ARM_LAM = 68, ARM_BIAS = 76, ARM_O = 84, ARM_AX = 105,
       kArmWords = 128 };
// global words per colour of the joint-space rows of the arm contact in that
// colour (g_n, g_t1, g_t2, then M^-1 g of each; 7 words apiece)
constexpr int kArmRowWords = 48;
// Articulated container parts in LDS (the limit rows): per part 16 words:
// body, kind (1 revolute, 2 prismatic), mass about the joint M, the two
// limit targets, the two limit impulses, 1 / M, axis x y z; at most
// kMaxParts parts per scene.  In the dyn region a part's inverse-mass word
// is a flag (-1 prismatic, -2 revolute), its inverse inertia the projector
// a a^T / M, and a revolute part's velocity is taken about its hinge point
// (linear part zero, w = qd a); dyn2's fourth word holds its part slot.
constexpr int kMaxParts = 16;
enum { PART_BODY = 0, PART_KIND = 1, PART_M = 2, PART_BIAS = 3, PART_LAM = 5, PART_IM = 7, PART_AX = 8,
       kPartStride = 16, kPartWords = 4 + kMaxParts * kPartStride };  // word 0 of the region: the part count
constexpr float kPrismaticFlag = -1.f, kRevoluteFlag = -2.f;
// articulation code of a batch for the layouts: the arm mode (0, 1, 2) plus
// kArtParts when it has container parts
constexpr int kArtParts = 8;
constexpr int kRec = 5;        // float4 per contact in the solver records

// float4 per scene of the solver-record buffer: the records of CM contacts,
// or, earlier in the step, the narrowphase's staging of up to 4 contacts
// (2 float4 each) for every one of PM pairs, whichever is larger.
inline __host__ __device__ long rec_stride(long PM, long CM) {
  return kRec * CM > 8 * PM ? kRec * CM : 8 * PM;
}

inline __host__ __device__ LdsLayout lds_layout(int NB, int PM, int CM, int waves, int solver, int warm, int arm) {
  LdsLayout L;
  int o = 0;
  auto take = [&](int words) { int r = o; o += (words + 3) & ~3; return r; };
  L.geo = take(12 * NB);
  take(2 * kDynWords);  // ground and sink slots
  L.dyn = take(kDynWords * NB);
  take(2 * 4);  // ground and sink slots of dyn2
  L.dyn2 = take(4 * NB);
  L.ckey = take(CM);
  L.lam = take(4 * CM);
  L.perm = take(CM);
  L.fresh = (warm == WARM_LEARNED) ? take((CM + 31) / 32) : -1;
  L.misc = take(kMiscWords);
  L.arm = (arm & 3) == 2 ? take(kArmWords) : -1;
  L.parts = (arm & kArtParts) ? take(kPartWords) : -1;
  L.hist = take(256 * waves);
  L.hbase = take(256);
  L.scr = o;
  int b = L.scr;
  auto tb = [&](int words) { int r = b; b += (words + 3) & ~3; return r; };
  L.pk = tb(PM);
  L.pk2 = tb(PM);
  L.lo = tb(4 * NB);
  L.hi = tb(4 * NB);
  L.skey = tb(NB);
  L.sval = tb(NB);
  L.skey2 = tb(NB);
  L.sval2 = tb(NB);
  int bend = b;
  // narrowphase (the AABBs and body sort are dead by then): class-sorted pair
  // order and contacts per pair (bytes), over the AABB region
  L.nperm = L.lo;
  L.ncnt = L.lo + ((PM + 3) & ~3);
  if (L.ncnt + (PM + 3) / 4 > bend) bend = L.ncnt + (((PM + 3) / 4 + 3) & ~3);
  int p = L.scr;
  auto tp = [&](int words) { int r = p; p += (words + 3) & ~3; return r; };
  L.colour = tp(CM);
  L.deg = tp(NB + 1);
  const int after_deg = p;
  L.lstart = tp(NB + 1);
  L.list = tp(2 * CM);
  L.rank = tp(CM);
  int cend = p;
  L.cv0 = L.list;       // colour sort after the colouring rounds
  L.ck1 = L.list + CM;
  int q = after_deg;    // solver and outputs: lists are dead, deg and colour live on
  auto tq = [&](int words) { int r = q; q += (words + 3) & ~3; return r; };
  L.vsave = (warm == WARM_LEARNED) ? tq(8 * NB) : -1;
  L.fval = (warm == WARM_LEARNED) ? tq(CM) : -1;
  L.snap = (solver == SOLVER_JACOBI) ? tq(8 * NB) : -1;
  L.dl = (solver == SOLVER_JACOBI) ? tq(4 * CM) : -1;
  L.force = after_deg;  // outputs run after the solve
  if (q < after_deg + CM) q = after_deg + ((CM + 3) & ~3);
  int m = bend;
  if (cend > m) m = cend;
  if (q > m) m = q;
  L.total = m;
  return L;
}

}  // namespace rbs

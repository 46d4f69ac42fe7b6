// api.hip -- host side of the C ABI declared in include/rbsim.h.
//
// Validates the batch descriptor, lays the whole simulation out in one
// caller-owned device workspace (structure-of-arrays planes, 256-byte
// aligned), uploads the initial state, and launches the step kernel with one
// workgroup per scene, largest scenes first.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/rbsim.h"
#include "sim_internal.h"

extern "C" int rbs_launch_step(const rbs::StepParams* P, const rbs::LdsLayout* L, int threads, int grid,
                               hipStream_t stream);
extern "C" int rbs_set_step_lds_limit(int bytes);
extern "C" int rbs_launch_step_hbm(const rbs::StepParams* P, const rbs::LdsLayout* L, int n, hipStream_t stream);
extern "C" int rbs_launch_persistent(const rbs::StepParams* P, const rbs::QueueParams* Q, int grid,
                                     hipStream_t stream);
extern "C" int rbs_mlp_forward(const rbs::MlpParams* M, const float* x, long n, float* y, hipStream_t st);
extern "C" size_t rbs_mlp_work_bytes(long n);
extern "C" int rbs_mlp_stats(const float* x, long n, float* mean, float* stdv, void* work, hipStream_t st);
extern "C" int rbs_mlp_grad(const float* prm, const float* mean, const float* stdv, const float* x, const float* t,
                            const int32_t* rows, long n, float* grad, float* loss, void* work, hipStream_t st);
extern "C" long rbs_mlp_grad_static_max_rows();
extern "C" int rbs_mlp_grad_static(const float* prm, const float* mean, const float* stdv, const float* x,
                                   const float* t, const int32_t* rows, long n, float* grad, float* loss,
                                   hipStream_t st);
extern "C" int rbs_mlp_adam(float* prm, float* m1, float* m2, const float* grad, int step, float lr, float clip,
                            float* gnorm, hipStream_t st);
extern "C" int rbs_mlp_export(const float* prm, uint16_t* wbf, float* bias, hipStream_t st);
extern "C" int rbs_gather(const int32_t* count, const int32_t* flags, int S, int CM, long scm, const float* feat,
                          const float* lam, float inv_gdt, float tclip, int64_t* offs, int32_t* cnt, float* x,
                          float* t, long cap, long long* total, hipStream_t st);
extern "C" int rbs_launch_query(int n_scenes, int max_bodies, long n_bodies, const int32_t* body_offset,
                                const uint8_t* shape, const float* prm, const float* pose, const float* arm_base,
                                const float* link_len, const float* theta, int M, float clearance, uint8_t* hit,
                                float* min_phi, const int32_t* hull_info, const float4* hull_vert,
                                const float4* hull_plane, const uint8_t* hull_loop, const uint8_t* hull_edge,
                                const float4* hull_ext, hipStream_t stream);
extern "C" int rbs_launch_arm_pose(const rbs::StepParams* P, const uint8_t* mask, hipStream_t stream);
extern "C" int rbs_launch_reset(const rbs::StepParams* P, const uint8_t* mask, int K, const int32_t* index,
                                const float* pool_pose, const float* pool_vel, const float* pool_theta,
                                const float* pool_joint, int32_t* count_a, int32_t* count_b, hipStream_t stream);

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

struct Layout {
  size_t off_body_offset, off_shape, off_motion, off_prm, off_inv_mass, off_inv_inertia, off_friction,
      off_restitution, off_pose, off_vel, off_rest, off_theta, off_arm_state, off_arm_base, off_scene_list;
  size_t off_arm_rows;
  size_t off_joint, off_joint_axis, off_joint_anchor, off_joint_limits, off_joint_parent, off_joint_state;
  size_t off_hull_info, off_hull_vert, off_hull_plane, off_hull_loop, off_hull_edge, off_hull_ext;
  size_t off_ckey[2], off_clam[2], off_ccount[2], off_ccol[2];
  size_t off_x_pair, off_x_npairs, off_x_normal, off_x_point, off_x_phi, off_x_lambda, off_x_colour, off_x_feat;
  size_t off_raw, off_crec;
  size_t off_st[7];
  size_t off_gather, off_gcount;
  size_t off_queue, off_head;
  size_t off_actions;
  size_t off_glist, off_gscr;
  size_t total;
};

size_t align256(size_t x) { return (x + 255u) & ~size_t(255u); }

// art: the arm mode plus rbs::kArtParts when the batch has container parts
// Sizes of the hull library's device tables (hulls, vertices, faces, edges).
struct HullSizes {
  long H = 0, V = 0, F = 0, E = 0;
};

Layout make_layout(long S, long N, long PM, long CM, long n_hbm, long hbm_words, int art, HullSizes hs = HullSizes()) {
  const int arm = art & 3;
  const bool parts = (art & rbs::kArtParts) != 0;
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  L.off_body_offset = take(4 * (S + 1));
  L.off_shape = take(N);
  L.off_motion = take(N);
  L.off_prm = take(4 * 3 * N);
  L.off_inv_mass = take(4 * N);
  L.off_inv_inertia = take(4 * 3 * N);
  L.off_friction = take(4 * N);
  L.off_restitution = take(4 * N);
  L.off_pose = take(4 * 7 * N);
  L.off_vel = take(4 * 6 * N);
  L.off_rest = take(4 * N);  // steps each body has ended at rest (sleeping)
  L.off_theta = take(4 * 7 * S);
  L.off_arm_state = take(arm == 2 ? 4 * 21 * S : 0);  // articulated arm: joint rates, motor targets, impulses
  L.off_arm_base = take(4 * 3 * S);
  // container parts: joint kinds, axes, anchors, limits, parents; q and qd
  L.off_joint = take(parts ? N : 0);
  L.off_joint_axis = take(parts ? 4 * 3 * N : 0);
  L.off_joint_anchor = take(parts ? 4 * 3 * N : 0);
  L.off_joint_limits = take(parts ? 4 * 2 * N : 0);
  L.off_joint_parent = take(parts ? 4 * N : 0);
  L.off_joint_state = take(parts ? 4 * 2 * N : 0);
  // convex hulls: per hull 8 ints and a float4; float4 vertices and planes;
  // 8-byte loops, 4-byte edges
  L.off_hull_info = take(4 * 8 * hs.H);
  L.off_hull_vert = take(16 * hs.V);
  L.off_hull_plane = take(16 * hs.F);
  L.off_hull_loop = take(8 * hs.F);
  L.off_hull_edge = take(4 * hs.E);
  L.off_hull_ext = take(16 * hs.H);
  L.off_scene_list = take(4 * S);
  for (int k = 0; k < 2; k++) {
    L.off_ckey[k] = take(4 * S * CM);
    L.off_clam[k] = take(4 * 4 * S * CM);
    L.off_ccount[k] = take(4 * S);
    L.off_ccol[k] = take(S * CM);  // colour hints: not state (any content gives the same step)
  }
  L.off_x_pair = take(4 * S * PM);
  L.off_x_npairs = 0;  // stats pairs array doubles as the pair count
  L.off_x_normal = take(4 * 3 * S * CM);
  L.off_x_point = take(4 * 3 * S * CM);
  L.off_x_phi = take(4 * S * CM);
  L.off_x_lambda = take(4 * 3 * S * CM);
  L.off_x_colour = take(4 * S * CM);
  L.off_x_feat = take(4 * 16 * S * CM);
  L.off_raw = take(4 * 8 * S * CM);
  L.off_crec = take(sizeof(float4) * rbs::rec_stride(PM, CM) * S);  // solver records, narrowphase staging
  // articulated arm: joint-space rows of the contact on the arm in each colour
  L.off_arm_rows = take(arm == 2 ? 4 * (size_t)rbs::kMaxColours * rbs::kArmRowWords * S : 0);
  for (int k = 0; k < 7; k++) L.off_st[k] = take(4 * S);
  L.off_gather = take(8 * S);  // per-scene row offsets and counts of sim_mlp_gather
  L.off_gcount = take(4 * S);
  L.off_queue = take(4 * 2 * S);  // persistent launch: team queue, wave queue
  L.off_head = take(256);
  L.off_actions = take(4 * 7 * S);  // persistent launch: the step's actions at a fixed address
  L.off_glist = take(4 * S);                    // scenes stepped with their working set in global memory
  L.off_gscr = take(4 * (size_t)n_hbm * hbm_words);  // and those working sets
  L.total = o;
  return L;
}

}  // namespace

struct sim_handle {
  int S;
  long N;
  int NB, PM, CM;
  int threads;
  hipStream_t stream;
  char* ws;
  Layout lay;
  int parity;  // cache buffer the next step reads
  int export_on;
  float last_dt;    // dt of the last step (0 before the first)
  int last_export;  // export was on during the last step
  int arm;                 // 0 none, 1 kinematic, 2 articulated with joint motors
  bool parts;              // articulated container parts
  long n_hulls = 0;        // convex hulls in the library
  int art;                 // arm | (rbs::kArtParts if parts): the layouts' articulation code
  float motor_kp, motor_max;
  float link_len[7];
  float arm_radius;
  float gravity[3], margin, baumgarte, slop, rest_thresh, ground_mu, ground_e;
  int solver, warm;
  float tol;
  float sleep_speed = 0.f;  // sleeping islands: off at 0
  int sleep_steps = 0;
  rbs::MlpParams mlp;
  bool mlp_set;
  uint64_t* trace;
  int lds_limit;
  std::vector<int> body_offset;  // host copy, [S + 1]
  // scenes whose working set lives in global memory, and the largest body
  // count of the others
  std::vector<int> hbm;
  long hbm_words = 0;
  int nb_lds = 0;
  hipStream_t capture_stream2 = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // persistent launch
  bool persistent = false;
  int wave_max_bodies = 0;
  bool wave_by_table = false;  // route by the bucket table instead of the threshold
  uint32_t wave_buckets = 0;   // bit k: the scenes of body-count bucket k go to single waves
  int n_team = 0, n_wave = 0, lds_words = 0, grid = 0;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  rbs::StepParams exec_key[2];
  ~sim_handle();
};

sim_handle::~sim_handle() {
  for (int k = 0; k < 2; k++)
    if (exec[k]) hipGraphExecDestroy(exec[k]);
  if (capture_stream) hipStreamDestroy(capture_stream);
  if (capture_stream2) hipStreamDestroy(capture_stream2);
  if (fork_ev) hipEventDestroy(fork_ev);
  if (join_ev) hipEventDestroy(join_ev);
}

namespace {

template <class T>
T* at(sim_handle* h, size_t off) {
  return reinterpret_cast<T*>(h->ws + off);
}

rbs::StepParams params(sim_handle* h) {
  rbs::StepParams P;
  memset(&P, 0, sizeof(P));
  const Layout& L = h->lay;
  P.num_scenes = h->S;
  P.n_bodies = h->N;
  P.scene_cm = (long)h->S * h->CM;
  P.scene_pm = (long)h->S * h->PM;
  P.NB = h->NB;
  P.PM = h->PM;
  P.CM = h->CM;
  P.body_offset = at<int32_t>(h, L.off_body_offset);
  P.shape = at<uint8_t>(h, L.off_shape);
  P.motion = at<uint8_t>(h, L.off_motion);
  P.prm = at<float>(h, L.off_prm);
  P.inv_mass = at<float>(h, L.off_inv_mass);
  P.inv_inertia = at<float>(h, L.off_inv_inertia);
  P.friction = at<float>(h, L.off_friction);
  P.restitution = at<float>(h, L.off_restitution);
  P.pose = at<float>(h, L.off_pose);
  P.vel = at<float>(h, L.off_vel);
  P.rest = at<int32_t>(h, L.off_rest);
  P.sleep_speed = h->sleep_speed;
  P.sleep_steps = h->sleep_steps;
  P.arm = h->arm;
  P.theta = at<float>(h, L.off_theta);
  P.arm_state = h->arm == 2 ? at<float>(h, L.off_arm_state) : nullptr;
  P.arm_rows = h->arm == 2 ? at<float>(h, L.off_arm_rows) : nullptr;
  if (h->parts) {
    P.joint = at<uint8_t>(h, L.off_joint);
    P.joint_axis = at<float>(h, L.off_joint_axis);
    P.joint_anchor = at<float>(h, L.off_joint_anchor);
    P.joint_limits = at<float>(h, L.off_joint_limits);
    P.joint_parent = at<int32_t>(h, L.off_joint_parent);
    P.joint_state = at<float>(h, L.off_joint_state);
  }
  P.art = h->art;
  if (h->n_hulls > 0) {
    P.hull_info = at<int32_t>(h, L.off_hull_info);
    P.hull_vert = at<float4>(h, L.off_hull_vert);
    P.hull_plane = at<float4>(h, L.off_hull_plane);
    P.hull_loop = at<uint8_t>(h, L.off_hull_loop);
    P.hull_edge = at<uint8_t>(h, L.off_hull_edge);
    P.hull_ext = at<float4>(h, L.off_hull_ext);
  }
  P.motor_kp = h->motor_kp;
  P.motor_max = h->motor_max;
  P.arm_base = at<float>(h, L.off_arm_base);
  for (int k = 0; k < 7; k++) P.link_len[k] = h->link_len[k];
  P.arm_radius = h->arm_radius;
  int rd = h->parity, wr = 1 - h->parity;
  P.prev_key = at<uint32_t>(h, L.off_ckey[rd]);
  P.prev_lam = at<float>(h, L.off_clam[rd]);
  P.prev_count = at<int32_t>(h, L.off_ccount[rd]);
  P.cur_key = at<uint32_t>(h, L.off_ckey[wr]);
  P.cur_lam = at<float>(h, L.off_clam[wr]);
  P.cur_count = at<int32_t>(h, L.off_ccount[wr]);
  P.prev_col = at<uint8_t>(h, L.off_ccol[rd]);
  P.cur_col = at<uint8_t>(h, L.off_ccol[wr]);
  P.export_on = h->export_on;
  P.x_pair = at<uint32_t>(h, L.off_x_pair);
  P.x_normal = at<float>(h, L.off_x_normal);
  P.x_point = at<float>(h, L.off_x_point);
  P.x_phi = at<float>(h, L.off_x_phi);
  P.x_lambda = at<float>(h, L.off_x_lambda);
  P.x_colour = at<int32_t>(h, L.off_x_colour);
  P.x_feat = at<float>(h, L.off_x_feat);
  P.raw = at<float4>(h, L.off_raw);
  P.crec = at<float4>(h, L.off_crec);
  P.st_pairs = at<int32_t>(h, L.off_st[0]);
  P.st_contacts = at<int32_t>(h, L.off_st[1]);
  P.st_colours = at<int32_t>(h, L.off_st[2]);
  P.st_sweeps = at<int32_t>(h, L.off_st[3]);
  P.st_flags = at<int32_t>(h, L.off_st[4]);
  P.st_residual = at<float>(h, L.off_st[5]);
  P.st_arm_force = at<float>(h, L.off_st[6]);
  P.gx = h->gravity[0];
  P.gy = h->gravity[1];
  P.gz = h->gravity[2];
  P.margin = h->margin;
  P.baumgarte = h->baumgarte;
  P.slop = h->slop;
  P.rest_thresh = h->rest_thresh;
  P.ground_mu = h->ground_mu;
  P.ground_e = h->ground_e;
  P.tol = h->tol;
  P.warm = h->warm;
  P.solver = h->solver;
  P.mlp = h->mlp;
  P.scene_list = at<int32_t>(h, L.off_scene_list);
  P.gscr = at<float>(h, L.off_gscr);
  P.gwords = h->hbm_words;
  P.glist = at<int32_t>(h, L.off_glist);
  P.trace = h->trace;
  return P;
}

// A hull of the library, prepared in double precision: face planes
// (Newell's normal of the loop through its mean vertex), edges (each
// undirected vertex pair once, in order of first appearance over the
// loops, with the faces of its first and second appearance), the local
// bounding box, and the solid's volume, centre of mass and inertia for a
// unit mass (tetrahedra from the origin over a fan of every loop: a
// tetrahedron (0, a, b, c) of volume v has second moment v/20 (a a^T +
// b b^T + c c^T + s s^T), s = a + b + c, and centroid s / 4).
struct HullPrep {
  int nv = 0, nf = 0;
  std::vector<double> v;          // [nv][3]
  std::vector<int> loop;          // [nf][8], -1 after the last
  std::vector<double> plane;      // [nf][4]
  std::vector<int> edge;          // [ne][4]: a, b, face 0, face 1
  double ext[3] = {0, 0, 0};
  double vol = 0, com[3] = {0, 0, 0}, I[3][3] = {{0}};
};

// Returns an empty string, or what makes the hull unusable.
std::string prepare_hull(const sim_batch_desc* d, int h, HullPrep& P) {
  const int32_t* ix = d->h_hull_index + 4 * h;
  const int v0 = ix[0], nv = ix[1], f0 = ix[2], nf = ix[3];
  if (v0 < 0 || f0 < 0 || nv < 4 || nv > 32 || nf < 4 || nf > 32) return "hull sizes out of range";
  P.nv = nv;
  P.nf = nf;
  P.v.assign(d->h_hull_vert + 3L * v0, d->h_hull_vert + 3L * (v0 + nv));
  for (double x : P.v)
    if (!std::isfinite(x)) return "hull vertices must be finite";
  P.loop.assign(d->h_hull_face + 8L * f0, d->h_hull_face + 8L * (f0 + nf));
  P.plane.assign(4L * nf, 0.0);
  auto V = [&](int k, int c) { return P.v[3 * k + c]; };
  for (int f = 0; f < nf; f++) {
    int n = 0;
    while (n < 8 && P.loop[8 * f + n] >= 0) n++;
    for (int k = n; k < 8; k++)
      if (P.loop[8 * f + k] >= 0) return "a face loop continues after -1";
    if (n < 3) return "a face needs at least 3 vertices";
    double nn[3] = {0, 0, 0}, c[3] = {0, 0, 0};
    for (int k = 0; k < n; k++) {
      const int a = P.loop[8 * f + k], b = P.loop[8 * f + (k + 1) % n];
      if (a >= nv || b >= nv) return "a face loop index is out of range";
      nn[0] += (V(a, 1) - V(b, 1)) * (V(a, 2) + V(b, 2));
      nn[1] += (V(a, 2) - V(b, 2)) * (V(a, 0) + V(b, 0));
      nn[2] += (V(a, 0) - V(b, 0)) * (V(a, 1) + V(b, 1));
      for (int q = 0; q < 3; q++) c[q] += V(a, q);
    }
    const double L = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
    if (!(L > 0)) return "a degenerate face";
    for (int q = 0; q < 3; q++) P.plane[4 * f + q] = nn[q] / L;
    P.plane[4 * f + 3] = (P.plane[4 * f] * c[0] + P.plane[4 * f + 1] * c[1] + P.plane[4 * f + 2] * c[2]) / n;
    for (int k = 0; k < n; k++) {
      const int a = P.loop[8 * f + k], b = P.loop[8 * f + (k + 1) % n];
      const int lo = std::min(a, b), hi = std::max(a, b);
      int seen = -1;
      for (size_t e = 0; e < P.edge.size() / 4; e++)
        if (P.edge[4 * e] == lo && P.edge[4 * e + 1] == hi) seen = (int)e;
      if (seen < 0) P.edge.insert(P.edge.end(), {lo, hi, f, -1});
      else if (P.edge[4 * seen + 3] < 0) P.edge[4 * seen + 3] = f;
      else return "an edge is shared by more than two faces";
    }
  }
  if (P.edge.size() / 4 > 64) return "more than 64 edges";
  for (size_t e = 0; e < P.edge.size() / 4; e++)
    if (P.edge[4 * e + 3] < 0) return "the faces do not close the surface";
  // convex: every vertex on or inside every face plane
  double ext = 0;
  for (int k = 0; k < nv; k++)
    for (int q = 0; q < 3; q++) {
      P.ext[q] = std::max(P.ext[q], std::fabs(V(k, q)));
      ext = std::max(ext, std::fabs(V(k, q)));
    }
  for (int f = 0; f < nf; f++)
    for (int k = 0; k < nv; k++) {
      const double s = P.plane[4 * f] * V(k, 0) + P.plane[4 * f + 1] * V(k, 1) + P.plane[4 * f + 2] * V(k, 2) -
                       P.plane[4 * f + 3];
      if (s > 1e-5 * ext) return "the hull is not convex (or a loop is clockwise)";
    }
  double C[3][3] = {{0}}, cm[3] = {0, 0, 0};
  for (int f = 0; f < nf; f++) {
    int n = 0;
    while (n < 8 && P.loop[8 * f + n] >= 0) n++;
    for (int k = 1; k + 1 < n; k++) {
      const int ia = P.loop[8 * f], ib = P.loop[8 * f + k], ic = P.loop[8 * f + k + 1];
      const double a[3] = {V(ia, 0), V(ia, 1), V(ia, 2)}, b[3] = {V(ib, 0), V(ib, 1), V(ib, 2)},
                   c[3] = {V(ic, 0), V(ic, 1), V(ic, 2)};
      const double vt = (a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                         a[2] * (b[0] * c[1] - b[1] * c[0])) / 6.0;
      const double sm[3] = {a[0] + b[0] + c[0], a[1] + b[1] + c[1], a[2] + b[2] + c[2]};
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
          C[i][j] += vt / 20.0 * (a[i] * a[j] + b[i] * b[j] + c[i] * c[j] + sm[i] * sm[j]);
      for (int i = 0; i < 3; i++) cm[i] += vt * sm[i] / 4.0;
      P.vol += vt;
    }
  }
  if (!(P.vol > 0)) return "the hull has no volume";
  for (int i = 0; i < 3; i++) P.com[i] = cm[i] / P.vol;
  const double tr = (C[0][0] + C[1][1] + C[2][2]) / P.vol;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) P.I[i][j] = (i == j ? tr : 0.0) - C[i][j] / P.vol;
  const double Imax = std::max(P.I[0][0], std::max(P.I[1][1], P.I[2][2]));
  for (int i = 0; i < 3; i++)
    if (std::fabs(P.com[i]) > 1e-6 * ext) return "the hull's origin is not its centre of mass";
  if (std::fabs(P.I[0][1]) > 1e-6 * Imax || std::fabs(P.I[0][2]) > 1e-6 * Imax || std::fabs(P.I[1][2]) > 1e-6 * Imax)
    return "the hull's axes are not its principal axes";
  return "";
}

struct Caps {
  int NB;
  long N;
  bool ok;
};

int validate(const sim_batch_desc* d, Caps* caps) {
  if (!d) return fail(SIM_EINVAL, "descriptor is NULL");
  if (d->abi_version != SIM_ABI_VERSION) return fail(SIM_EABI, "abi_version mismatch");
  if (d->num_scenes < 1) return fail(SIM_EINVAL, "num_scenes must be >= 1");
  if (!d->h_body_offset || !d->h_shape || !d->h_motion || !d->h_param || !d->h_mass || !d->h_friction ||
      !d->h_restitution || !d->h_pose || !d->h_vel)
    return fail(SIM_EINVAL, "a required host array is NULL");
  if (d->h_body_offset[0] != 0) return fail(SIM_EINVAL, "body_offset[0] must be 0");
  int NB = 0;
  for (int s = 0; s < d->num_scenes; s++) {
    int n = d->h_body_offset[s + 1] - d->h_body_offset[s];
    if (n < 0) return fail(SIM_EINVAL, "body_offset must be non-decreasing");
    if (n > rbs::kMaxBodiesPerScene) return fail(SIM_ECAPACITY, "a scene exceeds 2046 bodies");
    if (d->arm && n < 7) return fail(SIM_EINVAL, "arm scenes need at least 7 bodies");
    NB = std::max(NB, n);
  }
  long N = d->h_body_offset[d->num_scenes];
  for (long i = 0; i < N; i++) {
    if (d->h_shape[i] > SIM_HULL) return fail(SIM_EINVAL, "bad shape type");
    if (d->h_motion[i] > SIM_KINEMATIC) return fail(SIM_EINVAL, "bad motion type");
    const float* p = d->h_param + 3 * i;
    int sh = d->h_shape[i];
    if (sh == SIM_HULL) {
      if (!(p[0] >= 0.f && p[0] < (float)d->n_hulls) || p[0] != std::floor(p[0]))
        return fail(SIM_EINVAL, "a hull body needs the index of a hull in the library");
    } else {
      int need = sh == SIM_SPHERE ? 1 : (sh == SIM_BOX ? 3 : 2);
      for (int k = 0; k < need; k++)
        if (!(p[k] > 0.f) || !std::isfinite(p[k])) return fail(SIM_EINVAL, "shape parameters must be positive");
    }
    if (d->h_motion[i] == SIM_DYNAMIC && !(d->h_mass[i] > 0.f && std::isfinite(d->h_mass[i])))
      return fail(SIM_EINVAL, "dynamic bodies need a positive mass");
  }
  if (d->arm < 0 || d->arm > 2) return fail(SIM_EINVAL, "arm must be 0, 1 or 2");
  if (d->arm == 2 && (d->solver != SIM_PGS || d->warm_start == SIM_LEARNED))
    return fail(SIM_EINVAL, "the articulated arm needs the PGS solver without the learned warm start");
  if (d->arm) {
    if (!d->h_arm_base || !d->h_arm_theta) return fail(SIM_EINVAL, "arm needs base and theta arrays");
    const int want = d->arm == 2 ? SIM_DYNAMIC : SIM_KINEMATIC;
    for (int s = 0; s < d->num_scenes; s++)
      for (int k = 0; k < 7; k++) {
        long i = d->h_body_offset[s + 1] - 7 + k;
        if (d->h_shape[i] != SIM_CAPSULE || d->h_motion[i] != want)
          return fail(SIM_EINVAL, d->arm == 2 ? "the last 7 bodies of an articulated arm scene must be dynamic capsules"
                                              : "the last 7 bodies of an arm scene must be kinematic capsules");
      }
  }
  if (d->h_joint) {
    if (!d->h_joint_axis || !d->h_joint_anchor || !d->h_joint_limits || !d->h_joint_parent)
      return fail(SIM_EINVAL, "container parts need axis, anchor, limit and parent arrays");
    if (d->solver != SIM_PGS || d->warm_start == SIM_LEARNED)
      return fail(SIM_EINVAL, "container parts need the PGS solver without the learned warm start");
    for (int s = 0; s < d->num_scenes; s++) {
      const int b0 = d->h_body_offset[s], nb = d->h_body_offset[s + 1] - b0;
      int np = 0;
      for (int k = 0; k < nb; k++) {
        const long i = b0 + k;
        const int kind = d->h_joint[i];
        if (kind == 0) continue;
        if (kind > 2) return fail(SIM_EINVAL, "joint kind must be 0, 1 or 2");
        if (d->h_motion[i] != SIM_DYNAMIC) return fail(SIM_EINVAL, "a container part must be a dynamic body");
        if (d->arm && k >= nb - 7) return fail(SIM_EINVAL, "an arm link cannot be a container part");
        const float* a = d->h_joint_axis + 3 * i;
        const float* o = d->h_joint_anchor + 3 * i;
        const float* lim = d->h_joint_limits + 2 * i;
        const double n2 = (double)a[0] * a[0] + (double)a[1] * a[1] + (double)a[2] * a[2];
        if (!(std::fabs(n2 - 1.0) <= 1e-4)) return fail(SIM_EINVAL, "a joint axis must be a unit vector");
        if (!std::isfinite(o[0]) || !std::isfinite(o[1]) || !std::isfinite(o[2]))
          return fail(SIM_EINVAL, "joint anchors must be finite");
        if (!std::isfinite(lim[0]) || !std::isfinite(lim[1]) || !(lim[0] <= lim[1]))
          return fail(SIM_EINVAL, "joint limits must be finite with lower <= upper");
        const int par = d->h_joint_parent[i];
        if (par < -1 || par >= nb || par == k) return fail(SIM_EINVAL, "bad joint parent index");
        if (++np > rbs::kMaxParts) return fail(SIM_ECAPACITY, "a scene exceeds 16 container parts");
      }
    }
  }
  if (d->n_hulls < 0) return fail(SIM_EINVAL, "n_hulls must be >= 0");
  if (d->n_hulls > 0) {
    if (!d->h_hull_index || !d->h_hull_vert || !d->h_hull_face)
      return fail(SIM_EINVAL, "a hull library needs index, vertex and face arrays");
    if (d->warm_start == SIM_LEARNED) return fail(SIM_EINVAL, "convex hulls are not available with the learned warm start");
    for (int h = 0; h < d->n_hulls; h++) {
      HullPrep hp;
      const std::string why = prepare_hull(d, h, hp);
      if (!why.empty()) return fail(SIM_EINVAL, "hull " + std::to_string(h) + ": " + why);
    }
  }
  if (d->max_pairs < 1 || d->max_contacts < 1) return fail(SIM_EINVAL, "capacities must be >= 1");
  if (d->max_pairs > (1 << 20) || d->max_contacts > (1 << 20)) return fail(SIM_EINVAL, "capacity too large");
  // the narrowphase stages 4 contacts per pair in a contact record slot set
  int T = d->threads ? d->threads : 64;
  if (T != 64 && T != 128 && T != 192 && T != 256) return fail(SIM_EINVAL, "threads must be 64, 128, 192 or 256");
  if (d->solver != SIM_PGS && d->solver != SIM_JACOBI) return fail(SIM_EINVAL, "bad solver");
  if (d->warm_start < SIM_COLD || d->warm_start > SIM_LEARNED) return fail(SIM_EINVAL, "bad warm start");
  if (!(d->tolerance >= 0.f)) return fail(SIM_EINVAL, "tolerance must be >= 0");
  if (!(d->margin >= 0.f) || !(d->slop >= 0.f) || !(d->baumgarte >= 0.f)) return fail(SIM_EINVAL, "bad constants");
  if (d->hbm_min_bodies < 0) return fail(SIM_EINVAL, "hbm_min_bodies must be >= 0");
  caps->NB = NB;
  caps->N = N;
  caps->ok = true;
  return SIM_OK;
}

// articulation code of a descriptor (the layouts' last argument)
int desc_art(const sim_batch_desc* d) { return d->arm | (d->h_joint ? rbs::kArtParts : 0); }

// device table sizes of a validated descriptor's hull library
HullSizes hull_sizes(const sim_batch_desc* d) {
  HullSizes hs;
  hs.H = d->n_hulls;
  for (int h = 0; h < d->n_hulls; h++) {
    HullPrep hp;
    prepare_hull(d, h, hp);
    hs.V += hp.nv;
    hs.F += hp.nf;
    hs.E += (long)hp.edge.size() / 4;
  }
  return hs;
}

int lds_bytes(int NB, int PM, int CM, int T, int solver, int warm, int arm) {
  rbs::LdsLayout L = rbs::lds_layout(NB, PM, CM, T / 64, solver, warm, arm);
  return L.total * 4;
}

bool aligned(const void* p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

int device_lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
  return v;
}

// LDS words a 256-thread workgroup of the persistent launch may use for a
// scene (the device limit less the kernel's static words).
int team_lds_words(int lds_limit) { return ((lds_limit - 256) / 4) & ~15; }

// Working-set words of a scene of nb bodies in its largest solver mode
// (Jacobi with the learned start) for a 256-thread team.
long worst_words(int nb, int PM, int CM, int arm) {
  return rbs::lds_layout(nb, rbs::scene_cap(nb, PM), rbs::scene_cap(nb, CM), 4, rbs::SOLVER_JACOBI, rbs::WARM_LEARNED,
                         arm)
      .total;
}

// Scenes stepped with their working set in global memory: those whose
// largest working set exceeds a workgroup's LDS, and those of at least
// min_bodies bodies when min_bodies > 0.  Largest first; words: the region
// each gets (the largest such working set, a multiple of 64 words).
struct HbmSplit {
  std::vector<int> scenes;
  long words = 0;
  int nb_lds = 0;  // largest body count among the other scenes
};

HbmSplit hbm_split(const int32_t* off, int S, int PM, int CM, int lds_limit, int min_bodies, int arm) {
  HbmSplit r;
  const long budget = team_lds_words(lds_limit);
  for (int s = 0; s < S; s++) {
    const int nb = off[s + 1] - off[s];
    const long w = worst_words(nb, PM, CM, arm);
    if (w > budget || (min_bodies > 0 && nb >= min_bodies)) {
      r.scenes.push_back(s);
      r.words = std::max(r.words, (w + 63) & ~63L);
    } else {
      r.nb_lds = std::max(r.nb_lds, nb);
    }
  }
  std::stable_sort(r.scenes.begin(), r.scenes.end(),
                   [&](int a, int b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
  return r;
}

// Body-count buckets of the persistent launch's routing table: [1, 16],
// (16, 32], ..., (512, 1024], (1024, 2046].
constexpr int kBuckets = 8;
int body_bucket(int nb) {
  int k = 0;
  for (int hi = 16; k < kBuckets - 1 && nb > hi; hi *= 2) k++;
  return k;
}

// Persistent launch: a queue for whole-workgroup teams and one for single-wave
// teams, each in descending body count (ties by scene index).  A scene goes
// to a wave when its routing says so (at most wave_max_bodies bodies, or its
// body-count bucket's bit in the table) and its working set (for the current
// solver mode) fits a quarter of the workgroup's LDS.
int build_queues(sim_handle* h, int wave_max_bodies, bool by_table = false, uint32_t buckets = 0) {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SIM_EDEVICE, "hipGetDevice failed");
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
    return fail(SIM_EDEVICE, "multiprocessor count unavailable");
  // the workgroup's dynamic LDS: the device limit less its static words, a multiple of 16 words
  const int lds_words = team_lds_words(h->lds_limit);
  std::vector<int> team, wave;
  std::vector<char> in_hbm(h->S, 0);
  for (int s : h->hbm) in_hbm[s] = 1;
  for (int s = 0; s < h->S; s++) {
    if (in_hbm[s]) continue;
    const int nb = h->body_offset[s + 1] - h->body_offset[s];
    const int pm = rbs::scene_cap(nb, h->PM), cm = rbs::scene_cap(nb, h->CM);
    const int need_wave = rbs::lds_layout(nb, pm, cm, 1, h->solver, h->warm, h->art).total;
    const int need_team = rbs::lds_layout(nb, pm, cm, 4, h->solver, h->warm, h->art).total;
    const bool to_wave = by_table ? ((buckets >> body_bucket(nb)) & 1u) != 0u : nb <= wave_max_bodies;
    if (to_wave && need_wave <= lds_words / 4)
      wave.push_back(s);
    else if (need_team <= lds_words)
      team.push_back(s);
    else
      return fail(SIM_ECAPACITY, "scene " + std::to_string(s) + " does not fit a workgroup's LDS");
  }
  auto by_size = [&](int a, int b) {
    const int na = h->body_offset[a + 1] - h->body_offset[a], nb = h->body_offset[b + 1] - h->body_offset[b];
    return na != nb ? na > nb : a < b;
  };
  std::sort(team.begin(), team.end(), by_size);
  std::sort(wave.begin(), wave.end(), by_size);
  std::vector<int32_t> q(2 * (size_t)h->S, 0);
  std::copy(team.begin(), team.end(), q.begin());
  std::copy(wave.begin(), wave.end(), q.begin() + h->S);
  hipError_t e = hipMemcpyAsync(at<int32_t>(h, h->lay.off_queue), q.data(), q.size() * 4, hipMemcpyHostToDevice,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(SIM_EDEVICE, "queue upload failed");
  h->n_team = (int)team.size();
  h->n_wave = (int)wave.size();
  h->lds_words = lds_words;
  h->grid = ncu;
  h->wave_max_bodies = wave_max_bodies;
  h->wave_by_table = by_table;
  h->wave_buckets = buckets;
  for (int k = 0; k < 2; k++)
    if (h->exec[k]) {
      hipGraphExecDestroy(h->exec[k]);
      h->exec[k] = nullptr;
    }
  return SIM_OK;
}

rbs::QueueParams queue_params(sim_handle* h) {
  rbs::QueueParams Q;
  Q.team = at<int32_t>(h, h->lay.off_queue);
  Q.wave = at<int32_t>(h, h->lay.off_queue) + h->S;
  Q.n_team = h->n_team;
  Q.n_wave = h->n_wave;
  Q.head = at<uint32_t>(h, h->lay.off_head);
  Q.lds_words = h->lds_words;
  return Q;
}

// LDS layout shared by the scenes stepped out of global memory (their largest
// scene, current solver mode, 256-thread teams).
rbs::LdsLayout hbm_layout(const sim_handle* h) {
  int nb = 0;
  for (int s : h->hbm) nb = std::max(nb, h->body_offset[s + 1] - h->body_offset[s]);
  return rbs::lds_layout(nb, rbs::scene_cap(nb, h->PM), rbs::scene_cap(nb, h->CM), 4, h->solver, h->warm, h->art);
}

// One step through a graph of (queue reset, persistent kernel) captured once
// per cache parity and argument set, replayed on the handle's stream.  When
// scenes run out of global memory, their kernel is a parallel branch of the
// graph (forked onto a second capture stream), so that it shares the device
// with the persistent kernel.
int launch_persistent(sim_handle* h, const rbs::StepParams& P) {
  const int par = h->parity;
  if (!h->exec[par] || memcmp(&h->exec_key[par], &P, sizeof(P)) != 0) {
    if (h->exec[par]) {
      hipGraphExecDestroy(h->exec[par]);
      h->exec[par] = nullptr;
    }
    hipError_t e;
    if (!h->capture_stream) {
      e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return (int)e;
    }
    const bool fork = !h->hbm.empty();
    if (fork && !h->capture_stream2) {
      e = hipStreamCreateWithFlags(&h->capture_stream2, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming);
      if (e != hipSuccess) return (int)e;
    }
    rbs::QueueParams Q = queue_params(h);
    const rbs::LdsLayout LH = hbm_layout(h);
    e = hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return (int)e;
    int rc = 0;
    if (fork) {
      if (hipEventRecord(h->fork_ev, h->capture_stream) != hipSuccess ||
          hipStreamWaitEvent(h->capture_stream2, h->fork_ev, 0) != hipSuccess)
        rc = -1;
      if (rc == 0) rc = rbs_launch_step_hbm(&P, &LH, (int)h->hbm.size(), h->capture_stream2);
      if (rc == 0 && hipEventRecord(h->join_ev, h->capture_stream2) != hipSuccess) rc = -1;
    }
    if (rc == 0) rc = rbs_launch_persistent(&P, &Q, h->grid, h->capture_stream);
    if (fork && rc == 0 && hipStreamWaitEvent(h->capture_stream, h->join_ev, 0) != hipSuccess) rc = -1;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->capture_stream, &g);
    if (rc != 0) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return (int)e;
    e = hipGraphInstantiate(&h->exec[par], g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
      h->exec[par] = nullptr;
      return (int)e;
    }
    h->exec_key[par] = P;
  }
  return (int)hipGraphLaunch(h->exec[par], h->stream);
}

// State a step changes (and the autotuner restores): pose, velocity, joint
// angles and both contact caches.
struct StateSpan {
  size_t off, bytes;
};

std::vector<StateSpan> state_spans(const sim_handle* h) {
  const Layout& L = h->lay;
  const size_t S = h->S, N = h->N, CM = h->CM;
  std::vector<StateSpan> v = {{L.off_pose, 4 * 7 * N}, {L.off_vel, 4 * 6 * N}, {L.off_rest, 4 * N},
                              {L.off_theta, 4 * 7 * S}};
  if (h->arm == 2) v.push_back({L.off_arm_state, 4 * 21 * S});
  if (h->parts) v.push_back({L.off_joint_state, 4 * 2 * N});
  for (int k = 0; k < 2; k++) {
    v.push_back({L.off_ckey[k], 4 * S * CM});
    v.push_back({L.off_clam[k], 4 * 4 * S * CM});
    v.push_back({L.off_ccount[k], 4 * S});
  }
  return v;
}

size_t state_bytes(const sim_handle* h) {
  size_t t = 0;
  for (const StateSpan& sp : state_spans(h)) t += align256(sp.bytes);
  return t;
}

int copy_state(sim_handle* h, char* scratch, bool save) {
  size_t o = 0;
  for (const StateSpan& sp : state_spans(h)) {
    void* dev = h->ws + sp.off;
    hipError_t e = save ? hipMemcpyAsync(scratch + o, dev, sp.bytes, hipMemcpyDeviceToDevice, h->stream)
                        : hipMemcpyAsync(dev, scratch + o, sp.bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return (int)e;
    o += align256(sp.bytes);
  }
  return 0;
}

}  // namespace

extern "C" {

size_t sim_workspace_bytes(const sim_batch_desc* d) {
  Caps c;
  if (validate(d, &c) != SIM_OK) return 0;
  const HbmSplit sp = hbm_split(d->h_body_offset, d->num_scenes, d->max_pairs, d->max_contacts, device_lds_limit(),
                                d->hbm_min_bodies, desc_art(d));
  return make_layout(d->num_scenes, c.N, d->max_pairs, d->max_contacts, (long)sp.scenes.size(), sp.words, desc_art(d),
                     hull_sizes(d))
      .total;
}

int sim_create(const sim_batch_desc* d, void* d_workspace, size_t workspace_bytes, sim_handle** out) {
  if (!out) return fail(SIM_EINVAL, "out is NULL");
  *out = nullptr;
  Caps c;
  int rc = validate(d, &c);
  if (rc != SIM_OK) return rc;
  const int S = d->num_scenes;
  const long N = c.N;
  const int limit = device_lds_limit();
  const int art = desc_art(d);
  HbmSplit sp = hbm_split(d->h_body_offset, S, d->max_pairs, d->max_contacts, limit, d->hbm_min_bodies, art);
  const HullSizes hs = hull_sizes(d);
  Layout lay = make_layout(S, N, d->max_pairs, d->max_contacts, (long)sp.scenes.size(), sp.words, art, hs);
  if (!d_workspace || workspace_bytes < lay.total) return fail(SIM_EWORKSPACE, "workspace too small");
  if (((uintptr_t)d_workspace & 255u) != 0) return fail(SIM_EWORKSPACE, "workspace must be 256-byte aligned");
  const int T = d->threads ? d->threads : 64;
  // the working set of the largest scene kept in LDS, under any solver mode
  // (the split above sends every larger one to global memory)
  const int nbl = sp.nb_lds;
  int need = nbl ? lds_bytes(nbl, rbs::scene_cap(nbl, d->max_pairs), rbs::scene_cap(nbl, d->max_contacts), T,
                             rbs::SOLVER_JACOBI, rbs::WARM_LEARNED, art)
                 : 0;
  if (need > limit)
    return fail(SIM_ECAPACITY, "per-scene working set (" + std::to_string(need) + " B) exceeds LDS (" +
                                   std::to_string(limit) + " B)");
  if (rbs_set_step_lds_limit(limit) != 0) return fail(SIM_EDEVICE, "hipFuncSetAttribute failed");

  sim_handle* h = new sim_handle();
  h->S = S;
  h->N = N;
  h->NB = c.NB;
  h->PM = d->max_pairs;
  h->CM = d->max_contacts;
  h->threads = T;
  h->stream = (hipStream_t)d->stream;
  h->ws = (char*)d_workspace;
  h->lay = lay;
  h->parity = 0;
  h->export_on = 0;
  h->last_dt = 0.f;
  h->last_export = 0;
  h->arm = d->arm;
  h->parts = d->h_joint != nullptr;
  h->n_hulls = d->n_hulls;
  h->art = art;
  h->motor_kp = 0.3f;      // position gain of the joint motors (Sec. 5)
  h->motor_max = 10.0f;    // largest motor impulse per step, N s (Sec. 5)
  for (int k = 0; k < 7; k++) h->link_len[k] = d->link_len[k];
  h->arm_radius = d->arm_radius;
  for (int k = 0; k < 3; k++) h->gravity[k] = d->gravity[k];
  h->margin = d->margin;
  h->baumgarte = d->baumgarte;
  h->slop = d->slop;
  h->rest_thresh = d->rest_thresh;
  h->ground_mu = d->ground_friction;
  h->ground_e = d->ground_restitution;
  h->solver = d->solver;
  h->warm = d->warm_start;
  h->tol = d->tolerance;
  memset(&h->mlp, 0, sizeof(h->mlp));
  h->mlp_set = false;
  h->trace = nullptr;
  h->lds_limit = limit;
  h->body_offset.assign(d->h_body_offset, d->h_body_offset + S + 1);
  h->hbm = sp.scenes;
  h->hbm_words = sp.words;
  h->nb_lds = nbl;

  // the hull library, prepared once
  std::vector<HullPrep> preps(d->n_hulls > 0 ? d->n_hulls : 0);
  for (int hh = 0; hh < d->n_hulls; hh++) prepare_hull(d, hh, preps[hh]);
  // host staging: structure-of-arrays planes
  std::vector<float> prm(3 * N), inv_mass(N), inv_I(3 * N), pose(7 * N), vel(6 * N);
  for (long i = 0; i < N; i++) {
    for (int k = 0; k < 3; k++) prm[k * N + i] = d->h_param[3 * i + k];
    for (int k = 0; k < 7; k++) pose[k * N + i] = d->h_pose[7 * i + k];
    for (int k = 0; k < 6; k++) vel[k * N + i] = d->h_vel[6 * i + k];
    if (d->h_motion[i] == SIM_DYNAMIC) {
      double m = d->h_mass[i];
      const float* p = d->h_param + 3 * i;
      double I[3];
      if (d->h_shape[i] == SIM_HULL) {  // principal moments of the solid hull (its frame is principal)
        const HullPrep& hp = preps[(int)p[0]];
        for (int k = 0; k < 3; k++) I[k] = m * hp.I[k][k];
      } else if (d->h_shape[i] == SIM_SPHERE) {
        I[0] = I[1] = I[2] = 0.4 * m * (double)p[0] * p[0];
      } else if (d->h_shape[i] == SIM_BOX) {
        double x2 = (double)p[0] * p[0], y2 = (double)p[1] * p[1], z2 = (double)p[2] * p[2];
        I[0] = m / 3.0 * (y2 + z2);
        I[1] = m / 3.0 * (x2 + z2);
        I[2] = m / 3.0 * (x2 + y2);
      } else {
        // solid capsule: cylinder (length 2h) + two hemispheres, mass by volume
        double r = p[0], hh = p[1];
        double vc = 2.0 * M_PI * r * r * hh, vs = 4.0 / 3.0 * M_PI * r * r * r;
        double mc = m * vc / (vc + vs), ms = m - mc;
        I[2] = mc * r * r / 2.0 + 0.4 * ms * r * r;
        I[0] = I[1] = mc * (r * r / 4.0 + hh * hh / 3.0) + ms * (0.4 * r * r + hh * hh + 0.75 * hh * r);
      }
      inv_mass[i] = (float)(1.0 / m);
      for (int k = 0; k < 3; k++) inv_I[k * N + i] = (float)(1.0 / I[k]);
    } else {
      inv_mass[i] = 0.f;
      for (int k = 0; k < 3; k++) inv_I[k * N + i] = 0.f;
    }
  }
  // largest scenes first: the tail of the grid holds the cheap scenes; the
  // scenes stepped out of global memory have their own list
  std::vector<char> in_hbm(S, 0);
  for (int s : sp.scenes) in_hbm[s] = 1;
  std::vector<int32_t> order;
  for (int s = 0; s < S; s++)
    if (!in_hbm[s]) order.push_back(s);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return d->h_body_offset[a + 1] - d->h_body_offset[a] > d->h_body_offset[b + 1] - d->h_body_offset[b];
  });
  order.resize(S, 0);
  std::vector<int32_t> glist(sp.scenes.begin(), sp.scenes.end());
  glist.resize(S, 0);
  std::vector<float> theta(7 * S, 0.f), base(3 * S, 0.f);
  if (d->arm) {
    for (int i = 0; i < 7 * S; i++) theta[i] = d->h_arm_theta[i];
    for (int i = 0; i < 3 * S; i++) base[i] = d->h_arm_base[i];
  }
  hipStream_t st = h->stream;
  auto up = [&](size_t off, const void* src, size_t bytes) {
    return hipMemcpyAsync(h->ws + off, src, bytes, hipMemcpyHostToDevice, st);
  };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemsetAsync(h->ws, 0, lay.total, st);
  if (e == hipSuccess) e = up(lay.off_body_offset, d->h_body_offset, 4 * (S + 1));
  if (e == hipSuccess) e = up(lay.off_shape, d->h_shape, N);
  if (e == hipSuccess) e = up(lay.off_motion, d->h_motion, N);
  if (e == hipSuccess) e = up(lay.off_prm, prm.data(), 4 * 3 * N);
  if (e == hipSuccess) e = up(lay.off_inv_mass, inv_mass.data(), 4 * N);
  if (e == hipSuccess) e = up(lay.off_inv_inertia, inv_I.data(), 4 * 3 * N);
  if (e == hipSuccess) e = up(lay.off_friction, d->h_friction, 4 * N);
  if (e == hipSuccess) e = up(lay.off_restitution, d->h_restitution, 4 * N);
  if (e == hipSuccess) e = up(lay.off_pose, pose.data(), 4 * 7 * N);
  if (e == hipSuccess) e = up(lay.off_vel, vel.data(), 4 * 6 * N);
  if (e == hipSuccess) e = up(lay.off_theta, theta.data(), 4 * 7 * S);
  std::vector<float> arm_state;
  if (d->arm == 2) {  // at rest, motor targets at the initial angles, no motor impulses yet
    arm_state.assign(21 * (size_t)S, 0.f);
    for (int s2 = 0; s2 < S; s2++)
      for (int k = 0; k < 7; k++) arm_state[21 * s2 + 7 + k] = theta[7 * s2 + k];
    if (e == hipSuccess) e = up(lay.off_arm_state, arm_state.data(), 4 * 21 * S);
  }
  std::vector<float> jax, jan, jlim;
  if (d->h_joint) {  // planes [3][N], [3][N], [2][N]; q and qd start at 0 (the workspace is cleared)
    jax.assign(3 * (size_t)N, 0.f);
    jan.assign(3 * (size_t)N, 0.f);
    jlim.assign(2 * (size_t)N, 0.f);
    for (long i = 0; i < N; i++) {
      for (int k = 0; k < 3; k++) {
        jax[k * N + i] = d->h_joint_axis[3 * i + k];
        jan[k * N + i] = d->h_joint_anchor[3 * i + k];
      }
      for (int k = 0; k < 2; k++) jlim[k * N + i] = d->h_joint_limits[2 * i + k];
    }
    if (e == hipSuccess) e = up(lay.off_joint, d->h_joint, N);
    if (e == hipSuccess) e = up(lay.off_joint_axis, jax.data(), 4 * 3 * N);
    if (e == hipSuccess) e = up(lay.off_joint_anchor, jan.data(), 4 * 3 * N);
    if (e == hipSuccess) e = up(lay.off_joint_limits, jlim.data(), 4 * 2 * N);
    if (e == hipSuccess) e = up(lay.off_joint_parent, d->h_joint_parent, 4 * N);
  }
  if (d->n_hulls > 0) {  // the hull library's device tables
    std::vector<int32_t> info(8L * hs.H, 0);
    std::vector<float> hv(4 * hs.V, 0.f), hp4(4 * hs.F, 0.f), hext(4 * hs.H, 0.f);
    std::vector<uint8_t> hloop(8 * hs.F, 255u), hedge(4 * hs.E, 0u);
    long v0 = 0, f0 = 0, e0 = 0;
    for (int hh = 0; hh < d->n_hulls; hh++) {
      const HullPrep& q = preps[hh];
      const long ne = (long)q.edge.size() / 4;
      const int32_t row[8] = {(int32_t)v0, q.nv, (int32_t)f0, q.nf, (int32_t)e0, (int32_t)ne, 0, 0};
      for (int k = 0; k < 8; k++) info[8 * hh + k] = row[k];
      for (int k = 0; k < q.nv; k++)
        for (int c = 0; c < 3; c++) hv[4 * (v0 + k) + c] = (float)q.v[3 * k + c];
      for (int f = 0; f < q.nf; f++) {
        for (int c = 0; c < 4; c++) hp4[4 * (f0 + f) + c] = (float)q.plane[4 * f + c];
        for (int k = 0; k < 8; k++)
          if (q.loop[8 * f + k] >= 0) hloop[8 * (f0 + f) + k] = (uint8_t)q.loop[8 * f + k];
      }
      for (long k = 0; k < ne; k++)
        for (int c = 0; c < 4; c++) hedge[4 * (e0 + k) + c] = (uint8_t)q.edge[4 * k + c];
      for (int c = 0; c < 3; c++) hext[4 * hh + c] = (float)q.ext[c];
      v0 += q.nv;
      f0 += q.nf;
      e0 += ne;
    }
    if (e == hipSuccess) e = up(lay.off_hull_info, info.data(), 4 * info.size());
    if (e == hipSuccess) e = up(lay.off_hull_vert, hv.data(), 4 * hv.size());
    if (e == hipSuccess) e = up(lay.off_hull_plane, hp4.data(), 4 * hp4.size());
    if (e == hipSuccess) e = up(lay.off_hull_loop, hloop.data(), hloop.size());
    if (e == hipSuccess) e = up(lay.off_hull_edge, hedge.data(), hedge.size());
    if (e == hipSuccess) e = up(lay.off_hull_ext, hext.data(), 4 * hext.size());
  }
  if (e == hipSuccess) e = up(lay.off_arm_base, base.data(), 4 * 3 * S);
  if (e == hipSuccess) e = up(lay.off_scene_list, order.data(), 4 * S);
  if (e == hipSuccess) e = up(lay.off_glist, glist.data(), 4 * S);
  if (e == hipSuccess && h->arm) {
    rbs::StepParams P = params(h);
    e = (hipError_t)rbs_launch_arm_pose(&P, nullptr, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete h;
    return fail(SIM_EDEVICE, std::string("upload failed: ") + hipGetErrorString(e));
  }
  *out = h;
  return SIM_OK;
}

int sim_step(sim_handle* h, const float* d_actions, float dt, int iters) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (!(dt > 0.f) || !std::isfinite(dt)) return fail(SIM_EINVAL, "dt must be > 0");
  if (iters < 1) return fail(SIM_EINVAL, "iters must be >= 1");
  if (h->warm == SIM_LEARNED && !h->mlp_set) return fail(SIM_EINVAL, "learned warm start needs sim_set_mlp");
  rbs::StepParams P = params(h);
  P.actions = d_actions;
  P.dt = dt;
  P.iters = iters;
  int rc;
  if (h->persistent) {
    // The graph's kernel reads the actions from a fixed buffer, so that a
    // new action array each step does not force a new capture.
    if (h->arm) {
      float* fixed = at<float>(h, h->lay.off_actions);
      const size_t bytes = sizeof(float) * 7 * (size_t)h->S;
      hipError_t e = d_actions ? hipMemcpyAsync(fixed, d_actions, bytes, hipMemcpyDeviceToDevice, h->stream)
                               : hipMemsetAsync(fixed, 0, bytes, h->stream);
      if (e != hipSuccess) return fail(SIM_EDEVICE, std::string("action copy failed: ") + hipGetErrorString(e));
      P.actions = fixed;
    } else {
      P.actions = nullptr;
    }
    rc = launch_persistent(h, P);
    if (rc != 0) return fail(SIM_EDEVICE, std::string("persistent step failed: ") + hipGetErrorString((hipError_t)rc));
  } else {
    const int nl = h->S - (int)h->hbm.size(), nbl = h->nb_lds;
    rc = 0;
    if (nl > 0) {
      rbs::LdsLayout L = rbs::lds_layout(nbl, rbs::scene_cap(nbl, h->PM), rbs::scene_cap(nbl, h->CM),
                                         h->threads / 64, h->solver, h->warm, h->art);
      if (L.total * 4 > h->lds_limit) return fail(SIM_ECAPACITY, "working set exceeds LDS");
      rc = rbs_launch_step(&P, &L, h->threads, nl, h->stream);
    }
    if (rc == 0 && !h->hbm.empty()) {
      const rbs::LdsLayout LH = hbm_layout(h);
      rc = rbs_launch_step_hbm(&P, &LH, (int)h->hbm.size(), h->stream);
    }
    if (rc != 0) return fail(SIM_EDEVICE, std::string("step launch failed: ") + hipGetErrorString((hipError_t)rc));
  }
  h->parity ^= 1;
  h->last_dt = dt;
  h->last_export = h->export_on;
  return SIM_OK;
}

int sim_query_arm(sim_handle* h, const float* d_theta, int M, float clearance, uint8_t* d_hit, float* d_min_phi) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (!h->arm) return fail(SIM_EINVAL, "the batch has no arm");
  if (M < 0) return fail(SIM_EINVAL, "M must be >= 0");
  if (!(clearance >= 0.f) || !std::isfinite(clearance)) return fail(SIM_EINVAL, "clearance must be finite and >= 0");
  if (M == 0) return SIM_OK;
  if (!d_theta || !d_hit) return fail(SIM_EINVAL, "NULL pointer");
  if (!aligned(d_theta, 4) || (d_min_phi && !aligned(d_min_phi, 4))) return fail(SIM_EINVAL, "misaligned array");
  int nb_max = 0;
  for (int s = 0; s < h->S; s++) nb_max = std::max(nb_max, h->body_offset[s + 1] - h->body_offset[s]);
  const rbs::StepParams P = params(h);
  const int rc = rbs_launch_query(h->S, nb_max, h->N, P.body_offset, P.shape, P.prm, P.pose, P.arm_base,
                                  h->link_len, d_theta, M, clearance, d_hit, d_min_phi, P.hull_info, P.hull_vert,
                                  P.hull_plane, P.hull_loop, P.hull_edge, P.hull_ext, h->stream);
  if (rc == -2) return fail(SIM_EINVAL, "too many scenes x configuration blocks for one launch");
  if (rc != 0) return fail(SIM_EDEVICE, std::string("query launch failed: ") + hipGetErrorString((hipError_t)rc));
  return SIM_OK;
}

int sim_contacts(const sim_handle* hc, sim_contact_view* out) {
  if (!hc || !out) return fail(SIM_EINVAL, "NULL argument");
  sim_handle* h = const_cast<sim_handle*>(hc);
  const Layout& L = h->lay;
  int last = h->parity;  // the buffer the last step wrote is the one the next reads
  out->max_contacts = h->CM;
  out->max_pairs = h->PM;
  out->count = at<int32_t>(h, L.off_ccount[last]);
  out->key = at<uint32_t>(h, L.off_ckey[last]);
  out->normal = at<float>(h, L.off_x_normal);
  out->point = at<float>(h, L.off_x_point);
  out->phi = at<float>(h, L.off_x_phi);
  out->lambda = at<float>(h, L.off_x_lambda);
  out->colour = at<int32_t>(h, L.off_x_colour);
  out->features = at<float>(h, L.off_x_feat);
  out->n_pairs = at<int32_t>(h, L.off_st[0]);
  out->pair_key = at<uint32_t>(h, L.off_x_pair);
  return SIM_OK;
}

int sim_state(const sim_handle* hc, sim_state_view* out) {
  if (!hc || !out) return fail(SIM_EINVAL, "NULL argument");
  sim_handle* h = const_cast<sim_handle*>(hc);
  const Layout& L = h->lay;
  out->n_bodies = h->N;
  out->pose = at<float>(h, L.off_pose);
  out->vel = at<float>(h, L.off_vel);
  out->rest = at<int32_t>(h, L.off_rest);
  out->theta = h->arm ? at<float>(h, L.off_theta) : nullptr;
  out->arm_state = h->arm == 2 ? at<float>(h, L.off_arm_state) : nullptr;
  out->joint_state = h->parts ? at<float>(h, L.off_joint_state) : nullptr;
  out->cache_cap = h->CM;
  out->cache_count = at<int32_t>(h, L.off_ccount[h->parity]);
  out->cache_key = at<uint32_t>(h, L.off_ckey[h->parity]);
  out->cache_lam = at<float>(h, L.off_clam[h->parity]);
  return SIM_OK;
}

int sim_stats(const sim_handle* hc, sim_stats_view* out) {
  if (!hc || !out) return fail(SIM_EINVAL, "NULL argument");
  sim_handle* h = const_cast<sim_handle*>(hc);
  const Layout& L = h->lay;
  out->pairs = at<int32_t>(h, L.off_st[0]);
  out->contacts = at<int32_t>(h, L.off_st[1]);
  out->colours = at<int32_t>(h, L.off_st[2]);
  out->sweeps = at<int32_t>(h, L.off_st[3]);
  out->flags = at<int32_t>(h, L.off_st[4]);
  out->residual = at<float>(h, L.off_st[5]);
  out->arm_force = at<float>(h, L.off_st[6]);
  return SIM_OK;
}

int sim_set_export(sim_handle* h, int on) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  h->export_on = on ? 1 : 0;
  return SIM_OK;
}

int sim_set_motors(sim_handle* h, float kp, float max_impulse) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (h->arm != 2) return fail(SIM_EINVAL, "the batch has no articulated arm");
  if (!(kp >= 0.f && kp <= 1.f)) return fail(SIM_EINVAL, "motor gain must be in [0, 1]");
  if (!(max_impulse >= 0.f) || !std::isfinite(max_impulse)) return fail(SIM_EINVAL, "motor impulse bound must be >= 0");
  h->motor_kp = kp;
  h->motor_max = max_impulse;
  return SIM_OK;
}

int sim_set_solver(sim_handle* h, int solver, int warm_start, float tolerance) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (solver != SIM_PGS && solver != SIM_JACOBI) return fail(SIM_EINVAL, "bad solver");
  if (warm_start < SIM_COLD || warm_start > SIM_LEARNED) return fail(SIM_EINVAL, "bad warm start");
  if (!(tolerance >= 0.f)) return fail(SIM_EINVAL, "tolerance must be >= 0");
  if (warm_start == SIM_LEARNED && h->sleep_speed > 0.f)
    return fail(SIM_EINVAL, "the learned warm start is not available with sleeping islands");
  if (h->arm == 2 && (solver != SIM_PGS || warm_start == SIM_LEARNED))
    return fail(SIM_EINVAL, "the articulated arm needs the PGS solver without the learned warm start");
  if (h->parts && (solver != SIM_PGS || warm_start == SIM_LEARNED))
    return fail(SIM_EINVAL, "container parts need the PGS solver without the learned warm start");
  if (h->n_hulls > 0 && warm_start == SIM_LEARNED)
    return fail(SIM_EINVAL, "convex hulls are not available with the learned warm start");
  const int old_solver = h->solver, old_warm = h->warm;
  h->solver = solver;
  h->warm = warm_start;
  if (h->persistent && (solver != old_solver || warm_start != old_warm)) {
    // the working sets change size: route the scenes again
    int rc = build_queues(h, h->wave_max_bodies, h->wave_by_table, h->wave_buckets);
    if (rc != SIM_OK) {
      h->solver = old_solver;
      h->warm = old_warm;
      build_queues(h, h->wave_max_bodies, h->wave_by_table, h->wave_buckets);
      return rc;
    }
  }
  h->tol = tolerance;
  return SIM_OK;
}

int sim_set_mlp(sim_handle* h, const uint16_t* w1, const uint16_t* w2, const uint16_t* w3, const float* b1,
                const float* b2, const float* b3, const float* mean, const float* stdv) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (!w1 || !w2 || !w3 || !b1 || !b2 || !b3 || !mean || !stdv) return fail(SIM_EINVAL, "NULL weight pointer");
  if (!aligned(w1, 8) || !aligned(w2, 8) || !aligned(w3, 8)) return fail(SIM_EINVAL, "bf16 weights must be 8-byte aligned");
  h->mlp.w1 = w1;
  h->mlp.w2 = w2;
  h->mlp.w3 = w3;
  h->mlp.b1 = b1;
  h->mlp.b2 = b2;
  h->mlp.b3 = b3;
  h->mlp.mean = mean;
  h->mlp.stdv = stdv;
  h->mlp_set = true;
  return SIM_OK;
}

int sim_reset(sim_handle* h, const uint8_t* d_mask, const sim_reset_pool* pool) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (!d_mask || !pool || !pool->pose || !pool->vel) return fail(SIM_EINVAL, "mask, pool, pose and vel are required");
  if (pool->size < 1) return fail(SIM_EINVAL, "pool size must be >= 1");
  if (h->arm && !pool->theta) return fail(SIM_EINVAL, "arm scenes need theta");
  if (h->parts && !pool->joint_state) return fail(SIM_EINVAL, "container parts need joint_state");
  rbs::StepParams P = params(h);
  int rc = rbs_launch_reset(&P, d_mask, pool->size, pool->index, pool->pose, pool->vel, h->arm ? pool->theta : nullptr,
                            h->parts ? pool->joint_state : nullptr, at<int32_t>(h, h->lay.off_ccount[0]),
                            at<int32_t>(h, h->lay.off_ccount[1]), h->stream);
  if (rc == 0 && h->arm) rc = rbs_launch_arm_pose(&P, d_mask, h->stream);
  if (rc != 0) return fail(SIM_EDEVICE, "reset launch failed");
  return SIM_OK;
}

int sim_set_sleep(sim_handle* h, float speed, int steps) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (!(speed >= 0.f) || !std::isfinite(speed)) return fail(SIM_EINVAL, "speed must be finite and >= 0");
  if (speed > 0.f && steps < 1) return fail(SIM_EINVAL, "steps must be >= 1");
  if (speed > 0.f && h->warm == SIM_LEARNED)
    return fail(SIM_EINVAL, "sleeping islands are not available with the learned warm start");
  h->sleep_speed = speed;
  h->sleep_steps = speed > 0.f ? steps : 0;
  return SIM_OK;
}

int sim_set_trace(sim_handle* h, uint64_t* d_trace) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  h->trace = d_trace;
  return SIM_OK;
}

int sim_set_stream(sim_handle* h, void* stream) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  h->stream = (hipStream_t)stream;
  return SIM_OK;
}

void sim_destroy(sim_handle* h) { delete h; }

int sim_set_persistent(sim_handle* h, int on, int wave_max_bodies) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (!on) {
    h->persistent = false;
    return SIM_OK;
  }
  int rc = build_queues(h, wave_max_bodies < 0 ? rbs::kMaxBodiesPerScene : wave_max_bodies);
  if (rc != SIM_OK) return rc;
  h->persistent = true;
  return SIM_OK;
}

int sim_set_persistent_table(sim_handle* h, uint32_t wave_buckets) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (wave_buckets >> kBuckets) return fail(SIM_EINVAL, "bucket bits beyond the table");
  int rc = build_queues(h, 0, true, wave_buckets);
  if (rc != SIM_OK) return rc;
  h->persistent = true;
  return SIM_OK;
}

size_t sim_autotune_scratch_bytes(const sim_handle* h) { return h ? state_bytes(h) : 0; }

size_t sim_state_bytes(const sim_handle* h) { return h ? state_bytes(h) + 256 : 0; }

// Blob: 256-byte header (cache parity, scene and body counts) then the state
// spans in workspace order.
int sim_save_state(sim_handle* h, void* d_blob) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (!d_blob || ((uintptr_t)d_blob & 255u)) return fail(SIM_EINVAL, "blob must be 256-byte aligned device memory");
  static thread_local int32_t hdr[4];
  hdr[0] = h->parity;
  hdr[1] = h->S;
  hdr[2] = (int32_t)h->N;
  hdr[3] = h->CM;
  if (hipMemcpyAsync(d_blob, hdr, sizeof(hdr), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return fail(SIM_EDEVICE, "state header copy failed");
  if (copy_state(h, static_cast<char*>(d_blob) + 256, true) != 0) return fail(SIM_EDEVICE, "state copy failed");
  return SIM_OK;
}

int sim_load_state(sim_handle* h, const void* d_blob) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (!d_blob || ((uintptr_t)d_blob & 255u)) return fail(SIM_EINVAL, "blob must be 256-byte aligned device memory");
  int32_t hdr[4];
  if (hipMemcpyAsync(hdr, d_blob, sizeof(hdr), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess)
    return fail(SIM_EDEVICE, "state header copy failed");
  if (hdr[1] != h->S || hdr[2] != (int32_t)h->N || hdr[3] != h->CM || (hdr[0] != 0 && hdr[0] != 1))
    return fail(SIM_EINVAL, "blob was saved from a different batch layout");
  if (copy_state(h, const_cast<char*>(static_cast<const char*>(d_blob)) + 256, false) != 0)
    return fail(SIM_EDEVICE, "state copy failed");
  h->parity = hdr[0];
  return SIM_OK;
}

int sim_autotune(sim_handle* h, void* d_scratch, size_t scratch_bytes, int steps, float dt, int iters,
                 uint32_t* out_wave_buckets) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (steps < 1 || !(dt > 0.f) || iters < 1) return fail(SIM_EINVAL, "steps, dt and iters must be positive");
  if (!d_scratch || scratch_bytes < state_bytes(h) || ((uintptr_t)d_scratch & 255u))
    return fail(SIM_EWORKSPACE, "scratch too small or not 256-byte aligned");
  if (h->warm == SIM_LEARNED && !h->mlp_set) return fail(SIM_EINVAL, "learned warm start needs sim_set_mlp");
  // body-count buckets present in the batch (scenes stepped out of global
  // memory are not in the queues)
  std::vector<char> in_hbm(h->S, 0);
  for (int s : h->hbm) in_hbm[s] = 1;
  uint32_t present = 0;
  for (int s = 0; s < h->S; s++)
    if (!in_hbm[s]) present |= 1u << body_bucket(h->body_offset[s + 1] - h->body_offset[s]);
  const bool was_persistent = h->persistent, was_table = h->wave_by_table;
  const int was_threshold = h->wave_max_bodies, parity0 = h->parity;
  const uint32_t was_buckets = h->wave_buckets;
  char* scratch = static_cast<char*>(d_scratch);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return fail(SIM_EDEVICE, "event creation failed");
  }
  int rc = SIM_OK;
  if (copy_state(h, scratch, true) != 0) rc = fail(SIM_EDEVICE, "state save failed");
  // times `steps` steps of one routing (after an untimed step that captures
  // the graph) and restores the state
  auto trial = [&](uint32_t mask, float* ms) -> int {
    int r = build_queues(h, 0, true, mask);
    if (r != SIM_OK) return r;
    h->persistent = true;
    for (int it = 0; it <= steps && r == SIM_OK; it++) {
      if (it == 1 && hipEventRecord(e0, h->stream) != hipSuccess) r = fail(SIM_EDEVICE, "event record failed");
      if (r == SIM_OK) r = sim_step(h, nullptr, dt, iters);
    }
    if (r == SIM_OK && (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(ms, e0, e1) != hipSuccess))
      r = fail(SIM_EDEVICE, "timing failed");
    if (r == SIM_OK && copy_state(h, scratch, false) != 0) r = fail(SIM_EDEVICE, "state restore failed");
    h->parity = parity0;
    return r;
  };
  // greedy over the buckets in ascending size: a bucket's scenes go to single
  // waves if that makes the batch's step faster
  uint32_t best = 0;
  float best_ms = 0.f;
  if (rc == SIM_OK) rc = trial(0u, &best_ms);
  for (int k = 0; k < kBuckets && rc == SIM_OK; k++) {
    if (!((present >> k) & 1u)) continue;
    const uint32_t mask = best | (1u << k);
    float ms = 0.f;
    rc = trial(mask, &ms);
    if (rc == SIM_OK && h->n_wave > 0 && ms < best_ms) {
      best = mask;
      best_ms = ms;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc == SIM_OK) hipStreamSynchronize(h->stream);
  if (rc != SIM_OK) {
    h->persistent = was_persistent;
    if (was_persistent) build_queues(h, was_threshold, was_table, was_buckets);
    return rc;
  }
  rc = build_queues(h, 0, true, best);
  if (rc != SIM_OK) return rc;
  h->persistent = true;
  if (out_wave_buckets) *out_wave_buckets = best;
  return SIM_OK;
}

int sim_mlp_forward(const sim_mlp_weights* w, const float* d_x, long n, float* d_y, void* stream) {
  if (!w || !w->w1 || !w->w2 || !w->w3 || !w->b1 || !w->b2 || !w->b3 || !w->mean || !w->std)
    return fail(SIM_EINVAL, "NULL weight pointer");
  if (n < 0) return fail(SIM_EINVAL, "n must be >= 0");
  if (n > 0 && (!d_x || !d_y)) return fail(SIM_EINVAL, "x and y are required");
  if (!aligned(w->w1, 8) || !aligned(w->w2, 8) || !aligned(w->w3, 8) || !aligned(d_x, 16))
    return fail(SIM_EINVAL, "bf16 weights need 8-byte and x 16-byte alignment");
  rbs::MlpParams M{w->w1, w->w2, w->w3, w->b1, w->b2, w->b3, w->mean, w->std};
  if (rbs_mlp_forward(&M, d_x, n, d_y, (hipStream_t)stream) != 0) return fail(SIM_EDEVICE, "forward launch failed");
  return SIM_OK;
}

size_t sim_mlp_workspace_bytes(long n) { return n < 0 ? 0 : rbs_mlp_work_bytes(n); }

int sim_mlp_stats(const float* d_x, long n, float* d_mean, float* d_std, void* d_work, size_t work_bytes,
                  void* stream) {
  if (n < 1) return fail(SIM_EINVAL, "n must be >= 1");
  if (!d_x || !d_mean || !d_std) return fail(SIM_EINVAL, "NULL pointer");
  if (!d_work || work_bytes < rbs_mlp_work_bytes(n) || !aligned(d_work, 256))
    return fail(SIM_EWORKSPACE, "workspace too small or not 256-byte aligned");
  if (rbs_mlp_stats(d_x, n, d_mean, d_std, d_work, (hipStream_t)stream) != 0)
    return fail(SIM_EDEVICE, "stats launch failed");
  return SIM_OK;
}

int sim_mlp_grad(const float* d_params, const float* d_mean, const float* d_std, const float* d_x, const float* d_t,
                 const int32_t* d_rows, long n, float* d_grad, float* d_loss, void* d_work, size_t work_bytes,
                 void* stream) {
  if (n < 1) return fail(SIM_EINVAL, "n must be >= 1");
  if (n > (1L << 30)) return fail(SIM_EINVAL, "n too large");
  if (!d_params || !d_mean || !d_std || !d_x || !d_t || !d_grad) return fail(SIM_EINVAL, "NULL pointer");
  if (!d_work || work_bytes < rbs_mlp_work_bytes(n) || !aligned(d_work, 256))
    return fail(SIM_EWORKSPACE, "workspace too small or not 256-byte aligned");
  if (rbs_mlp_grad(d_params, d_mean, d_std, d_x, d_t, d_rows, n, d_grad, d_loss, d_work, (hipStream_t)stream) != 0)
    return fail(SIM_EDEVICE, "gradient launch failed");
  return SIM_OK;
}

long sim_mlp_grad_noalloc_max_rows(void) { return rbs_mlp_grad_static_max_rows(); }

int sim_mlp_grad_noalloc(const float* d_params, const float* d_mean, const float* d_std, const float* d_x,
                         const float* d_t, const int32_t* d_rows, long n, float* d_grad, float* d_loss, void* stream) {
  if (n < 1) return fail(SIM_EINVAL, "n must be >= 1");
  if (n > rbs_mlp_grad_static_max_rows())
    return fail(SIM_EINVAL, "n = " + std::to_string(n) + " exceeds the " +
                                std::to_string(rbs_mlp_grad_static_max_rows()) + " rows of the static scratch");
  if (!d_params || !d_mean || !d_std || !d_x || !d_t || !d_grad) return fail(SIM_EINVAL, "NULL pointer");
  const int rc = rbs_mlp_grad_static(d_params, d_mean, d_std, d_x, d_t, d_rows, n, d_grad, d_loss,
                                     (hipStream_t)stream);
  if (rc != 0) return fail(SIM_EDEVICE, "static scratch lookup or gradient launch failed");
  return SIM_OK;
}

int sim_mlp_adam(float* d_params, float* d_m, float* d_v, const float* d_grad, int step, float lr, float clip,
                 float* d_gnorm, void* stream) {
  if (!d_params || !d_m || !d_v || !d_grad) return fail(SIM_EINVAL, "NULL pointer");
  if (step < 1) return fail(SIM_EINVAL, "step counts from 1");
  if (!(lr >= 0.f) || !(clip >= 0.f)) return fail(SIM_EINVAL, "lr and clip must be >= 0");
  if (rbs_mlp_adam(d_params, d_m, d_v, d_grad, step, lr, clip, d_gnorm, (hipStream_t)stream) != 0)
    return fail(SIM_EDEVICE, "adam launch failed");
  return SIM_OK;
}

int sim_mlp_export(const float* d_params, uint16_t* d_wbf16, float* d_bias, void* stream) {
  if (!d_params || !d_wbf16 || !d_bias) return fail(SIM_EINVAL, "NULL pointer");
  if (rbs_mlp_export(d_params, d_wbf16, d_bias, (hipStream_t)stream) != 0)
    return fail(SIM_EDEVICE, "export launch failed");
  return SIM_OK;
}

int sim_mlp_gather(sim_handle* h, float* d_x, float* d_t, long cap, float target_clip, long long* d_total) {
  if (!h) return fail(SIM_EINVAL, "handle is NULL");
  if (!d_x || !d_t || !d_total || cap < 0) return fail(SIM_EINVAL, "bad output arguments");
  if (!(target_clip >= 0.f)) return fail(SIM_EINVAL, "target_clip must be >= 0");
  if (!(h->last_dt > 0.f) || !h->last_export) return fail(SIM_EINVAL, "gather needs a previous step with export on");
  const float gm = std::sqrt(h->gravity[0] * h->gravity[0] + h->gravity[1] * h->gravity[1] +
                             h->gravity[2] * h->gravity[2]);
  if (!(gm > 0.f)) return fail(SIM_EINVAL, "gather scales targets by |g| dt; gravity is zero");
  const Layout& L = h->lay;
  // the last step wrote its cache into the buffer the next step reads
  int rc = rbs_gather(at<int32_t>(h, L.off_ccount[h->parity]), at<int32_t>(h, L.off_st[4]), h->S, h->CM,
                      (long)h->S * h->CM, at<float>(h, L.off_x_feat), at<float>(h, L.off_x_lambda),
                      1.0f / (gm * h->last_dt), target_clip, at<int64_t>(h, L.off_gather),
                      at<int32_t>(h, L.off_gcount), d_x, d_t, cap, d_total, h->stream);
  if (rc != 0) return fail(SIM_EDEVICE, "gather launch failed");
  return SIM_OK;
}

const char* sim_last_error(void) { return g_err.c_str(); }

}  // extern "C"

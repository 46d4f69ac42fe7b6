/*
 * rbsim.h -- C ABI of the MI355X batched rigid-body step (librbsim.so).
 *
 * The library advances a batch of independent rearrangement scenes by one
 * physics step per call: the physics-engine transition (s_t, a_t) -> s_{t+1}
 * of the paper's simulator definition (Habitat 2.0, Sec. 2 "What is a
 * simulator?"), for rigid objects with mass, friction and restitution and
 * simplified collision proxies (Sec. 3, asset creation; Sec. 4.3 "simplify
 * and reuse"), base-constrained parts treated as static (Sec. 4.1) and an
 * arm moved kinematically by the agent's action (Sec. 5, 7-DoF arm), at
 * 1/120 s per step (Sec. 4.4).  The per-step arm collision force in newtons
 * is the quantity the Pick task consumes (Sec. 5; appendix, Pick reward).
 * The paper gives no engine algorithm; the step is sort-and-sweep
 * broadphase, sphere/box/capsule narrowphase, graph-coloured projected
 * Gauss-Seidel (or Jacobi) contact and friction impulses, and semi-implicit
 * Euler integration, all in hand-written HIP for gfx950.
 *
 * Memory.  The caller owns every buffer.  All device memory the library
 * touches lives in one caller-allocated workspace (sim_workspace_bytes);
 * the library never allocates device memory.  Host arrays in the
 * descriptor are read during sim_create only.
 *
 * Streams.  All work is enqueued on the stream given at creation (may be
 * changed with sim_set_stream).  Only sim_create synchronises that stream.
 *
 * Errors.  Functions return SIM_OK (0) or a negative code and leave the
 * simulation unchanged; sim_last_error() returns a thread-local message.
 * Per-scene soft faults are not return codes but bits in the stats flags
 * (SIM_FLAG_*); a scene with NONFINITE or CAPACITY is undefined until reset.
 *
 * Threading.  One handle per host thread; handles are independent.
 */
#ifndef RBSIM_H
#define RBSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_ABI_VERSION 6

enum { SIM_OK = 0, SIM_EINVAL = -1, SIM_EDEVICE = -2, SIM_EWORKSPACE = -3, SIM_EABI = -4, SIM_ECAPACITY = -5 };
enum { SIM_SPHERE = 0, SIM_BOX = 1, SIM_CAPSULE = 2, SIM_HULL = 3 };
enum { SIM_DYNAMIC = 0, SIM_STATIC = 1, SIM_KINEMATIC = 2 };
enum { SIM_COLD = 0, SIM_PREV = 1, SIM_LEARNED = 2 };
enum { SIM_PGS = 0, SIM_JACOBI = 1 };
enum { SIM_FLAG_NONFINITE = 1, SIM_FLAG_CAPACITY = 2, SIM_FLAG_NOT_CONVERGED = 4, SIM_FLAG_FELLBACK = 8,
       SIM_FLAG_BAD_RESET = 16 };

/* Batch descriptor.  N = body_offset[num_scenes] bodies in total; scene s
 * owns bodies [body_offset[s], body_offset[s+1]), at most 2046 bodies.  All
 * h_* pointers are host memory read during sim_create. */
typedef struct sim_batch_desc {
    int abi_version;             /* SIM_ABI_VERSION */
    int num_scenes;              /* S >= 1 */
    const int32_t *h_body_offset;/* [S+1], non-decreasing, body_offset[0] = 0 */
    const uint8_t *h_shape;      /* [N] SIM_SPHERE / SIM_BOX / SIM_CAPSULE */
    const uint8_t *h_motion;     /* [N] SIM_DYNAMIC / SIM_STATIC / SIM_KINEMATIC */
    const float *h_param;        /* [N*3] sphere (r,-,-); box half-extents; capsule (r, half-length, -), m;
                                    hull (index in the hull library, -, -) */
    const float *h_mass;         /* [N] kg, > 0 for dynamic bodies */
    const float *h_friction;     /* [N] */
    const float *h_restitution;  /* [N] */
    const float *h_pose;         /* [N*7] x y z (m), quaternion w x y z (body to world) */
    const float *h_vel;          /* [N*6] linear (m/s), angular (rad/s, world frame) */
    int arm;                     /* 1: the last 7 bodies of every scene are the arm links
                                    (kinematic capsules); their poses follow the joint angles.
                                    2: the same links as dynamic capsules (h_mass their masses)
                                    of one articulated body in reduced coordinates (Sec. 1:
                                    articulated robots; Sec. 5: joint motors under PD position
                                    control): the state is the joint angles and rates, link
                                    poses and velocities follow them, contacts on the links act
                                    on the joint rates through the link Jacobians, and motor k
                                    drives rate k towards Kp (target_k - theta_k) / dt with at
                                    most the motor impulse bound per step (sim_set_motors;
                                    Kp 0.3 and 10 N s by default).  Needs the PGS solver
                                    without the learned warm start.  Initial link poses follow
                                    h_arm_theta, at rest, motor targets at h_arm_theta. */
    const float *h_arm_base;     /* [S*3] arm base position (m), or NULL when arm = 0 */
    const float *h_arm_theta;    /* [S*7] initial joint angles (rad), or NULL when arm = 0 */
    float link_len[7];           /* arm link lengths (m) */
    float arm_radius;            /* arm capsule radius (m) */
    float gravity[3];            /* m/s^2, z up */
    float margin;                /* AABB fattening and contact keep distance (m) */
    float baumgarte;             /* penetration correction factor per step */
    float slop;                  /* allowed penetration (m) */
    float rest_thresh;           /* approach speed above which restitution applies (m/s) */
    float ground_friction;       /* friction of the plane z = 0 */
    float ground_restitution;
    int max_pairs;               /* per-scene capacity of broadphase pairs (a scene of n
                                    bodies holds at most min(max_pairs, max(64, 6 n))) */
    int max_contacts;            /* per-scene capacity of contacts (same rule) */
    int solver;                  /* SIM_PGS or SIM_JACOBI */
    int warm_start;              /* SIM_COLD, SIM_PREV or SIM_LEARNED */
    float tolerance;             /* > 0: stop sweeps once the residual (m/s) <= tolerance;
                                    0: always run the requested sweeps */
    int threads;                 /* threads per scene workgroup: 64, 128, 192 or 256 (0: 128) */
    void *stream;                /* hipStream_t for all work; NULL = default stream */
    int hbm_min_bodies;          /* 0: a scene keeps its step's working set in LDS when it fits
                                    a workgroup's LDS in every solver mode, else in global memory
                                    (HBM, through the caches); > 0: also every scene of at least
                                    this many bodies uses global memory.  Results do not depend
                                    on where the working set lives. */
    /* Articulated container parts (Sec. 3: doors and drawers of the
     * furniture turn about an axis or slide): NULL h_joint for none.  A part
     * is a dynamic body with one degree of freedom relative to the world,
     * its coordinate q (0 at the initial pose) and rate qd the state
     * (sim_state_view.joint_state): revolute (1) about the line through the
     * anchor along the axis, q in rad, or prismatic (2) along the axis, q in
     * m; q is held within [lower, upper] by limit rows solved after the
     * contacts in every sweep; gravity and contacts act on it through the
     * joint.  A part never collides with the body it is joined to (its
     * parent: the cabinet that carries the door).  At most 16 parts per
     * scene; not arm links.  Needs the PGS solver without the learned warm
     * start.  Parts start at rest (q = 0, qd = 0; h_vel is not read for them)
     * and never sleep. */
    const uint8_t *h_joint;        /* [N] 0 none, 1 revolute, 2 prismatic (only dynamic bodies) */
    const float *h_joint_axis;     /* [N*3] unit axis (world, at the initial pose) */
    const float *h_joint_anchor;   /* [N*3] a point of the hinge line (world, m; read for revolute) */
    const float *h_joint_limits;   /* [N*2] lower <= upper limit of q */
    const int32_t *h_joint_parent; /* [N] local index (within the scene) of the parent body, or -1 */
    /* Convex hulls (shape SIM_HULL; convex collision proxies, Sec. 3 and
     * Sec. 4.3): a library of convex polyhedra that hull bodies index.  A
     * hull's vertices are in its body frame, which must have its origin at
     * the centre of mass of the solid (uniform density) and its axes along
     * the principal axes of inertia (checked: SIM_EINVAL otherwise); faces
     * are vertex loops counter-clockwise seen from outside, 3 to 8 vertices,
     * -1 after the last; every vertex on or inside every face plane; at
     * most 32 vertices and 32 faces a hull.  Contacts with hulls: against
     * the ground (vertices), spheres (closest point), capsules and boxes
     * and other hulls (separating axes and face clipping); arm queries
     * test the links against hulls too.  Batches with hulls step without
     * the learned warm start. */
    int n_hulls;                   /* H (0: none) */
    const int32_t *h_hull_index;   /* [H*4]: first vertex, vertex count, first face, face count */
    const float *h_hull_vert;      /* [V*3] m */
    const int32_t *h_hull_face;    /* [F*8] */
} sim_batch_desc;

typedef struct sim_handle sim_handle;

/* Device pointers of the simulation state (structure of arrays, plane
 * stride N unless stated).  Valid until sim_destroy; the caller may read
 * and write them between steps on the handle's stream. */
typedef struct sim_state_view {
    long n_bodies;        /* N */
    float *pose;          /* [7][N]: x, y, z, qw, qx, qy, qz */
    float *vel;           /* [6][N]: vx, vy, vz, wx, wy, wz */
    int32_t *rest;        /* [N] steps each dynamic body has ended at rest (sleeping islands) */
    float *theta;         /* [S][7] arm joint angles, or NULL */
    float *arm_state;     /* articulated arm only (else NULL): [S][21] per scene the joint rates
                             (rad/s), the motor targets (rad) and the last step's motor impulses
                             (N m s, the motors' warm start), 7 each */
    float *joint_state;   /* container parts only (else NULL): [2][N] joint coordinate q and
                             rate qd of every part (0 for the other bodies); a caller that
                             writes q must move the part's pose to match */
    int cache_cap;        /* per-scene contact capacity (= max_contacts) */
    int32_t *cache_count; /* [S] contacts stored for the next step's warm start */
    uint32_t *cache_key;  /* [S][cache_cap] sorted contact keys */
    float *cache_lam;     /* [4][S*cache_cap]: normal impulse, world friction impulse x y z (N s) */
} sim_state_view;

/* Device pointers of the last step's contacts.  Contact q of scene s is at
 * index s*max_contacts + q, q < count[s]; arrays with a leading [k] are
 * planes of stride S*max_contacts.  Keys: (a << 20) | (b << 8) | feature,
 * b = 0xFFF for the ground; pairs: (a << 16) | b, b = 0xFFFF for the ground.
 * Normals point from body b to body a.  Filled only when export is on
 * (sim_set_export), except count and key which are always written. */
typedef struct sim_contact_view {
    int max_contacts, max_pairs;
    const int32_t *count;     /* [S] */
    const uint32_t *key;      /* [S*max_contacts] canonical (sorted) order */
    const float *normal;      /* [3][S*max_contacts] */
    const float *point;       /* [3][S*max_contacts] */
    const float *phi;         /* [S*max_contacts] signed separation (m) */
    const float *lambda;      /* [3][S*max_contacts] normal, tangent-1, tangent-2 impulses (N s) */
    const int32_t *colour;    /* [S*max_contacts]; -1 for a contact of sleeping bodies */
    const float *features;    /* [16][S*max_contacts] warm-start features */
    const int32_t *n_pairs;   /* [S] */
    const uint32_t *pair_key; /* [S*max_pairs] */
} sim_contact_view;

/* Per-scene statistics of the last step, device arrays of length S.
 * Flags: NOT_CONVERGED when the tolerance was set and the last sweep's
 * residual is above it (the step is not solved, whatever its start);
 * FELLBACK when the network's start impulses were rejected before the
 * sweeps (they raised the solver's objective) and the new contacts started
 * from zero. */
typedef struct sim_stats_view {
    const int32_t *pairs, *contacts, *colours, *sweeps, *flags;
    const float *residual;    /* last sweep's max |dlambda| * k (m/s) */
    const float *arm_force;   /* sum over arm contacts of |impulse| / dt (N) */
} sim_stats_view;

/* Bytes of device workspace the descriptor needs (0 on a bad descriptor):
 * the state, contact caches and step buffers of all the batch's scenes,
 * the many environments stepped in parallel of Sec. 4.4. */
size_t sim_workspace_bytes(const sim_batch_desc *desc);

/* The initial state s_0 of every scene (Sec. 2, the simulator's state;
 * rigid objects with mass, friction and restitution and simplified
 * collision proxies, Sec. 3 and Sec. 4.3; static parts, Sec. 4.1; the arm,
 * Sec. 5).  Validates the descriptor (SIM_EINVAL, SIM_EABI, SIM_ECAPACITY
 * when a scene's working set does not fit the device), lays out the
 * workspace (>= sim_workspace_bytes, 256-byte aligned device memory owned by
 * the caller; SIM_EWORKSPACE otherwise), uploads the initial state on
 * desc->stream and synchronises it.  *out receives the handle, which owns
 * host metadata only. */
int sim_create(const sim_batch_desc *desc, void *d_workspace, size_t workspace_bytes, sim_handle **out);

/* One transition (s_t, a_t) -> s_{t+1} of every scene (Sec. 2), a physics
 * step of dt (1/120 s in Sec. 4.4): d_actions [S*7] arm joint velocities
 * (rad/s; the agent's arm action of Sec. 5; with the articulated arm the
 * rates of the motor targets, which move by dt times them before the
 * step's motors aim at them), device memory, or NULL (zero);
 * dt > 0 seconds; iters >= 1 sweeps (the cap when a tolerance is set).
 * SIM_EINVAL on bad arguments (nothing launched).  Asynchronous on the
 * handle's stream; per-scene soft faults go to the stats flags. */
int sim_step(sim_handle *h, const float *d_actions, float dt, int iters);

/* Collision checks of candidate arm configurations, the test a sampling
 * motion planner runs at every configuration it visits (Sec. 4.5 and
 * App. C: the planner checks the arm against the scene at fine joint-space
 * steps): for each scene s and configuration j, the arm links placed by the
 * forward kinematics of d_theta[(s*M + j)*7 .. +7] (rad, device float32
 * [S][M][7]) are tested against every body of scene s that is not an arm
 * link, at its current pose, and against the ground plane; the arm itself
 * is left out.  d_hit[s*M + j] (device uint8 [S][M]) = 1 iff some link has a
 * contact with signed separation <= clearance (m, finite, >= 0);
 * d_min_phi (device float32 [S][M], or NULL) gets the least separation of
 * those contacts, +INF when none is within the clearance.  The scenes'
 * state is read, not changed; no solver runs.  SIM_EINVAL for a batch
 * without the arm, M < 0, a bad clearance or NULL/misaligned arrays
 * (nothing launched); M = 0 does nothing.  Asynchronous on the handle's
 * stream, after any step enqueued before it. */
int sim_query_arm(sim_handle *h, const float *d_theta, int M, float clearance, uint8_t *d_hit, float *d_min_phi);

/* Contact and pair views of the last step (device pointers into the
 * workspace, valid until the next step): the contacts whose impulses make
 * up the arm's collision force that the Pick task reads (Sec. 5; appendix,
 * Pick reward). */
int sim_contacts(const sim_handle *h, sim_contact_view *out);

/* State view (the s_t of Sec. 2: poses, velocities, joint angles and the
 * warm-start contact cache) and per-scene statistics of the last step
 * (pairs, contacts, colours, sweeps, residual, flags and the arm force of
 * Sec. 5).  Device pointers into the workspace; SIM_EINVAL on NULL. */
int sim_state(const sim_handle *h, sim_state_view *out);
int sim_stats(const sim_handle *h, sim_stats_view *out);

/* Export of normals, points, phi, impulses, colours, features and pairs on
 * (1) or off (0) for later steps (for analysis and for logging the learned
 * warm start's training rows; off in the hot loop). */
int sim_set_export(sim_handle *h, int on);

/* Change the solver settings used by later steps: SIM_PGS or SIM_JACOBI,
 * SIM_COLD / SIM_PREV / SIM_LEARNED start, residual tolerance (m/s; 0 =
 * fixed sweeps).  SIM_EINVAL on a bad value or on Jacobi or the learned
 * start with an articulated arm or container parts, SIM_ECAPACITY if a scene
 * no longer fits the persistent launch's LDS (settings unchanged). */
int sim_set_solver(sim_handle *h, int solver, int warm_start, float tolerance);

/* Sleeping islands for later steps (localized physics, Sec. 4.1: the robot
 * is the only source of forces besides gravity, and the engine's sleeping
 * state spares settled objects): speed > 0 (m/s) turns them on, 0 off.  An
 * island (dynamic bodies joined by the step's contacts between two dynamic
 * bodies) sleeps when every body in it has ended at least `steps` steps at
 * rest (speed and surface speed |w| r, r the body's bounding radius, both at
 * most `speed`; sim_state_view.rest counts them) and none of its bodies
 * touches a kinematic body (the arm).  A sleeping body keeps its pose with
 * zero velocity; its contacts are found as usual but are not coloured or
 * solved (exported colour -1) and keep their previous impulses in the
 * cache.  The counters are part of the state (checkpoints, resets clear
 * them).  SIM_EINVAL for a negative or non-finite speed, steps < 1 with
 * speed > 0, or speed > 0 with the learned warm start (and sim_set_solver
 * refuses the learned start while sleeping is on). */
int sim_set_sleep(sim_handle *h, float speed, int steps);

/* Joint motors of the articulated arm (Sec. 5: PD position control with
 * gain Kp = 0.3 and at most 10 N s of motor impulse per step, the
 * defaults): kp in [0, 1] is the fraction of a joint's angle error its motor
 * closes per step when unloaded; max_impulse >= 0 (N m s) bounds each
 * motor's impulse in a step.  Applies from the next step.  SIM_EINVAL
 * without an articulated arm (arm 2) or for a value out of range. */
int sim_set_motors(sim_handle *h, float kp, float max_impulse);

/* Learned warm start weights (this library's addition; the paper has no
 * learned solver), device memory read during every later step in
 * SIM_LEARNED mode: bf16 w1 [64*16], w2 [64*64], w3 [3*64] (row = output),
 * fp32 b1 [64], b2 [64], b3 [3], feature mean [16] and std [16].  The
 * pointers must stay valid while used. */
int sim_set_mlp(sim_handle *h, const uint16_t *d_w1, const uint16_t *d_w2, const uint16_t *d_w3,
                const float *d_b1, const float *d_b2, const float *d_b3, const float *d_mean, const float *d_std);

/* ---- Learned warm start: the network outside the step ------------------
 * The warm-start network maps 16 contact features (z-scored with a
 * training-set mean and std, std floored at 1e-6) through 64 -> ReLU -> 64
 * -> ReLU -> 3 outputs y.  Features, world frame, SI units: 0-2 relative
 * velocity along n, t1, t2; 3 depth -phi; 4-5 inverse masses of A and B;
 * 6-7 (r x n) . I^-1 (r x n) of A and B; 8-10 previous impulses along n,
 * t1, t2 in units of |g| dt / k_n; 11-13 the normal n; 14 friction
 * coefficient; 15 for a new contact 1 / max(n_A, n_B) (n_X: contacts
 * touching dynamic body X), 0 for a persisting one.  In SIM_LEARNED mode a contact that persists
 * from the previous step starts from its previous impulse (the classic warm
 * start, Catto 2005) and a new contact from y |g| dt / k_n, in units of the
 * impulse that cancels one step of gravity along the normal (features 8-10
 * are the previous impulses in the same units); starts are projected onto
 * the friction cone.  Before any sweep the solver scores the network's part
 * on its quadratic objective f(l) = 1/2 l^T A l + l^T (u_free - b) (rows:
 * normal with target velocity b = bias, two friction rows with b = 0): if
 * adding the new contacts' impulses raises f, they are dropped (the new
 * contacts start from zero as in SIM_PREV) and SIM_FLAG_FELLBACK is set.  The paper has no learned
 * solver: the network is this library's addition to the classic warm start.  Its z-scoring echoes the per-channel input normalization of
 * the appendix's monolithic policy (App. B.1), and the optimizer defaults
 * the caller is expected to use come from that policy's training setup
 * (App. B.2: Adam, lr 1e-4 decayed linearly, gradient norm clipped at 0.5).
 * Flat fp32 parameter vector (row = output unit):
 *   w1 [64][16] | b1 [64] | w2 [64][64] | b2 [64] | w3 [3][64] | b3 [3]. */
#define SIM_MLP_NPARAM 5443
#define SIM_MLP_NWEIGHT 5312  /* bf16 weights: w1 | w2 | w3 */
#define SIM_MLP_NBIAS 131     /* fp32 biases: b1 | b2 | b3 */

/* Inference weights in the form sim_set_mlp takes (device pointers; bf16
 * arrays 8-byte aligned). */
typedef struct sim_mlp_weights {
    const uint16_t *w1, *w2, *w3;
    const float *b1, *b2, *b3, *mean, *std;
} sim_mlp_weights;

/* y [n][3] = network(x [n][16]) exactly as the step's learned warm start
 * computes it: bf16 weights and layer inputs, fp32 accumulation on the
 * matrix cores.  x 16-byte aligned.  Asynchronous on stream (a hipStream_t,
 * NULL = default stream). */
int sim_mlp_forward(const sim_mlp_weights *w, const float *d_x, long n, float *d_y, void *stream);

/* Device scratch bytes sim_mlp_stats and sim_mlp_grad need for n rows
 * (caller-owned, 256-byte aligned). */
size_t sim_mlp_workspace_bytes(long n);

/* Population mean and std of each feature of x [n][16], accumulated in
 * double in a fixed order: the network's input normalisation (per-channel,
 * as for the appendix's policy inputs, App. B.1).  SIM_EINVAL for n < 1 or
 * NULL, SIM_EWORKSPACE for a short or misaligned d_work. */
int sim_mlp_stats(const float *d_x, long n, float *d_mean, float *d_std, void *d_work, size_t work_bytes,
                  void *stream);

/* Gradient of the mean squared error over the 3n outputs of a batch of n
 * rows against targets t [.][3], with respect to the flat parameters (the
 * training half of the learned warm start; optimizer setup after App. B.2).  Row
 * j of the batch is row d_rows[j] of x [.][16] and t (d_rows: int32 [n],
 * device, each index in range; NULL = rows 0..n-1).  The forward rounds
 * weights and activations to bf16 as inference does; the backward runs in
 * fp32 through the rounded weights.  d_grad [5443]; d_loss (may be NULL)
 * gets the loss.  Bitwise reproducible. */
int sim_mlp_grad(const float *d_params, const float *d_mean, const float *d_std, const float *d_x, const float *d_t,
                 const int32_t *d_rows, long n, float *d_grad, float *d_loss, void *d_work, size_t work_bytes,
                 void *stream);

/* sim_mlp_grad without a caller workspace, for callers that cannot allocate
 * device memory (code under stream capture, tight training loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and result as
 * sim_mlp_grad, bit for bit; the per-workgroup partial sums live in a
 * library-owned static device array of 5.6 MB, one copy per device, held
 * until the process ends.  n must lie in [1, sim_mlp_grad_noalloc_max_rows()]
 * (16384): SIM_EINVAL otherwise, before any device work.  Allocates nothing
 * (its first call on a device looks the array's address up).  Every call on
 * a device shares that device's array: calls that overlap in time on one
 * device (two streams, two host threads) race and give undefined gradients;
 * calls ordered on one stream are safe.  Asynchronous on stream. */
int sim_mlp_grad_noalloc(const float *d_params, const float *d_mean, const float *d_std, const float *d_x,
                         const float *d_t, const int32_t *d_rows, long n, float *d_grad, float *d_loss,
                         void *stream);
long sim_mlp_grad_noalloc_max_rows(void);

/* One Adam step (the optimizer of App. B.2; beta1 0.9, beta2 0.999, eps
 * 1e-8, bias-corrected; step counts from 1) on the fp32 master parameters, after scaling the gradient
 * to global L2 norm <= clip (clip 0: no clipping).  d_m, d_v: [5443]
 * moments, zero before the first step.  d_gnorm (may be NULL) gets the
 * gradient norm before clipping.  The caller owns the lr schedule. */
int sim_mlp_adam(float *d_params, float *d_m, float *d_v, const float *d_grad, int step, float lr, float clip,
                 float *d_gnorm, void *stream);

/* Inference copy of the parameters for sim_set_mlp: d_wbf16 [5312] = bf16 (round to
 * nearest even) of w1 | w2 | w3, d_bias [131] = b1 | b2 | b3. */
int sim_mlp_export(const float *d_params, uint16_t *d_wbf16, float *d_bias, void *stream);

/* Training rows from the last step (which must have run with export on;
 * SIM_EINVAL otherwise), the impulses the plain solver itself converged to:
 * for every new contact (feature 15 > 0) of every scene whose flags are all
 * clear, its 16 features into d_x [cap][16] and into d_t [cap][3] the
 * network's target, its converged impulses in units of |g| dt / k_n, i.e.
 * lambda k_n / (|g| dt) (k_n from the features: w_A + w_B + the two
 * angular terms), each saturated to [-target_clip, target_clip] when
 * target_clip > 0 (the converged impulses of stacked light bodies are
 * heavy-tailed and not unique), scenes in order, contacts in canonical
 * order.  Rows past cap are dropped; *d_total (device) receives the
 * number of rows there were.  Asynchronous on the handle's stream. */
int sim_mlp_gather(sim_handle *h, float *d_x, float *d_t, long cap, float target_clip, long long *d_total);

/* Masked reset of episodes from a pre-generated pool of fresh states
 * (Sec. 4.3 prefetches and caches assets so that an episode reset does not
 * reload them; Sec. 7 names reloading on reset as a bottleneck of the
 * training loop).  The pool holds `size` = K >= 1 complete states of the
 * batch, device memory laid out like the state: pose [K][7][N], velocity
 * [K][6][N] and, for arm batches, joint angles [K][S][7] (NULL otherwise).
 * For every scene s with d_mask[s] != 0 the library copies entry
 * k = index[s] of the pool into the scene's bodies (and joint angles,
 * recomputing the arm link poses) and clears its contact cache; index is a
 * device int32 [S] (NULL: entry 0 for every scene).  A scene whose index
 * lies outside [0, K) is left unchanged and gets SIM_FLAG_BAD_RESET in its
 * stats flags (visible until the next step).  Static and kinematic bodies
 * are copied like the others.  Asynchronous on the handle's stream;
 * SIM_EINVAL on NULL mask, pool, pose or vel, size < 1, or a missing theta
 * for an arm batch or joint_state for a batch with container parts. */
typedef struct sim_reset_pool {
    int size;                 /* K */
    const float *pose;        /* [K][7][N] */
    const float *vel;         /* [K][6][N] */
    const float *theta;       /* [K][S][7] or NULL when the batch has no arm */
    const int32_t *index;     /* [S] pool entry per scene, or NULL (entry 0) */
    const float *joint_state; /* [K][2][N] container parts' q and qd, or NULL when the batch has none */
} sim_reset_pool;

int sim_reset(sim_handle *h, const uint8_t *d_mask, const sim_reset_pool *pool);

/* Phase tracing (profiling aid, no counterpart in the paper): when d_trace (device, [S][16] uint64) is non-NULL, every
 * later step writes 15 wall-clock timestamps per scene (constant-rate
 * counter) at its phase boundaries: start, bodies loaded, arm, AABBs, body
 * sort, sweep, pair sort, narrowphase, setup, contact lists, colouring
 * rounds, colour sort, warm start, sweeps, integration, outputs end; slot
 * 15 holds the shader-clock cycles spent in the solver sweeps.
 * NULL turns it off.  For profiling; adds one store per phase. */
int sim_set_trace(sim_handle *h, uint64_t *d_trace);

/* ---- Batches of uneven scene sizes ---------------------------------------
 * The paper benchmarks many environments stepped in parallel (Sec. 4.4)
 * and names their synchronisation, and reloading on episode reset, as what
 * bounds the whole loop (Sec. 7).  Scene sizes differ, so one workgroup per
 * scene sized for the largest scene wastes the LDS.
 * With on = 1 every later sim_step is one persistent launch (after a queue
 * reset) replayed from a HIP graph captured on first use and again whenever
 * the step's arguments change: each workgroup (256 threads, the device's
 * whole LDS) first steps scenes from a queue of large scenes with all its
 * threads, then each of its four waves steps scenes from a queue of small
 * scenes alone in a quarter of the LDS.  Both queues run largest first.  A
 * scene is small when it has at most wave_max_bodies bodies (< 0: no limit)
 * and its working set fits a quarter of the LDS.  Results are identical to
 * the one-workgroup-per-scene launch.  on = 0 restores that launch.
 * SIM_ECAPACITY if a scene fits no workgroup. */
int sim_set_persistent(sim_handle *h, int on, int wave_max_bodies);

/* ---- Checkpoint and resume ----------------------------------------------
 * The state s_t of Sec. 2 as a blob, for resuming a batch: it holds what
 * later steps depend on: pose, velocity, joint
 * angles and both contact caches (the warm-start impulses), with a header
 * naming the batch layout.  sim_save_state copies the state into d_blob
 * (device memory, 256-byte aligned, sim_state_bytes long); sim_load_state
 * restores it into a handle created from the same batch layout (SIM_EINVAL
 * otherwise).  Both synchronise the handle's stream for the header; the
 * bulk copies are queued on it. */
size_t sim_state_bytes(const sim_handle *h);
int sim_save_state(sim_handle *h, void *d_blob);
int sim_load_state(sim_handle *h, const void *d_blob);

/* Device scratch (256-byte aligned) sim_autotune needs to save and restore
 * the simulation state: pose, velocity, joint angles and contact caches
 * (0 for a NULL handle). */
size_t sim_autotune_scratch_bytes(const sim_handle *h);

/* Routing table of the persistent launch: bit k of wave_buckets sends the
 * scenes of body-count bucket k to single-wave teams (four scenes per
 * workgroup), the others to whole-workgroup teams; buckets are [1, 16],
 * (16, 32], (32, 64], ..., (512, 1024], (1024, 2046] bodies (k = 0..7).  A
 * scene whose working set does not fit a quarter of the LDS stays with a
 * whole workgroup whatever the table says.  Turns the persistent launch on.
 * The table is what sim_autotune chooses and may be stored and applied to a
 * later batch of the same workload.  SIM_EINVAL for bits beyond bucket 7,
 * SIM_ECAPACITY if a scene fits no workgroup.  Results do not depend on it. */
int sim_set_persistent_table(sim_handle *h, uint32_t wave_buckets);

/* Autotuning of the persistent launch over the batch's own scenes (the
 * parallel environments of Sec. 4.4, whose synchronisation Sec. 7 names as
 * the loop's bound): the routing table, bucket by bucket in ascending body
 * count, each bucket's scenes moved to single waves if that makes `steps`
 * timed steps (zero actions, dt, iters sweeps, after an untimed one)
 * faster, the state restored after each trial; leaves the persistent
 * launch on with the table found and reports it in *out_wave_buckets (may
 * be NULL).  Synchronises the handle's stream; the last step's contact and
 * stats views then hold a trial step's values. */
int sim_autotune(sim_handle *h, void *d_scratch, size_t scratch_bytes, int steps, float dt, int iters,
                 uint32_t *out_wave_buckets);

/* The stream (hipStream_t, NULL = default) for later work of the handle. */
int sim_set_stream(sim_handle *h, void *stream);
/* Frees the handle's host metadata, graphs and capture stream (the
 * workspace stays the caller's).  NULL is ignored. */
void sim_destroy(sim_handle *h);
/* Message of the calling thread's last failed call. */
const char *sim_last_error(void);

#ifdef __cplusplus
}
#endif
#endif

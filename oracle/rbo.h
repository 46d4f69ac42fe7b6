/*
 * rbo.h -- FP64 CPU oracle of the batched rigid-body step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the package's smoke() check and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code with
 * the HIP path: no headers, no helpers, no tables.
 *
 * It computes, in plain double-precision loops and in the method's own order,
 * one step (s_t, a_t) -> s_{t+1} of the physics engine that the paper's
 * simulator definition names (Sec. 2, "What is a simulator?"), for a batch of
 * independent scenes made of rigid bodies with mass, friction and restitution
 * and simplified collision proxies (Sec. 3, asset creation; Sec. 4.3), with
 * parts constrained to the base treated as static (Sec. 4.1) and a
 * kinematically driven 7-DoF arm (Sec. 5, embodiment), at 1/120 s per step
 * (Sec. 4.4).  The paper does not specify the engine's algorithms; the steps
 * follow the readings written in the design notes: brute-force broadphase,
 * sphere/box/capsule narrowphase, first-fit colouring, colour-major projected
 * Gauss-Seidel (or Jacobi), semi-implicit Euler.
 *
 * Key layouts (identical on both sides by definition, not by shared code):
 *   pair key    = (a << 16) | b            b = 0xFFFF for the ground
 *   contact key = (a << 20) | (b << 8) | f b = 0xFFF  for the ground
 */
#ifndef RBO_H
#define RBO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_SPHERE = 0, ORA_BOX = 1, ORA_CAPSULE = 2, ORA_HULL = 3 };
enum { ORA_DYNAMIC = 0, ORA_STATIC = 1, ORA_KINEMATIC = 2 };
enum { ORA_COLD = 0, ORA_PREV = 1, ORA_LEARNED = 2 };
enum { ORA_PGS = 0, ORA_JACOBI = 1 };
enum { ORA_F_NONFINITE = 1, ORA_F_CAPACITY = 2, ORA_F_NOT_CONVERGED = 4, ORA_F_FELLBACK = 8 };

typedef struct ora_model {
    int n_scenes;
    const int32_t *body_offset;   /* [S+1] */
    const uint8_t *shape;         /* [N] */
    const uint8_t *motion;        /* [N] */
    const double *param;          /* [N*3] sphere r | box half-extents | capsule r, half-length */
    const double *mass;           /* [N] kg (ignored unless dynamic) */
    const double *friction;       /* [N] */
    const double *restitution;    /* [N] */
    int arm;                      /* 1: the last 7 bodies of every scene are the arm links,
                                     kinematic (poses follow theta); 2: the arm is one
                                     articulated body in reduced coordinates (theta and its
                                     rates) driven by PD position motors */
    const double *arm_base;       /* [S*3] */
    double link_len[7];
    double arm_radius;
    double gravity[3];
    double margin;                /* AABB fattening and contact keep distance (m) */
    double baumgarte;
    double slop;                  /* m */
    double rest_thresh;           /* m/s */
    double ground_friction;
    double ground_restitution;
    double sleep_speed;           /* m/s; > 0 with sleep_steps > 0 and a rest array: sleeping on */
    int sleep_steps;              /* steps at rest before an island may sleep */
    double motor_kp;              /* arm 2: position gain of the joint motors (fraction of the
                                     angle error closed per step) */
    double motor_max;             /* arm 2: largest motor impulse per step (N s) */
    /* Articulated container parts (doors, drawers): a dynamic body with
     * joint[i] = 1 turns about the world line through joint_anchor[i] along
     * joint_axis[i] (revolute, q in rad), with 2 it slides along joint_axis[i]
     * (prismatic, q in m); q = 0 at its initial pose, held within
     * joint_limits[i] = (lo, hi); it does not collide with joint_parent[i]
     * (local index of its static base, -1 for none).  NULL: no parts. */
    const uint8_t *joint;         /* [N] 0 none, 1 revolute, 2 prismatic */
    const double *joint_axis;     /* [N*3] unit, world */
    const double *joint_anchor;   /* [N*3] world point on the hinge line */
    const double *joint_limits;   /* [N*2] */
    const int32_t *joint_parent;  /* [N] */
    /* Convex hulls (shape ORA_HULL; convex collision proxies, Sec. 3 and
     * Sec. 4.3): param[3*i] of a hull body is the index of its hull in this
     * library.  A hull's vertices are in the body frame (origin at the
     * centre of mass of the solid, axes along its principal axes); its faces
     * are vertex loops counter-clockwise seen from outside, at most 8
     * vertices, -1 after the last; at most 32 vertices and 32 faces. */
    int n_hulls;
    const int32_t *hull_index;    /* [H*4]: first vertex, vertex count, first face, face count */
    const double *hull_vert;      /* [V*3] */
    const int32_t *hull_face;     /* [F*8] */
} ora_model;

typedef struct ora_cache {        /* previous step's contacts, sorted by key */
    int cap;                      /* per-scene capacity */
    int32_t *count;               /* [S] */
    uint32_t *key;                /* [S*cap] */
    double *lam;                  /* [S*cap*4]: lambda_n, world friction impulse xyz */
} ora_cache;

typedef struct ora_mlp {          /* 16-64-64-3 warm-start network */
    const double *w1, *b1;        /* [64*16], [64] row-major (out, in) */
    const double *w2, *b2;        /* [64*64], [64] */
    const double *w3, *b3;        /* [3*64], [3] */
    const double *mean, *std;     /* [16] feature normalisation */
    int bf16;                     /* 1: round weights and layer inputs to bf16 (RNE) */
} ora_mlp;

typedef struct ora_out {          /* optional per-scene outputs (any pointer may be NULL) */
    int max_pairs, max_contacts;
    int32_t *n_pairs;             /* [S] */
    uint32_t *pair_key;           /* [S*max_pairs] */
    int32_t *n_contacts;          /* [S] */
    uint32_t *c_key;              /* [S*max_contacts] */
    double *c_normal;             /* [S*max_contacts*3] unit, from body b to body a */
    double *c_point;              /* [S*max_contacts*3] */
    double *c_phi;                /* [S*max_contacts] signed separation (m) */
    double *c_lambda;             /* [S*max_contacts*3] impulses n, t1, t2 (N s) */
    int32_t *c_colour;            /* [S*max_contacts], -1 for a contact of sleeping bodies */
    double *c_feat;               /* [S*max_contacts*16] warm-start features */
    int32_t *n_colours;           /* [S] */
    int32_t *sweeps;              /* [S] */
    double *residual;             /* [S] last sweep's residual (m/s) */
    double *arm_force;            /* [S] N */
    int32_t *flags;               /* [S] */
    int32_t *ambiguous;           /* [S] decisions that fell inside the tie band */
    uint8_t *tied;                /* [N] 1 for the bodies of a pair with such a decision */
    double *tol_gap;              /* [S] min over the tested sweeps of |residual - tol| / tol */
} ora_out;

/* One step for scenes [s0, s1).  pose [N*7] (x, q w x y z), vel [N*6] (v, w),
 * theta [S*7] are read and overwritten.  rest [N] (may be NULL: no
 * sleeping) counts the steps each dynamic body has ended at rest and is
 * updated.  arm_state [S*21] (arm 2 only, PGS without the learned start;
 * may be NULL otherwise): per scene the joint rates (rad/s), the motor
 * targets (rad) and the motor impulses of the last step (N m s, the warm
 * start), 7 each, read and overwritten.  joint_state [N*2] (with parts;
 * may be NULL otherwise): per body the joint coordinate q and its rate,
 * read and overwritten.  cache may be NULL (then treated as
 * empty and not written).  actions [S*7] joint velocities (rad/s; arm 2:
 * velocities of the motor targets) or NULL.
 * iters: sweep cap.  tol > 0 stops a scene's sweeps once residual <= tol.
 * Returns 0, or -1 on a bad argument. */
int ora_step(const ora_model *m, double *pose, double *vel, double *theta, int32_t *rest,
             double *arm_state, double *joint_state, ora_cache *cache, const double *actions, double dt, int iters,
             double tol, int warm, int solver, const ora_mlp *mlp,
             ora_out *out, int s0, int s1);

/* Arm forward kinematics for all scenes: writes the arm links' pose. */
int ora_arm_pose(const ora_model *m, double *pose, const double *theta);


/* Narrowphase of one body pair, for unit tests.  Shapes as in the model;
 * poses [7].  ground: b is the plane z = 0 (shape_b, param_b, pose_b unused).
 * Writes up to 4 contacts (normal from b to a).  Returns the count. */
int ora_collide(int shape_a, const double *param_a, const double *pose_a,
                int shape_b, const double *param_b, const double *pose_b,
                int ground, double margin, int *feature, double *normal,
                double *point, double *phi, int *ambiguous);

/* ora_collide with a hull library (the model's hull fields; other fields
 * unused): shapes may be ORA_HULL, param[0] the hull index. */
int ora_collide_hulls(const ora_model *m, int shape_a, const double *param_a, const double *pose_a,
                      int shape_b, const double *param_b, const double *pose_b,
                      int ground, double margin, int *feature, double *normal,
                      double *point, double *phi, int *ambiguous);

/* Mass properties of hull h of the library for mass m: writes the inertia
 * tensor about the body origin (row-major 3x3), the centre of mass and the
 * volume.  Returns 0, or -1 for a bad index or an unusable hull. */
int ora_hull_mass(const ora_model *m, int h, double mass, double *I, double *com, double *volume);

/* Brute-force pair set of scene s at the given poses. Returns the count. */
int ora_pairs(const ora_model *m, const double *pose, int s, uint32_t *keys, int cap);

/* Collision queries of M arm configurations per scene (motion planning):
 * theta_q [S*M*7] joint angles; hit [S*M] 1 iff some arm link comes within
 * `clearance` of a body that is not an arm link or of the ground; min_phi
 * [S*M] (may be NULL) the least separation found (+INF if none within
 * reach); ambiguous [S*M] (may be NULL) 1 where min_phi is within the tie
 * band of the clearance.  pose [N*7].  Returns 0, or -1 on a bad argument. */
int ora_arm_query(const ora_model *m, const double *pose, const double *theta_q, int M, double clearance,
                  uint8_t *hit, double *min_phi, int32_t *ambiguous, int s0, int s1);

/* MLP: forward for n rows of 16 raw features -> n*3 outputs. */
void ora_mlp_forward(const ora_mlp *net, const double *x, int n, double *y);

/* Loss 1/(3n) sum (y - t)^2 and its gradient w.r.t. every parameter
 * (pure FP64, or with the forward pass rounded like the bf16 kernels when
 * net->bf16 = 1).  g* have the shapes of the weights.  Returns the loss. */
double ora_mlp_loss_grad(const ora_mlp *net, const double *x, const double *t, int n,
                         double *gw1, double *gb1, double *gw2, double *gb2,
                         double *gw3, double *gb3);

/* Round to the nearest bf16 (ties to even), returned as a double. */
double ora_bf16(double x);

#ifdef __cplusplus
}
#endif
#endif

/*
 * zema.h -- C interface of the MI355X (gfx950) library for the Newton step of the
 * soft/affine incremental-potential-contact method of Du et al., "Intersection-free
 * Robot Manipulation with Soft-Rigid Coupled Incremental Potential Contact"
 * (arXiv 2311.05945), Sec. III.
 *
 * Problem statement followed by every call: soft bodies are tetrahedral meshes with
 * a diagonal (lumped) mass and a hyper-elastic potential (Sec. III eq. 1, Sec. IV-D:
 * neo-Hookean with a logarithmic volume term); rigid bodies are affine bodies with
 * 12 DOFs q_b = (p, a1, a2, a3), x = A x0 + p, mass M_b = int rho J^T J and the
 * orthogonality potential lambda V |A A^T - I|_F^2 (eq. 2); both are integrated as
 * one barrier-augmented incremental potential (eqs. 3-5) with lagged smoothed
 * friction (eqs. 9-10), minimised by projected Newton (eqs. 6-8, 11) with an
 * intersection-free line search.  Driven bodies follow a kinematic target through
 * the penalty kappa_A/2 |q - q~|^2 (Sec. IV-C-1, multiplier zero).
 *
 * Conventions
 *   - Status: 0 ok, negative error (ZEMA_E_*).  Outputs are valid only on ok,
 *     except the required counts returned with ZEMA_E_CAPACITY.
 *   - The DOF vector y is [soft vertex xyz (3 per vertex, bodies in creation order) |
 *     q of every non-fixed affine body (12 each, creation order)].  Fixed affine
 *     bodies are Dirichlet: their DOFs are not in y.
 *   - Arrays of the hot-path calls (y, ydot, p, grad, xs, pair lists, rhs, sol, v,
 *     out) are DEVICE pointers on the scene's device; scalar outputs (terms, alpha,
 *     counts, stats) are HOST pointers.  Scene descriptors are host pointers and
 *     are copied at creation.  The caller owns every pointer it passes.
 *   - Positions are row-major (n,3) doubles in SI units; indices int32, zero-based.
 *   - Surface numbering (used by pair lists): surface vertices = boundary vertices
 *     of each soft body in ascending vertex order, then every vertex of each affine
 *     body, bodies in creation order; triangles are rotated so the smallest id comes
 *     first (orientation kept) and sorted; edges are (min,max) pairs, sorted.
 *   - A scene is bound to one HIP stream (NULL = default stream); calls on one scene
 *     are not thread-safe; different scenes are independent.
 */
#ifndef ZEMA_H
#define ZEMA_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ZEMA_OK = 0,
  ZEMA_E_ARG = -1,        /* bad argument or size */
  ZEMA_E_MESH = -2,       /* degenerate / inverted tet, open or inward affine surface */
  ZEMA_E_INTERSECT = -3,  /* a contact pair at zero distance (state not intersection-free) */
  ZEMA_E_CAPACITY = -4,   /* output buffer too small; required count returned */
  ZEMA_E_NEWTON = -5,     /* Newton did not converge in newton_max iterations */
  ZEMA_E_LINESEARCH = -6, /* line-search step fell below 1e-10 */
  ZEMA_E_PCG = -7,        /* PCG breakdown (p^T H p <= 0) or no convergence */
  ZEMA_E_NONFINITE = -8,  /* NaN / Inf in the state or a result */
  ZEMA_E_DEVICE = -9      /* HIP runtime error */
};

/* flags of zema_ip_assemble */
enum {
  ZEMA_GRAD = 1u,       /* write the gradient of the selected terms */
  ZEMA_HESS = 2u,       /* assemble the PSD-projected Hessian of the selected terms */
  ZEMA_REBUILD = 4u,    /* rebuild the candidate set statically at y (r = dhat) first */
  ZEMA_TERMS_SHIFT = 8u /* bits 8..13 select terms (0 inertia, 1 elastic,
                           2 orthogonality, 3 kinematic, 4 barrier, 5 friction);
                           0 selects all */
};

enum { ZEMA_FREE = 0, ZEMA_FIXED = 1, ZEMA_DRIVEN = 2 };
enum { ZEMA_FP64 = 0, ZEMA_MIXED = 1 };
enum { ZEMA_WARM_EXPLICIT = 0, ZEMA_WARM_LEARNED = 1 };

typedef struct zema_scene zema_scene;
typedef struct zema_mlp zema_mlp;

/* Solver parameters.  dt = h, dhat = barrier distance d-hat (eq. 5), kappa = barrier
 * stiffness (eq. 4; <= 0 selects the automatic rule: kappa0 = h^2 mbar |g| /
 * (dhat (ln 2 + 1/2)), doubled after an accepted iterate whose minimum distance
 * dropped below 1e-3 dhat and decreased), mu = friction coefficient and eps_v =
 * velocity threshold of eqs. 9-10, gravity (m/s^2), newton_tol (m/s: converged when
 * the largest vertex displacement of a Newton direction is <= newton_tol * dt),
 * pcg_rtol (relative residual), ccd_s (ACCD separation fraction, 0.1),
 * newton_max, pcg_max (<= 0: number of DOFs), precision (ZEMA_FP64: every array
 * FP64; ZEMA_MIXED: Hessian blocks, their products and the block-Jacobi
 * preconditioner in FP32, energies, gradients, line search, CCD and the convergence
 * test FP64), warm_start (ZEMA_WARM_EXPLICIT: y^t + alpha h ydot^t; ZEMA_WARM_LEARNED:
 * the network attached by zema_scene_set_mlp proposes the soft-vertex displacement,
 * filtered by the same CCD bound and kept only if its energy is not higher than the
 * explicit start's). */
typedef struct {
  double dt, dhat, kappa, mu, eps_v;
  double gravity[3];
  double newton_tol, pcg_rtol, ccd_s;
  int32_t newton_max, pcg_max, precision, warm_start;
} zema_params;

/* Soft tetrahedral body (Sec. III eq. 1): rest positions [n_verts][3], tets
 * [n_tets][4] (positive orientation expected, negative ones are reordered), optional
 * initial positions / velocities (NULL = rest / zero), Young's modulus E (Pa),
 * Poisson ratio nu, density rho (kg/m^3) and the constitutive model (Sec. IV-D):
 * ZEMA_NEO_HOOKEAN  Psi = mu/2 (|F|^2 - 3) - mu log J + lambda/2 (log J)^2,
 * ZEMA_STVK         Psi = mu |E|^2 + lambda/2 (tr E)^2, E = (F^T F - I)/2,
 * ZEMA_FIXED_COROTATED  Psi = mu |F - R|^2 + lambda/2 (J - 1)^2, F = R S;
 * mu, lambda the Lame parameters of E and nu; J <= 0 is infeasible for every model.
 * ZEMA_BARAFF_WITKIN makes the body a garment (Sec. IV-D): no tets (n_tets = 0) and
 * triangles tris [n_tris][3] instead; rest material coordinates (u, v) = rest (x, z)
 * of the vertices; per triangle of rest area A the incremental-potential energy
 * h^2 A (k_s/2 ((|w_u| - 1)^2 + (|w_v| - 1)^2) + k_sh/2 (w_u . w_v)^2), w_u, w_v the
 * columns of the deformation x = W (u, v)^T + const, with k_s = E and
 * k_sh = E / (2 (1 + nu)) (N/m); rho is the area density (kg/m^2), lumped as rho A / 3
 * per vertex; every triangle is a contact surface triangle; no bending.  A garment
 * body is accepted by zema_scene_create only (not in batches).
 * An unknown model, tets on a garment or triangles on a solid is ZEMA_E_ARG. */
enum { ZEMA_NEO_HOOKEAN = 0, ZEMA_STVK = 1, ZEMA_FIXED_COROTATED = 2, ZEMA_BARAFF_WITKIN = 3 };
typedef struct {
  int32_t n_verts, n_tets;
  const double* rest_pos;
  const int32_t* tets;
  const double* pos0;
  const double* vel0;
  double E, nu, rho;
  int32_t model, pad_;
  const int32_t* tris; /* garment triangles (ZEMA_BARAFF_WITKIN), else NULL */
  int32_t n_tris, pad2_;
} zema_soft_desc;

/* Affine body (Sec. III eq. 2): closed outward triangle surface in world
 * coordinates at t = 0 (the rest state), density, orthogonality stiffness lambda
 * (Pa), initial dq/dt (12), mode, and for driven bodies the kinematic penalty
 * kappa_A and a target that moves at target_vel (m/s) until target_stop (s). */
typedef struct {
  int32_t n_verts, n_tris;
  const double* rest_pos;
  const int32_t* tris;
  double rho, stiffness;
  double qdot0[12];
  int32_t mode, pad_;
  double kappa_A;
  double target_vel[3];
  double target_stop;
} zema_affine_desc;

/* Per-step statistics written by zema_step. */
typedef struct {
  int32_t status, newton_iters, pcg_iters, ls_backtracks;
  int32_t n_pt_active, n_ee_active, n_pt_cand, n_ee_cand;
  int32_t warm_learned;    /* 1 if the learned initial guess was kept */
  int32_t pcg_breakdowns;  /* PCG solves of the step ended at non-positive curvature */
  int32_t al_updates;      /* multiplier updates of the kinematic energy (zema_kinematic_al) */
  int32_t pad_;
  double alpha_ccd_min, kappa, d_min, energy;
  double ms_total, ms_assemble, ms_pcg, ms_broad, ms_ccd, ms_linesearch, ms_warm;
} zema_step_stats;

/* Create a scene from the problem statement of Sec. III (eqs. 1-3): tetrahedral soft
 * bodies with a lumped (diagonal) mass and affine bodies with M_b = int rho J^T J.
 * Copies every input, precomputes rest-shape inverses, volumes, lumped masses,
 * boundary surfaces, affine mass properties (volume, mass, centre, second moment;
 * the rest shape x0 is measured from the centre) and the static sparsity pattern,
 * and sets the initial state (rest or pos0, velocities vel0 / qdot0).  hip_stream:
 * a hipStream_t or NULL.  The scene owns its device memory until zema_scene_destroy.
 * Errors: ZEMA_E_ARG, ZEMA_E_MESH, ZEMA_E_INTERSECT, ZEMA_E_DEVICE. */
int zema_scene_create(const zema_params* params, const zema_soft_desc* soft, int32_t n_soft,
                      const zema_affine_desc* affine, int32_t n_affine, void* hip_stream,
                      zema_scene** out);
void zema_scene_destroy(zema_scene* s);
const char* zema_status_string(int status);
const char* zema_last_error(const zema_scene* s);

/* Sizes: [0] n_dof, [1] soft vertices, [2] tets, [3] surface vertices, [4] surface
 * triangles, [5] surface edges, [6] non-fixed affine bodies, [7] all bodies. */
int zema_sizes(const zema_scene* s, int64_t* out8);

/* Set / get the time-step state y^t, dy^t/dt (device, n_dof each), the barrier
 * stiffness (kappa <= 0 keeps the automatic rule's value) and the step index.
 * Setting the state recomputes the predictor of eq. 3, the kinematic targets and the
 * lagged friction table (eqs. 9-10) at y^t. */
int zema_set_state(zema_scene* s, const double* y, const double* ydot, double kappa, int32_t step);
int zema_get_state(zema_scene* s, double* y, double* ydot, double* kappa, int32_t* step);
/* Change kappa without recomputing the lagged friction table. */
int zema_set_kappa(zema_scene* s, double kappa);

/* Surface vertex positions xs [n_surf][3] (device) of the DOF vector y: soft
 * vertices copied, affine vertices ((a_k1 x0_1 + a_k2 x0_2) + a_k3 x0_3) + p_k
 * without fused multiply-add. */
int zema_surface_positions(zema_scene* s, const double* y, double* xs);

/* Candidate contact pairs (Sec. III: the set C of eq. 4 restricted by a broad
 * phase): every inter-body (surface vertex, triangle) pair and (edge a, edge b)
 * pair with a < b, not both on fixed bodies, whose boxes overlap, each box being
 * [min over the primitive's vertices of min(xs0, xs1)] - r .. [max of max] + r per
 * axis, closed intervals.  xs1 = NULL means static (xs1 = xs0).  Output pt [n][2]
 * = (vertex, triangle) sorted lexicographically, ee [n][2] = (a, b) sorted; device
 * buffers of capacity pt_cap / ee_cap pairs.  The set is also stored in the scene
 * as the current candidate set.  ZEMA_E_CAPACITY with *n_pt / *n_ee = required. */
int zema_contact_candidates(zema_scene* s, const double* xs0, const double* xs1, double r,
                            int32_t* pt, int64_t pt_cap, int64_t* n_pt, int32_t* ee, int64_t ee_cap,
                            int64_t* n_ee);

/* Barrier-augmented incremental potential of Sec. III (eqs. 1-5 with the lagged
 * friction of eqs. 9-10) at y (device, n_dof).  The active set is every pair of the
 * scene's current candidate set (the last one stored by zema_contact_candidates,
 * zema_set_state, a step or an earlier assemble) closer than dhat at y; with
 * ZEMA_REBUILD the set is first rebuilt statically at y (r = dhat), which stores it.
 * Outputs: energy terms (host, 8 doubles: inertia, elastic, orthogonality,
 * kinematic, barrier, friction, total, minimum candidate distance), the gradient
 * (device, n_dof; with ZEMA_GRAD) and, with ZEMA_HESS, the PSD-projected Hessian kept
 * in the scene (eqs. 6-8: x-space pair blocks projected, then mapped through the
 * affine Jacobian) for zema_hessian_matvec, zema_hessian_bsr and zema_pcg_solve.
 * ZEMA_E_INTERSECT if a tet is inverted or a candidate distance is zero (total =
 * +inf); ZEMA_E_ARG on a batch. */
int zema_ip_assemble(zema_scene* s, const double* y, uint32_t flags, double* terms, double* grad);

/* out = H v for the last assembled Hessian (device vectors, n_dof).  ZEMA_E_ARG
 * before the first assembly with ZEMA_HESS. */
int zema_hessian_matvec(zema_scene* s, const double* v, double* out);

/* The last assembled Hessian (the PSD-projected Newton matrix of eqs. 6-8) as block
 * sparse rows over 3-DOF nodes: node n holds DOFs 3n .. 3n+2 of y (soft vertex i is
 * node i; a free affine body's p, a1, a2, a3 are four consecutive nodes).  Device
 * outputs: row_ptr [n_dof/3 + 1], col [nnzb] (ascending within a row) and val
 * [nnzb][3][3] (row-major blocks, FP64; the mixed form's FP32 blocks are converted).
 * Both triangles are stored; the matrix is symmetric.  cap is the capacity of col
 * and val in blocks; *nnzb (host) receives the block count, also with
 * ZEMA_E_CAPACITY when cap is too small (row_ptr, col and val may then be NULL).
 * ZEMA_E_ARG without an assembled Hessian or on a batch. */
int zema_hessian_bsr(zema_scene* s, int32_t* row_ptr, int32_t* col, double* val, int64_t cap, int64_t* nnzb);

/* Surface topology that the pair lists of zema_contact_candidates and the
 * intersection check index (the primitives of the contact set C of Sec. III eq. 4):
 * tris [n_tris][3] and edges [n_edges][2] in surface vertex ids, the global body of
 * each surface vertex vbody [n_surf] (soft bodies first, then affine bodies, in
 * creation order) and its source vsrc [n_surf] (>= 0: the soft vertex, whose DOFs are
 * 3 vsrc .. 3 vsrc + 2; < 0: -(1 + affine body index), the vertex x = A x0 + p of that
 * body).  Device outputs, each optional (NULL skips it).  Errors: ZEMA_E_ARG. */
int zema_surface_view(zema_scene* s, int32_t* tris, int32_t* edges, int32_t* vbody, int32_t* vsrc);

/* The linear solve of a projected-Newton step (Sec. III; the runtime table of
 * Sec. V lists it as "Linear"): block-Jacobi preconditioned CG on the last assembled
 * Hessian, H sol = rhs, start at 0, stop at |r|_2 <= rtol |rhs|_2 or max_iter (<= 0:
 * n_dof) iterations.  The preconditioner inverts the 3x3 diagonal block of each soft
 * vertex and the 12x12 diagonal block of each free affine body.  rhs, sol device;
 * iters, rel_res host.  FP64 form: non-positive curvature (p.Hp <= 0) is
 * ZEMA_E_PCG.  Mixed form: the FP32 products' recurrence residual is checked at exit
 * against b - H sol recomputed with FP64 accumulation; while that true residual
 * exceeds rtol (at most twice), the residual equation is solved and its solution
 * added, and rel_res reports the true residual.  Non-positive curvature, which FP32
 * rounding of a PSD-projected Hessian can produce, ends a mixed solve with the
 * current iterate (M^-1 rhs at the first iteration).  ZEMA_E_PCG also on no
 * convergence or a singular preconditioner block. */
int zema_pcg_solve(zema_scene* s, const double* rhs, double* sol, double rtol, int32_t max_iter,
                   int32_t* iters, double* rel_res);

/* Largest step alpha in (0, 1] along p from y (device vectors) that additive CCD
 * (Li, Kaufman, Jiang 2021, Alg. 1; separation s = ccd_s, zero thickness) certifies
 * over the swept candidate set of [y, y + p] (r = dhat).  ZEMA_E_INTERSECT if a pair
 * starts at zero distance. */
int zema_ccd_max_step(zema_scene* s, const double* y, const double* p, double* alpha);

/* Advance n_steps time steps: each is the minimisation of eq. 11 by projected
 * Newton (Sec. III) -- predictor of eq. 3 and kinematic targets, lagged friction
 * (eqs. 9-10) at y^t, warm start, then per iteration assembly (eqs. 1-8), PCG,
 * convergence test, swept candidates, CCD bound, backtracking line search on the
 * energy with an inversion check (intersection-free), kappa rule -- and the velocity
 * update (y - y^t)/h.  On an error the scene keeps the last accepted state.  stats:
 * host array of n_steps * n_scenes entries, step-major (n_scenes = 1 for a single
 * scene). */
int zema_step(zema_scene* s, int32_t n_steps, zema_step_stats* stats);

/* Contact force sensing (Sec. IV-B): the force on a surface vertex is -dB/dx / h^2
 * (N), B the barrier energy of eq. 4 over the candidate set rebuilt statically at y
 * (device, n_dof) -- the incremental potential is h^2 times the potential energy --
 * and the force on a body the sum over its surface vertices.  forces: host
 * [n_bodies][3], soft bodies first, then affine bodies (fixed ones included), in
 * creation order.  Replaces the scene's current candidate set and assembled Hessian.
 * ZEMA_E_INTERSECT if the state is infeasible; ZEMA_E_ARG on NULL pointers. */
int zema_contact_forces(zema_scene* s, const double* y, double* forces);

/* Kinematic target q~ (eq. 13) of driven affine body `body` (index among the affine
 * bodies, creation order) for the steps that follow: q (host, 12 values: p, a1, a2,
 * a3), or NULL to return to the scheduled target (target_vel until target_stop).
 * ZEMA_E_ARG if the body is not driven. */
int zema_set_drive_target(zema_scene* s, int32_t body, const double* q);

/* Springs (Sec. IV-C-3): the energy k |x - target|^2 of each of n distinct surface
 * vertices sv (host int32 [n]; x = the soft vertex, or A x0 + p of an affine body's
 * vertex) with stiffness k (host [n], N/m) towards targets (host [n][3], m), added to
 * the incremental potential times h^2 and reported in the constraint term (energy
 * term 3, with the kinematic energy); n = 0 removes them.  Replaces the previous set.
 * ZEMA_E_ARG on a batch, an out-of-range or repeated vertex, or a negative k. */
int zema_set_springs(zema_scene* s, int32_t n, const int32_t* sv, const double* k, const double* targets);

/* Prismatic joints (Sec. IV-C-2) between affine bodies b12[i][0] = b1 and b12[i][1] = b2
 * (indices among the affine bodies, distinct, not both fixed), axis d = axes[i] in b1's
 * rest frame, stiffness kappa[i] (incremental-potential units, as kappa_A): the energy
 * kappa (|A1 - A2|_F^2 + |r x (A1 d)|^2), r the gap between the two bodies' images of
 * b1's rest centre of mass (in b1: p1; in b2: A2 (c1 - c2) + p2).  Its Hessian is the
 * Gauss-Newton matrix of the 12 residuals (PSD; the exact Hessian where the joint
 * holds).  The energy joins the constraint term (term 3).  n = 0 removes the joints;
 * host arrays b12 [n][2], axes [n][3], kappa [n].  ZEMA_E_ARG on a batch or bad
 * bodies. */
int zema_set_prismatic_joints(zema_scene* s, int32_t n, const int32_t* b12, const double* axes, const double* kappa);

/* Augmented Lagrangian of the kinematic energy (Sec. IV-C-1 eq. 13): E_A =
 * kappa_A/2 |q - q~|^2 - sqrt(m) lambda_A . (q - q~) per driven body (m its mass).
 * With tol > 0, a step whose Newton loop has converged checks max |q - q~| over the
 * driven bodies; while it exceeds tol (at most max_updates times per step) every
 * driven body's multiplier is updated, lambda_A <- lambda_A - kappa_A / sqrt(m)
 * (q - q~), and the Newton loop continues from the same state.  tol = 0 (the default)
 * keeps the multipliers (initially zero: the penalty alone).  lam (host [n_affine][12],
 * optional) receives the multipliers.  Single scenes only (ZEMA_E_ARG on a batch). */
int zema_kinematic_al(zema_scene* s, double tol, int32_t max_updates, double* lam);

/* Grasp procedure (Sec. V: AutoGrasp, Lift, Shake) on a single scene whose driven
 * affine bodies are the fingers, each closing along its target_vel at |target_vel|.
 * Before every step the contact forces are measured at the current state (as
 * zema_contact_forces) and every finger's target is set to its current state plus
 *   AutoGrasp: phi(f) h target_vel, f = |force on the finger|, with the controller of
 *     Sec. IV-A eq. 12: phi(f) = (exp(-k f) - exp(-k f*)) / (1 - exp(-k f*)) for
 *     0 <= f < f*, 0 for f >= f*; the phase ends when phi = 0 for every finger (each
 *     has reached f*) or after max_close_steps;
 *   Lift: lift_speed h along -gravity, lift_steps steps;
 *   Shake: a(t + h) - a(t) along shake_axis, a(t) = shake_amplitude
 *     sin(2 pi shake_frequency t) from the start of the phase, shake_steps steps.
 * The grasp succeeds when, at the end, the object body is still in contact with the
 * hand (a nonzero force on some finger) and not with the ground body (zero force).
 * trace (host, optional): per step [phase, |f_ground|, |f_finger| ...] (2 + fingers
 * doubles, at most trace_cap rows).  On a step error the procedure stops with that
 * status in res->status. */
typedef struct {
  double k, f_star;                /* 1/N, N */
  int32_t max_close_steps, lift_steps, shake_steps, object_body;
  double lift_speed;               /* m/s */
  double shake_amplitude, shake_frequency, shake_axis[3];
  int32_t ground_body, pad_;       /* global body ids (soft bodies first); ground -1: none */
} zema_grasp_params;

typedef struct {
  int32_t status, close_steps, total_steps, success, n_fingers, pad_;
  double ground_force, finger_force_max; /* |f| at the end */
} zema_grasp_result;

int zema_grasp_run(zema_scene* s, const zema_grasp_params* gp, zema_grasp_result* res, double* trace,
                   int32_t trace_cap);

/* ---------------------------------------------------------------- batches
 * Independent scenes stepped together (the paper evaluates grasps in parallel): one
 * object holds the concatenation of every scene's bodies, each phase of a step is one
 * launch over all of them, and every scene keeps its own Newton iteration, PCG
 * scalars, CCD bound, line search and barrier stiffness; a scene that has converged
 * stops moving until all have.  Scene k owns soft bodies [soft_off[k], soft_off[k+1])
 * and affine bodies [aff_off[k], aff_off[k+1]) of the descriptor arrays (offsets:
 * host [n_scenes + 1], starting at 0); params[k] (host [n_scenes]) must agree on every
 * field except mu.  Candidate pairs never join two scenes.
 * y (zema_get_state / zema_set_state) is [soft vertices of all scenes, scene by
 * scene | free affine bodies of all scenes, scene by scene]; surface vertices are
 * numbered scene by scene.  zema_step fills n_steps * n_scenes statistics; the
 * single-scene hot-path calls (ip_assemble, pcg_solve, ccd_max_step) return
 * ZEMA_E_ARG on a batch, zema_set_kappa sets every scene and zema_get_state reports
 * scene 0's kappa.  Errors: as zema_scene_create. */
int zema_batch_create(const zema_params* params, int32_t n_scenes, const zema_soft_desc* soft,
                      const int32_t* soft_off, const zema_affine_desc* affine, const int32_t* aff_off,
                      void* hip_stream, zema_scene** out);
/* Number of scenes and, when ranges is not NULL, per scene (host [n_scenes][8]):
 * soft vertex range, free affine body range, tet range, surface vertex range, each
 * [begin, end).  A scene's DOFs are 3 v0 .. 3 v1 and 3 n_soft_verts + 12 f0 ..
 * 3 n_soft_verts + 12 f1. */
int zema_batch_layout(const zema_scene* s, int32_t* n_scenes, int64_t* ranges);

/* Number of lagged friction pairs and their table (host outputs): ids5 [n][5] =
 * (kind 0 PT / 1 EE, 4 surface vertices), vals8 [n][8] = (lambda, n(3), w(4)). */
int zema_friction_table(zema_scene* s, int64_t* n, int32_t* ids5, double* vals8, int64_t cap);

/* Steps several scene objects (single scenes or batches) concurrently: one host thread
 * per object, each object's launches on its own stream (objects created on distinct
 * streams overlap on the GPU; objects sharing a stream still run correctly, in turn).
 * Splitting independent scenes into a few batch objects on a few streams (as many as
 * the device has hardware queues) overlaps one object's host synchronisation and
 * latency-bound launches with the others' work.  Each object is stepped exactly as by
 * zema_step; stats[k] is object k's array (n_steps x its scene count), status[k]
 * (host) its result.  Returns the first nonzero status, else 0.  Errors: ZEMA_E_ARG
 * (null pointers, an object listed twice). */
int zema_step_group(zema_scene* const* scenes, int32_t n_scenes, int32_t n_steps, zema_step_stats* const* stats,
                    int32_t* status);

/* Validation of the intersection-free guarantee: at y (device), the number of
 * inter-body (surface edge, surface triangle) pairs whose closed segment and closed
 * triangle intersect, the number of tets with non-positive volume, and the number of
 * pairs / tets whose orientation signs the FP64 filter (static error bound of
 * orient3d) cannot certify.  The first min(n_uncertain, cap) uncertain (edge,
 * triangle) pairs are written to uncertain_pairs (device, [cap][2]) for an exact
 * check by the caller; uncertain tets are only counted.  Counts are host outputs. */
int zema_intersection_count(zema_scene* s, const double* y, int64_t* n_intersect, int64_t* n_inverted,
                            int64_t* n_uncertain, int32_t* uncertain_pairs, int64_t cap);

/* Execution knobs of a single scene.
 * ZEMA_TUNE_PCG_GRAPH: 1 (default) replays PCG iterations in chunks of 16 from a
 *   captured HIP graph, 0 launches every kernel individually (as does the two-launch
 *   form while the PCG timer above is enabled); results are identical.
 * ZEMA_TUNE_SPMV_LANES: lanes per soft-vertex row of the PCG matrix-vector product
 *   (4 default, 8, 16, 32; the two-launch form below uses 8 where 4 is set);
 *   ZEMA_TUNE_UPDATE_BLOCK: threads per block of the two-launch form's vector update
 *   (64, 128, 256 default).  These change the floating-point summation order (results
 *   agree to rounding); a fixed setting is deterministic.
 * ZEMA_TUNE_PCG_FORM: 1 (default) runs each PCG iteration as one launch, with the
 *   two inner products of an iteration taken in one reduction (the Chronopoulos-Gear
 *   arrangement of the same iterates); 0 runs the textbook order in two launches per
 *   iteration.  In exact arithmetic both produce the same iterates; in floating point
 *   they agree to rounding (the update-block knob applies to form 0 only).
 * ZEMA_TUNE_BATCH_ASYNC (batches): 1 (default) lets each scene start its next time step
 *   as soon as its Newton loop has converged, so a call of n steps takes as many global
 *   iterations as its slowest scene needs over the n steps rather than the sum over
 *   steps of the slowest scene's; 0 steps all scenes in lockstep.  Each scene's
 *   arithmetic is the same either way (its trajectory agrees to rounding: the
 *   candidate set of its initial guess is the swept set of h ydot^t, and per-scene
 *   sums may group differently).  The learned initial guess always runs in lockstep.
 *   On failure every scene returns to the start of the step it was in.
 * ZEMA_TUNE_CG_ROWS: soft-vertex rows per workgroup of the single-launch PCG form
 *   (1..64, capped at 256 / lanes).  0 (default) spreads the rows over the device's
 *   compute units: ceil(soft rows / compute units), capped the same way, so a system
 *   of 10k rows runs on every compute unit instead of 256 / lanes rows on fewer.
 *   Each row's products do not depend on the setting; the inner products are summed
 *   per workgroup, so different settings agree to rounding (a fixed setting is
 *   deterministic).
 * ZEMA_TUNE_WARM_FIT (learned initial guess): 0 uses the network's per-vertex
 *   correction as it is; 1 replaces it on each soft body by its mass-weighted
 *   least-squares affine fit cbar + A (x_i - xbar) over the body's vertices at the
 *   step start (A = 0 for a body whose centred second moment S has
 *   det S <= 1e-9 (tr S)^3); 2 (default) by its mass-weighted mean cbar.  The fit
 *   removes the part of the network's error that varies from vertex to vertex
 *   (zema_warm_fit applies it to a given field).  Deterministic for a fixed setting.
 * Errors: ZEMA_E_ARG for an unknown knob or value. */
enum {
  ZEMA_TUNE_PCG_GRAPH = 0,
  ZEMA_TUNE_SPMV_LANES = 1,
  ZEMA_TUNE_UPDATE_BLOCK = 2,
  ZEMA_TUNE_PCG_FORM = 3,
  ZEMA_TUNE_BATCH_ASYNC = 4,
  ZEMA_TUNE_CG_ROWS = 5,
  ZEMA_TUNE_WARM_FIT = 6
};
int zema_tune(zema_scene* s, int32_t knob, int32_t value);
/* Current value of a knob (host output).  Errors: ZEMA_E_ARG for an unknown knob. */
int zema_tune_get(zema_scene* s, int32_t knob, int32_t* value);
/* Autotuner: times 64 PCG iterations on the last assembled Hessian (after
 * zema_ip_assemble or a step) for every launch shape of the current PCG form (lanes;
 * the two-launch form also the update block), keeps the fastest and returns it with
 * its time per iteration (microseconds, host outputs; update_block is unchanged for
 * the single-reduction form).
 * Overwrites the scene's internal PCG vectors only.  Errors: ZEMA_E_ARG (no Hessian,
 * batch), ZEMA_E_DEVICE. */
int zema_autotune(zema_scene* s, int32_t* lanes, int32_t* update_block, double* us_per_iter);

/* Launch timing for benchmarks: with enable != 0 the library records HIP events on
 * the scene's stream around launches of one kernel group (0 PCG iteration, 1 elastic
 * assembly: the per-tet kernel and the gradient and Hessian gathers of one assembly,
 * 2 contact pair assembly, 3 broad-phase query, 4 CCD) and
 * accumulates their durations; zema_kernel_time returns the total milliseconds, the
 * launch count and the algorithmic bytes of those launches (what the method must move:
 * for a single-reduction PCG iteration 76 B per stored 3x3 block plus 152 B per DOF
 * (r, w, s, p, x read and written, the 3x3 inverse blocks, the node records read and
 * written), for the two-launch form's product 76 B per block plus four DOF vectors,
 * for the elastic assembly 320 B per tet; 0 for the other groups) since the timer was
 * enabled.  Single-reduction PCG iterations are timed per replayed chunk of 16 (events
 * around the graph launch; chunks in which the solve converged are not counted), the
 * other groups per launch.  Both calls synchronise the stream; bytes may be NULL. */
int zema_kernel_timer(zema_scene* s, int32_t group, int32_t enable);
int zema_kernel_time(zema_scene* s, int32_t group, double* ms, int64_t* launches, double* bytes);

/* ---------------------------------------------------------------- learned initial guess
 * Not part of the paper's method: a per-soft-vertex network proposes the Newton
 * initial guess of a time step; the step itself (tolerance, CCD filter, line
 * search) is unchanged, so the result is accepted by the same Newton loop.
 *
 * Network: 16 -> 64 -> 64 -> 64 -> 3, ReLU, weight matrices used in bfloat16 (round to
 * nearest even from the FP32 master copy), biases FP32, FP32 accumulation on the
 * matrix cores.  Parameters: ZEMA_MLP_PARAMS floats in the order W1 [64][16], b1,
 * W2 [64][64], b2, W3 [64][64], b3, W4 [3][64], b4 (W row-major [out][in]).
 *
 * Features of soft vertex i (ZEMA_MLP_FEATURES floats; s = dt * 0.05 m/s):
 *   0-2 dt v_i / s;  3-5 dt (v_i - v_i of the previous step) / s;
 *   6   min(d_i, 4 dhat) / dhat, d_i the distance to the nearest triangle of another
 *       body (surface vertices; 4 for interior ones and none in range);
 *   7-9 unit vector to the closest point of that triangle; 10-12 dt (velocity of that
 *       point) / s; 13-15 dt (kinematic target velocity - velocity) / s of the driven
 *       body owning it (0 otherwise).  Entries 7-15 are 0 when no triangle is in range.
 * Output: the correction of dt v_i in units of s.  Training target of a step:
 * ((x_i^{t+1} - x_i^t) - dt v_i^t) / s. */
#define ZEMA_MLP_PARAMS 9603
#define ZEMA_MLP_FEATURES 16

/* Network object bound to hip_stream (NULL: the default stream); weights zero until
 * set.  Errors: ZEMA_E_ARG, ZEMA_E_DEVICE. */
int zema_mlp_create(void* hip_stream, zema_mlp** out);
void zema_mlp_destroy(zema_mlp* m);
const char* zema_mlp_last_error(const zema_mlp* m);
/* Host [ZEMA_MLP_PARAMS] FP32 parameters in / out; set also clears the Adam state. */
int zema_mlp_set_weights(zema_mlp* m, const float* theta);
int zema_mlp_get_weights(zema_mlp* m, float* theta);
/* out [n][3] = network(feat [n][16]); device pointers. */
int zema_mlp_forward(zema_mlp* m, const float* feat, int64_t n, float* out);
/* Mean-squared-error loss (1 / 3n) sum |out - target|^2 over rows 0..n-1 of feat and
 * target [n][3] (device) and its gradient grad [ZEMA_MLP_PARAMS] (device); loss is a
 * host output.  No update. */
int zema_mlp_grad(zema_mlp* m, const float* feat, const float* target, int64_t n, float* grad, double* loss);
/* zema_mlp_grad for callers that cannot allocate device memory (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid hipMalloc): the
 * same loss and gradient, with no hipMalloc / hipFree and no allocating library call.
 * Its partial sums live in a static array of the library (about 9.4 MiB per device,
 * 256 block partials; each device that runs it keeps its copy until the process
 * ends).  Every call on a device shares that array: calls that overlap on one device
 * (other streams, other threads) race and must be serialised by the caller.  For n <=
 * 16384 rows the result equals zema_mlp_grad's bitwise; above it the rows are summed
 * in 256 larger blocks (FP32 rounding order differs).  feat [n][16], target [n][3],
 * grad [ZEMA_MLP_PARAMS] device; loss host.  The network's device is made current for
 * the call.  ZEMA_E_ARG for n outside 1 .. ZEMA_MLP_NOALLOC_MAX_ROWS or NULL
 * pointers. */
#define ZEMA_MLP_NOALLOC_MAX_ROWS (1LL << 26)
int zema_mlp_grad_noalloc(zema_mlp* m, const float* feat, const float* target, int64_t n, float* grad,
                          double* loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, learning rate lr)
 * on the batch of rows idx [batch] (device int32, each in [0, n_rows); rows out of
 * range are skipped) of feat / target [n_rows]; loss of the batch before the step is
 * a host output. */
int zema_mlp_train_step(zema_mlp* m, const float* feat, const float* target, int64_t n_rows, const int32_t* idx,
                        int64_t batch, float lr, double* loss);

/* Network used by zema_step when params.warm_start == ZEMA_WARM_LEARNED (NULL
 * detaches).  The scene reads the weights on its own stream at every step; the
 * caller must not update them concurrently. */
int zema_scene_set_mlp(zema_scene* s, zema_mlp* m);
/* Features [n_soft_verts][16] (device) at the current state.  Replaces the stored
 * candidate set with the one at radius 4 dhat. */
int zema_scene_features(zema_scene* s, float* feat);
/* Training target [n_soft_verts][3] (device) of the last step taken by zema_step. */
int zema_scene_warm_target(zema_scene* s, float* target);
/* The per-soft-body fit of the learned initial guess (see ZEMA_TUNE_WARM_FIT; mode 0
 * copies, 1 affine fit, 2 mean) applied to a correction field at the scene's current
 * positions with its lumped masses: in, out device float [n_soft_verts][3] (the same
 * pointer fits in place).  Synchronous.  Errors: ZEMA_E_ARG (mode, null pointers),
 * ZEMA_E_DEVICE. */
int zema_warm_fit(zema_scene* s, int32_t mode, const float* in, float* out);

#ifdef __cplusplus
}
#endif
#endif

/*
 * zema_ref.h -- C interface of the CPU oracle (test infrastructure only).
 *
 * A plain, slow FP64 implementation of the barrier-augmented incremental-potential
 * Newton step of soft (tetrahedral neo-Hookean) and affine bodies.  It exists to
 * check the HIP library against; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code or header with the
 * HIP library.  All pointers are host pointers.  Status codes: 0 ok, negative error
 * (-1 argument, -2 mesh, -3 intersecting, -4 capacity, -5 Newton, -6 line search,
 * -7 PCG, -8 non-finite).
 */
#ifndef ZEMA_REF_H
#define ZEMA_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct zref_scene zref_scene;

typedef struct {
  double dt, dhat, kappa, mu, eps_v;
  double gravity[3];
  double newton_tol, pcg_rtol, ccd_s;
  int32_t newton_max, pcg_max, precision, warm_start;
} zref_params;

typedef struct {
  int32_t n_verts, n_tets;
  const double* rest_pos;
  const int32_t* tets;
  const double* pos0;
  const double* vel0;
  double E, nu, rho;
  int32_t model, pad_; /* 0 neo-Hookean, 1 Saint Venant-Kirchhoff, 2 fixed corotated,
                          3 Baraff-Witkin garment (triangles below, no tets) */
  const int32_t* tris; /* garment triangles [n_tris][3] */
  int32_t n_tris, pad2_;
} zref_soft_desc;

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
} zref_affine_desc;

typedef struct {
  int32_t status, newton_iters, pcg_iters, ls_backtracks;
  int32_t n_pt_active, n_ee_active, n_pt_cand, n_ee_cand;
  int32_t al_updates, pad_; /* augmented Lagrangian multiplier updates of the step */
  double alpha_ccd_min, kappa, d_min, energy;
} zref_step_stats;

int zref_scene_create(const zref_params* p, const zref_soft_desc* soft, int32_t n_soft,
                      const zref_affine_desc* aff, int32_t n_aff, zref_scene** out);
void zref_scene_destroy(zref_scene* s);
const char* zref_last_error(const zref_scene* s);
int zref_set_threads(int32_t n);

/* sizes: [0] n_dof, [1] n_soft_verts, [2] n_tets, [3] n_surf_verts, [4] n_tris,
 *        [5] n_edges, [6] n_free_bodies, [7] n_bodies */
int zref_sizes(const zref_scene* s, int64_t* out8);
/* surface topology (global surface ids): tris [n_tris][3], edges [n_edges][2],
 * vertex body id [n_surf], mass per DOF-owning soft vertex [n_soft_verts] */
int zref_surface(const zref_scene* s, int32_t* tris, int32_t* edges, int32_t* vbody);
int zref_lumped_mass(const zref_scene* s, double* mass);
/* affine body mass properties: per body [V, m, c(3), S(9)] = 14 doubles */
int zref_affine_props(const zref_scene* s, double* out14);

int zref_set_state(zref_scene* s, const double* y, const double* ydot, double kappa, int32_t step);
int zref_get_state(const zref_scene* s, double* y, double* ydot, double* kappa, int32_t* step);
int zref_set_kappa(zref_scene* s, double kappa);
int zref_surface_positions(const zref_scene* s, const double* y, double* xs);

int zref_candidates(zref_scene* s, const double* xs0, const double* xs1, double r,
                    int32_t* pt, int64_t pt_cap, int64_t* n_pt,
                    int32_t* ee, int64_t ee_cap, int64_t* n_ee);
/* energy terms: [0] inertia [1] elastic [2] orthogonality [3] kinematic [4] barrier
 * [5] friction [6] total [7] min distance over candidates. flags bit0 grad, bit1 hess */
int zref_ip_assemble(zref_scene* s, const double* y, uint32_t flags, double* terms, double* grad);
int zref_hessian_matvec(zref_scene* s, const double* v, double* out);
int zref_pcg_solve(zref_scene* s, const double* rhs, double* sol, double rtol, int32_t max_iter,
                   int32_t* iters, double* rel_res);
int zref_ccd_max_step(zref_scene* s, const double* y, const double* p, double* alpha);
int zref_friction_count(const zref_scene* s, int64_t* n);
/* lagged friction rows: [kind, v0, v1, v2, v3] ints and [lambda, n(3), w(4)] doubles */
int zref_friction_table(const zref_scene* s, int32_t* ids5, double* vals8);
int zref_step(zref_scene* s, int32_t n_steps, zref_step_stats* stats);

/* contact force sensing (Sec. IV-B): per body the sum over its surface vertices of
 * -dB/dx / h^2 (N), B the barrier energy over the static candidate set at y;
 * forces [n_bodies][3], soft bodies first.  The candidate set is rebuilt at y. */
int zref_contact_forces(zref_scene* s, const double* y, double* forces);
/* kinematic target of driven affine body `body` for the following steps (12 values),
 * NULL returns to the scheduled target */
int zref_set_drive_target(zref_scene* s, int32_t body, const double* q);
/* springs (Sec. IV-C-3): h^2 k |x - target|^2 per distinct surface vertex; n = 0 clears */
int zref_set_springs(zref_scene* s, int32_t n, const int32_t* sv, const double* k, const double* targets);
/* augmented Lagrangian updates of the kinematic multipliers (eq. 13): tolerance on
 * max |q - q~| (0: off), at most max_updates per step; lam (optional) reads them */
int zref_kinematic_al(zref_scene* s, double tol, int32_t max_updates, double* lam);
/* prismatic joints (Sec. IV-C-2): body pairs [n][2] (affine indices), axes [n][3] in the
 * first body's rest frame, stiffness [n]; n = 0 removes them */
int zref_set_prismatic_joints(zref_scene* s, int32_t n, const int32_t* b12, const double* axes,
                              const double* kappa);

/* iterate recording for per-iterate parity: when enabled every Newton iterate of
 * zref_step is stored: (step, kappa at lag, kappa, y^t, ydot^t, y_k). */
int zref_record(zref_scene* s, int32_t enable);
int zref_record_count(const zref_scene* s, int64_t* n);
int zref_record_get(const zref_scene* s, int64_t k, int32_t* step, double* kappa_lag, double* kappa,
                    double* y_t, double* ydot_t, double* y_k);

/* local kernels exposed for pinning: distance between a point and a triangle /
 * two edges (x: 12 doubles), barrier b(d) with derivatives, friction f0/f1. */
double zref_dist_pt(const double* x12, int32_t* type);
double zref_dist_ee(const double* x12, int32_t* type);
int zref_barrier(double d, double dhat, double* b3);
int zref_pair_energy(zref_scene* s, int32_t kind, const double* x12, const double* rest_len2,
                     double* e, double* g12, double* h144, int32_t project);
/* the same with the feature type given (type >= 0; -1: the closest feature): the
 * barrier of the squared distance of that type, for ties between two features */
int zref_pair_energy_typed(zref_scene* s, int32_t kind, const double* x12, const double* rest_len2, int32_t type,
                           double* e, double* g12, double* h144, int32_t project);
int zref_tet_energy(zref_scene* s, int32_t tet, const double* x12, double* e, double* g12,
                    double* h144, int32_t project);
int zref_project_psd(int32_t n, const double* a, double* out);
int zref_accd_pair(int32_t kind, const double* x12, const double* p12, double s, double* toi);

#ifdef __cplusplus
}
#endif
#endif

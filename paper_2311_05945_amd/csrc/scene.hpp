// Scene state of the HIP library and the launchers of its kernels.
//
// HBM layout (one scene):
//   y, ydot, y^t, ydot^t, yhat    AoS DOF vectors [3*nsv | 12*nfree] (double)
//   tets                          int4 [nt]                  (16 B, one load per tet)
//   Dm^-1                         SoA double [9][nt]         (coalesced planes)
//   h^2 V, mu, lambda             SoA double [nt] each
//   element Hessians              AoS double [nt][90]        (10 upper 3x3 blocks)
//   static BSR                    row_ptr [nodes+1], col [nnzb], val SoA [9][nnzb]
//   contact matrix (dynamic)      CSR over the same nodes, val SoA [9][nnz_c]
//   surface                       xs AoS [nsurf][3]; tris int [ntri][3]; edges int [ne][2]
// Nodes of the block system: soft vertex i -> node i; free affine body k -> nodes
// nsv + 4k + {0: p, 1: a1, 2: a2, 3: a3} (3 DOFs each), so every block is 3x3.
#pragma once
#include <memory>
#include <string>
#include <vector>

#include "../../include/zema.h"
#include "common.hpp"
#include "mlp.hpp"

namespace zema {

// Per-body device record (doubles): mass, volume, orthogonality stiffness, kappa_A,
// second moment S[9], the fixed q of a fixed body [12], the kinematic multiplier [12]
constexpr int BF = 48;
constexpr int BF_M = 0, BF_V = 1, BF_ST = 2, BF_KA = 3, BF_S = 4, BF_QF = 13, BF_LAM = 25;

struct Body {
  int mode = 0;
  int dof0 = -1, node0 = -1;       // -1 for fixed bodies
  int sv0 = 0, nsv = 0;            // surface vertex range
  double rho = 0, stiff = 0, kappaA = 0;
  double V = 0, m = 0, c[3] = {0, 0, 0}, S[9] = {0};
  double qrest[12], qdot0[12];
  double tvel[3] = {0, 0, 0}, tstop = 0;
  bool has_target = false;  // a kinematic target set by the caller replaces the schedule
  double target[12] = {0};
  double target_vel[3] = {0, 0, 0};  // (new target - previous target) / dt of the last set
  double lamA[12] = {0};             // augmented Lagrangian multiplier of the kinematic energy
};

// spring on a surface vertex (Sec. IV-C-3)
struct Spring {
  int sv;
  double k, target[3];
};

// prismatic joint between two affine bodies (Sec. IV-C-2)
struct Joint {
  int b1, b2;
  double d[3], kappa;
};

// Launch timing of one kernel group with HIP events on the scene's stream.
enum { KT_SPMV = 0, KT_TET = 1, KT_CONTACT = 2, KT_QUERY = 3, KT_CCD = 4, KT_N = 5 };
struct KTimer {
  bool on = false;
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  size_t used = 0;
  double ms = 0.0;
  long long launches = 0;
  double bytes = 0.0;           // algorithmic bytes of the timed launches
  std::vector<double> pending;  // bytes of launches not folded yet
};

// Ranges of one scene of a batch (a single scene is a batch of one).  Soft vertices,
// tets, affine bodies, free affine bodies (nodes nsv + 4 f ...) and surface vertices
// of a scene are contiguous; so are its candidate pairs, which are sorted by the
// scene-major surface numbering.
struct SceneRange {
  int v0 = 0, v1 = 0, t0 = 0, t1 = 0, b0 = 0, b1 = 0, f0 = 0, f1 = 0, s0 = 0, s1 = 0;
  double mu = 0.0, cell = 1.0, mbar = 1.0;
  double kappa = 0.0, kappa_lag = 0.0, dprev = 0.0;
};

// A captured chunk of PCG iterations (16 x [matvec, update]) and what it was captured
// with; replayed as long as every pointer and size matches.
struct PcgGraph {
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;
};

// Buffers for one radix sort of (key, value) pairs.
struct SortBufs {
  DBuf<unsigned long long> k0, k1;
  DBuf<int> v0, v1;
  DBuf<int> hist;
};

}  // namespace zema

struct zema_scene {
  zema_params P;
  hipStream_t st = nullptr;
  std::string err;
  // constraints of Sec. IV-C: springs (single scenes) and the multiplier updates of the
  // kinematic energy (al_tol > 0: at most al_max updates per step)
  std::vector<zema::Spring> springs;
  zema::DBuf<int> spr_sv;
  zema::DBuf<double> spr_kt, e_spr;  // [n][4] (k, target); energies of the springs, then of the joints
  std::vector<zema::Joint> joints;
  zema::DBuf<int> jnt_i;             // [nj][4] b1, b2, triplet offsets with / without Hessian
  zema::DBuf<double> jnt_d;          // [nj][8] axis (3), kappa, c1 - c2 (3), 0
  const double* y_asm = nullptr;     // the state of the assembly in progress
  double al_tol = 0.0;
  int al_max = 0;
  int n_soft_bodies = 0, n_bodies = 0;
  int nsv = 0, nt = 0, nsurf = 0, ntri = 0, nedge = 0, nfree = 0, ndof = 0, nnodes = 0;
  // ---- scene table (batches)
  int ns = 1;
  std::vector<zema::SceneRange> scn;
  zema::DBuf<int> body_scene, sv_scene, v_scene, f_scene;  // global body / surface vertex / soft vertex / free body
  zema::DBuf<double> sc_dots;                              // [ns][3] per-scene inner products
  zema::DBuf<int> scn_rng;                                 // [ns][8] v0 v1 t0 t1 b0 b1 f0 f1
  zema::DBuf<double> icell_sc, mu_sc, kappa_sc;                // per scene
  zema::DBuf<unsigned long long> sc_u64, sc_dmin, sc_tmin;      // per-scene extrema (bits)
  zema::DBuf<double> sc_alpha, sc_sum;                          // per-scene step sizes, sums [ns][8]
  zema::DBuf<double> sc_part;                                  // partial per-scene energy sums
  zema::DBuf<int> sc_mask, sc_rng;                              // per-scene flags; pair ranges [ns][8]
  zema::DBuf<unsigned int> sc_cnt;
  zema::DBuf<int> sc_act;                // scenes still iterating (batches), read by assembly
  bool masked = false;                   // assembly and candidate search skip converged scenes
  const int* act_dev() const { return masked ? sc_act.p : nullptr; }
  std::vector<double> kappa_h, scale_h;  // host staging of per-scene uploads
  std::vector<int> mask_h;
  std::vector<zema::Body> bodies;  // affine bodies, creation order
  std::vector<double> mass_h;
  double cell = 0.0;               // hash cell size

  // ---- soft (device)
  zema::DBuf<int4> tets;
  zema::DBuf<double> Dmi, h2vol, lmu, llam, mass;
  // ---- garment triangles (Baraff-Witkin; single-scene objects only)
  int ncl = 0;
  zema::DBuf<int4> cl_v;     // vertices (soft vertex ids)
  zema::DBuf<double> cl_d;   // [8]: inverse rest (u, v) edge matrix, rest area, k_stretch, k_shear, pad
  zema::DBuf<unsigned char> tmodel;  // per tet: 0 neo-Hookean, 1 Saint Venant-Kirchhoff, 2 fixed corotated
  zema::DBuf<int> vt_ptr, vt_list;       // vertex -> (tet*4 + local index), tet order
  zema::DBuf<double> e_tet, g_tet, h_tet, e_in;  // per-tet energy; gradient [4nt][3], Hessian [4nt][6] + [6nt][9] records
  zema::DBuf<float> h_tet32;                      // element Hessian blocks, mixed precision
  // ---- static BSR
  int nnzb = 0, bsr_row_soft_end = 0;
  zema::DBuf<int> bsr_ptr, bsr_col, bsr_row, bsr_diag, hc_ptr, hc_list;
  // element records in destination order: tslot [10][nt] (diagonal / gradient slot of
  // each tet vertex = its position in the vertex's incident list vt_ptr, then the slot
  // of each vertex pair in its upper off-diagonal block's list off_ptr); off_blk /
  // off_mir: BSR positions of those upper blocks and of their transposes
  zema::DBuf<int> tslot, off_ptr, off_blk, off_mir;
  zema::DBuf<double> bsr_val;
  zema::DBuf<float> bsr_val32;           // static block values, mixed precision
  bool mixed = false;                    // FP32 Hessian storage / products
  // ---- affine (device): per body packed
  zema::DBuf<double> body_f;  // [nb][32]: m, V, stiff, kappaA, S(9), qfix(12) ...
  zema::DBuf<int> body_i;     // [nb][4]: mode, dof0, node0, pad
  zema::DBuf<double> qtilde;  // [nb][12]
  zema::DBuf<double> e_body;  // [nb][3] inertia, orth, kinematic
  // ---- surface (device)
  zema::DBuf<int> sv_ref;      // >= 0 soft vertex, < 0 : -(body+1)
  zema::DBuf<int> sv_body;     // global body id (soft bodies first)
  zema::DBuf<double> sv_x0;    // [nsurf][3]
  zema::DBuf<int> tris, edges;
  zema::DBuf<double> elen2;
  zema::DBuf<unsigned char> body_fixed;  // per global body
  zema::DBuf<double> xs, xs1, xs2, dxs;  // surface positions / displacements
  // ---- learned initial guess
  zema_mlp* mlp = nullptr;               // network used when P.warm_start == 1 (not owned)
  bool stepped = false;                  // a step completed since the state was set
  zema::DBuf<int> soft_sv;               // soft vertex -> surface vertex or -1
  zema::DBuf<double> yd_prev, body_tv;   // velocity before the last step; target velocity [nb][3]
  std::vector<double> body_tv_h;
  zema::DBuf<unsigned long long> fdmin;  // per surface vertex: nearest other-body triangle distance
  zema::DBuf<int> fpick;                 // ... and the PT pair realising it
  zema::DBuf<float> feat, mlp_out;       // [nsv][16], [nsv][3]
  zema::DBuf<double> ywarm;              // learned initial guess [ndof]
  int warm_fit = 2;                      // 0 network output as is, 1 its affine fit per soft body, 2 its mean
  zema::DBuf<int> soft_vr, v_sbody;      // soft body -> first soft vertex [n_soft_bodies + 1]; soft vertex -> body
  zema::DBuf<double> wfit;               // per soft body: mean correction, centre, 3x3 map [15]
  // ---- state
  zema::DBuf<double> y, ydot, yt, ydt, yhat, ytmp, grad, pdir;
  int step = 0;
  std::vector<int> scene_step;  // per scene of a batch (scenes may be at different steps)
  std::vector<double> qt_h;     // host copy of the kinematic targets [nb][12]
  bool batch_async = true;      // a batch's scenes start their next step as they converge
  // ---- candidates (current set)
  zema::DBuf<int> pt, ee;       // [n][2]
  zema::DBuf<int> et_pairs, unc_pairs;  // intersection check work
  int64_t npt = 0, nee = 0;
  // broad phase work
  zema::DBuf<double> bb_lo, bb_hi;       // boxes of all primitives
  zema::DBuf<unsigned long long> body_blo, body_bhi;  // boxes of whole bodies (ordered encoding)
  zema::DBuf<int> scene_bodies;          // per scene: soft body range, affine body range (global ids)
  zema::DBuf<int> cnt, offs;
  zema::DBuf<unsigned long long> ent_cell;
  zema::DBuf<int> ent_prim, ent_body, bucket_lo, bucket_hi, big_list;
  zema::DBuf<double> ent_box;                 // sorted entries' boxes [n][6]
  zema::DBuf<int> q_cnt, q_off, q_big, q_item;  // query work items (query, cell)
  zema::DBuf<long long> tot_dev;                 // totals of the search's two count scans
  zema::DBuf<unsigned long long> pair_keys;
  zema::DBuf<int> counters;              // small device counters
  zema::SortBufs sort;
  std::vector<std::unique_ptr<zema::DBuf<int>>> scan_tmp;
  // ---- contact evaluation
  zema::DBuf<int> act_idx;               // compacted active candidate ids
  zema::DBuf<int> trip_cnt, trip_off;
  zema::DBuf<unsigned long long> trip_key;
  zema::DBuf<double> trip_val;           // [ntrip][9]
  zema::DBuf<double> item_h, item_g;     // per contact item: 12x12 Hessian, gradient
  zema::DBuf<double> body_force;         // [n_bodies][3] contact force sensing output
  zema::DBuf<double> e_pair, d_pair;     // per candidate energy / distance
  int n_act = 0;
  // contact matrix (CSR over nodes)
  int nnzc = 0;
  zema::DBuf<int> c_ptr, c_col, seg_start, seg_row;
  zema::DBuf<double> c_val;
  zema::DBuf<float> c_val32;
  // ---- friction (lagged)
  int nfric = 0;
  zema::DBuf<int> f_ids;       // [n][5]
  zema::DBuf<double> f_vals;   // [n][8] lambda, n, w
  zema::DBuf<double> f_xt;     // [n][12]
  zema::DBuf<int> f_ids2, fr_flag, fr_offs;  // partial rebuild of the table (batches)
  zema::DBuf<double> f_vals2, f_xt2;
  zema::DBuf<double> e_fric;
  // ---- PCG
  zema::DBuf<double> minv_soft;  // [9][nsv]
  zema::DBuf<double> minv_body;  // [nfree][144]
  zema::DBuf<double> pr, pz, pp0, pp1, pq, px;
  zema::DBuf<double> pdir2;  // second initial-guess direction of a batch's starting scenes
  zema::DBuf<double> res_q, res_r, res_d, res_out;  // FP64 residual check of the mixed form
  zema::DBuf<double> cg_z, cg_part;  // single-reduction PCG: node records, partials
  zema::DBuf<int4> cg_tab;   // its block layout: soft blocks (first row, rows, scene, slot)
  zema::DBuf<int2> cg_prng;  // per scene: partial slots
  zema::DBuf<int4> cg_binfo;  // per block: its scene's partial slots, scene, own slot
  std::vector<int> cg_key;
  int cg_nsoft_blocks = 0, cg_nslots = 0;
  int cg_rpb = 0;             // soft rows per block of that layout
  int tune_cg_rows = 0;       // requested rows per block (0: spread over the compute units)
  int n_cu = 0;               // compute units of the scene's device (0: not yet queried)
  double* poll_h = nullptr;  // pinned host copies of the PCG scalars (two slots)
  int poll_cap = 0;
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};  // timing of a replayed chunk
  zema::DBuf<double> partial;    // block partial sums
  zema::DBuf<double> scal;       // PCG scalars
  zema::DBuf<unsigned int> ticket;
  // ---- reductions / readback
  zema::DBuf<double> red;        // reduction results
  zema::DBuf<unsigned long long> umin;
  double* host_pinned = nullptr;  // small pinned readback area
  bool hess_valid = false;
  zema::KTimer kt[zema::KT_N];
  // ---- graph-captured PCG chunks
  bool use_graph = true;
  int tune_lanes = 4, tune_ublock = 256;   // launch shapes of the fused PCG kernels (form 0: 4 -> 8)
  int pcg_form = 1;                         // 1: single-reduction iteration, 0: two launches
  hipStream_t cap_st = nullptr;          // capture stream (default priority)
  zema::PcgGraph pcg_graph;               // captured chunk of PCG iterations
  zema::DBuf<unsigned char> mat_dev;     // matrix descriptors read by the captured kernels
  std::vector<unsigned char> mat_h;
  ~zema_scene();
};

namespace zema {

// -------- launch timing (api.cpp)
void kt_begin(zema_scene* s, int g);
void kt_end(zema_scene* s, int g, double bytes = 0.0);
void kt_fold(zema_scene* s);  // after a stream synchronisation: accumulate elapsed times
void kt_add(zema_scene* s, int g, double ms, double bytes, long long launches = 1);  // launches timed elsewhere

// -------- map / vectors (k_misc.hip)
void k_map_surface(zema_scene* s, const double* y, double* xs);
void k_surface_disp(zema_scene* s, const double* p, double* dx);
void k_axpy(zema_scene* s, int n, double a, const double* x, const double* y, double* out);  // out = y + a x
void k_scale(zema_scene* s, int n, double a, const double* x, double* out);
void k_iota(zema_scene* s, int* p, int64_t n);  // p[i] = i
void k_velocity(zema_scene* s, double inv_h);   // ydot = (y - yt) * inv_h
void k_velocity_to(zema_scene* s, double inv_h, double* out);  // (y - yt) * inv_h into out
void k_predict(zema_scene* s);                  // yhat from y^t, ydot^t
void k_predict_to(zema_scene* s, double* out);  // the prediction into out
void k_max_disp(zema_scene* s, const double* p, double* out);  // per scene: max vertex displacement of p
void k_axpy_scene(zema_scene* s, const double* alpha_host, const double* p, const double* y, double* out);
void k_select_scene(zema_scene* s, const int* mask_host, const double* a, const double* b, double* out);
void k_scale_scene(zema_scene* s, const double* alpha_host, double* p);
void k_scene_dots(zema_scene* s, const double* a, const double* b, double* out_host);  // per scene a.b, a.a, b.b
bool k_inverted(zema_scene* s, const double* y, int* out);  // per scene: any tet inverted
// multi-segment deterministic sums: out[k] = sum of seg k (host results)
// (extra: optional device word copied to out_host[nseg] in the same synchronisation)
void k_sums(zema_scene* s, int nseg, const double* const* ptr, const int64_t* len, double* out_host,
            const void* extra);
bool k_any_inverted(zema_scene* s, const double* y);

// -------- elastic (k_elastic.hip)
void k_tet_assemble(zema_scene* s, const double* y, bool hess);  // e_tet, g_tet, h_tet
void k_tet_energy(zema_scene* s, const double* y);               // e_tet only (inf if inverted)
void k_gather_grad_soft(zema_scene* s, const double* y, double* grad, unsigned mask);
void k_gather_hess_static(zema_scene* s, unsigned mask);
void k_inertia_energy(zema_scene* s, const double* y, double* e_out);

// -------- affine (k_affine.hip)
void k_body_terms(zema_scene* s, const double* y, double* grad, bool hess, unsigned mask);
void k_body_energy(zema_scene* s, const double* y);

// -------- contact (k_contact.hip)
// evaluate the current candidate set at xs: energies / distances; with derivatives,
// builds the contact matrix (CSR) and adds gradient contributions into grad.
void k_contact_energy(zema_scene* s);                 // e_pair, d_pair, e_fric at xs
void k_scene_sums(zema_scene* s, double* out_host);  // per scene [ns][8] energy terms, total, min distance
void k_contact_assemble(zema_scene* s, double* grad, bool hess, unsigned mask);
// springs (Sec. IV-C-3): per-spring energies at s->xs; gradient and Hessian added to the
// assembled ones (after the elastic gathers and the body terms)
void k_spring_energy(zema_scene* s);
void k_spring_terms(zema_scene* s, double* grad, bool hess);
// prismatic joints (Sec. IV-C-2): energies at y into e_out [n_joints]; their gradient
// and Hessian are emitted with the contact triplets (k_contact_assemble, mask bit 3)
void k_joint_energy(zema_scene* s, const double* y, double* e_out);
// contact force (N) on every body from the barrier items of the last assembly (host out)
void k_body_forces(zema_scene* s, double* out_host);
void k_friction_build(zema_scene* s);                 // lagged table from current candidates at xs
void k_friction_rebuild(zema_scene* s, const int* rebuild_host);  // the same for some scenes of a batch

// -------- broad phase (k_broad.hip)
void k_candidates(zema_scene* s, const double* xs0, const double* xs1, double r, const double* xs2 = nullptr);
void k_features(zema_scene* s, float* feat);
void k_cloth_energy(zema_scene* s, const double* y, double* e_out);  // per garment triangle
void k_cloth_emit(zema_scene* s, const double* y, bool hess, int64_t base, unsigned long long W,
                  unsigned long long* key, double* val);  // gradient (+ Hessian) triplets, 3 (12) per triangle
void k_warm_fit(zema_scene* s, int mode, float* out);   // per-soft-body fit of a correction field, in place
void k_warm_dir(zema_scene* s, float* out, double* p);  // applies the scene's fit to out first
void k_warm_target(zema_scene* s, float* target);
int64_t k_edge_tri_pairs(zema_scene* s, const double* xs, DBuf<int>& out);

// -------- intersection count (k_intersect.hip)
// counts of intersecting inter-body (edge, triangle) pairs, tets with J <= 0 and
// pairs / tets whose sign the floating-point filter cannot decide (listed in unc)
void k_intersections(zema_scene* s, const double* y, int64_t* n_int, int64_t* n_inv, int64_t* n_unc,
                     DBuf<int>& unc);

// -------- sort / scan (k_sort.hip)
int64_t k_exclusive_scan(zema_scene* s, const int* in, int* out, int64_t n, bool want_total = true);
void k_radix_sort(zema_scene* s, SortBufs& b, int64_t n, int key_bits);  // sorts (b.k0, b.v0) in place

// -------- sparse / PCG (k_sparse.hip)
void k_hess_matvec(zema_scene* s, const double* v, double* out);
// the Hessian as merged BSR (row_ptr, col, AoS 3x3 FP64 values); returns the block
// count and writes only when it fits cap
int64_t k_hessian_bsr(zema_scene* s, int* row_ptr, int* col, double* val, int64_t cap);
void k_build_precond(zema_scene* s);
int k_pcg(zema_scene* s, const double* rhs, double* sol, double rtol, int max_iter, int* iters, double* relres,
          int* breakdown = nullptr);
void k_autotune(zema_scene* s, int* lanes_out, int* ub_out, double* us_per_iter);
void k_pcg_batch(zema_scene* s, const double* rhs, double* sol, double rtol, int max_iter, const int* active_host,
                 int* iters, double* relres, int* status, int* breakdown = nullptr);
// the solve of every active scene with, in the mixed form, the FP64 residual check and
// refinement; breakdown[k]: the scene's solve ended at non-positive curvature
void k_pcg_solve(zema_scene* s, const double* rhs, double* sol, double rtol, int max_iter, const int* active_host,
                 int* iters, double* relres, int* status, int* breakdown);
void k_hess_matvec64(zema_scene* s, const double* v, double* out);  // FP64 accumulation

// -------- CCD (k_ccd.hip)
int k_ccd(zema_scene* s, const double* y, const double* p, double* alpha);

}  // namespace zema

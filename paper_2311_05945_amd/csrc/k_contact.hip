// Contact terms of the incremental potential: log-barrier pairs (Sec. III eqs.
// 4-5, edge-edge pairs mollified) and lagged smoothed friction (eqs. 9-10), with the
// soft-affine chain rule of eqs. 6-8: the 12x12 pair Hessian is projected to PSD in
// x-space and then mapped through the affine Jacobian J(x0) = [I | e_r x0^T].
//
// Assembly is deterministic: every active pair writes its y-space contributions as
// (row node, column node, 3x3 block) triplets and (node, 3-vector) gradient entries
// at scanned offsets; the triplets are radix-sorted by key and summed per key in
// sorted order into a CSR contact matrix over the 3-DOF nodes.
#include "geom.hpp"
#include "wave_jacobi.hpp"
#include "scene.hpp"

namespace zema {

__device__ inline void pair_slots(int k, int npt, const int* __restrict__ pt, const int* __restrict__ ee,
                                  const int* __restrict__ tris, const int* __restrict__ edges, int& kind, int sv[4],
                                  int& ea, int& eb) {
  if (k < npt) {
    kind = 0;
    int v = pt[2 * k], t = pt[2 * k + 1];
    sv[0] = v;
    sv[1] = tris[3 * t];
    sv[2] = tris[3 * t + 1];
    sv[3] = tris[3 * t + 2];
    ea = eb = -1;
  } else {
    kind = 1;
    int j = k - npt;
    ea = ee[2 * j];
    eb = ee[2 * j + 1];
    sv[0] = edges[2 * ea];
    sv[1] = edges[2 * ea + 1];
    sv[2] = edges[2 * eb];
    sv[3] = edges[2 * eb + 1];
  }
}

// ------------------------------------------------------------------ energies (line search)
// barrier energy and distance of every candidate pair; per-scene minimum distance
__global__ void contact_energy_kernel(int npt, int nee, const int* __restrict__ pt, const int* __restrict__ ee,
                                      const int* __restrict__ tris, const int* __restrict__ edges,
                                      const double* __restrict__ elen2, const double* __restrict__ xs,
                                      const double* __restrict__ kappa_sc, const int* __restrict__ sv_scene,
                                      double dhat, double* __restrict__ e_pair, double* __restrict__ d_pair,
                                      unsigned long long* __restrict__ dmin) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  double d = INFINITY;
  int sc = -1;
  if (k < npt + nee) {
    int kind, sv[4], ea, eb;
    pair_slots(k, npt, pt, ee, tris, edges, kind, sv, ea, eb);
    sc = sv_scene[sv[0]];
    V3 x[4];
    for (int a = 0; a < 4; ++a) x[a] = ld3(xs + 3 * sv[a]);
    double eps = kind == 1 ? 1e-3 * elen2[ea] * elen2[eb] : 0.0;
    e_pair[k] = pair_barrier_energy(kind, x, eps, kappa_sc[sc], dhat, &d);
    if (d != d) d = 0.0;  // a non-finite distance makes the state infeasible, never inactive
    d_pair[k] = d;
  }
  scene_atomic_ext<false>(dmin, sc, d);
}

// friction: f0 and the coefficients of the 3x3 core  alpha Pi - beta u u^T
__device__ inline double friction_core(double y, double ys, double& f1y, double& alpha, double& beta) {
  if (y < ys) {
    f1y = 2.0 / ys - y / (ys * ys);
    alpha = f1y;
    beta = y > 0.0 ? 1.0 / (ys * ys * y) : 0.0;
    return -y * y * y / (3.0 * ys * ys) + y * y / ys + ys / 3.0;
  }
  f1y = 1.0 / y;
  alpha = 1.0 / y;
  beta = 1.0 / (y * y * y);
  return y;
}

__device__ inline V3 friction_u(const double* __restrict__ fv, const double* __restrict__ xt, const V3* x) {
  V3 D = v3(0, 0, 0);
  for (int a = 0; a < 4; ++a) D = D + fv[4 + a] * (x[a] - ld3(xt + 3 * a));
  V3 n = ld3(fv + 1);
  return D - dot(n, D) * n;
}

__global__ void friction_energy_kernel(int nf, const int* __restrict__ fids, const double* __restrict__ fvals,
                                       const double* __restrict__ fxt, const double* __restrict__ xs,
                                       const double* __restrict__ mu_sc, const int* __restrict__ sv_scene, double ys,
                                       double* __restrict__ e) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const double mu = mu_sc[sv_scene[fids[5 * f + 1]]];
  V3 x[4];
  for (int a = 0; a < 4; ++a) x[a] = ld3(xs + 3 * fids[5 * f + 1 + a]);
  V3 u = friction_u(fvals + 8 * f, fxt + 12 * f, x);
  double y = sqrt(dot(u, u)), f1y, al, be;
  double f0 = friction_core(y, ys, f1y, al, be);
  e[f] = mu * fvals[8 * f] * f0;
}

// ------------------------------------------------------------------ lagged friction table
// only : per-scene flags of the scenes whose entries are built, or null for all
__global__ void friction_flag_kernel(int npt, int nee, const int* __restrict__ pt, const int* __restrict__ ee,
                                     const int* __restrict__ tris, const int* __restrict__ edges,
                                     const double* __restrict__ xs, double dhat, const int* __restrict__ only,
                                     const int* __restrict__ sv_scene, int* __restrict__ flag) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npt + nee) return;
  int kind, sv[4], ea, eb;
  pair_slots(k, npt, pt, ee, tris, edges, kind, sv, ea, eb);
  if (only && !only[sv_scene[sv[0]]]) {
    flag[k] = 0;
    return;
  }
  V3 x[4];
  for (int a = 0; a < 4; ++a) x[a] = ld3(xs + 3 * sv[a]);
  double d = pair_dist(kind, x, nullptr);
  flag[k] = (d < dhat && d > 0.0) ? 1 : 0;
}

// lambda = kappa m |b'(d)| (normal force in IP units), n = unit vector between the
// closest points, w = closest-point weights (PT: 1, -beta_i; EE: 1-ga, ga, -(1-gb), -gb)
__global__ void friction_fill_kernel(int npt, int nee, const int* __restrict__ pt, const int* __restrict__ ee,
                                     const int* __restrict__ tris, const int* __restrict__ edges,
                                     const double* __restrict__ elen2, const double* __restrict__ xs,
                                     const double* __restrict__ kappa_sc, const int* __restrict__ sv_scene,
                                     double dhat, const int* __restrict__ flag, const int* __restrict__ offs,
                                     int* __restrict__ fids, double* __restrict__ fvals, double* __restrict__ fxt) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npt + nee || !flag[k]) return;
  int f = offs[k];
  int kind, sv[4], ea, eb;
  pair_slots(k, npt, pt, ee, tris, edges, kind, sv, ea, eb);
  const double kappa = kappa_sc[sv_scene[sv[0]]];
  V3 x[4];
  for (int a = 0; a < 4; ++a) x[a] = ld3(xs + 3 * sv[a]);
  double w[4];
  V3 c0, c1;
  double m = 1.0;
  if (kind == 0) {
    double b[3];
    pt_closest_bary(x, b);
    w[0] = 1.0;
    w[1] = -b[0];
    w[2] = -b[1];
    w[3] = -b[2];
    c0 = x[0];
    c1 = b[0] * x[1] + b[1] * x[2] + b[2] * x[3];
  } else {
    double sa, tb;
    ee_type(x[0], x[1], x[2], x[3], &sa, &tb);
    w[0] = 1.0 - sa;
    w[1] = sa;
    w[2] = -(1.0 - tb);
    w[3] = -tb;
    c0 = (1.0 - sa) * x[0] + sa * x[1];
    c1 = (1.0 - tb) * x[2] + tb * x[3];
    V3 n = cross(x[1] - x[0], x[3] - x[2]);
    double m1, m2;
    mollifier(dot(n, n), 1e-3 * elen2[ea] * elen2[eb], m, m1, m2);
  }
  double d = pair_dist(kind, x, nullptr);
  double b, b1, b2;
  barrier3(d, dhat, b, b1, b2);
  V3 n = c0 - c1;
  double nn = sqrt(dot(n, n));
  n = nn > 0.0 ? (1.0 / nn) * n : v3(0, 0, 0);
  fids[5 * f] = kind;
  for (int a = 0; a < 4; ++a) fids[5 * f + 1 + a] = sv[a];
  fvals[8 * f] = nn > 0.0 ? kappa * m * fabs(b1) : 0.0;
  fvals[8 * f + 1] = n.x;
  fvals[8 * f + 2] = n.y;
  fvals[8 * f + 3] = n.z;
  for (int a = 0; a < 4; ++a) fvals[8 * f + 4 + a] = w[a];
  for (int a = 0; a < 4; ++a) {
    fxt[12 * f + 3 * a] = x[a].x;
    fxt[12 * f + 3 * a + 1] = x[a].y;
    fxt[12 * f + 3 * a + 2] = x[a].z;
  }
}

// ------------------------------------------------------------------ entities and emission
struct Ent {
  int n;            // number of entities
  int id[4];        // soft vertex id or -(body+1)
  int node0[4];     // first node
  int nn[4];        // nodes per entity (1 soft, 4 affine)
  int of_slot[4];   // entity of each slot, -1 for fixed
};

__device__ inline void entities(const int sv[4], const int* __restrict__ sv_ref, const int* __restrict__ bi, Ent& E) {
  E.n = 0;
  for (int a = 0; a < 4; ++a) {
    int r = sv_ref[sv[a]];
    int node0, nn;
    if (r >= 0) {
      node0 = r;
      nn = 1;
    } else {
      node0 = bi[4 * (-r - 1) + 2];
      nn = 4;
      if (node0 < 0) {
        E.of_slot[a] = -1;
        continue;
      }
    }
    int found = -1;
    for (int k = 0; k < E.n; ++k)
      if (E.id[k] == r) found = k;
    if (found < 0) {
      found = E.n++;
      E.id[found] = r;
      E.node0[found] = node0;
      E.nn[found] = nn;
    }
    E.of_slot[a] = found;
  }
}

__device__ inline int ent_dofs(const Ent& E) {
  int t = 0;
  for (int k = 0; k < E.n; ++k) t += E.nn[k];
  return t;
}

// item i < n_act: barrier pair act_idx[i]; else friction pair i - n_act
struct ItemArgs {
  int npt, nee, n_act, nfric;
  const int *pt, *ee, *tris, *edges, *act, *sv_ref, *bi, *fids;
  const double *elen2, *xs, *sv_x0, *fvals, *fxt;
  const double *kappa_sc, *mu_sc;
  const int *sv_scene, *active;
  double dhat, ys;
  int nn_total, hess;
};

__device__ inline void item_slots(const ItemArgs& A, int i, int& kind, int sv[4], int& ea, int& eb, bool& fric) {
  if (i < A.n_act) {
    fric = false;
    pair_slots(A.act[i], A.npt, A.pt, A.ee, A.tris, A.edges, kind, sv, ea, eb);
  } else {
    fric = true;
    int f = i - A.n_act;
    kind = A.fids[5 * f];
    for (int a = 0; a < 4; ++a) sv[a] = A.fids[5 * f + 1 + a];
    ea = eb = -1;
  }
}

// barrier pairs closer than dhat (of scenes still iterating, when a mask is given)
__global__ void active_flag_kernel(int n, int npt, const int* __restrict__ pt, const int* __restrict__ ee,
                                   const int* __restrict__ edges, const int* __restrict__ sv_scene,
                                   const int* __restrict__ active, const double* __restrict__ d_pair, double dhat,
                                   int* __restrict__ flag) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int f = d_pair[k] < dhat ? 1 : 0;
  if (f && active) f = active[sv_scene[k < npt ? pt[2 * k] : edges[2 * ee[2 * (k - npt)]]]];
  flag[k] = f;
}

__global__ void compact_kernel(int n, const int* __restrict__ flag, const int* __restrict__ offs, int* __restrict__ out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && flag[k]) out[offs[k]] = k;
}

__global__ void item_count_kernel(ItemArgs A, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n_act + A.nfric) return;
  int kind, sv[4], ea, eb;
  bool fric;
  item_slots(A, i, kind, sv, ea, eb, fric);
  Ent E;
  entities(sv, A.sv_ref, A.bi, E);
  int nd = ent_dofs(E);
  cnt[i] = nd + (A.hess ? nd * nd : 0);
}

// K1: one wavefront per item: gradient (12) and full 12x12 Hessian in x-space.  Lane 0
// classifies the pair and forms the variable-space derivatives of the squared
// distance (and of the edge-edge mollifier's argument) in LDS, with the barrier's
// scalar factors; then every lane forms its entries of the slot-space gradient and
// Hessian (barrier: kappa (m (b'' terms + b' terms) + mollifier terms); friction:
// c w_a w_b core).  Barrier pairs store the unprojected Hessian (projected by K2);
// friction Hessians are PSD by construction.
__global__ void __launch_bounds__(64) pair_deriv_kernel(ItemArgs A, double* __restrict__ hout,
                                                        double* __restrict__ gout) {
  __shared__ DVars Dd, Dc, Dw;          // distance, mollifier argument, scratch
  __shared__ double gD[12], gC[12];     // slot gradients of D and of the mollifier argument
  __shared__ double fw[4], core[9], U3[3];
  __shared__ double k_cg, k_ch, k_kappa, k_m, k_m1, k_m2, k_b, k_c, k_cf;
  __shared__ int mode;                  // 0 zero, 1 barrier, 2 mollified barrier, 3 friction
  const int i = blockIdx.x, lane = threadIdx.x;
  if (i >= A.n_act + A.nfric) return;
  if (lane == 0) {
    int kind, sv[4], ea, eb;
    bool fric;
    item_slots(A, i, kind, sv, ea, eb, fric);
    mode = 0;
    if (!(fric && A.active && !A.active[A.sv_scene[sv[0]]])) {  // else a converged scene of a batch
      V3 x[4];
      for (int a = 0; a < 4; ++a) x[a] = ld3(A.xs + 3 * sv[a]);
      if (!fric) {
        int type;
        double d = pair_dist(kind, x, &type);
        if (d < A.dhat) {
          double D = d2_vars(kind, type, x, Dd);
          d = sqrt(D);
          double b, b1, b2;
          barrier3(d, A.dhat, b, b1, b2);
          k_cg = b1 / (2.0 * d);
          k_ch = b2 / (4.0 * D) - b1 / (4.0 * D * d);
          k_kappa = A.kappa_sc[A.sv_scene[sv[0]]];
          k_b = b;
          mode = 1;
          if (kind == 1) {
            const double eps = 1e-3 * A.elen2[ea] * A.elen2[eb];
            V3 u = x[1] - x[0], v = x[3] - x[2];
            V3 nn = cross(u, v);
            double c = dot(nn, nn);
            if (c < eps) {
              double m, m1, m2;
              mollifier(c, eps, m, m1, m2);
              k_m = m;
              k_m1 = m1;
              k_m2 = m2;
              // gradient / Hessian of c = |u x v|^2 with u = a1 - a0, v = b1 - b0
              dvar_triple(x[2] - x[0], u, v, Dw, &Dc);
              Dc.C[0][2] = 1;
              Dc.C[0][0] = -1;
              Dc.C[1][1] = 1;
              Dc.C[1][0] = -1;
              Dc.C[2][3] = 1;
              Dc.C[2][2] = -1;
              mode = 2;
            }
          }
        }
      } else {
        int f = i - A.n_act;
        const double* fv = A.fvals + 8 * f;
        V3 u = friction_u(fv, A.fxt + 12 * f, x);
        double y = sqrt(dot(u, u)), f1y, al, be;
        friction_core(y, A.ys, f1y, al, be);
        const double c = A.mu_sc[A.sv_scene[sv[0]]] * fv[0];
        V3 n = ld3(fv + 1);
        double N[3] = {n.x, n.y, n.z};
        U3[0] = u.x;
        U3[1] = u.y;
        U3[2] = u.z;
        for (int a = 0; a < 4; ++a) fw[a] = fv[4 + a];
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) core[3 * r + q] = al * ((r == q ? 1.0 : 0.0) - N[r] * N[q]) - be * U3[r] * U3[q];
        k_c = c;
        k_cf = c * f1y;
        mode = 3;
      }
    }
  }
  __syncthreads();
  const int md = mode;
  if ((md == 1 || md == 2) && lane < 12) {
    gD[lane] = dv_grad_entry(Dd, lane / 3, lane % 3);
    if (md == 2) gC[lane] = dv_grad_entry(Dc, lane / 3, lane % 3);
  }
  __syncthreads();
  if (lane < 12) {
    double g = 0.0;
    if (md == 1 || md == 2) {
      g = k_cg * gD[lane];
      if (md == 2) g = k_m * g + k_b * k_m1 * gC[lane];
      g *= k_kappa;
    } else if (md == 3) {
      g = k_cf * fw[lane / 3] * U3[lane % 3];
    }
    gout[(size_t)12 * i + lane] = g;
  }
  if (!A.hess) return;
  for (int e = lane; e < 144; e += 64) {
    const int r = e / 12, q = e % 12;
    double H = 0.0;
    if (md == 1 || md == 2) {
      H = k_ch * gD[r] * gD[q] + k_cg * dv_hess_entry(Dd, r / 3, r % 3, q / 3, q % 3);
      if (md == 2) {
        const double gr = k_cg * gD[r], gq = k_cg * gD[q];
        H = k_m * H + k_m1 * (gr * gC[q] + gC[r] * gq) +
            k_b * (k_m2 * gC[r] * gC[q] + k_m1 * dv_hess_entry(Dc, r / 3, r % 3, q / 3, q % 3));
      }
      H *= k_kappa;
    } else if (md == 3) {
      H = k_c * fw[r / 3] * fw[q / 3] * core[3 * (r % 3) + q % 3];
    }
    hout[(size_t)144 * i + e] = H;
  }
}

// K2: one wavefront (block of 64) per item.  Barrier Hessians are projected to PSD by
// parallel cyclic Jacobi in LDS (six disjoint rotations per round, the update
// A <- J^T A J and V <- V J applied to all 144 entries by the 64 lanes); then the
// item's node-pair blocks J_a^T P_ab J_b and gradient entries J_a^T g_a are emitted
// with the lanes splitting the blocks.
constexpr int LDA = 13;
__global__ void __launch_bounds__(64) project_emit_kernel(ItemArgs A, const double* __restrict__ hin,
                                                          const double* __restrict__ gin,
                                                          const int* __restrict__ offs,
                                                          unsigned long long* __restrict__ key,
                                                          double* __restrict__ val) {
  __shared__ double M[12 * LDA], Vm[12 * LDA], G[12], X0[12], cs[24];
  __shared__ int partner[12];
  const int i = blockIdx.x, lane = threadIdx.x;
  if (i >= A.n_act + A.nfric) return;
  int kind, sv[4], ea, eb;
  bool fric;
  item_slots(A, i, kind, sv, ea, eb, fric);
  if (lane < 12) {
    G[lane] = gin[(size_t)12 * i + lane];
    X0[lane] = A.sv_x0[3 * sv[lane / 3] + lane % 3];
  }
  if (A.hess) {
    for (int e = lane; e < 144; e += 64) M[(e / 12) * LDA + e % 12] = hin[(size_t)144 * i + e];
    __syncthreads();
    if (!fric) wave_psd_project<12, LDA>(M, Vm, cs, partner, lane);  // block-uniform branch
  }
  __syncthreads();
  // node list of the item: entities (soft vertex: one node; free affine body: p, a1..a3)
  Ent E;
  entities(sv, A.sv_ref, A.bi, E);
  int nd = ent_dofs(E);
  int ntot = nd + (A.hess ? nd * nd : 0);
  unsigned long long W = (unsigned long long)A.nn_total + 1;
  int o0 = offs[i];
  for (int t = lane; t < ntot; t += 64) {
    int o = o0 + t;
    if (t < nd) {
      int e = 0, j = t;
      while (j >= E.nn[e]) j -= E.nn[e++];
      double acc[3] = {0, 0, 0};
#pragma unroll 1
      for (int a = 0; a < 4; ++a) {
        if (E.of_slot[a] != e) continue;
        if (E.nn[e] == 1 || j == 0) {
          for (int c = 0; c < 3; ++c) acc[c] += G[3 * a + c];
        } else {
          double gr = G[3 * a + j - 1];
          for (int c = 0; c < 3; ++c) acc[c] += X0[3 * a + c] * gr;
        }
      }
      key[o] = (unsigned long long)(E.node0[e] + j) * W + (unsigned long long)A.nn_total;
      for (int c = 0; c < 3; ++c) val[(size_t)9 * o + c] = acc[c];
      for (int c = 3; c < 9; ++c) val[(size_t)9 * o + c] = 0.0;
    } else {
      int bidx = t - nd, n = bidx / nd, m = bidx % nd;
      int e = 0, j = n, f = 0, l = m;
      while (j >= E.nn[e]) j -= E.nn[e++];
      while (l >= E.nn[f]) l -= E.nn[f++];
      bool Ij = (E.nn[e] == 1 || j == 0), Il = (E.nn[f] == 1 || l == 0);
      double K[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 1
      for (int a = 0; a < 4; ++a) {
        if (E.of_slot[a] != e) continue;
#pragma unroll 1
        for (int b = 0; b < 4; ++b) {
          if (E.of_slot[b] != f) continue;
          const double* P = M + (3 * a) * LDA + 3 * b;  // P_ab[r][c] = P[r * LDA + c]
          if (Ij && Il) {
            for (int r = 0; r < 3; ++r)
              for (int c = 0; c < 3; ++c) K[3 * r + c] += P[r * LDA + c];
          } else if (Ij) {  // P_ab e_s x0_b^T
            int sI = l - 1;
            for (int r = 0; r < 3; ++r)
              for (int c = 0; c < 3; ++c) K[3 * r + c] += P[r * LDA + sI] * X0[3 * b + c];
          } else if (Il) {  // x0_a e_r^T P_ab
            int rI = j - 1;
            for (int r = 0; r < 3; ++r)
              for (int c = 0; c < 3; ++c) K[3 * r + c] += X0[3 * a + r] * P[rI * LDA + c];
          } else {  // P_ab[r][s] x0_a x0_b^T
            double prs = P[(j - 1) * LDA + (l - 1)];
            for (int r = 0; r < 3; ++r)
              for (int c = 0; c < 3; ++c) K[3 * r + c] += prs * X0[3 * a + r] * X0[3 * b + c];
          }
        }
      }
      key[o] = (unsigned long long)(E.node0[e] + j) * W + (unsigned long long)(E.node0[f] + l);
      for (int q = 0; q < 9; ++q) val[(size_t)9 * o + q] = K[q];
    }
  }
}

// segment heads of sorted keys: head[j] = 1 if key differs from the previous one;
// hess_head additionally requires a Hessian key (column < nn)
__global__ void heads_kernel(int n, const unsigned long long* __restrict__ k, unsigned long long W, int* __restrict__ head,
                             int* __restrict__ hhead) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  bool h = (j == 0) || (k[j] != k[j - 1]);
  head[j] = h ? 1 : 0;
  hhead[j] = (h && (k[j] % W) != W - 1) ? 1 : 0;
}

__global__ void seg_start_kernel(int n, const int* __restrict__ head, const int* __restrict__ sid,
                                 int* __restrict__ start) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n && head[j]) start[sid[j]] = j;
}

// one wavefront per segment: lanes sum strided entries in sorted order, then a fixed
// shuffle tree; gradient keys add into grad, Hessian keys become CSR entries
template <class T>
__global__ void seg_reduce_kernel(int nseg, int n, const int* __restrict__ start, const unsigned long long* __restrict__ k,
                                  const int* __restrict__ perm, const double* __restrict__ val, unsigned long long W,
                                  const int* __restrict__ hid, double* __restrict__ grad, int* __restrict__ crow,
                                  int* __restrict__ ccol, T* __restrict__ cval, int nnzc) {
  int u = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (u >= nseg) return;
  int j0 = start[u], j1 = u + 1 < nseg ? start[u + 1] : n;
  unsigned long long key = k[j0];
  int row = (int)(key / W), col = (int)(key % W);
  bool is_grad = (unsigned long long)col == W - 1;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int j = j0 + lane; j < j1; j += 64) {
    const double* v = val + (size_t)9 * perm[j];
    for (int q = 0; q < 9; ++q) acc[q] += v[q];
  }
  for (int q = 0; q < 9; ++q) acc[q] = wave_sum(acc[q]);
  if (lane != 0) return;
  if (is_grad) {
    if (grad)
      for (int q = 0; q < 3; ++q) grad[3 * row + q] += acc[q];
  } else {
    int h = hid[j0];
    crow[h] = row;
    ccol[h] = col;
    for (int q = 0; q < 9; ++q) cval[(size_t)q * nnzc + h] = T(acc[q]);
  }
}

__global__ void row_ptr_kernel(int nrows, int nnzc, const int* __restrict__ crow, int* __restrict__ cptr) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r > nrows) return;
  int lo = 0, hi = nnzc;  // first index with crow >= r
  while (lo < hi) {
    int m = (lo + hi) >> 1;
    if (crow[m] < r)
      lo = m + 1;
    else
      hi = m;
  }
  cptr[r] = lo;
}

// ------------------------------------------------------------------ per-scene energy sums (batches)
// Candidate and friction lists are sorted by the scene-major surface numbering, so
// every scene owns one run of PT pairs, one of EE pairs and (PT items first) one run
// of each friction kind; run bounds go to rng[8 sc + slot], rng[8 sc + slot + 1].
__global__ void runs_kernel(int mode, int n, int base, const int* __restrict__ a, const int* __restrict__ edges,
                            const int* __restrict__ sv_scene, int ns, int* __restrict__ rng) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto key = [&](int j, int& sc, int& slot) {
    if (mode == 0) {
      sc = sv_scene[a[2 * j]];
      slot = 0;
    } else if (mode == 1) {
      sc = sv_scene[edges[2 * a[2 * j]]];
      slot = 2;
    } else {
      int kind = a[5 * j];
      sc = sv_scene[a[5 * j + 1]];
      slot = 4 + 2 * kind;
    }
    return slot * ns + sc;
  };
  int sc, slot, o1, o2;
  int k = key(i, sc, slot);
  if (i == 0 || key(i - 1, o1, o2) != k) rng[8 * sc + slot] = base + i;
  if (i == n - 1 || key(i + 1, o1, o2) != k) rng[8 * sc + slot + 1] = base + i + 1;
}

constexpr int kSumParts = 32;  // blocks per scene of the energy sums

// part p of kSumParts equal contiguous parts of [lo, hi)
__device__ inline double range_part_sum(const double* __restrict__ a, int lo, int hi, int p, double* sh) {
  const int64_t len = hi - lo;
  const int a0 = lo + (int)(len * p / kSumParts), a1 = lo + (int)(len * (p + 1) / kSumParts);
  double acc = 0.0;
  for (int i = a0 + threadIdx.x; i < a1; i += kBlock) acc += a[i];
  return block_sum<kBlock>(acc, sh);
}

// block (p, k): part p of every energy array range of scene k -> part[k][p][6]
// (inertia, elastic, orthogonality, kinematic, barrier, friction)
__global__ void scene_sums_kernel(const int* __restrict__ srng, const int* __restrict__ drng,
                                  const double* __restrict__ e_in, const double* __restrict__ e_tet,
                                  const double* __restrict__ e_body, int nb, const double* __restrict__ e_pair,
                                  const double* __restrict__ e_fric, double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  const int p = blockIdx.x, k = blockIdx.y;
  const int* R = srng + 8 * k;
  const int* D = drng + 8 * k;
  double in_s = range_part_sum(e_in, R[0], R[1], p, sh);
  double in_b = range_part_sum(e_body, R[4], R[5], p, sh);
  double el = range_part_sum(e_tet, R[2], R[3], p, sh);
  double orth = range_part_sum(e_body + nb, R[4], R[5], p, sh);
  double kin = range_part_sum(e_body + 2 * nb, R[4], R[5], p, sh);
  double bar = range_part_sum(e_pair, D[0], D[1], p, sh) + range_part_sum(e_pair, D[2], D[3], p, sh);
  double fr = range_part_sum(e_fric, D[4], D[5], p, sh) + range_part_sum(e_fric, D[6], D[7], p, sh);
  if (threadIdx.x == 0) {
    double* o = part + 6 * ((size_t)k * kSumParts + p);
    o[0] = in_s + in_b;
    o[1] = el;
    o[2] = orth;
    o[3] = kin;
    o[4] = bar;
    o[5] = fr;
  }
}

// one wavefront per scene: T[0] inertia, 1 elastic, 2 orthogonality, 3 kinematic,
// 4 barrier, 5 friction, 6 total, 7 minimum distance (+inf without pairs); the parts
// are added in order
__global__ void scene_sums_fin(int ns, const double* __restrict__ part, const unsigned long long* __restrict__ dmin,
                               double* __restrict__ out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ns) return;
  double t[6] = {0, 0, 0, 0, 0, 0};
  for (int p = 0; p < kSumParts; ++p)
    for (int q = 0; q < 6; ++q) t[q] += part[6 * ((size_t)k * kSumParts + p) + q];
  double* T = out + 8 * k;
  for (int q = 0; q < 6; ++q) T[q] = t[q];
  T[6] = T[0] + T[1] + T[2] + T[3] + T[4] + T[5];
  unsigned long long u = dmin[k];
  T[7] = u == ~0ull ? INFINITY : __longlong_as_double((long long)u);
}

void k_scene_sums(zema_scene* s, double* out_host) {
  const int ns = s->ns;
  ZCHK(hipMemsetAsync(s->sc_rng.p, 0, sizeof(int) * 8 * ns, s->st));
  if (s->npt)
    runs_kernel<<<nblocks(s->npt), kBlock, 0, s->st>>>(0, (int)s->npt, 0, s->pt.p, s->edges.p, s->sv_scene.p, ns,
                                                       s->sc_rng.p);
  if (s->nee)
    runs_kernel<<<nblocks(s->nee), kBlock, 0, s->st>>>(1, (int)s->nee, (int)s->npt, s->ee.p, s->edges.p,
                                                       s->sv_scene.p, ns, s->sc_rng.p);
  if (s->nfric)
    runs_kernel<<<nblocks(s->nfric), kBlock, 0, s->st>>>(2, s->nfric, 0, s->f_ids.p, s->edges.p, s->sv_scene.p, ns,
                                                         s->sc_rng.p);
  int nb = (int)s->bodies.size();
  s->sc_part.reserve((size_t)6 * kSumParts * ns);
  scene_sums_kernel<<<dim3(kSumParts, ns), kBlock, 0, s->st>>>(s->scn_rng.p, s->sc_rng.p, s->e_in.p, s->e_tet.p,
                                                                s->e_body.p, nb, s->e_pair.p, s->e_fric.p,
                                                                s->sc_part.p);
  scene_sums_fin<<<nblocks(ns), kBlock, 0, s->st>>>(ns, s->sc_part.p, s->sc_dmin.p, s->sc_sum.p);
  ZCHK(hipMemcpyAsync(out_host, s->sc_sum.p, sizeof(double) * 8 * ns, hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
}

// ------------------------------------------------------------------ prismatic joints
// Sec. IV-C-2: E = kappa (|A1 - A2|_F^2 + |r x u|^2), u = A1 d (d in b1's rest frame),
// r = p1 - (A2 (c1 - c2) + p2) the gap between the two bodies' images of b1's rest
// centre of mass c1 (x0 is measured from each body's centre).  Residuals R (12): the
// 9 entries of A1 - A2 and the 3 of r x u; Jacobian Jm [12][24] over (q1, q2); Hessian
// the Gauss-Newton matrix 2 kappa Jm^T Jm.
__device__ inline void joint_residuals(const double* q1, const double* q2, const double* d, const double* dc,
                                       double R[12], double Jm[12][24]) {
  for (int i = 0; i < 12; ++i)
    for (int k = 0; k < 24; ++k) Jm[i][k] = 0.0;
  for (int k = 0; k < 9; ++k) {
    R[k] = q1[3 + k] - q2[3 + k];
    Jm[k][3 + k] = 1.0;
    Jm[k][15 + k] = -1.0;
  }
  double r[3], u[3], dr[3][24], du[3][24];
  for (int i = 0; i < 3; ++i) {
    for (int k = 0; k < 24; ++k) dr[i][k] = du[i][k] = 0.0;
    r[i] = q1[i] - q2[i];
    u[i] = 0.0;
    dr[i][i] = 1.0;
    dr[i][12 + i] = -1.0;
    for (int j = 0; j < 3; ++j) {
      r[i] -= dc[j] * q2[3 + 3 * i + j];
      dr[i][15 + 3 * i + j] = -dc[j];
      u[i] += d[j] * q1[3 + 3 * i + j];
      du[i][3 + 3 * i + j] = d[j];
    }
  }
  for (int i = 0; i < 3; ++i) {
    const int a = (i + 1) % 3, b = (i + 2) % 3;  // w_i = r_a u_b - r_b u_a
    R[9 + i] = r[a] * u[b] - r[b] * u[a];
    for (int k = 0; k < 24; ++k) Jm[9 + i][k] = u[b] * dr[a][k] + r[a] * du[b][k] - u[a] * dr[b][k] - r[b] * du[a][k];
  }
}

struct JointArgs {
  int nj;
  const int* ji;       // [nj][4]: b1, b2, triplet offset within the joints' block with / without Hessian
  const double* jd;    // [nj][8]: d (3), kappa, c1 - c2 (3), 0
  const double* bf;    // body records (fixed q)
  const int* bi;       // body ints (mode, dof0, node0)
  const double* y;
};

__device__ inline const double* joint_q(const JointArgs& J, int b) {
  const int dof0 = J.bi[4 * b + 1];
  return dof0 >= 0 ? J.y + dof0 : J.bf + BF * b + BF_QF;
}

__global__ void joint_energy_kernel(JointArgs J, double* __restrict__ e) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J.nj) return;
  double R[12], Jm[12][24];
  joint_residuals(joint_q(J, J.ji[4 * j]), joint_q(J, J.ji[4 * j + 1]), J.jd + 8 * j, J.jd + 8 * j + 4, R, Jm);
  double acc = 0.0;
  for (int i = 0; i < 12; ++i) acc += R[i] * R[i];
  e[j] = J.jd[8 * j + 3] * acc;
}

// one thread per joint: gradient triplets (node, n_nodes) and, with hess, the node-pair
// blocks of 2 kappa Jm^T Jm, for the nodes of the joint's non-fixed bodies
__global__ void joint_emit_kernel(JointArgs J, int hess, int64_t base, unsigned long long W, int nn_total,
                                  unsigned long long* __restrict__ key, double* __restrict__ val) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J.nj) return;
  const int b[2] = {J.ji[4 * j], J.ji[4 * j + 1]};
  const double kappa = J.jd[8 * j + 3];
  double R[12], Jm[12][24];
  joint_residuals(joint_q(J, b[0]), joint_q(J, b[1]), J.jd + 8 * j, J.jd + 8 * j + 4, R, Jm);
  int node[8], nn = 0, loc[8];  // nodes of non-fixed bodies and their first local index
  for (int k = 0; k < 2; ++k) {
    const int dof0 = J.bi[4 * b[k] + 1], node0 = J.bi[4 * b[k] + 2];
    if (dof0 < 0) continue;
    for (int m = 0; m < 4; ++m) {
      node[nn] = node0 + m;
      loc[nn] = 12 * k + 3 * m;
      ++nn;
    }
  }
  int64_t o = base + J.ji[4 * j + (hess ? 2 : 3)];
  for (int a = 0; a < nn; ++a, ++o) {
    key[o] = (unsigned long long)node[a] * W + (unsigned long long)nn_total;
    for (int c = 0; c < 3; ++c) {
      double g = 0.0;
      for (int i = 0; i < 12; ++i) g += Jm[i][loc[a] + c] * R[i];
      val[(size_t)9 * o + c] = 2.0 * kappa * g;
    }
    for (int c = 3; c < 9; ++c) val[(size_t)9 * o + c] = 0.0;
  }
  if (!hess) return;
  for (int a = 0; a < nn; ++a)
    for (int bb = 0; bb < nn; ++bb, ++o) {
      key[o] = (unsigned long long)node[a] * W + (unsigned long long)node[bb];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double h = 0.0;
          for (int i = 0; i < 12; ++i) h += Jm[i][loc[a] + r] * Jm[i][loc[bb] + c];
          val[(size_t)9 * o + 3 * r + c] = 2.0 * kappa * h;
        }
    }
}

static JointArgs joint_args(zema_scene* s, const double* y) {
  JointArgs J;
  J.nj = (int)s->joints.size();
  J.ji = s->jnt_i.p;
  J.jd = s->jnt_d.p;
  J.bf = s->body_f.p;
  J.bi = s->body_i.p;
  J.y = y;
  return J;
}

void k_joint_energy(zema_scene* s, const double* y, double* e_out) {
  const int nj = (int)s->joints.size();
  if (nj) joint_energy_kernel<<<nblocks(nj, 64), 64, 0, s->st>>>(joint_args(s, y), e_out);
}

// ------------------------------------------------------------------ contact force sensing
// Sec. IV-B: the force on a surface vertex is -dB/dx / h^2 (B the barrier energy of
// eq. 4 in incremental-potential units), and the resultant on a body the sum over its
// surface vertices.  One workgroup per body walks the active barrier items in order;
// item i's x-space gradient (12 slot entries) was written by pair_deriv_kernel.
__global__ void body_force_kernel(int n_act, ItemArgs A, const int* __restrict__ sv_body,
                                  const double* __restrict__ item_g, double inv_h2, double* __restrict__ out) {
  __shared__ double sh[kBlock / 64];
  const int b = blockIdx.x;
  double f[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n_act; i += kBlock) {
    int kind, sv[4], ea, eb;
    bool fric;
    item_slots(A, i, kind, sv, ea, eb, fric);
    for (int a = 0; a < 4; ++a)
      if (sv_body[sv[a]] == b)
        for (int k = 0; k < 3; ++k) f[k] += item_g[(size_t)12 * i + 3 * a + k];
  }
  for (int k = 0; k < 3; ++k) {
    const double t = block_sum<kBlock>(f[k], sh);
    if (threadIdx.x == 0) out[3 * b + k] = -t * inv_h2;
  }
}

void k_body_forces(zema_scene* s, double* out_host) {
  const int nb = s->n_bodies;
  s->body_force.reserve((size_t)3 * std::max(nb, 1));
  ItemArgs A{};
  A.npt = (int)s->npt;
  A.nee = (int)s->nee;
  A.n_act = s->n_act;
  A.nfric = 0;
  A.pt = s->pt.p;
  A.ee = s->ee.p;
  A.tris = s->tris.p;
  A.edges = s->edges.p;
  A.act = s->act_idx.p;
  if (nb > 0)
    body_force_kernel<<<nb, kBlock, 0, s->st>>>(s->n_act, A, s->sv_body.p, s->item_g.p,
                                                1.0 / (s->P.dt * s->P.dt), s->body_force.p);
  ZCHK(hipMemcpyAsync(out_host, s->body_force.p, sizeof(double) * 3 * nb, hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
}

// ------------------------------------------------------------------ launchers
static int bits_for(unsigned long long v) {
  int b = 0;
  while (b < 64 && (v >> b)) ++b;
  return b;
}

void k_contact_energy(zema_scene* s) {
  int nc = (int)(s->npt + s->nee);
  s->e_pair.reserve(nc + 1);
  s->d_pair.reserve(nc + 1);
  // all-ones bits: no pair in the scene (read back as +infinity)
  ZCHK(hipMemsetAsync(s->sc_dmin.p, 0xff, sizeof(unsigned long long) * s->ns, s->st));
  if (nc)
    contact_energy_kernel<<<nblocks(nc), kBlock, 0, s->st>>>((int)s->npt, (int)s->nee, s->pt.p, s->ee.p, s->tris.p,
                                                             s->edges.p, s->elen2.p, s->xs.p, s->kappa_sc.p,
                                                             s->sv_scene.p, s->P.dhat, s->e_pair.p, s->d_pair.p,
                                                             s->sc_dmin.p);
  s->e_fric.reserve(s->nfric + 1);
  if (s->nfric)
    friction_energy_kernel<<<nblocks(s->nfric), kBlock, 0, s->st>>>(s->nfric, s->f_ids.p, s->f_vals.p, s->f_xt.p,
                                                                     s->xs.p, s->mu_sc.p, s->sv_scene.p,
                                                                     s->P.eps_v * s->P.dt, s->e_fric.p);
}

void k_friction_build(zema_scene* s) {
  int nc = (int)(s->npt + s->nee);
  s->nfric = 0;
  if (!nc) return;
  s->cnt.reserve(nc + 1);
  s->offs.reserve(nc + 1);
  friction_flag_kernel<<<nblocks(nc), kBlock, 0, s->st>>>((int)s->npt, (int)s->nee, s->pt.p, s->ee.p, s->tris.p,
                                                          s->edges.p, s->xs.p, s->P.dhat, nullptr, s->sv_scene.p,
                                                          s->cnt.p);
  int64_t nf = k_exclusive_scan(s, s->cnt.p, s->offs.p, nc);
  s->nfric = (int)nf;
  s->f_ids.reserve(5 * nf + 5);
  s->f_vals.reserve(8 * nf + 8);
  s->f_xt.reserve(12 * nf + 12);
  if (nf)
    friction_fill_kernel<<<nblocks(nc), kBlock, 0, s->st>>>((int)s->npt, (int)s->nee, s->pt.p, s->ee.p, s->tris.p,
                                                            s->edges.p, s->elen2.p, s->xs.p, s->kappa_sc.p,
                                                            s->sv_scene.p, s->P.dhat, s->cnt.p, s->offs.p, s->f_ids.p,
                                                            s->f_vals.p, s->f_xt.p);
}

// entries of the scenes that keep their table: flag = 1
__global__ void friction_keep_kernel(int nf, const int* __restrict__ fids, const int* __restrict__ sv_scene,
                                     const int* __restrict__ rebuild, int* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nf) flag[i] = rebuild[sv_scene[fids[5 * i + 1]]] ? 0 : 1;
}

__global__ void friction_move_kernel(int nf, const int* __restrict__ flag, const int* __restrict__ offs,
                                     const int* __restrict__ fids, const double* __restrict__ fvals,
                                     const double* __restrict__ fxt, int* __restrict__ oids, double* __restrict__ ovals,
                                     double* __restrict__ oxt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf || !flag[i]) return;
  int o = offs[i];
  for (int q = 0; q < 5; ++q) oids[5 * (size_t)o + q] = fids[5 * (size_t)i + q];
  for (int q = 0; q < 8; ++q) ovals[8 * (size_t)o + q] = fvals[8 * (size_t)i + q];
  for (int q = 0; q < 12; ++q) oxt[12 * (size_t)o + q] = fxt[12 * (size_t)i + q];
}

// Rebuilds the lagged friction entries of the scenes flagged in rebuild_host from the
// current candidates at s->xs (their state at the start of their step) and keeps the
// entries of every other scene: kept entries first, in their order, then the new ones
// in pair order, so each scene's point-triangle and edge-edge entries stay contiguous.
void k_friction_rebuild(zema_scene* s, const int* rebuild_host) {
  const int ns = s->ns;
  ZCHK(hipMemcpyAsync(s->sc_mask.p, rebuild_host, sizeof(int) * ns, hipMemcpyHostToDevice, s->st));
  const int nold = s->nfric;
  int64_t nk = 0;
  s->fr_flag.reserve(nold + 1);
  s->fr_offs.reserve(nold + 1);
  if (nold) {
    friction_keep_kernel<<<nblocks(nold), kBlock, 0, s->st>>>(nold, s->f_ids.p, s->sv_scene.p, s->sc_mask.p,
                                                              s->fr_flag.p);
    nk = k_exclusive_scan(s, s->fr_flag.p, s->fr_offs.p, nold);
  }
  const int nc = (int)(s->npt + s->nee);
  int64_t nn = 0;
  s->cnt.reserve(nc + 1);
  s->offs.reserve(nc + 1);
  if (nc) {
    friction_flag_kernel<<<nblocks(nc), kBlock, 0, s->st>>>((int)s->npt, (int)s->nee, s->pt.p, s->ee.p, s->tris.p,
                                                            s->edges.p, s->xs.p, s->P.dhat, s->sc_mask.p,
                                                            s->sv_scene.p, s->cnt.p);
    nn = k_exclusive_scan(s, s->cnt.p, s->offs.p, nc);
  }
  const int64_t nf = nk + nn;
  s->f_ids2.reserve(5 * nf + 5);
  s->f_vals2.reserve(8 * nf + 8);
  s->f_xt2.reserve(12 * nf + 12);
  if (nk)
    friction_move_kernel<<<nblocks(nold), kBlock, 0, s->st>>>(nold, s->fr_flag.p, s->fr_offs.p, s->f_ids.p,
                                                              s->f_vals.p, s->f_xt.p, s->f_ids2.p, s->f_vals2.p,
                                                              s->f_xt2.p);
  if (nn)
    friction_fill_kernel<<<nblocks(nc), kBlock, 0, s->st>>>((int)s->npt, (int)s->nee, s->pt.p, s->ee.p, s->tris.p,
                                                            s->edges.p, s->elen2.p, s->xs.p, s->kappa_sc.p,
                                                            s->sv_scene.p, s->P.dhat, s->cnt.p, s->offs.p,
                                                            s->f_ids2.p + 5 * nk, s->f_vals2.p + 8 * nk,
                                                            s->f_xt2.p + 12 * nk);
  std::swap(s->f_ids.p, s->f_ids2.p);
  std::swap(s->f_ids.cap, s->f_ids2.cap);
  std::swap(s->f_vals.p, s->f_vals2.p);
  std::swap(s->f_vals.cap, s->f_vals2.cap);
  std::swap(s->f_xt.p, s->f_xt2.p);
  std::swap(s->f_xt.cap, s->f_xt2.cap);
  s->nfric = (int)nf;
}

void k_contact_assemble(zema_scene* s, double* grad, bool hess, unsigned mask) {
  int nc = (int)(s->npt + s->nee);
  // active barrier pairs (distances come from k_contact_energy at the same xs)
  s->n_act = 0;
  if ((mask & 16u) && nc) {
    s->cnt.reserve(nc + 1);
    s->offs.reserve(nc + 1);
    active_flag_kernel<<<nblocks(nc), kBlock, 0, s->st>>>(nc, (int)s->npt, s->pt.p, s->ee.p, s->edges.p,
                                                          s->sv_scene.p, s->act_dev(), s->d_pair.p, s->P.dhat,
                                                          s->cnt.p);
    s->n_act = (int)k_exclusive_scan(s, s->cnt.p, s->offs.p, nc);
    s->act_idx.reserve(s->n_act + 1);
    compact_kernel<<<nblocks(nc), kBlock, 0, s->st>>>(nc, s->cnt.p, s->offs.p, s->act_idx.p);
  }
  int nfr = (mask & 32u) ? s->nfric : 0;
  int nitems = s->n_act + nfr;
  s->nnzc = 0;
  s->c_ptr.reserve(s->nnodes + 1);
  // prismatic joints emit their triplets after the items' (constraint term, mask bit 3)
  // (offsets within the joints' block: jnt_i, uploaded when the joints are set)
  const int nj = (mask & 8u) ? (int)s->joints.size() : 0;
  int64_t ntrip_j = 0;
  for (int j = 0; j < nj; ++j) {
    const Joint& J = s->joints[j];
    const int nodes = 4 * ((s->bodies[J.b1].dof0 >= 0) + (s->bodies[J.b2].dof0 >= 0));
    ntrip_j += nodes + (hess ? nodes * nodes : 0);
  }
  // garment triangles emit theirs after the joints' (elastic term, mask bit 1)
  const int64_t ntrip_c = (mask & 2u) ? (int64_t)s->ncl * (hess ? 12 : 3) : 0;
  if (nitems == 0 && ntrip_j == 0 && ntrip_c == 0) {
    ZCHK(hipMemsetAsync(s->c_ptr.p, 0, sizeof(int) * (s->nnodes + 1), s->st));
    return;
  }
  ItemArgs A;
  A.npt = (int)s->npt;
  A.nee = (int)s->nee;
  A.n_act = s->n_act;
  A.nfric = nfr;
  A.pt = s->pt.p;
  A.ee = s->ee.p;
  A.tris = s->tris.p;
  A.edges = s->edges.p;
  A.act = s->act_idx.p;
  A.sv_ref = s->sv_ref.p;
  A.bi = s->body_i.p;
  A.fids = s->f_ids.p;
  A.elen2 = s->elen2.p;
  A.xs = s->xs.p;
  A.sv_x0 = s->sv_x0.p;
  A.fvals = s->f_vals.p;
  A.fxt = s->f_xt.p;
  A.kappa_sc = s->kappa_sc.p;
  A.mu_sc = s->mu_sc.p;
  A.sv_scene = s->sv_scene.p;
  A.active = s->act_dev();
  A.dhat = s->P.dhat;
  A.ys = s->P.eps_v * s->P.dt;
  A.nn_total = s->nnodes;
  A.hess = hess ? 1 : 0;
  int64_t ntrip_items = 0;
  if (nitems) {
    s->trip_cnt.reserve(nitems + 1);
    s->trip_off.reserve(nitems + 1);
    item_count_kernel<<<nblocks(nitems), kBlock, 0, s->st>>>(A, s->trip_cnt.p);
    ntrip_items = k_exclusive_scan(s, s->trip_cnt.p, s->trip_off.p, nitems);
  }
  const int64_t ntrip = ntrip_items + ntrip_j + ntrip_c;
  if (ntrip == 0) {  // every item touches only fixed bodies
    ZCHK(hipMemsetAsync(s->c_ptr.p, 0, sizeof(int) * (s->nnodes + 1), s->st));
    return;
  }
  SortBufs& sb = s->sort;
  sb.k0.reserve(ntrip + 1);
  sb.v0.reserve(ntrip + 1);
  s->trip_val.reserve((size_t)9 * ntrip + 9);
  unsigned long long W = (unsigned long long)s->nnodes + 1;
  if (nitems) {
    s->item_h.reserve((size_t)144 * nitems + 144);
    s->item_g.reserve((size_t)12 * nitems + 12);
    pair_deriv_kernel<<<nitems, 64, 0, s->st>>>(A, s->item_h.p, s->item_g.p);
    kt_begin(s, KT_CONTACT);
    project_emit_kernel<<<nitems, 64, 0, s->st>>>(A, s->item_h.p, s->item_g.p, s->trip_off.p, sb.k0.p,
                                                  s->trip_val.p);
    kt_end(s, KT_CONTACT);
  }
  if (nj)
    joint_emit_kernel<<<nblocks(nj, 64), 64, 0, s->st>>>(joint_args(s, s->y_asm), hess ? 1 : 0, ntrip_items, W,
                                                        s->nnodes, sb.k0.p, s->trip_val.p);
  if (ntrip_c) k_cloth_emit(s, s->y_asm, hess, ntrip_items + ntrip_j, W, sb.k0.p, s->trip_val.p);
  k_iota(s, sb.v0.p, ntrip);  // sort values = triplet ids
  k_radix_sort(s, sb, ntrip, bits_for((unsigned long long)s->nnodes * W + W));
  // segments
  s->cnt.reserve(ntrip + 1);
  s->offs.reserve(ntrip + 1);
  s->trip_cnt.reserve(ntrip + 1);
  s->seg_start.reserve(ntrip + 1);
  int* head = s->cnt.p;
  int* hhead = s->trip_cnt.p;
  heads_kernel<<<nblocks(ntrip), kBlock, 0, s->st>>>((int)ntrip, sb.k0.p, W, head, hhead);
  int64_t nseg = k_exclusive_scan(s, head, s->offs.p, ntrip);
  seg_start_kernel<<<nblocks(ntrip), kBlock, 0, s->st>>>((int)ntrip, head, s->offs.p, s->seg_start.p);
  int64_t nh = k_exclusive_scan(s, hhead, hhead, ntrip);  // Hessian segment ids
  s->nnzc = (int)nh;
  s->c_col.reserve(nh + 1);
  s->c_val.reserve((size_t)9 * nh + 9);
  s->seg_row.reserve(nh + 1);
  if (s->mixed) {
    s->c_val32.reserve((size_t)9 * nh + 9);
    seg_reduce_kernel<float><<<nblocks(nseg, 4), kBlock, 0, s->st>>>((int)nseg, (int)ntrip, s->seg_start.p, sb.k0.p,
                                                                     sb.v0.p, s->trip_val.p, W, hhead, grad,
                                                                     s->seg_row.p, s->c_col.p, s->c_val32.p, (int)nh);
  } else {
    seg_reduce_kernel<double><<<nblocks(nseg, 4), kBlock, 0, s->st>>>((int)nseg, (int)ntrip, s->seg_start.p, sb.k0.p,
                                                                      sb.v0.p, s->trip_val.p, W, hhead, grad,
                                                                      s->seg_row.p, s->c_col.p, s->c_val.p, (int)nh);
  }
  row_ptr_kernel<<<nblocks(s->nnodes + 1), kBlock, 0, s->st>>>(s->nnodes, (int)nh, s->seg_row.p, s->c_ptr.p);
}

}  // namespace zema

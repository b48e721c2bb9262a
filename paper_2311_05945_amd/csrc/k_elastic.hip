// Soft-body terms of the incremental potential (Sec. III eq. 1): per-tet
// neo-Hookean energy, gradient and projected Hessian blocks (one tet per lane,
// SoA element streams), and deterministic gathers of the per-tet results into the
// gradient and the static block-sparse Hessian, together with the diagonal inertia
// term 1/2 m_i |x_i - xhat_i|^2.
#include "material.hpp"
#include "scene.hpp"

namespace zema {

__device__ inline void load_tet(int e, int nt, const int4* __restrict__ tets, const double* __restrict__ Dmi,
                                const double* __restrict__ y, double F[3][3], double G[4][3], int4& t) {
  t = tets[e];
  double x[4][3];
  const int id[4] = {t.x, t.y, t.z, t.w};
  for (int a = 0; a < 4; ++a)
    for (int k = 0; k < 3; ++k) x[a][k] = y[3 * id[a] + k];
  double D[3][3];
  for (int m = 0; m < 3; ++m)
    for (int j = 0; j < 3; ++j) D[m][j] = Dmi[(3 * m + j) * nt + e];
  for (int j = 0; j < 3; ++j) {
    G[1][j] = D[0][j];
    G[2][j] = D[1][j];
    G[3][j] = D[2][j];
    G[0][j] = -(D[0][j] + D[1][j] + D[2][j]);
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      F[i][j] = (x[1][i] - x[0][i]) * D[0][j] + (x[2][i] - x[0][i]) * D[1][j] + (x[3][i] - x[0][i]) * D[2][j];
}

template <class T>
__global__ void __launch_bounds__(128) tet_assemble_kernel(int nt, const int4* __restrict__ tets,
                                                            const double* __restrict__ Dmi,
                                                            const double* __restrict__ h2vol,
                                                            const double* __restrict__ lmu,
                                                            const double* __restrict__ llam,
                                                            const double* __restrict__ y, double* __restrict__ e_out,
                                                            double* __restrict__ g_out, T* __restrict__ h_out,
                                                            int want_h, const int* __restrict__ v_scene,
                                                            const int* __restrict__ active) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt) return;
  if (active && !active[v_scene[tets[e].x]]) return;  // converged scene of a batch: blocks kept
  double F[3][3], G[4][3];
  int4 t;
  load_tet(e, nt, tets, Dmi, y, F, G, t);
  double g[12];
  double E = nh_element(F, G, lmu[e], llam[e], h2vol[e], g, nullptr);
  e_out[e] = E;
  for (int k = 0; k < 12; ++k) g_out[(size_t)12 * e + k] = g[k];
  if (want_h && E < INFINITY) nh_hess_blocks<T>(F, G, lmu[e], llam[e], h2vol[e], h_out + (size_t)90 * e);
}

__global__ void tet_energy_kernel(int nt, const int4* __restrict__ tets, const double* __restrict__ Dmi,
                                  const double* __restrict__ h2vol, const double* __restrict__ lmu,
                                  const double* __restrict__ llam, const double* __restrict__ y,
                                  double* __restrict__ e_out) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt) return;
  double F[3][3], G[4][3];
  int4 t;
  load_tet(e, nt, tets, Dmi, y, F, G, t);
  e_out[e] = nh_energy(F, lmu[e], llam[e], h2vol[e]);
}

// gradient of soft vertices: elastic contributions in tet order + inertia
__global__ void gather_grad_soft_kernel(int nsv, const int* __restrict__ vt_ptr, const int* __restrict__ vt_list,
                                        const double* __restrict__ g_tet, const double* __restrict__ mass,
                                        const double* __restrict__ y, const double* __restrict__ yhat,
                                        double* __restrict__ grad, unsigned mask) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsv) return;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  if (mask & 2u)
    for (int k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) {
      int ent = vt_list[k];
      const double* gt = g_tet + (size_t)12 * (ent >> 2) + 3 * (ent & 3);
      g0 += gt[0];
      g1 += gt[1];
      g2 += gt[2];
    }
  if (mask & 1u) {
    double m = mass[i];
    g0 += m * (y[3 * i] - yhat[3 * i]);
    g1 += m * (y[3 * i + 1] - yhat[3 * i + 1]);
    g2 += m * (y[3 * i + 2] - yhat[3 * i + 2]);
  }
  grad[3 * i] = g0;
  grad[3 * i + 1] = g1;
  grad[3 * i + 2] = g2;
}

// index of the upper block (a <= b) among the 10 stored per tet
__device__ inline int upper_index(int a, int b) {
  // rows start at 0, 4, 7, 9
  const int base[4] = {0, 4, 7, 9};
  return base[a] + (b - a);
}

// static BSR blocks of soft rows: sum of tet blocks (list order = tet order) and
// the inertia mass on the diagonal
template <class T>
__global__ void gather_hess_kernel(int nnzb_soft, const int* __restrict__ brow, const int* __restrict__ bcol,
                                   const int* __restrict__ hc_ptr, const int* __restrict__ hc_list,
                                   const T* __restrict__ h_tet, const double* __restrict__ mass,
                                   T* __restrict__ val, int nnzb, unsigned mask) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nnzb_soft) return;
  T acc[9];
  for (int k = 0; k < 9; ++k) acc[k] = T(0);
  if (mask & 2u)
    for (int k = hc_ptr[j]; k < hc_ptr[j + 1]; ++k) {
      int ent = hc_list[k];
      int e = ent >> 4, a = (ent >> 2) & 3, b = ent & 3;
      if (a <= b) {
        const T* h = h_tet + (size_t)90 * e + 9 * upper_index(a, b);
        for (int q = 0; q < 9; ++q) acc[q] += h[q];
      } else {
        const T* h = h_tet + (size_t)90 * e + 9 * upper_index(b, a);
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) acc[3 * r + c] += h[3 * c + r];
      }
    }
  int row = brow[j];
  if ((mask & 1u) && bcol[j] == row) {
    T m = T(mass[row]);
    acc[0] += m;
    acc[4] += m;
    acc[8] += m;
  }
  for (int q = 0; q < 9; ++q) val[(size_t)q * nnzb + j] = acc[q];
}

__global__ void inertia_energy_kernel(int nsv, const double* __restrict__ mass, const double* __restrict__ y,
                                      const double* __restrict__ yhat, double* __restrict__ e) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsv) return;
  double d0 = y[3 * i] - yhat[3 * i], d1 = y[3 * i + 1] - yhat[3 * i + 1], d2 = y[3 * i + 2] - yhat[3 * i + 2];
  e[i] = 0.5 * mass[i] * (d0 * d0 + d1 * d1 + d2 * d2);
}

void k_tet_assemble(zema_scene* s, const double* y, bool hess) {
  if (!s->nt) return;
  kt_begin(s, KT_TET);
  if (s->mixed)
    tet_assemble_kernel<float><<<nblocks(s->nt, 128), 128, 0, s->st>>>(s->nt, s->tets.p, s->Dmi.p, s->h2vol.p,
                                                                       s->lmu.p, s->llam.p, y, s->e_tet.p,
                                                                       s->g_tet.p, s->h_tet32.p, hess ? 1 : 0,
                                                                       s->v_scene.p, s->act_dev());
  else
    tet_assemble_kernel<double><<<nblocks(s->nt, 128), 128, 0, s->st>>>(s->nt, s->tets.p, s->Dmi.p, s->h2vol.p,
                                                                        s->lmu.p, s->llam.p, y, s->e_tet.p,
                                                                        s->g_tet.p, s->h_tet.p, hess ? 1 : 0,
                                                                        s->v_scene.p, s->act_dev());
  kt_end(s, KT_TET, (s->mixed ? 170.0 : 320.0) * s->nt);
}

void k_tet_energy(zema_scene* s, const double* y) {
  if (!s->nt) return;
  tet_energy_kernel<<<nblocks(s->nt), kBlock, 0, s->st>>>(s->nt, s->tets.p, s->Dmi.p, s->h2vol.p, s->lmu.p, s->llam.p,
                                                          y, s->e_tet.p);
}

void k_gather_grad_soft(zema_scene* s, const double* y, double* grad, unsigned mask) {
  if (!s->nsv) return;
  gather_grad_soft_kernel<<<nblocks(s->nsv), kBlock, 0, s->st>>>(s->nsv, s->vt_ptr.p, s->vt_list.p, s->g_tet.p,
                                                                  s->mass.p, y, s->yhat.p, grad, mask);
}

void k_gather_hess_static(zema_scene* s, unsigned mask) {
  // soft rows come first in node order
  int nsoft_blocks = s->nsv ? s->bsr_row_soft_end : 0;
  if (!nsoft_blocks) return;
  if (s->mixed)
    gather_hess_kernel<float><<<nblocks(nsoft_blocks), kBlock, 0, s->st>>>(nsoft_blocks, s->bsr_row.p, s->bsr_col.p,
                                                                          s->hc_ptr.p, s->hc_list.p, s->h_tet32.p,
                                                                          s->mass.p, s->bsr_val32.p, s->nnzb, mask);
  else
    gather_hess_kernel<double><<<nblocks(nsoft_blocks), kBlock, 0, s->st>>>(nsoft_blocks, s->bsr_row.p, s->bsr_col.p,
                                                                           s->hc_ptr.p, s->hc_list.p, s->h_tet.p,
                                                                           s->mass.p, s->bsr_val.p, s->nnzb, mask);
}

void k_inertia_energy(zema_scene* s, const double* y, double* e_out) {
  if (!s->nsv) return;
  inertia_energy_kernel<<<nblocks(s->nsv), kBlock, 0, s->st>>>(s->nsv, s->mass.p, y, s->yhat.p, e_out);
}

}  // namespace zema

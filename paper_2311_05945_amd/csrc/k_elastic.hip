// Soft-body terms of the incremental potential (Sec. III eq. 1): per-tet
// energy, gradient and projected Hessian blocks of the tet's constitutive model
// (Sec. IV-D: neo-Hookean, Saint Venant-Kirchhoff, fixed corotated; one tet per lane,
// SoA element streams), and deterministic gathers of the per-tet results into the
// gradient and the static block-sparse Hessian, together with the diagonal inertia
// term 1/2 m_i |x_i - xhat_i|^2.
//
// The tet kernel writes each contribution to the slot its destination reads: the
// records of one soft vertex (its gradient shares and diagonal blocks, slots in the
// vertex's incident-tet list) and of one upper off-diagonal block (slots in that
// block's tet list) are contiguous, in tet order, so the gathers read contiguous
// streams and sum them in a fixed order (bitwise repeatable, no atomics).
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

// Destination slots of one tet's records: diagonal / gradient slot of each vertex,
// off-diagonal slot of each pair (tet_pair order), transposed when the pair's global
// order is reversed (the stored block is the upper one, row vertex < column vertex).
template <class T>
struct SlotHess {
  T* hd;  // [4 nt][6] diagonal records
  T* ho;  // [6 nt][9] off-diagonal records
  int sd[4], so[6];
  unsigned tr;
  __device__ void diag(int a, int k, T v) const { hd[(size_t)6 * sd[a] + k] = v; }
  __device__ void off(int p, int r, int c, T v) const {
    ho[(size_t)9 * so[p] + (((tr >> p) & 1u) ? 3 * c + r : 3 * r + c)] = v;
  }
};

template <class T>
__global__ void __launch_bounds__(128) tet_assemble_kernel(int nt, const int4* __restrict__ tets,
                                                            const double* __restrict__ Dmi,
                                                            const double* __restrict__ h2vol,
                                                            const double* __restrict__ lmu,
                                                            const double* __restrict__ llam,
                                                            const unsigned char* __restrict__ tmodel,
                                                            const int* __restrict__ slot, const double* __restrict__ y,
                                                            double* __restrict__ e_out, double* __restrict__ g_out,
                                                            T* __restrict__ h_out, int want_h,
                                                            const int* __restrict__ v_scene,
                                                            const int* __restrict__ active) {
  // a single scene spreads contiguous tet runs over the XCDs (a batch keeps the plain
  // order, so that converged scenes do not idle whole XCDs)
  const int blk = active ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
  int e = blk * blockDim.x + threadIdx.x;
  if (e >= nt) return;
  if (active && !active[v_scene[tets[e].x]]) return;  // converged scene of a batch: records kept
  double F[3][3], G[4][3];
  int4 t;
  load_tet(e, nt, tets, Dmi, y, F, G, t);
  double g[12];
  const int model = tmodel[e];
  double E = tet_element(model, F, G, lmu[e], llam[e], h2vol[e], g, nullptr);
  e_out[e] = E;
  SlotHess<T> out;
#pragma unroll
  for (int a = 0; a < 4; ++a) out.sd[a] = slot[(size_t)a * nt + e];
#pragma unroll
  for (int q = 0; q < 6; ++q) out.so[q] = slot[(size_t)(4 + q) * nt + e];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 3; ++r) g_out[(size_t)3 * out.sd[a] + r] = g[3 * a + r];
  if (want_h && E < INFINITY) {
    const int id[4] = {t.x, t.y, t.z, t.w};
    out.tr = 0u;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a + 1; b < 4; ++b) out.tr |= (id[a] > id[b] ? 1u : 0u) << tet_pair(a, b);
    out.hd = h_out;
    out.ho = h_out + (size_t)24 * nt;
    tet_hess_blocks<T>(model, F, G, lmu[e], llam[e], h2vol[e], out);
  }
}

__global__ void tet_energy_kernel(int nt, const int4* __restrict__ tets, const double* __restrict__ Dmi,
                                  const double* __restrict__ h2vol, const double* __restrict__ lmu,
                                  const double* __restrict__ llam, const unsigned char* __restrict__ tmodel,
                                  const double* __restrict__ y, double* __restrict__ e_out) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt) return;
  double F[3][3], G[4][3];
  int4 t;
  load_tet(e, nt, tets, Dmi, y, F, G, t);
  e_out[e] = tet_psi(tmodel[e], F, lmu[e], llam[e], h2vol[e]);
}

// gradient of soft vertices: elastic contributions (the vertex's contiguous records,
// tet order) + inertia
__global__ void gather_grad_soft_kernel(int nsv, const int* __restrict__ vt_ptr, const double* __restrict__ g_rec,
                                        const double* __restrict__ mass, const double* __restrict__ y,
                                        const double* __restrict__ yhat, double* __restrict__ grad, unsigned mask) {
  int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= nsv) return;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  if (mask & 2u)
    for (int k = vt_ptr[i]; k < vt_ptr[i + 1]; ++k) {
      const double* gt = g_rec + (size_t)3 * k;
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

// Static BSR blocks of soft rows, kGatherLanes lanes per block: blocks [0, nsv) the
// diagonal block of a vertex (its contiguous diagonal records + the lumped mass),
// blocks [nsv, nsv + n_off) one upper off-diagonal block (its contiguous records), also
// written transposed at the mirror position.  Lane l of a group sums records l, l + L,
// l + 2L, ... of the block's run (the group reads the run as one coalesced stream), then
// the group adds its lanes by a fixed butterfly: a deterministic order.
constexpr int kGatherLanes = 8;

template <class T>
__global__ void __launch_bounds__(kBlock) gather_hess_kernel(int nsv, int n_off, const int* __restrict__ vt_ptr,
                                                             const int* __restrict__ bdiag,
                                                             const int* __restrict__ off_ptr,
                                                             const int* __restrict__ off_blk,
                                                             const int* __restrict__ off_mir, const T* __restrict__ hd,
                                                             const T* __restrict__ ho, const double* __restrict__ mass,
                                                             T* __restrict__ val, int nnzb, unsigned mask) {
  constexpr int L = kGatherLanes;
  const int tid = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int u = tid / L, l = tid % L;
  const bool diag = u < nsv;
  if (!diag && u - nsv >= n_off) return;  // whole groups leave together
  int k0, k1;
  if (diag) {
    k0 = vt_ptr[u];
    k1 = vt_ptr[u + 1];
  } else {
    k0 = off_ptr[u - nsv];
    k1 = off_ptr[u - nsv + 1];
  }
  if (!(mask & 2u)) k1 = k0;
  T acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = T(0);
  if (diag) {
    for (int k = k0 + l; k < k1; k += L) {
      const T* h = hd + (size_t)6 * k;
#pragma unroll
      for (int q = 0; q < 6; ++q) acc[q] += h[q];
    }
  } else {
    for (int k = k0 + l; k < k1; k += L) {
      const T* h = ho + (size_t)9 * k;
#pragma unroll
      for (int q = 0; q < 9; ++q) acc[q] += h[q];
    }
  }
#pragma unroll
  for (int o = L / 2; o >= 1; o >>= 1)
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] += __shfl_xor(acc[q], o, L);
  if (diag) {
    const int j = bdiag[u];
    if (j < 0) return;  // a vertex of no tet has no static block
    if (mask & 1u) {
      const T m = T(mass[u]);
      acc[0] += m;
      acc[3] += m;
      acc[5] += m;
    }
    const T full[9] = {acc[0], acc[1], acc[2], acc[1], acc[3], acc[4], acc[2], acc[4], acc[5]};
#pragma unroll
    for (int q = 0; q < 9; ++q)
      if (q % L == l) val[(size_t)q * nnzb + j] = full[q];
    return;
  }
  const int j = off_blk[u - nsv], jm = off_mir[u - nsv];
#pragma unroll
  for (int q = 0; q < 9; ++q)
    if (q % L == l) {
      const int r = q / 3, c = q % 3;
      val[(size_t)q * nnzb + j] = acc[q];
      val[(size_t)(3 * c + r) * nnzb + jm] = acc[q];
    }
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
  if (s->mixed)
    tet_assemble_kernel<float><<<nblocks(s->nt, 128), 128, 0, s->st>>>(s->nt, s->tets.p, s->Dmi.p, s->h2vol.p,
                                                                       s->lmu.p, s->llam.p, s->tmodel.p, s->tslot.p,
                                                                       y, s->e_tet.p, s->g_tet.p, s->h_tet32.p,
                                                                       hess ? 1 : 0,
                                                                       s->v_scene.p, s->act_dev());
  else
    tet_assemble_kernel<double><<<nblocks(s->nt, 128), 128, 0, s->st>>>(s->nt, s->tets.p, s->Dmi.p, s->h2vol.p,
                                                                        s->lmu.p, s->llam.p, s->tmodel.p, s->tslot.p,
                                                                        y, s->e_tet.p, s->g_tet.p, s->h_tet.p,
                                                                        hess ? 1 : 0,
                                                                        s->v_scene.p, s->act_dev());
}

void k_tet_energy(zema_scene* s, const double* y) {
  if (!s->nt) return;
  tet_energy_kernel<<<nblocks(s->nt), kBlock, 0, s->st>>>(s->nt, s->tets.p, s->Dmi.p, s->h2vol.p, s->lmu.p, s->llam.p,
                                                          s->tmodel.p, y, s->e_tet.p);
}

void k_gather_grad_soft(zema_scene* s, const double* y, double* grad, unsigned mask) {
  if (!s->nsv) return;
  gather_grad_soft_kernel<<<nblocks(s->nsv), kBlock, 0, s->st>>>(s->nsv, s->vt_ptr.p, s->g_tet.p, s->mass.p, y,
                                                                  s->yhat.p, grad, mask);
}

void k_gather_hess_static(zema_scene* s, unsigned mask) {
  // soft rows come first in node order: one thread per diagonal block, then one per
  // upper off-diagonal block of those rows
  if (!s->nsv) return;
  const int n_off = (int)s->off_blk.n;
  const int64_t n = (int64_t)kGatherLanes * (s->nsv + n_off);
  const size_t ho = (size_t)24 * s->nt;
  if (s->mixed)
    gather_hess_kernel<float><<<nblocks(n), kBlock, 0, s->st>>>(s->nsv, n_off, s->vt_ptr.p, s->bsr_diag.p,
                                                                s->off_ptr.p, s->off_blk.p, s->off_mir.p, s->h_tet32.p,
                                                                s->h_tet32.p + ho, s->mass.p, s->bsr_val32.p, s->nnzb,
                                                                mask);
  else
    gather_hess_kernel<double><<<nblocks(n), kBlock, 0, s->st>>>(s->nsv, n_off, s->vt_ptr.p, s->bsr_diag.p,
                                                                 s->off_ptr.p, s->off_blk.p, s->off_mir.p, s->h_tet.p,
                                                                 s->h_tet.p + ho, s->mass.p, s->bsr_val.p, s->nnzb,
                                                                 mask);
}

void k_inertia_energy(zema_scene* s, const double* y, double* e_out) {
  if (!s->nsv) return;
  inertia_energy_kernel<<<nblocks(s->nsv), kBlock, 0, s->st>>>(s->nsv, s->mass.p, y, s->yhat.p, e_out);
}

}  // namespace zema

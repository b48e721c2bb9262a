// Affine-body terms (Sec. III eq. 2): inertia 1/2 (q - qhat)^T M_b (q - qhat) with
// M_b = diag(m I, S, S, S) for a centred rest frame, orthogonality potential
// h^2 lambda V |A A^T - I|_F^2 (9x9 Hessian projected to PSD), and for driven bodies
// the kinematic energy of Sec. IV-C-1 eq. 13, kappa_A/2 |q - q~|^2 - sqrt(m)
// lambda_A . (q - q~).  One lane per body.  Also the springs of Sec. IV-C-3,
// h^2 k |x - x_target|^2 per constrained surface vertex.
#include "geom.hpp"
#include "scene.hpp"
#include "wave_jacobi.hpp"

namespace zema {


// energies [inertia, orthogonality, kinematic]; optional gradient (12) and Hessian
__device__ inline void body_terms(const double* q, const double* qh, const double* qt, const double* bf, int mode,
                                  double h2, double* E3, double* g, double (*H)[12], unsigned mask) {
  double m = bf[BF_M], V = bf[BF_V], lam = bf[BF_ST], kA = bf[BF_KA];
  const double* S = bf + BF_S;
  double dq[12];
  for (int k = 0; k < 12; ++k) dq[k] = q[k] - qh[k];
  // inertia
  double Mdq[12];
  for (int k = 0; k < 3; ++k) Mdq[k] = m * dq[k];
  for (int blk = 0; blk < 3; ++blk)
    for (int i = 0; i < 3; ++i)
      Mdq[3 + 3 * blk + i] = S[3 * i] * dq[3 + 3 * blk] + S[3 * i + 1] * dq[4 + 3 * blk] + S[3 * i + 2] * dq[5 + 3 * blk];
  double ein = 0.0;
  for (int k = 0; k < 12; ++k) ein += 0.5 * dq[k] * Mdq[k];
  // orthogonality: A rows a_i = q[3+3i .. 5+3i]; R = A A^T - I
  double A[3][3], R[3][3], AtA[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = q[3 + 3 * i + j];
  double phi = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = A[i][0] * A[j][0] + A[i][1] * A[j][1] + A[i][2] * A[j][2];
      R[i][j] = acc - (i == j ? 1.0 : 0.0);
      AtA[i][j] = A[0][i] * A[0][j] + A[1][i] * A[1][j] + A[2][i] * A[2][j];
      phi += R[i][j] * R[i][j];
    }
  double c = h2 * lam * V;
  double eorth = c * phi;
  double ekin = 0.0;
  const double sm = sqrt(m);
  const double* lamA = bf + BF_LAM;
  if (mode == ZEMA_DRIVEN)
    for (int k = 0; k < 12; ++k) {
      double d = q[k] - qt[k];
      ekin += 0.5 * kA * d * d - sm * lamA[k] * d;
    }
  E3[0] = ein;
  E3[1] = eorth;
  E3[2] = ekin;
  if (g) {
    for (int k = 0; k < 12; ++k) g[k] = (mask & 1u) ? Mdq[k] : 0.0;
    if (mask & 4u)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          g[3 + 3 * i + j] += 4.0 * c * (R[i][0] * A[0][j] + R[i][1] * A[1][j] + R[i][2] * A[2][j]);
    if ((mask & 8u) && mode == ZEMA_DRIVEN)
      for (int k = 0; k < 12; ++k) g[k] += kA * (q[k] - qt[k]) - sm * lamA[k];
  }
  if (H) {
    for (int i = 0; i < 12; ++i)
      for (int j = 0; j < 12; ++j) H[i][j] = 0.0;
    if (mask & 4u) {
      // d2/dA_ij dA_kl of |A A^T - I|^2 = 4 (delta_ik (A^T A)_lj + A_il A_kj + R_ik delta_jl)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
              double v = (i == k ? AtA[l][j] : 0.0) + A[i][l] * A[k][j] + (j == l ? R[i][k] : 0.0);
              H[3 * i + j][3 * k + l] = 4.0 * c * v;
            }
      psd_project<9>(H);
      // move the 9x9 into the a-block (indices 3..11)
      for (int i = 8; i >= 0; --i)
        for (int j = 8; j >= 0; --j) H[3 + i][3 + j] = H[i][j];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 12; ++j) {
          H[i][j] = 0.0;
          H[j][i] = 0.0;
        }
    }
    if (mask & 1u) {
      for (int k = 0; k < 3; ++k) H[k][k] += m;
      for (int blk = 0; blk < 3; ++blk)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) H[3 + 3 * blk + i][3 + 3 * blk + j] += S[3 * i + j];
    }
    if ((mask & 8u) && mode == ZEMA_DRIVEN)
      for (int k = 0; k < 12; ++k) H[k][k] += kA;
  }
}

template <class T>
__global__ void body_assemble_kernel(int nb, const double* __restrict__ bf, const int* __restrict__ bi,
                                     const double* __restrict__ qtilde, const double* __restrict__ y,
                                     const double* __restrict__ yhat, double* __restrict__ grad,
                                     double* __restrict__ e_body, const int* __restrict__ bsr_ptr,
                                     T* __restrict__ val, int nnzb, int want_h, double h2, unsigned mask) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  int mode = bi[4 * b], dof0 = bi[4 * b + 1], node0 = bi[4 * b + 2];
  if (dof0 < 0) {
    e_body[b] = e_body[nb + b] = e_body[2 * nb + b] = 0.0;
    return;
  }
  double E3[3], g[12];
  double H[12][12];
  body_terms(y + dof0, yhat + dof0, qtilde + 12 * b, bf + BF * b, mode, h2, E3, grad ? g : nullptr,
             want_h ? H : nullptr, mask);
  for (int k = 0; k < 3; ++k) e_body[k * nb + b] = E3[k];  // SoA: [inertia | orth | kinematic]
  if (grad)
    for (int k = 0; k < 12; ++k) grad[dof0 + k] = g[k];
  if (want_h)
    for (int r = 0; r < 4; ++r) {
      int base = bsr_ptr[node0 + r];
      for (int c = 0; c < 4; ++c)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) val[(size_t)(3 * i + j) * nnzb + base + c] = T(H[3 * r + i][3 * c + j]);
    }
}

// Hessian of the body terms, one wavefront per body: the 9x9 orthogonality Hessian
// is formed entry-parallel in LDS (padded to 10x10 with a zero row and column, which
// the projection leaves at zero), projected by parallel Jacobi, and written with the
// inertia and kinematic diagonals as the body's 4x4 node blocks.
template <class T>
__global__ void __launch_bounds__(64) body_hess_kernel(const double* __restrict__ bf, const int* __restrict__ bi,
                                                       const double* __restrict__ y, const int* __restrict__ bsr_ptr,
                                                       T* __restrict__ val, int nnzb, double h2, unsigned mask) {
  constexpr int N = 10, LD = 11;
  __shared__ double M[N * LD], Vm[N * LD], cs[2 * N];
  __shared__ int partner[N];
  __shared__ double A[9], R[9], AtA[9];
  const int b = blockIdx.x, lane = threadIdx.x;
  const int mode = bi[4 * b], dof0 = bi[4 * b + 1], node0 = bi[4 * b + 2];
  if (dof0 < 0) return;  // fixed body: no DOFs (uniform over the block)
  const double* f = bf + BF * b;
  const double m = f[BF_M], c = h2 * f[BF_ST] * f[BF_V], kA = f[BF_KA];
  const double* S = f + BF_S;
  const double* q = y + dof0;
  if (lane < 9) A[lane] = q[3 + lane];  // rows a_i = q[3 + 3i .. 5 + 3i]
  __syncthreads();
  if (lane < 9) {
    int i = lane / 3, j = lane % 3;
    R[lane] = A[3 * i] * A[3 * j] + A[3 * i + 1] * A[3 * j + 1] + A[3 * i + 2] * A[3 * j + 2] - (i == j ? 1.0 : 0.0);
    AtA[lane] = A[i] * A[j] + A[3 + i] * A[3 + j] + A[6 + i] * A[6 + j];
  }
  __syncthreads();
  for (int e = lane; e < N * N; e += 64) {
    int r = e / N, cc = e % N;
    double v = 0.0;
    if (r < 9 && cc < 9 && (mask & 4u)) {
      int i = r / 3, j = r % 3, k = cc / 3, l = cc % 3;
      // d2/dA_ij dA_kl of |A A^T - I|^2 = 4 (delta_ik (A^T A)_lj + A_il A_kj + R_ik delta_jl)
      v = 4.0 * c * ((i == k ? AtA[3 * l + j] : 0.0) + A[3 * i + l] * A[3 * k + j] + (j == l ? R[3 * i + k] : 0.0));
    }
    M[r * LD + cc] = v;
  }
  __syncthreads();
  if (mask & 4u) wave_psd_project<N, LD>(M, Vm, cs, partner, lane);
  // 12x12 entry (r, cc): p-block inertia m I, a-blocks the projection plus S, kinematic diagonal
  for (int e = lane; e < 144; e += 64) {
    int r = e / 12, cc = e % 12;
    double v = (r >= 3 && cc >= 3) ? M[(r - 3) * LD + (cc - 3)] : 0.0;
    if (mask & 1u) {
      if (r < 3 && r == cc) v += m;
      if (r >= 3 && cc >= 3 && (r - 3) / 3 == (cc - 3) / 3) v += S[3 * ((r - 3) % 3) + (cc - 3) % 3];
    }
    if ((mask & 8u) && mode == ZEMA_DRIVEN && r == cc) v += kA;
    int nr = r / 3, nc = cc / 3;
    val[(size_t)(3 * (r % 3) + cc % 3) * nnzb + bsr_ptr[node0 + nr] + nc] = T(v);
  }
}

// ------------------------------------------------------------------ springs (Sec. IV-C-3)
// energy h^2 k |x - t|^2 of each spring at the surface positions xs
__global__ void spring_energy_kernel(int n, const int* __restrict__ sv, const double* __restrict__ kt,
                                     const double* __restrict__ xs, double h2, double* __restrict__ e) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* x = xs + 3 * sv[i];
  const double* c = kt + 4 * i;
  double d0 = x[0] - c[1], d1 = x[1] - c[2], d2 = x[2] - c[3];
  e[i] = h2 * c[0] * (d0 * d0 + d1 * d1 + d2 * d2);
}

// gradient 2 h^2 k (x - t) and Hessian 2 h^2 k I of the springs on soft vertices (one
// spring per vertex: each thread owns its vertex's DOFs and diagonal block), added to
// the assembled gradient and static blocks
template <class T>
__global__ void spring_soft_kernel(int n, const int* __restrict__ sv, const double* __restrict__ kt,
                                   const int* __restrict__ sv_ref, const double* __restrict__ xs, double h2,
                                   double* __restrict__ grad, const int* __restrict__ bdiag, T* __restrict__ val,
                                   int nnzb) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int v = sv_ref[sv[i]];
  if (v < 0) return;  // an affine body's vertex
  const double* x = xs + 3 * sv[i];
  const double* c = kt + 4 * i;
  const double w = 2.0 * h2 * c[0];
  if (grad)
    for (int k = 0; k < 3; ++k) grad[3 * v + k] += w * (x[k] - c[1 + k]);
  if (val) {
    const int j = bdiag[v];
    for (int k = 0; k < 3; ++k) val[(size_t)(4 * k) * nnzb + j] += T(w);
  }
}

// springs on the vertices of free or driven affine bodies, one lane per body walking
// the springs in order: x = A x0 + p, gradient J^T 2 h^2 k (x - t), Hessian
// 2 h^2 k J^T J on the body's 4x4 node blocks
template <class T>
__global__ void spring_body_kernel(int nb, int n, const int* __restrict__ sv, const double* __restrict__ kt,
                                   const int* __restrict__ sv_ref, const double* __restrict__ sv_x0,
                                   const double* __restrict__ xs, const int* __restrict__ bi, double h2,
                                   double* __restrict__ grad, const int* __restrict__ bsr_ptr, T* __restrict__ val,
                                   int nnzb) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int dof0 = bi[4 * b + 1], node0 = bi[4 * b + 2];
  if (dof0 < 0) return;
  for (int i = 0; i < n; ++i) {
    const int s = sv[i];
    if (sv_ref[s] != -1 - b) continue;
    const double* x = xs + 3 * s;
    const double* x0 = sv_x0 + 3 * s;
    const double* c = kt + 4 * i;
    const double w = 2.0 * h2 * c[0];
    // J: row r has 1 at p_r and x0_j at a_{r j} (DOF 3 + 3 r + j)
    if (grad)
      for (int r = 0; r < 3; ++r) {
        const double gr = w * (x[r] - c[1 + r]);
        grad[dof0 + r] += gr;
        for (int j = 0; j < 3; ++j) grad[dof0 + 3 + 3 * r + j] += gr * x0[j];
      }
    if (val)
      for (int u = 0; u < 12; ++u)
        for (int v = 0; v < 12; ++v) {
          // (J^T J)_{uv} = sum_r J_ru J_rv; J_ru nonzero only for u = r or u = 3 + 3 r + j
          const int ru = u < 3 ? u : (u - 3) / 3, rv = v < 3 ? v : (v - 3) / 3;
          if (ru != rv) continue;
          const double ju = u < 3 ? 1.0 : x0[(u - 3) % 3], jv = v < 3 ? 1.0 : x0[(v - 3) % 3];
          val[(size_t)(3 * (u % 3) + v % 3) * nnzb + bsr_ptr[node0 + u / 3] + v / 3] += T(w * ju * jv);
        }
  }
}

void k_spring_energy(zema_scene* s) {
  const int n = (int)s->springs.size();
  if (n) spring_energy_kernel<<<nblocks(n), kBlock, 0, s->st>>>(n, s->spr_sv.p, s->spr_kt.p, s->xs.p,
                                                                 s->P.dt * s->P.dt, s->e_spr.p);
}

void k_spring_terms(zema_scene* s, double* grad, bool hess) {
  const int n = (int)s->springs.size(), nb = (int)s->bodies.size();
  if (!n) return;
  const double h2 = s->P.dt * s->P.dt;
  if (s->mixed) {
    spring_soft_kernel<float><<<nblocks(n), kBlock, 0, s->st>>>(n, s->spr_sv.p, s->spr_kt.p, s->sv_ref.p, s->xs.p, h2,
                                                                grad, s->bsr_diag.p, hess ? s->bsr_val32.p : nullptr,
                                                                s->nnzb);
    if (nb)
      spring_body_kernel<float><<<nblocks(nb, 64), 64, 0, s->st>>>(nb, n, s->spr_sv.p, s->spr_kt.p, s->sv_ref.p,
                                                                   s->sv_x0.p, s->xs.p, s->body_i.p, h2, grad,
                                                                   s->bsr_ptr.p, hess ? s->bsr_val32.p : nullptr,
                                                                   s->nnzb);
  } else {
    spring_soft_kernel<double><<<nblocks(n), kBlock, 0, s->st>>>(n, s->spr_sv.p, s->spr_kt.p, s->sv_ref.p, s->xs.p, h2,
                                                                 grad, s->bsr_diag.p, hess ? s->bsr_val.p : nullptr,
                                                                 s->nnzb);
    if (nb)
      spring_body_kernel<double><<<nblocks(nb, 64), 64, 0, s->st>>>(nb, n, s->spr_sv.p, s->spr_kt.p, s->sv_ref.p,
                                                                    s->sv_x0.p, s->xs.p, s->body_i.p, h2, grad,
                                                                    s->bsr_ptr.p, hess ? s->bsr_val.p : nullptr,
                                                                    s->nnzb);
  }
}

void k_body_terms(zema_scene* s, const double* y, double* grad, bool hess, unsigned mask) {
  int nb = (int)s->bodies.size();
  if (!nb) return;
  const double h2 = s->P.dt * s->P.dt;
  if (s->mixed) {
    body_assemble_kernel<float><<<nblocks(nb, 64), 64, 0, s->st>>>(nb, s->body_f.p, s->body_i.p, s->qtilde.p, y,
                                                                   s->yhat.p, grad, s->e_body.p, s->bsr_ptr.p,
                                                                   s->bsr_val32.p, s->nnzb, 0, h2, mask);
    if (hess)
      body_hess_kernel<float><<<nb, 64, 0, s->st>>>(s->body_f.p, s->body_i.p, y, s->bsr_ptr.p, s->bsr_val32.p, s->nnzb,
                                                    h2, mask);
  } else {
    body_assemble_kernel<double><<<nblocks(nb, 64), 64, 0, s->st>>>(nb, s->body_f.p, s->body_i.p, s->qtilde.p, y,
                                                                    s->yhat.p, grad, s->e_body.p, s->bsr_ptr.p,
                                                                    s->bsr_val.p, s->nnzb, 0, h2, mask);
    if (hess)
      body_hess_kernel<double><<<nb, 64, 0, s->st>>>(s->body_f.p, s->body_i.p, y, s->bsr_ptr.p, s->bsr_val.p,
                                                     s->nnzb, h2, mask);
  }
}

void k_body_energy(zema_scene* s, const double* y) {
  int nb = (int)s->bodies.size();
  if (!nb) return;
  body_assemble_kernel<double><<<nblocks(nb, 64), 64, 0, s->st>>>(nb, s->body_f.p, s->body_i.p, s->qtilde.p, y,
                                                                  s->yhat.p, nullptr, s->e_body.p, s->bsr_ptr.p,
                                                                  s->bsr_val.p, s->nnzb, 0, s->P.dt * s->P.dt, 0x3fu);
}

}  // namespace zema

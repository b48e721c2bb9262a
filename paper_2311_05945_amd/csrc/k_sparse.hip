// Block-sparse Hessian products and the block-Jacobi preconditioned CG solve of
// the Newton system H p = -g.  H = static BSR (tets + affine bodies) + contact CSR,
// both over 3-DOF nodes with 3x3 blocks stored as 9 SoA planes.  Soft rows are
// handled by 16-lane groups (one block per lane, shuffle reduction); affine rows,
// which collect every contacting soft vertex, get a full workgroup each.
//
// PCG (start at 0, stop at |r| <= rtol |b|): each iteration is spmv (with the
// search-direction update p = z + beta p_old folded into the gathers), a one-block
// scalar step, the vector update with the preconditioner, and a one-block scalar
// step; scalars stay on the device and the host polls a flag every few iterations.
#include "scene.hpp"

namespace zema {

constexpr int RG = 16;  // lanes per soft row

struct Mat {
  int nsv, nnodes, nnzb, nnzc;
  const int *bp, *bc, *cp, *cc;
  const double *bv, *cv;
};

struct Vec {
  const double* a;  // value = a + beta * b (b may be null)
  const double* b;
  const double* beta;
  __device__ inline V3 at(int j) const {
    V3 v = ld3(a + 3 * j);
    if (b) {
      double be = *beta;
      V3 w = ld3(b + 3 * j);
      v = v + be * w;
    }
    return v;
  }
};

__device__ inline V3 blk_mul(const double* v, int stride, int j, V3 x) {
  return v3(v[j] * x.x + v[stride + j] * x.y + v[2 * stride + j] * x.z,
            v[3 * stride + j] * x.x + v[4 * stride + j] * x.y + v[5 * stride + j] * x.z,
            v[6 * stride + j] * x.x + v[7 * stride + j] * x.y + v[8 * stride + j] * x.z);
}

__device__ inline V3 row_partial(const Mat& M, int row, int lane, int nl, const Vec& x) {
  V3 acc = v3(0, 0, 0);
  for (int j = M.bp[row] + lane; j < M.bp[row + 1]; j += nl) acc = acc + blk_mul(M.bv, M.nnzb, j, x.at(M.bc[j]));
  if (M.cp)
    for (int j = M.cp[row] + lane; j < M.cp[row + 1]; j += nl) acc = acc + blk_mul(M.cv, M.nnzc, j, x.at(M.cc[j]));
  return acc;
}

// out = H x; optionally writes xo = x (own rows) and block partials of x.out
__global__ void spmv_kernel(Mat M, Vec x, double* __restrict__ out, double* __restrict__ xo,
                            double* __restrict__ partial, const double* __restrict__ done) {
  if (done && *done != 0.0) return;
  __shared__ double sh[kBlock / 64];
  __shared__ double red[3][kBlock / 64];
  int nsoft_blocks = (M.nsv + (kBlock / RG) - 1) / (kBlock / RG);
  double dotv = 0.0;
  if ((int)blockIdx.x < nsoft_blocks) {
    int row = blockIdx.x * (kBlock / RG) + threadIdx.x / RG;
    int lane = threadIdx.x % RG;
    V3 acc = v3(0, 0, 0);
    if (row < M.nsv) acc = row_partial(M, row, lane, RG, x);
    for (int o = RG / 2; o > 0; o >>= 1) {
      acc.x += __shfl_xor(acc.x, o, RG);
      acc.y += __shfl_xor(acc.y, o, RG);
      acc.z += __shfl_xor(acc.z, o, RG);
    }
    if (lane == 0 && row < M.nsv) {
      st3(out + 3 * row, acc);
      V3 xv = x.at(row);
      if (xo) st3(xo + 3 * row, xv);
      dotv = dot(xv, acc);
    }
  } else {
    int row = M.nsv + (blockIdx.x - nsoft_blocks);
    V3 acc = row_partial(M, row, threadIdx.x, kBlock, x);
    acc.x = wave_sum(acc.x);
    acc.y = wave_sum(acc.y);
    acc.z = wave_sum(acc.z);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
      red[0][w] = acc.x;
      red[1][w] = acc.y;
      red[2][w] = acc.z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      V3 s = v3(0, 0, 0);
      for (int k = 0; k < kBlock / 64; ++k) s = s + v3(red[0][k], red[1][k], red[2][k]);
      st3(out + 3 * row, s);
      V3 xv = x.at(row);
      if (xo) st3(xo + 3 * row, xv);
      dotv = dot(xv, s);
    }
    __syncthreads();
  }
  if (partial) {
    double r = block_sum<kBlock>(dotv, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
  }
}

// ------------------------------------------------------------------ preconditioner
__device__ inline int find_col(const int* cc, int j0, int j1, int col) {
  while (j0 < j1) {
    int m = (j0 + j1) >> 1;
    if (cc[m] < col)
      j0 = m + 1;
    else
      j1 = m;
  }
  return j0;
}

__device__ inline void add_block(const Mat& M, int row, int col, double* D, int ld, int r0, int c0) {
  // static
  int j0 = M.bp[row], j1 = M.bp[row + 1];
  int j = find_col(M.bc, j0, j1, col);
  if (j < j1 && M.bc[j] == col)
    for (int q = 0; q < 9; ++q) D[(r0 + q / 3) * ld + c0 + q % 3] += M.bv[(size_t)q * M.nnzb + j];
  if (M.cp) {
    j0 = M.cp[row];
    j1 = M.cp[row + 1];
    j = find_col(M.cc, j0, j1, col);
    if (j < j1 && M.cc[j] == col)
      for (int q = 0; q < 9; ++q) D[(r0 + q / 3) * ld + c0 + q % 3] += M.cv[(size_t)q * M.nnzc + j];
  }
}

__host__ __device__ inline bool inv3(const double* a, double* o) {
  double c00 = a[4] * a[8] - a[5] * a[7], c01 = a[5] * a[6] - a[3] * a[8], c02 = a[3] * a[7] - a[4] * a[6];
  double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  if (!(det != 0.0)) return false;
  double id = 1.0 / det;
  o[0] = c00 * id;
  o[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  o[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  o[3] = c01 * id;
  o[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  o[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  o[6] = c02 * id;
  o[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  o[8] = (a[0] * a[4] - a[1] * a[3]) * id;
  return true;
}

__global__ void precond_soft_kernel(Mat M, double* __restrict__ minv, int* __restrict__ bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.nsv) return;
  double D[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, I[9];
  add_block(M, i, i, D, 3, 0, 0);
  if (!inv3(D, I)) {
    atomicAdd(bad, 1);
    for (int q = 0; q < 9; ++q) I[q] = 0.0;
  }
  for (int q = 0; q < 9; ++q) minv[(size_t)q * M.nsv + i] = I[q];
}

// 12x12 inverse by Gauss-Jordan with partial pivoting, one lane per affine body
__global__ void precond_body_kernel(Mat M, int nfree, double* __restrict__ minv, int* __restrict__ bad) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nfree) return;
  int node0 = M.nsv + 4 * k;
  double A[144], I[144];
  for (int q = 0; q < 144; ++q) {
    A[q] = 0.0;
    I[q] = (q % 13 == 0) ? 1.0 : 0.0;
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) add_block(M, node0 + r, node0 + c, A, 12, 3 * r, 3 * c);
  for (int c = 0; c < 12; ++c) {
    int piv = c;
    for (int r = c + 1; r < 12; ++r)
      if (fabs(A[r * 12 + c]) > fabs(A[piv * 12 + c])) piv = r;
    if (A[piv * 12 + c] == 0.0) {
      atomicAdd(bad, 1);
      return;
    }
    if (piv != c)
      for (int q = 0; q < 12; ++q) {
        double t = A[c * 12 + q];
        A[c * 12 + q] = A[piv * 12 + q];
        A[piv * 12 + q] = t;
        t = I[c * 12 + q];
        I[c * 12 + q] = I[piv * 12 + q];
        I[piv * 12 + q] = t;
      }
    double d = 1.0 / A[c * 12 + c];
    for (int q = 0; q < 12; ++q) {
      A[c * 12 + q] *= d;
      I[c * 12 + q] *= d;
    }
    for (int r = 0; r < 12; ++r) {
      if (r == c) continue;
      double f = A[r * 12 + c];
      if (f == 0.0) continue;
      for (int q = 0; q < 12; ++q) {
        A[r * 12 + q] -= f * A[c * 12 + q];
        I[r * 12 + q] -= f * I[c * 12 + q];
      }
    }
  }
  for (int q = 0; q < 144; ++q) minv[(size_t)144 * k + q] = I[q];
}

// ------------------------------------------------------------------ PCG kernels
// scalars: 0 rz, 1 pq, 2 alpha, 3 beta, 4 rr, 5 bb, 6 done, 7 iters, 8 breakdown, 9 tol2
__device__ inline void apply_minv(int i, int nsv, const double* __restrict__ ms, const double* __restrict__ mb,
                                  const double* __restrict__ r, double* __restrict__ z) {
  if (i < nsv) {
    V3 rv = ld3(r + 3 * i);
    z[3 * i] = ms[i] * rv.x + ms[nsv + i] * rv.y + ms[2 * nsv + i] * rv.z;
    z[3 * i + 1] = ms[3 * nsv + i] * rv.x + ms[4 * nsv + i] * rv.y + ms[5 * nsv + i] * rv.z;
    z[3 * i + 2] = ms[6 * nsv + i] * rv.x + ms[7 * nsv + i] * rv.y + ms[8 * nsv + i] * rv.z;
  } else {
    int k = i - nsv;
    const double* m = mb + 144 * k;
    const double* rr = r + 3 * nsv + 12 * k;
    double* zz = z + 3 * nsv + 12 * k;
    for (int a = 0; a < 12; ++a) {
      double acc = 0.0;
      for (int b = 0; b < 12; ++b) acc += m[12 * a + b] * rr[b];
      zz[a] = acc;
    }
  }
}

__global__ void pcg_init_kernel(int nsv, int nfree, const double* __restrict__ b, const double* __restrict__ ms,
                                const double* __restrict__ mb, double* __restrict__ x, double* __restrict__ r,
                                double* __restrict__ z, double* __restrict__ p, double* __restrict__ partial) {
  __shared__ double sh[kBlock / 64];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, bb = 0.0;
  if (i < nsv + nfree) {
    int o = i < nsv ? 3 * i : 3 * nsv + 12 * (i - nsv), n = i < nsv ? 3 : 12;
    for (int k = 0; k < n; ++k) {
      x[o + k] = 0.0;
      r[o + k] = b[o + k];
      p[o + k] = 0.0;
    }
    apply_minv(i, nsv, ms, mb, b, z);
    for (int k = 0; k < n; ++k) {
      rz += b[o + k] * z[o + k];
      bb += b[o + k] * b[o + k];
    }
  }
  double s1 = block_sum<kBlock>(rz, sh);
  double s2 = block_sum<kBlock>(bb, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1;
    partial[2 * blockIdx.x + 1] = s2;
  }
}

__global__ void pcg_init_fin(int nb, const double* __restrict__ partial, double* __restrict__ sc, double rtol) {
  __shared__ double sh[kBlock / 64];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  double rz = block_sum<kBlock>(a, sh);
  double bb = block_sum<kBlock>(b, sh);
  if (threadIdx.x == 0) {
    sc[0] = rz;
    sc[3] = 0.0;
    sc[4] = bb;
    sc[5] = bb;
    sc[6] = bb == 0.0 ? 1.0 : 0.0;
    sc[7] = 0.0;
    sc[8] = 0.0;
    sc[9] = rtol * rtol * bb;
  }
}

__global__ void pcg_alpha_kernel(int nb, const double* __restrict__ partial, double* __restrict__ sc) {
  if (sc[6] != 0.0) return;
  __shared__ double sh[kBlock / 64];
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) a += partial[i];
  double pq = block_sum<kBlock>(a, sh);
  if (threadIdx.x == 0) {
    sc[1] = pq;
    if (!(pq > 0.0)) {
      sc[8] = 1.0;
      sc[6] = 1.0;
    } else {
      sc[2] = sc[0] / pq;
    }
  }
}

__global__ void pcg_update_kernel(int nsv, int nfree, const double* __restrict__ p, const double* __restrict__ q,
                                  const double* __restrict__ ms, const double* __restrict__ mb, double* __restrict__ x,
                                  double* __restrict__ r, double* __restrict__ z, const double* __restrict__ sc,
                                  double* __restrict__ partial) {
  if (sc[6] != 0.0) return;
  __shared__ double sh[kBlock / 64];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double alpha = sc[2];
  double rz = 0.0, rr = 0.0;
  if (i < nsv + nfree) {
    int o = i < nsv ? 3 * i : 3 * nsv + 12 * (i - nsv), n = i < nsv ? 3 : 12;
    for (int k = 0; k < n; ++k) {
      x[o + k] += alpha * p[o + k];
      r[o + k] -= alpha * q[o + k];
    }
    apply_minv(i, nsv, ms, mb, r, z);
    for (int k = 0; k < n; ++k) {
      rz += r[o + k] * z[o + k];
      rr += r[o + k] * r[o + k];
    }
  }
  double s1 = block_sum<kBlock>(rz, sh);
  double s2 = block_sum<kBlock>(rr, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1;
    partial[2 * blockIdx.x + 1] = s2;
  }
}

__global__ void pcg_beta_kernel(int nb, const double* __restrict__ partial, double* __restrict__ sc) {
  if (sc[6] != 0.0) return;
  __shared__ double sh[kBlock / 64];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  double rz = block_sum<kBlock>(a, sh);
  double rr = block_sum<kBlock>(b, sh);
  if (threadIdx.x == 0) {
    sc[7] += 1.0;
    sc[4] = rr;
    if (rr <= sc[9]) {
      sc[6] = 1.0;
    } else {
      sc[3] = rz / sc[0];
      sc[0] = rz;
    }
  }
}

static Mat make_mat(zema_scene* s) {
  Mat M;
  M.nsv = s->nsv;
  M.nnodes = s->nnodes;
  M.nnzb = s->nnzb;
  M.nnzc = s->nnzc;
  M.bp = s->bsr_ptr.p;
  M.bc = s->bsr_col.p;
  M.bv = s->bsr_val.p;
  bool has_c = s->nnzc > 0;
  M.cp = has_c ? s->c_ptr.p : nullptr;
  M.cc = s->c_col.p;
  M.cv = s->c_val.p;
  return M;
}

static int spmv_grid(zema_scene* s) { return (s->nsv + (kBlock / RG) - 1) / (kBlock / RG) + 4 * s->nfree; }

void k_hess_matvec(zema_scene* s, const double* v, double* out) {
  Mat M = make_mat(s);
  Vec x{v, nullptr, nullptr};
  int g = spmv_grid(s);
  if (g) spmv_kernel<<<g, kBlock, 0, s->st>>>(M, x, out, nullptr, nullptr, nullptr);
}

void k_build_precond(zema_scene* s) {
  Mat M = make_mat(s);
  s->minv_soft.reserve((size_t)9 * s->nsv + 9);
  s->minv_body.reserve((size_t)144 * s->nfree + 144);
  int* bad = s->counters.p + 4;
  ZCHK(hipMemsetAsync(bad, 0, sizeof(int), s->st));
  if (s->nsv) precond_soft_kernel<<<nblocks(s->nsv), kBlock, 0, s->st>>>(M, s->minv_soft.p, bad);
  if (s->nfree) precond_body_kernel<<<nblocks(s->nfree, 64), 64, 0, s->st>>>(M, s->nfree, s->minv_body.p, bad);
}

int k_pcg(zema_scene* s, const double* rhs, double* sol, double rtol, int max_iter, int* iters, double* relres) {
  int n = s->ndof;
  if (max_iter <= 0) max_iter = n;
  k_build_precond(s);
  s->pr.reserve(n);
  s->pz.reserve(n);
  s->pp0.reserve(n);
  s->pp1.reserve(n);
  s->pq.reserve(n);
  int nunits = s->nsv + s->nfree;
  int nbv = nblocks(nunits);
  int g = spmv_grid(s);
  s->partial.reserve(2 * (size_t)std::max(nbv, g) + 2);
  s->scal.reserve(16);
  double* sc = s->scal.p;
  Mat M = make_mat(s);
  pcg_init_kernel<<<nbv, kBlock, 0, s->st>>>(s->nsv, s->nfree, rhs, s->minv_soft.p, s->minv_body.p, sol, s->pr.p,
                                             s->pz.p, s->pp0.p, s->partial.p);
  pcg_init_fin<<<1, kBlock, 0, s->st>>>(nbv, s->partial.p, sc, rtol);
  double* pold = s->pp0.p;
  double* pnew = s->pp1.p;
  const int chunk = 8;
  double hs[10];
  int it = 0;
  for (;;) {
    for (int k = 0; k < chunk && it < max_iter; ++k, ++it) {
      Vec x{s->pz.p, pold, sc + 3};
      kt_begin(s, KT_SPMV);
      spmv_kernel<<<g, kBlock, 0, s->st>>>(M, x, s->pq.p, pnew, s->partial.p, sc + 6);
      kt_end(s, KT_SPMV, 76.0 * (s->nnzb + s->nnzc) + 32.0 * s->ndof);
      pcg_alpha_kernel<<<1, kBlock, 0, s->st>>>(g, s->partial.p, sc);
      pcg_update_kernel<<<nbv, kBlock, 0, s->st>>>(s->nsv, s->nfree, pnew, s->pq.p, s->minv_soft.p, s->minv_body.p,
                                                   sol, s->pr.p, s->pz.p, sc, s->partial.p);
      pcg_beta_kernel<<<1, kBlock, 0, s->st>>>(nbv, s->partial.p, sc);
      std::swap(pold, pnew);
    }
    ZCHK(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, s->st));
    ZCHK(hipStreamSynchronize(s->st));
    if (hs[6] != 0.0 || it >= max_iter) break;
  }
  int bad;
  ZCHK(hipMemcpyAsync(&bad, s->counters.p + 4, sizeof(int), hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
  *iters = (int)hs[7];
  *relres = hs[5] > 0.0 ? sqrt(hs[4] / hs[5]) : 0.0;
  if (bad) return ZEMA_E_PCG;
  if (hs[8] != 0.0) return ZEMA_E_PCG;
  if (hs[6] == 0.0) return ZEMA_E_PCG;
  return 0;
}

}  // namespace zema

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
#include <cstring>

#include "scene.hpp"

namespace zema {

constexpr int RG = 16;  // lanes per soft row

// matrix with block values of type V (double, or float for the mixed-precision
// form, where products also accumulate in float)
template <class V>
struct Mat {
  int nsv, nnodes, nnzb, nnzc;
  const int *bp, *bc, *cp, *cc;
  const V *bv, *cv;
};

template <class V>
struct Acc3 {
  V x, y, z;
};

// x = a + beta b at node c (DOF vectors stay FP64; converted to V for the product)
template <class V>
__device__ inline void blk_acc(const V* __restrict__ v, int stride, int j, const double* a, const double* b,
                               double beta, int c, Acc3<V>& acc) {
  double u0 = a[3 * c], u1 = a[3 * c + 1], u2 = a[3 * c + 2];
  if (b) {
    u0 += beta * b[3 * c];
    u1 += beta * b[3 * c + 1];
    u2 += beta * b[3 * c + 2];
  }
  V x0 = V(u0), x1 = V(u1), x2 = V(u2);
  acc.x += v[j] * x0 + v[stride + j] * x1 + v[2 * stride + j] * x2;
  acc.y += v[3 * stride + j] * x0 + v[4 * stride + j] * x1 + v[5 * stride + j] * x2;
  acc.z += v[6 * stride + j] * x0 + v[7 * stride + j] * x1 + v[8 * stride + j] * x2;
}

template <class V>
__device__ inline Acc3<V> row_partial(const Mat<V>& M, int row, int lane, int nl, const double* a, const double* b,
                                      double beta) {
  Acc3<V> acc{V(0), V(0), V(0)};
  for (int j = M.bp[row] + lane; j < M.bp[row + 1]; j += nl) blk_acc(M.bv, M.nnzb, j, a, b, beta, M.bc[j], acc);
  if (M.cp)
    for (int j = M.cp[row] + lane; j < M.cp[row + 1]; j += nl) blk_acc(M.cv, M.nnzc, j, a, b, beta, M.cc[j], acc);
  return acc;
}

// q = H x with x = a + beta b.  Writes xo = x for the rows it owns and the block
// partial of x . q when those pointers are given.  Soft rows: 16 lanes each; affine
// rows: one block each.
template <class V>
__device__ inline double spmv_rows(const Mat<V>& M, const double* a, const double* b, double beta, double* q,
                                   double* xo, double* sh_red /* 3 * waves */) {
  int nsoft_blocks = (M.nsv + (kBlock / RG) - 1) / (kBlock / RG);
  double dotv = 0.0;
  if ((int)blockIdx.x < nsoft_blocks) {
    int row = blockIdx.x * (kBlock / RG) + threadIdx.x / RG;
    int lane = threadIdx.x % RG;
    Acc3<V> acc{V(0), V(0), V(0)};
    if (row < M.nsv) acc = row_partial(M, row, lane, RG, a, b, beta);
    for (int o = RG / 2; o > 0; o >>= 1) {
      acc.x += __shfl_xor(acc.x, o, RG);
      acc.y += __shfl_xor(acc.y, o, RG);
      acc.z += __shfl_xor(acc.z, o, RG);
    }
    if (lane == 0 && row < M.nsv) {
      V3 qv = v3(double(acc.x), double(acc.y), double(acc.z));
      st3(q + 3 * row, qv);
      V3 xv = ld3(a + 3 * row);
      if (b) xv = xv + beta * ld3(b + 3 * row);
      if (xo) st3(xo + 3 * row, xv);
      dotv = dot(xv, qv);
    }
  } else {
    int row = M.nsv + (blockIdx.x - nsoft_blocks);
    Acc3<V> acc = row_partial(M, row, threadIdx.x, kBlock, a, b, beta);
    for (int o = 32; o > 0; o >>= 1) {
      acc.x += __shfl_xor(acc.x, o, 64);
      acc.y += __shfl_xor(acc.y, o, 64);
      acc.z += __shfl_xor(acc.z, o, 64);
    }
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
      sh_red[3 * w] = double(acc.x);
      sh_red[3 * w + 1] = double(acc.y);
      sh_red[3 * w + 2] = double(acc.z);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      V3 sq = v3(0, 0, 0);
      for (int k = 0; k < kBlock / 64; ++k) sq = sq + v3(sh_red[3 * k], sh_red[3 * k + 1], sh_red[3 * k + 2]);
      st3(q + 3 * row, sq);
      V3 xv = ld3(a + 3 * row);
      if (b) xv = xv + beta * ld3(b + 3 * row);
      if (xo) st3(xo + 3 * row, xv);
      dotv = dot(xv, sq);
    }
    __syncthreads();
  }
  return dotv;
}

template <class V>
__global__ void spmv_kernel(Mat<V> M, const double* __restrict__ x, double* __restrict__ out) {
  __shared__ double red[3 * (kBlock / 64)];
  spmv_rows(M, x, nullptr, 0.0, out, nullptr, red);
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

template <class V>
__device__ inline void add_block(const Mat<V>& M, int row, int col, double* D, int ld, int r0, int c0) {
  // static
  int j0 = M.bp[row], j1 = M.bp[row + 1];
  int j = find_col(M.bc, j0, j1, col);
  if (j < j1 && M.bc[j] == col)
    for (int q = 0; q < 9; ++q) D[(r0 + q / 3) * ld + c0 + q % 3] += double(M.bv[(size_t)q * M.nnzb + j]);
  if (M.cp) {
    j0 = M.cp[row];
    j1 = M.cp[row + 1];
    j = find_col(M.cc, j0, j1, col);
    if (j < j1 && M.cc[j] == col)
      for (int q = 0; q < 9; ++q) D[(r0 + q / 3) * ld + c0 + q % 3] += double(M.cv[(size_t)q * M.nnzc + j]);
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

template <class V>
__global__ void precond_soft_kernel(Mat<V> M, double* __restrict__ minv, int* __restrict__ bad) {
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

// 12x12 inverse of an affine body's diagonal block by Gauss-Jordan with partial
// pivoting: one wavefront per body, the augmented matrix [D | I] in LDS.
template <class V>
__global__ void __launch_bounds__(64) precond_body_kernel(Mat<V> M, int nfree, double* __restrict__ minv,
                                                          int* __restrict__ bad) {
  __shared__ double Aug[12][25];
  __shared__ int piv_row;
  int k = blockIdx.x, lane = threadIdx.x;
  if (k >= nfree) return;
  int node0 = M.nsv + 4 * k;
  for (int e = lane; e < 12 * 24; e += 64) {
    int r = e / 24, c = e % 24;
    Aug[r][c] = c >= 12 ? (c - 12 == r ? 1.0 : 0.0) : 0.0;
  }
  __syncthreads();
  if (lane < 16) add_block(M, node0 + lane / 4, node0 + lane % 4, &Aug[0][0], 25, 3 * (lane / 4), 3 * (lane % 4));
  __syncthreads();
  for (int c = 0; c < 12; ++c) {
    if (lane == 0) {
      int pr = c;
      for (int r = c + 1; r < 12; ++r)
        if (fabs(Aug[r][c]) > fabs(Aug[pr][c])) pr = r;
      piv_row = pr;
    }
    __syncthreads();
    int pr = piv_row;
    if (Aug[pr][c] == 0.0) {
      if (lane == 0) atomicAdd(bad, 1);
      return;
    }
    if (pr != c && lane < 24) {
      double t = Aug[c][lane];
      Aug[c][lane] = Aug[pr][lane];
      Aug[pr][lane] = t;
    }
    __syncthreads();
    double d = 1.0 / Aug[c][c];
    __syncthreads();
    if (lane < 24) Aug[c][lane] *= d;
    __syncthreads();
    // eliminate column c from every other row (factors read before any update)
    double f[12];
    for (int r = 0; r < 12; ++r) f[r] = Aug[r][c];
    __syncthreads();
    for (int e = lane; e < 12 * 24; e += 64) {
      int r = e / 24, cc = e % 24;
      if (r != c) Aug[r][cc] -= f[r] * Aug[c][cc];
    }
    __syncthreads();
  }
  for (int e = lane; e < 144; e += 64) minv[(size_t)144 * k + e] = Aug[e / 12][12 + e % 12];
}

// ------------------------------------------------------------------ PCG kernels
// scalars: 0/1 rz (ping-pong by iteration parity), 2 alpha, 4 rr, 5 bb, 6 done,
// 7 iters, 8 breakdown, 9 tol^2 = rtol^2 bb
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

// every block sums the same partials in the same order (deterministic, identical)
__device__ inline void reduce_partials2(const double* __restrict__ partial, int nb, double* sh, double& a, double& b) {
  double x = 0.0, y = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    x += partial[2 * i];
    y += partial[2 * i + 1];
  }
  a = block_sum<kBlock>(x, sh);
  b = block_sum<kBlock>(y, sh);
  __shared__ double bc[2];
  if (threadIdx.x == 0) {
    bc[0] = a;
    bc[1] = b;
  }
  __syncthreads();
  a = bc[0];
  b = bc[1];
  __syncthreads();
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
  double rz, bb;
  reduce_partials2(partial, nb, sh, rz, bb);
  if (threadIdx.x == 0) {
    sc[0] = rz;
    sc[1] = rz;
    sc[4] = bb;
    sc[5] = bb;
    sc[6] = bb == 0.0 ? 1.0 : 0.0;
    sc[7] = 0.0;
    sc[8] = 0.0;
    sc[9] = rtol * rtol * bb;
  }
}

// Two accumulators per row: H a and H b over the same gathers, so the product can be
// formed before beta is known (q = H a + beta H b).
template <class V>
__device__ inline void blk_acc2(const V* __restrict__ v, int stride, int j, const double* a, const double* b, int c,
                                Acc3<V>& A, Acc3<V>& B) {
  V a0 = V(a[3 * c]), a1 = V(a[3 * c + 1]), a2 = V(a[3 * c + 2]);
  V b0 = V(b[3 * c]), b1 = V(b[3 * c + 1]), b2 = V(b[3 * c + 2]);
  V m0 = v[j], m1 = v[stride + j], m2 = v[2 * stride + j], m3 = v[3 * stride + j], m4 = v[4 * stride + j],
    m5 = v[5 * stride + j], m6 = v[6 * stride + j], m7 = v[7 * stride + j], m8 = v[8 * stride + j];
  A.x += m0 * a0 + m1 * a1 + m2 * a2;
  A.y += m3 * a0 + m4 * a1 + m5 * a2;
  A.z += m6 * a0 + m7 * a1 + m8 * a2;
  B.x += m0 * b0 + m1 * b1 + m2 * b2;
  B.y += m3 * b0 + m4 * b1 + m5 * b2;
  B.z += m6 * b0 + m7 * b1 + m8 * b2;
}

template <class V>
__device__ inline void row_partial2(const Mat<V>& M, int row, int lane, int nl, const double* a, const double* b,
                                    Acc3<V>& A, Acc3<V>& B) {
  for (int j = M.bp[row] + lane; j < M.bp[row + 1]; j += nl) blk_acc2(M.bv, M.nnzb, j, a, b, M.bc[j], A, B);
  if (M.cp)
    for (int j = M.cp[row] + lane; j < M.cp[row + 1]; j += nl) blk_acc2(M.cv, M.nnzc, j, a, b, M.cc[j], A, B);
}

// sums of two per-thread values over the block (fixed tree), broadcast to all threads
__device__ inline void block_sum2_bcast(double& a, double& b, double* sh, double* bc) {
  double x = block_sum<kBlock>(a, sh);
  double y = block_sum<kBlock>(b, sh);
  if (threadIdx.x == 0) {
    bc[0] = x;
    bc[1] = y;
  }
  __syncthreads();
  a = bc[0];
  b = bc[1];
}

// Iteration k, first half: (k > 0) reduce the previous update's partials into
// rz_k, rr_k, stop if converged, beta = rz_k / rz_{k-1}; q = H p_k with
// p_k = z + beta p_{k-1} (gathered as H z and H p_{k-1}, combined once beta is known),
// p_k stored, block partials of p_k . q.  The scalars, the partials and the matrix
// gathers are independent loads, issued before any reduction.
// The matrix descriptor is read from device memory so that a captured launch stays
// valid when the contact matrix is rebuilt; k only selects parities (and k > 0), so a
// captured chunk of an even number of iterations can be replayed at any odd start;
// sc[7] counts the iterations on the device.
template <class V, int G>
__global__ void pcg_spmv_kernel(const Mat<V>* __restrict__ Mp, int k, int nbu, const double* __restrict__ upart,
                                const double* __restrict__ z, const double* __restrict__ pold,
                                double* __restrict__ pnew, double* __restrict__ q, double* __restrict__ spart,
                                double* __restrict__ sc) {
  const Mat<V> M = *Mp;
  __shared__ double sh[kBlock / 64];
  __shared__ double bc[2];
  __shared__ double red[6 * (kBlock / 64)];
  __shared__ double done_s;  // block 0 may set the flag during this launch: read once per block
  if (threadIdx.x == 0) done_s = sc[6];
  const double tol2 = sc[9], rz_prev = k > 0 ? sc[(k - 1) & 1] : 1.0;
  double u1 = 0.0, u2 = 0.0;
  if (k > 0)
    for (int i = threadIdx.x; i < nbu; i += kBlock) {
      u1 += upart[2 * i];
      u2 += upart[2 * i + 1];
    }
  const int nsoft_blocks = (M.nsv + (kBlock / G) - 1) / (kBlock / G);
  const bool soft = (int)blockIdx.x < nsoft_blocks;
  int row;
  Acc3<V> A{V(0), V(0), V(0)}, B{V(0), V(0), V(0)};
  if (soft) {
    row = blockIdx.x * (kBlock / G) + threadIdx.x / G;
    int lane = threadIdx.x % G;
    if (row < M.nsv) row_partial2(M, row, lane, G, z, pold, A, B);
    for (int o = G / 2; o > 0; o >>= 1) {
      A.x += __shfl_xor(A.x, o, G);
      A.y += __shfl_xor(A.y, o, G);
      A.z += __shfl_xor(A.z, o, G);
      B.x += __shfl_xor(B.x, o, G);
      B.y += __shfl_xor(B.y, o, G);
      B.z += __shfl_xor(B.z, o, G);
    }
  } else {
    row = M.nsv + (blockIdx.x - nsoft_blocks);
    row_partial2(M, row, threadIdx.x, kBlock, z, pold, A, B);
    for (int o = 32; o > 0; o >>= 1) {
      A.x += __shfl_xor(A.x, o, 64);
      A.y += __shfl_xor(A.y, o, 64);
      A.z += __shfl_xor(A.z, o, 64);
      B.x += __shfl_xor(B.x, o, 64);
      B.y += __shfl_xor(B.y, o, 64);
      B.z += __shfl_xor(B.z, o, 64);
    }
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
      red[6 * w] = double(A.x);
      red[6 * w + 1] = double(A.y);
      red[6 * w + 2] = double(A.z);
      red[6 * w + 3] = double(B.x);
      red[6 * w + 4] = double(B.y);
      red[6 * w + 5] = double(B.z);
    }
  }
  __syncthreads();  // done_s and red[] visible to the whole block
  if (done_s != 0.0) return;
  double beta = 0.0;
  if (k > 0) {
    block_sum2_bcast(u1, u2, sh, bc);  // rz_k, rr_k
    bool conv = u2 <= tol2;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc[7] += 1.0;  // iterations completed
      sc[4] = u2;
      sc[k & 1] = u1;
      if (conv) sc[6] = 1.0;
    }
    if (conv) return;
    beta = u1 / rz_prev;
  }
  double dotv = 0.0;
  if (soft) {
    if (threadIdx.x % G == 0 && row < M.nsv) {
      V3 qv = v3(double(A.x) + beta * double(B.x), double(A.y) + beta * double(B.y),
                 double(A.z) + beta * double(B.z));
      st3(q + 3 * row, qv);
      V3 pv = ld3(z + 3 * row) + beta * ld3(pold + 3 * row);
      st3(pnew + 3 * row, pv);
      dotv = dot(pv, qv);
    }
  } else if (threadIdx.x == 0) {
    V3 sa = v3(0, 0, 0), sb = v3(0, 0, 0);
    for (int w = 0; w < kBlock / 64; ++w) {
      sa = sa + v3(red[6 * w], red[6 * w + 1], red[6 * w + 2]);
      sb = sb + v3(red[6 * w + 3], red[6 * w + 4], red[6 * w + 5]);
    }
    V3 qv = sa + beta * sb;
    st3(q + 3 * row, qv);
    V3 pv = ld3(z + 3 * row) + beta * ld3(pold + 3 * row);
    st3(pnew + 3 * row, pv);
    dotv = dot(pv, qv);
  }
  double r = block_sum<kBlock>(dotv, sh);
  if (threadIdx.x == 0) spart[blockIdx.x] = r;
}

// Iteration k, second half: pq from the spmv partials, alpha = rz_k / pq (breakdown
// if pq <= 0), x += alpha p, r -= alpha q, z = M^-1 r, partials of r.z and r.r.  A
// soft vertex's vectors and preconditioner block are loaded with the partials,
// before the reduction.
template <int UB>
__global__ void __launch_bounds__(UB) pcg_update_kernel(int nsv, int nfree, int k, int nbs, const double* __restrict__ spart,
                                  const double* __restrict__ p, const double* __restrict__ q,
                                  const double* __restrict__ ms, const double* __restrict__ mb, double* __restrict__ x,
                                  double* __restrict__ r, double* __restrict__ z, double* __restrict__ sc,
                                  double* __restrict__ upart) {
  __shared__ double sh[UB / 64];
  __shared__ double pq_s;
  __shared__ double done_s;  // block 0 may set the flag during this launch: read once per block
  if (threadIdx.x == 0) done_s = sc[6];
  const double rzk = sc[k & 1];
  double a = 0.0;
  for (int i = threadIdx.x; i < nbs; i += UB) a += spart[i];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool sv = i < nsv;
  V3 pv{}, qv{}, xv{}, rv{};
  double m[9];
  if (sv) {
    pv = ld3(p + 3 * i);
    qv = ld3(q + 3 * i);
    xv = ld3(x + 3 * i);
    rv = ld3(r + 3 * i);
    for (int t = 0; t < 9; ++t) m[t] = ms[(size_t)t * nsv + i];
  }
  __syncthreads();
  if (done_s != 0.0) return;
  {
    double t = block_sum<UB>(a, sh);
    if (threadIdx.x == 0) pq_s = t;
    __syncthreads();
  }
  const double pq = pq_s;
  if (!(pq > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc[8] = 1.0;
      sc[6] = 1.0;
    }
    return;
  }
  const double alpha = rzk / pq;
  double rz = 0.0, rr = 0.0;
  if (sv) {
    xv = xv + alpha * pv;
    rv = rv - alpha * qv;
    st3(x + 3 * i, xv);
    st3(r + 3 * i, rv);
    V3 zv = v3(m[0] * rv.x + m[1] * rv.y + m[2] * rv.z, m[3] * rv.x + m[4] * rv.y + m[5] * rv.z,
               m[6] * rv.x + m[7] * rv.y + m[8] * rv.z);
    st3(z + 3 * i, zv);
    rz = dot(rv, zv);
    rr = dot(rv, rv);
  } else if (i < nsv + nfree) {
    int o = 3 * nsv + 12 * (i - nsv);
    for (int kk = 0; kk < 12; ++kk) {
      x[o + kk] += alpha * p[o + kk];
      r[o + kk] -= alpha * q[o + kk];
    }
    apply_minv(i, nsv, ms, mb, r, z);
    for (int kk = 0; kk < 12; ++kk) {
      rz += r[o + kk] * z[o + kk];
      rr += r[o + kk] * r[o + kk];
    }
  }
  double s1 = block_sum<UB>(rz, sh);
  double s2 = block_sum<UB>(rr, sh);
  if (threadIdx.x == 0) {
    upart[2 * blockIdx.x] = s1;
    upart[2 * blockIdx.x + 1] = s2;
  }
}

// after the last update: residual and convergence of iteration k
__global__ void pcg_final_kernel(int k, int nbu, const double* __restrict__ upart, double* __restrict__ sc) {
  if (sc[6] != 0.0) return;
  __shared__ double sh[kBlock / 64];
  double rz, rr;
  reduce_partials2(upart, nbu, sh, rz, rr);
  if (threadIdx.x == 0) {
    sc[7] = k;
    sc[4] = rr;
    if (rr <= sc[9]) sc[6] = 1.0;
  }
}

template <class V>
static Mat<V> make_mat(zema_scene* s, const V* bv, const V* cv) {
  Mat<V> M;
  M.nsv = s->nsv;
  M.nnodes = s->nnodes;
  M.nnzb = s->nnzb;
  M.nnzc = s->nnzc;
  M.bp = s->bsr_ptr.p;
  M.bc = s->bsr_col.p;
  M.bv = bv;
  M.cp = s->nnzc > 0 ? s->c_ptr.p : nullptr;
  M.cc = s->c_col.p;
  M.cv = cv;
  return M;
}

static int spmv_grid(zema_scene* s) { return (s->nsv + (kBlock / RG) - 1) / (kBlock / RG) + 4 * s->nfree; }
static int spmv_grid_g(zema_scene* s, int g) { return (s->nsv + (kBlock / g) - 1) / (kBlock / g) + 4 * s->nfree; }

void k_hess_matvec(zema_scene* s, const double* v, double* out) {
  int g = spmv_grid(s);
  if (!g) return;
  if (s->mixed)
    spmv_kernel<float><<<g, kBlock, 0, s->st>>>(make_mat<float>(s, s->bsr_val32.p, s->c_val32.p), v, out);
  else
    spmv_kernel<double><<<g, kBlock, 0, s->st>>>(make_mat<double>(s, s->bsr_val.p, s->c_val.p), v, out);
}

void k_build_precond(zema_scene* s) {
  s->minv_soft.reserve((size_t)9 * s->nsv + 9);
  s->minv_body.reserve((size_t)144 * s->nfree + 144);
  int* bad = s->counters.p + 4;
  ZCHK(hipMemsetAsync(bad, 0, sizeof(int), s->st));
  if (s->mixed) {
    auto M = make_mat<float>(s, s->bsr_val32.p, s->c_val32.p);
    if (s->nsv) precond_soft_kernel<float><<<nblocks(s->nsv), kBlock, 0, s->st>>>(M, s->minv_soft.p, bad);
    if (s->nfree) precond_body_kernel<float><<<s->nfree, 64, 0, s->st>>>(M, s->nfree, s->minv_body.p, bad);
  } else {
    auto M = make_mat<double>(s, s->bsr_val.p, s->c_val.p);
    if (s->nsv) precond_soft_kernel<double><<<nblocks(s->nsv), kBlock, 0, s->st>>>(M, s->minv_soft.p, bad);
    if (s->nfree) precond_body_kernel<double><<<s->nfree, 64, 0, s->st>>>(M, s->nfree, s->minv_body.p, bad);
  }
}

static constexpr int kChunk = 16;  // PCG iterations per captured chunk (even)

// launch shapes of the fused PCG kernels (tuned per scene): lanes per soft row of the
// matrix-vector product, threads per block of the vector update
struct PcgArgs {
  const void* mat;
  int g, nbu, lanes, ub;
  double *upart, *spart, *sc, *sol;
  double bytes;
};

template <class V>
static void pcg_iteration_v(zema_scene* s, const PcgArgs& a, int k, double* pold, double* pnew, hipStream_t st) {
  const Mat<V>* M = (const Mat<V>*)a.mat;
#define ZEMA_SPMV(G)                                                                                            \
  pcg_spmv_kernel<V, G><<<a.g, kBlock, 0, st>>>(M, k, a.nbu, a.upart, s->pz.p, pold, pnew, s->pq.p, a.spart, \
                                                a.sc)
  if (a.lanes == 8)
    ZEMA_SPMV(8);
  else if (a.lanes == 32)
    ZEMA_SPMV(32);
  else
    ZEMA_SPMV(16);
#undef ZEMA_SPMV
}

static void pcg_iteration(zema_scene* s, const PcgArgs& a, int k, double* pold, double* pnew, hipStream_t st) {
  if (s->mixed)
    pcg_iteration_v<float>(s, a, k, pold, pnew, st);
  else
    pcg_iteration_v<double>(s, a, k, pold, pnew, st);
}

static void pcg_update(zema_scene* s, const PcgArgs& a, int k, double* p, hipStream_t st) {
  int nb = nblocks(s->nsv + s->nfree, a.ub);
#define ZEMA_UPD(B)                                                                                              \
  pcg_update_kernel<B><<<nb, B, 0, st>>>(s->nsv, s->nfree, k, a.g, a.spart, p, s->pq.p, s->minv_soft.p,       \
                                         s->minv_body.p, a.sol, s->pr.p, s->pz.p, a.sc, a.upart)
  if (a.ub == 64)
    ZEMA_UPD(64);
  else if (a.ub == 128)
    ZEMA_UPD(128);
  else
    ZEMA_UPD(256);
#undef ZEMA_UPD
}

// the chunk of iterations k = 1 .. kChunk (pold = pp1 at an odd start), captured once
// per set of buffers; returns false when capture is unavailable.  Launch timing needs
// events around every matvec, so timed solves launch individually.
static bool pcg_graph_ready(zema_scene* s, const PcgArgs& a) {
  std::vector<const void*> key = {a.mat, a.upart, a.spart, a.sc, a.sol, s->pz.p, s->pp0.p, s->pp1.p, s->pq.p,
                                  s->pr.p, s->minv_soft.p, s->minv_body.p, (const void*)(intptr_t)a.g,
                                  (const void*)(intptr_t)a.nbu, (const void*)(intptr_t)a.lanes,
                                  (const void*)(intptr_t)a.ub, (const void*)(intptr_t)s->mixed,
                                  (const void*)(intptr_t)s->nsv, (const void*)(intptr_t)s->nfree};
  PcgGraph& G = s->pcg_graph;
  if (G.exec && G.key == key) return true;
  if (G.exec) {
    ZCHK(hipGraphExecDestroy(G.exec));
    G.exec = nullptr;
  }
  if (!s->cap_st) ZCHK(hipStreamCreate(&s->cap_st));
  if (hipStreamBeginCapture(s->cap_st, hipStreamCaptureModeRelaxed) != hipSuccess) return false;
  double* pold = s->pp1.p;
  double* pnew = s->pp0.p;
  bool ok = true;
  for (int c = 0; c < kChunk; ++c) {
    int k = 1 + c;
    pcg_iteration(s, a, k, pold, pnew, s->cap_st);
    pcg_update(s, a, k, pnew, s->cap_st);
    std::swap(pold, pnew);
  }
  hipGraph_t graph = nullptr;
  ok = (hipStreamEndCapture(s->cap_st, &graph) == hipSuccess) && ok && graph;
  if (ok) ok = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0) == hipSuccess;
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipGetLastError();
  if (!ok) {
    G.exec = nullptr;
    return false;
  }
  G.key = key;
  return true;
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
  const int lanes = s->tune_lanes, ub = s->tune_ublock;
  int g = spmv_grid_g(s, lanes);
  int nbu = nblocks(nunits, ub);
  size_t np = (size_t)std::max(nbv, nbu);
  s->partial.reserve(2 * np + (size_t)g + 4);
  s->scal.reserve(16);
  // matrix descriptors in device memory (the captured kernels read them there)
  s->mat_h.resize(sizeof(Mat<double>) + sizeof(Mat<float>));
  Mat<double> M64 = make_mat<double>(s, s->bsr_val.p, s->c_val.p);
  Mat<float> M32 = make_mat<float>(s, s->bsr_val32.p, s->c_val32.p);
  std::memcpy(s->mat_h.data(), &M64, sizeof(M64));
  std::memcpy(s->mat_h.data() + sizeof(M64), &M32, sizeof(M32));
  s->mat_dev.reserve(s->mat_h.size());
  ZCHK(hipMemcpyAsync(s->mat_dev.p, s->mat_h.data(), s->mat_h.size(), hipMemcpyHostToDevice, s->st));
  PcgArgs a;
  a.mat = s->mixed ? (const void*)(s->mat_dev.p + sizeof(Mat<double>)) : (const void*)s->mat_dev.p;
  a.g = g;
  a.nbu = nbu;
  a.lanes = lanes;
  a.ub = ub;
  a.upart = s->partial.p;
  a.spart = s->partial.p + 2 * np + 2;
  a.sc = s->scal.p;
  a.sol = sol;
  a.bytes = (s->mixed ? 40.0 : 76.0) * (s->nnzb + s->nnzc) + 32.0 * s->ndof;
  pcg_init_kernel<<<nbv, kBlock, 0, s->st>>>(s->nsv, s->nfree, rhs, s->minv_soft.p, s->minv_body.p, sol, s->pr.p,
                                             s->pz.p, s->pp0.p, a.upart);
  pcg_init_fin<<<1, kBlock, 0, s->st>>>(nbv, a.upart, a.sc, rtol);
  const bool timed = s->kt[KT_SPMV].on;
  double* pold = s->pp0.p;
  double* pnew = s->pp1.p;
  double hs[10];
  int it = 0;
  for (;;) {
    if (it == 0) {  // iteration 0 eagerly; every later round starts at an odd iteration
      kt_begin(s, KT_SPMV);
      pcg_iteration(s, a, 0, pold, pnew, s->st);
      kt_end(s, KT_SPMV, a.bytes);
      pcg_update(s, a, 0, pnew, s->st);
      std::swap(pold, pnew);
      it = 1;
    }
    bool graph = (it & 1) && max_iter - it >= kChunk && s->use_graph && !timed && pcg_graph_ready(s, a);
    if (graph) {
      ZCHK(hipGraphLaunch(s->pcg_graph.exec, s->st));
      it += kChunk;  // even: pold / pnew are where they were
    } else {
      for (int c = 0; c < kChunk && it < max_iter; ++c, ++it) {
        kt_begin(s, KT_SPMV);
        pcg_iteration(s, a, it, pold, pnew, s->st);
        kt_end(s, KT_SPMV, a.bytes);
        pcg_update(s, a, it, pnew, s->st);
        std::swap(pold, pnew);
      }
    }
    if (it >= max_iter) pcg_final_kernel<<<1, kBlock, 0, s->st>>>(it, nbu, a.upart, a.sc);
    ZCHK(hipMemcpyAsync(hs, a.sc, sizeof(hs), hipMemcpyDeviceToHost, s->st));
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

// ------------------------------------------------------------------ launch-shape autotuner
__global__ void probe_rhs_kernel(int n, double* __restrict__ b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)((i * 2654435761u) & 1023u) / 512.0 - 1.0;  // deterministic, not smooth
}

// Times a fixed number of PCG iterations on the last assembled Hessian for every
// (lanes per soft row, update block) shape and keeps the fastest.  The shapes change
// summation order only; the choice is fixed until the next call.
void k_autotune(zema_scene* s, int* lanes_out, int* ub_out, double* us_per_iter) {
  const int n = s->ndof, iters = 64;
  if (n == 0) {
    *lanes_out = s->tune_lanes;
    *ub_out = s->tune_ublock;
    return;
  }
  s->ytmp.reserve(n);
  probe_rhs_kernel<<<nblocks(n), kBlock, 0, s->st>>>(n, s->ytmp.p);
  const int L[3] = {8, 16, 32}, U[3] = {64, 128, 256};
  double best = 1e300;
  int bl = s->tune_lanes, bu = s->tune_ublock;
  hipEvent_t e0, e1;
  ZCHK(hipEventCreate(&e0));
  ZCHK(hipEventCreate(&e1));
  for (int li = 0; li < 3; ++li)
    for (int ui = 0; ui < 3; ++ui) {
      s->tune_lanes = L[li];
      s->tune_ublock = U[ui];
      int it;
      double rr;
      float ms = 0.0f;
      for (int rep = 0; rep < 2; ++rep) {  // the first run captures the graph
        ZCHK(hipEventRecord(e0, s->st));
        (void)k_pcg(s, s->ytmp.p, s->pdir.p, 0.0, iters, &it, &rr);
        ZCHK(hipEventRecord(e1, s->st));
        ZCHK(hipEventSynchronize(e1));
        ZCHK(hipEventElapsedTime(&ms, e0, e1));
      }
      if (ms < best) {
        best = ms;
        bl = L[li];
        bu = U[ui];
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  s->tune_lanes = bl;
  s->tune_ublock = bu;
  *lanes_out = bl;
  *ub_out = bu;
  *us_per_iter = 1e3 * best / iters;
}

// ------------------------------------------------------------------ batched PCG
// A batch of scenes has a block-diagonal Newton system; each scene runs its own CG
// (own alpha, beta, residual test and breakdown flag) in lockstep with the others.
// Per-scene dot products are summed by one block per scene over the scene's nodes in
// a fixed order.  Per-scene scalars [ns][16]: 0 rz, 2 alpha, 3 beta, 4 rr, 5 bb,
// 6 done, 7 iterations, 8 breakdown, 9 rtol^2 bb.

__device__ inline int node_scene(int node, int nsv, const int* v_scene, const int* f_scene) {
  return node < nsv ? v_scene[node] : f_scene[(node - nsv) >> 2];
}

// per-node values of r.z, b.b (init) or r.z, r.r (update): unit-major writes
__global__ void pcgb_init_kernel(int nsv, int nfree, const double* __restrict__ b, const double* __restrict__ ms,
                                 const double* __restrict__ mb, double* __restrict__ x, double* __restrict__ r,
                                 double* __restrict__ z, double* __restrict__ p, double* __restrict__ d1,
                                 double* __restrict__ d2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsv + nfree) return;
  int o = i < nsv ? 3 * i : 3 * nsv + 12 * (i - nsv), n = i < nsv ? 3 : 12;
  for (int k = 0; k < n; ++k) {
    x[o + k] = 0.0;
    r[o + k] = b[o + k];
    p[o + k] = 0.0;
  }
  apply_minv(i, nsv, ms, mb, b, z);
  double rz = 0.0, bb = 0.0;
  for (int k = 0; k < n; ++k) {
    rz += b[o + k] * z[o + k];
    bb += b[o + k] * b[o + k];
  }
  d1[i] = rz;
  d2[i] = bb;
}

// sum of a per-unit array over scene k's units (soft vertices, then free bodies)
__device__ inline double scene_unit_sum(const double* __restrict__ a, const int* __restrict__ rng, int k, int nsv,
                                        double* sh) {
  const int* R = rng + 8 * k;
  int nv = R[1] - R[0], nf = R[7] - R[6];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nv + nf; i += kBlock) acc += i < nv ? a[R[0] + i] : a[nsv + R[6] + (i - nv)];
  return block_sum<kBlock>(acc, sh);
}

__global__ void pcgb_init_fin(const double* __restrict__ d1, const double* __restrict__ d2,
                              const int* __restrict__ rng, const int* __restrict__ active, int nsv,
                              double* __restrict__ sc, double rtol) {
  __shared__ double sh[kBlock / 64];
  int k = blockIdx.x;
  double rz = scene_unit_sum(d1, rng, k, nsv, sh);
  double bb = scene_unit_sum(d2, rng, k, nsv, sh);
  if (threadIdx.x == 0) {
    double* c = sc + 16 * k;
    c[0] = rz;
    c[2] = 0.0;
    c[3] = 0.0;
    c[4] = bb;
    c[5] = bb;
    c[6] = (bb == 0.0 || !active[k]) ? 1.0 : 0.0;
    c[7] = 0.0;
    c[8] = 0.0;
    c[9] = rtol * rtol * bb;
  }
}

// q = H p with p = z + beta_scene p_old formed in the gathers; p stored; per-node
// p.q.  Rows of finished scenes are skipped.
template <class V>
__global__ void pcgb_spmv_kernel(const Mat<V>* __restrict__ Mp, const int* __restrict__ v_scene,
                                 const int* __restrict__ f_scene,
                                 const double* __restrict__ sc, const double* __restrict__ z,
                                 const double* __restrict__ pold, double* __restrict__ pnew, double* __restrict__ q,
                                 double* __restrict__ pq) {
  const Mat<V> M = *Mp;
  __shared__ double red[3 * (kBlock / 64)];
  int nsoft_blocks = (M.nsv + (kBlock / RG) - 1) / (kBlock / RG);
  if ((int)blockIdx.x < nsoft_blocks) {
    int row = blockIdx.x * (kBlock / RG) + threadIdx.x / RG;
    int lane = threadIdx.x % RG;
    if (row >= M.nsv) return;
    const double* c = sc + 16 * v_scene[row];
    if (c[6] != 0.0) return;  // the whole 16-lane group leaves together
    double beta = c[3];
    Acc3<V> acc = row_partial(M, row, lane, RG, z, pold, beta);
    for (int o = RG / 2; o > 0; o >>= 1) {
      acc.x += __shfl_xor(acc.x, o, RG);
      acc.y += __shfl_xor(acc.y, o, RG);
      acc.z += __shfl_xor(acc.z, o, RG);
    }
    if (lane == 0) {
      V3 qv = v3(double(acc.x), double(acc.y), double(acc.z));
      st3(q + 3 * row, qv);
      V3 xv = ld3(z + 3 * row) + beta * ld3(pold + 3 * row);
      st3(pnew + 3 * row, xv);
      pq[row] = dot(xv, qv);
    }
  } else {
    int row = M.nsv + (blockIdx.x - nsoft_blocks);
    const double* c = sc + 16 * f_scene[(row - M.nsv) >> 2];
    if (c[6] != 0.0) return;  // uniform over the block
    double beta = c[3];
    Acc3<V> acc = row_partial(M, row, threadIdx.x, kBlock, z, pold, beta);
    for (int o = 32; o > 0; o >>= 1) {
      acc.x += __shfl_xor(acc.x, o, 64);
      acc.y += __shfl_xor(acc.y, o, 64);
      acc.z += __shfl_xor(acc.z, o, 64);
    }
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
      red[3 * w] = double(acc.x);
      red[3 * w + 1] = double(acc.y);
      red[3 * w + 2] = double(acc.z);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      V3 sq = v3(0, 0, 0);
      for (int k = 0; k < kBlock / 64; ++k) sq = sq + v3(red[3 * k], red[3 * k + 1], red[3 * k + 2]);
      st3(q + 3 * row, sq);
      V3 xv = ld3(z + 3 * row) + beta * ld3(pold + 3 * row);
      st3(pnew + 3 * row, xv);
      pq[row] = dot(xv, sq);
    }
  }
}

// per scene: pq over its nodes (soft vertices, then 4 nodes per free body) -> alpha
__global__ void pcgb_alpha_kernel(const double* __restrict__ pq, const int* __restrict__ rng, int nsv,
                                  double* __restrict__ sc) {
  __shared__ double sh[kBlock / 64];
  int k = blockIdx.x;
  double* c = sc + 16 * k;
  if (c[6] != 0.0) return;
  const int* R = rng + 8 * k;
  int nv = R[1] - R[0], nn = 4 * (R[7] - R[6]);
  double acc = 0.0;
  for (int i = threadIdx.x; i < nv + nn; i += kBlock) acc += i < nv ? pq[R[0] + i] : pq[nsv + 4 * R[6] + (i - nv)];
  double t = block_sum<kBlock>(acc, sh);
  if (threadIdx.x == 0) {
    if (!(t > 0.0)) {
      c[8] = 1.0;
      c[6] = 1.0;
    } else {
      c[2] = c[0] / t;
    }
  }
}

__global__ void pcgb_update_kernel(int nsv, int nfree, const int* __restrict__ v_scene,
                                   const int* __restrict__ f_scene, const double* __restrict__ sc,
                                   const double* __restrict__ p, const double* __restrict__ q,
                                   const double* __restrict__ ms, const double* __restrict__ mb,
                                   double* __restrict__ x, double* __restrict__ r, double* __restrict__ z,
                                   double* __restrict__ d1, double* __restrict__ d2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsv + nfree) return;
  const double* c = sc + 16 * (i < nsv ? v_scene[i] : f_scene[i - nsv]);
  if (c[6] != 0.0) return;
  double alpha = c[2];
  int o = i < nsv ? 3 * i : 3 * nsv + 12 * (i - nsv), n = i < nsv ? 3 : 12;
  for (int k = 0; k < n; ++k) {
    x[o + k] += alpha * p[o + k];
    r[o + k] -= alpha * q[o + k];
  }
  apply_minv(i, nsv, ms, mb, r, z);
  double rz = 0.0, rr = 0.0;
  for (int k = 0; k < n; ++k) {
    rz += r[o + k] * z[o + k];
    rr += r[o + k] * r[o + k];
  }
  d1[i] = rz;
  d2[i] = rr;
}

__global__ void pcgb_beta_kernel(const double* __restrict__ d1, const double* __restrict__ d2,
                                 const int* __restrict__ rng, int nsv, int it, double* __restrict__ sc) {
  __shared__ double sh[kBlock / 64];
  int k = blockIdx.x;
  double* c = sc + 16 * k;
  if (c[6] != 0.0) return;
  double rz = scene_unit_sum(d1, rng, k, nsv, sh);
  double rr = scene_unit_sum(d2, rng, k, nsv, sh);
  if (threadIdx.x == 0) {
    c[7] += 1.0;  // iterations completed by this scene
    c[4] = rr;
    if (rr <= c[9]) {
      c[6] = 1.0;
    } else {
      c[3] = rz / c[0];
      c[0] = rz;
    }
  }
}

// Batched solve: scenes with active[k] == 0 get x = 0 and count as converged.
// iters / relres / status: host arrays [ns].
void k_pcg_batch(zema_scene* s, const double* rhs, double* sol, double rtol, int max_iter, const int* active_host,
                 int* iters, double* relres, int* status) {
  const int ns = s->ns, n = s->ndof, nunits = s->nsv + s->nfree;
  if (max_iter <= 0) max_iter = std::max(n, 1);
  k_build_precond(s);  // block-Jacobi inverses of the current Hessian (allocates them)
  s->pr.reserve(n);
  s->pz.reserve(n);
  s->pp0.reserve(n);
  s->pp1.reserve(n);
  s->pq.reserve(n);
  s->partial.reserve((size_t)2 * nunits + s->nnodes + 8);
  double* d1 = s->partial.p;
  double* d2 = s->partial.p + nunits + 1;
  double* pqn = s->partial.p + 2 * (size_t)nunits + 2;
  s->scal.reserve((size_t)16 * ns);
  double* sc = s->scal.p;
  ZCHK(hipMemcpyAsync(s->sc_mask.p, active_host, sizeof(int) * ns, hipMemcpyHostToDevice, s->st));
  if (nunits)
    pcgb_init_kernel<<<nblocks(nunits), kBlock, 0, s->st>>>(s->nsv, s->nfree, rhs, s->minv_soft.p, s->minv_body.p,
                                                            sol, s->pr.p, s->pz.p, s->pp0.p, d1, d2);
  pcgb_init_fin<<<ns, kBlock, 0, s->st>>>(d1, d2, s->scn_rng.p, s->sc_mask.p, s->nsv, sc, rtol);
  s->mat_h.resize(sizeof(Mat<double>) + sizeof(Mat<float>));
  Mat<double> M64 = make_mat<double>(s, s->bsr_val.p, s->c_val.p);
  Mat<float> M32 = make_mat<float>(s, s->bsr_val32.p, s->c_val32.p);
  std::memcpy(s->mat_h.data(), &M64, sizeof(M64));
  std::memcpy(s->mat_h.data() + sizeof(M64), &M32, sizeof(M32));
  s->mat_dev.reserve(s->mat_h.size());
  ZCHK(hipMemcpyAsync(s->mat_dev.p, s->mat_h.data(), s->mat_h.size(), hipMemcpyHostToDevice, s->st));
  const Mat<double>* D64 = (const Mat<double>*)s->mat_dev.p;
  const Mat<float>* D32 = (const Mat<float>*)(s->mat_dev.p + sizeof(Mat<double>));
  const int g = spmv_grid(s);
  const double bytes = (s->mixed ? 40.0 : 76.0) * (s->nnzb + s->nnzc) + 32.0 * s->ndof;
  auto iteration = [&](double* pold, double* pnew, hipStream_t st) {
    if (g) {
      if (s->mixed)
        pcgb_spmv_kernel<float><<<g, kBlock, 0, st>>>(D32, s->v_scene.p, s->f_scene.p, sc, s->pz.p, pold, pnew, s->pq.p,
                                                      pqn);
      else
        pcgb_spmv_kernel<double><<<g, kBlock, 0, st>>>(D64, s->v_scene.p, s->f_scene.p, sc, s->pz.p, pold, pnew,
                                                       s->pq.p, pqn);
    }
  };
  auto rest = [&](double* pnew, hipStream_t st) {
    pcgb_alpha_kernel<<<ns, kBlock, 0, st>>>(pqn, s->scn_rng.p, s->nsv, sc);
    if (nunits)
      pcgb_update_kernel<<<nblocks(nunits), kBlock, 0, st>>>(s->nsv, s->nfree, s->v_scene.p, s->f_scene.p, sc, pnew,
                                                             s->pq.p, s->minv_soft.p, s->minv_body.p, sol, s->pr.p,
                                                             s->pz.p, d1, d2);
    pcgb_beta_kernel<<<ns, kBlock, 0, st>>>(d1, d2, s->scn_rng.p, s->nsv, 0, sc);
  };
  // a chunk of 16 iterations (even: p_old is pp0 at every chunk start), captured once
  // per set of buffers and replayed
  const bool timed = s->kt[KT_SPMV].on;
  bool graph_ok = false;
  if (s->use_graph && !timed) {
    std::vector<const void*> key = {D64, sc, sol, pqn, d1, d2, s->pz.p, s->pp0.p, s->pp1.p, s->pq.p, s->pr.p,
                                    s->minv_soft.p, s->minv_body.p, (const void*)(intptr_t)g,
                                    (const void*)(intptr_t)s->mixed, (const void*)(intptr_t)ns};
    PcgGraph& G = s->pcgb_graph;
    graph_ok = G.exec && G.key == key;
    if (!graph_ok) {
      if (G.exec) {
        ZCHK(hipGraphExecDestroy(G.exec));
        G.exec = nullptr;
      }
      if (!s->cap_st) ZCHK(hipStreamCreate(&s->cap_st));
      if (hipStreamBeginCapture(s->cap_st, hipStreamCaptureModeRelaxed) == hipSuccess) {
        double* po = s->pp0.p;
        double* pn = s->pp1.p;
        for (int c = 0; c < 16; ++c) {
          iteration(po, pn, s->cap_st);
          rest(pn, s->cap_st);
          std::swap(po, pn);
        }
        hipGraph_t graph = nullptr;
        bool ok = hipStreamEndCapture(s->cap_st, &graph) == hipSuccess && graph;
        if (ok) ok = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        if (ok) {
          G.key = key;
          graph_ok = true;
        } else {
          G.exec = nullptr;
        }
      }
    }
  }
  double* pold = s->pp0.p;
  double* pnew = s->pp1.p;
  std::vector<double> hs((size_t)16 * ns);
  const int chunk = 16;
  int it = 0;
  for (;;) {
    if (graph_ok && max_iter - it >= chunk) {
      ZCHK(hipGraphLaunch(s->pcgb_graph.exec, s->st));
      it += chunk;
    } else {
      for (int c = 0; c < chunk && it < max_iter; ++c, ++it) {
        kt_begin(s, KT_SPMV);
        iteration(pold, pnew, s->st);
        kt_end(s, KT_SPMV, bytes);
        rest(pnew, s->st);
        std::swap(pold, pnew);
      }
    }
    ZCHK(hipMemcpyAsync(hs.data(), sc, sizeof(double) * 16 * ns, hipMemcpyDeviceToHost, s->st));
    ZCHK(hipStreamSynchronize(s->st));
    bool all = true;
    for (int k = 0; k < ns; ++k) all = all && hs[16 * k + 6] != 0.0;
    if (all || it >= max_iter) break;
  }
  int bad;
  ZCHK(hipMemcpyAsync(&bad, s->counters.p + 4, sizeof(int), hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
  for (int k = 0; k < ns; ++k) {
    const double* c = hs.data() + 16 * k;
    iters[k] = (int)c[7];
    relres[k] = c[5] > 0.0 ? std::sqrt(c[4] / c[5]) : 0.0;
    status[k] = (bad || c[8] != 0.0 || c[6] == 0.0) ? ZEMA_E_PCG : 0;
  }
}

}  // namespace zema

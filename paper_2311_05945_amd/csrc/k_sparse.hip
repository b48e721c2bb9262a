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
#include <climits>
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

// x = a + beta b at node c (DOF vectors stay FP64; converted to the accumulation type
// A for the product: A = V, or double for the FP64 residual check of FP32 blocks)
template <class V, class A = V>
__device__ inline void blk_acc(const V* __restrict__ v, int stride, int j, const double* a, const double* b,
                               double beta, int c, Acc3<A>& acc) {
  double u0 = a[3 * c], u1 = a[3 * c + 1], u2 = a[3 * c + 2];
  if (b) {
    u0 += beta * b[3 * c];
    u1 += beta * b[3 * c + 1];
    u2 += beta * b[3 * c + 2];
  }
  A x0 = A(u0), x1 = A(u1), x2 = A(u2);
  acc.x += A(v[j]) * x0 + A(v[stride + j]) * x1 + A(v[2 * stride + j]) * x2;
  acc.y += A(v[3 * stride + j]) * x0 + A(v[4 * stride + j]) * x1 + A(v[5 * stride + j]) * x2;
  acc.z += A(v[6 * stride + j]) * x0 + A(v[7 * stride + j]) * x1 + A(v[8 * stride + j]) * x2;
}

template <class V, class A = V>
__device__ inline Acc3<A> row_partial(const Mat<V>& M, int row, int lane, int nl, const double* a, const double* b,
                                      double beta) {
  Acc3<A> acc{A(0), A(0), A(0)};
  for (int j = M.bp[row] + lane; j < M.bp[row + 1]; j += nl)
    blk_acc<V, A>(M.bv, M.nnzb, j, a, b, beta, M.bc[j], acc);
  if (M.cp)
    for (int j = M.cp[row] + lane; j < M.cp[row + 1]; j += nl)
      blk_acc<V, A>(M.cv, M.nnzc, j, a, b, beta, M.cc[j], acc);
  return acc;
}

// q = H x with x = a + beta b.  Writes xo = x for the rows it owns and the block
// partial of x . q when those pointers are given.  Soft rows: 16 lanes each; affine
// rows: one block each.
template <class V, class A = V>
__device__ inline double spmv_rows(const Mat<V>& M, const double* a, const double* b, double beta, double* q,
                                   double* xo, double* sh_red /* 3 * waves */) {
  int nsoft_blocks = (M.nsv + (kBlock / RG) - 1) / (kBlock / RG);
  double dotv = 0.0;
  if ((int)blockIdx.x < nsoft_blocks) {
    int row = blockIdx.x * (kBlock / RG) + threadIdx.x / RG;
    int lane = threadIdx.x % RG;
    Acc3<A> acc{A(0), A(0), A(0)};
    if (row < M.nsv) acc = row_partial<V, A>(M, row, lane, RG, a, b, beta);
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
    Acc3<A> acc = row_partial<V, A>(M, row, threadIdx.x, kBlock, a, b, beta);
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

template <class V, class A = V>
__global__ void spmv_kernel(Mat<V> M, const double* __restrict__ x, double* __restrict__ out) {
  __shared__ double red[3 * (kBlock / 64)];
  spmv_rows<V, A>(M, x, nullptr, 0.0, out, nullptr, red);
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

// ------------------------------------------------------------------ BSR export
// Static blocks (tets, affine bodies) and contact blocks share the node numbering and
// both keep ascending columns per row; a row of the export is their merge, a column
// present in both summed in FP64.  One thread per row (an export, not the hot loop).
template <class V>
__global__ void bsr_export_count_kernel(Mat<V> M, int* __restrict__ cnt) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= M.nnodes) return;
  int i = M.bp[r], ie = M.bp[r + 1], j = 0, je = 0;
  if (M.cp) {
    j = M.cp[r];
    je = M.cp[r + 1];
  }
  int n = 0;
  while (i < ie || j < je) {
    int ci = i < ie ? M.bc[i] : INT_MAX, cj = j < je ? M.cc[j] : INT_MAX;
    if (ci <= cj) ++i;
    if (cj <= ci) ++j;
    ++n;
  }
  cnt[r] = n;
}

template <class V>
__global__ void bsr_export_fill_kernel(Mat<V> M, const int* __restrict__ off, int* __restrict__ col,
                                       double* __restrict__ val) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= M.nnodes) return;
  int i = M.bp[r], ie = M.bp[r + 1], j = 0, je = 0;
  if (M.cp) {
    j = M.cp[r];
    je = M.cp[r + 1];
  }
  int o = off[r];
  while (i < ie || j < je) {
    int ci = i < ie ? M.bc[i] : INT_MAX, cj = j < je ? M.cc[j] : INT_MAX;
    int c = ci < cj ? ci : cj;
    double b[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (ci == c) {
      for (int q = 0; q < 9; ++q) b[q] += double(M.bv[(size_t)q * M.nnzb + i]);
      ++i;
    }
    if (cj == c) {
      for (int q = 0; q < 9; ++q) b[q] += double(M.cv[(size_t)q * M.nnzc + j]);
      ++j;
    }
    col[o] = c;
    for (int q = 0; q < 9; ++q) val[(size_t)9 * o + q] = b[q];
    ++o;
  }
}

int64_t k_hessian_bsr(zema_scene* s, int* row_ptr, int* col, double* val, int64_t cap) {
  const int n = s->nnodes;
  s->cnt.reserve((size_t)n + 1);
  s->offs.reserve((size_t)n + 1);
  if (n == 0) return 0;
  if (s->mixed)
    bsr_export_count_kernel<float><<<nblocks(n), kBlock, 0, s->st>>>(make_mat<float>(s, s->bsr_val32.p, s->c_val32.p),
                                                                     s->cnt.p);
  else
    bsr_export_count_kernel<double><<<nblocks(n), kBlock, 0, s->st>>>(make_mat<double>(s, s->bsr_val.p, s->c_val.p),
                                                                      s->cnt.p);
  int64_t total = k_exclusive_scan(s, s->cnt.p, s->offs.p, n, true);
  if (total > cap || !row_ptr || !col || !val) return total;
  if (s->mixed)
    bsr_export_fill_kernel<float><<<nblocks(n), kBlock, 0, s->st>>>(make_mat<float>(s, s->bsr_val32.p, s->c_val32.p),
                                                                    s->offs.p, col, val);
  else
    bsr_export_fill_kernel<double><<<nblocks(n), kBlock, 0, s->st>>>(make_mat<double>(s, s->bsr_val.p, s->c_val.p),
                                                                     s->offs.p, col, val);
  int tot32 = (int)total;
  ZCHK(hipMemcpyAsync(row_ptr, s->offs.p, sizeof(int) * n, hipMemcpyDeviceToDevice, s->st));
  ZCHK(hipMemcpyAsync(row_ptr + n, &tot32, sizeof(int), hipMemcpyHostToDevice, s->st));
  ZCHK(hipStreamSynchronize(s->st));
  return total;
}

// out = H v with FP64 accumulation (the mixed form's FP32 blocks converted exactly)
void k_hess_matvec64(zema_scene* s, const double* v, double* out) {
  int g = spmv_grid(s);
  if (!g) return;
  if (s->mixed)
    spmv_kernel<float, double><<<g, kBlock, 0, s->st>>>(make_mat<float>(s, s->bsr_val32.p, s->c_val32.p), v, out);
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
  if (!s->cap_st) ZCHK(hipStreamCreateWithFlags(&s->cap_st, hipStreamNonBlocking));
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

static void k_pcg_cg(zema_scene* s, const void* mat, int lanes, double bytes, const double* rhs, double* sol,
                     double rtol, int max_iter, const int* active_host, int* iters, double* relres, int* status,
                     int* breakdown);

int k_pcg(zema_scene* s, const double* rhs, double* sol, double rtol, int max_iter, int* iters, double* relres,
          int* breakdown) {
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
  // 4 lanes per soft row exist for the single-reduction kernel only
  const int lanes = (s->tune_lanes == 4 && s->pcg_form != 1) ? 8 : s->tune_lanes, ub = s->tune_ublock;
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
  if (s->pcg_form == 1) {
    // matrix once; r, w, s, p, x read and written once per DOF; 3x3 inverse blocks;
    // node records read and written once
    a.bytes = (s->mixed ? 40.0 : 76.0) * (s->nnzb + s->nnzc) + 152.0 * s->ndof;
    int one = 1, st = 0;
    k_pcg_cg(s, a.mat, lanes, a.bytes, rhs, sol, rtol, max_iter, &one, iters, relres, &st, breakdown);
    return st;
  }
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
  if (breakdown) *breakdown = hs[8] != 0.0;
  if (bad) return ZEMA_E_PCG;
  if (hs[8] != 0.0) return ZEMA_E_PCG;
  if (hs[6] == 0.0) return ZEMA_E_PCG;
  return 0;
}

// ------------------------------------------------------------------ single-reduction PCG
// The same preconditioned CG iterates, rearranged after Chronopoulos and Gear (1989) so
// that both inner products of an iteration come from one reduction:
//   gamma_k = r_k . z_k,  delta_k = z_k . w_k  (z_k = M^-1 r_k, w_k = H z_k)
//   beta_k = gamma_k / gamma_{k-1},  alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1})
//   p_k = z_k + beta_k p_{k-1},  s_k = w_k + beta_k s_{k-1}  (s_k = H p_k)
//   x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k s_k
// (delta_k - beta_k gamma_k / alpha_{k-1} equals p_k . H p_k, the standard denominator.)
// One launch per iteration.  Every block reduces the previous launch's partials of its
// scene into gamma_k, delta_k, |r_k|^2 (same order in every block of the scene).  The
// product w_{k+1} = H z_{k+1}, z_{k+1} = M^-1 r_k - alpha_k (M^-1 w_k + beta_k M^-1 s_{k-1}),
// is gathered as three accumulators over a per-node record Z = (M^-1 r_k, M^-1 w_k,
// M^-1 s_{k-1}) written by the previous launch (double-buffered by parity), so the
// gathers are issued before the reduction.  r, w, s, p and x are read and written only
// by the owning row (in place).  An affine body's four node rows share one block,
// which applies the body's 12x12 inverse block to form the body's Z records.
//
// Batches: the Newton system of a batch is block diagonal, and every scene runs its own
// CG (own scalars, residual test, breakdown flag, iteration count) in the same
// launches.  Soft-row blocks never straddle scenes, so a scene's blocks, partials and
// summation order are those it has alone.  Per-scene scalars [ns][16]: 0/1 gamma,
// 2/3 alpha (by parity), 4 rr, 5 bb, 6 done, 7 iterations, 8 breakdown, 9 tol^2.
constexpr int kZs = 16;  // doubles per node record: M^-1 r, M^-1 w, M^-1 s (9 used, one cache line)

struct CgVec {
  const double *ms, *mb;  // preconditioner: 3x3 soft blocks (9 planes), 12x12 body blocks
  double *x, *p, *r, *w, *s;
  const double* zin;      // node records of iteration k
  double* zout;           // node records of iteration k + 1
  const double* cin;      // partials (gamma_k, delta_k, rr_k) per block, scene-contiguous
  double* cout;           // partials of iteration k + 1
  double* sc;             // per-scene scalars
  const int4* tab;        // soft workgroups in launch order: first row, rows, scene, partial slot
  const int4* binfo;      // every block: its scene's partial slots [x, y), scene, own slot
  int nsoft_blocks;
  int nslots;             // partial slots of all scenes
  int rpb;                // soft rows per block
  int nsv_single;  // a single scene: its soft rows (the block table is then implied), else -1
  double rtol;
};

template <class V>
__device__ inline void mul_acc(const V* m, double u0, double u1, double u2, Acc3<V>& acc) {
  V x0 = V(u0), x1 = V(u1), x2 = V(u2);
  acc.x += m[0] * x0 + m[1] * x1 + m[2] * x2;
  acc.y += m[3] * x0 + m[4] * x1 + m[5] * x2;
  acc.z += m[6] * x0 + m[7] * x1 + m[8] * x2;
}

// loads through global-memory pointers (the matrix descriptor is read from device
// memory, so its pointers would otherwise be generic and load through the flat path)
template <class T>
__device__ inline T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// Entries [j, end) step nl of one part of a row, software-pipelined: the column index
// and values of the next entry are requested while the current entry's node record
// is in flight, so each entry costs about one memory round trip instead of two.
template <class V>
__device__ inline void cg_seg(const V* v, int stride, const int* cols, int j, int end, int nl, const double* Z,
                              Acc3<V>& A, Acc3<V>& B, Acc3<V>& C) {
  if (j >= end) return;
  int c = gld(cols + j);
  V m[9];
  for (int t = 0; t < 9; ++t) m[t] = gld(v + (size_t)t * stride + j);
  for (;;) {
    const double* z = Z + (size_t)kZs * c;
    double zz[9];
    for (int t = 0; t < 9; ++t) zz[t] = z[t];
    const int jn = j + nl;
    const bool more = jn < end;
    int cn = 0;
    V mn[9];
    if (more) {
      cn = gld(cols + jn);
      for (int t = 0; t < 9; ++t) mn[t] = gld(v + (size_t)t * stride + jn);
    }
    mul_acc(m, zz[0], zz[1], zz[2], A);
    mul_acc(m, zz[3], zz[4], zz[5], B);
    mul_acc(m, zz[6], zz[7], zz[8], C);
    if (!more) break;
    j = jn;
    c = cn;
    for (int t = 0; t < 9; ++t) m[t] = mn[t];
  }
}

// row extents [b0, b1) of the static part and [c0, c1) of the contact part
template <class V>
__device__ inline void cg_row(const Mat<V>& M, const double* Z, int4 e, int lane, int nl, Acc3<V>& A, Acc3<V>& B,
                              Acc3<V>& C) {
  cg_seg(M.bv, M.nnzb, M.bc, e.x + lane, e.y, nl, Z, A, B, C);
  cg_seg(M.cv, M.nnzc, M.cc, e.z + lane, e.w, nl, Z, A, B, C);
}

template <class V>
__device__ inline void acc_xor(Acc3<V>& A, int o, int w) {
  A.x += __shfl_xor(A.x, o, w);
  A.y += __shfl_xor(A.y, o, w);
  A.z += __shfl_xor(A.z, o, w);
}

__device__ inline V3 m3v(const double* m, V3 v) {
  return v3(m[0] * v.x + m[1] * v.y + m[2] * v.z, m[3] * v.x + m[4] * v.y + m[5] * v.z,
            m[6] * v.x + m[7] * v.y + m[8] * v.z);
}

// Sums of three per-thread values over the block, each in block_sum's order (wave tree,
// then waves in order); the results are returned to every thread.
__device__ inline void block_sum3(double& a, double& b, double& c, double* sh /* 3 * waves + 3 */) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    sh[3 * w] = a;
    sh[3 * w + 1] = b;
    sh[3 * w + 2] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0.0, y = 0.0, z = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) {
      x += sh[3 * i];
      y += sh[3 * i + 1];
      z += sh[3 * i + 2];
    }
    sh[3 * (kBlock / 64)] = x;
    sh[3 * (kBlock / 64) + 1] = y;
    sh[3 * (kBlock / 64) + 2] = z;
  }
  __syncthreads();
  a = sh[3 * (kBlock / 64)];
  b = sh[3 * (kBlock / 64) + 1];
  c = sh[3 * (kBlock / 64) + 2];
}

// Scalars: zero, done for scenes that do not solve (their x stays 0).
__global__ void cg_scal_init(int ns, const int* __restrict__ active, double* __restrict__ sc) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ns) return;
  for (int t = 0; t < 16; ++t) sc[16 * k + t] = 0.0;
  sc[16 * k + 6] = active[k] ? 0.0 : 1.0;
}

// Set-up: x = 0, r_0 = b, w = s = p = 0 and the records (M^-1 b, 0, 0).  Soft nodes one
// per thread; then one block per free body (12 threads: M^-1 applied to its 12 DOFs).
__global__ void cg_setup_kernel(int nsv, int nfree, const double* __restrict__ rhs, CgVec a) {
  const int nsb = (nsv + kBlock - 1) / kBlock;
  if ((int)blockIdx.x < nsb) {
    int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nsv) return;
    double m[9];
    for (int t = 0; t < 9; ++t) m[t] = a.ms[(size_t)t * nsv + i];
    V3 b = ld3(rhs + 3 * i), z0 = v3(0, 0, 0);
    st3(a.r + 3 * i, b);
    st3(a.x + 3 * i, z0);
    st3(a.w + 3 * i, z0);
    st3(a.s + 3 * i, z0);
    st3(a.p + 3 * i, z0);
    double* z = a.zout + (size_t)kZs * i;
    V3 zr = m3v(m, b);
    z[0] = zr.x;
    z[1] = zr.y;
    z[2] = zr.z;
    for (int t = 3; t < 9; ++t) z[t] = 0.0;
  } else {
    int bi = blockIdx.x - nsb, t = threadIdx.x;
    if (bi >= nfree || t >= 12) return;
    size_t o = 3 * (size_t)nsv + 12 * (size_t)bi;
    a.r[o + t] = rhs[o + t];
    a.x[o + t] = 0.0;
    a.w[o + t] = 0.0;
    a.s[o + t] = 0.0;
    a.p[o + t] = 0.0;
    double acc = 0.0;
    const double* M = a.mb + 144 * (size_t)bi + 12 * t;
    for (int d = 0; d < 12; ++d) acc += M[d] * rhs[o + d];
    double* z = a.zout + (size_t)kZs * (nsv + 4 * bi + t / 3);
    z[t % 3] = acc;
    z[3 + t % 3] = 0.0;
    z[6 + t % 3] = 0.0;
  }
}

// Workgroups of a launch are dispatched round-robin over the device's 8 XCDs, each
// with its own L2.  In a single-scene solve, soft workgroup b takes logical block
// xcd_block(b, n) (common.hpp), so each XCD holds a contiguous run of rows: the
// neighbour records its rows gather are shared in its own L2 rather than fetched by
// every XCD, and each XCD works on the same rows in every iteration.  (Batches keep
// the plain order: there a contiguous run would be about one scene per XCD, and the
// XCDs of scenes that have converged would idle.)

// One iteration (START: the first product w_0 = H M^-1 b with alpha = beta = 0 and no
// reduction; it leaves p = M^-1 b, which the first iteration scales by beta = 0).
// Blocks of a finished scene return before gathering.
template <class V, int G, bool START>
__global__ void __launch_bounds__(kBlock) pcg_cg_kernel(const Mat<V>* __restrict__ Mp, int k, CgVec a) {
  const Mat<V> M = *Mp;
  __shared__ double sh[3 * (kBlock / 64) + 3];
  __shared__ double bv[3][12];  // a body's r_{k+1}, w_{k+1}, s_k
  const bool soft = (int)blockIdx.x < a.nsoft_blocks;
  const int blk = soft && a.nsv_single >= 0 ? xcd_block(blockIdx.x, a.nsoft_blocks) : (int)blockIdx.x;
  int scene, slot, row, lane;
  int2 pr;
  bool valid;
  if (a.nsv_single >= 0) {  // one scene: logical block b holds partial slot b
    scene = 0;
    slot = blk;
    pr = make_int2(0, a.nslots);
  } else {
    const int4 b = a.binfo[blk];
    pr = make_int2(b.x, b.y);
    scene = b.z;
    slot = b.w;
  }
  if (soft) {
    lane = threadIdx.x % G;
    if (a.nsv_single >= 0) {  // block b holds rows b * rpb onward
      row = blk * a.rpb + threadIdx.x / G;
      valid = (int)threadIdx.x / G < a.rpb && row < a.nsv_single;
    } else {
      const int4 t = a.tab[blk];
      valid = (int)threadIdx.x / G < t.y;
      row = t.x + threadIdx.x / G;
    }
  } else {  // wavefront m of the block: node row m of the body
    lane = threadIdx.x & 63;
    valid = true;
    row = M.nsv + 4 * (blockIdx.x - a.nsoft_blocks) + (threadIdx.x >> 6);
  }
  double* c = a.sc + 16 * scene;
  // row extents, the scene's scalars and its flag are independent loads; the flag is
  // read once per block (the scene's first block may set it during this launch)
  __shared__ int skip_s;
  int4 ext = make_int4(0, 0, 0, 0);
  if (valid) {
    ext.x = gld(M.bp + row);
    ext.y = gld(M.bp + row + 1);
    if (M.cp) {
      ext.z = gld(M.cp + row);
      ext.w = gld(M.cp + row + 1);
    }
  }
  double gprev = 1.0, aprev = 1.0, tol2 = 0.0;
  double c1 = 0.0, c2 = 0.0, c3 = 0.0;
  const int i0 = pr.x + threadIdx.x;
  if (!START) {
    if (k > 0) {
      gprev = c[(k - 1) & 1];
      aprev = c[2 + ((k - 1) & 1)];
      tol2 = c[9];
    }
  }
  if (threadIdx.x == 0) skip_s = START ? 0 : c[6] != 0.0;
  __syncthreads();
  if (skip_s) return;
  if (!START)  // a scene with more partial slots than threads per block
    for (int i = i0; i < pr.y; i += kBlock) {
      c1 += a.cin[3 * i];
      c2 += a.cin[3 * i + 1];
      c3 += a.cin[3 * i + 2];
    }
  Acc3<V> A{V(0), V(0), V(0)}, B{V(0), V(0), V(0)}, C{V(0), V(0), V(0)};
  if (soft) {
    cg_row(M, a.zin, ext, lane, G, A, B, C);
    for (int o = G / 2; o > 0; o >>= 1) {
      acc_xor(A, o, G);
      acc_xor(B, o, G);
      acc_xor(C, o, G);
    }
  } else {
    cg_row(M, a.zin, ext, lane, 64, A, B, C);
    for (int o = 32; o > 0; o >>= 1) {
      acc_xor(A, o, 64);
      acc_xor(B, o, 64);
      acc_xor(C, o, 64);
    }
  }
  const bool own = lane == 0 && valid;
  V3 rv{}, wv{}, sv{}, pv{}, xv{}, zr{}, zw{}, zs{};
  double mi[9];
  if (own) {
    rv = ld3(a.r + 3 * row);
    wv = ld3(a.w + 3 * row);
    sv = ld3(a.s + 3 * row);
    pv = ld3(a.p + 3 * row);
    xv = ld3(a.x + 3 * row);
    const double* z = a.zin + (size_t)kZs * row;
    zr = v3(z[0], z[1], z[2]);
    zw = v3(z[3], z[4], z[5]);
    zs = v3(z[6], z[7], z[8]);
    if (soft)
      for (int t = 0; t < 9; ++t) mi[t] = a.ms[(size_t)t * M.nsv + row];
  }
  double alpha = 0.0, beta = 0.0;
  if (!START) {
    block_sum3(c1, c2, c3, sh);
    const double gam = c1, del = c2, rr = c3;
    if (k == 0) tol2 = a.rtol * a.rtol * rr;
    const bool first = slot == pr.x && threadIdx.x == 0;  // the scene's first block
    if (first) {
      c[4] = rr;
      if (k == 0) {
        c[5] = rr;
        c[9] = tol2;
      }
    }
    if (rr <= tol2) {
      if (first) c[6] = 1.0;
      return;
    }
    beta = k > 0 ? gam / gprev : 0.0;
    const double den = k > 0 ? del - beta * gam / aprev : del;
    if (!(den > 0.0)) {
      if (first) {
        c[8] = 1.0;
        c[6] = 1.0;
      }
      return;
    }
    alpha = gam / den;
    if (first) {
      c[k & 1] = gam;
      c[2 + (k & 1)] = alpha;
      c[7] += 1.0;  // iterations completed after this launch
    }
  }
  double g1 = 0.0, d1 = 0.0, r1 = 0.0;
  if (own) {
    const V3 wn = v3(double(A.x), double(A.y), double(A.z)) -
                  alpha * (v3(double(B.x), double(B.y), double(B.z)) + beta * v3(double(C.x), double(C.y), double(C.z)));
    const V3 sk = wv + beta * sv;
    const V3 pk = zr + beta * pv;
    const V3 rn = rv - alpha * sk;
    const V3 zn = zr - alpha * (zw + beta * zs);
    st3(a.s + 3 * row, sk);
    st3(a.p + 3 * row, pk);
    st3(a.x + 3 * row, xv + alpha * pk);
    st3(a.r + 3 * row, rn);
    st3(a.w + 3 * row, wn);
    g1 = dot(rn, zn);
    d1 = dot(zn, wn);
    r1 = dot(rn, rn);
    if (soft) {
      double* z = a.zout + (size_t)kZs * row;
      V3 q = m3v(mi, rn);
      z[0] = q.x;
      z[1] = q.y;
      z[2] = q.z;
      q = m3v(mi, wn);
      z[3] = q.x;
      z[4] = q.y;
      z[5] = q.z;
      q = m3v(mi, sk);
      z[6] = q.x;
      z[7] = q.y;
      z[8] = q.z;
    } else {
      int m = threadIdx.x >> 6;
      bv[0][3 * m] = rn.x;
      bv[0][3 * m + 1] = rn.y;
      bv[0][3 * m + 2] = rn.z;
      bv[1][3 * m] = wn.x;
      bv[1][3 * m + 1] = wn.y;
      bv[1][3 * m + 2] = wn.z;
      bv[2][3 * m] = sk.x;
      bv[2][3 * m + 1] = sk.y;
      bv[2][3 * m + 2] = sk.z;
    }
  }
  if (!soft) {  // the body's records: its 12x12 inverse block applied to r, w and s
    __syncthreads();
    int t = threadIdx.x;
    if (t < 36) {
      int q = t / 12, i = t % 12, bi = blockIdx.x - a.nsoft_blocks;
      const double* Mb = a.mb + 144 * (size_t)bi + 12 * i;
      double acc = 0.0;
      for (int d = 0; d < 12; ++d) acc += Mb[d] * bv[q][d];
      a.zout[(size_t)kZs * (M.nsv + 4 * bi + i / 3) + 3 * q + i % 3] = acc;
    }
  }
  block_sum3(g1, d1, r1, sh);
  if (threadIdx.x == 0) {
    a.cout[3 * slot] = g1;
    a.cout[3 * slot + 1] = d1;
    a.cout[3 * slot + 2] = r1;
  }
}

// x = M^-1 b for the units of the scenes flagged in mask (a solve that met
// non-positive curvature at its first iteration)
__global__ void cg_precond_rhs_kernel(int nsv, int nfree, const double* __restrict__ ms, const double* __restrict__ mb,
                                      const double* __restrict__ rhs, double* __restrict__ sol,
                                      const int* __restrict__ mask, const int* __restrict__ v_scene,
                                      const int* __restrict__ f_scene) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsv + nfree) return;
  if (!mask[i < nsv ? v_scene[i] : f_scene[i - nsv]]) return;
  apply_minv(i, nsv, ms, mb, rhs, sol);
}

// after the last iteration: |r|^2 and convergence of every unfinished scene
__global__ void pcg_cg_final_kernel(const int2* __restrict__ prng, const double* __restrict__ cin,
                                    double* __restrict__ sc) {
  double* c = sc + 16 * blockIdx.x;
  if (c[6] != 0.0) return;
  __shared__ double sh[kBlock / 64];
  const int2 pr = prng[blockIdx.x];
  double rr = 0.0;
  for (int i = pr.x + threadIdx.x; i < pr.y; i += kBlock) rr += cin[3 * i + 2];
  rr = block_sum<kBlock>(rr, sh);
  if (threadIdx.x == 0) {
    c[4] = rr;
    if (rr <= c[9]) c[6] = 1.0;
  }
}

// Soft rows per workgroup: the requested number, else enough rows for one workgroup
// per compute unit (a 10k-row system on 256 compute units: 40), at most kBlock / lanes.
static int cg_rows_per_block(zema_scene* s, int lanes) {
  const int cap = kBlock / lanes;
  if (s->tune_cg_rows > 0) return std::min(s->tune_cg_rows, cap);
  if (s->n_cu <= 0) {
    int dev = 0;
    ZCHK(hipGetDevice(&dev));
    ZCHK(hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  }
  return std::min(cap, std::max(1, (s->nsv + s->n_cu - 1) / std::max(s->n_cu, 1)));
}

// Block layout of the single-reduction kernels for the given lanes per soft row:
// scene-aligned soft blocks, then one block per free body; partial slots grouped by
// scene (its soft blocks, then its bodies).
static void cg_layout(zema_scene* s, int lanes) {
  const int rpb = cg_rows_per_block(s, lanes);
  std::vector<int> key = {lanes, s->ns, s->nsv, s->nfree, rpb};
  if (s->cg_key == key) return;
  std::vector<int4> tab;
  std::vector<int2> prng(s->ns);
  std::vector<int> fslot(std::max(s->nfree, 1)), fscene(std::max(s->nfree, 1));
  int slot = 0;
  std::vector<int> soft_slot0(s->ns), nsb(s->ns);
  for (int k = 0; k < s->ns; ++k) {
    const SceneRange& R = s->scn[k];
    prng[k].x = slot;
    soft_slot0[k] = slot;
    nsb[k] = (R.v1 - R.v0 + rpb - 1) / rpb;
    slot += nsb[k] + (R.f1 - R.f0);
    prng[k].y = slot;
  }
  for (int k = 0; k < s->ns; ++k) {
    const SceneRange& R = s->scn[k];
    for (int b = 0; b < nsb[k]; ++b) {
      int r0 = R.v0 + b * rpb;
      tab.push_back(make_int4(r0, std::min(rpb, R.v1 - r0), k, soft_slot0[k] + b));
    }
    for (int f = R.f0; f < R.f1; ++f) {
      fslot[f] = soft_slot0[k] + nsb[k] + (f - R.f0);
      fscene[f] = k;
    }
  }
  // Batches: soft workgroup b runs on XCD b mod 8 (round-robin dispatch).  Each scene's
  // blocks are cut into 8 contiguous runs, run x placed on XCD x, so a scene's rows stay
  // in the same XCD's L2 from one iteration to the next while every XCD holds a share of
  // every scene (a converged scene frees all XCDs alike).  A permutation of the table:
  // slots, and so every sum, are unchanged.
  const int nsoft = (int)tab.size();
  if (s->ns > 1 && nsoft >= 8) {
    std::vector<std::vector<int>> q(8);
    int l0 = 0;
    for (int k = 0; k < s->ns; ++k) {
      for (int x = 0; x < 8; ++x)
        for (int l = l0 + x * nsb[k] / 8; l < l0 + (x + 1) * nsb[k] / 8; ++l) q[x].push_back(l);
      l0 += nsb[k];
    }
    std::vector<int> spill;
    for (int x = 0; x < 8; ++x) {
      const size_t cap = nsoft / 8 + (x < nsoft % 8 ? 1 : 0);
      while (q[x].size() > cap) {
        spill.push_back(q[x].back());
        q[x].pop_back();
      }
    }
    for (int x = 0; x < 8; ++x) {
      const size_t cap = nsoft / 8 + (x < nsoft % 8 ? 1 : 0);
      while (q[x].size() < cap) {
        q[x].push_back(spill.back());
        spill.pop_back();
      }
    }
    std::vector<int4> perm(nsoft);
    for (int b = 0; b < nsoft; ++b) perm[b] = tab[q[b % 8][b / 8]];
    tab.swap(perm);
  }
  std::vector<int4> binfo;
  for (const int4& t : tab) binfo.push_back(make_int4(prng[t.z].x, prng[t.z].y, t.z, t.w));
  for (int f = 0; f < s->nfree; ++f)
    binfo.push_back(make_int4(prng[fscene[f]].x, prng[fscene[f]].y, fscene[f], fslot[f]));
  s->cg_nsoft_blocks = (int)tab.size();
  s->cg_nslots = slot;
  s->cg_rpb = rpb;
  if (tab.empty()) tab.push_back(make_int4(0, 0, 0, 0));
  s->cg_tab.upload(tab, s->st);
  s->cg_prng.upload(prng, s->st);
  if (binfo.empty()) binfo.push_back(make_int4(0, 0, 0, 0));
  s->cg_binfo.upload(binfo, s->st);
  s->cg_key = key;
}

// records by parity: launch k reads Z and partials of slot k & 1 and writes slot
// (k + 1) & 1; k = -1 is the first product (the set-up writes slot 1)
static CgVec cg_vec(zema_scene* s, int k, double* sol, double rtol) {
  int e = k & 1, o = (k + 1) & 1;
  size_t zn = (size_t)kZs * s->nnodes;
  size_t pn = (size_t)3 * s->cg_nslots;
  CgVec a;
  a.ms = s->minv_soft.p;
  a.mb = s->minv_body.p;
  a.x = sol;
  a.p = s->pp0.p;
  a.r = s->pr.p;
  a.w = s->pq.p;
  a.s = s->pz.p;
  a.zin = s->cg_z.p + zn * e;
  a.zout = s->cg_z.p + zn * o;
  a.cin = s->cg_part.p + pn * e;
  a.cout = s->cg_part.p + pn * o;
  a.sc = s->scal.p;
  a.tab = s->cg_tab.p;
  a.binfo = s->cg_binfo.p;
  a.nsoft_blocks = s->cg_nsoft_blocks;
  a.nslots = s->cg_nslots;
  a.rpb = s->cg_rpb;
  a.nsv_single = s->ns == 1 ? s->nsv : -1;
  a.rtol = rtol;
  return a;
}

template <class V, bool START>
static void cg_launch_v(const void* mat, int lanes, int g, int k, const CgVec& a, hipStream_t st) {
  const Mat<V>* M = (const Mat<V>*)mat;
  if (lanes == 4)
    pcg_cg_kernel<V, 4, START><<<g, kBlock, 0, st>>>(M, k, a);
  else if (lanes == 8)
    pcg_cg_kernel<V, 8, START><<<g, kBlock, 0, st>>>(M, k, a);
  else if (lanes == 32)
    pcg_cg_kernel<V, 32, START><<<g, kBlock, 0, st>>>(M, k, a);
  else
    pcg_cg_kernel<V, 16, START><<<g, kBlock, 0, st>>>(M, k, a);
}

template <bool START>
static void cg_launch(zema_scene* s, const void* mat, int lanes, int k, const CgVec& a, hipStream_t st) {
  int g = s->cg_nsoft_blocks + s->nfree;
  if (g == 0) return;
  if (s->mixed)
    cg_launch_v<float, START>(mat, lanes, g, k, a, st);
  else
    cg_launch_v<double, START>(mat, lanes, g, k, a, st);
}

static bool cg_graph_ready(zema_scene* s, const void* mat, int lanes, double* sol) {
  std::vector<const void*> key = {mat, s->cg_part.p, s->scal.p, sol, s->pp0.p, s->pr.p, s->pq.p, s->pz.p, s->cg_z.p,
                                  s->minv_soft.p, s->minv_body.p, s->cg_tab.p, s->cg_prng.p, s->cg_binfo.p,
                                  (const void*)(intptr_t)s->cg_nslots,
                                  (const void*)(intptr_t)s->cg_nsoft_blocks, (const void*)(intptr_t)lanes,
                                  (const void*)(intptr_t)s->cg_rpb,
                                  (const void*)(intptr_t)s->mixed, (const void*)(intptr_t)s->nsv,
                                  (const void*)(intptr_t)s->nfree, (const void*)(intptr_t)s->nnodes,
                                  (const void*)(intptr_t)s->ns};
  PcgGraph& G = s->pcg_graph;
  if (G.exec && G.key == key) return true;
  if (G.exec) {
    ZCHK(hipGraphExecDestroy(G.exec));
    G.exec = nullptr;
  }
  if (!s->cap_st) ZCHK(hipStreamCreateWithFlags(&s->cap_st, hipStreamNonBlocking));
  if (hipStreamBeginCapture(s->cap_st, hipStreamCaptureModeRelaxed) != hipSuccess) return false;
  for (int c = 0; c < kChunk; ++c) {
    int k = 1 + c;
    cg_launch<false>(s, mat, lanes, k, cg_vec(s, k, sol, 0.0), s->cap_st);
  }
  hipGraph_t graph = nullptr;
  bool ok = (hipStreamEndCapture(s->cap_st, &graph) == hipSuccess) && graph;
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

// Single-reduction solve of every scene whose active flag is set (others get x = 0);
// per-scene iterations, relative residuals and status on the host.
static void k_pcg_cg(zema_scene* s, const void* mat, int lanes, double bytes, const double* rhs, double* sol,
                     double rtol, int max_iter, const int* active_host, int* iters, double* relres, int* status,
                     int* breakdown) {
  const int ns = s->ns, n = s->ndof;
  s->pr.reserve(n);
  s->pz.reserve(n);
  s->pp0.reserve(n);
  s->pq.reserve(n);
  cg_layout(s, lanes);
  s->cg_z.reserve((size_t)2 * kZs * s->nnodes + kZs);
  s->cg_part.reserve((size_t)6 * s->cg_nslots + 6);
  s->scal.reserve((size_t)16 * ns);
  ZCHK(hipMemcpyAsync(s->sc_mask.p, active_host, sizeof(int) * ns, hipMemcpyHostToDevice, s->st));
  cg_scal_init<<<nblocks(ns), kBlock, 0, s->st>>>(ns, s->sc_mask.p, s->scal.p);
  {
    int nsb = (s->nsv + kBlock - 1) / kBlock;
    if (nsb + s->nfree > 0)
      cg_setup_kernel<<<nsb + s->nfree, kBlock, 0, s->st>>>(s->nsv, s->nfree, rhs, cg_vec(s, 0, sol, rtol));
    cg_launch<true>(s, mat, lanes, -1, cg_vec(s, -1, sol, rtol), s->st);
  }
  // The scalars of every chunk are copied to pinned host memory behind it; the host
  // checks the previous chunk's copy while the next chunk runs, so the device does not
  // wait for the host.  Launches after convergence return at once (the scene flags).
  // With the launch timer on, every chunk is checked before the next is launched, and
  // a replayed chunk whose 16 launches all iterated is timed by events around it.
  const bool timed = s->kt[KT_SPMV].on;
  if (s->poll_cap < 16 * ns) {
    if (s->poll_h) ZCHK(hipHostFree(s->poll_h));
    ZCHK(hipHostMalloc((void**)&s->poll_h, sizeof(double) * 32 * ns, hipHostMallocDefault));
    s->poll_cap = 16 * ns;
  }
  for (hipEvent_t& e : s->poll_ev)
    if (!e) ZCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (hipEvent_t& e : s->chunk_ev)
    if (!e) ZCHK(hipEventCreate(&e));
  auto all_done = [&](const double* h) {
    for (int k = 0; k < ns; ++k)
      if (h[16 * k + 6] == 0.0) return false;
    return true;
  };
  int it = 0, slot = 0, pending = -1;
  double iters_before = 0.0;
  for (;;) {
    bool graph = it > 0 && (it & 1) && max_iter - it >= kChunk && s->use_graph && cg_graph_ready(s, mat, lanes, sol);
    if (graph) {
      if (timed) ZCHK(hipEventRecord(s->chunk_ev[0], s->st));
      ZCHK(hipGraphLaunch(s->pcg_graph.exec, s->st));
      if (timed) ZCHK(hipEventRecord(s->chunk_ev[1], s->st));
      it += kChunk;
    } else {  // the first launch alone (replays start at odd iterations), then chunks
      const int nl = it == 0 ? 1 : kChunk;
      for (int c = 0; c < nl && it < max_iter; ++c, ++it)
        cg_launch<false>(s, mat, lanes, it, cg_vec(s, it, sol, rtol), s->st);
    }
    if (it >= max_iter)
      pcg_cg_final_kernel<<<ns, kBlock, 0, s->st>>>(s->cg_prng.p,
                                                     s->cg_part.p + (size_t)3 * s->cg_nslots * (it & 1), s->scal.p);
    double* h = s->poll_h + (size_t)16 * ns * slot;
    ZCHK(hipMemcpyAsync(h, s->scal.p, sizeof(double) * 16 * ns, hipMemcpyDeviceToHost, s->st));
    ZCHK(hipEventRecord(s->poll_ev[slot], s->st));
    if (timed) {
      ZCHK(hipEventSynchronize(s->poll_ev[slot]));
      if (graph && ns == 1 && h[7] - iters_before == kChunk) {
        float ms = 0.0f;
        ZCHK(hipEventElapsedTime(&ms, s->chunk_ev[0], s->chunk_ev[1]));
        kt_add(s, KT_SPMV, ms, kChunk * bytes, kChunk);
      }
      iters_before = h[7];
      if (all_done(h) || it >= max_iter) break;
      continue;
    }
    if (it >= max_iter) break;
    if (pending >= 0) {
      ZCHK(hipEventSynchronize(s->poll_ev[pending]));
      if (all_done(s->poll_h + (size_t)16 * ns * pending)) break;
    }
    pending = slot;
    slot ^= 1;
  }
  ZCHK(hipStreamSynchronize(s->st));
  const double* hs = s->poll_h + (size_t)16 * ns * slot;  // the last copy
  int bad;
  ZCHK(hipMemcpyAsync(&bad, s->counters.p + 4, sizeof(int), hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
  // Non-positive curvature (p.Hp <= 0, possible when FP32 rounding leaves the Hessian
  // slightly indefinite) ends a scene's solve with its current iterate, a descent
  // direction; at the first iteration that iterate is 0 and M^-1 b is taken instead.
  std::vector<int> first(ns, 0);
  bool any_first = false;
  for (int k = 0; k < ns; ++k) {
    const double* c = hs + 16 * k;
    iters[k] = (int)c[7];
    relres[k] = c[5] > 0.0 ? std::sqrt(c[4] / c[5]) : 0.0;
    status[k] = (bad || c[6] == 0.0) ? ZEMA_E_PCG : 0;
    if (breakdown) breakdown[k] = active_host[k] && c[8] != 0.0;
    if (c[8] != 0.0 && iters[k] == 0 && active_host[k]) {
      first[k] = 1;
      any_first = true;
    }
  }
  if (any_first && s->nsv + s->nfree > 0) {
    ZCHK(hipMemcpyAsync(s->sc_mask.p, first.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s->st));
    cg_precond_rhs_kernel<<<nblocks(s->nsv + s->nfree), kBlock, 0, s->st>>>(
        s->nsv, s->nfree, s->minv_soft.p, s->minv_body.p, rhs, sol, s->sc_mask.p, s->v_scene.p, s->f_scene.p);
    ZCHK(hipStreamSynchronize(s->st));
  }
}

// ------------------------------------------------------------------ launch-shape autotuner
__global__ void probe_rhs_kernel(int n, double* __restrict__ b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)((i * 2654435761u) & 1023u) / 512.0 - 1.0;  // deterministic, not smooth
}

// Times a fixed number of PCG iterations on the last assembled Hessian for every
// launch shape of the current form (lanes per soft row; with the two-launch form also
// the update block) and keeps the fastest.  The shapes change
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
  // the single-reduction form has no separate update kernel: its shapes are the lanes
  const bool cg = s->pcg_form == 1;
  const int L[4] = {4, 8, 16, 32}, U[3] = {64, 128, 256};
  const int l0 = cg ? 0 : 1, nu = cg ? 1 : 3;
  double best = 1e300;
  int bl = s->tune_lanes, bu = s->tune_ublock;
  hipEvent_t e0, e1;
  ZCHK(hipEventCreate(&e0));
  ZCHK(hipEventCreate(&e1));
  for (int li = l0; li < 4; ++li)
    for (int ui = 0; ui < nu; ++ui) {
      s->tune_lanes = L[li];
      s->tune_ublock = cg ? bu : U[ui];
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
        bu = s->tune_ublock;
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
// A batch of scenes has a block-diagonal Newton system; every scene runs its own CG in
// the same single-reduction launches (scenes with active[k] == 0 get x = 0 and count
// as converged).  iters / relres / status: host arrays [ns].
void k_pcg_batch(zema_scene* s, const double* rhs, double* sol, double rtol, int max_iter, const int* active_host,
                 int* iters, double* relres, int* status, int* breakdown) {
  if (max_iter <= 0) max_iter = std::max(s->ndof, 1);
  k_build_precond(s);  // block-Jacobi inverses of the current Hessian (allocates them)
  s->mat_h.resize(sizeof(Mat<double>) + sizeof(Mat<float>));
  Mat<double> M64 = make_mat<double>(s, s->bsr_val.p, s->c_val.p);
  Mat<float> M32 = make_mat<float>(s, s->bsr_val32.p, s->c_val32.p);
  std::memcpy(s->mat_h.data(), &M64, sizeof(M64));
  std::memcpy(s->mat_h.data() + sizeof(M64), &M32, sizeof(M32));
  s->mat_dev.reserve(s->mat_h.size());
  ZCHK(hipMemcpyAsync(s->mat_dev.p, s->mat_h.data(), s->mat_h.size(), hipMemcpyHostToDevice, s->st));
  const void* mat = s->mixed ? (const void*)(s->mat_dev.p + sizeof(Mat<double>)) : (const void*)s->mat_dev.p;
  const double bytes = (s->mixed ? 40.0 : 76.0) * (s->nnzb + s->nnzc) + 152.0 * s->ndof;
  k_pcg_cg(s, mat, s->tune_lanes, bytes, rhs, sol, rtol, max_iter, active_host, iters, relres, status, breakdown);
}

// ------------------------------------------------------------------ FP64 residual check
// Per scene k: r = b - q over its DOFs (soft rows, then its free bodies' rows) and
// out[k] = (|r|^2, |b|^2), summed in a fixed order by one block per scene.
__global__ void scene_resid_kernel(int nsv, const int* __restrict__ rng, const double* __restrict__ b,
                                   const double* __restrict__ q, double* __restrict__ r, double* __restrict__ out) {
  __shared__ double sh[2][kBlock / 64];
  const int k = blockIdx.x;
  const int64_t s0 = 3 * (int64_t)rng[8 * k], s1 = 3 * (int64_t)rng[8 * k + 1];
  const int64_t a0 = 3 * (int64_t)nsv + 12 * (int64_t)rng[8 * k + 6], a1 = 3 * (int64_t)nsv + 12 * (int64_t)rng[8 * k + 7];
  double rr = 0.0, bb = 0.0;
  for (int64_t i = s0 + threadIdx.x; i < s1; i += kBlock) {
    double ri = b[i] - q[i];
    r[i] = ri;
    rr += ri * ri;
    bb += b[i] * b[i];
  }
  for (int64_t i = a0 + threadIdx.x; i < a1; i += kBlock) {
    double ri = b[i] - q[i];
    r[i] = ri;
    rr += ri * ri;
    bb += b[i] * b[i];
  }
  for (int o = 32; o > 0; o >>= 1) {
    rr += __shfl_xor(rr, o, 64);
    bb += __shfl_xor(bb, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = rr;
    sh[1][threadIdx.x >> 6] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t0 = 0.0, t1 = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      t0 += sh[0][w];
      t1 += sh[1][w];
    }
    out[2 * k] = t0;
    out[2 * k + 1] = t1;
  }
}

// The Newton system's solve for every active scene.  In the mixed form the FP32
// products' recurrence residual is checked against b - H x recomputed with FP64
// accumulation: while that true residual exceeds rtol |b| (at most twice), the
// residual equation H d = r is solved to the tolerance still missing and d added;
// relres then reports the true residual.
void k_pcg_solve(zema_scene* s, const double* rhs, double* sol, double rtol, int max_iter, const int* active_host,
                 int* iters, double* relres, int* status, int* breakdown) {
  const int ns = s->ns, n = s->ndof;
  auto solve = [&](const double* b, double* x, double tol, const int* act, int* it, double* rr, int* st, int* bd) {
    if (ns == 1) {
      st[0] = act[0] ? k_pcg(s, b, x, tol, max_iter, it, rr, bd) : 0;
      if (!act[0]) it[0] = bd[0] = 0;
    } else {
      k_pcg_batch(s, b, x, tol, max_iter, act, it, rr, st, bd);
    }
  };
  solve(rhs, sol, rtol, active_host, iters, relres, status, breakdown);
  if (!s->mixed || n == 0) return;
  s->res_q.reserve(n);
  s->res_r.reserve(n);
  s->res_d.reserve(n);
  s->res_out.reserve((size_t)2 * ns);
  std::vector<double> h((size_t)2 * ns), one(ns);
  std::vector<int> need(ns), it2(ns), st2(ns), bd2(ns);
  std::vector<double> rr2(ns);
  for (int pass = 0;; ++pass) {
    k_hess_matvec64(s, sol, s->res_q.p);
    scene_resid_kernel<<<ns, kBlock, 0, s->st>>>(s->nsv, s->scn_rng.p, rhs, s->res_q.p, s->res_r.p, s->res_out.p);
    ZCHK(hipMemcpyAsync(h.data(), s->res_out.p, sizeof(double) * 2 * ns, hipMemcpyDeviceToHost, s->st));
    ZCHK(hipStreamSynchronize(s->st));
    double tol = rtol;
    bool any = false;
    for (int k = 0; k < ns; ++k) {
      need[k] = 0;
      if (!active_host[k] || status[k]) continue;
      double tr = h[2 * k + 1] > 0.0 ? std::sqrt(h[2 * k] / h[2 * k + 1]) : 0.0;
      relres[k] = tr;
      if (tr > rtol) {
        need[k] = 1;
        any = true;
        tol = std::min(tol, 0.5 * rtol / tr);
      }
    }
    if (!any || pass == 2) break;
    solve(s->res_r.p, s->res_d.p, tol, need.data(), it2.data(), rr2.data(), st2.data(), bd2.data());
    for (int k = 0; k < ns; ++k) {
      one[k] = need[k] && !st2[k] ? 1.0 : 0.0;
      if (need[k]) {
        iters[k] += it2[k];
        breakdown[k] |= bd2[k];
      }
    }
    k_axpy_scene(s, one.data(), s->res_d.p, sol, sol);
  }
}

}  // namespace zema

// PSD projection of a small symmetric matrix by one wavefront: parallel cyclic Jacobi
// (Golub and Van Loan, "parallel ordering": in each round the index pairs
// (L_k, L_{N-1-k}) are disjoint, L_0 = 0 fixed and L_1..L_{N-1} rotating), then
// P = V max(Lambda, 0) V^T.  The matrix lives in LDS with row stride LD.
#pragma once
#include "common.hpp"

namespace zema {

template <int N>
__device__ inline int rr_pair(int r, int i) {
  return i == 0 ? 0 : ((i - 1 + r) % (N - 1)) + 1;
}

// M: N x N symmetric (row stride LD), Vm: scratch of the same shape, cs: [2N],
// partner: [N].  N even.  Called by all 64 lanes of the block (one wavefront).
template <int N, int LD>
__device__ void wave_psd_project(double* M, double* Vm, double* cs, int* partner, int lane) {
  static_assert(N % 2 == 0, "even order");
  constexpr int NE = N * N;
  constexpr int PER = (NE + 63) / 64;
  for (int e = lane; e < NE; e += 64) Vm[(e / N) * LD + e % N] = (e / N == e % N) ? 1.0 : 0.0;
  __syncthreads();
  double fro = 0.0;
  for (int e = lane; e < NE; e += 64) fro += M[(e / N) * LD + e % N] * M[(e / N) * LD + e % N];
  fro = wave_sum(fro);
  double off_prev = INFINITY;
  for (int sweep = 0; sweep < 20; ++sweep) {
    double off = 0.0;
    for (int e = lane; e < NE; e += 64) {
      int r = e / N, c = e % N;
      if (r < c) off += M[r * LD + c] * M[r * LD + c];
    }
    off = wave_sum(off);
    // Stop once the off-diagonal norm is 1e-13 of the Frobenius norm (the eigenvalues
    // are then those of a matrix within that distance), or, once it is below 1e-12,
    // when a sweep no longer halves it: there the sweeps converge quadratically until
    // rounding stalls them, which for badly scaled matrices (barrier Hessians) happens
    // above 1e-15.  Above 1e-12 a sweep may shrink it less than that (the linear phase
    // of cyclic Jacobi, seen on mollified edge-edge Hessians), so no stop there.
    if (!(off > 1e-26 * fro) || (off < 1e-24 * fro && off > 0.25 * off_prev)) break;
    off_prev = off;
    for (int rd = 0; rd < N - 1; ++rd) {
      if (lane < N / 2) {
        int p = rr_pair<N>(rd, lane), q = rr_pair<N>(rd, N - 1 - lane);
        double apq = M[p * LD + q], c = 1.0, sn = 0.0;
        if (apq != 0.0) {
          double th = (M[q * LD + q] - M[p * LD + p]) / (2.0 * apq);
          double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          sn = t * c;
        }
        // rotation J: column p = (p: c, q: -s), column q = (p: s, q: c)
        partner[p] = q;
        partner[q] = p;
        cs[2 * p] = c;
        cs[2 * p + 1] = -sn;
        cs[2 * q] = c;
        cs[2 * q + 1] = sn;
      }
      __syncthreads();
      double na[PER], nv[PER];
      int cnt = 0;
      for (int e = lane; e < NE; e += 64, ++cnt) {
        int r = e / N, c = e % N;
        int rp = partner[r], cp = partner[c];
        double jrr = cs[2 * r], jpr = cs[2 * r + 1];
        double jcc = cs[2 * c], jpc = cs[2 * c + 1];
        double arc = M[r * LD + c] * jcc + M[r * LD + cp] * jpc;
        double apc = M[rp * LD + c] * jcc + M[rp * LD + cp] * jpc;
        na[cnt] = jrr * arc + jpr * apc;  // (J^T M J)[r][c]
        nv[cnt] = Vm[r * LD + c] * jcc + Vm[r * LD + cp] * jpc;  // (V J)[r][c]
      }
      __syncthreads();
      cnt = 0;
      for (int e = lane; e < NE; e += 64, ++cnt) {
        M[(e / N) * LD + e % N] = na[cnt];
        Vm[(e / N) * LD + e % N] = nv[cnt];
      }
      __syncthreads();
    }
  }
  double pv[PER];
  int cnt = 0;
  for (int e = lane; e < NE; e += 64, ++cnt) {
    int r = e / N, c = e % N;
    double acc = 0.0;
    for (int k = 0; k < N; ++k) {
      double l = M[k * LD + k];
      if (l > 0.0) acc += l * Vm[r * LD + k] * Vm[c * LD + k];
    }
    pv[cnt] = acc;
  }
  __syncthreads();
  cnt = 0;
  for (int e = lane; e < NE; e += 64, ++cnt) M[(e / N) * LD + e % N] = pv[cnt];
  __syncthreads();
}

}  // namespace zema

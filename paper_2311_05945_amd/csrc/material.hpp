// Soft-body elements (Sec. IV-D names three isotropic potentials), each scaled by
// h^2 V as in Sec. III eq. 1:
//   neo-Hookean with logarithmic volume terms
//     Psi = mu/2 (|F|^2 - 3) - mu log J + lambda/2 (log J)^2,
//   Saint Venant-Kirchhoff
//     Psi = mu |E|^2 + lambda/2 (tr E)^2,  E = (F^T F - I) / 2,
//   fixed corotated
//     Psi = mu |F - R|^2 + lambda/2 (J - 1)^2,  R the rotation of F = R S;
// every model is infinite for J <= 0 (an inverting step is infeasible).
//
// The Hessian d2Psi/dF2 is projected to PSD through its analytic eigensystem in the
// singular values of the rotation-variant SVD F = U diag(s) V^T (Smith, de Goes, Kim
// 2019, "Analytic eigensystems for isotropic distortion energies"): three scaling
// modes U diag(e) V^T from the 3x3 Hessian of Psi in s, and for each pair (i, j) a
// twist mode (u_i v_j^T - u_j v_i^T)/sqrt2 with eigenvalue (psi_i + psi_j)/(s_i + s_j)
// and a flip mode (u_i v_j^T + u_j v_i^T)/sqrt2 with eigenvalue
// (psi_i - psi_j)/(s_i - s_j), psi_i = dPsi/ds_i, both written without the division.
#pragma once
#include "common.hpp"

namespace zema {

// symmetric 3x3 eigen-decomposition by cyclic Jacobi: A overwritten by its
// eigenvalues on the diagonal, V columns are eigenvectors
template <class T>
__host__ __device__ inline void eig3(T A[3][3], T V[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = i == j ? T(1) : T(0);
  for (int sweep = 0; sweep < 12; ++sweep) {
    T off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    T dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    const T rel = sizeof(T) == 8 ? T(1e-34) : T(1e-15);
    if (off <= rel * dg || off == T(0)) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        T apq = A[p][q];
        if (apq == T(0)) continue;
        T th = (A[q][q] - A[p][p]) / (T(2) * apq);
        T t = (th >= T(0) ? T(1) : T(-1)) / (fabs(th) + sqrt(th * th + T(1)));
        T c = T(1) / sqrt(t * t + T(1)), s = t * c;
        for (int k = 0; k < 3; ++k) {
          T akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          T apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          T vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
}

// index of (i, j), i <= j, in the packed upper triangle of a 9x9 matrix
__host__ __device__ inline int up9(int i, int j) { return i * 9 - (i * (i - 1)) / 2 + (j - i); }

// Rotation-variant SVD F = U diag(s) V^T with U, V rotations (s[2] carries the sign
// of det F), singular values descending in magnitude.
__host__ __device__ inline void svd3(const double F[3][3], double U[3][3], double s[3], double V[3][3]) {
  double C[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
  double W[3][3];
  eig3(C, W);
  double lam[3] = {C[0][0], C[1][1], C[2][2]};
  int o[3] = {0, 1, 2};
  for (int a = 0; a < 2; ++a)
    for (int b = a + 1; b < 3; ++b)
      if (lam[o[b]] > lam[o[a]]) {
        int t = o[a];
        o[a] = o[b];
        o[b] = t;
      }
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) V[i][k] = W[i][o[k]];
  // make V a rotation
  double dv = V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) - V[0][1] * (V[1][0] * V[2][2] - V[1][2] * V[2][0]) +
              V[0][2] * (V[1][0] * V[2][1] - V[1][1] * V[2][0]);
  if (dv < 0.0)
    for (int i = 0; i < 3; ++i) V[i][2] = -V[i][2];
  V3 v0 = v3(V[0][0], V[1][0], V[2][0]), v1 = v3(V[0][1], V[1][1], V[2][1]), v2 = v3(V[0][2], V[1][2], V[2][2]);
  auto mulF = [&](V3 v) {
    return v3(F[0][0] * v.x + F[0][1] * v.y + F[0][2] * v.z, F[1][0] * v.x + F[1][1] * v.y + F[1][2] * v.z,
              F[2][0] * v.x + F[2][1] * v.y + F[2][2] * v.z);
  };
  V3 f0 = mulF(v0), f1 = mulF(v1), f2 = mulF(v2);
  double n0 = sqrt(dot(f0, f0));
  V3 u0 = n0 > 0.0 ? (1.0 / n0) * f0 : v3(1, 0, 0);
  V3 w1 = f1 - dot(u0, f1) * u0;
  double n1 = sqrt(dot(w1, w1));
  V3 u1;
  if (n1 > 1e-300) {
    u1 = (1.0 / n1) * w1;
  } else {  // any unit vector orthogonal to u0
    V3 t = fabs(u0.x) < 0.9 ? v3(1, 0, 0) : v3(0, 1, 0);
    V3 c = cross(u0, t);
    u1 = (1.0 / sqrt(dot(c, c))) * c;
  }
  V3 u2 = cross(u0, u1);
  s[0] = dot(u0, f0);
  s[1] = dot(u1, f1);
  s[2] = dot(u2, f2);
  U[0][0] = u0.x;
  U[1][0] = u0.y;
  U[2][0] = u0.z;
  U[0][1] = u1.x;
  U[1][1] = u1.y;
  U[2][1] = u1.z;
  U[0][2] = u2.x;
  U[1][2] = u2.y;
  U[2][2] = u2.z;
}

enum : int { MAT_NEO_HOOKEAN = 0, MAT_STVK = 1, MAT_FIXED_COROTATED = 2 };

__host__ __device__ inline double det3(const double F[3][3]) {
  return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
         F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
}

// Energy h^2 V Psi(F) of one tet (c = h^2 V); +inf for J <= 0.
__host__ __device__ inline double tet_psi(int model, const double F[3][3], double mu, double lam, double c) {
  double J = det3(F);
  if (!(J > 0.0)) return INFINITY;
  if (model == MAT_STVK) {
    double E[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        E[i][j] = 0.5 * (F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j] - (i == j ? 1.0 : 0.0));
    double ee = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) ee += E[i][j] * E[i][j];
    double tr = E[0][0] + E[1][1] + E[2][2];
    return c * (mu * ee + 0.5 * lam * tr * tr);
  }
  if (model == MAT_FIXED_COROTATED) {  // singular values of the same SVD as the gradient's
    double U[3][3], s[3], V[3][3];
    svd3(F, U, s, V);
    double d = (s[0] - 1.0) * (s[0] - 1.0) + (s[1] - 1.0) * (s[1] - 1.0) + (s[2] - 1.0) * (s[2] - 1.0);
    return c * (mu * d + 0.5 * lam * (J - 1.0) * (J - 1.0));
  }
  double I = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) I += F[i][j] * F[i][j];
  double L = log(J);
  return c * (0.5 * mu * (I - 3.0) - mu * L + 0.5 * lam * L * L);
}

// Element Hessian layout (kTetHess values per tet): the diagonal blocks (a, a),
// a = 0..3, as their upper entries xx, xy, xz, yy, yz, zz (6 each), then the
// off-diagonal blocks (a, b), a < b, in the pair order (0,1), (0,2), (0,3), (1,2),
// (1,3), (2,3), row-major 3x3 (rows of vertex a).  78 values: the upper triangle of the
// 12x12 element matrix.
constexpr int kTetOff = 24, kTetHess = 78;
__host__ __device__ constexpr int sym3(int r, int c) { return r == 0 ? c : (r == 1 ? 2 + c : 5); }  // r <= c
__host__ __device__ constexpr int tet_pair(int a, int b) { return a == 0 ? b - 1 : (a == 1 ? 1 + b : 5); }  // a < b

// The upper triangle of c B^T P9 B (layout above), P9 the PSD projection of
// d2Psi/dF2, in arithmetic type T (double, or float for the mixed-precision form).
// With F = sum_a x_a G_a^T, a mode Q of eigenvalue l adds l w_a w_b^T to block (a, b),
// w_a = Q G_a = U M (V^T G_a) for Q = U M V^T; the blocks of vertices 1..3 are
// accumulated mode by mode and vertex 0 follows from G_0 = -(G_1 + G_2 + G_3).
// Output sink of tet_hess_blocks: diag(a, k, v) receives entry k (sym3 order) of block
// (a, a), off(p, r, c, v) entry (r, c) of the off-diagonal block of pair p (tet_pair).
template <class T>
struct PackedHess {  // the element layout above, kTetHess values at h
  T* h;
  __host__ __device__ void diag(int a, int k, T v) const { h[6 * a + k] = v; }
  __host__ __device__ void off(int p, int r, int c, T v) const { h[kTetOff + 9 * p + 3 * r + c] = v; }
};

template <class T, class Out>
__host__ __device__ inline void tet_hess_blocks(int model, const double F[3][3], const double Gd[4][3], double mu_d,
                                                double lam_d, double c_d, const Out& out) {
  const double J = det3(F);
  double Ud[3][3], sd[3], Vd[3][3];
  svd3(F, Ud, sd, Vd);
  const T mu = T(mu_d), lam = T(lam_d);
  T U[3][3], s[3], gt[3][3];  // gt[a-1] = V^T G_a
  for (int i = 0; i < 3; ++i) {
    s[i] = T(sd[i]);
    for (int j = 0; j < 3; ++j) U[i][j] = T(Ud[i][j]);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      gt[a][k] = T(Vd[0][k] * Gd[a + 1][0] + Vd[1][k] * Gd[a + 1][1] + Vd[2][k] * Gd[a + 1][2]);
  // 3x3 Hessian of Psi in the singular values, and the twist / flip eigenvalues
  T A[3][3], twist[3], flip[3];
  const int pi[3] = {0, 1, 0}, pj[3] = {1, 2, 2}, pk[3] = {2, 0, 1};
  if (model == MAT_STVK) {
    T tr = T(0.5) * (s[0] * s[0] + s[1] * s[1] + s[2] * s[2] - T(3));
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        A[i][j] = (i == j ? mu * (T(3) * s[i] * s[i] - T(1)) + lam * tr : T(0)) + lam * s[i] * s[j];
    for (int t = 0; t < 3; ++t) {
      T si = s[pi[t]], sj = s[pj[t]];
      twist[t] = mu * (si * si - si * sj + sj * sj - T(1)) + lam * tr;
      flip[t] = mu * (si * si + si * sj + sj * sj - T(1)) + lam * tr;
    }
  } else if (model == MAT_FIXED_COROTATED) {
    const T Jm = T(J - 1.0), two_mu = T(2) * mu;
    T P[3] = {s[1] * s[2], s[0] * s[2], s[0] * s[1]};  // J / s_i
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) A[i][j] = i == j ? two_mu + lam * P[i] * P[i] : lam * P[i] * P[j] + lam * Jm * s[3 - i - j];
    for (int t = 0; t < 3; ++t) {
      T si = s[pi[t]], sj = s[pj[t]], sk = s[pk[t]];
      twist[t] = two_mu - T(2) * two_mu / (si + sj) + lam * Jm * sk;
      flip[t] = two_mu - lam * Jm * sk;
    }
  } else {
    const T L = T(log(J));
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        A[i][j] = i == j ? mu + (mu + lam - lam * L) / (s[i] * s[i]) : lam / (s[i] * s[j]);
    for (int t = 0; t < 3; ++t) {
      T q = (lam * L - mu) / (s[pi[t]] * s[pj[t]]);
      twist[t] = mu + q;
      flip[t] = mu - q;
    }
  }
  T Ev[3][3];
  eig3<T>(A, Ev);
  // the nine eigenvalues clamped at zero (a clamped mode adds exact zeros)
  T lm[9];
#pragma unroll
  for (int m = 0; m < 3; ++m) lm[m] = A[m][m] > T(0) ? A[m][m] : T(0);
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    lm[3 + 2 * t] = twist[t] > T(0) ? twist[t] : T(0);
    lm[4 + 2 * t] = flip[t] > T(0) ? flip[t] : T(0);
  }
  // K: blocks (a, b), a, b = 1..3, as the upper triangle of a 9x9 matrix
  T K[45];
#pragma unroll
  for (int k = 0; k < 45; ++k) K[k] = T(0);
  const T is2 = T(0.70710678118654752440);
#pragma unroll
  for (int mode = 0; mode < 9; ++mode) {
    T w[9];
    if (mode < 3) {  // scaling mode U diag(e) V^T, e = column `mode` of Ev
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        T e0 = Ev[0][mode] * gt[a][0], e1 = Ev[1][mode] * gt[a][1], e2 = Ev[2][mode] * gt[a][2];
#pragma unroll
        for (int r = 0; r < 3; ++r) w[3 * a + r] = U[r][0] * e0 + U[r][1] * e1 + U[r][2] * e2;
      }
    } else {  // twist (antisymmetric) or flip (symmetric) mode of the pair (i, j)
      const int t = (mode - 3) / 2, i = pi[t], j = pj[t];
      const T sg = (mode - 3) % 2 == 0 ? T(-1) : T(1);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int r = 0; r < 3; ++r) w[3 * a + r] = is2 * (U[r][i] * gt[a][j] + sg * U[r][j] * gt[a][i]);
    }
#pragma unroll
    for (int x = 0; x < 9; ++x) {
      const T lw = lm[mode] * w[x];
#pragma unroll
      for (int y = x; y < 9; ++y) K[up9(x, y)] += lw * w[y];
    }
  }
  const T c = T(c_d);
  // off-diagonal blocks (0, b) = -sum_a K(a, b), b = 1..3; diagonal block (0, 0) =
  // -sum_b block (0, b), upper entries only
  T D00[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) D00[k] = T(0);
#pragma unroll
  for (int b = 1; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        T v = T(0);
#pragma unroll
        for (int a = 1; a < 4; ++a) {
          const int x = 3 * (a - 1) + r, y = 3 * (b - 1) + cc;
          v += x <= y ? K[up9(x, y)] : K[up9(y, x)];
        }
        v = -v;
        out.off(b - 1, r, cc, c * v);  // pairs (0,1), (0,2), (0,3)
        if (cc >= r) D00[sym3(r, cc)] += v;
      }
#pragma unroll
  for (int k = 0; k < 6; ++k) out.diag(0, k, -c * D00[k]);
  // diagonal blocks (a, a) and off-diagonal blocks (1,2), (1,3), (2,3) from K
#pragma unroll
  for (int a = 1; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = r; cc < 3; ++cc) out.diag(a, sym3(r, cc), c * K[up9(3 * (a - 1) + r, 3 * (a - 1) + cc)]);
#pragma unroll
  for (int a = 1; a < 3; ++a)
#pragma unroll
    for (int b = a + 1; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
          out.off(tet_pair(a, b), r, cc, c * K[up9(3 * (a - 1) + r, 3 * (b - 1) + cc)]);
}

// Energy c Psi(F) and gradient (12: vertex a, coordinate r) of one tet; with hblk
// the projected Hessian in the element layout (tet_hess_blocks<double>).
__host__ __device__ inline double tet_element(int model, const double F[3][3], const double G[4][3], double mu,
                                              double lam, double c, double* g, double* hblk) {
  double J = det3(F);
  if (!(J > 0.0)) {
    for (int k = 0; k < 12; ++k) g[k] = 0.0;
    if (hblk)
      for (int k = 0; k < kTetHess; ++k) hblk[k] = 0.0;
    return INFINITY;
  }
  double cof[3][3];  // cofactor matrix dJ/dF
  cof[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  cof[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  cof[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  cof[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
  cof[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
  cof[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
  cof[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
  cof[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
  cof[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  double E, P[3][3];  // energy and first Piola-Kirchhoff stress dPsi/dF
  if (model == MAT_STVK) {
    double Eg[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        Eg[i][j] = 0.5 * (F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j] - (i == j ? 1.0 : 0.0));
    double ee = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) ee += Eg[i][j] * Eg[i][j];
    double tr = Eg[0][0] + Eg[1][1] + Eg[2][2];
    E = c * (mu * ee + 0.5 * lam * tr * tr);
    double S[3][3];  // second Piola-Kirchhoff stress 2 mu E + lambda tr(E) I; P = F S
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) S[i][j] = 2.0 * mu * Eg[i][j] + (i == j ? lam * tr : 0.0);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) P[i][j] = F[i][0] * S[0][j] + F[i][1] * S[1][j] + F[i][2] * S[2][j];
  } else if (model == MAT_FIXED_COROTATED) {
    double U[3][3], s[3], V[3][3];
    svd3(F, U, s, V);
    double d = (s[0] - 1.0) * (s[0] - 1.0) + (s[1] - 1.0) * (s[1] - 1.0) + (s[2] - 1.0) * (s[2] - 1.0);
    E = c * (mu * d + 0.5 * lam * (J - 1.0) * (J - 1.0));
    // P = 2 mu (F - R) + lambda (J - 1) cof(F), R = U V^T
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double R = U[i][0] * V[j][0] + U[i][1] * V[j][1] + U[i][2] * V[j][2];
        P[i][j] = 2.0 * mu * (F[i][j] - R) + lam * (J - 1.0) * cof[i][j];
      }
  } else {
    double L = log(J);
    double I = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) I += F[i][j] * F[i][j];
    E = c * (0.5 * mu * (I - 3.0) - mu * L + 0.5 * lam * L * L);
    // P = mu F + (lambda log J - mu) F^-T, F^-T = cof(F) / J
    double k = (lam * L - mu) / J;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) P[i][j] = mu * F[i][j] + k * cof[i][j];
  }
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 3; ++r) g[3 * a + r] = c * (P[r][0] * G[a][0] + P[r][1] * G[a][1] + P[r][2] * G[a][2]);
  if (hblk) tet_hess_blocks<double>(model, F, G, mu, lam, c, PackedHess<double>{hblk});
  return E;
}

}  // namespace zema

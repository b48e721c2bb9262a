// Neo-Hookean element (Sec. IV-D: the model with logarithmic volume terms,
// Psi = mu/2 (|F|^2 - 3) - mu log J + lambda/2 (log J)^2, infinite for J <= 0),
// scaled by h^2 V as in Sec. III eq. 1, with the PSD projection of d2Psi/dF2 built
// from its analytic eigensystem (Smith, de Goes, Kim 2019, "Analytic eigensystems
// for isotropic distortion energies"): three scaling modes from the 3x3 Hessian in
// the singular values, and per pair (i,j) a twist and a flip mode with eigenvalues
// mu + (lambda log J - mu)/(s_i s_j) and mu - (lambda log J - mu)/(s_i s_j).
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

// Energy h^2 V Psi(F) of one tet; G is the 4x3 map with F = sum_a x_a G_a^T
// (G_a = row a-1 of Dm^-1 for a >= 1, G_0 = -sum of rows).  Returns +inf for J <= 0.
__host__ __device__ inline double nh_energy(const double F[3][3], double mu, double lam, double c) {
  double J = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
             F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  if (!(J > 0.0)) return INFINITY;
  double I = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) I += F[i][j] * F[i][j];
  double L = log(J);
  return c * (0.5 * mu * (I - 3.0) - mu * L + 0.5 * lam * L * L);
}

// index of (i, j), i <= j, in the packed upper triangle of a 9x9 matrix
__host__ __device__ inline int up9(int i, int j) { return i * 9 - (i * (i - 1)) / 2 + (j - i); }

// The 10 upper 3x3 blocks (order (0,0),(0,1),(0,2),(0,3),(1,1),(1,2),(1,3),(2,2),
// (2,3),(3,3)) of h^2 V B^T P9 B, P9 the PSD projection of d2Psi/dF2, computed in
// arithmetic type T (double, or float for the mixed-precision form).  P9 is
// accumulated mode by mode from the analytic eigensystem, then contracted with the
// rows of G (F = sum_a x_a G_a^T).
template <class T>
__host__ __device__ inline void nh_hess_blocks(const double F[3][3], const double Gd[4][3], double mu_d, double lam_d,
                                               double c_d, T* hblk) {
  double J = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
             F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  const T mu = T(mu_d), lam = T(lam_d), L = T(log(J));
  double Ud[3][3], sd[3], Vd[3][3];
  svd3(F, Ud, sd, Vd);
  T U[3][3], V[3][3], s[3], G[4][3];
  for (int i = 0; i < 3; ++i) {
    s[i] = T(sd[i]);
    for (int j = 0; j < 3; ++j) {
      U[i][j] = T(Ud[i][j]);
      V[i][j] = T(Vd[i][j]);
    }
  }
  for (int a = 0; a < 4; ++a)
    for (int j = 0; j < 3; ++j) G[a][j] = T(Gd[a][j]);
  T A[3][3], Ev[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      A[i][j] = i == j ? mu + (mu + lam - lam * L) / (s[i] * s[i]) : lam / (s[i] * s[j]);
  eig3<T>(A, Ev);
  T P[45];
  for (int k = 0; k < 45; ++k) P[k] = T(0);
  T q[9];
  // scaling modes: U diag(e_m) V^T
  for (int m = 0; m < 3; ++m) {
    T lm = A[m][m];
    if (!(lm > T(0))) continue;
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc)
        q[3 * r + cc] = Ev[0][m] * U[r][0] * V[cc][0] + Ev[1][m] * U[r][1] * V[cc][1] + Ev[2][m] * U[r][2] * V[cc][2];
    for (int i = 0; i < 9; ++i)
      for (int j = i; j < 9; ++j) P[up9(i, j)] += lm * q[i] * q[j];
  }
  // twist (antisymmetric) and flip (symmetric) modes of each pair of singular values
  const T is2 = T(0.70710678118654752440);
  const int pi[3] = {0, 1, 0}, pj[3] = {1, 2, 2};
  for (int t = 0; t < 3; ++t) {
    int i = pi[t], j = pj[t];
    T qq = (lam * L - mu) / (s[i] * s[j]);
    for (int mode = 0; mode < 2; ++mode) {
      T lm = mode == 0 ? mu + qq : mu - qq;
      if (!(lm > T(0))) continue;
      T sg = mode == 0 ? T(-1) : T(1);
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) q[3 * r + cc] = is2 * (U[r][i] * V[cc][j] + sg * U[r][j] * V[cc][i]);
      for (int a = 0; a < 9; ++a)
        for (int b = a; b < 9; ++b) P[up9(a, b)] += lm * q[a] * q[b];
    }
  }
  const T c = T(c_d);
  int blk = 0;
  for (int a = 0; a < 4; ++a)
    for (int bb = a; bb < 4; ++bb, ++blk)
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) {
          T acc = T(0);
          for (int j = 0; j < 3; ++j)
            for (int l = 0; l < 3; ++l) {
              int x = 3 * r + j, y = 3 * cc + l;
              T pv = x <= y ? P[up9(x, y)] : P[up9(y, x)];
              acc += G[a][j] * G[bb][l] * pv;
            }
          hblk[9 * blk + 3 * r + cc] = c * acc;
        }
}

// Gradient (12) and optionally the 10 upper 3x3 blocks of the projected Hessian
// (order (0,0),(0,1),(0,2),(0,3),(1,1),(1,2),(1,3),(2,2),(2,3),(3,3), row-major 3x3).
__host__ __device__ inline double nh_element(const double F[3][3], const double G[4][3], double mu, double lam, double c,
                                             double* g, double* hblk) {
  double J = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
             F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  if (!(J > 0.0)) {
    for (int k = 0; k < 12; ++k) g[k] = 0.0;
    if (hblk)
      for (int k = 0; k < 90; ++k) hblk[k] = 0.0;
    return INFINITY;
  }
  double L = log(J);
  double I = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) I += F[i][j] * F[i][j];
  double E = c * (0.5 * mu * (I - 3.0) - mu * L + 0.5 * lam * L * L);
  // first Piola P = mu F + (lambda log J - mu) F^-T, F^-T = cof(F) / J
  double cof[3][3];
  cof[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  cof[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  cof[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  cof[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
  cof[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
  cof[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
  cof[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
  cof[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
  cof[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  double k = (lam * L - mu) / J;
  double P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[i][j] = mu * F[i][j] + k * cof[i][j];
  for (int a = 0; a < 4; ++a)
    for (int r = 0; r < 3; ++r) g[3 * a + r] = c * (P[r][0] * G[a][0] + P[r][1] * G[a][1] + P[r][2] * G[a][2]);
  if (hblk) nh_hess_blocks<double>(F, G, mu, lam, c, hblk);
  return E;
}

}  // namespace zema

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
__host__ __device__ inline void eig3(double A[3][3], double V[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 12; ++sweep) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double dg = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-34 * dg || off == 0.0) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        double apq = A[p][q];
        if (apq == 0.0) continue;
        double th = (A[q][q] - A[p][p]) / (2.0 * apq);
        double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {
          double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
          double vkp = V[k][p], vkq = V[k][q];
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
  if (!hblk) return E;
  double U[3][3], s[3], V[3][3];
  svd3(F, U, s, V);
  // 3x3 Hessian in the singular values (scaling modes)
  double A[3][3], Ev[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      A[i][j] = i == j ? mu + (mu + lam - lam * L) / (s[i] * s[i]) : lam / (s[i] * s[j]);
  eig3(A, Ev);
  double lamk[9];
  double Q[9][3][3];
  for (int m = 0; m < 3; ++m) {
    lamk[m] = A[m][m];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc)
        Q[m][r][cc] = Ev[0][m] * U[r][0] * V[cc][0] + Ev[1][m] * U[r][1] * V[cc][1] + Ev[2][m] * U[r][2] * V[cc][2];
  }
  const double is2 = 0.70710678118654752440;
  int pi[3] = {0, 1, 0}, pj[3] = {1, 2, 2};
  for (int t = 0; t < 3; ++t) {
    int i = pi[t], j = pj[t];
    double q = (lam * L - mu) / (s[i] * s[j]);
    lamk[3 + t] = mu + q;  // twist
    lamk[6 + t] = mu - q;  // flip
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) {
        double a1 = U[r][i] * V[cc][j], a2 = U[r][j] * V[cc][i];
        Q[3 + t][r][cc] = is2 * (a1 - a2);
        Q[6 + t][r][cc] = is2 * (a1 + a2);
      }
  }
  double b[9][12];
  for (int m = 0; m < 9; ++m)
    for (int a = 0; a < 4; ++a)
      for (int r = 0; r < 3; ++r) b[m][3 * a + r] = Q[m][r][0] * G[a][0] + Q[m][r][1] * G[a][1] + Q[m][r][2] * G[a][2];
  int blk = 0;
  for (int a = 0; a < 4; ++a)
    for (int bb = a; bb < 4; ++bb, ++blk)
      for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) {
          double acc = 0.0;
          for (int m = 0; m < 9; ++m)
            if (lamk[m] > 0.0) acc += lamk[m] * b[m][3 * a + r] * b[m][3 * bb + cc];
          hblk[9 * blk + 3 * r + cc] = c * acc;
        }
  return E;
}

}  // namespace zema

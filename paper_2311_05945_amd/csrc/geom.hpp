// Device geometry of the contact terms: closed-primitive distances with their
// feature type, analytic gradients / Hessians of the squared distance, the log
// barrier (Sec. III eq. 5) with the edge-edge mollifier, the lagged friction block
// (eqs. 9-10) and a cyclic-Jacobi PSD projection.
//
// Slot order of a pair's 12 coordinates: point-triangle (p, t0, t1, t2),
// edge-edge (a0, a1, b0, b1).
#pragma once
#include "common.hpp"

namespace zema {

// Feature types.  PT: 0..2 point-vertex t_i, 3 edge t0t1, 4 edge t1t2, 5 edge t2t0,
// 6 face.  EE: 0..3 endpoints (a_i, b_j) = 2i+j, 4..5 a_i to edge b, 6..7 b_j to
// edge a, 8 interior-interior.
enum { PT_FACE = 6, EE_LINE = 8 };

// Closest feature of a point to a triangle by Voronoi-region tests
// (Ericson, Real-Time Collision Detection, Sec. 5.1.5).
__host__ __device__ inline int pt_type(V3 p, V3 a, V3 b, V3 c) {
  V3 ab = b - a, ac = c - a, ap = p - a;
  double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0.0 && d2 <= 0.0) return 0;
  V3 bp = p - b;
  double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0.0 && d4 <= d3) return 1;
  double vc = d1 * d4 - d3 * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) return 3;
  V3 cp = p - c;
  double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) return 2;
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return 5;
  double va = d3 * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) return 4;
  return PT_FACE;
}

// Closest features of two segments (Ericson, Sec. 5.1.9) mapped to a type; nearly
// parallel segments (|a x b|^2 <= 1e-20 |a|^2 |b|^2) take the endpoint branch, so the
// interior-interior type always has |a x b| > 0.
__host__ __device__ inline int ee_type(V3 a0, V3 a1, V3 b0, V3 b1, double* sp, double* tp) {
  V3 d1 = a1 - a0, d2 = b1 - b0, r = a0 - b0;
  double A = dot(d1, d1), E = dot(d2, d2), f = dot(d2, r), c = dot(d1, r), bb = dot(d1, d2);
  // |d1 x d2|^2 from the cross product: exactly zero for parallel axis-aligned edges,
  // where A E - bb^2 would round to a small non-zero value
  V3 nx = cross(d1, d2);
  double den = dot(nx, nx);
  double s = 0.0, t;
  if (den > 1e-20 * A * E) {
    s = (bb * f - c * E) / den;
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  }
  t = (bb * s + f) / E;
  if (t <= 0.0) {
    t = 0.0;
    s = -c / A;
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  } else if (t >= 1.0) {
    t = 1.0;
    s = (bb - c) / A;
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  }
  if (sp) *sp = s;
  if (tp) *tp = t;
  bool s_end = (s <= 0.0 || s >= 1.0), t_end = (t <= 0.0 || t >= 1.0);
  int si = s >= 1.0 ? 1 : 0, ti = t >= 1.0 ? 1 : 0;
  if (s_end && t_end) return 2 * si + ti;
  if (s_end) return 4 + si;
  if (t_end) return 6 + ti;
  return EE_LINE;
}

// squared distance of a given type (value only)
__host__ __device__ inline double d2_pe_val(V3 p, V3 a, V3 b) {
  V3 e = b - a;
  V3 c = cross(p - a, e);
  return dot(c, c) / dot(e, e);
}
__host__ __device__ inline double d2_triple_val(V3 w, V3 u, V3 v) {
  V3 n = cross(u, v);
  double s = dot(w, n);
  return s * s / dot(n, n);
}

__host__ __device__ inline double pt_d2(const V3* x, int type) {
  if (type <= 2) {
    V3 r = x[0] - x[1 + type];
    return dot(r, r);
  }
  if (type <= 5) {
    int i = type - 3, j = (i + 1) % 3;
    return d2_pe_val(x[0], x[1 + i], x[1 + j]);
  }
  return d2_triple_val(x[0] - x[1], x[2] - x[1], x[3] - x[1]);
}
__host__ __device__ inline double ee_d2(const V3* x, int type) {
  if (type <= 3) {
    V3 r = x[type / 2] - x[2 + type % 2];
    return dot(r, r);
  }
  if (type <= 5) return d2_pe_val(x[type - 4], x[2], x[3]);
  if (type <= 7) return d2_pe_val(x[2 + type - 6], x[0], x[1]);
  return d2_triple_val(x[2] - x[0], x[1] - x[0], x[3] - x[2]);
}

// barycentric weights of the closest point of triangle (x1, x2, x3) to x0, on the
// feature pt_type selects (vertex, clamped edge parameter, or face projection)
__host__ __device__ inline void pt_closest_bary(const V3* x, double b[3]) {
  int t = pt_type(x[0], x[1], x[2], x[3]);
  b[0] = b[1] = b[2] = 0.0;
  if (t <= 2) {
    b[t] = 1.0;
  } else if (t <= 5) {
    int i = t - 3, j = (i + 1) % 3;
    V3 e = x[1 + j] - x[1 + i];
    double s = dot(x[0] - x[1 + i], e) / dot(e, e);
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
    b[i] = 1.0 - s;
    b[j] = s;
  } else {
    V3 u = x[2] - x[1], v = x[3] - x[1], ww = x[0] - x[1];
    V3 n = cross(u, v);
    double nn = dot(n, n);
    b[1] = dot(cross(ww, v), n) / nn;
    b[2] = dot(cross(u, ww), n) / nn;
    b[0] = 1.0 - b[1] - b[2];
  }
}

__host__ __device__ inline double pair_dist(int kind, const V3* x, int* type_out) {
  int t;
  double D;
  if (kind == 0) {
    t = pt_type(x[0], x[1], x[2], x[3]);
    D = pt_d2(x, t);
  } else {
    t = ee_type(x[0], x[1], x[2], x[3], nullptr, nullptr);
    D = ee_d2(x, t);
  }
  if (type_out) *type_out = t;
  return sqrt(D);
}

// ------------------------------------------------------------------ derivatives of d^2
// Variables are differences of slot positions: var_u = sum_m C[u][m] x_m with
// coefficients in {-1, 0, 1}.  Gradient / Hessian in variable space are mapped to
// slots: g_m = sum_u C[u][m] g_u, H_mn = sum_uv C[u][m] C[v][n] H_uv.
struct DVars {
  int nv;
  int C[3][4];
  double g[3][3];
  double H[3][3][3][3];  // [u][v][i][j]
};

__device__ inline void dv_zero(DVars& d, int nv) {
  d.nv = nv;
  for (int u = 0; u < 3; ++u)
    for (int m = 0; m < 4; ++m) d.C[u][m] = 0;
  for (int u = 0; u < 3; ++u)
    for (int i = 0; i < 3; ++i) {
      d.g[u][i] = 0.0;
      for (int v = 0; v < 3; ++v)
        for (int j = 0; j < 3; ++j) d.H[u][v][i][j] = 0.0;
    }
}

// |r|^2 with r = x_i - x_j
__device__ inline double dvar_pp(const V3* x, int i, int j, DVars& d) {
  dv_zero(d, 1);
  d.C[0][i] = 1;
  d.C[0][j] = -1;
  V3 r = x[i] - x[j];
  d.g[0][0] = 2 * r.x;
  d.g[0][1] = 2 * r.y;
  d.g[0][2] = 2 * r.z;
  for (int k = 0; k < 3; ++k) d.H[0][0][k][k] = 2.0;
  return dot(r, r);
}

// point i to the line through edge j->k: b = x_i - x_j, a = x_k - x_j,
// D = b.b - (a.b)^2 / (a.a)
__device__ inline double dvar_pe(const V3* x, int i, int j, int k, DVars& d) {
  dv_zero(d, 2);
  d.C[0][i] = 1;
  d.C[0][j] = -1;
  d.C[1][k] = 1;
  d.C[1][j] = -1;
  V3 b = x[i] - x[j], a = x[k] - x[j];
  double s = dot(a, b), t = dot(a, a), it = 1.0 / t;
  double A[3] = {a.x, a.y, a.z}, Bv[3] = {b.x, b.y, b.z};
  for (int r = 0; r < 3; ++r) {
    d.g[0][r] = 2 * Bv[r] - 2 * s * it * A[r];
    d.g[1][r] = -2 * s * it * Bv[r] + 2 * s * s * it * it * A[r];
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double dl = r == c ? 1.0 : 0.0;
      d.H[0][0][r][c] = 2 * dl - 2 * A[r] * A[c] * it;
      double hba = -2 * (A[r] * Bv[c] + s * dl) * it + 4 * s * A[r] * A[c] * it * it;  // d2/db_r da_c
      d.H[0][1][r][c] = hba;
      d.H[1][0][c][r] = hba;
      d.H[1][1][r][c] = -2 * Bv[r] * Bv[c] * it + 4 * s * (Bv[r] * A[c] + A[r] * Bv[c]) * it * it +
                        2 * s * s * dl * it * it - 8 * s * s * A[r] * A[c] * it * it * it;
    }
  return dot(b, b) - s * s * it;
}

// cross-product matrix [a]x with [a]x v = a x v
__device__ inline void crossmat(V3 a, double M[3][3]) {
  M[0][0] = 0;
  M[0][1] = -a.z;
  M[0][2] = a.y;
  M[1][0] = a.z;
  M[1][1] = 0;
  M[1][2] = -a.x;
  M[2][0] = -a.y;
  M[2][1] = a.x;
  M[2][2] = 0;
}

// D = s^2 / W with s = w.(u x v), W = |u x v|^2 (point-plane and line-line).
// Also returns W with its gradient / Hessian (for the edge-edge mollifier) when
// dW != nullptr.
__device__ inline double dvar_triple(V3 w, V3 u, V3 v, DVars& d, DVars* dW) {
  dv_zero(d, 3);
  V3 n = cross(u, v);
  double s = dot(w, n), W = dot(n, n), iW = 1.0 / W;
  V3 gs[3] = {n, cross(v, w), cross(w, u)};
  double uu = dot(u, u), vv = dot(v, v), uv = dot(u, v);
  V3 gW[3] = {v3(0, 0, 0), 2.0 * (vv * u - uv * v), 2.0 * (uu * v - uv * u)};
  double Hs[3][3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Hs[a][b][i][j] = 0.0;
  double M[3][3];
  crossmat(v, M);  // H_wu = -[v]x
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Hs[0][1][i][j] = -M[i][j];
      Hs[1][0][j][i] = -M[i][j];
    }
  crossmat(u, M);  // H_wv = [u]x
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Hs[0][2][i][j] = M[i][j];
      Hs[2][0][j][i] = M[i][j];
    }
  crossmat(w, M);  // H_uv = -[w]x
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Hs[1][2][i][j] = -M[i][j];
      Hs[2][1][j][i] = -M[i][j];
    }
  double U[3] = {u.x, u.y, u.z}, Vv[3] = {v.x, v.y, v.z};
  double HW[3][3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) HW[a][b][i][j] = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double dl = i == j ? 1.0 : 0.0;
      HW[1][1][i][j] = 2 * (vv * dl - Vv[i] * Vv[j]);
      HW[2][2][i][j] = 2 * (uu * dl - U[i] * U[j]);
      HW[1][2][i][j] = 2 * (2 * U[i] * Vv[j] - Vv[i] * U[j] - uv * dl);
      HW[2][1][j][i] = HW[1][2][i][j];
    }
  double c1 = 2 * s * iW, c2 = s * s * iW * iW;
  for (int a = 0; a < 3; ++a)
    for (int i = 0; i < 3; ++i) d.g[a][i] = c1 * comp(gs[a], i) - c2 * comp(gW[a], i);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double si = comp(gs[a], i), sj = comp(gs[b], j), wi = comp(gW[a], i), wj = comp(gW[b], j);
          d.H[a][b][i][j] = 2 * iW * si * sj + c1 * Hs[a][b][i][j] - 2 * s * iW * iW * (si * wj + wi * sj) -
                            c2 * HW[a][b][i][j] + 2 * s * s * iW * iW * iW * wi * wj;
        }
  if (dW) {
    dv_zero(*dW, 3);
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < 3; ++i) dW->g[a][i] = comp(gW[a], i);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) dW->H[a][b][i][j] = HW[a][b][i][j];
  }
  return s * s * iW;
}

// slot-space gradient entry (slot m, component i) and Hessian entry ((m, i), (n, j))
// from variable space
__device__ inline double dv_grad_entry(const DVars& d, int m, int i) {
  double acc = 0.0;
  for (int u = 0; u < d.nv; ++u) acc += d.C[u][m] * d.g[u][i];
  return acc;
}
__device__ inline double dv_hess_entry(const DVars& d, int m, int i, int n, int j) {
  double acc = 0.0;
  for (int u = 0; u < d.nv; ++u) {
    if (!d.C[u][m]) continue;
    for (int v = 0; v < d.nv; ++v)
      if (d.C[v][n]) acc += d.C[u][m] * d.C[v][n] * d.H[u][v][i][j];
  }
  return acc;
}

// Squared distance of the given type with its variable-space derivatives in d.
__device__ inline double d2_vars(int kind, int type, const V3* x, DVars& d) {
  double D;
  if (kind == 0) {
    if (type <= 2)
      D = dvar_pp(x, 0, 1 + type, d);
    else if (type <= 5) {
      int i = type - 3, j = (i + 1) % 3;
      D = dvar_pe(x, 0, 1 + i, 1 + j, d);
    } else {
      D = dvar_triple(x[0] - x[1], x[2] - x[1], x[3] - x[1], d, nullptr);
      // w = p - t0, u = t1 - t0, v = t2 - t0
      d.C[0][0] = 1;
      d.C[0][1] = -1;
      d.C[1][2] = 1;
      d.C[1][1] = -1;
      d.C[2][3] = 1;
      d.C[2][1] = -1;
    }
  } else {
    if (type <= 3)
      D = dvar_pp(x, type / 2, 2 + type % 2, d);
    else if (type <= 5)
      D = dvar_pe(x, type - 4, 2, 3, d);
    else if (type <= 7)
      D = dvar_pe(x, 2 + type - 6, 0, 1, d);
    else {
      D = dvar_triple(x[2] - x[0], x[1] - x[0], x[3] - x[2], d, nullptr);
      // w = b0 - a0, u = a1 - a0, v = b1 - b0
      d.C[0][2] = 1;
      d.C[0][0] = -1;
      d.C[1][1] = 1;
      d.C[1][0] = -1;
      d.C[2][3] = 1;
      d.C[2][2] = -1;
    }
  }
  return D;
}

// ------------------------------------------------------------------ barrier
// b(d) = -(d - dhat)^2 log(d / dhat) on (0, dhat), zero beyond; b' and b''.
__host__ __device__ inline void barrier3(double d, double dhat, double& b, double& b1, double& b2) {
  if (d >= dhat) {
    b = b1 = b2 = 0.0;
    return;
  }
  double t = d - dhat, L = log(d / dhat);
  b = -t * t * L;
  b1 = -2.0 * t * L - t * t / d;
  b2 = -2.0 * L - 4.0 * t / d + t * t / (d * d);
}

// edge-edge mollifier m(c) = 2c/eps - (c/eps)^2 for c < eps, else 1
__host__ __device__ inline void mollifier(double c, double eps, double& m, double& m1, double& m2) {
  if (c < eps) {
    double ie = 1.0 / eps;
    m = 2.0 * c * ie - c * c * ie * ie;
    m1 = 2.0 * ie - 2.0 * c * ie * ie;
    m2 = -2.0 * ie * ie;
  } else {
    m = 1.0;
    m1 = m2 = 0.0;
  }
}

// barrier energy only (line search)
__device__ inline double pair_barrier_energy(int kind, const V3* x, double eps_x, double kappa, double dhat,
                                             double* dist) {
  double d = pair_dist(kind, x, nullptr);
  if (dist) *dist = d;
  if (!(d < dhat)) return 0.0;
  double b, b1, b2;
  barrier3(d, dhat, b, b1, b2);
  double m = 1.0;
  if (kind == 1) {
    V3 n = cross(x[1] - x[0], x[3] - x[2]);
    double m1, m2;
    mollifier(dot(n, n), eps_x, m, m1, m2);
  }
  return kappa * m * b;
}

// ------------------------------------------------------------------ PSD projection
// Cyclic Jacobi on a symmetric n x n matrix (n <= 12); A is replaced by
// V max(Lambda, 0) V^T.
template <int N>
__device__ inline void psd_project(double (*A)[12]) {
  double V[N][N];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  double fro = 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) fro += A[i][j] * A[i][j];
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < N; ++p)
      for (int q = p + 1; q < N; ++q) off += A[p][q] * A[p][q];
    if (off <= 1e-34 * fro) break;
    for (int p = 0; p < N - 1; ++p)
      for (int q = p + 1; q < N; ++q) {
        double apq = A[p][q];
        if (apq == 0.0) continue;
        double th = (A[q][q] - A[p][p]) / (2.0 * apq);
        double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < N; ++k) {
          double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < N; ++k) {
          double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < N; ++k) {
          double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  double lam[N];
  for (int k = 0; k < N; ++k) lam[k] = A[k][k] > 0.0 ? A[k][k] : 0.0;
  for (int i = 0; i < N; ++i)
    for (int j = i; j < N; ++j) {
      double acc = 0.0;
      for (int k = 0; k < N; ++k) acc += lam[k] * V[i][k] * V[j][k];
      A[i][j] = acc;
      A[j][i] = acc;
    }
}

}  // namespace zema

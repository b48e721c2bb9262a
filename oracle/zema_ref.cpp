/*
 * zema_ref.cpp -- FP64 CPU oracle of the soft/affine incremental-potential-contact
 * Newton step.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow and written to be checked by eye against
 * the paper (Du et al., "Intersection-free Robot Manipulation with Soft-Rigid Coupled
 * Incremental Potential Contact", arXiv 2311.05945).  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * What it computes, with the passage each part follows:
 *   soft IP energy 1/2 (x-xhat)^T M (x-xhat) + h^2 Phi(x), diagonal M   Sec. III, eq. 1
 *   affine IP energy with orthogonality potential lambda V |AA^T-I|_F^2  Sec. III, eq. 2
 *   coupled energy, xhat and qhat predictors                             Sec. III, eq. 3
 *   barrier-augmented energy B_t = E + kappa sum b(d_k)                  Sec. III, eq. 4
 *   log barrier b(d)                                                     Sec. III, eq. 5
 *   soft-affine Jacobian and chain rule for gradient / Hessian          Sec. III, eqs. 6-8
 *   PSD projection of the x-space pair Hessian before mapping            Sec. III, text after eq. 8
 *   lagged smoothed friction D_k = mu lambda_k f0(|u_k|)                  Sec. III, eqs. 9-10
 *   minimisation of B_t + D and the velocity update                       Sec. III, eq. 11 and after
 *   kinematic penalty kappa_A/2 |q - qtilde|^2 (multiplier zero)          Sec. IV-C-1, kinematic energy
 *   neo-Hookean with logarithmic volume term                              Sec. IV-D
 * Readings where the paper is silent (lumping, distance types, mollifier, ACCD,
 * PCG, kappa rule, convergence norm) are listed in the design notes of the
 * repository; each is marked "reading" below.
 *
 * Derivatives: second-order forward-mode automatic differentiation (value, gradient,
 * Hessian carried together) of the hand-written energies.  PSD projection: cyclic
 * Jacobi eigen-decomposition, eigenvalues clamped at zero.
 */
#include "zema_ref.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <tuple>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double INF = std::numeric_limits<double>::infinity();

// ------------------------------------------------------------------ second-order jets
template <int N>
struct J2 {
  double v;
  double g[N];
  double h[N][N];
};

template <int N>
J2<N> jconst(double c) {
  J2<N> r;
  r.v = c;
  for (int i = 0; i < N; ++i) {
    r.g[i] = 0.0;
    for (int j = 0; j < N; ++j) r.h[i][j] = 0.0;
  }
  return r;
}

template <int N>
J2<N> jvar(double x, int k) {
  J2<N> r = jconst<N>(x);
  r.g[k] = 1.0;
  return r;
}

template <int N>
J2<N> operator+(const J2<N>& a, const J2<N>& b) {
  J2<N> r;
  r.v = a.v + b.v;
  for (int i = 0; i < N; ++i) {
    r.g[i] = a.g[i] + b.g[i];
    for (int j = 0; j < N; ++j) r.h[i][j] = a.h[i][j] + b.h[i][j];
  }
  return r;
}

template <int N>
J2<N> operator-(const J2<N>& a, const J2<N>& b) {
  J2<N> r;
  r.v = a.v - b.v;
  for (int i = 0; i < N; ++i) {
    r.g[i] = a.g[i] - b.g[i];
    for (int j = 0; j < N; ++j) r.h[i][j] = a.h[i][j] - b.h[i][j];
  }
  return r;
}

template <int N>
J2<N> operator*(double c, const J2<N>& a) {
  J2<N> r;
  r.v = c * a.v;
  for (int i = 0; i < N; ++i) {
    r.g[i] = c * a.g[i];
    for (int j = 0; j < N; ++j) r.h[i][j] = c * a.h[i][j];
  }
  return r;
}

template <int N>
J2<N> operator+(const J2<N>& a, double c) {
  J2<N> r = a;
  r.v += c;
  return r;
}

template <int N>
J2<N> operator*(const J2<N>& a, const J2<N>& b) {
  J2<N> r;
  r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) {
    r.g[i] = a.v * b.g[i] + b.v * a.g[i];
    for (int j = 0; j < N; ++j)
      r.h[i][j] = a.v * b.h[i][j] + b.v * a.h[i][j] + a.g[i] * b.g[j] + b.g[i] * a.g[j];
  }
  return r;
}

// f(a) given f(a.v), f'(a.v), f''(a.v)
template <int N>
J2<N> junary(const J2<N>& a, double f, double f1, double f2) {
  J2<N> r;
  r.v = f;
  for (int i = 0; i < N; ++i) {
    r.g[i] = f1 * a.g[i];
    for (int j = 0; j < N; ++j) r.h[i][j] = f1 * a.h[i][j] + f2 * a.g[i] * a.g[j];
  }
  return r;
}

template <int N>
J2<N> jinv(const J2<N>& a) {
  double x = a.v;
  return junary(a, 1.0 / x, -1.0 / (x * x), 2.0 / (x * x * x));
}
template <int N>
J2<N> operator/(const J2<N>& a, const J2<N>& b) {
  return a * jinv(b);
}
template <int N>
J2<N> jlog(const J2<N>& a) {
  double x = a.v;
  return junary(a, std::log(x), 1.0 / x, -1.0 / (x * x));
}
template <int N>
J2<N> jsqrt(const J2<N>& a) {
  double s = std::sqrt(a.v);
  return junary(a, s, 0.5 / s, -0.25 / (s * a.v));
}
template <int N>
J2<N> jsq(const J2<N>& a) {
  return a * a;
}

template <int N>
struct V3 {
  J2<N> c[3];
};
template <int N>
V3<N> vsub(const V3<N>& a, const V3<N>& b) {
  return {{a.c[0] - b.c[0], a.c[1] - b.c[1], a.c[2] - b.c[2]}};
}
template <int N>
J2<N> vdot(const V3<N>& a, const V3<N>& b) {
  return a.c[0] * b.c[0] + a.c[1] * b.c[1] + a.c[2] * b.c[2];
}
template <int N>
V3<N> vcross(const V3<N>& a, const V3<N>& b) {
  return {{a.c[1] * b.c[2] - a.c[2] * b.c[1], a.c[2] * b.c[0] - a.c[0] * b.c[2],
           a.c[0] * b.c[1] - a.c[1] * b.c[0]}};
}

// ------------------------------------------------------------------ small dense algebra
struct D3 {
  double x, y, z;
};
D3 d3(const double* p) { return {p[0], p[1], p[2]}; }
D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
D3 cross(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major).
void jacobi_eig(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  double fro = 0.0;
  for (double a : A) fro += a * a;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off <= 1e-34 * fro || off == 0.0) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // A <- R^T A R with R the rotation in the (p,q) plane
        for (int k = 0; k < n; ++k) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
    }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

// nearest symmetric PSD matrix: V max(Lambda,0) V^T
std::vector<double> project_psd(int n, const std::vector<double>& A) {
  std::vector<double> S(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) S[i * n + j] = 0.5 * (A[i * n + j] + A[j * n + i]);
  std::vector<double> w, V;
  jacobi_eig(n, S, w, V);
  std::vector<double> P(n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    if (w[k] <= 0.0) continue;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) P[i * n + j] += w[k] * V[i * n + k] * V[j * n + k];
  }
  return P;
}

// inverse by Gauss-Jordan with partial pivoting; returns false if singular
bool invert(int n, std::vector<double> A, std::vector<double>& Inv) {
  Inv.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) Inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[c * n + k], A[piv * n + k]);
        std::swap(Inv[c * n + k], Inv[piv * n + k]);
      }
    double d = A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] /= d;
      Inv[c * n + k] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        Inv[r * n + k] -= f * Inv[c * n + k];
      }
    }
  }
  return true;
}

// ------------------------------------------------------------------ barrier (eq. 5)
// b(d) = -(d - dhat)^2 log(d/dhat) for 0 < d < dhat, else 0, with b' and b''.
void barrier3(double d, double dhat, double* b) {
  if (d >= dhat) {
    b[0] = b[1] = b[2] = 0.0;
    return;
  }
  double t = d - dhat, L = std::log(d / dhat);
  b[0] = -t * t * L;
  b[1] = -2.0 * t * L - t * t / d;
  b[2] = -2.0 * L - 4.0 * t / d + t * t / (d * d);
}

// ------------------------------------------------------------------ distances
// Reading: distance between closed primitives = minimum over the feature pairs
// whose foot point lies in the closed feature.  Enumeration order decides ties.
// PT types: 0..2 point-vertex t_i, 3..5 point-edge (t0t1, t1t2, t2t0), 6 face.
// EE types: 0..3 endpoint pairs (a0b0,a0b1,a1b0,a1b1), 4..5 a_i to edge b,
//           6..7 b_j to edge a, 8 interior-interior.
double seg_param(D3 p, D3 a, D3 b, bool* ok) {
  D3 e = b - a;
  double ee = dot(e, e);
  if (ee <= 0.0) {
    *ok = false;
    return 0.0;
  }
  double s = dot(p - a, e) / ee;
  *ok = (s >= 0.0 && s <= 1.0);
  return s;
}
double d2_pe(D3 p, D3 a, D3 b) {
  D3 e = b - a;
  D3 c = cross(p - a, e);
  return dot(c, c) / dot(e, e);
}

double pt_type_d2(const double* x, int* type, double bary[3]) {
  D3 p = d3(x), t[3] = {d3(x + 3), d3(x + 6), d3(x + 9)};
  double best = INF;
  int bt = -1;
  double bb[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    D3 r = p - t[i];
    double v = dot(r, r);
    if (v < best) {
      best = v;
      bt = i;
      bb[0] = bb[1] = bb[2] = 0;
      bb[i] = 1;
    }
  }
  for (int k = 0; k < 3; ++k) {
    int i = k, j = (k + 1) % 3;
    bool ok;
    double s = seg_param(p, t[i], t[j], &ok);
    if (!ok) continue;
    double v = d2_pe(p, t[i], t[j]);
    if (v < best) {
      best = v;
      bt = 3 + k;
      bb[0] = bb[1] = bb[2] = 0;
      bb[i] = 1.0 - s;
      bb[j] = s;
    }
  }
  D3 u = t[1] - t[0], v = t[2] - t[0], w = p - t[0];
  D3 n = cross(u, v);
  double nn = dot(n, n);
  if (nn > 0.0) {
    double b1 = dot(cross(w, v), n) / nn, b2 = dot(cross(u, w), n) / nn, b0 = 1.0 - b1 - b2;
    if (b0 >= 0.0 && b1 >= 0.0 && b2 >= 0.0) {
      double sd = dot(w, n);
      double val = sd * sd / nn;
      if (val < best) {
        best = val;
        bt = 6;
        bb[0] = b0;
        bb[1] = b1;
        bb[2] = b2;
      }
    }
  }
  *type = bt;
  if (bary) std::memcpy(bary, bb, sizeof(bb));
  return best;
}

double ee_type_d2(const double* x, int* type, double gam[2]) {
  D3 a0 = d3(x), a1 = d3(x + 3), b0 = d3(x + 6), b1 = d3(x + 9);
  double best = INF;
  int bt = -1;
  double ga = 0, gb = 0;
  D3 A[2] = {a0, a1}, B[2] = {b0, b1};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      D3 r = A[i] - B[j];
      double v = dot(r, r);
      if (v < best) {
        best = v;
        bt = 2 * i + j;
        ga = i;
        gb = j;
      }
    }
  for (int i = 0; i < 2; ++i) {
    bool ok;
    double s = seg_param(A[i], b0, b1, &ok);
    if (!ok) continue;
    double v = d2_pe(A[i], b0, b1);
    if (v < best) {
      best = v;
      bt = 4 + i;
      ga = i;
      gb = s;
    }
  }
  for (int j = 0; j < 2; ++j) {
    bool ok;
    double s = seg_param(B[j], a0, a1, &ok);
    if (!ok) continue;
    double v = d2_pe(B[j], a0, a1);
    if (v < best) {
      best = v;
      bt = 6 + j;
      ga = s;
      gb = j;
    }
  }
  D3 ea = a1 - a0, eb = b1 - b0, r = a0 - b0;
  D3 n = cross(ea, eb);
  double D = dot(n, n);
  if (D > 0.0) {
    double aa = dot(ea, ea), bb = dot(eb, eb), ab = dot(ea, eb), ar = dot(ea, r), br = dot(eb, r);
    double s = (ab * br - bb * ar) / D, t = (aa * br - ab * ar) / D;
    if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
      double sd = dot(b0 - a0, n);
      double val = sd * sd / D;
      if (val < best) {
        best = val;
        bt = 8;
        ga = s;
        gb = t;
      }
    }
  }
  *type = bt;
  if (gam) {
    gam[0] = ga;
    gam[1] = gb;
  }
  return best;
}

// squared distance of the selected type as a jet over the 12 coordinates
template <int N>
V3<N> jpt(const J2<N>* X, int v) {
  return {{X[3 * v], X[3 * v + 1], X[3 * v + 2]}};
}
template <int N>
J2<N> jd2_pp(const V3<N>& p, const V3<N>& q) {
  V3<N> r = vsub(p, q);
  return vdot(r, r);
}
template <int N>
J2<N> jd2_pe(const V3<N>& p, const V3<N>& a, const V3<N>& b) {
  V3<N> e = vsub(b, a);
  V3<N> c = vcross(vsub(p, a), e);
  return vdot(c, c) / vdot(e, e);
}
template <int N>
J2<N> jd2_plane(const V3<N>& p, const V3<N>& o, const V3<N>& u, const V3<N>& v) {
  V3<N> n = vcross(u, v);
  J2<N> s = vdot(vsub(p, o), n);
  return (s * s) / vdot(n, n);
}

J2<12> pt_d2_jet(const J2<12>* X, int type) {
  V3<12> p = jpt(X, 0), t[3] = {jpt(X, 1), jpt(X, 2), jpt(X, 3)};
  if (type <= 2) return jd2_pp(p, t[type]);
  if (type <= 5) {
    int i = type - 3, j = (i + 1) % 3;
    return jd2_pe(p, t[i], t[j]);
  }
  return jd2_plane(p, t[0], vsub(t[1], t[0]), vsub(t[2], t[0]));
}
J2<12> ee_d2_jet(const J2<12>* X, int type) {
  V3<12> A[2] = {jpt(X, 0), jpt(X, 1)}, B[2] = {jpt(X, 2), jpt(X, 3)};
  if (type <= 3) return jd2_pp(A[type / 2], B[type % 2]);
  if (type <= 5) return jd2_pe(A[type - 4], B[0], B[1]);
  if (type <= 7) return jd2_pe(B[type - 6], A[0], A[1]);
  return jd2_plane(B[0], A[0], vsub(A[1], A[0]), vsub(B[1], B[0]));
}

// ------------------------------------------------------------------ scene
struct Elem {
  std::vector<int> dofs;
  std::vector<double> M;  // dofs.size()^2, row-major
};

struct Body {
  int mode = 0;  // 0 free, 1 fixed, 2 driven
  double rho = 0, stiff = 0, kappaA = 0;
  double V = 0, m = 0, c[3] = {0, 0, 0}, S[9] = {0};
  double tvel[3] = {0, 0, 0}, tstop = 0;
  bool has_target = false;  // a target set by the caller replaces the schedule
  double target[12] = {0};
  double lamA[12] = {0};    // augmented Lagrangian multiplier of the kinematic energy
  double qrest[12];
  double qdot0[12];
  int dof0 = -1;              // first DOF or -1 if fixed
  int sv0 = 0, nsv = 0;       // surface vertex range
  std::vector<double> x0;     // rest positions relative to the centre of mass
};

struct Fric {
  int kind;  // 0 PT, 1 EE
  int v[4];
  double lam, n[3], w[4];
  double xt[12];
};

struct Pair {
  int a, b;
};

struct Rec {
  int step;
  double kappa_lag, kappa;
  std::vector<double> yt, ydt, yk;
};

}  // namespace

struct Spring {
  int sv;          // surface vertex
  double k;        // stiffness (N/m)
  double target[3];
};

struct Joint {
  int b1, b2;     // affine body indices
  double d[3];    // axis in b1's rest frame
  double kappa;   // penalty stiffness (incremental-potential units, as kappa_A)
};

struct zref_scene {
  zref_params P;
  std::string err;
  std::vector<Spring> springs;
  std::vector<Joint> joints;
  double al_tol = 0.0;  // kinematic constraint tolerance of the multiplier updates (0: off)
  int al_max = 0;       // at most this many multiplier updates per step
  int n_soft_bodies = 0;
  // soft
  int nsv = 0;
  std::vector<double> X;      // rest positions [nsv*3]
  std::vector<double> x_init, v_init;
  std::vector<int> tets;      // [nt*4]
  std::vector<double> Dminv;  // [nt*9] row-major
  std::vector<double> vol;    // [nt]
  std::vector<double> lam_mu; // [nt*2] (mu, lambda)
  std::vector<int> tet_model; // [nt] constitutive model (0 neo-Hookean, 1 StVK, 2 fixed corotated)
  std::vector<double> mass;   // [nsv]
  std::vector<int> vbody;     // soft vertex -> body
  std::vector<int> cloth_v;     // garment triangles [nc*3] (soft vertex ids)
  std::vector<double> cloth_d;  // per triangle: rest (u, v) edge-matrix inverse [4], area, k_stretch, k_shear
  // affine
  std::vector<Body> bodies;   // index = affine body index
  // surface
  int nsurf = 0;
  std::vector<int> sv_kind, sv_id, sv_body;  // kind 0 soft (id = soft vertex), 1 affine (id = body)
  std::vector<double> sv_x0;                 // affine vertex x0 [nsurf*3]
  std::vector<int> tris, edges;
  std::vector<double> edge_len2;
  std::vector<char> body_fixed;              // per global body id
  int ndof = 0;
  // state
  std::vector<double> y, ydot, yt, ydt;
  double kappa = 0, kappa_lag = 0;
  int step = 0;
  double dprev = INF;
  std::vector<double> yhat;    // predictor for every DOF
  std::vector<double> qtilde;  // per affine body, 12
  std::vector<Fric> fric;
  std::vector<Pair> pt, ee;    // current candidate set
  std::vector<Elem> H;
  bool record = false;
  std::vector<Rec> recs;
};

namespace {

int fail(zref_scene* s, int code, const std::string& m) {
  if (s) s->err = m;
  return code;
}

int nthreads_req = 0;

// affine vertex position ((a_k0 x0_0 + a_k1 x0_1) + a_k2 x0_2) + p_k
void affine_point(const double* q, const double* x0, double* out) {
  for (int k = 0; k < 3; ++k) {
    const double* a = q + 3 + 3 * k;
    double s = a[0] * x0[0];
    s = s + a[1] * x0[1];
    s = s + a[2] * x0[2];
    out[k] = s + q[k];
  }
}

const double* body_q(const zref_scene* s, int b, const double* y) {
  const Body& B = s->bodies[b];
  return B.dof0 >= 0 ? y + B.dof0 : B.qrest;
}

void surface_positions(const zref_scene* s, const double* y, double* xs) {
  for (int i = 0; i < s->nsurf; ++i) {
    if (s->sv_kind[i] == 0) {
      const double* p = y + 3 * s->sv_id[i];
      xs[3 * i] = p[0];
      xs[3 * i + 1] = p[1];
      xs[3 * i + 2] = p[2];
    } else {
      affine_point(body_q(s, s->sv_id[i], y), &s->sv_x0[3 * i], xs + 3 * i);
    }
  }
}

// displacement of surface vertices for a DOF-space direction p (linear in p)
void surface_disp(const zref_scene* s, const double* p, double* dx) {
  for (int i = 0; i < s->nsurf; ++i) {
    if (s->sv_kind[i] == 0) {
      for (int k = 0; k < 3; ++k) dx[3 * i + k] = p[3 * s->sv_id[i] + k];
    } else {
      const Body& B = s->bodies[s->sv_id[i]];
      if (B.dof0 < 0) {
        dx[3 * i] = dx[3 * i + 1] = dx[3 * i + 2] = 0.0;
      } else {
        const double* q = p + B.dof0;
        const double* x0 = &s->sv_x0[3 * i];
        for (int k = 0; k < 3; ++k)
          dx[3 * i + k] = q[3 + 3 * k] * x0[0] + q[3 + 3 * k + 1] * x0[1] + q[3 + 3 * k + 2] * x0[2] + q[k];
      }
    }
  }
}

// DOF map of a surface vertex: returns the number of y-DOFs (0, 3 or 12), fills the
// DOF ids and the 3 x n Jacobian (row-major, n <= 12).
int vertex_map(const zref_scene* s, int sv, int* dofs, double* J) {
  if (s->sv_kind[sv] == 0) {
    int i = s->sv_id[sv];
    for (int k = 0; k < 3; ++k) dofs[k] = 3 * i + k;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r * 3 + c] = (r == c) ? 1.0 : 0.0;
    return 3;
  }
  const Body& B = s->bodies[s->sv_id[sv]];
  if (B.dof0 < 0) return 0;
  const double* x0 = &s->sv_x0[3 * sv];
  for (int k = 0; k < 12; ++k) dofs[k] = B.dof0 + k;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 12; ++c) J[r * 12 + c] = 0.0;
  for (int r = 0; r < 3; ++r) {
    J[r * 12 + r] = 1.0;                       // d x_r / d p_r
    for (int j = 0; j < 3; ++j) J[r * 12 + 3 + 3 * r + j] = x0[j];  // d x_r / d (a_r)_j
  }
  return 12;
}

// map a 4-vertex x-space gradient / Hessian into y-space (eqs. 6-8)
void map_pair(const zref_scene* s, const int* v4, const double* g12, const double* H144,
              std::vector<double>& grad, Elem* e) {
  int dofs[4][12];
  double J[4][36];
  int nd[4];
  for (int a = 0; a < 4; ++a) nd[a] = vertex_map(s, v4[a], dofs[a], J[a]);
  // gradient
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < nd[a]; ++c) {
      double acc = 0.0;
      for (int r = 0; r < 3; ++r) acc += J[a][r * nd[a] + c] * g12[3 * a + r];
      grad[dofs[a][c]] += acc;
    }
  if (!e) return;
  int n = 0;
  for (int a = 0; a < 4; ++a) n += nd[a];
  e->dofs.clear();
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < nd[a]; ++c) e->dofs.push_back(dofs[a][c]);
  // Jt: 12 x n dense
  std::vector<double> Jt(12 * n, 0.0);
  int col = 0;
  for (int a = 0; a < 4; ++a) {
    for (int c = 0; c < nd[a]; ++c) {
      for (int r = 0; r < 3; ++r) Jt[(3 * a + r) * n + col + c] = J[a][r * nd[a] + c];
    }
    col += nd[a];
  }
  // M = Jt^T H Jt
  std::vector<double> HJ(12 * n, 0.0);
  for (int i = 0; i < 12; ++i)
    for (int k = 0; k < 12; ++k) {
      double h = H144[i * 12 + k];
      if (h == 0.0) continue;
      for (int c = 0; c < n; ++c) HJ[i * n + c] += h * Jt[k * n + c];
    }
  e->M.assign(n * n, 0.0);
  for (int i = 0; i < 12; ++i)
    for (int r = 0; r < n; ++r) {
      double jr = Jt[i * n + r];
      if (jr == 0.0) continue;
      for (int c = 0; c < n; ++c) e->M[r * n + c] += jr * HJ[i * n + c];
    }
}

// ------------------------------------------------------------------ constitutive models (Sec. IV-D)
// The soft-body potentials the paper names: neo-Hookean with the logarithmic volume
// term (model 0), Saint Venant-Kirchhoff (model 1) and fixed corotated (model 2), each
// written from its definition on F with second-order jets:
//   0  Psi = mu/2 (tr F^T F - 3) - mu log J + lambda/2 (log J)^2, +inf for J <= 0;
//   1  Psi = mu |E|_F^2 + lambda/2 (tr E)^2,  E = (F^T F - I) / 2;
//   2  Psi = mu |F - R|_F^2 + lambda/2 (J - 1)^2,  R the rotation of the polar
//      decomposition F = R S.
// Every model returns false (infeasible) for J <= 0: a step that inverts a tet is
// rejected by the line search whatever the material (reading).
template <int N>
void jmat3_inv_t(const J2<N>* X, J2<N>* out, J2<N>& det) {
  // X^{-T} = cof(X) / det X (row-major 3x3)
  J2<N> c[9];
  c[0] = X[4] * X[8] - X[5] * X[7];
  c[1] = X[5] * X[6] - X[3] * X[8];
  c[2] = X[3] * X[7] - X[4] * X[6];
  c[3] = X[2] * X[7] - X[1] * X[8];
  c[4] = X[0] * X[8] - X[2] * X[6];
  c[5] = X[1] * X[6] - X[0] * X[7];
  c[6] = X[1] * X[5] - X[2] * X[4];
  c[7] = X[2] * X[3] - X[0] * X[5];
  c[8] = X[0] * X[4] - X[1] * X[3];
  det = X[0] * c[0] + X[1] * c[1] + X[2] * c[2];
  J2<N> id = jinv(det);
  for (int k = 0; k < 9; ++k) out[k] = c[k] * id;
}

// Rotation of the polar decomposition by Newton's iteration X <- (X + X^{-T}) / 2
// from X = F (Higham 1986), run on the jets until the values have converged and then
// twice more: the map's derivative vanishes at its fixed point, so the first and
// second derivatives converge with the values.
void polar_rotation_jet(const J2<9>* f, J2<9>* R) {
  for (int k = 0; k < 9; ++k) R[k] = f[k];
  int extra = -1;
  for (int it = 0; it < 60 && extra != 0; ++it) {
    J2<9> Xit[9], det;
    jmat3_inv_t(R, Xit, det);
    double change = 0.0;
    for (int k = 0; k < 9; ++k) {
      J2<9> nx = 0.5 * (R[k] + Xit[k]);
      change = std::max(change, std::fabs(nx.v - R[k].v));
      R[k] = nx;
    }
    if (extra > 0) --extra;
    else if (change <= 1e-15) extra = 2;
  }
}

bool psi_jet(const double* F, int model, double mu, double lam, J2<9>& out) {
  J2<9> f[9];
  for (int k = 0; k < 9; ++k) f[k] = jvar<9>(F[k], k);
  J2<9> J = f[0] * (f[4] * f[8] - f[5] * f[7]) - f[1] * (f[3] * f[8] - f[5] * f[6]) +
            f[2] * (f[3] * f[7] - f[4] * f[6]);
  if (!(J.v > 0.0)) return false;
  if (model == 1) {
    J2<9> E[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        J2<9> c = f[i] * f[j] + f[3 + i] * f[3 + j] + f[6 + i] * f[6 + j];  // (F^T F)_ij
        E[3 * i + j] = 0.5 * (i == j ? c + (-1.0) : c);
      }
    J2<9> ee = jconst<9>(0.0);
    for (int k = 0; k < 9; ++k) ee = ee + E[k] * E[k];
    J2<9> tr = E[0] + E[4] + E[8];
    out = mu * ee + (0.5 * lam) * (tr * tr);
    return true;
  }
  if (model == 2) {
    J2<9> R[9];
    polar_rotation_jet(f, R);
    J2<9> d2 = jconst<9>(0.0);
    for (int k = 0; k < 9; ++k) {
      J2<9> d = f[k] - R[k];
      d2 = d2 + d * d;
    }
    J2<9> jm = J + (-1.0);
    out = mu * d2 + (0.5 * lam) * (jm * jm);
    return true;
  }
  J2<9> Ic = jconst<9>(0.0);
  for (int k = 0; k < 9; ++k) Ic = Ic + f[k] * f[k];
  J2<9> L = jlog(J);
  out = (0.5 * mu) * (Ic + (-3.0)) - mu * L + (0.5 * lam) * (L * L);
  return true;
}

// F = Ds Dm^{-1}; B = dvec(F)/dx (9 x 12), row index 3i+j, column 3a+c
void tet_F_B(const double* x12, const double* Dmi, double* F, double* B) {
  double Ds[9];
  for (int i = 0; i < 3; ++i)
    for (int m = 0; m < 3; ++m) Ds[3 * i + m] = x12[3 * (m + 1) + i] - x12[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int m = 0; m < 3; ++m) acc += Ds[3 * i + m] * Dmi[3 * m + j];
      F[3 * i + j] = acc;
    }
  if (!B) return;
  for (int k = 0; k < 108; ++k) B[k] = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s0 = 0.0;
      for (int m = 0; m < 3; ++m) s0 += Dmi[3 * m + j];
      B[(3 * i + j) * 12 + 3 * 0 + i] = -s0;
      for (int a = 1; a < 4; ++a) B[(3 * i + j) * 12 + 3 * a + i] = Dmi[3 * (a - 1) + j];
    }
}

// per-tet elastic IP term h^2 V Psi with gradient and projected Hessian
bool tet_term(const zref_scene* s, int e, const double* x12, double* E, double* g12, double* H144,
              bool project) {
  double F[9], B[108];
  tet_F_B(x12, &s->Dminv[9 * e], F, B);
  J2<9> psi;
  if (!psi_jet(F, s->tet_model[e], s->lam_mu[2 * e], s->lam_mu[2 * e + 1], psi)) {
    *E = INF;
    return false;
  }
  double h2V = s->P.dt * s->P.dt * s->vol[e];
  *E = h2V * psi.v;
  if (g12)
    for (int c = 0; c < 12; ++c) {
      double acc = 0.0;
      for (int k = 0; k < 9; ++k) acc += B[k * 12 + c] * psi.g[k];
      g12[c] = h2V * acc;
    }
  if (H144) {
    std::vector<double> Hf(81);
    for (int i = 0; i < 9; ++i)
      for (int j = 0; j < 9; ++j) Hf[i * 9 + j] = psi.h[i][j];
    std::vector<double> P = project ? project_psd(9, Hf) : Hf;
    for (int a = 0; a < 12; ++a)
      for (int b = 0; b < 12; ++b) {
        double acc = 0.0;
        for (int i = 0; i < 9; ++i) {
          double bi = B[i * 12 + a];
          if (bi == 0.0) continue;
          for (int j = 0; j < 9; ++j) acc += bi * P[i * 9 + j] * B[j * 12 + b];
        }
        H144[a * 12 + b] = h2V * acc;
      }
  }
  return true;
}

// ------------------------------------------------------------------ garment (Sec. IV-D)
// Baraff-Witkin membrane on a triangle with rest material coordinates (u, v): the
// deformation's columns w_u, w_v (x = W (u, v)^T + const over the triangle) enter the
// stretch conditions |w_u| - 1, |w_v| - 1 and the shear condition w_u . w_v; each
// energy density k/2 C^2 is integrated over the rest area A (reading) and scaled by
// h^2 into the incremental potential:
//   h^2 A (k_s/2 ((|w_u| - 1)^2 + (|w_v| - 1)^2) + k_sh/2 (w_u . w_v)^2).
// Hessian (reading): the stretch and the shear parts are each projected to PSD in the
// six coordinates of (w_u, w_v) and the sum is mapped to the vertices (W is linear in
// x).  Bending is not modelled.
void cloth_term(const zref_scene* s, int c, const double* x9, double* E, double* g9, double* H81) {
  const double* d = &s->cloth_d[7 * c];
  const double m00 = d[0], m01 = d[1], m10 = d[2], m11 = d[3];
  const double h2A = s->P.dt * s->P.dt * d[4], ks = d[5], ksh = d[6];
  // dW/dx: w_u = sum_a cu[a] x_a, w_v = sum_a cv[a] x_a
  const double cu[3] = {-(m00 + m10), m00, m10}, cv[3] = {-(m01 + m11), m01, m11};
  J2<6> w[6];
  for (int k = 0; k < 3; ++k) {
    double wu = 0.0, wv = 0.0;
    for (int a = 0; a < 3; ++a) {
      wu += cu[a] * x9[3 * a + k];
      wv += cv[a] * x9[3 * a + k];
    }
    w[k] = jvar<6>(wu, k);
    w[3 + k] = jvar<6>(wv, 3 + k);
  }
  J2<6> nu = jsqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  J2<6> nv = jsqrt(w[3] * w[3] + w[4] * w[4] + w[5] * w[5]);
  J2<6> su = nu + (-1.0), sv = nv + (-1.0);
  J2<6> st = (0.5 * h2A * ks) * (su * su + sv * sv);
  J2<6> cs = w[0] * w[3] + w[1] * w[4] + w[2] * w[5];
  J2<6> sh = (0.5 * h2A * ksh) * (cs * cs);
  *E = st.v + sh.v;
  const double* col[2] = {cu, cv};
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k)
      g9[3 * a + k] = col[0][a] * (st.g[k] + sh.g[k]) + col[1][a] * (st.g[3 + k] + sh.g[3 + k]);
  if (!H81) return;
  std::vector<double> A(36), B(36);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      A[6 * i + j] = st.h[i][j];
      B[6 * i + j] = sh.h[i][j];
    }
  std::vector<double> PA = project_psd(6, A), PB = project_psd(6, B);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double acc = 0.0;
          for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
              const int i = 3 * p + k, j = 3 * q + l;
              acc += col[p][a] * col[q][b] * (PA[6 * i + j] + PB[6 * i + j]);
            }
          H81[(3 * a + k) * 9 + 3 * b + l] = acc;
        }
}

// ------------------------------------------------------------------ affine body terms (eq. 2)
// h^2 lambda V |A A^T - I|_F^2 on the 9 entries of A, A rows = a1, a2, a3
void orth_term(const zref_scene* s, const Body& B, const double* q, double* E, double* g12,
               double* H144) {
  J2<9> a[9];
  for (int k = 0; k < 9; ++k) a[k] = jvar<9>(q[3 + k], k);
  J2<9> phi = jconst<9>(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      J2<9> m = a[3 * i] * a[3 * j] + a[3 * i + 1] * a[3 * j + 1] + a[3 * i + 2] * a[3 * j + 2];
      if (i == j) m = m + (-1.0);
      phi = phi + m * m;
    }
  double c = s->P.dt * s->P.dt * B.stiff * B.V;
  *E = c * phi.v;
  if (g12) {
    for (int k = 0; k < 3; ++k) g12[k] = 0.0;
    for (int k = 0; k < 9; ++k) g12[3 + k] = c * phi.g[k];
  }
  if (H144) {
    std::vector<double> Hf(81);
    for (int i = 0; i < 9; ++i)
      for (int j = 0; j < 9; ++j) Hf[i * 9 + j] = phi.h[i][j];
    std::vector<double> P = project_psd(9, Hf);
    for (int k = 0; k < 144; ++k) H144[k] = 0.0;
    for (int i = 0; i < 9; ++i)
      for (int j = 0; j < 9; ++j) H144[(3 + i) * 12 + 3 + j] = c * P[i * 9 + j];
  }
}

// ------------------------------------------------------------------ contact pair energy
// kappa * m_k * b(d): m_k = 1 for point-triangle; for edge-edge the mollifier
// (reading) m = 2c/eps - (c/eps)^2 for c < eps, c = |(a1-a0)x(b1-b0)|^2,
// eps = 1e-3 |A1-A0|^2 |B1-B0|^2 at rest.
// force_type >= 0 (test use only) evaluates the squared distance of that feature type
// in place of the closest one, e.g. the other side of a tie between two features.
bool pair_energy_jet(const zref_scene* s, int kind, const double* x12, double eps_x, double kappa,
                     J2<12>& out, double* dist, int force_type = -1) {
  int type;
  double d2 = kind == 0 ? pt_type_d2(x12, &type, nullptr) : ee_type_d2(x12, &type, nullptr);
  if (force_type >= 0) {
    type = force_type;
    J2<12> X0[12];
    for (int k = 0; k < 12; ++k) X0[k] = jconst<12>(x12[k]);
    d2 = (kind == 0 ? pt_d2_jet(X0, type) : ee_d2_jet(X0, type)).v;
  }
  double dhat = s->P.dhat;
  if (dist) *dist = std::sqrt(d2);
  if (!(std::sqrt(d2) < dhat)) {
    out = jconst<12>(0.0);
    return false;
  }
  J2<12> X[12];
  for (int k = 0; k < 12; ++k) X[k] = jvar<12>(x12[k], k);
  J2<12> D2 = kind == 0 ? pt_d2_jet(X, type) : ee_d2_jet(X, type);
  J2<12> d = jsqrt(D2);
  J2<12> t = d + (-dhat);
  J2<12> b = jconst<12>(-1.0) * (t * t) * jlog((1.0 / dhat) * d);
  if (kind == 1) {
    V3<12> ea = vsub(jpt(X, 1), jpt(X, 0)), eb = vsub(jpt(X, 3), jpt(X, 2));
    V3<12> n = vcross(ea, eb);
    J2<12> c = vdot(n, n);
    if (c.v < eps_x) {
      J2<12> r = (1.0 / eps_x) * c;
      J2<12> m = 2.0 * r - r * r;
      b = m * b;
    }
  }
  out = kappa * b;
  return true;
}

double ee_eps(const zref_scene* s, int ea, int eb) {
  return 1e-3 * s->edge_len2[ea] * s->edge_len2[eb];
}

void gather12(const double* xs, const int* v4, double* x12) {
  for (int a = 0; a < 4; ++a)
    for (int k = 0; k < 3; ++k) x12[3 * a + k] = xs[3 * v4[a] + k];
}

void pair_vertices(const zref_scene* s, int kind, const Pair& p, int* v4) {
  if (kind == 0) {
    v4[0] = p.a;
    v4[1] = s->tris[3 * p.b];
    v4[2] = s->tris[3 * p.b + 1];
    v4[3] = s->tris[3 * p.b + 2];
  } else {
    v4[0] = s->edges[2 * p.a];
    v4[1] = s->edges[2 * p.a + 1];
    v4[2] = s->edges[2 * p.b];
    v4[3] = s->edges[2 * p.b + 1];
  }
}

// ------------------------------------------------------------------ friction (eqs. 9-10)
// D = mu lambda f0(|Pi W (x - x^t)|), f0(y) = -y^3/(3 y*^2) + y^2/y* + y*/3 for
// y < y* = eps_v h, else y.  Written in s = |u|^2 so the jet stays finite at 0.
J2<12> friction_jet(const zref_scene* s, const Fric& f, const double* x12) {
  J2<12> X[12];
  for (int k = 0; k < 12; ++k) X[k] = jvar<12>(x12[k], k);
  J2<12> D[3];
  for (int k = 0; k < 3; ++k) {
    D[k] = jconst<12>(0.0);
    for (int a = 0; a < 4; ++a) D[k] = D[k] + f.w[a] * (X[3 * a + k] + (-f.xt[3 * a + k]));
  }
  J2<12> nd = f.n[0] * D[0] + f.n[1] * D[1] + f.n[2] * D[2];
  J2<12> u[3];
  for (int k = 0; k < 3; ++k) u[k] = D[k] - f.n[k] * nd;
  J2<12> sq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double ys = s->P.eps_v * s->P.dt;
  J2<12> f0;
  if (std::sqrt(sq.v) < ys) {
    double sv = sq.v, r = std::sqrt(sv);
    // s^(3/2): second derivative 3/(4 sqrt(s)) multiplies grad(s) grad(s)^T = O(s), limit 0
    J2<12> s32 = junary(sq, sv * r, 1.5 * r, sv > 0.0 ? 0.75 / r : 0.0);
    f0 = (-1.0 / (3.0 * ys * ys)) * s32 + (1.0 / ys) * sq + ys / 3.0;
  } else {
    f0 = jsqrt(sq);
  }
  return (s->P.mu * f.lam) * f0;
}

// ------------------------------------------------------------------ candidates
struct Box {
  double lo[3], hi[3];
};

void prim_box(const double* xs0, const double* xs1, const int* v, int n, double r, Box& b) {
  for (int k = 0; k < 3; ++k) {
    double lo = INF, hi = -INF;
    for (int a = 0; a < n; ++a) {
      lo = std::min(lo, std::min(xs0[3 * v[a] + k], xs1[3 * v[a] + k]));
      hi = std::max(hi, std::max(xs0[3 * v[a] + k], xs1[3 * v[a] + k]));
    }
    b.lo[k] = lo - r;
    b.hi[k] = hi + r;
  }
}

bool overlap(const Box& a, const Box& b) {
  for (int k = 0; k < 3; ++k)
    if (!(a.lo[k] <= b.hi[k] && b.lo[k] <= a.hi[k])) return false;
  return true;
}

// Candidate set: every inter-body (surface vertex, triangle) and (edge, edge) pair
// whose inflated swept boxes overlap (brute force over all pairs).
void candidates(zref_scene* s, const double* xs0, const double* xs1, double r, std::vector<Pair>& pt,
                std::vector<Pair>& ee) {
  int nt = (int)s->tris.size() / 3, ne = (int)s->edges.size() / 2;
  std::vector<Box> vb(s->nsurf), tb(nt), eb(ne);
  for (int i = 0; i < s->nsurf; ++i) prim_box(xs0, xs1, &i, 1, r, vb[i]);
  for (int t = 0; t < nt; ++t) prim_box(xs0, xs1, &s->tris[3 * t], 3, r, tb[t]);
  for (int e = 0; e < ne; ++e) prim_box(xs0, xs1, &s->edges[2 * e], 2, r, eb[e]);
  auto both_fixed = [&](int b0, int b1) { return s->body_fixed[b0] && s->body_fixed[b1]; };
  std::vector<std::vector<Pair>> tpt(s->nsurf), tee(ne);
#pragma omp parallel for schedule(dynamic, 64)
  for (int i = 0; i < s->nsurf; ++i) {
    int bi = s->sv_body[i];
    for (int t = 0; t < nt; ++t) {
      int bt = s->sv_body[s->tris[3 * t]];
      if (bt == bi || both_fixed(bi, bt)) continue;
      if (overlap(vb[i], tb[t])) tpt[i].push_back({i, t});
    }
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int a = 0; a < ne; ++a) {
    int ba = s->sv_body[s->edges[2 * a]];
    for (int b = a + 1; b < ne; ++b) {
      int bb = s->sv_body[s->edges[2 * b]];
      if (bb == ba || both_fixed(ba, bb)) continue;
      if (overlap(eb[a], eb[b])) tee[a].push_back({a, b});
    }
  }
  pt.clear();
  ee.clear();
  for (auto& v : tpt) pt.insert(pt.end(), v.begin(), v.end());
  for (auto& v : tee) ee.insert(ee.end(), v.begin(), v.end());
}

void candidates_static(zref_scene* s, const double* y) {
  std::vector<double> xs(3 * s->nsurf);
  surface_positions(s, y, xs.data());
  candidates(s, xs.data(), xs.data(), s->P.dhat, s->pt, s->ee);
}

void candidates_swept(zref_scene* s, const double* y, const double* p) {
  std::vector<double> xs0(3 * s->nsurf), xs1(3 * s->nsurf), y1(s->ndof);
  for (int i = 0; i < s->ndof; ++i) y1[i] = y[i] + p[i];
  surface_positions(s, y, xs0.data());
  surface_positions(s, y1.data(), xs1.data());
  candidates(s, xs0.data(), xs1.data(), s->P.dhat, s->pt, s->ee);
}

// ------------------------------------------------------------------ energy evaluation
struct EvalOut {
  double terms[8];
  bool feasible;
  int n_pt_active, n_ee_active;
};

// Energy terms at y on the current candidate set; optional gradient / Hessian.
// mask: bit k selects term k (0 inertia, 1 elastic, 2 orthogonality, 3 kinematic,
// 4 barrier, 5 friction) for the gradient and Hessian; energies are always reported.
EvalOut evaluate(zref_scene* s, const double* y, std::vector<double>* grad, bool hess,
                 unsigned mask = 0x3f) {
  EvalOut o;
  for (double& t : o.terms) t = 0.0;
  o.feasible = true;
  o.n_pt_active = o.n_ee_active = 0;
  if (grad) grad->assign(s->ndof, 0.0);
  if (hess) s->H.clear();
  std::vector<double> g_local(s->ndof, 0.0), g_drop(s->ndof, 0.0);
  std::vector<double>& g_all = grad ? *grad : g_local;
  auto G = [&](int term) -> std::vector<double>& { return (mask >> term) & 1 ? g_all : g_drop; };
  auto HS = [&](int term) { return hess && ((mask >> term) & 1); };
  // inertia, soft (eq. 1): 1/2 m_i |x_i - xhat_i|^2
  for (int i = 0; i < s->nsv; ++i) {
    double e = 0.0;
    for (int k = 0; k < 3; ++k) {
      double d = y[3 * i + k] - s->yhat[3 * i + k];
      e += 0.5 * s->mass[i] * d * d;
      G(0)[3 * i + k] += s->mass[i] * d;
    }
    o.terms[0] += e;
    if (HS(0)) {
      Elem el;
      el.dofs = {3 * i, 3 * i + 1, 3 * i + 2};
      el.M.assign(9, 0.0);
      for (int k = 0; k < 3; ++k) el.M[4 * k] = s->mass[i];
      s->H.push_back(el);
    }
  }
  // affine bodies: inertia 1/2 (q-qhat)^T M_b (q-qhat), M_b = diag(m I, S, S, S);
  // orthogonality; kinematic penalty for driven bodies
  for (size_t b = 0; b < s->bodies.size(); ++b) {
    const Body& B = s->bodies[b];
    if (B.dof0 < 0) continue;
    const double* q = y + B.dof0;
    double Mb[144] = {0};
    for (int k = 0; k < 3; ++k) Mb[k * 12 + k] = B.m;
    for (int blk = 0; blk < 3; ++blk)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Mb[(3 + 3 * blk + i) * 12 + 3 + 3 * blk + j] = B.S[3 * i + j];
    double dq[12];
    for (int k = 0; k < 12; ++k) dq[k] = q[k] - s->yhat[B.dof0 + k];
    double ein = 0.0;
    for (int i = 0; i < 12; ++i) {
      double acc = 0.0;
      for (int j = 0; j < 12; ++j) acc += Mb[i * 12 + j] * dq[j];
      ein += 0.5 * dq[i] * acc;
      G(0)[B.dof0 + i] += acc;
    }
    o.terms[0] += ein;
    double eo, go[12], Ho[144];
    orth_term(s, B, q, &eo, go, hess ? Ho : nullptr);
    o.terms[2] += eo;
    for (int k = 0; k < 12; ++k) G(2)[B.dof0 + k] += go[k];
    double ek = 0.0;
    if (B.mode == 2) {
      // eq. 13: kappa_A/2 |q - q~|^2 - sqrt(m) lambda_A . (q - q~)
      const double* qt = &s->qtilde[12 * b];
      const double sm = std::sqrt(B.m);
      for (int k = 0; k < 12; ++k) {
        double d = q[k] - qt[k];
        ek += 0.5 * B.kappaA * d * d - sm * B.lamA[k] * d;
        G(3)[B.dof0 + k] += B.kappaA * d - sm * B.lamA[k];
      }
    }
    o.terms[3] += ek;
    if (HS(0) || HS(2) || HS(3)) {
      Elem el;
      for (int k = 0; k < 12; ++k) el.dofs.push_back(B.dof0 + k);
      el.M.assign(144, 0.0);
      for (int k = 0; k < 144; ++k) el.M[k] = (HS(0) ? Mb[k] : 0.0) + (HS(2) ? Ho[k] : 0.0);
      if (B.mode == 2 && HS(3))
        for (int k = 0; k < 12; ++k) el.M[13 * k] += B.kappaA;
      s->H.push_back(el);
    }
  }
  // elastic (eq. 1, Sec. IV-D)
  int nt = (int)s->tets.size() / 4;
  std::vector<double> te(nt);
  std::vector<std::array<double, 12>> tg(grad ? nt : 0);
  std::vector<Elem> th(hess ? nt : 0);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
  for (int e = 0; e < nt; ++e) {
    double x12[12];
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 3; ++k) x12[3 * a + k] = y[3 * s->tets[4 * e + a] + k];
    double H144[144];
    bool ok = tet_term(s, e, x12, &te[e], grad ? tg[e].data() : nullptr, hess ? H144 : nullptr, true);
    if (!ok) {
      ++bad;
      continue;
    }
    if (hess) {
      th[e].dofs.resize(12);
      for (int a = 0; a < 4; ++a)
        for (int k = 0; k < 3; ++k) th[e].dofs[3 * a + k] = 3 * s->tets[4 * e + a] + k;
      th[e].M.assign(H144, H144 + 144);
    }
  }
  if (bad) {
    o.feasible = false;
    o.terms[1] = INF;
  } else {
    for (int e = 0; e < nt; ++e) o.terms[1] += te[e];
    if (grad)
      for (int e = 0; e < nt; ++e)
        for (int a = 0; a < 4; ++a)
          for (int k = 0; k < 3; ++k) G(1)[3 * s->tets[4 * e + a] + k] += tg[e][3 * a + k];
    if (HS(1))
      for (int e = 0; e < nt; ++e) s->H.push_back(std::move(th[e]));
  }
  // garment triangles (Sec. IV-D, Baraff-Witkin stretch and shear), elastic term
  const int ncl = (int)s->cloth_v.size() / 3;
  for (int c = 0; c < ncl && o.feasible; ++c) {
    double x9[9], e, g9[9], H81[81];
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 3; ++k) x9[3 * a + k] = y[3 * s->cloth_v[3 * c + a] + k];
    cloth_term(s, c, x9, &e, g9, HS(1) ? H81 : nullptr);
    o.terms[1] += e;
    for (int a = 0; a < 3; ++a)
      for (int k = 0; k < 3; ++k) G(1)[3 * s->cloth_v[3 * c + a] + k] += g9[3 * a + k];
    if (HS(1)) {
      Elem el;
      for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) el.dofs.push_back(3 * s->cloth_v[3 * c + a] + k);
      el.M.assign(H81, H81 + 81);
      s->H.push_back(el);
    }
  }
  // barrier over the active subset of the candidates (eqs. 4-8)
  std::vector<double> xs(3 * s->nsurf);
  surface_positions(s, y, xs.data());
  // prismatic joints (Sec. IV-C-2): kappa (|A1 - A2|_F^2 + |r x (A1 d)|^2), r the gap
  // between the two bodies' images of b1's rest centre of mass c: in b1 (x0 measured
  // from its centre) that image is p1, in b2 A2 (c - c2) + p2.  Hessian: the
  // Gauss-Newton matrix 2 kappa sum_i grad R_i grad R_i^T of the 12 residuals R (PSD;
  // the exact Hessian at R = 0).  The energy joins the constraint term (index 3).
  for (const Joint& jt : s->joints) {
    const Body* Bj[2] = {&s->bodies[jt.b1], &s->bodies[jt.b2]};
    J2<24> q[2][12];
    for (int b = 0; b < 2; ++b) {
      const double* qb = body_q(s, b == 0 ? jt.b1 : jt.b2, y);
      for (int k = 0; k < 12; ++k)
        q[b][k] = Bj[b]->dof0 >= 0 ? jvar<24>(qb[k], 12 * b + k) : jconst<24>(qb[k]);
    }
    J2<24> R[12];
    for (int k = 0; k < 9; ++k) R[k] = q[0][3 + k] + (-1.0) * q[1][3 + k];
    J2<24> r[3], u[3];
    for (int i = 0; i < 3; ++i) {
      J2<24> a2c = jconst<24>(0.0), a1d = jconst<24>(0.0);
      for (int j = 0; j < 3; ++j) {
        a2c = a2c + (Bj[0]->c[j] - Bj[1]->c[j]) * q[1][3 + 3 * i + j];
        a1d = a1d + jt.d[j] * q[0][3 + 3 * i + j];
      }
      r[i] = q[0][i] + (-1.0) * q[1][i] + (-1.0) * a2c;
      u[i] = a1d;
    }
    R[9] = r[1] * u[2] + (-1.0) * (r[2] * u[1]);
    R[10] = r[2] * u[0] + (-1.0) * (r[0] * u[2]);
    R[11] = r[0] * u[1] + (-1.0) * (r[1] * u[0]);
    double e = 0.0, g24[24] = {0}, H[24][24] = {{0}};
    for (int i = 0; i < 12; ++i) {
      e += jt.kappa * R[i].v * R[i].v;
      for (int a = 0; a < 24; ++a) {
        g24[a] += 2.0 * jt.kappa * R[i].v * R[i].g[a];
        for (int b = 0; b < 24; ++b) H[a][b] += 2.0 * jt.kappa * R[i].g[a] * R[i].g[b];
      }
    }
    o.terms[3] += e;
    std::vector<int> loc;  // local indices (0..23) that are DOFs
    Elem el;
    for (int b = 0; b < 2; ++b)
      if (Bj[b]->dof0 >= 0)
        for (int k = 0; k < 12; ++k) {
          loc.push_back(12 * b + k);
          el.dofs.push_back(Bj[b]->dof0 + k);
        }
    for (size_t a = 0; a < loc.size(); ++a) G(3)[el.dofs[a]] += g24[loc[a]];
    if (HS(3) && !loc.empty()) {
      const size_t n = loc.size();
      el.M.assign(n * n, 0.0);
      for (size_t a = 0; a < n; ++a)
        for (size_t b = 0; b < n; ++b) el.M[a * n + b] = H[loc[a]][loc[b]];
      s->H.push_back(el);
    }
  }
  // springs (Sec. IV-C-3): k |x - x_target|^2 per constrained surface vertex, times h^2
  // in incremental-potential units, chained to the DOFs through the vertex map; the
  // energy joins the constraint term (index 3)
  for (const Spring& sp : s->springs) {
    const double h2 = s->P.dt * s->P.dt;
    double dx[3], e = 0.0;
    for (int k = 0; k < 3; ++k) {
      dx[k] = xs[3 * sp.sv + k] - sp.target[k];
      e += h2 * sp.k * dx[k] * dx[k];
    }
    o.terms[3] += e;
    int dofs[12];
    double J[36];
    int nd = vertex_map(s, sp.sv, dofs, J);
    for (int c = 0; c < nd; ++c) {
      double acc = 0.0;
      for (int r = 0; r < 3; ++r) acc += J[r * nd + c] * 2.0 * h2 * sp.k * dx[r];
      G(3)[dofs[c]] += acc;
    }
    if (HS(3) && nd > 0) {
      Elem el;
      el.dofs.assign(dofs, dofs + nd);
      el.M.assign(nd * nd, 0.0);
      for (int a = 0; a < nd; ++a)
        for (int c = 0; c < nd; ++c) {
          double acc = 0.0;
          for (int r = 0; r < 3; ++r) acc += J[r * nd + a] * J[r * nd + c];
          el.M[a * nd + c] = 2.0 * h2 * sp.k * acc;
        }
      s->H.push_back(el);
    }
  }
  double dmin = INF;
  for (int kind = 0; kind < 2; ++kind) {
    const std::vector<Pair>& L = kind == 0 ? s->pt : s->ee;
    int np = (int)L.size();
    std::vector<double> pe(np, 0.0), pd(np, INF);
    std::vector<char> act(np, 0);
    std::vector<std::array<double, 12>> pg(np);
    std::vector<std::vector<double>> ph(hess ? np : 0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < np; ++k) {
      int v4[4];
      pair_vertices(s, kind, L[k], v4);
      double x12[12];
      gather12(xs.data(), v4, x12);
      double eps = kind == 1 ? ee_eps(s, L[k].a, L[k].b) : 0.0;
      J2<12> E;
      double d;
      if (!pair_energy_jet(s, kind, x12, eps, s->kappa, E, &d)) {
        pd[k] = d;
        continue;
      }
      pd[k] = d;
      act[k] = 1;
      pe[k] = E.v;
      for (int i = 0; i < 12; ++i) pg[k][i] = E.g[i];
      if (hess) {
        std::vector<double> Hx(144);
        for (int i = 0; i < 12; ++i)
          for (int j = 0; j < 12; ++j) Hx[i * 12 + j] = E.h[i][j];
        ph[k] = project_psd(12, Hx);
      }
    }
    for (int k = 0; k < np; ++k) {
      dmin = std::min(dmin, pd[k]);
      if (!act[k]) continue;
      if (kind == 0)
        o.n_pt_active++;
      else
        o.n_ee_active++;
      o.terms[4] += pe[k];
      int v4[4];
      pair_vertices(s, kind, L[k], v4);
      Elem el;
      map_pair(s, v4, pg[k].data(), HS(4) ? ph[k].data() : nullptr, G(4), HS(4) ? &el : nullptr);
      if (HS(4)) s->H.push_back(std::move(el));
    }
  }
  if (dmin <= 0.0) o.feasible = false;
  o.terms[7] = dmin;
  // lagged friction (eqs. 9-11)
  for (const Fric& f : s->fric) {
    double x12[12];
    gather12(xs.data(), f.v, x12);
    J2<12> D = friction_jet(s, f, x12);
    o.terms[5] += D.v;
    double g12[12], H144[144];
    for (int i = 0; i < 12; ++i) g12[i] = D.g[i];
    for (int i = 0; i < 12; ++i)
      for (int j = 0; j < 12; ++j) H144[i * 12 + j] = D.h[i][j];
    Elem el;
    map_pair(s, f.v, g12, HS(5) ? H144 : nullptr, G(5), HS(5) ? &el : nullptr);
    if (HS(5)) s->H.push_back(std::move(el));
  }
  o.terms[6] = o.terms[0] + o.terms[1] + o.terms[2] + o.terms[3] + o.terms[4] + o.terms[5];
  if (!o.feasible) o.terms[6] = INF;
  return o;
}

void hess_matvec(const zref_scene* s, const double* v, double* out) {
  std::fill(out, out + s->ndof, 0.0);
  for (const Elem& e : s->H) {
    int n = (int)e.dofs.size();
    for (int r = 0; r < n; ++r) {
      double acc = 0.0;
      for (int c = 0; c < n; ++c) acc += e.M[r * n + c] * v[e.dofs[c]];
      out[e.dofs[r]] += acc;
    }
  }
}

// ------------------------------------------------------------------ PCG (reading)
// block-Jacobi: exact inverses of the 3x3 soft-vertex and 12x12 affine diagonal blocks
struct Precond {
  std::vector<std::vector<int>> blocks;
  std::vector<std::vector<double>> inv;
};

bool build_precond(const zref_scene* s, Precond& P) {
  P.blocks.clear();
  P.inv.clear();
  std::vector<int> blk_of(s->ndof), pos_in(s->ndof);
  for (int i = 0; i < s->nsv; ++i) {
    std::vector<int> b = {3 * i, 3 * i + 1, 3 * i + 2};
    for (int k = 0; k < 3; ++k) {
      blk_of[3 * i + k] = (int)P.blocks.size();
      pos_in[3 * i + k] = k;
    }
    P.blocks.push_back(b);
  }
  for (const Body& B : s->bodies) {
    if (B.dof0 < 0) continue;
    std::vector<int> b;
    for (int k = 0; k < 12; ++k) {
      b.push_back(B.dof0 + k);
      blk_of[B.dof0 + k] = (int)P.blocks.size();
      pos_in[B.dof0 + k] = k;
    }
    P.blocks.push_back(b);
  }
  std::vector<std::vector<double>> D(P.blocks.size());
  for (size_t b = 0; b < P.blocks.size(); ++b) D[b].assign(P.blocks[b].size() * P.blocks[b].size(), 0.0);
  for (const Elem& e : s->H) {
    int n = (int)e.dofs.size();
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) {
        int br = blk_of[e.dofs[r]], bc = blk_of[e.dofs[c]];
        if (br != bc) continue;
        int m = (int)P.blocks[br].size();
        D[br][pos_in[e.dofs[r]] * m + pos_in[e.dofs[c]]] += e.M[r * n + c];
      }
  }
  P.inv.resize(P.blocks.size());
  for (size_t b = 0; b < P.blocks.size(); ++b)
    if (!invert((int)P.blocks[b].size(), D[b], P.inv[b])) return false;
  return true;
}

void apply_precond(const Precond& P, const double* r, double* z) {
  for (size_t b = 0; b < P.blocks.size(); ++b) {
    int m = (int)P.blocks[b].size();
    for (int i = 0; i < m; ++i) {
      double acc = 0.0;
      for (int j = 0; j < m; ++j) acc += P.inv[b][i * m + j] * r[P.blocks[b][j]];
      z[P.blocks[b][i]] = acc;
    }
  }
}

double vdotd(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

int pcg(zref_scene* s, const double* b, double* x, double rtol, int maxit, int* iters, double* relres) {
  int n = s->ndof;
  if (maxit <= 0) maxit = n;
  Precond P;
  if (!build_precond(s, P)) return fail(s, -7, "singular preconditioner block");
  std::vector<double> r(b, b + n), z(n), p(n), q(n);
  std::fill(x, x + n, 0.0);
  double bn = std::sqrt(vdotd(r, r));
  *iters = 0;
  *relres = 0.0;
  if (bn == 0.0) return 0;
  apply_precond(P, r.data(), z.data());
  p = z;
  double rz = vdotd(r, z);
  for (int k = 1; k <= maxit; ++k) {
    hess_matvec(s, p.data(), q.data());
    double pq = vdotd(p, q);
    if (!(pq > 0.0)) {
      *iters = k;
      return fail(s, -7, "PCG breakdown: p^T H p <= 0");
    }
    double alpha = rz / pq;
    for (int i = 0; i < n; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    double rn = std::sqrt(vdotd(r, r));
    *relres = rn / bn;
    *iters = k;
    if (rn <= rtol * bn) return 0;
    apply_precond(P, r.data(), z.data());
    double rz2 = vdotd(r, z);
    double beta = rz2 / rz;
    rz = rz2;
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  return fail(s, -7, "PCG did not converge");
}

// ------------------------------------------------------------------ ACCD (reading)
// Additive CCD (Li, Kaufman, Jiang 2021, Codimensional IPC, Alg. 1), thickness 0,
// t_c = 1, iteration cap 1e4.
double pair_dist(int kind, const double* x12) {
  int t;
  return std::sqrt(kind == 0 ? pt_type_d2(x12, &t, nullptr) : ee_type_d2(x12, &t, nullptr));
}

bool accd(int kind, const double* x12in, const double* p12in, double s, double* toi) {
  double x[12], p[12];
  std::memcpy(x, x12in, sizeof(x));
  std::memcpy(p, p12in, sizeof(p));
  double mean[3] = {0, 0, 0};
  for (int a = 0; a < 4; ++a)
    for (int k = 0; k < 3; ++k) mean[k] += 0.25 * p[3 * a + k];
  for (int a = 0; a < 4; ++a)
    for (int k = 0; k < 3; ++k) p[3 * a + k] -= mean[k];
  double nrm[4];
  for (int a = 0; a < 4; ++a) nrm[a] = std::sqrt(p[3 * a] * p[3 * a] + p[3 * a + 1] * p[3 * a + 1] + p[3 * a + 2] * p[3 * a + 2]);
  double lp = kind == 0 ? nrm[0] + std::max(nrm[1], std::max(nrm[2], nrm[3]))
                        : std::max(nrm[0], nrm[1]) + std::max(nrm[2], nrm[3]);
  if (lp == 0.0) {
    *toi = 1.0;
    return true;
  }
  double d = pair_dist(kind, x);
  if (!(d > 0.0)) return false;
  double g = s * d, t = 0.0, tl = (1.0 - s) * d / lp;
  for (int it = 0; it < 10000; ++it) {
    for (int k = 0; k < 12; ++k) x[k] += tl * p[k];
    d = pair_dist(kind, x);
    if (t > 0.0 && d < g) break;
    t += tl;
    if (t > 1.0) {
      *toi = 1.0;
      return true;
    }
    tl = (1.0 - s) * d / lp;
  }
  *toi = t;
  return true;
}

int ccd_bound(zref_scene* s, const double* y, const double* p, double* alpha) {
  std::vector<double> xs(3 * s->nsurf), dx(3 * s->nsurf);
  surface_positions(s, y, xs.data());
  surface_disp(s, p, dx.data());
  double amin = 1.0;
  int bad = 0;
  for (int kind = 0; kind < 2; ++kind) {
    const std::vector<Pair>& L = kind == 0 ? s->pt : s->ee;
    int np = (int)L.size();
    std::vector<double> tk(np, 1.0);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
    for (int k = 0; k < np; ++k) {
      int v4[4];
      pair_vertices(s, kind, L[k], v4);
      double x12[12], p12[12];
      gather12(xs.data(), v4, x12);
      gather12(dx.data(), v4, p12);
      if (!accd(kind, x12, p12, s->P.ccd_s, &tk[k])) ++bad;
    }
    for (int k = 0; k < np; ++k) amin = std::min(amin, tk[k]);
  }
  *alpha = amin;
  if (bad) return fail(s, -3, "intersecting pair at CCD start");
  return 0;
}

// ------------------------------------------------------------------ step setup
// predictor (eq. 3): xhat = x + h v + h^2 g; qhat = q + h qdot + h^2 (g, 0, 0, 0)
// (centred x0 makes the affine gravity force (m g, 0, 0, 0), so M_b^{-1} f = (g,0,0,0))
void begin_step(zref_scene* s) {
  const double h = s->P.dt;
  s->yhat.assign(s->ndof, 0.0);
  for (int i = 0; i < s->nsv; ++i)
    for (int k = 0; k < 3; ++k) s->yhat[3 * i + k] = s->y[3 * i + k] + h * s->ydot[3 * i + k] + h * h * s->P.gravity[k];
  s->qtilde.assign(12 * s->bodies.size(), 0.0);
  double tnext = (s->step + 1) * h;
  for (size_t b = 0; b < s->bodies.size(); ++b) {
    Body& B = s->bodies[b];
    if (B.dof0 < 0) continue;
    for (int k = 0; k < 12; ++k) {
      double gk = k < 3 ? s->P.gravity[k] : 0.0;
      s->yhat[B.dof0 + k] = s->y[B.dof0 + k] + h * s->ydot[B.dof0 + k] + h * h * gk;
    }
    // kinematic target (Sec. IV-C-1): rest state moved at target_vel until target_stop,
    // or the target the caller set (the force controller of Sec. IV-A)
    if (B.has_target) {
      for (int k = 0; k < 12; ++k) s->qtilde[12 * b + k] = B.target[k];
      continue;
    }
    double tt = std::min(tnext, B.tstop);
    for (int k = 0; k < 12; ++k) s->qtilde[12 * b + k] = B.qrest[k];
    for (int k = 0; k < 3; ++k) s->qtilde[12 * b + k] += tt * B.tvel[k];
  }
  // lagged friction at y^t (eqs. 9-10, lambda = kappa m |b'(d)| in IP units)
  s->kappa_lag = s->kappa;
  candidates_static(s, s->y.data());
  std::vector<double> xs(3 * s->nsurf);
  surface_positions(s, s->y.data(), xs.data());
  s->fric.clear();
  for (int kind = 0; kind < 2; ++kind) {
    const std::vector<Pair>& L = kind == 0 ? s->pt : s->ee;
    for (const Pair& pr : L) {
      Fric f;
      f.kind = kind;
      pair_vertices(s, kind, pr, f.v);
      gather12(xs.data(), f.v, f.xt);
      int type;
      double d2, cp0[3], cp1[3];
      if (kind == 0) {
        double bary[3];
        d2 = pt_type_d2(f.xt, &type, bary);
        f.w[0] = 1.0;
        for (int i = 0; i < 3; ++i) f.w[1 + i] = -bary[i];
        for (int k = 0; k < 3; ++k) {
          cp0[k] = f.xt[k];
          cp1[k] = bary[0] * f.xt[3 + k] + bary[1] * f.xt[6 + k] + bary[2] * f.xt[9 + k];
        }
      } else {
        double gm[2];
        d2 = ee_type_d2(f.xt, &type, gm);
        f.w[0] = 1.0 - gm[0];
        f.w[1] = gm[0];
        f.w[2] = -(1.0 - gm[1]);
        f.w[3] = -gm[1];
        for (int k = 0; k < 3; ++k) {
          cp0[k] = (1.0 - gm[0]) * f.xt[k] + gm[0] * f.xt[3 + k];
          cp1[k] = (1.0 - gm[1]) * f.xt[6 + k] + gm[1] * f.xt[9 + k];
        }
      }
      double d = std::sqrt(d2);
      if (!(d < s->P.dhat) || !(d > 0.0)) continue;
      double b3[3];
      barrier3(d, s->P.dhat, b3);
      double m = 1.0;
      if (kind == 1) {
        D3 ea = d3(f.xt + 3) - d3(f.xt), eb = d3(f.xt + 9) - d3(f.xt + 6);
        D3 n = cross(ea, eb);
        double c = dot(n, n), eps = ee_eps(s, pr.a, pr.b);
        if (c < eps) m = 2.0 * c / eps - (c / eps) * (c / eps);
      }
      f.lam = s->kappa * m * std::fabs(b3[1]);
      double nn = 0.0;
      for (int k = 0; k < 3; ++k) {
        f.n[k] = cp0[k] - cp1[k];
        nn += f.n[k] * f.n[k];
      }
      nn = std::sqrt(nn);
      if (!(nn > 0.0)) continue;
      for (int k = 0; k < 3; ++k) f.n[k] /= nn;
      s->fric.push_back(f);
    }
  }
}

double auto_kappa(const zref_scene* s) {
  // reading: the barrier alone holds one mean soft vertex against gravity at d = dhat/2
  double g = std::sqrt(s->P.gravity[0] * s->P.gravity[0] + s->P.gravity[1] * s->P.gravity[1] +
                       s->P.gravity[2] * s->P.gravity[2]);
  double mbar = 0.0;
  for (double m : s->mass) mbar += m;
  mbar = s->nsv ? mbar / s->nsv : 1.0;
  if (g == 0.0) g = 9.81;
  return s->P.dt * s->P.dt * mbar * g / (s->P.dhat * (std::log(2.0) + 0.5));
}

double max_vertex_disp(const zref_scene* s, const double* p) {
  double m = 0.0;
  for (int i = 0; i < s->nsv; ++i) {
    double n = std::sqrt(p[3 * i] * p[3 * i] + p[3 * i + 1] * p[3 * i + 1] + p[3 * i + 2] * p[3 * i + 2]);
    m = std::max(m, n);
  }
  for (const Body& B : s->bodies) {
    if (B.dof0 < 0) continue;
    const double* q = p + B.dof0;
    for (int v = 0; v < (int)B.x0.size() / 3; ++v) {
      double dx[3];
      for (int k = 0; k < 3; ++k)
        dx[k] = q[3 + 3 * k] * B.x0[3 * v] + q[3 + 3 * k + 1] * B.x0[3 * v + 1] + q[3 + 3 * k + 2] * B.x0[3 * v + 2] + q[k];
      m = std::max(m, std::sqrt(dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2]));
    }
  }
  return m;
}

double min_dist(zref_scene* s, const double* y) {
  std::vector<double> xs(3 * s->nsurf);
  surface_positions(s, y, xs.data());
  double dmin = INF;
  for (int kind = 0; kind < 2; ++kind) {
    const std::vector<Pair>& L = kind == 0 ? s->pt : s->ee;
    for (const Pair& pr : L) {
      int v4[4];
      pair_vertices(s, kind, pr, v4);
      double x12[12];
      gather12(xs.data(), v4, x12);
      dmin = std::min(dmin, pair_dist(kind, x12));
    }
  }
  return dmin;
}

bool any_inverted(const zref_scene* s, const double* y) {
  int nt = (int)s->tets.size() / 4;
  for (int e = 0; e < nt; ++e) {
    double x12[12], F[9];
    for (int a = 0; a < 4; ++a)
      for (int k = 0; k < 3; ++k) x12[3 * a + k] = y[3 * s->tets[4 * e + a] + k];
    tet_F_B(x12, &s->Dminv[9 * e], F, nullptr);
    double J = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) + F[2] * (F[3] * F[7] - F[4] * F[6]);
    if (!(J > 0.0)) return true;
  }
  return false;
}

// one time step of the Newton method (Sec. III eq. 11; loop structure is a reading)
int time_step(zref_scene* s, zref_step_stats* st) {
  const double h = s->P.dt;
  const int n = s->ndof;
  std::memset(st, 0, sizeof(*st));
  st->alpha_ccd_min = 1.0;
  begin_step(s);
  s->yt = s->y;
  s->ydt = s->ydot;
  // warm start y^t + alpha h ydot^t, alpha from ACCD over that sweep
  std::vector<double> p(n), grad(n), y1(n);
  for (int i = 0; i < n; ++i) p[i] = h * s->ydot[i];
  candidates_swept(s, s->y.data(), p.data());
  double a0;
  int rc = ccd_bound(s, s->y.data(), p.data(), &a0);
  if (rc) return rc;
  for (;;) {
    for (int i = 0; i < n; ++i) y1[i] = s->y[i] + a0 * p[i];
    if (!any_inverted(s, y1.data())) break;
    a0 *= 0.5;
    if (a0 < 1e-10) {
      y1 = s->y;
      break;
    }
  }
  s->y = y1;
  candidates_static(s, s->y.data());
  s->dprev = min_dist(s, s->y.data());
  const bool auto_k = s->P.kappa <= 0.0;
  const double tol = s->P.newton_tol * h;
  int it = 0;
  bool conv = false;
  for (; it < s->P.newton_max; ++it) {
    if (s->record) s->recs.push_back({s->step, s->kappa_lag, s->kappa, s->yt, s->ydt, s->y});
    EvalOut eo = evaluate(s, s->y.data(), &grad, true);
    st->energy = eo.terms[6];
    st->n_pt_active = eo.n_pt_active;
    st->n_ee_active = eo.n_ee_active;
    std::vector<double> rhs(n);
    for (int i = 0; i < n; ++i) rhs[i] = -grad[i];
    int pit;
    double rr;
    rc = pcg(s, rhs.data(), p.data(), s->P.pcg_rtol, s->P.pcg_max, &pit, &rr);
    st->pcg_iters += pit;
    if (rc) return rc;
    if (max_vertex_disp(s, p.data()) <= tol) {
      // augmented Lagrangian (eq. 13): while a driven body misses its target by more
      // than al_tol, lambda_A <- lambda_A - kappa_A / sqrt(m) (q - q~) and Newton goes on
      double worst = 0.0;
      for (size_t b = 0; b < s->bodies.size(); ++b) {
        const Body& B = s->bodies[b];
        if (B.mode != 2) continue;
        for (int k = 0; k < 12; ++k)
          worst = std::max(worst, std::fabs(s->y[B.dof0 + k] - s->qtilde[12 * b + k]));
      }
      if (s->al_tol > 0.0 && worst > s->al_tol && st->al_updates < s->al_max) {
        for (size_t b = 0; b < s->bodies.size(); ++b) {
          Body& B = s->bodies[b];
          if (B.mode != 2) continue;
          const double c = B.kappaA / std::sqrt(B.m);
          for (int k = 0; k < 12; ++k) B.lamA[k] -= c * (s->y[B.dof0 + k] - s->qtilde[12 * b + k]);
        }
        st->al_updates++;
        continue;
      }
      conv = true;
      break;
    }
    candidates_swept(s, s->y.data(), p.data());
    st->n_pt_cand = (int)s->pt.size();
    st->n_ee_cand = (int)s->ee.size();
    double alpha;
    rc = ccd_bound(s, s->y.data(), p.data(), &alpha);
    if (rc) return rc;
    st->alpha_ccd_min = std::min(st->alpha_ccd_min, alpha);
    double E0 = evaluate(s, s->y.data(), nullptr, false).terms[6];
    for (;;) {
      for (int i = 0; i < n; ++i) y1[i] = s->y[i] + alpha * p[i];
      EvalOut e1 = evaluate(s, y1.data(), nullptr, false);
      if (e1.feasible && e1.terms[6] <= E0) break;
      alpha *= 0.5;
      st->ls_backtracks++;
      if (alpha < 1e-10) return fail(s, -6, "line search failed");
    }
    s->y = y1;
    double dm = min_dist(s, s->y.data());
    if (auto_k && dm < 1e-3 * s->P.dhat && dm < s->dprev) s->kappa *= 2.0;
    s->dprev = dm;
  }
  st->newton_iters = it;
  st->kappa = s->kappa;
  st->d_min = min_dist(s, s->y.data());
  if (!conv) return fail(s, -5, "Newton did not converge");
  // velocity update (text after eq. 11)
  for (int i = 0; i < n; ++i) s->ydot[i] = (s->y[i] - s->yt[i]) / h;
  s->step += 1;
  return 0;
}

}  // namespace

// ================================================================== C interface
extern "C" {

// Contact force sensing (Sec. IV-B): the barrier energy B of eq. 4 over the static
// candidate set at y (every inter-body pair closer than dhat) is differentiated with
// respect to the surface vertex positions; the force on a vertex is -dB/dx divided by
// h^2 (the incremental potential is h^2 times the potential energy), and the resultant
// on a body is the sum over its surface vertices.  forces: [n_bodies][3], soft bodies
// first, then affine bodies, in Newtons.
int zref_contact_forces(zref_scene* s, const double* y, double* forces) {
  if (!s || !y || !forces) return -1;
  const int nb = s->n_soft_bodies + (int)s->bodies.size();
  std::vector<double> f(3 * (size_t)nb, 0.0);
  candidates_static(s, y);
  std::vector<double> xs(3 * s->nsurf);
  surface_positions(s, y, xs.data());
  const double h2 = s->P.dt * s->P.dt;
  for (int kind = 0; kind < 2; ++kind) {
    const std::vector<Pair>& L = kind == 0 ? s->pt : s->ee;
    for (const Pair& pr : L) {
      int v4[4];
      pair_vertices(s, kind, pr, v4);
      double x12[12];
      gather12(xs.data(), v4, x12);
      double eps = kind == 1 ? ee_eps(s, pr.a, pr.b) : 0.0;
      J2<12> E;
      double d;
      if (!pair_energy_jet(s, kind, x12, eps, s->kappa, E, &d)) continue;
      for (int a = 0; a < 4; ++a) {
        int b = s->sv_body[v4[a]];
        for (int k = 0; k < 3; ++k) f[3 * b + k] -= E.g[3 * a + k] / h2;
      }
    }
  }
  std::copy(f.begin(), f.end(), forces);
  return 0;
}

// Kinematic target of driven affine body `body` (its index among the affine bodies)
// for the following steps: q (12, host), or NULL to return to the scheduled target.
int zref_set_drive_target(zref_scene* s, int32_t body, const double* q) {
  if (!s || body < 0 || body >= (int)s->bodies.size() || s->bodies[body].mode != 2) return -1;
  Body& B = s->bodies[body];
  B.has_target = q != nullptr;
  if (q)
    for (int k = 0; k < 12; ++k) B.target[k] = q[k];
  return 0;
}

// Springs (Sec. IV-C-3): n constrained surface vertices sv (distinct), stiffness k (N/m)
// and targets [n][3]; n = 0 removes them.  Replaces the previous set.
int zref_set_springs(zref_scene* s, int32_t n, const int32_t* sv, const double* k, const double* targets) {
  if (!s || n < 0 || (n && (!sv || !k || !targets))) return -1;
  std::vector<Spring> v;
  std::vector<char> seen(s->nsurf, 0);
  for (int i = 0; i < n; ++i) {
    if (sv[i] < 0 || sv[i] >= s->nsurf || seen[sv[i]] || !(k[i] >= 0.0)) return -1;
    seen[sv[i]] = 1;
    Spring sp;
    sp.sv = sv[i];
    sp.k = k[i];
    for (int c = 0; c < 3; ++c) sp.target[c] = targets[3 * i + c];
    v.push_back(sp);
  }
  s->springs = v;
  return 0;
}

// Augmented Lagrangian multiplier updates of the kinematic energy (eq. 13): at Newton
// convergence, while max |q - q~| over the driven bodies exceeds tol, update every
// driven body's multiplier and continue, at most max_updates times per step.
// tol = 0 keeps the multipliers at their values.  lam (optional, [n_affine][12]) reads
// the multipliers.
int zref_kinematic_al(zref_scene* s, double tol, int32_t max_updates, double* lam) {
  if (!s || tol < 0.0 || max_updates < 0) return -1;
  s->al_tol = tol;
  s->al_max = max_updates;
  if (lam)
    for (size_t b = 0; b < s->bodies.size(); ++b)
      for (int k = 0; k < 12; ++k) lam[12 * b + k] = s->bodies[b].lamA[k];
  return 0;
}

// Prismatic joints (Sec. IV-C-2) between affine bodies b12[i][0] and b12[i][1] (distinct,
// not both fixed) with axis axes[i] (b1's rest frame) and stiffness kappa[i]; n = 0
// removes them.  Replaces the previous set.
int zref_set_prismatic_joints(zref_scene* s, int32_t n, const int32_t* b12, const double* axes,
                              const double* kappa) {
  if (!s || n < 0 || (n && (!b12 || !axes || !kappa))) return -1;
  std::vector<Joint> v;
  const int nb = (int)s->bodies.size();
  for (int i = 0; i < n; ++i) {
    Joint j;
    j.b1 = b12[2 * i];
    j.b2 = b12[2 * i + 1];
    if (j.b1 < 0 || j.b1 >= nb || j.b2 < 0 || j.b2 >= nb || j.b1 == j.b2 || !(kappa[i] >= 0.0)) return -1;
    if (s->bodies[j.b1].dof0 < 0 && s->bodies[j.b2].dof0 < 0) return -1;
    for (int k = 0; k < 3; ++k) j.d[k] = axes[3 * i + k];
    j.kappa = kappa[i];
    v.push_back(j);
  }
  s->joints = v;
  return 0;
}

int zref_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  nthreads_req = n;
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

const char* zref_last_error(const zref_scene* s) { return s ? s->err.c_str() : "null scene"; }

int zref_scene_create(const zref_params* p, const zref_soft_desc* soft, int32_t n_soft,
                      const zref_affine_desc* aff, int32_t n_aff, zref_scene** out) {
  if (!p || !out || n_soft < 0 || n_aff < 0) return -1;
  zref_scene* s = new zref_scene();
  s->P = *p;
  s->n_soft_bodies = n_soft;
  int nbodies = n_soft + n_aff;
  s->body_fixed.assign(nbodies, 0);
  // --- soft bodies: Dm, V, Lame parameters, lumped mass, boundary faces (Sec. III eq. 1)
  std::vector<std::array<int, 3>> surf_tris;  // in soft vertex ids, outward
  for (int b = 0; b < n_soft; ++b) {
    const zref_soft_desc& d = soft[b];
    int v0 = s->nsv;
    if (d.model < 0 || d.model > 3 || (d.model == 3) != (d.n_tris > 0) || (d.model == 3 && d.n_tets) ||
        (d.n_tris && !d.tris)) {
      delete s;
      return -1;
    }
    double mu = d.E / (2.0 * (1.0 + d.nu)), lam = d.E * d.nu / ((1.0 + d.nu) * (1.0 - 2.0 * d.nu));
    for (int i = 0; i < d.n_verts; ++i) {
      for (int k = 0; k < 3; ++k) {
        s->X.push_back(d.rest_pos[3 * i + k]);
        s->x_init.push_back(d.pos0 ? d.pos0[3 * i + k] : d.rest_pos[3 * i + k]);
        s->v_init.push_back(d.vel0 ? d.vel0[3 * i + k] : 0.0);
      }
      s->vbody.push_back(b);
      s->mass.push_back(0.0);
    }
    s->nsv += d.n_verts;
    std::map<std::array<int, 3>, std::pair<int, std::array<int, 3>>> faces;
    for (int e = 0; e < d.n_tets; ++e) {
      int t[4];
      for (int a = 0; a < 4; ++a) {
        t[a] = d.tets[4 * e + a];
        if (t[a] < 0 || t[a] >= d.n_verts) {
          delete s;
          return -2;
        }
        t[a] += v0;
      }
      double Dm[9];
      for (int i = 0; i < 3; ++i)
        for (int m = 0; m < 3; ++m) Dm[3 * i + m] = s->X[3 * t[m + 1] + i] - s->X[3 * t[0] + i];
      double det = Dm[0] * (Dm[4] * Dm[8] - Dm[5] * Dm[7]) - Dm[1] * (Dm[3] * Dm[8] - Dm[5] * Dm[6]) +
                   Dm[2] * (Dm[3] * Dm[7] - Dm[4] * Dm[6]);
      if (det < 0.0) {  // reading: reorder vertices 1 and 2 of a negative tet
        std::swap(t[1], t[2]);
        for (int i = 0; i < 3; ++i)
          for (int m = 0; m < 3; ++m) Dm[3 * i + m] = s->X[3 * t[m + 1] + i] - s->X[3 * t[0] + i];
        det = -det;
      }
      double L = 0.0;
      for (int k = 0; k < 9; ++k) L = std::max(L, std::fabs(Dm[k]));
      if (!(det > 1e-14 * L * L * L)) {
        delete s;
        return -2;
      }
      std::vector<double> Dmi;
      invert(3, std::vector<double>(Dm, Dm + 9), Dmi);
      for (int k = 0; k < 4; ++k) s->tets.push_back(t[k]);
      for (int k = 0; k < 9; ++k) s->Dminv.push_back(Dmi[k]);
      double V = det / 6.0;
      s->vol.push_back(V);
      s->lam_mu.push_back(mu);
      s->lam_mu.push_back(lam);
      s->tet_model.push_back(d.model);
      for (int a = 0; a < 4; ++a) s->mass[t[a]] += d.rho * V / 4.0;  // reading: equal lumping
      // faces; outward orientation decided by the side of the opposite vertex
      for (int j = 0; j < 4; ++j) {
        int f[3], k = 0;
        for (int a = 0; a < 4; ++a)
          if (a != j) f[k++] = t[a];
        D3 A = d3(&s->X[3 * f[0]]), Bv = d3(&s->X[3 * f[1]]), C = d3(&s->X[3 * f[2]]), O = d3(&s->X[3 * t[j]]);
        if (dot(cross(Bv - A, C - A), O - A) > 0.0) std::swap(f[1], f[2]);
        std::array<int, 3> key = {f[0], f[1], f[2]};
        std::sort(key.begin(), key.end());
        auto it = faces.find(key);
        if (it == faces.end())
          faces[key] = {1, {f[0], f[1], f[2]}};
        else
          it->second.first++;
      }
    }
    // garment (reading): rest material coordinates (u, v) = rest (x, z); per triangle
    // the inverse of the rest edge matrix [[du1, du2], [dv1, dv2]], the rest area, the
    // stretch stiffness E and the shear stiffness E / (2 (1 + nu)) (N/m), mass rho A / 3
    // per vertex (rho in kg/m^2); every triangle is a surface triangle as given
    for (int e = 0; e < d.n_tris; ++e) {
      int t[3];
      for (int a = 0; a < 3; ++a) {
        t[a] = d.tris[3 * e + a];
        if (t[a] < 0 || t[a] >= d.n_verts) {
          delete s;
          return -2;
        }
        t[a] += v0;
      }
      double du1 = s->X[3 * t[1]] - s->X[3 * t[0]], du2 = s->X[3 * t[2]] - s->X[3 * t[0]];
      double dv1 = s->X[3 * t[1] + 2] - s->X[3 * t[0] + 2], dv2 = s->X[3 * t[2] + 2] - s->X[3 * t[0] + 2];
      double det = du1 * dv2 - du2 * dv1;
      double L = std::max({std::fabs(du1), std::fabs(du2), std::fabs(dv1), std::fabs(dv2)});
      if (!(std::fabs(det) > 1e-12 * L * L)) {
        delete s;
        return -2;
      }
      // inverse of [[du1, du2], [dv1, dv2]]
      double M[4] = {dv2 / det, -du2 / det, -dv1 / det, du1 / det};
      double A = 0.5 * std::fabs(det);
      for (int a = 0; a < 3; ++a) s->cloth_v.push_back(t[a]);
      for (int k = 0; k < 4; ++k) s->cloth_d.push_back(M[k]);
      s->cloth_d.push_back(A);
      s->cloth_d.push_back(d.E);
      s->cloth_d.push_back(d.E / (2.0 * (1.0 + d.nu)));
      for (int a = 0; a < 3; ++a) s->mass[t[a]] += d.rho * A / 3.0;
      std::array<int, 3> key = {t[0], t[1], t[2]};
      std::sort(key.begin(), key.end());
      auto it = faces.find(key);
      if (it == faces.end())
        faces[key] = {1, {t[0], t[1], t[2]}};
      else
        it->second.first++;
    }
    for (auto& kv : faces)
      if (kv.second.first == 1) surf_tris.push_back(kv.second.second);
  }
  s->ndof = 3 * s->nsv;
  // --- surface numbering: soft surface vertices ascending, then affine vertices
  std::vector<int> soft_sid(s->nsv, -1);
  {
    std::vector<char> on(s->nsv, 0);
    for (auto& t : surf_tris)
      for (int k = 0; k < 3; ++k) on[t[k]] = 1;
    for (int i = 0; i < s->nsv; ++i)
      if (on[i]) {
        soft_sid[i] = s->nsurf++;
        s->sv_kind.push_back(0);
        s->sv_id.push_back(i);
        s->sv_body.push_back(s->vbody[i]);
        for (int k = 0; k < 3; ++k) s->sv_x0.push_back(0.0);
      }
  }
  std::vector<std::array<int, 3>> all_tris;
  for (auto& t : surf_tris) all_tris.push_back({soft_sid[t[0]], soft_sid[t[1]], soft_sid[t[2]]});
  // --- affine bodies: mass properties by the divergence theorem over origin tets
  for (int b = 0; b < n_aff; ++b) {
    const zref_affine_desc& d = aff[b];
    Body B;
    B.mode = d.mode;
    B.rho = d.rho;
    B.stiff = d.stiffness;
    B.kappaA = d.kappa_A;
    for (int k = 0; k < 3; ++k) B.tvel[k] = d.target_vel[k];
    B.tstop = d.target_stop;
    for (int k = 0; k < 12; ++k) B.qdot0[k] = d.qdot0[k];
    double V = 0.0, m1[3] = {0, 0, 0}, m2[9] = {0};
    for (int t = 0; t < d.n_tris; ++t) {
      int i0 = d.tris[3 * t], i1 = d.tris[3 * t + 1], i2 = d.tris[3 * t + 2];
      if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= d.n_verts || i1 >= d.n_verts || i2 >= d.n_verts) {
        delete s;
        return -2;
      }
      D3 a = d3(d.rest_pos + 3 * i0), bb = d3(d.rest_pos + 3 * i1), c = d3(d.rest_pos + 3 * i2);
      double vt = dot(a, cross(bb, c)) / 6.0;  // signed volume of (0, a, b, c)
      V += vt;
      D3 sm = a + bb + c;
      m1[0] += vt * sm.x / 4.0;
      m1[1] += vt * sm.y / 4.0;
      m1[2] += vt * sm.z / 4.0;
      // int_T x x^T = V/20 (sum_i v_i v_i^T + s s^T), vertices 0, a, b, c
      double P[3][3] = {{a.x, a.y, a.z}, {bb.x, bb.y, bb.z}, {c.x, c.y, c.z}};
      double S[3] = {sm.x, sm.y, sm.z};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double acc = S[i] * S[j];
          for (int r = 0; r < 3; ++r) acc += P[r][i] * P[r][j];
          m2[3 * i + j] += vt / 20.0 * acc;
        }
    }
    if (!(V > 0.0)) {
      delete s;
      s = nullptr;
      return -2;
    }
    B.V = V;
    B.m = d.rho * V;
    for (int k = 0; k < 3; ++k) B.c[k] = m1[k] / V;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) B.S[3 * i + j] = d.rho * (m2[3 * i + j] - V * B.c[i] * B.c[j]);
    for (int k = 0; k < 12; ++k) B.qrest[k] = 0.0;
    for (int k = 0; k < 3; ++k) {
      B.qrest[k] = B.c[k];
      B.qrest[3 + 4 * k] = 1.0;
    }
    B.sv0 = s->nsurf;
    B.nsv = d.n_verts;
    for (int i = 0; i < d.n_verts; ++i) {
      for (int k = 0; k < 3; ++k) {
        double x0 = d.rest_pos[3 * i + k] - B.c[k];
        B.x0.push_back(x0);
        s->sv_x0.push_back(x0);
      }
      s->sv_kind.push_back(1);
      s->sv_id.push_back(b);
      s->sv_body.push_back(n_soft + b);
      s->nsurf++;
    }
    for (int t = 0; t < d.n_tris; ++t)
      all_tris.push_back({B.sv0 + d.tris[3 * t], B.sv0 + d.tris[3 * t + 1], B.sv0 + d.tris[3 * t + 2]});
    if (B.mode == 1) {
      s->body_fixed[n_soft + b] = 1;
    } else {
      B.dof0 = s->ndof;
      s->ndof += 12;
    }
    s->bodies.push_back(B);
  }
  // --- canonical triangles: smallest id first (orientation kept), sorted
  for (auto& t : all_tris) {
    int k = (t[1] < t[0] && t[1] < t[2]) ? 1 : (t[2] < t[0] && t[2] < t[1]) ? 2 : 0;
    t = {t[k], t[(k + 1) % 3], t[(k + 2) % 3]};
  }
  std::sort(all_tris.begin(), all_tris.end());
  for (auto& t : all_tris)
    for (int k = 0; k < 3; ++k) s->tris.push_back(t[k]);
  std::vector<std::array<int, 2>> E;
  for (auto& t : all_tris)
    for (int k = 0; k < 3; ++k) {
      int a = t[k], b = t[(k + 1) % 3];
      E.push_back({std::min(a, b), std::max(a, b)});
    }
  std::sort(E.begin(), E.end());
  E.erase(std::unique(E.begin(), E.end()), E.end());
  for (auto& e : E) {
    s->edges.push_back(e[0]);
    s->edges.push_back(e[1]);
    // rest length^2: soft from rest positions, affine from x0
    double l2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      double xa = s->sv_kind[e[0]] == 0 ? s->X[3 * s->sv_id[e[0]] + k] : s->sv_x0[3 * e[0] + k];
      double xb = s->sv_kind[e[1]] == 0 ? s->X[3 * s->sv_id[e[1]] + k] : s->sv_x0[3 * e[1] + k];
      l2 += (xb - xa) * (xb - xa);
    }
    s->edge_len2.push_back(l2);
  }
  // --- initial state
  std::vector<double> y0(s->ndof), yd0(s->ndof);
  for (int i = 0; i < 3 * s->nsv; ++i) {
    y0[i] = s->x_init[i];
    yd0[i] = s->v_init[i];
  }
  for (const Body& B : s->bodies)
    if (B.dof0 >= 0)
      for (int k = 0; k < 12; ++k) {
        y0[B.dof0 + k] = B.qrest[k];
        yd0[B.dof0 + k] = B.qdot0[k];
      }
  int rc = zref_set_state(s, y0.data(), yd0.data(), 0.0, 0);
  if (rc) {
    delete s;
    return rc;
  }
  *out = s;
  return 0;
}

void zref_scene_destroy(zref_scene* s) { delete s; }

int zref_sizes(const zref_scene* s, int64_t* o) {
  o[0] = s->ndof;
  o[1] = s->nsv;
  o[2] = (int64_t)s->tets.size() / 4;
  o[3] = s->nsurf;
  o[4] = (int64_t)s->tris.size() / 3;
  o[5] = (int64_t)s->edges.size() / 2;
  int nf = 0;
  for (const Body& B : s->bodies) nf += B.dof0 >= 0;
  o[6] = nf;
  o[7] = (int64_t)s->bodies.size() + s->n_soft_bodies;
  return 0;
}

int zref_surface(const zref_scene* s, int32_t* tris, int32_t* edges, int32_t* vbody) {
  if (tris) std::copy(s->tris.begin(), s->tris.end(), tris);
  if (edges) std::copy(s->edges.begin(), s->edges.end(), edges);
  if (vbody) std::copy(s->sv_body.begin(), s->sv_body.end(), vbody);
  return 0;
}

int zref_lumped_mass(const zref_scene* s, double* m) {
  std::copy(s->mass.begin(), s->mass.end(), m);
  return 0;
}

int zref_affine_props(const zref_scene* s, double* o) {
  for (size_t b = 0; b < s->bodies.size(); ++b) {
    const Body& B = s->bodies[b];
    o[14 * b] = B.V;
    o[14 * b + 1] = B.m;
    for (int k = 0; k < 3; ++k) o[14 * b + 2 + k] = B.c[k];
    for (int k = 0; k < 9; ++k) o[14 * b + 5 + k] = B.S[k];
  }
  return 0;
}

int zref_set_state(zref_scene* s, const double* y, const double* ydot, double kappa, int32_t step) {
  s->y.assign(y, y + s->ndof);
  s->ydot.assign(ydot, ydot + s->ndof);
  for (double v : s->y)
    if (!std::isfinite(v)) return fail(s, -8, "non-finite state");
  s->step = step;
  s->kappa = kappa > 0.0 ? kappa : (s->P.kappa > 0.0 ? s->P.kappa : auto_kappa(s));
  if (any_inverted(s, s->y.data())) return fail(s, -2, "inverted tet in state");
  begin_step(s);
  if (min_dist(s, s->y.data()) <= 0.0) return fail(s, -3, "intersecting state");
  return 0;
}

int zref_get_state(const zref_scene* s, double* y, double* ydot, double* kappa, int32_t* step) {
  if (y) std::copy(s->y.begin(), s->y.end(), y);
  if (ydot) std::copy(s->ydot.begin(), s->ydot.end(), ydot);
  if (kappa) *kappa = s->kappa;
  if (step) *step = s->step;
  return 0;
}

int zref_set_kappa(zref_scene* s, double kappa) {
  if (!(kappa > 0.0)) return -1;
  s->kappa = kappa;
  return 0;
}

int zref_surface_positions(const zref_scene* s, const double* y, double* xs) {
  surface_positions(s, y, xs);
  return 0;
}

int zref_candidates(zref_scene* s, const double* xs0, const double* xs1, double r, int32_t* pt,
                    int64_t pt_cap, int64_t* n_pt, int32_t* ee, int64_t ee_cap, int64_t* n_ee) {
  candidates(s, xs0, xs1 ? xs1 : xs0, r, s->pt, s->ee);
  *n_pt = (int64_t)s->pt.size();
  *n_ee = (int64_t)s->ee.size();
  if (*n_pt > pt_cap || *n_ee > ee_cap) return fail(s, -4, "candidate capacity");
  for (size_t k = 0; k < s->pt.size(); ++k) {
    pt[2 * k] = s->pt[k].a;
    pt[2 * k + 1] = s->pt[k].b;
  }
  for (size_t k = 0; k < s->ee.size(); ++k) {
    ee[2 * k] = s->ee[k].a;
    ee[2 * k + 1] = s->ee[k].b;
  }
  return 0;
}

int zref_ip_assemble(zref_scene* s, const double* y, uint32_t flags, double* terms, double* grad) {
  candidates_static(s, y);
  std::vector<double> g;
  unsigned mask = (flags >> 8) & 0x3f;
  EvalOut o = evaluate(s, y, (flags & 1) ? &g : nullptr, (flags & 2) != 0, mask ? mask : 0x3f);
  std::copy(o.terms, o.terms + 8, terms);
  if ((flags & 1) && grad) std::copy(g.begin(), g.end(), grad);
  if (!o.feasible) return fail(s, -3, "infeasible state (inverted tet or zero distance)");
  return 0;
}

int zref_hessian_matvec(zref_scene* s, const double* v, double* out) {
  hess_matvec(s, v, out);
  return 0;
}

int zref_pcg_solve(zref_scene* s, const double* rhs, double* sol, double rtol, int32_t max_iter,
                   int32_t* iters, double* rel_res) {
  return pcg(s, rhs, sol, rtol, max_iter, iters, rel_res);
}

int zref_ccd_max_step(zref_scene* s, const double* y, const double* p, double* alpha) {
  candidates_swept(s, y, p);
  return ccd_bound(s, y, p, alpha);
}

int zref_friction_count(const zref_scene* s, int64_t* n) {
  *n = (int64_t)s->fric.size();
  return 0;
}

int zref_friction_table(const zref_scene* s, int32_t* ids5, double* vals8) {
  for (size_t k = 0; k < s->fric.size(); ++k) {
    const Fric& f = s->fric[k];
    ids5[5 * k] = f.kind;
    for (int a = 0; a < 4; ++a) ids5[5 * k + 1 + a] = f.v[a];
    vals8[8 * k] = f.lam;
    for (int a = 0; a < 3; ++a) vals8[8 * k + 1 + a] = f.n[a];
    for (int a = 0; a < 4; ++a) vals8[8 * k + 4 + a] = f.w[a];
  }
  return 0;
}

int zref_step(zref_scene* s, int32_t n_steps, zref_step_stats* stats) {
  for (int k = 0; k < n_steps; ++k) {
    int rc = time_step(s, &stats[k]);
    stats[k].status = rc;
    if (rc) return rc;
  }
  return 0;
}

int zref_record(zref_scene* s, int32_t enable) {
  s->record = enable != 0;
  s->recs.clear();
  return 0;
}

int zref_record_count(const zref_scene* s, int64_t* n) {
  *n = (int64_t)s->recs.size();
  return 0;
}

int zref_record_get(const zref_scene* s, int64_t k, int32_t* step, double* kappa_lag, double* kappa,
                    double* y_t, double* ydot_t, double* y_k) {
  if (k < 0 || k >= (int64_t)s->recs.size()) return -1;
  const Rec& r = s->recs[k];
  *step = r.step;
  *kappa_lag = r.kappa_lag;
  *kappa = r.kappa;
  std::copy(r.yt.begin(), r.yt.end(), y_t);
  std::copy(r.ydt.begin(), r.ydt.end(), ydot_t);
  std::copy(r.yk.begin(), r.yk.end(), y_k);
  return 0;
}

double zref_dist_pt(const double* x12, int32_t* type) {
  int t;
  double d2 = pt_type_d2(x12, &t, nullptr);
  if (type) *type = t;
  return std::sqrt(d2);
}

double zref_dist_ee(const double* x12, int32_t* type) {
  int t;
  double d2 = ee_type_d2(x12, &t, nullptr);
  if (type) *type = t;
  return std::sqrt(d2);
}

int zref_barrier(double d, double dhat, double* b3) {
  barrier3(d, dhat, b3);
  return 0;
}

int zref_pair_energy(zref_scene* s, int32_t kind, const double* x12, const double* rest_len2,
                     double* e, double* g12, double* h144, int32_t project) {
  return zref_pair_energy_typed(s, kind, x12, rest_len2, -1, e, g12, h144, project);
}

int zref_pair_energy_typed(zref_scene* s, int32_t kind, const double* x12, const double* rest_len2, int32_t type,
                           double* e, double* g12, double* h144, int32_t project) {
  if (type > (kind == 0 ? 6 : 8)) return -1;
  double eps = kind == 1 ? 1e-3 * rest_len2[0] * rest_len2[1] : 0.0;
  J2<12> E;
  double d;
  pair_energy_jet(s, kind, x12, eps, s->kappa, E, &d, type);
  *e = E.v;
  for (int i = 0; i < 12; ++i) g12[i] = E.g[i];
  std::vector<double> Hx(144);
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < 12; ++j) Hx[i * 12 + j] = E.h[i][j];
  if (project) Hx = project_psd(12, Hx);
  std::copy(Hx.begin(), Hx.end(), h144);
  return 0;
}

int zref_tet_energy(zref_scene* s, int32_t tet, const double* x12, double* e, double* g12, double* h144,
                    int32_t project) {
  if (tet < 0 || tet >= (int)s->vol.size()) return -1;
  return tet_term(s, tet, x12, e, g12, h144, project != 0) ? 0 : -2;
}

int zref_accd_pair(int32_t kind, const double* x12, const double* p12, double s, double* toi) {
  return accd(kind, x12, p12, s, toi) ? 0 : -3;
}

int zref_project_psd(int32_t n, const double* a, double* out) {
  std::vector<double> A(a, a + n * n);
  std::vector<double> P = project_psd(n, A);
  std::copy(P.begin(), P.end(), out);
  return 0;
}

}  // extern "C"

// Inputs and output of the learned initial guess of a time step (an extension of the
// method's explicit-velocity start y^t + h ydot^t, Sec. III).
//
// Features of soft vertex i at the step start, in units of s = h * 0.05 m/s where
// they are displacements:
//   0-2   h v_i / s
//   3-5   h (v_i - v_i^prev) / s                     (velocity change of the last step)
//   6     min(d_i, 4 dhat) / dhat                    d_i: distance to the nearest
//                                                    triangle of another body
//   7-9   unit vector to the closest point of that triangle (0 if none within 4 dhat)
//   10-12 h (velocity of that closest point) / s
//   13-15 h (kinematic target velocity - velocity) / s of the driven body owning the
//         triangle (0 for other bodies)
// Output of the network: the correction of h v_i in units of s; the proposal is
// x_i^t + h v_i + s * out_i for soft vertices and q^t + h qdot for affine bodies.
#include "geom.hpp"
#include "mlp.hpp"
#include "scene.hpp"

namespace zema {

constexpr double kFeatSpeed = 0.05;  // m/s: the displacement unit is h times this speed
constexpr int kNoPair = 0x7f7f7f7f;  // fill pattern of the pick array: no triangle in range

__global__ void feat_min_kernel(int npt, const int* __restrict__ pt, const int* __restrict__ tris,
                                const int* __restrict__ sv_ref, const double* __restrict__ xs,
                                unsigned long long* __restrict__ dmin) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npt) return;
  int v = pt[2 * k], t = pt[2 * k + 1];
  if (sv_ref[v] < 0) return;
  V3 x[4] = {ld3(xs + 3 * v), ld3(xs + 3 * tris[3 * t]), ld3(xs + 3 * tris[3 * t + 1]), ld3(xs + 3 * tris[3 * t + 2])};
  double d = pair_dist(0, x, nullptr);
  atomicMin(dmin + v, dbits(d));
}

__global__ void feat_pick_kernel(int npt, const int* __restrict__ pt, const int* __restrict__ tris,
                                 const int* __restrict__ sv_ref, const double* __restrict__ xs,
                                 const unsigned long long* __restrict__ dmin, int* __restrict__ pick) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npt) return;
  int v = pt[2 * k], t = pt[2 * k + 1];
  if (sv_ref[v] < 0) return;
  V3 x[4] = {ld3(xs + 3 * v), ld3(xs + 3 * tris[3 * t]), ld3(xs + 3 * tris[3 * t + 1]), ld3(xs + 3 * tris[3 * t + 2])};
  if (dbits(pair_dist(0, x, nullptr)) == dmin[v]) atomicMin(pick + v, k);
}

__global__ void feat_kernel(int nsv, const int* __restrict__ soft_sv, const int* __restrict__ pick,
                            const int* __restrict__ pt, const int* __restrict__ tris, const int* __restrict__ sv_ref,
                            const double* __restrict__ xs, const double* __restrict__ vs,
                            const double* __restrict__ ydot, const double* __restrict__ yprev,
                            const int* __restrict__ bi, const double* __restrict__ body_tv, double h, double dhat,
                            float* __restrict__ feat) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsv) return;
  const double inv = h / (h * kFeatSpeed);  // h / s
  double f[16];
  V3 v = ld3(ydot + 3 * i), vp = ld3(yprev + 3 * i);
  f[0] = inv * v.x;
  f[1] = inv * v.y;
  f[2] = inv * v.z;
  f[3] = inv * (v.x - vp.x);
  f[4] = inv * (v.y - vp.y);
  f[5] = inv * (v.z - vp.z);
  f[6] = 4.0;
  for (int k = 7; k < 16; ++k) f[k] = 0.0;
  int sv = soft_sv[i];
  int k = sv >= 0 ? pick[sv] : kNoPair;
  if (k != kNoPair) {
    int t = pt[2 * k + 1];
    int a = tris[3 * t], b = tris[3 * t + 1], c = tris[3 * t + 2];
    V3 x[4] = {ld3(xs + 3 * sv), ld3(xs + 3 * a), ld3(xs + 3 * b), ld3(xs + 3 * c)};
    double w[3];
    pt_closest_bary(x, w);
    V3 cp = w[0] * x[1] + w[1] * x[2] + w[2] * x[3];
    V3 dv = cp - x[0];
    double d = sqrt(dot(dv, dv));
    if (d < 4.0 * dhat) {
      f[6] = d / dhat;
      if (d > 0.0) {
        f[7] = dv.x / d;
        f[8] = dv.y / d;
        f[9] = dv.z / d;
      }
      V3 vc = w[0] * ld3(vs + 3 * a) + w[1] * ld3(vs + 3 * b) + w[2] * ld3(vs + 3 * c);
      f[10] = inv * vc.x;
      f[11] = inv * vc.y;
      f[12] = inv * vc.z;
      int r = sv_ref[a];
      if (r < 0) {
        int body = -r - 1;
        if (bi[4 * body] == ZEMA_DRIVEN) {
          V3 pd = ld3(ydot + bi[4 * body + 1]);
          V3 tv = ld3(body_tv + 3 * body);
          f[13] = inv * (tv.x - pd.x);
          f[14] = inv * (tv.y - pd.y);
          f[15] = inv * (tv.z - pd.z);
        }
      }
    }
  }
  for (int q = 0; q < 16; ++q) feat[16 * (size_t)i + q] = (float)f[q];
}

// p = h ydot on every DOF, plus s * out_i on soft vertex i
__global__ void warm_dir_kernel(int nsv, int ndof, double h, const double* __restrict__ ydot,
                                const float* __restrict__ out, double* __restrict__ p) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ndof) return;
  double v = h * ydot[j];
  if (j < 3 * nsv) v += h * kFeatSpeed * (double)out[j];
  p[j] = v;
}

// target of the network for the step just taken: ((x^{t+1} - x^t) - h v^t) / s
__global__ void warm_target_kernel(int n3, double h, const double* __restrict__ y, const double* __restrict__ yt,
                                   const double* __restrict__ ydt, float* __restrict__ target) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n3) return;
  target[j] = (float)(((y[j] - yt[j]) - h * ydt[j]) / (h * kFeatSpeed));
}

void k_features(zema_scene* s, float* feat) {
  if (!s->nsv) return;
  k_map_surface(s, s->y.p, s->xs.p);
  k_candidates(s, s->xs.p, s->xs.p, 4.0 * s->P.dhat);
  k_surface_disp(s, s->ydot.p, s->dxs.p);
  s->fdmin.reserve(s->nsurf + 1);
  s->fpick.reserve(s->nsurf + 1);
  ZCHK(hipMemsetAsync(s->fdmin.p, 0xff, sizeof(unsigned long long) * (s->nsurf + 1), s->st));
  ZCHK(hipMemsetAsync(s->fpick.p, 0x7f, sizeof(int) * (s->nsurf + 1), s->st));  // kNoPair
  int npt = (int)s->npt;
  if (npt) {
    feat_min_kernel<<<nblocks(npt), kBlock, 0, s->st>>>(npt, s->pt.p, s->tris.p, s->sv_ref.p, s->xs.p, s->fdmin.p);
    feat_pick_kernel<<<nblocks(npt), kBlock, 0, s->st>>>(npt, s->pt.p, s->tris.p, s->sv_ref.p, s->xs.p, s->fdmin.p,
                                                         s->fpick.p);
  }
  feat_kernel<<<nblocks(s->nsv), kBlock, 0, s->st>>>(s->nsv, s->soft_sv.p, s->fpick.p, s->pt.p, s->tris.p,
                                                     s->sv_ref.p, s->xs.p, s->dxs.p, s->ydot.p, s->yd_prev.p,
                                                     s->body_i.p, s->body_tv.p, s->P.dt, s->P.dhat, feat);
}

// Fit of the network's correction field over each soft body (mass-weighted least
// squares): c_i ~ cbar + A (x_i - xbar), with A = 0 when only the mean is kept or the
// body's second moment is singular.  One workgroup per body; the sums are taken about
// the body's first vertex, per thread in a fixed stride and then over a fixed tree, so
// the fit is bitwise repeatable.
constexpr int kFitThreads = 256;
constexpr int kFitSums = 22;  // m, m dx (3), m c (3), m dx dx^T (6), m c dx^T (9)

__global__ void __launch_bounds__(kFitThreads)
    warm_fit_kernel(const int* __restrict__ vr, const double* __restrict__ y, const double* __restrict__ mass,
                    const float* __restrict__ out, int affine, double* __restrict__ fit) {
  __shared__ double sh[kFitSums][kFitThreads];
  const int b = blockIdx.x, t = threadIdx.x;
  const int v0 = vr[b], v1 = vr[b + 1];
  double a[kFitSums];
#pragma unroll
  for (int q = 0; q < kFitSums; ++q) a[q] = 0.0;
  if (v1 > v0) {
    const V3 x0 = ld3(y + 3 * (size_t)v0);
    for (int i = v0 + t; i < v1; i += kFitThreads) {
      const double m = mass[i];
      const V3 xi = ld3(y + 3 * (size_t)i);
      const double d[3] = {xi.x - x0.x, xi.y - x0.y, xi.z - x0.z};
      const double c[3] = {(double)out[3 * (size_t)i], (double)out[3 * (size_t)i + 1], (double)out[3 * (size_t)i + 2]};
      a[0] += m;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        a[1 + k] += m * d[k];
        a[4 + k] += m * c[k];
      }
      a[7] += m * d[0] * d[0];
      a[8] += m * d[0] * d[1];
      a[9] += m * d[0] * d[2];
      a[10] += m * d[1] * d[1];
      a[11] += m * d[1] * d[2];
      a[12] += m * d[2] * d[2];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) a[13 + 3 * r + k] += m * c[r] * d[k];
    }
  }
#pragma unroll
  for (int q = 0; q < kFitSums; ++q) sh[q][t] = a[q];
  __syncthreads();
  for (int w = kFitThreads / 2; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int q = 0; q < kFitSums; ++q) sh[q][t] += sh[q][t + w];
    __syncthreads();
  }
  if (t != 0) return;
  double* f = fit + 15 * (size_t)b;
  for (int q = 0; q < 15; ++q) f[q] = 0.0;
  const double M = sh[0][0];
  if (v1 <= v0 || !(M > 0.0)) return;
  const V3 x0 = ld3(y + 3 * (size_t)v0);
  double xb[3], cb[3];
  for (int k = 0; k < 3; ++k) {
    xb[k] = sh[1 + k][0] / M;
    cb[k] = sh[4 + k][0] / M;
  }
  f[0] = cb[0];
  f[1] = cb[1];
  f[2] = cb[2];
  f[3] = x0.x + xb[0];
  f[4] = x0.y + xb[1];
  f[5] = x0.z + xb[2];
  if (!affine) return;
  // centred second moment S and cross moment C = sum m (c - cbar)(x - xbar)^T
  const int si[3][3] = {{7, 8, 9}, {8, 10, 11}, {9, 11, 12}};
  double S[3][3], C[3][3];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      S[r][k] = sh[si[r][k]][0] - M * xb[r] * xb[k];
      C[r][k] = sh[13 + 3 * r + k][0] - M * cb[r] * xb[k];
    }
  // S^-1 by cofactors; a body whose vertices are (nearly) coplanar keeps the mean only
  double co[3][3];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      const int r1 = (r + 1) % 3, r2 = (r + 2) % 3, k1 = (k + 1) % 3, k2 = (k + 2) % 3;
      co[r][k] = S[r1][k1] * S[r2][k2] - S[r1][k2] * S[r2][k1];
    }
  const double det = S[0][0] * co[0][0] + S[0][1] * co[0][1] + S[0][2] * co[0][2];
  const double tr = S[0][0] + S[1][1] + S[2][2];
  if (!(det > 1e-9 * tr * tr * tr)) return;
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k)  // (C S^-1)[r][k] = sum_j C[r][j] co[k][j] / det (S symmetric)
      f[6 + 3 * r + k] = (C[r][0] * co[k][0] + C[r][1] * co[k][1] + C[r][2] * co[k][2]) / det;
}

__global__ void warm_fit_apply_kernel(int nsv, const int* __restrict__ vbody, const double* __restrict__ y,
                                      const double* __restrict__ fit, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsv) return;
  const double* f = fit + 15 * (size_t)vbody[i];
  const V3 x = ld3(y + 3 * (size_t)i);
  const double d[3] = {x.x - f[3], x.y - f[4], x.z - f[5]};
#pragma unroll
  for (int r = 0; r < 3; ++r)
    out[3 * (size_t)i + r] = (float)(f[r] + f[6 + 3 * r] * d[0] + f[7 + 3 * r] * d[1] + f[8 + 3 * r] * d[2]);
}

void k_warm_fit(zema_scene* s, int mode, float* out) {
  if (mode && s->nsv && s->n_soft_bodies) {
    s->wfit.reserve(15 * (size_t)s->n_soft_bodies);
    warm_fit_kernel<<<s->n_soft_bodies, kFitThreads, 0, s->st>>>(s->soft_vr.p, s->y.p, s->mass.p, out, mode == 1,
                                                                s->wfit.p);
    warm_fit_apply_kernel<<<nblocks(s->nsv), kBlock, 0, s->st>>>(s->nsv, s->v_sbody.p, s->y.p, s->wfit.p, out);
  }
}

void k_warm_dir(zema_scene* s, float* out, double* p) {
  k_warm_fit(s, s->warm_fit, out);
  if (s->ndof)
    warm_dir_kernel<<<nblocks(s->ndof), kBlock, 0, s->st>>>(s->nsv, s->ndof, s->P.dt, s->ydot.p, out, p);
}

void k_warm_target(zema_scene* s, float* target) {
  int n3 = 3 * s->nsv;
  if (n3) warm_target_kernel<<<nblocks(n3), kBlock, 0, s->st>>>(n3, s->P.dt, s->y.p, s->yt.p, s->ydt.p, target);
}

}  // namespace zema

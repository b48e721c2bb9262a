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

void k_warm_dir(zema_scene* s, const float* out, double* p) {
  if (s->ndof)
    warm_dir_kernel<<<nblocks(s->ndof), kBlock, 0, s->st>>>(s->nsv, s->ndof, s->P.dt, s->ydot.p, out, p);
}

void k_warm_target(zema_scene* s, float* target) {
  int n3 = 3 * s->nsv;
  if (n3) warm_target_kernel<<<nblocks(n3), kBlock, 0, s->st>>>(n3, s->P.dt, s->y.p, s->yt.p, s->ydt.p, target);
}

}  // namespace zema

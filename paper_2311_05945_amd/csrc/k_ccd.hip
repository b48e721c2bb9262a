// Step bound of the intersection-free line search: additive CCD (Li, Kaufman,
// Jiang 2021, "Codimensional Incremental Potential Contact", Alg. 1) with zero
// thickness and t_c = 1, one candidate pair per lane.  Affine vertices move
// linearly in the step size because x = A x0 + p is linear in q, so linear CCD is
// exact for them too.  The global bound is min(1, min_k t_k).
#include <cstring>
#include <vector>

#include "geom.hpp"
#include "scene.hpp"

namespace zema {

__global__ void accd_kernel(int npt, int nee, const int* __restrict__ pt, const int* __restrict__ ee,
                            const int* __restrict__ tris, const int* __restrict__ edges, const double* __restrict__ xs,
                            const double* __restrict__ dx, double s_sep, const int* __restrict__ sv_scene,
                            unsigned long long* __restrict__ tmin, int* __restrict__ bad) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  double t = 1.0;
  int sc = -1;
  if (k < npt + nee) {
    int kind, sv[4];
    if (k < npt) {
      kind = 0;
      int v = pt[2 * k], tr = pt[2 * k + 1];
      sv[0] = v;
      sv[1] = tris[3 * tr];
      sv[2] = tris[3 * tr + 1];
      sv[3] = tris[3 * tr + 2];
    } else {
      kind = 1;
      int j = k - npt, ea = ee[2 * j], eb = ee[2 * j + 1];
      sv[0] = edges[2 * ea];
      sv[1] = edges[2 * ea + 1];
      sv[2] = edges[2 * eb];
      sv[3] = edges[2 * eb + 1];
    }
    sc = sv_scene[sv[0]];
    V3 x[4], p[4];
    for (int a = 0; a < 4; ++a) {
      x[a] = ld3(xs + 3 * sv[a]);
      p[a] = ld3(dx + 3 * sv[a]);
    }
    V3 mean = 0.25 * (p[0] + p[1] + p[2] + p[3]);
    double n[4];
    for (int a = 0; a < 4; ++a) {
      p[a] = p[a] - mean;
      n[a] = sqrt(dot(p[a], p[a]));
    }
    double lp = kind == 0 ? n[0] + fmax(n[1], fmax(n[2], n[3])) : fmax(n[0], n[1]) + fmax(n[2], n[3]);
    if (lp > 0.0) {
      double d = pair_dist(kind, x, nullptr);
      if (!(d > 0.0)) {
        atomicAdd(bad, 1);
        t = 0.0;
      } else {
        double g = s_sep * d, tl = (1.0 - s_sep) * d / lp;
        t = 0.0;
        bool capped = false;
        for (int it = 0; it < 10000; ++it) {
          for (int a = 0; a < 4; ++a) x[a] = x[a] + tl * p[a];
          d = pair_dist(kind, x, nullptr);
          if (t > 0.0 && d < g) break;
          t += tl;
          if (t > 1.0) {
            capped = true;
            break;
          }
          tl = (1.0 - s_sep) * d / lp;
        }
        if (capped) t = 1.0;
      }
    }
  }
  scene_atomic_ext<false>(tmin, sc, t);
}

// per scene: alpha_max over the current candidate set for the move y -> y + p
// (alpha [ns], host); a pair already at zero distance fails the call
int k_ccd(zema_scene* s, const double* y, const double* p, double* alpha) {
  k_map_surface(s, y, s->xs.p);
  k_surface_disp(s, p, s->dxs.p);
  int n = (int)(s->npt + s->nee);
  ZCHK(hipMemsetAsync(s->sc_tmin.p, 0xff, sizeof(unsigned long long) * s->ns, s->st));  // no pair: 1
  int* bad = s->counters.p + 5;
  ZCHK(hipMemsetAsync(bad, 0, sizeof(int), s->st));
  if (n) {
    kt_begin(s, KT_CCD);
    accd_kernel<<<nblocks(n), kBlock, 0, s->st>>>((int)s->npt, (int)s->nee, s->pt.p, s->ee.p, s->tris.p, s->edges.p,
                                                  s->xs.p, s->dxs.p, s->P.ccd_s, s->sv_scene.p, s->sc_tmin.p, bad);
    kt_end(s, KT_CCD);
  }
  std::vector<unsigned long long> u(s->ns);
  int b;
  ZCHK(hipMemcpyAsync(u.data(), s->sc_tmin.p, sizeof(unsigned long long) * s->ns, hipMemcpyDeviceToHost, s->st));
  ZCHK(hipMemcpyAsync(&b, bad, sizeof(b), hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
  for (int k = 0; k < s->ns; ++k) {
    double t = 1.0;
    if (u[k] != ~0ull) std::memcpy(&t, &u[k], sizeof(t));
    alpha[k] = t < 1.0 ? t : 1.0;
  }
  return b ? ZEMA_E_INTERSECT : 0;
}

}  // namespace zema

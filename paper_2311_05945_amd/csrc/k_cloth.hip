// Garment triangles (Sec. IV-D, Baraff-Witkin membrane): stretch and shear of each
// triangle from its deformation columns w_u, w_v (x = W (u, v)^T + const over the
// triangle, (u, v) the rest material coordinates), in incremental-potential units
//   h^2 A (k_s/2 ((|w_u| - 1)^2 + (|w_v| - 1)^2) + k_sh/2 (w_u . w_v)^2),
// A the rest area.  The Hessian takes each part's PSD projection in the six
// coordinates of (w_u, w_v), both in closed form:
//   stretch, per column w: k_s (w^ w^T + max(0, 1 - 1/|w|) (I - w^ w^T));
//   shear, with s = (w_u + w_v)/2, t = (w_u - w_v)/2, C = w_u . w_v = |s|^2 - |t|^2 and
//   g = (w_v, w_u) = g+ + g-, g+ = (s, s), g- = (-t, t): the unprojected k_sh (g g^T +
//   C [[0, I], [I, 0]]) has eigenvalue C on the (e, e) directions orthogonal to g+,
//   -C on the (e, -e) directions orthogonal to g-, and on span(g+, g-) the 2x2 matrix
//   [[|g+|^2 + C, |g+| |g-|], [|g+| |g-|, |g-|^2 - C]];
// the sum is mapped to the three vertices (W is linear in x).  The element terms enter
// the contact triplet stream (elastic mask bit), one thread per triangle.
#include "scene.hpp"

namespace zema {

struct ClothArgs {
  int n;
  const int4* v;      // vertices (soft vertex ids), w unused
  const double* d;    // [8]: inverse rest edge matrix m00 m01 m10 m11, area, k_s, k_sh, pad
  const double* y;
  double h2;
};

struct ClothGeo {
  double cu[3], cv[3];  // dW/dx per vertex
  double wu[3], wv[3];
  double h2A, ks, ksh;
};

__device__ inline ClothGeo cloth_geo(const ClothArgs& C, int c) {
  ClothGeo G;
  const double* d = C.d + 8 * (size_t)c;
  const int4 t = C.v[c];
  const int vid[3] = {t.x, t.y, t.z};
  G.cu[0] = -(d[0] + d[2]);
  G.cu[1] = d[0];
  G.cu[2] = d[2];
  G.cv[0] = -(d[1] + d[3]);
  G.cv[1] = d[1];
  G.cv[2] = d[3];
  for (int k = 0; k < 3; ++k) {
    G.wu[k] = 0.0;
    G.wv[k] = 0.0;
  }
  for (int a = 0; a < 3; ++a) {
    const double* x = C.y + 3 * (size_t)vid[a];
    for (int k = 0; k < 3; ++k) {
      G.wu[k] += G.cu[a] * x[k];
      G.wv[k] += G.cv[a] * x[k];
    }
  }
  G.h2A = C.h2 * d[4];
  G.ks = d[5];
  G.ksh = d[6];
  return G;
}

__global__ void cloth_energy_kernel(ClothArgs C, double* __restrict__ e_out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.n) return;
  const ClothGeo G = cloth_geo(C, c);
  const double nu = sqrt(G.wu[0] * G.wu[0] + G.wu[1] * G.wu[1] + G.wu[2] * G.wu[2]);
  const double nv = sqrt(G.wv[0] * G.wv[0] + G.wv[1] * G.wv[1] + G.wv[2] * G.wv[2]);
  const double cs = G.wu[0] * G.wv[0] + G.wu[1] * G.wv[1] + G.wu[2] * G.wv[2];
  e_out[c] = G.h2A * (0.5 * G.ks * ((nu - 1.0) * (nu - 1.0) + (nv - 1.0) * (nv - 1.0)) + 0.5 * G.ksh * cs * cs);
}

// H += lam u u^T on the 6x6 (upper triangle and diagonal kept full)
__device__ inline void rank1(double H[6][6], double lam, const double u[6]) {
  if (!(lam > 0.0)) return;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) H[i][j] += lam * u[i] * u[j];
}

__global__ void cloth_emit_kernel(ClothArgs C, int hess, int64_t base, unsigned long long W, int nn_total,
                                  unsigned long long* __restrict__ key, double* __restrict__ val) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.n) return;
  const ClothGeo G = cloth_geo(C, c);
  const int4 t = C.v[c];
  const int vid[3] = {t.x, t.y, t.z};
  const double nu = sqrt(G.wu[0] * G.wu[0] + G.wu[1] * G.wu[1] + G.wu[2] * G.wu[2]);
  const double nv = sqrt(G.wv[0] * G.wv[0] + G.wv[1] * G.wv[1] + G.wv[2] * G.wv[2]);
  const double cs = G.wu[0] * G.wv[0] + G.wu[1] * G.wv[1] + G.wu[2] * G.wv[2];
  double hu[3], hv[3];  // unit columns (0 for a collapsed column)
  for (int k = 0; k < 3; ++k) {
    hu[k] = nu > 0.0 ? G.wu[k] / nu : 0.0;
    hv[k] = nv > 0.0 ? G.wv[k] / nv : 0.0;
  }
  // gradient in W: (dE/dw_u, dE/dw_v)
  double gW[6];
  for (int k = 0; k < 3; ++k) {
    gW[k] = G.h2A * (G.ks * (nu - 1.0) * hu[k] + G.ksh * cs * G.wv[k]);
    gW[3 + k] = G.h2A * (G.ks * (nv - 1.0) * hv[k] + G.ksh * cs * G.wu[k]);
  }
  const double* col[2] = {G.cu, G.cv};
  int64_t o = base + (int64_t)c * (hess ? 12 : 3);
  for (int a = 0; a < 3; ++a, ++o) {
    key[o] = (unsigned long long)vid[a] * W + (unsigned long long)nn_total;
    for (int k = 0; k < 3; ++k) val[(size_t)9 * o + k] = col[0][a] * gW[k] + col[1][a] * gW[3 + k];
    for (int k = 3; k < 9; ++k) val[(size_t)9 * o + k] = 0.0;
  }
  if (!hess) return;
  double H[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) H[i][j] = 0.0;
  // stretch: per column k_s (w^ w^T + max(0, 1 - 1/|w|) (I - w^ w^T))
  const double lu = nu > 0.0 ? fmax(0.0, 1.0 - 1.0 / nu) : 0.0, lv = nv > 0.0 ? fmax(0.0, 1.0 - 1.0 / nv) : 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double id = i == j ? 1.0 : 0.0;
      H[i][j] += G.ks * (hu[i] * hu[j] + lu * (id - hu[i] * hu[j]));
      H[3 + i][3 + j] += G.ks * (hv[i] * hv[j] + lv * (id - hv[i] * hv[j]));
    }
  // shear (closed-form eigensystem, see the header)
  double sv[3], tv[3];
  for (int k = 0; k < 3; ++k) {
    sv[k] = 0.5 * (G.wu[k] + G.wv[k]);
    tv[k] = 0.5 * (G.wu[k] - G.wv[k]);
  }
  const double ns = sqrt(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2]);
  const double nt = sqrt(tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2]);
  const double gp = 1.41421356237309515 * ns, gm = 1.41421356237309515 * nt;  // |g+|, |g-|
  double up[6], um[6];  // unit g+ = (s, s)/|g+|, unit g- = (-t, t)/|g-| (0 when zero)
  for (int k = 0; k < 3; ++k) {
    up[k] = up[3 + k] = ns > 0.0 ? sv[k] / gp : 0.0;
    um[k] = nt > 0.0 ? -tv[k] / gm : 0.0;
    um[3 + k] = -um[k];
  }
  // max(C, 0) (Pi+ - up up^T) + max(-C, 0) (Pi- - um um^T)
  const double cp = fmax(cs, 0.0), cm = fmax(-cs, 0.0);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      const bool same = (i % 3) == (j % 3);
      const double pip = same ? 0.5 : 0.0;                              // Pi+ entry
      const double pim = same ? ((i < 3) == (j < 3) ? 0.5 : -0.5) : 0.0;  // Pi- entry
      H[i][j] += G.ksh * (cp * (pip - up[i] * up[j]) + cm * (pim - um[i] * um[j]));
    }
  // the 2x2 block on span(g+, g-)
  const double p = gp * gp + cs, q = gm * gm - cs, r = gp * gm;
  const double th = 0.5 * atan2(2.0 * r, p - q);
  const double co = cos(th), si = sin(th);
  const double l1 = p * co * co + 2.0 * r * co * si + q * si * si;
  const double l2 = p * si * si - 2.0 * r * co * si + q * co * co;
  double e1[6], e2[6];
  for (int i = 0; i < 6; ++i) {
    e1[i] = co * up[i] + si * um[i];
    e2[i] = -si * up[i] + co * um[i];
  }
  double Hs[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) Hs[i][j] = 0.0;
  rank1(Hs, l1, e1);
  rank1(Hs, l2, e2);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) H[i][j] = G.h2A * (H[i][j] + G.ksh * Hs[i][j]);
  // vertex blocks: sum over the column pairs of c_p[a] c_q[b] H_pq
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b, ++o) {
      key[o] = (unsigned long long)vid[a] * W + (unsigned long long)vid[b];
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double acc = 0.0;
          for (int pp = 0; pp < 2; ++pp)
            for (int qq = 0; qq < 2; ++qq) acc += col[pp][a] * col[qq][b] * H[3 * pp + k][3 * qq + l];
          val[(size_t)9 * o + 3 * k + l] = acc;
        }
    }
}

static ClothArgs cloth_args(zema_scene* s, const double* y) {
  ClothArgs C;
  C.n = s->ncl;
  C.v = s->cl_v.p;
  C.d = s->cl_d.p;
  C.y = y;
  C.h2 = s->P.dt * s->P.dt;
  return C;
}

void k_cloth_energy(zema_scene* s, const double* y, double* e_out) {
  if (s->ncl) cloth_energy_kernel<<<nblocks(s->ncl), kBlock, 0, s->st>>>(cloth_args(s, y), e_out);
}

void k_cloth_emit(zema_scene* s, const double* y, bool hess, int64_t base, unsigned long long W,
                  unsigned long long* key, double* val) {
  if (s->ncl)
    cloth_emit_kernel<<<nblocks(s->ncl), kBlock, 0, s->st>>>(cloth_args(s, y), hess ? 1 : 0, base, W, s->nnodes,
                                                             key, val);
}

}  // namespace zema

// Intersection count (validation of the intersection-free guarantee of Sec. III):
// inter-body (edge, triangle) pairs whose closed segment and closed triangle
// intersect, and tets with non-positive volume.  Orientation signs are computed in
// FP64 with a static error bound (Shewchuk 1997, orient3d: |det| > (7 + 56 eps) eps
// times the permanent); a sign the bound cannot certify makes the pair "uncertain"
// and it is listed for an exact check by the caller.
#include <algorithm>

#include "scene.hpp"

namespace zema {

// sign of det[a-d, b-d, c-d] (+1, -1, 0) or 2 when the filter cannot decide
__device__ inline int orient3d_f(V3 a, V3 b, V3 c, V3 d) {
  double adx = a.x - d.x, bdx = b.x - d.x, cdx = c.x - d.x;
  double ady = a.y - d.y, bdy = b.y - d.y, cdy = c.y - d.y;
  double adz = a.z - d.z, bdz = b.z - d.z, cdz = c.z - d.z;
  double bdxcdy = bdx * cdy, cdxbdy = cdx * bdy;
  double cdxady = cdx * ady, adxcdy = adx * cdy;
  double adxbdy = adx * bdy, bdxady = bdx * ady;
  double det = adz * (bdxcdy - cdxbdy) + bdz * (cdxady - adxcdy) + cdz * (adxbdy - bdxady);
  double perm = (fabs(bdxcdy) + fabs(cdxbdy)) * fabs(adz) + (fabs(cdxady) + fabs(adxcdy)) * fabs(bdz) +
                (fabs(adxbdy) + fabs(bdxady)) * fabs(cdz);
  const double eps = 1.1102230246251565e-16;  // 2^-53
  double bound = (7.0 + 56.0 * eps) * eps * perm;
  if (det > bound) return 1;
  if (-det > bound) return -1;
  if (perm == 0.0) return 0;  // exactly degenerate inputs
  return 2;
}

__global__ void seg_tri_kernel(int n, const int* __restrict__ pairs, const int* __restrict__ edges,
                               const int* __restrict__ tris, const double* __restrict__ xs,
                               unsigned long long* __restrict__ cnt, int* __restrict__ unc, int cap) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int e = pairs[2 * k], t = pairs[2 * k + 1];
  V3 p = ld3(xs + 3 * edges[2 * e]), q = ld3(xs + 3 * edges[2 * e + 1]);
  V3 a = ld3(xs + 3 * tris[3 * t]), b = ld3(xs + 3 * tris[3 * t + 1]), c = ld3(xs + 3 * tris[3 * t + 2]);
  int s1 = orient3d_f(a, b, c, p), s2 = orient3d_f(a, b, c, q);
  int verdict;  // 0 no, 1 yes, 2 uncertain
  if (s1 != 2 && s2 != 2 && s1 * s2 > 0) {
    verdict = 0;
  } else if (s1 == 2 || s2 == 2 || (s1 == 0 && s2 == 0)) {
    verdict = 2;  // undecided or coplanar
  } else {
    int t0 = orient3d_f(p, q, a, b), t1 = orient3d_f(p, q, b, c), t2 = orient3d_f(p, q, c, a);
    if (t0 == 2 || t1 == 2 || t2 == 2)
      verdict = 2;
    else
      verdict = ((t0 >= 0 && t1 >= 0 && t2 >= 0) || (t0 <= 0 && t1 <= 0 && t2 <= 0)) ? 1 : 0;
  }
  if (verdict == 1) atomicAdd(cnt, 1ull);
  if (verdict == 2) {
    unsigned long long u = atomicAdd(cnt + 1, 1ull);
    if ((int)u < cap) {
      unc[2 * u] = e;
      unc[2 * u + 1] = t;
    }
  }
}

__global__ void tet_sign_kernel(int nt, const int4* __restrict__ tets, const double* __restrict__ y,
                                unsigned long long* __restrict__ cnt) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt) return;
  int4 t = tets[e];
  // positive volume <=> x3 lies on the positive side of (x0, x1, x2)
  int s = orient3d_f(ld3(y + 3 * t.y), ld3(y + 3 * t.z), ld3(y + 3 * t.w), ld3(y + 3 * t.x));
  if (s == 2) atomicAdd(cnt + 3, 1ull);
  else if (s <= 0) atomicAdd(cnt + 2, 1ull);
}

void k_intersections(zema_scene* s, const double* y, int64_t* n_int, int64_t* n_inv, int64_t* n_unc,
                     DBuf<int>& unc) {
  k_map_surface(s, y, s->xs.p);
  int64_t np = k_edge_tri_pairs(s, s->xs.p, s->et_pairs);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(s->umin.p + 4);  // 4 counters
  ZCHK(hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned long long), s->st));
  int cap = (int)std::max<int64_t>(unc.cap / 2, 0);
  if (np) seg_tri_kernel<<<nblocks(np), kBlock, 0, s->st>>>((int)np, s->et_pairs.p, s->edges.p, s->tris.p, s->xs.p,
                                                            cnt, unc.p, cap);
  if (s->nt) tet_sign_kernel<<<nblocks(s->nt), kBlock, 0, s->st>>>(s->nt, s->tets.p, y, cnt);
  unsigned long long h[4];
  ZCHK(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
  *n_int = (int64_t)h[0];
  *n_unc = (int64_t)(h[1] + h[3]);
  *n_inv = (int64_t)h[2];
}

}  // namespace zema

// Vector kernels of the Newton step: affine vertex map (Sec. III eq. 2,
// x = A x0 + p), predictor (eq. 3), velocity update (text after eq. 11),
// convergence norm, deterministic multi-segment sums and inversion count.
#include <cstring>

#include "scene.hpp"

namespace zema {


__device__ inline const double* body_q(const double* y, const double* bf, const int* bi, int b) {
  int dof0 = bi[4 * b + 1];
  return dof0 >= 0 ? y + dof0 : bf + BF * b + BF_QF;
}

// ((a_k1 x0_1 + a_k2 x0_2) + a_k3 x0_3) + p_k, each operation rounded separately
__global__ void map_surface_kernel(int nsurf, const int* __restrict__ ref, const double* __restrict__ x0,
                                   const double* __restrict__ y, const double* __restrict__ bf,
                                   const int* __restrict__ bi, double* __restrict__ xs) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsurf) return;
  int r = ref[i];
  if (r >= 0) {
    xs[3 * i] = y[3 * r];
    xs[3 * i + 1] = y[3 * r + 1];
    xs[3 * i + 2] = y[3 * r + 2];
    return;
  }
  const double* q = body_q(y, bf, bi, -r - 1);
  double a = x0[3 * i], b = x0[3 * i + 1], c = x0[3 * i + 2];
  for (int k = 0; k < 3; ++k) {
    double s = __dmul_rn(q[3 + 3 * k], a);
    s = __dadd_rn(s, __dmul_rn(q[4 + 3 * k], b));
    s = __dadd_rn(s, __dmul_rn(q[5 + 3 * k], c));
    xs[3 * i + k] = __dadd_rn(s, q[k]);
  }
}

__global__ void surface_disp_kernel(int nsurf, const int* __restrict__ ref, const double* __restrict__ x0,
                                    const double* __restrict__ p, const int* __restrict__ bi,
                                    double* __restrict__ dx) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsurf) return;
  int r = ref[i];
  if (r >= 0) {
    dx[3 * i] = p[3 * r];
    dx[3 * i + 1] = p[3 * r + 1];
    dx[3 * i + 2] = p[3 * r + 2];
    return;
  }
  int dof0 = bi[4 * (-r - 1) + 1];
  if (dof0 < 0) {
    dx[3 * i] = dx[3 * i + 1] = dx[3 * i + 2] = 0.0;
    return;
  }
  const double* q = p + dof0;
  double a = x0[3 * i], b = x0[3 * i + 1], c = x0[3 * i + 2];
  for (int k = 0; k < 3; ++k) dx[3 * i + k] = q[3 + 3 * k] * a + q[4 + 3 * k] * b + q[5 + 3 * k] * c + q[k];
}

__global__ void axpy_kernel(int n, double a, const double* __restrict__ x, const double* __restrict__ y,
                            double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = y[i] + a * x[i];
}

__global__ void scale_kernel(int n, double a, const double* __restrict__ x, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i];
}

__global__ void iota_kernel(int64_t n, int* __restrict__ p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int)i;
}

__global__ void velocity_kernel(int n, double inv_h, const double* __restrict__ y, const double* __restrict__ yt,
                                double* __restrict__ v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (y[i] - yt[i]) * inv_h;
}

// xhat = x + h v + h^2 g; qhat = q + h qdot + h^2 (g, 0, 0, 0)
__global__ void predict_kernel(int nsoft3, int ndof, double h, double gx, double gy, double gz,
                               const double* __restrict__ y, const double* __restrict__ v, double* __restrict__ yhat) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndof) return;
  double g = 0.0;
  int k;
  if (i < nsoft3)
    k = i % 3;
  else
    k = (i - nsoft3) % 12;
  if (k < 3) g = k == 0 ? gx : (k == 1 ? gy : gz);
  yhat[i] = y[i] + h * v[i] + h * h * g;
}

// per scene: the largest vertex displacement |(J p)_i| over soft and affine vertices
__global__ void max_disp_kernel(int nsv, int nsurf, const int* __restrict__ ref, const double* __restrict__ x0,
                                const double* __restrict__ p, const int* __restrict__ bi,
                                const int* __restrict__ v_scene, const int* __restrict__ sv_scene,
                                unsigned long long* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  double m = 0.0;
  int sc = -1;
  if (i < nsv) {
    sc = v_scene[i];
    double a = p[3 * i], b = p[3 * i + 1], c = p[3 * i + 2];
    m = sqrt(a * a + b * b + c * c);
  } else if (i < nsv + nsurf) {
    int j = i - nsv;
    int r = ref[j];
    if (r < 0) {
      int dof0 = bi[4 * (-r - 1) + 1];
      sc = sv_scene[j];
      if (dof0 >= 0) {
        const double* q = p + dof0;
        double s2 = 0.0;
        for (int k = 0; k < 3; ++k) {
          double d = q[3 + 3 * k] * x0[3 * j] + q[4 + 3 * k] * x0[3 * j + 1] + q[5 + 3 * k] * x0[3 * j + 2] + q[k];
          s2 += d * d;
        }
        m = sqrt(s2);
      }
    }
  }
  scene_atomic_ext<true>(out, sc, m);
}

// out = y + alpha[scene] p, the scene of a DOF taken from its soft vertex or free body
__global__ void axpy_scene_kernel(int ndof, int nsv, const double* __restrict__ alpha, const int* __restrict__ v_scene,
                                  const int* __restrict__ f_scene, const double* __restrict__ p,
                                  const double* __restrict__ y, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndof) return;
  int sc = i < 3 * nsv ? v_scene[i / 3] : f_scene[(i - 3 * nsv) / 12];
  out[i] = y[i] + alpha[sc] * p[i];
}

// p *= alpha[scene] in place
__global__ void scale_scene_kernel(int ndof, int nsv, const double* __restrict__ alpha,
                                   const int* __restrict__ v_scene, const int* __restrict__ f_scene, double* p) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndof) return;
  int sc = i < 3 * nsv ? v_scene[i / 3] : f_scene[(i - 3 * nsv) / 12];
  p[i] *= alpha[sc];
}

// out = mask[scene] ? a : b per DOF
__global__ void select_scene_kernel(int ndof, int nsv, const int* __restrict__ mask, const int* __restrict__ v_scene,
                                    const int* __restrict__ f_scene, const double* __restrict__ a,
                                    const double* __restrict__ b, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndof) return;
  int sc = i < 3 * nsv ? v_scene[i / 3] : f_scene[(i - 3 * nsv) / 12];
  out[i] = mask[sc] ? a[i] : b[i];
}

constexpr int kSumGrid = 256;

struct SegTab {
  const double* p[8];
  int64_t n[8];
};

__global__ void sums_l1(SegTab tab, double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  int k = blockIdx.y;
  const double* a = tab.p[k];
  int64_t n = tab.n[k];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)kSumGrid * kBlock) acc += a[i];
  double r = block_sum<kBlock>(acc, sh);
  if (threadIdx.x == 0) part[k * kSumGrid + blockIdx.x] = r;
}

__global__ void sums_l2(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[kBlock / 64];
  int k = blockIdx.x;
  double r = block_sum<kBlock>(part[k * kSumGrid + threadIdx.x], sh);
  if (threadIdx.x == 0) out[k] = r;
}

// per scene: number of tets with non-positive volume at y
__global__ void inverted_kernel(int nt, const int4* __restrict__ tets, const double* __restrict__ y,
                                const int* __restrict__ v_scene, unsigned int* __restrict__ cnt) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nt) return;
  int4 t = tets[e];
  V3 x0 = ld3(y + 3 * t.x), x1 = ld3(y + 3 * t.y), x2 = ld3(y + 3 * t.z), x3 = ld3(y + 3 * t.w);
  double J = dot(x1 - x0, cross(x2 - x0, x3 - x0));
  if (!(J > 0.0)) atomicAdd(cnt + v_scene[t.x], 1u);
}

// ------------------------------------------------------------------ launchers
void k_map_surface(zema_scene* s, const double* y, double* xs) {
  if (!s->nsurf) return;
  map_surface_kernel<<<nblocks(s->nsurf), kBlock, 0, s->st>>>(s->nsurf, s->sv_ref.p, s->sv_x0.p, y, s->body_f.p,
                                                              s->body_i.p, xs);
}

void k_surface_disp(zema_scene* s, const double* p, double* dx) {
  if (!s->nsurf) return;
  surface_disp_kernel<<<nblocks(s->nsurf), kBlock, 0, s->st>>>(s->nsurf, s->sv_ref.p, s->sv_x0.p, p, s->body_i.p, dx);
}

void k_axpy(zema_scene* s, int n, double a, const double* x, const double* y, double* out) {
  if (n) axpy_kernel<<<nblocks(n), kBlock, 0, s->st>>>(n, a, x, y, out);
}

void k_scale(zema_scene* s, int n, double a, const double* x, double* out) {
  if (n) scale_kernel<<<nblocks(n), kBlock, 0, s->st>>>(n, a, x, out);
}

void k_iota(zema_scene* s, int* p, int64_t n) {
  if (n > 0) iota_kernel<<<nblocks(n), kBlock, 0, s->st>>>(n, p);
}

void k_velocity(zema_scene* s, double inv_h) {
  if (s->ndof) velocity_kernel<<<nblocks(s->ndof), kBlock, 0, s->st>>>(s->ndof, inv_h, s->y.p, s->yt.p, s->ydot.p);
}

void k_velocity_to(zema_scene* s, double inv_h, double* out) {
  if (s->ndof) velocity_kernel<<<nblocks(s->ndof), kBlock, 0, s->st>>>(s->ndof, inv_h, s->y.p, s->yt.p, out);
}

void k_predict_to(zema_scene* s, double* out) {
  if (s->ndof)
    predict_kernel<<<nblocks(s->ndof), kBlock, 0, s->st>>>(3 * s->nsv, s->ndof, s->P.dt, s->P.gravity[0],
                                                           s->P.gravity[1], s->P.gravity[2], s->y.p, s->ydot.p, out);
}

void k_predict(zema_scene* s) {
  if (s->ndof)
    predict_kernel<<<nblocks(s->ndof), kBlock, 0, s->st>>>(3 * s->nsv, s->ndof, s->P.dt, s->P.gravity[0],
                                                           s->P.gravity[1], s->P.gravity[2], s->y.p, s->ydot.p,
                                                           s->yhat.p);
}

void k_max_disp(zema_scene* s, const double* p, double* out) {
  unsigned long long* u = s->sc_u64.p;
  ZCHK(hipMemsetAsync(u, 0, sizeof(unsigned long long) * s->ns, s->st));
  int n = s->nsv + s->nsurf;
  if (n)
    max_disp_kernel<<<nblocks(n), kBlock, 0, s->st>>>(s->nsv, s->nsurf, s->sv_ref.p, s->sv_x0.p, p, s->body_i.p,
                                                      s->v_scene.p, s->sv_scene.p, u);
  ZCHK(hipMemcpyAsync(out, u, sizeof(double) * s->ns, hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
}

// per scene: a.b, a.a, b.b over the scene's soft and free-body DOFs (one block each)
__global__ void scene_dots_kernel(int nsv, const int* __restrict__ rng, const double* __restrict__ a,
                                  const double* __restrict__ b, double* __restrict__ out) {
  __shared__ double sh[3][kBlock / 64];
  const int k = blockIdx.x;
  const int64_t r[4] = {3 * (int64_t)rng[8 * k], 3 * (int64_t)rng[8 * k + 1],
                        3 * (int64_t)nsv + 12 * (int64_t)rng[8 * k + 6], 3 * (int64_t)nsv + 12 * (int64_t)rng[8 * k + 7]};
  double ab = 0.0, aa = 0.0, bb = 0.0;
  for (int part = 0; part < 2; ++part)
    for (int64_t i = r[2 * part] + threadIdx.x; i < r[2 * part + 1]; i += kBlock) {
      ab += a[i] * b[i];
      aa += a[i] * a[i];
      bb += b[i] * b[i];
    }
  for (int o = 32; o > 0; o >>= 1) {
    ab += __shfl_xor(ab, o, 64);
    aa += __shfl_xor(aa, o, 64);
    bb += __shfl_xor(bb, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = ab;
    sh[1][threadIdx.x >> 6] = aa;
    sh[2][threadIdx.x >> 6] = bb;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += sh[threadIdx.x][w];
    out[3 * k + threadIdx.x] = t;
  }
}

void k_scene_dots(zema_scene* s, const double* a, const double* b, double* out_host) {
  s->sc_dots.reserve((size_t)3 * s->ns);
  scene_dots_kernel<<<s->ns, kBlock, 0, s->st>>>(s->nsv, s->scn_rng.p, a, b, s->sc_dots.p);
  ZCHK(hipMemcpyAsync(out_host, s->sc_dots.p, sizeof(double) * 3 * s->ns, hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
}

void k_axpy_scene(zema_scene* s, const double* alpha_host, const double* p, const double* y, double* out) {
  ZCHK(hipMemcpyAsync(s->sc_alpha.p, alpha_host, sizeof(double) * s->ns, hipMemcpyHostToDevice, s->st));
  if (s->ndof)
    axpy_scene_kernel<<<nblocks(s->ndof), kBlock, 0, s->st>>>(s->ndof, s->nsv, s->sc_alpha.p, s->v_scene.p,
                                                              s->f_scene.p, p, y, out);
}

void k_scale_scene(zema_scene* s, const double* alpha_host, double* p) {
  ZCHK(hipMemcpyAsync(s->sc_alpha.p, alpha_host, sizeof(double) * s->ns, hipMemcpyHostToDevice, s->st));
  if (s->ndof)
    scale_scene_kernel<<<nblocks(s->ndof), kBlock, 0, s->st>>>(s->ndof, s->nsv, s->sc_alpha.p, s->v_scene.p,
                                                               s->f_scene.p, p);
}

void k_select_scene(zema_scene* s, const int* mask_host, const double* a, const double* b, double* out) {
  ZCHK(hipMemcpyAsync(s->sc_mask.p, mask_host, sizeof(int) * s->ns, hipMemcpyHostToDevice, s->st));
  if (s->ndof)
    select_scene_kernel<<<nblocks(s->ndof), kBlock, 0, s->st>>>(s->ndof, s->nsv, s->sc_mask.p, s->v_scene.p,
                                                                s->f_scene.p, a, b, out);
}

void k_sums(zema_scene* s, int nseg, const double* const* ptr, const int64_t* len, double* out_host,
            const void* extra) {
  SegTab tab;
  for (int k = 0; k < 8; ++k) {
    tab.p[k] = k < nseg ? ptr[k] : nullptr;
    tab.n[k] = k < nseg ? len[k] : 0;
  }
  s->red.reserve(32 + 8 * kSumGrid);
  sums_l1<<<dim3(kSumGrid, nseg), kBlock, 0, s->st>>>(tab, s->red.p + 32);
  sums_l2<<<nseg, kBlock, 0, s->st>>>(s->red.p + 32, s->red.p);
  ZCHK(hipMemcpyAsync(out_host, s->red.p, nseg * sizeof(double), hipMemcpyDeviceToHost, s->st));
  if (extra) ZCHK(hipMemcpyAsync(out_host + nseg, extra, sizeof(double), hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
}

// per scene: 1 if any tet of the scene is inverted at y; returns whether any is
bool k_inverted(zema_scene* s, const double* y, int* out) {
  unsigned int* c = s->sc_cnt.p;
  ZCHK(hipMemsetAsync(c, 0, sizeof(unsigned int) * s->ns, s->st));
  if (s->nt) inverted_kernel<<<nblocks(s->nt), kBlock, 0, s->st>>>(s->nt, s->tets.p, y, s->v_scene.p, c);
  std::vector<unsigned int> h(s->ns);
  ZCHK(hipMemcpyAsync(h.data(), c, sizeof(unsigned int) * s->ns, hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
  bool any = false;
  for (int k = 0; k < s->ns; ++k) {
    if (out) out[k] = h[k] != 0;
    any = any || h[k] != 0;
  }
  return any;
}

bool k_any_inverted(zema_scene* s, const double* y) { return k_inverted(s, y, nullptr); }

}  // namespace zema

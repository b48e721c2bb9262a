// Per-vertex warm-start network 16-64-64-64-3 (ReLU) on bf16 matrix cores.
//
// Every layer is computed transposed, Z^T = W H^T, with the 16 vertices of a tile as
// the N dimension of v_mfma_f32_16x16x16_bf16: the accumulator a lane holds for output
// tile t (rows 16t + 4(lane/16) + j of vertex lane%16) is exactly the B operand the
// next layer needs for its k-step t, so activations stay in registers between layers.
// Weights live in LDS as bf16 (rounded to nearest even from the FP32 master copy),
// biases in FP32; accumulation is FP32.
//
// Training: the same forward pass, then the backward pass in the same transposed form
// (delta^T_{l-1} = W_l^T delta^T_l masked by the ReLU), weight gradients
// dW_l = delta_l^T H_{l-1} by MFMA with the vertex tile as the K dimension (operands
// transposed through a per-wave LDS tile), per-block partial gradients reduced in a
// fixed order, then Adam (Kingma and Ba 2015) on the FP32 master weights.
#include <algorithm>
#include <mutex>

#include "mlp.hpp"

namespace zema {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int OW1 = 0, OB1 = 1024, OW2 = 1088, OB2 = 5184, OW3 = 5248, OB3 = 9344, OW4 = 9408, OB4 = 9600;
static_assert(OB4 + 3 == kMlpParams, "parameter layout");

__device__ inline unsigned short f2bf(float x) {  // round to nearest, ties to even
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ inline bf4 pack_relu(f4 a) {
  bf4 r;
  r[0] = (short)f2bf(fmaxf(a[0], 0.0f));
  r[1] = (short)f2bf(fmaxf(a[1], 0.0f));
  r[2] = (short)f2bf(fmaxf(a[2], 0.0f));
  r[3] = (short)f2bf(fmaxf(a[3], 0.0f));
  return r;
}

__device__ inline bf4 pack(f4 a) {
  bf4 r;
  for (int j = 0; j < 4; ++j) r[j] = (short)f2bf(a[j]);
  return r;
}

struct __align__(16) MlpLds {
  unsigned short W1[64 * 16], W2[64 * 64], W3[64 * 64], W4[16 * 64];  // [out][in], W4 rows 3..15 zero
  unsigned short W2T[64 * 64], W3T[64 * 64], W4T[64 * 16];             // [in][out]
  float b1[64], b2[64], b3[64], b4[16];
};

// four consecutive bf16 of row `row` starting at column `col` (col % 4 == 0, ld % 4 == 0)
__device__ inline bf4 lds4(const unsigned short* W, int ld, int row, int col) {
  return *reinterpret_cast<const bf4*>(W + row * ld + col);
}

__device__ void load_weights(const float* __restrict__ th, MlpLds& L, bool transposed) {
  for (int e = threadIdx.x; e < 64 * 16; e += blockDim.x) L.W1[e] = f2bf(th[OW1 + e]);
  for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
    int o = e / 64, i = e % 64;
    unsigned short w2 = f2bf(th[OW2 + e]), w3 = f2bf(th[OW3 + e]);
    L.W2[e] = w2;
    L.W3[e] = w3;
    if (transposed) {
      L.W2T[i * 64 + o] = w2;
      L.W3T[i * 64 + o] = w3;
    }
  }
  for (int e = threadIdx.x; e < 16 * 64; e += blockDim.x) {
    int c = e / 64, i = e % 64;
    unsigned short w = c < 3 ? f2bf(th[OW4 + e]) : (unsigned short)0;
    L.W4[e] = w;
    if (transposed) L.W4T[i * 16 + c] = w;
  }
  for (int e = threadIdx.x; e < 64; e += blockDim.x) {
    L.b1[e] = th[OB1 + e];
    L.b2[e] = th[OB2 + e];
    L.b3[e] = th[OB3 + e];
  }
  for (int e = threadIdx.x; e < 16; e += blockDim.x) L.b4[e] = e < 3 ? th[OB4 + e] : 0.0f;
}

struct Fwd {
  bf4 x, h1[4], h2[4], h3[4];
  f4 y;
};

// forward pass of one 16-vertex tile; m = lane % 16 (vertex), q = lane / 16
__device__ inline void forward_tile(const MlpLds& L, bf4 x, int m, int q, Fwd& F) {
  F.x = x;
  for (int t = 0; t < 4; ++t) {
    f4 a = {L.b1[16 * t + 4 * q], L.b1[16 * t + 4 * q + 1], L.b1[16 * t + 4 * q + 2], L.b1[16 * t + 4 * q + 3]};
    a = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(L.W1, 16, 16 * t + m, 4 * q), x, a, 0, 0, 0);
    F.h1[t] = pack_relu(a);
  }
  for (int t = 0; t < 4; ++t) {
    f4 a = {L.b2[16 * t + 4 * q], L.b2[16 * t + 4 * q + 1], L.b2[16 * t + 4 * q + 2], L.b2[16 * t + 4 * q + 3]};
    for (int k = 0; k < 4; ++k)
      a = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(L.W2, 64, 16 * t + m, 16 * k + 4 * q), F.h1[k], a, 0, 0, 0);
    F.h2[t] = pack_relu(a);
  }
  for (int t = 0; t < 4; ++t) {
    f4 a = {L.b3[16 * t + 4 * q], L.b3[16 * t + 4 * q + 1], L.b3[16 * t + 4 * q + 2], L.b3[16 * t + 4 * q + 3]};
    for (int k = 0; k < 4; ++k)
      a = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(L.W3, 64, 16 * t + m, 16 * k + 4 * q), F.h2[k], a, 0, 0, 0);
    F.h3[t] = pack_relu(a);
  }
  f4 a = {L.b4[4 * q], L.b4[4 * q + 1], L.b4[4 * q + 2], L.b4[4 * q + 3]};
  for (int k = 0; k < 4; ++k)
    a = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(L.W4, 64, m, 16 * k + 4 * q), F.h3[k], a, 0, 0, 0);
  F.y = a;  // rows 4q + j: outputs 0..2 live in lanes with q == 0
}

__device__ inline bf4 load_x(const float* __restrict__ feat, long row, int q, bool valid) {
  bf4 x = {0, 0, 0, 0};
  if (valid) {
    const float* f = feat + 16 * row + 4 * q;
    for (int j = 0; j < 4; ++j) x[j] = (short)f2bf(f[j]);
  }
  return x;
}

__global__ void __launch_bounds__(256) mlp_forward_kernel(const float* __restrict__ th, const float* __restrict__ feat,
                                                          long n, float* __restrict__ out) {
  __shared__ MlpLds L;
  load_weights(th, L, false);
  __syncthreads();
  const int lane = threadIdx.x & 63, m = lane & 15, q = lane >> 4;
  const long ntiles = (n + 15) / 16;
  const long wstride = (long)gridDim.x * (blockDim.x / 64);
  for (long tile = (long)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); tile < ntiles; tile += wstride) {
    long v = 16 * tile + m;
    Fwd F;
    forward_tile(L, load_x(feat, v, q, v < n), m, q, F);
    if (q == 0 && v < n)
      for (int c = 0; c < 3; ++c) out[3 * v + c] = F.y[c];
  }
}

// One wavefront per block; block b owns tiles [b * tpb, (b + 1) * tpb).  Writes the
// block's whole gradient partial (kMlpParams floats) and its loss partial.
__global__ void __launch_bounds__(64) mlp_grad_kernel(const float* __restrict__ th, const float* __restrict__ feat,
                                                      const float* __restrict__ target, const int* __restrict__ idx,
                                                      long nrows, long n, int tpb, float* __restrict__ gpart,
                                                      double* __restrict__ lpart) {
  __shared__ MlpLds L;
  __shared__ __align__(16) unsigned short Td[64 * 16];  // [row][vertex] transposition tiles
  __shared__ __align__(16) unsigned short Th[64 * 16];
  load_weights(th, L, true);
  __syncthreads();
  const int lane = threadIdx.x, m = lane & 15, q = lane >> 4;
  const float gs = 2.0f / (3.0f * (float)n);
  f4 g1[4], g2[4][4], g3[4][4], g4[4];
  f4 gb1[4], gb2[4], gb3[4], gb4;
  const f4 z = {0, 0, 0, 0};
  for (int a = 0; a < 4; ++a) {
    g1[a] = z;
    g4[a] = z;
    gb1[a] = z;
    gb2[a] = z;
    gb3[a] = z;
    for (int b = 0; b < 4; ++b) {
      g2[a][b] = z;
      g3[a][b] = z;
    }
  }
  gb4 = z;
  double lsum = 0.0;
  const long ntiles = (n + 15) / 16;
  for (int k = 0; k < tpb; ++k) {
    long tile = (long)blockIdx.x * tpb + k;
    if (tile >= ntiles) break;
    long v = 16 * tile + m;
    long row = v < n ? (idx ? (long)idx[v] : v) : -1;
    bool valid = row >= 0 && row < nrows;  // out-of-range sample indices are skipped
    if (!valid) row = 0;
    Fwd F;
    forward_tile(L, load_x(feat, row, q, valid), m, q, F);
    // output error
    f4 dy = z;
    if (q == 0 && valid)
      for (int c = 0; c < 3; ++c) {
        float e = F.y[c] - target[3 * row + c];
        lsum += (double)e * (double)e;
        dy[c] = gs * e;
      }
    gb4 += dy;
    bf4 d4 = pack(dy);
    // delta3 = (W4^T dy) * [h3 > 0]
    f4 d3[4], d2[4], d1[4];
    for (int t = 0; t < 4; ++t) {
      f4 a = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(L.W4T, 16, 16 * t + m, 4 * q), d4, z, 0, 0, 0);
      for (int j = 0; j < 4; ++j) a[j] = F.h3[t][j] != 0 ? a[j] : 0.0f;
      d3[t] = a;
      gb3[t] += a;
    }
    bf4 d3b[4];
    for (int t = 0; t < 4; ++t) d3b[t] = pack(d3[t]);
    for (int t = 0; t < 4; ++t) {
      f4 a = z;
      for (int kk = 0; kk < 4; ++kk)
        a = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(L.W3T, 64, 16 * t + m, 16 * kk + 4 * q), d3b[kk], a, 0, 0,
                                                      0);
      for (int j = 0; j < 4; ++j) a[j] = F.h2[t][j] != 0 ? a[j] : 0.0f;
      d2[t] = a;
      gb2[t] += a;
    }
    bf4 d2b[4];
    for (int t = 0; t < 4; ++t) d2b[t] = pack(d2[t]);
    for (int t = 0; t < 4; ++t) {
      f4 a = z;
      for (int kk = 0; kk < 4; ++kk)
        a = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(L.W2T, 64, 16 * t + m, 16 * kk + 4 * q), d2b[kk], a, 0, 0,
                                                      0);
      for (int j = 0; j < 4; ++j) a[j] = F.h1[t][j] != 0 ? a[j] : 0.0f;
      d1[t] = a;
      gb1[t] += a;
    }
    bf4 d1b[4];
    for (int t = 0; t < 4; ++t) d1b[t] = pack(d1[t]);
    // weight gradients dW[o][i] += sum_v delta[o][v] h[i][v]: stage delta and h as
    // [row][vertex] tiles so both operands read four consecutive vertices
    auto stage = [&](unsigned short* T, const bf4* src, int ntile) {
      for (int t = 0; t < ntile; ++t)
        for (int j = 0; j < 4; ++j) T[(16 * t + 4 * q + j) * 16 + m] = (unsigned short)src[t][j];
    };
    // layer 4 (rows 0..15 of which 0..2 are real) x h3
    __syncthreads();
    stage(Td, &d4, 1);
    stage(Th, F.h3, 4);
    __syncthreads();
    for (int ti = 0; ti < 4; ++ti)
      g4[ti] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(Td, 16, m, 4 * q), lds4(Th, 16, 16 * ti + m, 4 * q),
                                                         g4[ti], 0, 0, 0);
    __syncthreads();
    stage(Td, d3b, 4);
    stage(Th, F.h2, 4);
    __syncthreads();
    for (int to = 0; to < 4; ++to)
      for (int ti = 0; ti < 4; ++ti)
        g3[to][ti] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(Td, 16, 16 * to + m, 4 * q),
                                                               lds4(Th, 16, 16 * ti + m, 4 * q), g3[to][ti], 0, 0, 0);
    __syncthreads();
    stage(Td, d2b, 4);
    stage(Th, F.h1, 4);
    __syncthreads();
    for (int to = 0; to < 4; ++to)
      for (int ti = 0; ti < 4; ++ti)
        g2[to][ti] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(Td, 16, 16 * to + m, 4 * q),
                                                               lds4(Th, 16, 16 * ti + m, 4 * q), g2[to][ti], 0, 0, 0);
    __syncthreads();
    stage(Td, d1b, 4);
    stage(Th, &F.x, 1);
    __syncthreads();
    for (int to = 0; to < 4; ++to)
      g1[to] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lds4(Td, 16, 16 * to + m, 4 * q), lds4(Th, 16, m, 4 * q),
                                                         g1[to], 0, 0, 0);
  }
  // write the block partial: accumulator element j of a lane is row 16 to + 4q + j,
  // column 16 ti + m
  float* P = gpart + (size_t)blockIdx.x * kMlpParams;
  for (int to = 0; to < 4; ++to)
    for (int j = 0; j < 4; ++j) {
      int o = 16 * to + 4 * q + j;
      P[OW1 + o * 16 + m] = g1[to][j];
      for (int ti = 0; ti < 4; ++ti) {
        P[OW2 + o * 64 + 16 * ti + m] = g2[to][ti][j];
        P[OW3 + o * 64 + 16 * ti + m] = g3[to][ti][j];
      }
    }
  for (int ti = 0; ti < 4; ++ti)
    for (int j = 0; j < 3; ++j)
      if (q == 0) P[OW4 + j * 64 + 16 * ti + m] = g4[ti][j];
  // bias gradients: sum the per-vertex deltas over the 16 lanes of each group
  auto vsum = [&](float x) {
    for (int o = 1; o < 16; o <<= 1) x += __shfl_xor(x, o, 64);
    return x;
  };
  for (int t = 0; t < 4; ++t)
    for (int j = 0; j < 4; ++j) {
      float s1 = vsum(gb1[t][j]), s2 = vsum(gb2[t][j]), s3 = vsum(gb3[t][j]);
      if (m == 0) {
        P[OB1 + 16 * t + 4 * q + j] = s1;
        P[OB2 + 16 * t + 4 * q + j] = s2;
        P[OB3 + 16 * t + 4 * q + j] = s3;
      }
    }
  for (int j = 0; j < 3; ++j) {
    float s4 = vsum(gb4[j]);
    if (m == 0 && q == 0) P[OB4 + j] = s4;
  }
  double l = wave_sum(lsum);
  if (lane == 0) lpart[blockIdx.x] = l;
}

// g = sum of block partials in block order; then either store g or take an Adam step
__global__ void mlp_reduce_kernel(int nblk, const float* __restrict__ gpart, float* __restrict__ grad,
                                  float* __restrict__ th, float* __restrict__ mo, float* __restrict__ ve, int adam,
                                  float lr, float c1, float c2) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float g = 0.0f;
  for (int b = 0; b < nblk; ++b) g += gpart[(size_t)b * kMlpParams + p];
  grad[p] = g;
  if (adam) {
    float mm = 0.9f * mo[p] + 0.1f * g;
    float vv = 0.999f * ve[p] + 0.001f * g * g;
    mo[p] = mm;
    ve[p] = vv;
    th[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
  }
}

__global__ void mlp_loss_kernel(int nblk, const double* __restrict__ lpart, long n, double* __restrict__ out) {
  __shared__ double sh[kBlock / 64];
  double a = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kBlock) a += lpart[b];
  a = block_sum<kBlock>(a, sh);
  if (threadIdx.x == 0) out[0] = a / (3.0 * (double)n);
}

void mlp_forward(const zema_mlp* M, hipStream_t st, const float* feat, long n, float* out) {
  if (n <= 0) return;
  long ntiles = (n + 15) / 16;
  int grid = (int)std::min<long>((ntiles + 3) / 4, 2048);
  mlp_forward_kernel<<<grid, 256, 0, st>>>(M->theta.p, feat, n, out);
}

double mlp_grad(zema_mlp* M, const float* feat, const float* target, const int* idx, long nrows, long n, bool adam,
                float lr) {
  long ntiles = (n + 15) / 16;
  int nblk = (int)((ntiles + kTilesPerBlock - 1) / kTilesPerBlock);
  M->gpart.reserve((size_t)nblk * kMlpParams);
  M->lpart.reserve(nblk + 1);
  mlp_grad_kernel<<<nblk, 64, 0, M->st>>>(M->theta.p, feat, target, idx, nrows, n, kTilesPerBlock, M->gpart.p,
                                          M->lpart.p);
  float c1 = 1.0f, c2 = 1.0f;
  if (adam) {
    M->step += 1;
    c1 = (float)(1.0 - std::pow(0.9, M->step));
    c2 = (float)(1.0 - std::pow(0.999, M->step));
  }
  mlp_reduce_kernel<<<nblocks(kMlpParams), kBlock, 0, M->st>>>(nblk, M->gpart.p, M->grad.p, M->theta.p, M->mom.p,
                                                                M->vel.p, adam ? 1 : 0, lr, c1, c2);
  mlp_loss_kernel<<<1, kBlock, 0, M->st>>>(nblk, M->lpart.p, n, M->loss.p);
  double l = 0.0;
  ZCHK(hipMemcpyAsync(&l, M->loss.p, sizeof(double), hipMemcpyDeviceToHost, M->st));
  ZCHK(hipStreamSynchronize(M->st));
  return l;
}

// ------------------------------------------------------------ allocation-free gradient
// Scratch of mlp_grad_noalloc: kNoAllocBlocks gradient partials (FP32), as many loss
// partials and the loss (FP64).  Each device holds its own copy; its address on a
// device comes from hipGetSymbolAddress with that device current (the array's name in
// host code is not a device address).  Every block overwrites its whole partial, so
// nothing needs clearing between calls; calls that overlap on one device race.
constexpr size_t kNoAllocGradBytes = (size_t)kNoAllocBlocks * kMlpParams * sizeof(float);
constexpr size_t kNoAllocBytes = kNoAllocGradBytes + (kNoAllocBlocks + 1) * sizeof(double);
static_assert(kNoAllocGradBytes % 256 == 0, "loss partials stay 256-byte aligned");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch[kMaxDevices] = {};

// device address of this device's scratch (looked up once per device)
static unsigned char* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error(ZEMA_E_DEVICE, "device id out of range for the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(ZEMA_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = (unsigned char*)p;
  }
  return g_scratch[dev];
}

double mlp_grad_noalloc(zema_mlp* M, const float* feat, const float* target, long n, float* grad) {
  int cur = 0;
  ZCHK(hipGetDevice(&cur));
  if (cur != M->dev) ZCHK(hipSetDevice(M->dev));
  struct Restore {
    int d, c;
    ~Restore() {
      if (d != c) (void)hipSetDevice(c);
    }
  } restore{M->dev, cur};
  unsigned char* base = scratch_on(M->dev);
  float* gpart = (float*)base;
  double* lpart = (double*)(base + kNoAllocGradBytes);
  double* loss = lpart + kNoAllocBlocks;
  long ntiles = (n + 15) / 16;
  long tpb = std::max<long>(kTilesPerBlock, (ntiles + kNoAllocBlocks - 1) / kNoAllocBlocks);
  int nblk = (int)((ntiles + tpb - 1) / tpb);
  mlp_grad_kernel<<<nblk, 64, 0, M->st>>>(M->theta.p, feat, target, nullptr, n, n, (int)tpb, gpart, lpart);
  mlp_reduce_kernel<<<nblocks(kMlpParams), kBlock, 0, M->st>>>(nblk, gpart, grad, M->theta.p, M->mom.p, M->vel.p, 0,
                                                                0.0f, 1.0f, 1.0f);
  mlp_loss_kernel<<<1, kBlock, 0, M->st>>>(nblk, lpart, n, loss);
  double l = 0.0;
  ZCHK(hipMemcpyAsync(&l, loss, sizeof(double), hipMemcpyDeviceToHost, M->st));
  ZCHK(hipStreamSynchronize(M->st));
  return l;
}

}  // namespace zema

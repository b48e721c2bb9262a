// Shared host/device utilities of the HIP library: error handling, device buffers,
// launch helpers and small vector math.  gfx950 (CDNA4), wave64.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace zema {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define ZCHK(call)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::zema::Error(-9, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

constexpr int kBlock = 256;
inline int nblocks(int64_t n, int b = kBlock) { return (int)((n + b - 1) / b); }

// Workgroup b of a launch runs on XCD b mod 8 (round-robin dispatch, 8 XCDs with an
// L2 each).  xcd_block(b, n) is the logical block of workgroup b when each XCD takes a
// contiguous run of the n logical blocks (XCD x: runs of q or q + 1 blocks, n = 8q + r),
// so neighbouring blocks share their XCD's L2.  A bijection of [0, n).
__device__ inline int xcd_block(int b, int n) {
  const int x = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + k;
}

// Device buffer with capacity; growing discards the old contents.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0, cap = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  void reserve(size_t c) {
    if (c <= cap) return;
    size_t nc = c < 2 * cap ? 2 * cap : c;
    if (nc < 16) nc = 16;
    if (p) ZCHK(hipFree(p));
    p = nullptr;
    ZCHK(hipMalloc(&p, nc * sizeof(T)));
    cap = nc;
  }
  void resize(size_t m) {
    reserve(m);
    n = m;
  }
  // st: copy on that stream and wait for it (uploads while other threads capture graphs
  // must stay off the legacy stream); null: a synchronous copy
  void upload(const std::vector<T>& v, hipStream_t st = nullptr) {
    resize(v.size());
    if (v.empty()) return;
    if (st) {
      ZCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
      ZCHK(hipStreamSynchronize(st));
    } else {
      ZCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    }
  }
  void upload(const T* v, size_t m) {
    resize(m);
    if (m) ZCHK(hipMemcpy(p, v, m * sizeof(T), hipMemcpyHostToDevice));
  }
  std::vector<T> download(hipStream_t s) const {
    std::vector<T> v(n);
    if (n) {
      ZCHK(hipMemcpyAsync(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
      ZCHK(hipStreamSynchronize(s));
    }
    return v;
  }
};

// ------------------------------------------------------------------ 3-vectors
struct V3 {
  double x, y, z;
};
__host__ __device__ inline V3 v3(double x, double y, double z) { return {x, y, z}; }
__host__ __device__ inline V3 ld3(const double* p) { return {p[0], p[1], p[2]}; }
__host__ __device__ inline void st3(double* p, V3 a) {
  p[0] = a.x;
  p[1] = a.y;
  p[2] = a.z;
}
__host__ __device__ inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__host__ __device__ inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__host__ __device__ inline V3 operator-(V3 a) { return {-a.x, -a.y, -a.z}; }
__host__ __device__ inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__host__ __device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__host__ __device__ inline double comp(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

// ordered-bits of a non-negative double (monotone as an unsigned integer)
__device__ inline unsigned long long dbits(double d) { return (unsigned long long)__double_as_longlong(d); }

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Per-scene extremum of non-negative doubles (ordered as their bits): one atomic per
// wavefront when all its lanes belong to the same scene, else one per lane.  sc < 0
// contributes nothing.  Min and max are order-independent, so the result is exact.
template <bool MAX>
__device__ inline void scene_atomic_ext(unsigned long long* out, int sc, double v) {
  int sc0 = __shfl(sc, 0, 64);
  if (__all(sc == sc0)) {
    for (int o = 32; o > 0; o >>= 1) {
      double w = __shfl_xor(v, o, 64);
      v = MAX ? fmax(v, w) : fmin(v, w);
    }
    if ((threadIdx.x & 63) == 0 && sc0 >= 0) {
      if (MAX)
        atomicMax(out + sc0, dbits(v));
      else
        atomicMin(out + sc0, dbits(v));
    }
  } else if (sc >= 0) {
    if (MAX)
      atomicMax(out + sc, dbits(v));
    else
      atomicMin(out + sc, dbits(v));
  }
}

// Deterministic block sum (fixed tree), result valid in thread 0.
template <int B>
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < B / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}

}  // namespace zema

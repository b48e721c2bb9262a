// Exclusive prefix sum and stable LSD radix sort of (64-bit key, int value) pairs.
// The radix sort ranks equal digits inside a 64-lane wave with ballots (one ballot
// per digit bit), combines waves through LDS and keeps input order within a digit,
// so the result is deterministic.
#include "scene.hpp"

namespace zema {

constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = kBlock * SCAN_ITEMS;

__device__ inline int block_exclusive_scan(int v, int* sh, int* total) {
  // wave inclusive scan
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int i = 0; i < kBlock / 64; ++i) {
      int t = sh[i];
      sh[i] = acc;
      acc += t;
    }
    sh[kBlock / 64] = acc;
  }
  __syncthreads();
  int r = x - v + sh[w];
  *total = sh[kBlock / 64];
  __syncthreads();
  return r;
}

__global__ void scan_tiles(const int* __restrict__ in, int* __restrict__ out, int64_t n, int* __restrict__ sums) {
  __shared__ int sh[kBlock / 64 + 1];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int loc = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    loc += v[k];
  }
  int tot;
  int off = block_exclusive_scan(loc, sh, &tot);
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = off;
    off += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void scan_add(int* __restrict__ out, int64_t n, const int* __restrict__ offs) {
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int o = offs[blockIdx.x];
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) out[base + k] += o;
}

// returns the total when want_total (one host synchronisation); out may alias in
static int64_t scan_rec(zema_scene* s, const int* in, int* out, int64_t n, int lvl, bool want_total) {
  int nb = (int)((n + SCAN_TILE - 1) / SCAN_TILE);
  while ((int)s->scan_tmp.size() <= lvl) s->scan_tmp.emplace_back(new DBuf<int>());
  DBuf<int>& sums = *s->scan_tmp[lvl];
  sums.reserve(nb + 1);
  scan_tiles<<<nb, kBlock, 0, s->st>>>(in, out, n, sums.p);
  if (nb == 1) {
    if (!want_total) return -1;
    int t;
    ZCHK(hipMemcpyAsync(&t, sums.p, sizeof(int), hipMemcpyDeviceToHost, s->st));
    ZCHK(hipStreamSynchronize(s->st));
    return t;
  }
  int64_t total = scan_rec(s, sums.p, sums.p, nb, lvl + 1, want_total);
  scan_add<<<nb, kBlock, 0, s->st>>>(out, n, sums.p);
  return total;
}

int64_t k_exclusive_scan(zema_scene* s, const int* in, int* out, int64_t n, bool want_total) {
  if (n <= 0) return 0;
  return scan_rec(s, in, out, n, 0, want_total);
}

// ------------------------------------------------------------------ radix sort
constexpr int RS_ROUNDS = 8;
constexpr int RS_TILE = kBlock * RS_ROUNDS;

__global__ void rs_hist(const unsigned long long* __restrict__ keys, int64_t n, int shift, int nblk,
                        int* __restrict__ hist) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t i = base + r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void rs_scatter(const unsigned long long* __restrict__ kin, const int* __restrict__ vin,
                           unsigned long long* __restrict__ kout, int* __restrict__ vout, int64_t n, int shift,
                           int nblk, const int* __restrict__ offs) {
  __shared__ int base[256];
  __shared__ int wcnt[kBlock / 64][256];
  base[threadIdx.x] = offs[(int64_t)threadIdx.x * nblk + blockIdx.x];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int64_t tile = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    for (int k = 0; k < kBlock / 64; ++k) wcnt[k][threadIdx.x] = 0;
    __syncthreads();
    int64_t i = tile + r * kBlock + threadIdx.x;
    bool valid = i < n;
    unsigned long long key = valid ? kin[i] : 0ull;
    int val = valid ? vin[i] : 0;
    int d = (int)((key >> shift) & 255u);
    unsigned long long match = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      unsigned long long bal = __ballot((d >> b) & 1);
      match &= ((d >> b) & 1) ? bal : ~bal;
    }
    int rank = __popcll(match & lt);
    if (valid && rank == 0) wcnt[w][d] = __popcll(match);
    __syncthreads();
    if (valid) {
      int off = base[d];
      for (int k = 0; k < w; ++k) off += wcnt[k][d];
      kout[off + rank] = key;
      vout[off + rank] = val;
    }
    __syncthreads();
    {
      int dd = threadIdx.x, add = 0;
      for (int k = 0; k < kBlock / 64; ++k) add += wcnt[k][dd];
      base[dd] += add;
    }
    __syncthreads();
  }
}

// Small inputs: one workgroup sorts (key, value) pairs in LDS by a bitonic network,
// ordering equal keys by value.  Every caller's values are distinct input positions
// or its keys are distinct, so the result equals the stable radix sort's, in one
// launch instead of several per digit.
constexpr int kSmallSort = 4096;

__global__ void __launch_bounds__(1024) small_sort_kernel(int n, int m, unsigned long long* __restrict__ keys,
                                                          int* __restrict__ vals) {
  __shared__ unsigned long long K[kSmallSort];
  __shared__ int Vs[kSmallSort];
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    K[i] = i < n ? keys[i] : ~0ull;
    Vs[i] = i < n ? vals[i] : 0x7fffffff;
  }
  __syncthreads();
  for (int k = 2; k <= m; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const unsigned long long a = K[i], c = K[l];
          const int va = Vs[i], vc = Vs[l];
          const bool gt = a > c || (a == c && va > vc);
          if (gt == up) {
            K[i] = c;
            K[l] = a;
            Vs[i] = vc;
            Vs[l] = va;
          }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    keys[i] = K[i];
    vals[i] = Vs[i];
  }
}

void k_radix_sort(zema_scene* s, SortBufs& b, int64_t n, int key_bits) {
  if (n <= 1) return;
  if (n <= kSmallSort) {
    int m = 2;
    while (m < n) m <<= 1;
    small_sort_kernel<<<1, 1024, 0, s->st>>>((int)n, m, b.k0.p, b.v0.p);
    return;
  }
  int nblk = (int)((n + RS_TILE - 1) / RS_TILE);
  b.k1.reserve(n);
  b.v1.reserve(n);
  b.hist.reserve((size_t)256 * nblk);
  for (int shift = 0; shift < key_bits; shift += 8) {
    rs_hist<<<nblk, kBlock, 0, s->st>>>(b.k0.p, n, shift, nblk, b.hist.p);
    k_exclusive_scan(s, b.hist.p, b.hist.p, (int64_t)256 * nblk, false);
    rs_scatter<<<nblk, kBlock, 0, s->st>>>(b.k0.p, b.v0.p, b.k1.p, b.v1.p, n, shift, nblk, b.hist.p);
    std::swap(b.k0.p, b.k1.p);
    std::swap(b.k0.cap, b.k1.cap);
    std::swap(b.v0.p, b.v1.p);
    std::swap(b.v0.cap, b.v1.cap);
  }
}

}  // namespace zema

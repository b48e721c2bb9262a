// Broad phase: the candidate set of the contact term (Sec. III eq. 4, inter-body
// point-triangle and edge-edge pairs) is defined by an exact box predicate on the
// caller's positions -- per axis lo = min over the primitive's vertices of
// min(xs0, xs1) - r, hi = max of max + r, pairs kept when the closed intervals
// overlap on all three axes.  A uniform spatial hash (cell size ~ mean surface edge
// length, hash of Teschner et al. 2003) only accelerates the search: entries are
// sorted by bucket with the radix sort, every query walks the cells of its box, and a
// pair is reported only from the cell that contains the componentwise maximum of
// the two lower corners, which both boxes contain, so each pair appears exactly
// once.  Boxes spanning more than kBigCells cells skip the table and are tested
// against every primitive.  The output is sorted by (first, second) id.
#include <algorithm>

#include "scene.hpp"

namespace zema {

constexpr int kBigCells = 512;
constexpr int kCellBias = 1 << 20;

__device__ inline int cell_of(double z, double inv_c) { return (int)floor(__dmul_rn(z, inv_c)); }

// cells of different scenes of a batch hash apart (scene 0 leaves the hash unchanged)
__device__ inline unsigned hash3(int ix, int iy, int iz, int sc, unsigned mask) {
  return (((unsigned)ix * 73856093u) ^ ((unsigned)iy * 19349663u) ^ ((unsigned)iz * 83492791u) ^
          ((unsigned)sc * 2654435761u)) &
         mask;
}

__device__ inline unsigned long long pack_cell(int ix, int iy, int iz) {
  return ((unsigned long long)(ix + kCellBias) << 42) | ((unsigned long long)(iy + kCellBias) << 21) |
         (unsigned long long)(iz + kCellBias);
}

// boxes of vertices [0, nv), triangles [nv, nv+nt), edges [nv+nt, nv+nt+ne) over the
// positions xs0, xs1 and, when given, xs2
__global__ void boxes_kernel(int nv, int nt, int ne, const int* __restrict__ tris, const int* __restrict__ edges,
                             const double* __restrict__ xs0, const double* __restrict__ xs1,
                             const double* __restrict__ xs2, double r, double* __restrict__ lo,
                             double* __restrict__ hi) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv + nt + ne) return;
  int v[3], n;
  if (i < nv) {
    v[0] = i;
    n = 1;
  } else if (i < nv + nt) {
    const int* t = tris + 3 * (i - nv);
    v[0] = t[0];
    v[1] = t[1];
    v[2] = t[2];
    n = 3;
  } else {
    const int* e = edges + 2 * (i - nv - nt);
    v[0] = e[0];
    v[1] = e[1];
    n = 2;
  }
  for (int k = 0; k < 3; ++k) {
    double l = INFINITY, h = -INFINITY;
    for (int a = 0; a < n; ++a) {
      double p = xs0[3 * v[a] + k], q = xs1[3 * v[a] + k];
      l = fmin(l, fmin(p, q));
      h = fmax(h, fmax(p, q));
      if (xs2) {
        double w = xs2[3 * v[a] + k];
        l = fmin(l, w);
        h = fmax(h, w);
      }
    }
    lo[3 * i + k] = __dsub_rn(l, r);
    hi[3 * i + k] = __dadd_rn(h, r);
  }
}

__device__ inline bool overlap(const double* lo, const double* hi, int a, int b) {
  for (int k = 0; k < 3; ++k)
    if (!(lo[3 * a + k] <= hi[3 * b + k] && lo[3 * b + k] <= hi[3 * a + k])) return false;
  return true;
}

// cell range of a box; returns the number of cells or -1 when large / out of range
__device__ inline long long cell_range(const double* lo, const double* hi, int i, double inv_c, int c0[3], int c1[3]) {
  long long n = 1;
  for (int k = 0; k < 3; ++k) {
    double a = __dmul_rn(lo[3 * i + k], inv_c), b = __dmul_rn(hi[3 * i + k], inv_c);
    if (!(a > -(double)(kCellBias - 2) && b < (double)(kCellBias - 2))) return -1;
    c0[k] = (int)floor(a);
    c1[k] = (int)floor(b);
    n *= (long long)(c1[k] - c0[k] + 1);
  }
  return n > kBigCells ? -1 : n;
}

struct PrimSet {
  int base;  // index of the first primitive in the box arrays
  int n;
};

__device__ inline int prim_body(int kind, int id, const int* tris, const int* edges, const int* sv_body) {
  if (kind == 0) return sv_body[id];
  if (kind == 1) return sv_body[tris[3 * id]];
  return sv_body[edges[2 * id]];
}

// scene tables of the search: per surface vertex and per body scene, per-scene 1/cell,
// per-scene body ranges [soft b0, b1, affine b0, b1] (global body ids), and the
// boxes of whole bodies (order-preserving integer encoding, [nb][3])
struct SceneTab {
  const int *sv_body, *body_scene;
  const double* icell;
  const int* scene_bodies;
  const unsigned long long *blo, *bhi;
  const int* active;  // per-scene flags of a batch whose finished scenes are left out, or null
};

// order-preserving map of doubles to unsigned integers, and back
__device__ inline unsigned long long ord_enc(double d) {
  unsigned long long u = (unsigned long long)__double_as_longlong(d);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline double ord_dec(unsigned long long u) {
  u = (u >> 63) ? (u & 0x7fffffffffffffffull) : ~u;
  return __longlong_as_double((long long)u);
}

// box of every body = union of the boxes of its surface vertices (a triangle's or an
// edge's box is the union of its vertices' boxes); one atomic per wavefront when the
// wavefront's vertices share a body
__global__ void body_box_kernel(int nv, const double* __restrict__ lo, const double* __restrict__ hi,
                                const int* __restrict__ sv_body, unsigned long long* __restrict__ blo,
                                unsigned long long* __restrict__ bhi) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int b = i < nv ? sv_body[i] : -1;
  int b0 = __shfl(b, 0, 64);
  bool uni = __all(b == b0);
  for (int k = 0; k < 3; ++k) {
    unsigned long long l = i < nv ? ord_enc(lo[3 * i + k]) : ~0ull;
    unsigned long long h = i < nv ? ord_enc(hi[3 * i + k]) : 0ull;
    if (uni) {
      for (int o = 32; o > 0; o >>= 1) {
        unsigned long long l2 = __shfl_xor(l, o, 64), h2 = __shfl_xor(h, o, 64);
        l = l2 < l ? l2 : l;
        h = h2 > h ? h2 : h;
      }
      if ((threadIdx.x & 63) == 0 && b0 >= 0) {
        atomicMin(blo + 3 * b0 + k, l);
        atomicMax(bhi + 3 * b0 + k, h);
      }
    } else if (b >= 0) {
      atomicMin(blo + 3 * b + k, l);
      atomicMax(bhi + 3 * b + k, h);
    }
  }
}

// does box i overlap the box of another body of scene sc?  A candidate pair needs
// its two boxes to overlap, so each primitive of a pair passes this test for the
// other's body: skipping primitives that fail it leaves the candidate set unchanged.
__device__ inline bool near_other_body(const SceneTab& S, int body, int sc, const double* lo, const double* hi,
                                       int i) {
  if (S.active && !S.active[sc]) return false;  // a finished scene of the batch: no pairs needed
  const int* R = S.scene_bodies + 4 * sc;
  for (int part = 0; part < 2; ++part)
    for (int b = R[2 * part]; b < R[2 * part + 1]; ++b) {
      if (b == body) continue;
      bool ov = true;
      for (int k = 0; k < 3 && ov; ++k)
        ov = ord_dec(S.blo[3 * b + k]) <= hi[3 * i + k] && lo[3 * i + k] <= ord_dec(S.bhi[3 * b + k]);
      if (ov) return true;
    }
  return false;
}

__device__ inline int prim_scene(int kind, int id, const int* tris, const int* edges, const SceneTab& S) {
  return S.body_scene[prim_body(kind, id, tris, edges, S.sv_body)];
}

// entries: count cells of every entry primitive (0 for large ones, flagged in big)
__global__ void entry_count_kernel(PrimSet E, int ekind, const double* __restrict__ lo, const double* __restrict__ hi,
                                   SceneTab S, const int* __restrict__ tris, const int* __restrict__ edges,
                                   int* __restrict__ cnt, int* __restrict__ big_flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E.n) return;
  int c0[3], c1[3];
  int body = prim_body(ekind, i, tris, edges, S.sv_body), sc = S.body_scene[body];
  if (!near_other_body(S, body, sc, lo, hi, E.base + i)) {
    cnt[i] = 0;
    big_flag[i] = 0;
    return;
  }
  long long n = cell_range(lo, hi, E.base + i, S.icell[sc], c0, c1);
  cnt[i] = n < 0 ? 0 : (int)n;
  big_flag[i] = n < 0 ? 1 : 0;
}

__global__ void entry_insert_kernel(PrimSet E, int ekind, const double* __restrict__ lo, const double* __restrict__ hi,
                                    SceneTab S, const int* __restrict__ offs, unsigned mask,
                                    unsigned long long* __restrict__ key, int* __restrict__ val,
                                    unsigned long long* __restrict__ ecell, int* __restrict__ eprim,
                                    int* __restrict__ ebody, const int* __restrict__ tris,
                                    const int* __restrict__ edges) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E.n) return;
  int c0[3], c1[3];
  int body = prim_body(ekind, i, tris, edges, S.sv_body);
  int sc = S.body_scene[body];
  if (!near_other_body(S, body, sc, lo, hi, E.base + i)) return;
  if (cell_range(lo, hi, E.base + i, S.icell[sc], c0, c1) < 0) return;
  int o = offs[i];
  for (int x = c0[0]; x <= c1[0]; ++x)
    for (int y = c0[1]; y <= c1[1]; ++y)
      for (int z = c0[2]; z <= c1[2]; ++z, ++o) {
        key[o] = hash3(x, y, z, sc, mask);
        val[o] = o;
        ecell[o] = pack_cell(x, y, z);
        eprim[o] = i;
        ebody[o] = body;
      }
}

__global__ void bucket_bounds_kernel(int n, const unsigned long long* __restrict__ skey, int* __restrict__ blo,
                                     int* __restrict__ bhi) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  unsigned h = (unsigned)skey[j];
  if (j == 0 || (unsigned)skey[j - 1] != h) blo[h] = j;
  if (j == n - 1 || (unsigned)skey[j + 1] != h) bhi[h] = j + 1;
}

// gather entry cell / prim into sorted order
// gather entry cell / prim / body and the entry's box into bucket order, so a query
// reads one bucket's entries from contiguous arrays without indirection
__global__ void entry_permute_kernel(int n, int ebase, const int* __restrict__ sval,
                                     const unsigned long long* __restrict__ ecell, const int* __restrict__ eprim,
                                     const int* __restrict__ ebody, const double* __restrict__ lo,
                                     const double* __restrict__ hi, unsigned long long* __restrict__ scell,
                                     int* __restrict__ sprim, int* __restrict__ sbody, double* __restrict__ sbox) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int o = sval[j];
  int e = eprim[o];
  scell[j] = ecell[o];
  sprim[j] = e;
  sbody[j] = ebody[o];
  int ei = ebase + e;
  for (int k = 0; k < 3; ++k) {
    sbox[6 * (size_t)j + k] = lo[3 * ei + k];
    sbox[6 * (size_t)j + 3 + k] = hi[3 * ei + k];
  }
}

// totals of two exclusive scans: out[0] = offs_a[na-1] + cnt_a[na-1], out[1] likewise
__global__ void totals_kernel(int na, const int* __restrict__ cnt_a, const int* __restrict__ offs_a, int nb,
                              const int* __restrict__ cnt_b, const int* __restrict__ offs_b, long long* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = na > 0 ? (long long)offs_a[na - 1] + cnt_a[na - 1] : 0;
  if (threadIdx.x == 1) out[1] = nb > 0 ? (long long)offs_b[nb - 1] + cnt_b[nb - 1] : 0;
}

struct PairRule {
  int qkind, ekind;  // 0 vertex, 1 triangle, 2 edge
  int same_set;      // edge-edge: report (q, e) only when q < e
};

// inter-body pairs of one scene, not both on fixed bodies
__device__ inline bool admissible(PairRule R, int q, int e, const int* tris, const int* edges, const SceneTab& S,
                                  const unsigned char* fixed) {
  if (R.same_set && !(q < e)) return false;
  int bq = prim_body(R.qkind, q, tris, edges, S.sv_body), be = prim_body(R.ekind, e, tris, edges, S.sv_body);
  if (bq == be) return false;
  if (S.body_scene[bq] != S.body_scene[be]) return false;
  if (fixed[bq] && fixed[be]) return false;
  return true;
}

__device__ inline void emit(unsigned long long key, unsigned long long* out, int* counter, int cap) {
  int k = atomicAdd(counter, 1);
  if (k < cap) out[k] = key;
}

// Queries run as (query, cell) work items: a count pass (0 for queries far from every
// other body, flagged when the box is large), a scan, an expansion writing the query of
// every item, and one thread per item walking that cell's bucket.
__global__ void query_count_kernel(PrimSet Q, PairRule R, const double* __restrict__ lo,
                                   const double* __restrict__ hi, SceneTab S, const int* __restrict__ tris,
                                   const int* __restrict__ edges, int* __restrict__ cnt, int* __restrict__ big) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q.n) return;
  int qi = Q.base + q;
  int c0[3], c1[3];
  const int bq = prim_body(R.qkind, q, tris, edges, S.sv_body);
  const int sq = S.body_scene[bq];
  cnt[q] = 0;
  big[q] = 0;
  if (!near_other_body(S, bq, sq, lo, hi, qi)) return;
  long long n = cell_range(lo, hi, qi, S.icell[sq], c0, c1);
  if (n < 0)
    big[q] = 1;
  else
    cnt[q] = (int)n;
}

__global__ void query_expand_kernel(int nq, const int* __restrict__ cnt, const int* __restrict__ off,
                                    int* __restrict__ item_q) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  int o = off[q];
  for (int t = 0; t < cnt[q]; ++t) item_q[o + t] = q;
}

__global__ void query_items_kernel(int nitems, PrimSet Q, PrimSet E, PairRule R, const double* __restrict__ lo,
                                   const double* __restrict__ hi, SceneTab S, unsigned mask,
                                   const int* __restrict__ item_q, const int* __restrict__ off,
                                   const int* __restrict__ blo, const int* __restrict__ bhi,
                                   const unsigned long long* __restrict__ scell, const int* __restrict__ sprim,
                                   const int* __restrict__ sbody, const double* __restrict__ sbox,
                                   const int* __restrict__ tris, const int* __restrict__ edges,
                                   const unsigned char* __restrict__ fixed, unsigned long long nE,
                                   unsigned long long* __restrict__ out, int* __restrict__ counter, int cap) {
  int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitems) return;
  const int q = item_q[it], t = it - off[q];
  const int qi = Q.base + q;
  const int bq = prim_body(R.qkind, q, tris, edges, S.sv_body);
  const int sq = S.body_scene[bq];
  const double inv_c = S.icell[sq];
  int c0[3], c1[3];
  cell_range(lo, hi, qi, inv_c, c0, c1);
  const int ny = c1[1] - c0[1] + 1, nz = c1[2] - c0[2] + 1;
  const int x = c0[0] + t / (ny * nz), y = c0[1] + (t / nz) % ny, z = c0[2] + t % nz;
  const double ql[3] = {lo[3 * qi], lo[3 * qi + 1], lo[3 * qi + 2]};
  const double qh[3] = {hi[3 * qi], hi[3 * qi + 1], hi[3 * qi + 2]};
  const unsigned h = hash3(x, y, z, sq, mask);
  const unsigned long long ck = pack_cell(x, y, z);
  const int j1 = bhi[h];
  for (int j = blo[h]; j < j1; ++j) {
    const int be = sbody[j];
    if (be == bq || scell[j] != ck) continue;  // same body, or another cell in this bucket
    if (S.body_scene[be] != sq || (fixed[bq] && fixed[be])) continue;
    const int e = sprim[j];
    if (R.same_set && !(q < e)) continue;
    const double* eb = sbox + 6 * (size_t)j;
    bool ov = true;
    for (int k = 0; k < 3; ++k) ov = ov && eb[k] <= qh[k] && ql[k] <= eb[3 + k];
    if (!ov) continue;
    // report only from the cell holding max(lo_q, lo_e)
    if (cell_of(fmax(ql[0], eb[0]), inv_c) != x || cell_of(fmax(ql[1], eb[1]), inv_c) != y ||
        cell_of(fmax(ql[2], eb[2]), inv_c) != z)
      continue;
    emit((unsigned long long)q * nE + e, out, counter, cap);
  }
}

// large query boxes: test every small entry directly (for a shared set every pair with
// a large member is reported by big_entry_kernel)
__global__ void query_big_kernel(PrimSet Q, PrimSet E, PairRule R, const double* __restrict__ lo,
                                 const double* __restrict__ hi, SceneTab S, const int* __restrict__ qbig,
                                 const int* __restrict__ ebig, const int* __restrict__ tris,
                                 const int* __restrict__ edges, const unsigned char* __restrict__ fixed,
                                 unsigned long long nE, unsigned long long* __restrict__ out, int* __restrict__ counter,
                                 int cap) {
  if (R.same_set) return;
  for (int q = blockIdx.x; q < Q.n; q += gridDim.x) {
    if (!qbig[q]) continue;
    for (int e = threadIdx.x; e < E.n; e += blockDim.x) {
      if (ebig[e]) continue;
      if (!admissible(R, q, e, tris, edges, S, fixed)) continue;
      if (overlap(lo, hi, Q.base + q, E.base + e)) emit((unsigned long long)q * nE + e, out, counter, cap);
    }
  }
}

// large entries: test against every query primitive (for a shared set only pairs
// not already covered: the other primitive small, or large with a larger id)
__global__ void big_entry_kernel(PrimSet Q, PrimSet E, PairRule R, const double* __restrict__ lo,
                                 const double* __restrict__ hi, const int* __restrict__ ebig,
                                 const int* __restrict__ tris, const int* __restrict__ edges, SceneTab S,
                                 const unsigned char* __restrict__ fixed,
                                 unsigned long long nE, unsigned long long* __restrict__ out, int* __restrict__ counter,
                                 int cap) {
  for (int e = blockIdx.x; e < E.n; e += gridDim.x) {
  if (!ebig[e]) continue;
  for (int q = threadIdx.x; q < Q.n; q += blockDim.x) {
    if (R.same_set) {
      if (q == e) continue;
      int a = q < e ? q : e, b = q < e ? e : q;
      if (ebig[q] && !(e < q)) continue;  // both large: reported by the smaller id
      if (!admissible(R, a, b, tris, edges, S, fixed)) continue;
      if (overlap(lo, hi, Q.base + q, E.base + e)) emit((unsigned long long)a * nE + b, out, counter, cap);
    } else {
      if (!admissible(R, q, e, tris, edges, S, fixed)) continue;
      if (overlap(lo, hi, Q.base + q, E.base + e)) emit((unsigned long long)q * nE + e, out, counter, cap);
    }
  }
  }
}

__global__ void decode_pairs_kernel(int n, const unsigned long long* __restrict__ k, unsigned long long nE,
                                    int* __restrict__ out) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  out[2 * j] = (int)(k[j] / nE);
  out[2 * j + 1] = (int)(k[j] % nE);
}

static int bits_for(unsigned long long v) {
  int b = 0;
  while (b < 64 && (v >> b)) ++b;
  return b;
}

// boxes of whole bodies from the current primitive boxes
static void body_boxes(zema_scene* s) {
  int nb = std::max(s->n_bodies, 1);
  s->body_blo.reserve(3 * (size_t)nb);
  s->body_bhi.reserve(3 * (size_t)nb);
  ZCHK(hipMemsetAsync(s->body_blo.p, 0xff, sizeof(unsigned long long) * 3 * nb, s->st));
  ZCHK(hipMemsetAsync(s->body_bhi.p, 0, sizeof(unsigned long long) * 3 * nb, s->st));
  if (s->nsurf)
    body_box_kernel<<<nblocks(s->nsurf), kBlock, 0, s->st>>>(s->nsurf, s->bb_lo.p, s->bb_hi.p, s->sv_body.p,
                                                             s->body_blo.p, s->body_bhi.p);
}

// One candidate search (PT or EE); result sorted into out (n x 2 ints).
static int64_t search(zema_scene* s, PrimSet Q, PrimSet E, PairRule R, DBuf<int>& out) {
  if (Q.n == 0 || E.n == 0) {
    out.resize(0);
    return 0;
  }
  const SceneTab S{s->sv_body.p,     s->body_scene.p, s->icell_sc.p, s->scene_bodies.p,
                   s->body_blo.p,     s->body_bhi.p,   s->act_dev()};
  s->cnt.reserve(E.n + 1);
  s->offs.reserve(E.n + 1);
  s->big_list.reserve(E.n + 1);
  s->q_cnt.reserve(Q.n + 1);
  s->q_off.reserve(Q.n + 1);
  s->q_big.reserve(Q.n + 1);
  // entry cells and query work items are counted and scanned together, their totals
  // read back in one transfer
  entry_count_kernel<<<nblocks(E.n), kBlock, 0, s->st>>>(E, R.ekind, s->bb_lo.p, s->bb_hi.p, S, s->tris.p, s->edges.p,
                                                         s->cnt.p, s->big_list.p);
  query_count_kernel<<<nblocks(Q.n), kBlock, 0, s->st>>>(Q, R, s->bb_lo.p, s->bb_hi.p, S, s->tris.p, s->edges.p,
                                                         s->q_cnt.p, s->q_big.p);
  k_exclusive_scan(s, s->cnt.p, s->offs.p, E.n, false);
  k_exclusive_scan(s, s->q_cnt.p, s->q_off.p, Q.n, false);
  long long tot2[2];
  s->tot_dev.reserve(2);
  totals_kernel<<<1, 64, 0, s->st>>>(E.n, s->cnt.p, s->offs.p, Q.n, s->q_cnt.p, s->q_off.p, s->tot_dev.p);
  ZCHK(hipMemcpyAsync(tot2, s->tot_dev.p, sizeof(tot2), hipMemcpyDeviceToHost, s->st));
  ZCHK(hipStreamSynchronize(s->st));
  const int64_t total = tot2[0], nitems = tot2[1];
  unsigned tsize = 1024;
  while (tsize < 2 * total) tsize <<= 1;
  unsigned mask = tsize - 1;
  SortBufs& sb = s->sort;
  sb.k0.reserve(total + 1);
  sb.v0.reserve(total + 1);
  s->ent_cell.reserve(2 * total + 2);
  s->ent_prim.reserve(2 * total + 2);
  s->ent_body.reserve(2 * total + 2);
  s->bucket_lo.reserve(tsize);
  s->bucket_hi.reserve(tsize);
  if (total > 0) {
    entry_insert_kernel<<<nblocks(E.n), kBlock, 0, s->st>>>(E, R.ekind, s->bb_lo.p, s->bb_hi.p, S, s->offs.p, mask,
                                                            sb.k0.p, sb.v0.p, s->ent_cell.p, s->ent_prim.p,
                                                            s->ent_body.p, s->tris.p, s->edges.p);
    k_radix_sort(s, sb, total, bits_for(mask));
    // sorted copies live in the second halves of ent_cell / ent_prim
    s->ent_box.reserve(6 * (size_t)total + 6);
    entry_permute_kernel<<<nblocks(total), kBlock, 0, s->st>>>((int)total, E.base, sb.v0.p, s->ent_cell.p,
                                                               s->ent_prim.p, s->ent_body.p, s->bb_lo.p, s->bb_hi.p,
                                                               s->ent_cell.p + total, s->ent_prim.p + total,
                                                               s->ent_body.p + total, s->ent_box.p);
  }
  ZCHK(hipMemsetAsync(s->bucket_lo.p, 0, sizeof(int) * tsize, s->st));
  ZCHK(hipMemsetAsync(s->bucket_hi.p, 0, sizeof(int) * tsize, s->st));
  if (total > 0)
    bucket_bounds_kernel<<<nblocks(total), kBlock, 0, s->st>>>((int)total, sb.k0.p, s->bucket_lo.p, s->bucket_hi.p);
  unsigned long long nE = (unsigned long long)E.n;
  int* counter = s->counters.p;
  // query work items
  s->q_item.reserve(nitems + 1);
  if (nitems) query_expand_kernel<<<nblocks(Q.n), kBlock, 0, s->st>>>(Q.n, s->q_cnt.p, s->q_off.p, s->q_item.p);
  for (int attempt = 0; attempt < 2; ++attempt) {
    int cap = (int)std::min<size_t>(s->pair_keys.cap, (size_t)INT32_MAX);
    ZCHK(hipMemsetAsync(counter, 0, sizeof(int), s->st));
    kt_begin(s, KT_QUERY);
    if (nitems)
      query_items_kernel<<<nblocks(nitems), kBlock, 0, s->st>>>(
          (int)nitems, Q, E, R, s->bb_lo.p, s->bb_hi.p, S, mask, s->q_item.p, s->q_off.p, s->bucket_lo.p,
          s->bucket_hi.p, s->ent_cell.p + total, s->ent_prim.p + total, s->ent_body.p + total, s->ent_box.p,
          s->tris.p, s->edges.p, s->body_fixed.p, nE, s->pair_keys.p, counter, cap);
    kt_end(s, KT_QUERY);
    query_big_kernel<<<std::min(Q.n, 1024), kBlock, 0, s->st>>>(Q, E, R, s->bb_lo.p, s->bb_hi.p, S, s->q_big.p,
                                                                s->big_list.p, s->tris.p, s->edges.p,
                                                                s->body_fixed.p, nE, s->pair_keys.p, counter, cap);
    big_entry_kernel<<<std::min(E.n, 1024), kBlock, 0, s->st>>>(Q, E, R, s->bb_lo.p, s->bb_hi.p, s->big_list.p,
                                                                s->tris.p, s->edges.p, S, s->body_fixed.p, nE,
                                                                s->pair_keys.p, counter, cap);
    int n;
    ZCHK(hipMemcpyAsync(&n, counter, sizeof(int), hipMemcpyDeviceToHost, s->st));
    ZCHK(hipStreamSynchronize(s->st));
    if (n <= cap) {
      // sort the pair keys (values unused)
      sb.k0.reserve(n + 1);
      sb.v0.reserve(n + 1);
      if (n > 0) ZCHK(hipMemcpyAsync(sb.k0.p, s->pair_keys.p, sizeof(unsigned long long) * n,
                                     hipMemcpyDeviceToDevice, s->st));
      k_radix_sort(s, sb, n, bits_for((unsigned long long)Q.n * nE));
      out.resize((size_t)2 * n);
      if (n > 0) decode_pairs_kernel<<<nblocks(n), kBlock, 0, s->st>>>(n, sb.k0.p, nE, out.p);
      return n;
    }
    s->pair_keys.reserve((size_t)n + n / 4 + 1024);
  }
  throw Error(ZEMA_E_CAPACITY, "candidate buffer growth failed");
}

// inter-body (edge, triangle) pairs whose exact (uninflated) boxes overlap at xs
int64_t k_edge_tri_pairs(zema_scene* s, const double* xs, DBuf<int>& out) {
  int nv = s->nsurf, nt = s->ntri, ne = s->nedge;
  int np = nv + nt + ne;
  s->bb_lo.reserve(3 * (size_t)np);
  s->bb_hi.reserve(3 * (size_t)np);
  if (s->pair_keys.cap < 4096) s->pair_keys.reserve(1 << 16);
  if (np)
    boxes_kernel<<<nblocks(np), kBlock, 0, s->st>>>(nv, nt, ne, s->tris.p, s->edges.p, xs, xs, nullptr, 0.0, s->bb_lo.p,
                                                    s->bb_hi.p);
  body_boxes(s);
  return search(s, PrimSet{nv + nt, ne}, PrimSet{nv, nt}, PairRule{2, 1, 0}, out);
}

void k_candidates(zema_scene* s, const double* xs0, const double* xs1, double r, const double* xs2) {
  int nv = s->nsurf, nt = s->ntri, ne = s->nedge;
  int np = nv + nt + ne;
  s->bb_lo.reserve(3 * (size_t)np);
  s->bb_hi.reserve(3 * (size_t)np);
  if (s->pair_keys.cap < 4096) s->pair_keys.reserve(1 << 16);
  if (np)
    boxes_kernel<<<nblocks(np), kBlock, 0, s->st>>>(nv, nt, ne, s->tris.p, s->edges.p, xs0, xs1 ? xs1 : xs0, xs2, r,
                                                    s->bb_lo.p, s->bb_hi.p);
  body_boxes(s);
  s->npt = search(s, PrimSet{0, nv}, PrimSet{nv, nt}, PairRule{0, 1, 0}, s->pt);
  s->nee = search(s, PrimSet{nv + nt, ne}, PrimSet{nv + nt, ne}, PairRule{2, 2, 1}, s->ee);
}

}  // namespace zema

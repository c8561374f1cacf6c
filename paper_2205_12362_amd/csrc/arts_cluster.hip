// DM-width clustering of threshold candidates on the GPU (Sect. 6b.2, "Clustering"): the
// candidates that one plan appended to a device list are replaced, in place, by one candidate
// per cluster.
//
// A candidate (beam b, DM index d, width w, sample t) covers the boxcar window [t, t + w - 1].
// Step 1 groups, within one (b, d) row, candidates whose windows overlap (transitively); a
// group covers the union of its windows, an interval.  Step 2 joins groups of rows (b, d) and
// (b, d + 1) whose intervals overlap, again transitively.  Each resulting cluster reports its
// member with the highest S/N, ties to the lowest d, then the earliest t, then the smallest w.
//
// Device pipeline (all launches on one stream, no host round trip):
//   init     zero the per-row counters; read the list range [beg, end) from the device
//   count    candidates per row (atomics)
//   scan     row offsets (tile sums, then tile scans); the list is truncated to beg
//   scatter  copy the candidates into row-grouped scratch
//   rows     per row: sort by (t, w) and form the step-1 groups, one group per slot: rows of
//            up to 64 candidates in the registers of one wave, longer ones in LDS or in place
//   link     union-find over the groups of neighbouring rows (lock-free CAS hooking)
//   best     per cluster root: max over its groups of the packed (S/N, position) key
//   rank     prefix sum over the root flags (tile sums, then tile scans)
//   emit     each root's best candidate to the list at beg + its rank
// The list is left as it was if the range holds more than `cap` candidates (overflowed
// appends), or a record is invalid (beam or DM index outside the plan, width < 1, NaN S/N).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "arts_internal.h"

namespace arts {

namespace {

constexpr int kClThreads = 256;    // grid-stride kernels
constexpr int kClRowThreads = 64;  // one wave per row
constexpr int kClRowLds = 256;     // long rows of up to this many candidates are sorted in LDS
constexpr int kScanPer = 8;        // rows per scan thread (two 16-byte loads)
constexpr int kScanTile = kClThreads * kScanPer;

struct ClHead {
  long long beg, n;
  int skip, bad;
  int nbig, pad;  // rows longer than one wave, listed for the long-row kernel
};

__device__ __forceinline__ int32_t wave_sum(int32_t v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

// Sum over a 256-thread workgroup, returned to every thread.
__device__ int32_t block_sum(int32_t v) {
  __shared__ int32_t ws[kClThreads / 64];
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  int32_t t = 0;
  for (int i = 0; i < kClThreads / 64; ++i) t += ws[i];
  return t;
}

__device__ __forceinline__ uint32_t snr_key(float f) {
  if (f == 0.0f) f = 0.0f;  // -0 and +0 compare equal
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// (sample, width) order of a row
__device__ __forceinline__ bool before(const arts_candidate& a, const arts_candidate& b) {
  return a.sample < b.sample || (a.sample == b.sample && a.width < b.width);
}

__device__ __forceinline__ int load_rel(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x, halving the path on the way (every pointer written is an ancestor of x).
__device__ int find_root(int* parent, int x) {
  while (true) {
    const int p = load_rel(parent + x);
    if (p == x) return x;
    const int g = load_rel(parent + p);
    if (g != p) atomicCAS(parent + x, p, g);
    x = g;
  }
}

// Join the trees of a and b: the larger root is hooked under the smaller one.  A failed CAS
// means that root was hooked meanwhile; retry from the new roots.
__device__ void unite(int* parent, int a, int b) {
  while (true) {
    a = find_root(parent, a);
    b = find_root(parent, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(parent + a, a, b) == a) return;
  }
}

__global__ __launch_bounds__(kClThreads) void cl_init_kernel(
    int32_t* rowcnt, int64_t nrows, const unsigned long long* count,
    const unsigned long long* mark, int64_t cap, ClHead* h) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < nrows;
       r += stride)
    rowcnt[r] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const long long end = static_cast<long long>(*count);
    const long long beg = mark ? static_cast<long long>(*mark) : 0;
    h->beg = beg;
    h->n = end - beg;
    h->skip = (end > cap || beg > end) ? 1 : 0;
    h->bad = 0;
    h->nbig = 0;
  }
}

__global__ __launch_bounds__(kClThreads) void cl_count_kernel(
    const arts_candidate* __restrict__ cand, ClHead* h, int32_t nbeam, int32_t ndm,
    int32_t beam_offset, int32_t* rowcnt) {
  if (h->skip) return;
  const long long beg = h->beg, n = h->n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    const arts_candidate& c = cand[beg + i];
    const int b = c.beam - beam_offset;
    if (b < 0 || b >= nbeam || c.dm_index < 0 || c.dm_index >= ndm || c.width < 1 ||
        c.snr != c.snr) {
      atomicOr(&h->bad, 1);
      continue;
    }
    atomicAdd(rowcnt + static_cast<int64_t>(b) * ndm + c.dm_index, 1);
  }
}

// Exclusive prefix sum of rowcnt [nrows] into rowoff [nrows + 1] and cursor [nrows], in tiles
// of kScanTile rows: the first kernel sums each tile, the second adds the sums of the tiles
// before its own and scans the tile (each thread owns kScanPer consecutive rows).
__device__ __forceinline__ void load_counts(const int32_t* rowcnt, int64_t nrows, int64_t base,
                                            int32_t (&v)[kScanPer]) {
  if (base + kScanPer <= nrows) {
    const int4 a = *reinterpret_cast<const int4*>(rowcnt + base);
    const int4 b = *reinterpret_cast<const int4*>(rowcnt + base + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
    for (int k = 0; k < kScanPer; ++k) v[k] = base + k < nrows ? rowcnt[base + k] : 0;
  }
}

// DEV: the length is the candidate count on the device (the root flags); otherwise nrows.
template <bool DEV>
__global__ __launch_bounds__(kClThreads) void cl_scan_part_kernel(
    const int32_t* __restrict__ in, int64_t nrows, int32_t* __restrict__ part, const ClHead* h) {
  if (h->skip || h->bad) return;
  const int64_t n = DEV ? h->n : nrows;
  if (static_cast<int64_t>(blockIdx.x) * kScanTile >= n) return;
  int32_t v[kScanPer];
  load_counts(in, n, static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanPer, v);
  int32_t s = 0;
  for (int k = 0; k < kScanPer; ++k) s += v[k];
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Rows (DEV false): out = rowoff [nrows + 1], cursor = a copy, and the list is cut back to beg.
// Roots (DEV true): out = each root's rank among the roots; the list count becomes beg plus
// the number of roots.
template <bool DEV>
__global__ __launch_bounds__(kClThreads) void cl_scan_final_kernel(
    const int32_t* __restrict__ in, int64_t nrows, const int32_t* __restrict__ part,
    int32_t* __restrict__ out, int32_t* __restrict__ cursor, const ClHead* h,
    unsigned long long* count) {
  if (h->skip || h->bad) return;
  const int64_t n = DEV ? h->n : nrows;
  const int64_t ntile = (n + kScanTile - 1) / kScanTile;
  if (static_cast<int64_t>(blockIdx.x) >= ntile) return;
  __shared__ int32_t wtot[kClThreads / 64];
  int32_t before = 0;
  for (int i = threadIdx.x; i < static_cast<int>(blockIdx.x); i += kClThreads) before += part[i];
  before = block_sum(before);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanPer;
  int32_t v[kScanPer];
  load_counts(in, n, base, v);
  int32_t tot = 0;
  for (int k = 0; k < kScanPer; ++k) tot += v[k];
  // exclusive scan of the thread totals: within the wave, then across the 4 waves
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t inc = tot;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t u = __shfl_up(inc, off);
    if (lane >= off) inc += u;
  }
  if (lane == 63) wtot[wv] = inc;
  __syncthreads();
  int32_t run = before + inc - tot;
  for (int i = 0; i < wv; ++i) run += wtot[i];
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) {
      out[base + k] = run;
      if (!DEV) cursor[base + k] = run;
    }
    run += v[k];
  }
  const bool last = blockIdx.x == ntile - 1 && threadIdx.x == kClThreads - 1;
  if (DEV) {
    if (last) *count = static_cast<unsigned long long>(h->beg + run);
  } else {
    if (last) out[n] = run;
    if (blockIdx.x == 0 && threadIdx.x == 0)
      *count = static_cast<unsigned long long>(h->beg);  // emit appends the clusters from beg
  }
}

__global__ __launch_bounds__(kClThreads) void cl_scatter_kernel(
    const arts_candidate* __restrict__ cand, const ClHead* h, int32_t ndm, int32_t beam_offset,
    int32_t* cursor, arts_candidate* __restrict__ rec) {
  if (h->skip || h->bad) return;
  const long long beg = h->beg, n = h->n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    const arts_candidate c = cand[beg + i];
    const int64_t r = static_cast<int64_t>(c.beam - beam_offset) * ndm + c.dm_index;
    rec[atomicAdd(cursor + r, 1)] = c;
  }
}

// Bitonic sort of a[0, n) by (sample, width) with the all-ascending network (each merge opens
// with a mirrored compare), so that missing elements beyond n act as +infinity and are never
// touched.  `a` is LDS or global memory private to this workgroup.
__device__ void sort_row(arts_candidate* a, int n) {
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (int k = 2; k <= n2; k <<= 1) {
    for (int p = threadIdx.x; p < n2 / 2; p += blockDim.x) {
      const int half = k / 2, blk = p / half, off = p % half;
      const int i = blk * k + off, j = blk * k + k - 1 - off;
      if (j < n && before(a[j], a[i])) {
        const arts_candidate t = a[i];
        a[i] = a[j];
        a[j] = t;
      }
    }
    __syncthreads();
    for (int hd = k / 4; hd >= 1; hd >>= 1) {
      for (int p = threadIdx.x; p < n2 / 2; p += blockDim.x) {
        const int blk = p / hd, off = p % hd;
        const int i = blk * 2 * hd + off, j = i + hd;
        if (j < n && before(a[j], a[i])) {
          const arts_candidate t = a[i];
          a[i] = a[j];
          a[j] = t;
        }
      }
      __syncthreads();
    }
  }
}

// Step 1.  A row's candidates are sorted by (sample, width) and walked in that order: one whose
// window starts after everything the current group covers opens a new group.  Group g of row
// r lives in slot rowoff[r] + g: covered interval [gt0, gt1], best key (S/N in the high word,
// the complement of its sorted position in the low word, so that ties go to the earlier
// position), its row, and its union-find parent (itself); unused slots get grow = -1.
// perm[sorted position] is the scratch slot of the candidate at that position.

// Compare-exchange of the lane's record with lane ^ mask: the lower lane keeps the one that
// comes first in (sample, width, scratch slot) order, a strict total order.
__device__ __forceinline__ void cmpx(int64_t& t, int32_t& w, int32_t& idx, uint32_t& key,
                                     int mask) {
  const int lane = threadIdx.x & 63;
  const int64_t pt = __shfl_xor(t, mask);
  const int32_t pw = __shfl_xor(w, mask), pi = __shfl_xor(idx, mask);
  const uint32_t pk = static_cast<uint32_t>(__shfl_xor(static_cast<int>(key), mask));
  const bool pfirst = pt < t || (pt == t && (pw < w || (pw == w && pi < idx)));
  const bool lower = (lane & mask) == 0 || (lane ^ mask) > lane;
  if (lower == pfirst) {
    t = pt;
    w = pw;
    idx = pi;
    key = pk;
  }
}

// Rows of up to 64 candidates: one wave, one candidate per lane; bitonic sort across lanes, a
// prefix maximum of the window ends finds the group starts, LDS atomics the groups' best keys.
// Longer rows are listed for cl_rows_long_kernel.
__global__ __launch_bounds__(kClRowThreads) void cl_rows_kernel(
    ClHead* h, int64_t nrows, const int32_t* __restrict__ rowoff,
    const arts_candidate* __restrict__ rec, int32_t* __restrict__ gcnt, int64_t* __restrict__ gt0,
    int64_t* __restrict__ gt1, unsigned long long* __restrict__ gkey,
    unsigned long long* __restrict__ bkey, int32_t* __restrict__ parent,
    int32_t* __restrict__ grow, int32_t* __restrict__ perm, int32_t* __restrict__ big) {
  if (h->skip || h->bad) return;
  __shared__ unsigned long long s_key[kClRowThreads];
  const int lane = threadIdx.x;
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int o = rowoff[r], n = rowoff[r + 1] - o;
    if (n > kClRowThreads) {
      if (lane == 0) big[atomicAdd(&h->nbig, 1)] = static_cast<int32_t>(r);
      continue;
    }
    if (n == 0) {
      if (lane == 0) gcnt[r] = 0;
      continue;
    }
    const bool act = lane < n;
    int64_t t = LLONG_MAX;
    int32_t w = INT_MAX, idx = o + lane;
    uint32_t key = 0;
    if (act) {
      const arts_candidate& c = rec[o + lane];
      t = c.sample;
      w = c.width;
      key = snr_key(c.snr);
    }
    int n2 = 1;
    while (n2 < n) n2 <<= 1;
    for (int k = 2; k <= n2; k <<= 1) {
      cmpx(t, w, idx, key, k - 1);  // mirrored compare opens each merge
      for (int hd = k >> 2; hd >= 1; hd >>= 1) cmpx(t, w, idx, key, hd);
    }
    // lanes 0 .. n-1 now hold the row in order
    const int64_t e = act ? t + w - 1 : LLONG_MIN;
    int64_t m = e;  // inclusive prefix maximum of the window ends
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t u = __shfl_up(m, off);
      if (lane >= off) m = max(m, u);
    }
    int64_t ex = __shfl_up(m, 1);
    if (lane == 0) ex = LLONG_MIN;
    const bool first = act && t > ex;
    const unsigned long long fm = __ballot(first);
    const int g = __popcll(fm & (lane == 63 ? ~0ULL : ((2ULL << lane) - 1))) - 1;
    const int ng = __popcll(fm);
    const bool last = act && (lane == n - 1 || ((fm >> (lane + 1)) & 1ULL));
    if (lane < ng) s_key[lane] = 0;
    __syncthreads();
    if (act)
      atomicMax(s_key + g, (static_cast<unsigned long long>(key) << 32) |
                               (0xffffffffu - static_cast<uint32_t>(o + lane)));
    __syncthreads();
    if (first) {
      gt0[o + g] = t;
      gkey[o + g] = s_key[g];
    }
    if (last) gt1[o + g] = m;  // the group's largest end: earlier groups end before it starts
    if (act) {
      grow[o + lane] = lane < ng ? static_cast<int32_t>(r) : -1;
      parent[o + lane] = o + lane;
      bkey[o + lane] = 0;
      perm[o + lane] = idx;
    }
    if (lane == 0) gcnt[r] = ng;
    __syncthreads();
  }
}

// Rows longer than one wave: sorted in LDS (up to kClRowLds candidates) or in place in the
// scratch records, then walked by lane 0 in steps of 64 staged candidates.
__global__ __launch_bounds__(kClRowThreads) void cl_rows_long_kernel(
    const ClHead* h, const int32_t* __restrict__ big, const int32_t* __restrict__ rowoff,
    arts_candidate* __restrict__ rec, int32_t* __restrict__ gcnt, int64_t* __restrict__ gt0,
    int64_t* __restrict__ gt1, unsigned long long* __restrict__ gkey,
    unsigned long long* __restrict__ bkey, int32_t* __restrict__ parent,
    int32_t* __restrict__ grow, int32_t* __restrict__ perm) {
  if (h->skip || h->bad) return;
  __shared__ arts_candidate lds[kClRowLds];
  __shared__ int64_t st0[kClRowThreads], st1[kClRowThreads];
  __shared__ uint32_t skey[kClRowThreads];
  __shared__ int s_ng;
  const int tid = threadIdx.x;
  const int nbig = h->nbig;
  for (int bi = blockIdx.x; bi < nbig; bi += gridDim.x) {
    const int32_t r = big[bi];
    const int o = rowoff[r], n = rowoff[r + 1] - o;
    arts_candidate* a = rec + o;
    if (n <= kClRowLds) {
      for (int i = tid; i < n; i += kClRowThreads) lds[i] = a[i];
      __syncthreads();
      a = lds;
    }
    sort_row(a, n);
    // lane 0 walks the sorted row; the lanes stage 64 entries at a time
    int ng = 0, gbest = 0;
    int64_t g0 = 0, g1 = 0;
    uint32_t bk = 0;
    for (int base = 0; base < n; base += kClRowThreads) {
      const int i = base + tid;
      if (i < n) {
        st0[tid] = a[i].sample;
        st1[tid] = a[i].sample + a[i].width - 1;
        skey[tid] = snr_key(a[i].snr);
      }
      __syncthreads();
      if (tid == 0) {
        const int m = min(kClRowThreads, n - base);
        for (int q = 0; q < m; ++q) {
          const int k = base + q;
          if (k == 0 || st0[q] > g1) {
            if (k > 0) {  // close the previous group
              const int slot = o + ng - 1;
              gt0[slot] = g0;
              gt1[slot] = g1;
              gkey[slot] = (static_cast<unsigned long long>(bk) << 32) |
                           (0xffffffffu - static_cast<uint32_t>(o + gbest));
            }
            ++ng;
            g0 = st0[q];
            g1 = st1[q];
            bk = skey[q];
            gbest = k;
          } else {
            g1 = max(g1, st1[q]);
            if (skey[q] > bk) {
              bk = skey[q];
              gbest = k;
            }
          }
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      const int slot = o + ng - 1;
      gt0[slot] = g0;
      gt1[slot] = g1;
      gkey[slot] = (static_cast<unsigned long long>(bk) << 32) |
                   (0xffffffffu - static_cast<uint32_t>(o + gbest));
      gcnt[r] = ng;
      s_ng = ng;
    }
    __syncthreads();
    const int ngr = s_ng;
    if (a == lds)
      for (int i = tid; i < n; i += kClRowThreads) rec[o + i] = lds[i];
    for (int g = tid; g < n; g += kClRowThreads) {
      const int slot = o + g;
      grow[slot] = g < ngr ? r : -1;
      parent[slot] = slot;
      bkey[slot] = 0;
      perm[slot] = slot;  // sorted in place
    }
    __syncthreads();
  }
}

// Step 2: each group is joined with the groups of the next DM trial (same beam) whose interval
// overlaps its own.  A row's groups are sorted and disjoint, so those form one index range.
__global__ __launch_bounds__(kClThreads) void cl_link_kernel(
    const ClHead* h, int32_t ndm, const int32_t* __restrict__ rowoff,
    const int32_t* __restrict__ gcnt, const int64_t* __restrict__ gt0,
    const int64_t* __restrict__ gt1, const int32_t* __restrict__ grow, int32_t* parent) {
  if (h->skip || h->bad) return;
  const long long n = h->n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    const int32_t r = grow[i];
    if (r < 0 || r % ndm == ndm - 1) continue;
    const int lo0 = rowoff[r + 1], hi = lo0 + gcnt[r + 1];
    const int64_t a0 = gt0[i], a1 = gt1[i];
    int lo = lo0, up = hi;  // first group of the next row with gt1 >= a0
    while (lo < up) {
      const int mid = (lo + up) / 2;
      if (gt1[mid] < a0)
        lo = mid + 1;
      else
        up = mid;
    }
    for (int g = lo; g < hi && gt0[g] <= a1; ++g) unite(parent, static_cast<int>(i), g);
  }
}

// Per cluster root: the largest key of its groups.  Also flags the roots (final once the link
// kernel is done: roots are never hooked here).
__global__ __launch_bounds__(kClThreads) void cl_best_kernel(
    const ClHead* h, const int32_t* __restrict__ grow, const unsigned long long* __restrict__ gkey,
    int32_t* parent, unsigned long long* bkey, int32_t* __restrict__ rflag) {
  if (h->skip || h->bad) return;
  const long long n = h->n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    if (grow[i] < 0) {
      rflag[i] = 0;
      continue;
    }
    const int root = find_root(parent, static_cast<int>(i));
    rflag[i] = root == i ? 1 : 0;
    atomicMax(bkey + root, gkey[i]);
  }
}

// Each root writes its best candidate at beg + its rank among the roots, so the clusters come
// out in (beam, DM, sample, width) order of their groups.
__global__ __launch_bounds__(kClThreads) void cl_emit_kernel(
    const ClHead* h, const int32_t* __restrict__ rflag, const int32_t* __restrict__ rank,
    const unsigned long long* __restrict__ bkey, const int32_t* __restrict__ perm,
    const arts_candidate* __restrict__ rec, arts_candidate* __restrict__ cand) {
  if (h->skip || h->bad) return;
  const long long n = h->n, beg = h->beg;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    if (!rflag[i]) continue;
    const uint32_t pos = 0xffffffffu - static_cast<uint32_t>(bkey[i] & 0xffffffffu);
    cand[beg + rank[i]] = rec[perm[pos]];
  }
}

// Workspace layout: every array starts on a 256-byte boundary.
struct ClLayout {
  ClHead* head;
  unsigned long long* mark;
  int32_t *rowcnt, *rowoff, *cursor, *gcnt, *parent, *grow, *perm, *big, *part;
  int32_t *rflag, *rank, *part2;
  arts_candidate* rec;
  int64_t *gt0, *gt1;
  unsigned long long *gkey, *bkey;
  int64_t bytes;
};

template <typename T>
T* carve(uintptr_t base, int64_t& off, int64_t n) {
  T* q = reinterpret_cast<T*>(base + off);
  off += (n * static_cast<int64_t>(sizeof(T)) + 255) / 256 * 256;
  return q;
}

ClLayout layout(void* mem, int64_t cap, int64_t rows) {
  const uintptr_t b = reinterpret_cast<uintptr_t>(mem);
  int64_t off = 0;
  ClLayout l;
  l.head = carve<ClHead>(b, off, 1);
  l.mark = carve<unsigned long long>(b, off, 1);
  l.rowcnt = carve<int32_t>(b, off, rows);
  l.rowoff = carve<int32_t>(b, off, rows + 1);
  l.cursor = carve<int32_t>(b, off, rows);
  l.gcnt = carve<int32_t>(b, off, rows);
  l.big = carve<int32_t>(b, off, rows);
  l.part = carve<int32_t>(b, off, (rows + kScanTile - 1) / kScanTile);
  l.rec = carve<arts_candidate>(b, off, cap);
  l.gt0 = carve<int64_t>(b, off, cap);
  l.gt1 = carve<int64_t>(b, off, cap);
  l.gkey = carve<unsigned long long>(b, off, cap);
  l.bkey = carve<unsigned long long>(b, off, cap);
  l.parent = carve<int32_t>(b, off, cap);
  l.grow = carve<int32_t>(b, off, cap);
  l.perm = carve<int32_t>(b, off, cap);
  l.rflag = carve<int32_t>(b, off, cap);
  l.rank = carve<int32_t>(b, off, cap);
  l.part2 = carve<int32_t>(b, off, (cap + kScanTile - 1) / kScanTile);
  l.bytes = off;
  return l;
}

__global__ void cl_mark_kernel(const unsigned long long* count, unsigned long long* mark) {
  *mark = *count;
}

// ---------------------------------------------------------------- offline clustering
// Whole-observation clustering over time and DM windows: each kept candidate hashes its
// (time window, DM window) key into an open-addressing table (at most half full, so every
// probe sequence ends) and raises that slot's best (S/N, input order) key; one candidate per
// occupied slot is then written out.
constexpr unsigned long long kEmptyKey = ~0ULL;

struct OffHead {
  unsigned long long count;
  int bad, pad;
};

__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
  x ^= x >> 33;  // a 64-bit finaliser: spreads neighbouring windows over the table
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

__global__ __launch_bounds__(kClThreads) void off_init_kernel(unsigned long long* keys,
                                                               unsigned long long* best,
                                                               int64_t size, OffHead* h) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < size;
       i += stride) {
    keys[i] = kEmptyKey;
    best[i] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h->count = 0;
    h->bad = 0;
  }
}

__global__ __launch_bounds__(kClThreads) void off_insert_kernel(
    const arts_candidate* __restrict__ cand, int64_t n, int64_t t_window,
    const double* __restrict__ edges, int32_t nedge, float min_snr, unsigned long long* keys,
    unsigned long long* best, unsigned long long mask, OffHead* h) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    const arts_candidate c = cand[i];
    // native starts within +-2^42 keep the packed key below 2^63 (never the empty key)
    const int64_t lim = 1LL << 42;
    const bool sane = c.width >= 1 && c.downsample >= 1 && c.downsample < (1 << 20) &&
                      c.sample > -lim && c.sample < lim;
    const int64_t start = sane ? c.sample * c.downsample : 0;
    if (!sane || start <= -lim || start >= lim || c.snr != c.snr || c.dm != c.dm) {
      atomicOr(&h->bad, 1);
      continue;
    }
    const double dm = static_cast<double>(c.dm);
    if (dm < edges[0] || c.snr < min_snr) continue;
    const int64_t tw = start >= 0 ? start / t_window : -((-start + t_window - 1) / t_window);
    int lo = 0, hi = nedge;  // number of edges <= dm
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (edges[mid] <= dm)
        lo = mid + 1;
      else
        hi = mid;
    }
    const unsigned long long key =
        (static_cast<unsigned long long>(tw + (1LL << 42)) << 20) | static_cast<unsigned>(lo - 1);
    const unsigned long long val = (static_cast<unsigned long long>(snr_key(c.snr)) << 32) |
                                   (0xffffffffu - static_cast<uint32_t>(i));
    unsigned long long slot = mix64(key) & mask;
    while (true) {
      const unsigned long long prev = atomicCAS(keys + slot, kEmptyKey, key);
      if (prev == kEmptyKey || prev == key) {
        atomicMax(best + slot, val);
        break;
      }
      slot = (slot + 1) & mask;
    }
  }
}

__global__ __launch_bounds__(kClThreads) void off_emit_kernel(
    const arts_candidate* __restrict__ cand, const unsigned long long* __restrict__ keys,
    const unsigned long long* __restrict__ best, int64_t size, arts_candidate* __restrict__ out,
    OffHead* h) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < size;
       i += stride) {
    if (keys[i] == kEmptyKey) continue;
    const uint32_t idx = 0xffffffffu - static_cast<uint32_t>(best[i] & 0xffffffffu);
    out[atomicAdd(&h->count, 1ULL)] = cand[idx];
  }
}

}  // namespace

int64_t cluster_ws_bytes(int64_t cap, int64_t rows) { return layout(nullptr, cap, rows).bytes; }

int ensure_cluster_ws(ClusterWs& w, int64_t cap, int64_t rows) {
  if (cap < 1 || rows < 1) return fail(ARTS_E_INVAL, "clustering workspace: empty");
  if (cap >= INT_MAX || rows >= INT_MAX)
    return fail(ARTS_E_INVAL, "clustering: capacity and rows must stay below 2^31");
  if (w.d_mem && cap <= w.cap && rows <= w.rows) return ARTS_OK;
  free_cluster_ws(w);
  const int64_t bytes = layout(nullptr, cap, rows).bytes;
  ARTS_HIP(hipMalloc(&w.d_mem, bytes));
  w.cap = cap;
  w.rows = rows;
  w.bytes = bytes;
  return ARTS_OK;
}

void free_cluster_ws(ClusterWs& w) {
  if (w.d_mem) (void)hipFree(w.d_mem);
  w.d_mem = nullptr;
  w.cap = w.rows = w.bytes = 0;
}

int launch_cluster_mark(ClusterWs& w, const unsigned long long* count, hipStream_t s) {
  if (!w.d_mem) return fail(ARTS_E_STATE, "clustering workspace missing");
  const ClLayout l = layout(w.d_mem, w.cap, w.rows);
  (void)hipGetLastError();
  hipLaunchKernelGGL(cl_mark_kernel, dim3(1), dim3(1), 0, s, count, l.mark);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

int launch_cluster(ClusterWs& w, arts_candidate* cand, unsigned long long* count, int64_t cap,
                   bool from_mark, int32_t nbeam, int32_t ndm, int32_t beam_offset,
                   hipStream_t s) {
  const int64_t rows = static_cast<int64_t>(nbeam) * ndm;
  if (nbeam < 1 || ndm < 1) return fail(ARTS_E_INVAL, "clustering: nbeam, ndm >= 1");
  if (!w.d_mem || rows > w.rows || cap > w.cap)
    return fail(ARTS_E_STATE, "internal: clustering workspace not prepared");
  const ClLayout l = layout(w.d_mem, w.cap, w.rows);
  const unsigned gs = 1024;  // grid-stride kernels
  const unsigned grows = static_cast<unsigned>(std::min<int64_t>(rows, 16384));
  (void)hipGetLastError();
  hipLaunchKernelGGL(cl_init_kernel, dim3(gs), dim3(kClThreads), 0, s, l.rowcnt, rows, count,
                     from_mark ? l.mark : nullptr, cap, l.head);
  hipLaunchKernelGGL(cl_count_kernel, dim3(gs), dim3(kClThreads), 0, s, cand, l.head, nbeam, ndm,
                     beam_offset, l.rowcnt);
  const unsigned ntile = static_cast<unsigned>((rows + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(cl_scan_part_kernel<false>, dim3(ntile), dim3(kClThreads), 0, s, l.rowcnt,
                     rows, l.part, l.head);
  hipLaunchKernelGGL(cl_scan_final_kernel<false>, dim3(ntile), dim3(kClThreads), 0, s, l.rowcnt,
                     rows, l.part, l.rowoff, l.cursor, l.head, count);
  hipLaunchKernelGGL(cl_scatter_kernel, dim3(gs), dim3(kClThreads), 0, s, cand, l.head, ndm,
                     beam_offset, l.cursor, l.rec);
  hipLaunchKernelGGL(cl_rows_kernel, dim3(grows), dim3(kClRowThreads), 0, s, l.head, rows,
                     l.rowoff, l.rec, l.gcnt, l.gt0, l.gt1, l.gkey, l.bkey, l.parent, l.grow,
                     l.perm, l.big);
  hipLaunchKernelGGL(cl_rows_long_kernel, dim3(1024), dim3(kClRowThreads), 0, s, l.head, l.big,
                     l.rowoff, l.rec, l.gcnt, l.gt0, l.gt1, l.gkey, l.bkey, l.parent, l.grow,
                     l.perm);
  hipLaunchKernelGGL(cl_link_kernel, dim3(gs), dim3(kClThreads), 0, s, l.head, ndm, l.rowoff,
                     l.gcnt, l.gt0, l.gt1, l.grow, l.parent);
  hipLaunchKernelGGL(cl_best_kernel, dim3(gs), dim3(kClThreads), 0, s, l.head, l.grow, l.gkey,
                     l.parent, l.bkey, l.rflag);
  const unsigned ctile =
      static_cast<unsigned>(std::max<int64_t>(1, (cap + kScanTile - 1) / kScanTile));
  hipLaunchKernelGGL(cl_scan_part_kernel<true>, dim3(ctile), dim3(kClThreads), 0, s, l.rflag, 0,
                     l.part2, l.head);
  hipLaunchKernelGGL(cl_scan_final_kernel<true>, dim3(ctile), dim3(kClThreads), 0, s, l.rflag, 0,
                     l.part2, l.rank, nullptr, l.head, count);
  hipLaunchKernelGGL(cl_emit_kernel, dim3(gs), dim3(kClThreads), 0, s, l.head, l.rflag, l.rank,
                     l.bkey, l.perm, l.rec, cand);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

int read_cluster_status(ClusterWs& w, int* skipped, int* bad, hipStream_t s) {
  if (!w.d_mem) return fail(ARTS_E_STATE, "clustering workspace missing");
  const ClLayout l = layout(w.d_mem, w.cap, w.rows);
  ClHead h;
  ARTS_HIP(hipMemcpyAsync(&h, l.head, sizeof h, hipMemcpyDeviceToHost, s));
  ARTS_HIP(hipStreamSynchronize(s));
  *skipped = h.skip;
  *bad = h.bad;
  return ARTS_OK;
}

int64_t offline_table_size(int64_t n) {
  int64_t t = 1024;
  while (t < 2 * n) t <<= 1;
  return t;
}

int64_t offline_ws_bytes(int64_t n, int32_t nedge) {
  const int64_t t = offline_table_size(n);
  return 256 + (16 * t + 255) / 256 * 256 + (8LL * nedge + 255) / 256 * 256 +
         (static_cast<int64_t>(sizeof(arts_candidate)) * std::max<int64_t>(n, 1) + 255) / 256 * 256;
}

int launch_cluster_offline(const arts_candidate* cand, int64_t n, int64_t t_window,
                           const double* d_edges, int32_t nedge, float min_snr, void* ws,
                           arts_candidate** out, unsigned long long** d_count, int** d_bad,
                           hipStream_t s) {
  const int64_t t = offline_table_size(n);
  uint8_t* p = static_cast<uint8_t*>(ws);
  OffHead* h = reinterpret_cast<OffHead*>(p);
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(p + 256);
  unsigned long long* best = keys + t;
  *out = reinterpret_cast<arts_candidate*>(p + 256 + (16 * t + 255) / 256 * 256 +
                                           (8LL * nedge + 255) / 256 * 256);
  *d_count = &h->count;
  *d_bad = &h->bad;
  (void)hipGetLastError();
  hipLaunchKernelGGL(off_init_kernel, dim3(1024), dim3(kClThreads), 0, s, keys, best, t, h);
  if (n > 0) {
    hipLaunchKernelGGL(off_insert_kernel, dim3(1024), dim3(kClThreads), 0, s, cand, n, t_window,
                       d_edges, nedge, min_snr, keys, best,
                       static_cast<unsigned long long>(t - 1), h);
    hipLaunchKernelGGL(off_emit_kernel, dim3(1024), dim3(kClThreads), 0, s, cand, keys, best, t,
                       *out, h);
  }
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

// Where the offline workspace keeps the DM edges (after the table).
double* offline_edges(void* ws, int64_t n) {
  const int64_t t = offline_table_size(n);
  return reinterpret_cast<double*>(static_cast<uint8_t*>(ws) + 256 + (16 * t + 255) / 256 * 256);
}

}  // namespace arts

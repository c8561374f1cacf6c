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
//   scan     row offsets (one workgroup); the list is truncated to beg
//   scatter  copy the candidates into row-sorted scratch
//   rows     per row: sort by (t, w) and form the step-1 groups; one group per slot
//   link     union-find over the groups of neighbouring rows (lock-free CAS hooking)
//   best     per cluster root: max over its groups of the packed (S/N, position) key
//   emit     append each root's best candidate to the list
// The list is left as it was if the range holds more than `cap` candidates (overflowed
// appends), or a record is invalid (beam or DM index outside the plan, width < 1, NaN S/N).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "arts_internal.h"

namespace arts {

namespace {

constexpr int kClThreads = 256;  // grid-stride kernels
constexpr int kClRowThreads = 64;  // one wave per row
constexpr int kClRowLds = 256;   // rows of up to this many candidates are sorted in LDS
constexpr int kClScanThreads = 1024;

struct ClHead {
  long long beg, n;
  int skip, bad;
};

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

// Exclusive prefix sum of rowcnt [nrows] into rowoff [nrows + 1] and cursor [nrows]; one
// workgroup, each thread owning a contiguous span of rows.
__global__ __launch_bounds__(kClScanThreads) void cl_scan_kernel(
    const int32_t* __restrict__ rowcnt, int64_t nrows, int32_t* __restrict__ rowoff,
    int32_t* __restrict__ cursor, ClHead* h, unsigned long long* count) {
  if (h->skip || h->bad) return;
  __shared__ int32_t part[kClScanThreads];
  const int tid = threadIdx.x;
  const int64_t span = (nrows + kClScanThreads - 1) / kClScanThreads;
  const int64_t r0 = tid * span, r1 = min(nrows, r0 + span);
  int32_t s = 0;
  for (int64_t r = r0; r < r1; ++r) s += rowcnt[r];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < kClScanThreads; off <<= 1) {  // Hillis-Steele inclusive scan
    const int32_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int32_t run = part[tid] - s;
  for (int64_t r = r0; r < r1; ++r) {
    rowoff[r] = run;
    cursor[r] = run;
    run += rowcnt[r];
  }
  if (tid == kClScanThreads - 1) {
    rowoff[nrows] = part[tid];
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

// Step 1, one wave per row: sort the row's candidates, then walk them in order.  A candidate
// whose window starts after everything the current group covers opens a new group.  Group g of
// row r lives in slot rowoff[r] + g: covered interval [gt0, gt1], best key (S/N in the high
// word, the complement of its sorted position in the low word, so ties go to the earlier
// position), its row, and its union-find parent (itself).  Unused slots get grow = -1.
__global__ __launch_bounds__(kClRowThreads) void cl_rows_kernel(
    const ClHead* h, int64_t nrows, const int32_t* __restrict__ rowoff,
    arts_candidate* __restrict__ rec, int32_t* __restrict__ gcnt, int64_t* __restrict__ gt0,
    int64_t* __restrict__ gt1, unsigned long long* __restrict__ gkey,
    unsigned long long* __restrict__ bkey, int32_t* __restrict__ parent,
    int32_t* __restrict__ grow) {
  if (h->skip || h->bad) return;
  __shared__ arts_candidate lds[kClRowLds];
  __shared__ int64_t st0[kClRowThreads], st1[kClRowThreads];
  __shared__ uint32_t skey[kClRowThreads];
  __shared__ int s_ng;
  const int tid = threadIdx.x;
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int o = rowoff[r], n = rowoff[r + 1] - o;
    if (n == 0) {
      if (tid == 0) gcnt[r] = 0;
      continue;
    }
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
      grow[slot] = g < ngr ? static_cast<int32_t>(r) : -1;
      parent[slot] = slot;
      bkey[slot] = 0;
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

__global__ __launch_bounds__(kClThreads) void cl_best_kernel(
    const ClHead* h, const int32_t* __restrict__ grow, const unsigned long long* __restrict__ gkey,
    int32_t* parent, unsigned long long* bkey) {
  if (h->skip || h->bad) return;
  const long long n = h->n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    if (grow[i] < 0) continue;
    atomicMax(bkey + find_root(parent, static_cast<int>(i)), gkey[i]);
  }
}

__global__ __launch_bounds__(kClThreads) void cl_emit_kernel(
    const ClHead* h, const int32_t* __restrict__ grow, const int32_t* __restrict__ parent,
    const unsigned long long* __restrict__ bkey, const arts_candidate* __restrict__ rec,
    arts_candidate* __restrict__ cand, unsigned long long* count) {
  if (h->skip || h->bad) return;
  const long long n = h->n;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    if (grow[i] < 0 || parent[i] != i) continue;
    const uint32_t pos = 0xffffffffu - static_cast<uint32_t>(bkey[i] & 0xffffffffu);
    cand[atomicAdd(count, 1ULL)] = rec[pos];
  }
}

// Workspace layout: every array starts on a 256-byte boundary.
struct ClLayout {
  ClHead* head;
  unsigned long long* mark;
  int32_t *rowcnt, *rowoff, *cursor, *gcnt, *parent, *grow;
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
  l.rec = carve<arts_candidate>(b, off, cap);
  l.gt0 = carve<int64_t>(b, off, cap);
  l.gt1 = carve<int64_t>(b, off, cap);
  l.gkey = carve<unsigned long long>(b, off, cap);
  l.bkey = carve<unsigned long long>(b, off, cap);
  l.parent = carve<int32_t>(b, off, cap);
  l.grow = carve<int32_t>(b, off, cap);
  l.bytes = off;
  return l;
}

__global__ void cl_mark_kernel(const unsigned long long* count, unsigned long long* mark) {
  *mark = *count;
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
  hipLaunchKernelGGL(cl_scan_kernel, dim3(1), dim3(kClScanThreads), 0, s, l.rowcnt, rows,
                     l.rowoff, l.cursor, l.head, count);
  hipLaunchKernelGGL(cl_scatter_kernel, dim3(gs), dim3(kClThreads), 0, s, cand, l.head, ndm,
                     beam_offset, l.cursor, l.rec);
  hipLaunchKernelGGL(cl_rows_kernel, dim3(grows), dim3(kClRowThreads), 0, s, l.head, rows,
                     l.rowoff, l.rec, l.gcnt, l.gt0, l.gt1, l.gkey, l.bkey, l.parent, l.grow);
  hipLaunchKernelGGL(cl_link_kernel, dim3(gs), dim3(kClThreads), 0, s, l.head, ndm, l.rowoff,
                     l.gcnt, l.gt0, l.gt1, l.grow, l.parent);
  hipLaunchKernelGGL(cl_best_kernel, dim3(gs), dim3(kClThreads), 0, s, l.head, l.grow, l.gkey,
                     l.parent, l.bkey);
  hipLaunchKernelGGL(cl_emit_kernel, dim3(gs), dim3(kClThreads), 0, s, l.head, l.grow, l.parent,
                     l.bkey, l.rec, cand, count);
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

}  // namespace arts

// Streaming search: chunks of Stokes-I data arrive one by one (the real-time search processes
// 1.024 s chunks, Sect. 6b.2; the S/N is based on those 1.024 s, Sect. 6b.1).  The stream keeps
// the previous samples every trial still needs (the overlap, or halo) resident in device memory,
// so a chunk's search sees exactly the data a one-shot search of the concatenated series sees.
//
// Layout: native plans (D = 1) share one uint8 ring of nsrc * nchan rows holding Hmax + chunk
// samples (Hmax the largest of their halos; the row pitch W is rounded up to a multiple of 4 so
// rows stay dword-aligned); plan p reads each row's last H_p + chunk samples.  Each downsampled
// plan (D > 1) has its own 16-bit ring of rows of halo_p + chunk / D sums (even pitch).
// Every ring exists twice and the two copies alternate: a push copies the overlap out of the
// previous copy and appends the new chunk (downsampled for the 16-bit rings) to the other.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "arts_internal.h"

using namespace arts;

namespace {

constexpr uint32_t kGraph = 1u, kProfile = 2u;

int nphases(const arts_stream_s* s) { return static_cast<int>(s->plans.size()) + 2; }

void stream_free(arts_stream_s* s) {
  if (!s) return;
  if (s->hs) (void)hipStreamSynchronize(s->hs);
  for (auto& kv : s->graphs)
    if (kv.second) (void)hipGraphExecDestroy(kv.second);
  for (auto* r : s->ring)
    if (r) (void)hipFree(r);
  for (auto& v : s->ring16)
    for (auto* r : v)
      if (r) (void)hipFree(r);
  if (s->input) (void)hipFree(s->input);
  for (auto* p : s->series)
    if (p) (void)hipFree(p);
  for (auto* y : s->ybuf)
    if (y) (void)hipFree(y);
  if (s->d_cand) (void)hipFree(s->d_cand);
  if (s->d_count) (void)hipFree(s->d_count);
  if (s->h_count) (void)hipHostFree(s->h_count);
  if (s->d_flags) (void)hipFree(s->d_flags);
  free_cluster_ws(s->cl);
  if (s->rfi_ws) (void)hipFree(s->rfi_ws);
  for (auto e : s->pev)
    if (e) (void)hipEventDestroy(e);
  if (s->ev_in) (void)hipEventDestroy(s->ev_in);
  if (s->ev_done) (void)hipEventDestroy(s->ev_done);
  if (s->hs) (void)hipStreamDestroy(s->hs);
  delete s;
}

int dev_alloc(arts_stream_s* s, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? ARTS_E_NOMEM : ARTS_E_DEVICE,
                "stream allocation of %zu bytes: %s", bytes, hipGetErrorString(e));
  s->device_bytes += static_cast<int64_t>(bytes);
  return ARTS_OK;
}

// Step-1 row layout of a subband plan in a stream: L1 = halo + chunk - max step-1 delay samples
// per window, a front pad that puts each chunk's new rows 8-byte aligned, and room for the
// window to move m = 2 floor(L1 / chunk) chunks (at least 1) before it is compacted back to
// the front (the copy then never overlaps: it starts (m + 1) chunks in, past the L1 - chunk
// samples kept).
struct YLayout {
  int64_t l1 = 0, pitch = 0, rows = 0;
  int32_t pad = 0, m = 0;
};

YLayout y_layout(const arts_plan_s* pl, int32_t nbeam, int64_t chunk) {
  YLayout y;
  if (pl->nsub == 0) return y;
  const int64_t H = static_cast<int64_t>(pl->ds) * pl->halo;
  y.l1 = H + chunk - pl->max_d1;
  const int64_t keep = y.l1 - chunk;
  y.pad = static_cast<int32_t>((4 - keep % 4) % 4);
  // m moves between copies: twice the fewest that keep the copy from overlapping itself, so
  // that the copy runs half as often for the memory of m - l1 / chunk more chunks
  y.m = static_cast<int32_t>(std::max<int64_t>(1, 2 * (y.l1 / chunk)));
  y.pitch = (y.pad + y.l1 + y.m * chunk + 3) & ~int64_t(3);
  y.rows = static_cast<int64_t>(nbeam) * pl->nsub * pl->ncoarse;
  return y;
}
}  // namespace

// Phases of one push, reused by the serving engine (which batches the dedispersion of many
// streams into one launch).  All enqueue on `hs`.
namespace arts {

int stream_advance(arts_stream_s* s, int parity, hipStream_t hs) {
  if (s->rfi_ws && (s->rfi_nt > 0 || s->rfi_nf > 0))  // clean the new chunk before it is used
    if (int st = launch_rfi(s->input, s->nsrc, s->nchan, s->chunk, s->chunk, s->rfi_kt,
                            s->rfi_nt, s->rfi_kf, s->rfi_nf, s->rfi_ws, hs))
      return st;
  uint8_t* dst = s->ring[parity];
  const uint8_t* src = s->ring[parity ^ 1];
  const int64_t rows = static_cast<int64_t>(s->nsrc) * s->nchan;
  const int64_t ring_bytes = rows * s->W;
  if (dst) {
    if (int st = launch_copy_rows(dst, s->W, src + s->chunk, s->W, rows, s->hmax, src,
                                  src + ring_bytes, hs))
      return st;
    if (int st = launch_copy_rows(dst + s->hmax, s->W, s->input, s->chunk, rows, s->chunk,
                                  s->input, s->input + rows * s->chunk, hs))
      return st;
  }
  for (size_t p = 0; p < s->plans.size(); ++p) {
    uint16_t* d16 = s->ring16[parity][p];
    if (!d16) continue;
    const uint16_t* s16 = s->ring16[parity ^ 1][p];
    const int32_t D = s->plans[p]->ds;
    const int64_t W16 = s->W16[p], new16 = s->chunk / D, keep = s->N16[p] - new16;
    const uint8_t* sb = reinterpret_cast<const uint8_t*>(s16);
    if (int st = launch_copy_rows(reinterpret_cast<uint8_t*>(d16), 2 * W16, sb + 2 * new16,
                                  2 * W16, rows, 2 * keep, sb, sb + rows * W16 * 2, hs))
      return st;
    if (int st = launch_downsample(d16 + keep, W16, s->input, s->chunk, rows, new16, D, hs))
      return st;
  }
  return ARTS_OK;
}

// Device bytes arts_stream_create allocates for these arguments (the serving engine's admission
// test uses it before allocating anything).
int64_t stream_bytes_needed(const arts_plan_t* plans, int32_t nplan, int32_t nsrc, int32_t nbeam,
                            int64_t chunk, int64_t cand_capacity) {
  if (!plans || nplan < 1 || !plans[0]) return -1;
  const int64_t rows = static_cast<int64_t>(nsrc) * plans[0]->nchan;
  int64_t hmax = 0, total = rows * chunk + cand_capacity * sizeof(arts_candidate) + 64;
  bool native = false;
  for (int32_t i = 0; i < nplan; ++i) {
    const arts_plan_s* p = plans[i];
    if (!p) return -1;
    total += static_cast<int64_t>(nbeam) * p->ndm * (chunk / p->ds + p->wmax - 1) * 4;
    if (p->ds == 1) {
      native = true;
      hmax = std::max<int64_t>(hmax, static_cast<int64_t>(p->halo));
    } else {
      const int64_t n16 = p->halo + chunk / p->ds;
      total += 2 * rows * ((n16 + 1) & ~int64_t(1)) * 2;
    }
  }
  if (native) total += 2 * rows * ((hmax + chunk + 3) & ~int64_t(3));
  for (int32_t i = 0; i < nplan; ++i) {  // 16-bit step-1 rows
    const YLayout y = y_layout(plans[i], nbeam, chunk);
    total += 2 * y.rows * y.pitch;
  }
  int64_t max_rows = 0;  // candidate pre-pass flags
  for (int32_t i = 0; i < nplan; ++i)
    max_rows = std::max<int64_t>(max_rows, static_cast<int64_t>(nbeam) * plans[i]->ndm);
  total += max_rows;
  int64_t cl_rows = 0;  // clustering workspace
  for (int32_t i = 0; i < nplan; ++i)
    if (plans[i]->cluster) cl_rows = std::max<int64_t>(cl_rows, static_cast<int64_t>(nbeam) * plans[i]->ndm);
  if (cl_rows > 0) total += cluster_ws_bytes(cand_capacity, cl_rows);
  return total;
}

DedispJob stream_job(arts_stream_s* s, int parity, size_t p) {
  const arts_plan_s* pl = s->plans[p];
  const int64_t rows = static_cast<int64_t>(s->nsrc) * s->nchan;
  DedispJob job;
  job.nsrc = s->nsrc;
  job.sb_table = s->sb_table;
  job.nbeam = s->nbeam;
  job.out = s->series[p];
  job.nout = s->L[p];
  if (pl->ds == 1) {
    const int64_t off = s->hmax - s->H[p];
    job.in = s->ring[parity] + off;
    job.in_bytes = rows * s->W - off;
    job.nin = s->H[p] + s->chunk;
    job.pitch = s->W;
    if (pl->nsub > 0) {
      uint16_t* b = s->ybuf[p];
      const int64_t at = s->y_at[p] * s->chunk;
      job.y = b + at;
      job.y_prev = s->y_from[p] < 0 ? nullptr : b + s->y_from[p] * s->chunk;
      job.y_elems = s->y_elems[p] - at;
      job.y_new = s->chunk;
      job.y_pad = s->y_pad[p];
      job.y_pitch = s->y_pitch[p];
      job.y_lo = b;
      job.y_hi = b + s->y_elems[p];
    }
  } else {
    job.in = s->input;  // unused: the kernel reads the 16-bit ring
    job.in_bytes = rows * s->chunk;
    job.nin = s->N16[p] * pl->ds;
    job.pitch = s->chunk;
    job.in16 = s->ring16[parity][p];
    job.in16_elems = rows * s->W16[p];
    job.pitch16 = s->W16[p];
  }
  return job;
}

void stream_y_step(arts_stream_s* s) {
  for (size_t p = 0; p < s->plans.size(); ++p) {
    if (!s->ybuf[p]) continue;
    if (s->y_stale) {  // recompute the whole window at the front
      s->y_from[p] = -1;
      s->y_at[p] = 0;
    } else {
      s->y_from[p] = s->y_at[p];
      s->y_at[p] = s->y_at[p] < s->y_m[p] ? s->y_at[p] + 1 : 0;
    }
  }
}

int64_t stream_warmup(const arts_stream_s* s, size_t p, int64_t k) {
  const int64_t nrep = s->chunk / s->plans[p]->ds;
  const int64_t halo = s->H[p] / s->plans[p]->ds;
  // output t of chunk k starts its window at downsampled input sample k * nrep - halo + t
  if (k >= (halo + nrep - 1) / nrep) return 0;
  return std::min(nrep, halo - k * nrep);
}

bool stream_warm(const arts_stream_s* s, int64_t k) {
  for (size_t p = 0; p < s->plans.size(); ++p)
    if (stream_warmup(s, p, k) > 0) return false;
  return true;
}

// Decimated integration in a stream: chunk samples are numbered relative to the chunk, so each
// width's grid is the absolute one only if every width divides the chunk's searched length.
bool integration_grid_ok(const arts_plan_s* p, int64_t nrep) {
  if (p->integration == 0) return true;
  for (int32_t w : p->widths)
    if (nrep % w != 0) return false;
  return true;
}

int stream_candidates(arts_stream_s* s, hipStream_t hs) {
  for (size_t p = 0; p < s->plans.size(); ++p)
    if (!integration_grid_ok(s->plans[p], s->chunk / s->plans[p]->ds))
      return fail(ARTS_E_INVAL, "plan %zu searches with decimated integration: every width must "
                  "divide chunk / downsampling (%lld)", p, (long long)(s->chunk / s->plans[p]->ds));
  if (int st = launch_zero_u64(s->d_count, 1, hs)) return st;
  for (size_t p = 0; p < s->plans.size(); ++p) {
    const arts_plan_s* pl = s->plans[p];
    const int64_t nrep = s->chunk / pl->ds;
    const int64_t t0 = stream_warmup(s, p, s->pushed);
    if (t0 >= nrep) continue;
    const bool clu = s->cluster[p] != 0;
    if (clu)
      if (int st = launch_cluster_mark(s->cl, s->d_count, hs)) return st;
    // sample numbers are made absolute on the host: chunk-relative start minus the halo
    if (int st = launch_candidates(pl, s->series[p], s->nbeam, s->L[p], nrep, s->thr,
                                   -s->H[p] / pl->ds, 0, nullptr, nullptr, s->d_cand,
                                   s->d_count, s->cap, hs, t0, s->d_flags))
      return st;
    if (clu)
      if (int st = launch_cluster(s->cl, s->d_cand, s->d_count, s->cap, true, s->nbeam, pl->ndm,
                                  0, hs))
        return st;
  }
  ARTS_HIP(hipMemcpyAsync(s->h_count, s->d_count, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, hs));
  return ARTS_OK;
}

}  // namespace arts

namespace {

int enqueue_push(arts_stream_s* s, int parity, bool profile) {
  auto mark = [&](int i) -> int {
    if (profile) ARTS_HIP(hipEventRecord(s->pev[i], s->hs));
    return ARTS_OK;
  };
  int ev = 0;
  if (int st = mark(ev++)) return st;
  if (int st = stream_advance(s, parity, s->hs)) return st;
  if (int st = mark(ev++)) return st;
  for (size_t p = 0; p < s->plans.size(); ++p) {
    const DedispJob job = stream_job(s, parity, p);
    if (int st = launch_dedisperse(s->plans[p], job, s->hs)) return st;
    if (int st = mark(ev++)) return st;
  }
  if (int st = stream_candidates(s, s->hs)) return st;
  if (int st = mark(ev++)) return st;
  return ARTS_OK;
}

// Ring segments in snapshot order: the native ring, then each plan's 16-bit ring.
std::vector<std::pair<uint8_t*, int64_t>> ring_parts(arts_stream_s* s, int parity) {
  const int64_t rows = static_cast<int64_t>(s->nsrc) * s->nchan;
  std::vector<std::pair<uint8_t*, int64_t>> v;
  if (s->ring[parity]) v.push_back({s->ring[parity], rows * s->W});
  for (size_t p = 0; p < s->plans.size(); ++p)
    if (s->ring16[parity][p])
      v.push_back({reinterpret_cast<uint8_t*>(s->ring16[parity][p]), rows * s->W16[p] * 2});
  return v;
}

int64_t ring_bytes_total(arts_stream_s* s) {
  int64_t n = 0;
  for (auto& pr : ring_parts(s, 0)) n += pr.second;
  return n;
}

}  // namespace

extern "C" {

int arts_stream_create(const arts_plan_t* plans, int32_t nplan, int32_t nsrc,
                       const uint8_t* sb_table, int32_t nbeam, int64_t chunk, float threshold,
                       int64_t cand_capacity, uint32_t flags, arts_stream_t* out) {
  if (!out) return fail(ARTS_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!plans || nplan < 1) return fail(ARTS_E_INVAL, "need at least one plan");
  if (nsrc < 1 || nbeam < 1 || chunk < 1 || cand_capacity < 1 || !std::isfinite(threshold))
    return fail(ARTS_E_INVAL, "nsrc, nbeam, chunk, capacity must be >= 1; finite threshold");
  if (!sb_table && nbeam != nsrc)
    return fail(ARTS_E_INVAL, "without an SB table every source row is one beam");
  if (sb_table && nsrc > 256) return fail(ARTS_E_INVAL, "at most 256 source beams with a table");
  if ((flags & kGraph) && (flags & kProfile))
    return fail(ARTS_E_INVAL, "profiling events are not recorded inside graphs");
  arts_stream_s* s = new (std::nothrow) arts_stream_s;
  if (!s) return fail(ARTS_E_NOMEM, "host allocation failed");
  s->nsrc = nsrc;
  s->nbeam = nbeam;
  s->sb_table = sb_table;
  s->chunk = chunk;
  s->thr = threshold;
  s->flags = flags;
  s->cap = cand_capacity;
  for (int32_t i = 0; i < nplan; ++i) {
    arts_plan_s* p = plans[i];
    if (!p) {
      stream_free(s);
      return fail(ARTS_E_INVAL, "plan %d is NULL", i);
    }
    if (i > 0 && p->nchan != plans[0]->nchan) {
      stream_free(s);
      return fail(ARTS_E_INVAL, "all plans of a stream must have the same channel count");
    }
    if (chunk % p->ds != 0) {
      stream_free(s);
      return fail(ARTS_E_INVAL, "chunk %lld is not a multiple of plan %d's downsampling %d",
                  (long long)chunk, i, p->ds);
    }
    if (!integration_grid_ok(p, chunk / p->ds)) {
      stream_free(s);
      return fail(ARTS_E_INVAL, "plan %d searches with decimated integration: every width must "
                  "divide chunk / downsampling (%lld)", i, (long long)(chunk / p->ds));
    }
    if (p->nsub > 0 && chunk % 4 != 0) {  // the step-1 window moves by whole 8-byte groups
      stream_free(s);
      return fail(ARTS_E_INVAL, "plan %d is a subband plan: the chunk must be a multiple of 4",
                  i);
    }
    s->plans.push_back(p);
    s->H.push_back(static_cast<int64_t>(p->ds) * p->halo);
    s->L.push_back(chunk / p->ds + p->wmax - 1);
    s->N16.push_back(p->ds > 1 ? p->halo + chunk / p->ds : 0);
    s->W16.push_back((s->N16.back() + 1) & ~int64_t(1));
  }
  s->nchan = plans[0]->nchan;
  s->hmax = 0;
  bool native = false;
  for (size_t p = 0; p < s->plans.size(); ++p)
    if (s->plans[p]->ds == 1) {
      native = true;
      s->hmax = std::max(s->hmax, s->H[p]);
    }
  s->W = (s->hmax + chunk + 3) & ~int64_t(3);
  const int64_t rows = static_cast<int64_t>(nsrc) * s->nchan;
  int st = ARTS_OK;
  for (int r = 0; r < 2 && st == ARTS_OK; ++r) {
    s->ring16[r].assign(s->plans.size(), nullptr);
    if (native) {
      st = dev_alloc(s, reinterpret_cast<void**>(&s->ring[r]), rows * s->W);
      if (st == ARTS_OK && hipMemset(s->ring[r], 0, rows * s->W) != hipSuccess)
        st = fail(ARTS_E_DEVICE, "ring clear failed");
    }
    for (size_t p = 0; p < s->plans.size() && st == ARTS_OK; ++p) {
      if (s->plans[p]->ds == 1) continue;
      const int64_t bytes = rows * s->W16[p] * 2;
      st = dev_alloc(s, reinterpret_cast<void**>(&s->ring16[r][p]), bytes);
      if (st == ARTS_OK && hipMemset(s->ring16[r][p], 0, bytes) != hipSuccess)
        st = fail(ARTS_E_DEVICE, "ring clear failed");
    }
  }
  if (st == ARTS_OK) st = dev_alloc(s, reinterpret_cast<void**>(&s->input), rows * chunk);
  // offset tables for the alignment class of each plan's window start, made now so that no
  // allocation happens inside a push (or a captured graph)
  for (size_t p = 0; p < s->plans.size() && st == ARTS_OK; ++p) {
    const int g0 = s->plans[p]->ds == 1
                       ? static_cast<int>((reinterpret_cast<uintptr_t>(s->ring[0]) + s->hmax - s->H[p]) & 3u)
                       : static_cast<int>((reinterpret_cast<uintptr_t>(s->ring16[0][p]) >> 1) & 1u);
    st = prepare_plan(s->plans[p], nbeam, s->H[p] + chunk, g0, false);
  }
  // subband plans: one buffer of step-1 rows, zero like the history they stand for (the first
  // window sits at the front; every push moves it by one chunk)
  for (size_t p = 0; p < s->plans.size() && st == ARTS_OK; ++p) {
    const YLayout y = y_layout(s->plans[p], nbeam, chunk);
    const int64_t e = y.rows * y.pitch;
    s->y_elems.push_back(e);
    s->y_pitch.push_back(y.pitch);
    s->y_pad.push_back(y.pad);
    s->y_m.push_back(y.m);
    s->y_at.push_back(0);
    s->y_from.push_back(-1);
    uint16_t* b = nullptr;
    if (e > 0) {
      st = dev_alloc(s, reinterpret_cast<void**>(&b), e * sizeof(uint16_t));
      if (st == ARTS_OK && hipMemset(b, 0, e * sizeof(uint16_t)) != hipSuccess)
        st = fail(ARTS_E_DEVICE, "subband row clear failed");
    }
    s->ybuf.push_back(b);
  }
  for (size_t p = 0; p < s->plans.size() && st == ARTS_OK; ++p) {
    int32_t* ser = nullptr;
    const int64_t nrow = static_cast<int64_t>(nbeam) * s->plans[p]->ndm;
    st = dev_alloc(s, reinterpret_cast<void**>(&ser), nrow * s->L[p] * sizeof(int32_t));
    s->series.push_back(ser);
  }
  if (st == ARTS_OK)
    st = dev_alloc(s, reinterpret_cast<void**>(&s->d_cand), cand_capacity * sizeof(arts_candidate));
  if (st == ARTS_OK) st = dev_alloc(s, reinterpret_cast<void**>(&s->d_count), 64);
  int64_t max_rows = 0;  // candidate pre-pass flags
  for (auto* pl : s->plans) max_rows = std::max<int64_t>(max_rows, static_cast<int64_t>(nbeam) * pl->ndm);
  if (st == ARTS_OK) st = dev_alloc(s, reinterpret_cast<void**>(&s->d_flags), max_rows);
  // DM-width clustering, for the plans that ask for it when the stream is created
  int64_t cl_rows = 0;
  for (auto* pl : s->plans) {
    s->cluster.push_back(pl->cluster ? 1 : 0);
    if (pl->cluster) cl_rows = std::max<int64_t>(cl_rows, static_cast<int64_t>(nbeam) * pl->ndm);
  }
  if (st == ARTS_OK && cl_rows > 0) {
    st = ensure_cluster_ws(s->cl, cand_capacity, cl_rows);
    if (st == ARTS_OK) s->device_bytes += s->cl.bytes;
  }
  if (st == ARTS_OK && hipHostMalloc(reinterpret_cast<void**>(&s->h_count), 64) != hipSuccess)
    st = fail(ARTS_E_NOMEM, "pinned allocation failed");
  if (st == ARTS_OK && hipStreamCreateWithFlags(&s->hs, hipStreamNonBlocking) != hipSuccess)
    st = fail(ARTS_E_DEVICE, "stream creation failed");
  if (st == ARTS_OK && (hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming) != hipSuccess ||
                        hipEventCreateWithFlags(&s->ev_done, hipEventDisableTiming) != hipSuccess))
    st = fail(ARTS_E_DEVICE, "event creation failed");
  if (st == ARTS_OK && (flags & kProfile)) {
    s->pev.assign(nphases(s) + 1, nullptr);
    for (auto& e : s->pev)
      if (hipEventCreate(&e) != hipSuccess) st = fail(ARTS_E_DEVICE, "event creation failed");
    s->phase_ms.assign(nphases(s), 0.0);
    s->phase_n.assign(nphases(s), 0);
  }
  if (st != ARTS_OK) {
    stream_free(s);
    return st;
  }
  *out = s;
  return ARTS_OK;
}

int arts_stream_input(arts_stream_t s, uint8_t** chunk_buffer) {
  if (!s || !chunk_buffer) return fail(ARTS_E_INVAL, "NULL argument");
  *chunk_buffer = s->input;
  return ARTS_OK;
}

int arts_stream_push(arts_stream_t s, const uint8_t* chunk, void* stream) {
  TraceRange range("arts_stream_push");
  if (!s) return fail(ARTS_E_INVAL, "stream is NULL");
  if (s->pushed != s->waited)
    return fail(ARTS_E_STATE, "the previous chunk has not been collected with arts_stream_wait");
  // captured pushes read the plans' tables and modes as they were at capture: after any
  // change (a new tiling frees the old tables; clustering or integration mode) capture again
  std::vector<uint64_t> gen;
  for (const arts_plan_s* p : s->plans) gen.push_back(p->generation);
  if (gen != s->plan_gen) {
    for (auto& kv : s->graphs)
      if (kv.second) (void)hipGraphExecDestroy(kv.second);
    s->graphs.clear();
    s->plan_gen = gen;
    s->eager_next = true;  // lazily built tables must exist before a capture
  }
  hipStream_t caller = static_cast<hipStream_t>(stream);
  ARTS_HIP(hipEventRecord(s->ev_in, caller));
  ARTS_HIP(hipStreamWaitEvent(s->hs, s->ev_in, 0));
  const int64_t rows = static_cast<int64_t>(s->nsrc) * s->nchan;
  if (chunk && chunk != s->input)
    ARTS_HIP(hipMemcpyAsync(s->input, chunk, rows * s->chunk, hipMemcpyDeviceToDevice, s->hs));
  const int parity = static_cast<int>(s->pushed & 1);
  stream_y_step(s);
  // warm-up chunks search a chunk-dependent part of each series: they run eagerly, and the
  // graphs are captured once every plan searches its whole chunk, one per ring parity and
  // step-1 window position
  if ((s->flags & kGraph) && stream_warm(s, s->pushed) && !s->y_stale && !s->eager_next) {
    std::vector<int> key{parity};
    for (size_t p = 0; p < s->plans.size(); ++p) key.push_back(s->ybuf[p] ? s->y_at[p] : 0);
    hipGraphExec_t& ge = s->graphs[key];
    if (!ge) {
      hipGraph_t g = nullptr;
      ARTS_HIP(hipStreamBeginCapture(s->hs, hipStreamCaptureModeThreadLocal));
      const int st = enqueue_push(s, parity, false);
      const hipError_t ce = hipStreamEndCapture(s->hs, &g);
      if (st != ARTS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (ce != hipSuccess) return fail(ARTS_E_DEVICE, "graph capture: %s", hipGetErrorString(ce));
      const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        ge = nullptr;
        return fail(ARTS_E_DEVICE, "graph instantiate: %s", hipGetErrorString(ie));
      }
    }
    ARTS_HIP(hipGraphLaunch(ge, s->hs));
  } else {
    if (int st = enqueue_push(s, parity, (s->flags & kProfile) != 0)) return st;
    s->pending_profile = (s->flags & kProfile) != 0;
  }
  ARTS_HIP(hipEventRecord(s->ev_done, s->hs));
  ++s->pushed;
  s->y_stale = false;
  s->eager_next = false;
  return ARTS_OK;
}

int arts_stream_wait(arts_stream_t s, arts_candidate* host_out, int64_t capacity, int64_t* count,
                     int64_t* chunk_index) {
  TraceRange range("arts_stream_wait");
  if (!s || !count) return fail(ARTS_E_INVAL, "NULL argument");
  if (s->pushed == s->waited) return fail(ARTS_E_STATE, "nothing pushed");
  ARTS_HIP(hipEventSynchronize(s->ev_done));
  const int64_t k = s->pushed - 1;
  if (chunk_index) *chunk_index = k;
  if (s->pending_profile) {
    for (int i = 0; i < nphases(s); ++i) {
      float ms = 0;
      ARTS_HIP(hipEventElapsedTime(&ms, s->pev[i], s->pev[i + 1]));
      s->phase_ms[i] += ms;
      s->phase_n[i] += 1;
    }
    s->pending_profile = false;
  }
  s->waited = s->pushed;
  const int64_t n = static_cast<int64_t>(*s->h_count);
  *count = n;
  if (n > s->cap) return fail(ARTS_E_CAPACITY, "%lld candidates, stream capacity %lld",
                              (long long)n, (long long)s->cap);
  if (n > capacity) return fail(ARTS_E_CAPACITY, "%lld candidates, capacity %lld",
                                (long long)n, (long long)capacity);
  if (n == 0) return ARTS_OK;
  if (!host_out) return fail(ARTS_E_INVAL, "host_out is NULL");
  ARTS_HIP(hipMemcpy(host_out, s->d_cand, n * sizeof(arts_candidate), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i) host_out[i].sample += k * s->chunk / host_out[i].downsample;
  std::sort(host_out, host_out + n, [](const arts_candidate& a, const arts_candidate& b) {
    if (a.beam != b.beam) return a.beam < b.beam;
    if (a.downsample != b.downsample) return a.downsample < b.downsample;
    if (a.dm_index != b.dm_index) return a.dm_index < b.dm_index;
    if (a.width != b.width) return a.width < b.width;
    return a.sample < b.sample;
  });
  return ARTS_OK;
}

int arts_stream_info(arts_stream_t s, int64_t* chunks_pushed, int64_t* device_bytes,
                     int64_t* halo_native) {
  if (!s) return fail(ARTS_E_INVAL, "stream is NULL");
  if (chunks_pushed) *chunks_pushed = s->pushed;
  if (device_bytes) *device_bytes = s->device_bytes;
  if (halo_native) *halo_native = s->hmax;
  return ARTS_OK;
}

int arts_stream_warmup(arts_stream_t s, int32_t plan_index, int64_t chunk_index,
                       int64_t* t_begin) {
  if (!s || !t_begin) return fail(ARTS_E_INVAL, "NULL argument");
  if (plan_index < 0 || plan_index >= static_cast<int32_t>(s->plans.size()) || chunk_index < 0)
    return fail(ARTS_E_INVAL, "plan or chunk index out of range");
  *t_begin = stream_warmup(s, static_cast<size_t>(plan_index), chunk_index);
  return ARTS_OK;
}

int arts_stream_timing(arts_stream_t s, int32_t phase, double* total_ms, int64_t* n) {
  if (!s || !total_ms || !n) return fail(ARTS_E_INVAL, "NULL argument");
  if (!(s->flags & kProfile)) return fail(ARTS_E_STATE, "stream was created without profiling");
  if (phase < 0 || phase >= nphases(s)) return fail(ARTS_E_INVAL, "phase out of range");
  *total_ms = s->phase_ms[phase];
  *n = s->phase_n[phase];
  return ARTS_OK;
}

int arts_stream_series(arts_stream_t s, int32_t plan_index, const int32_t** series, int64_t* L) {
  if (!s || !series || !L) return fail(ARTS_E_INVAL, "NULL argument");
  if (plan_index < 0 || plan_index >= static_cast<int32_t>(s->plans.size()))
    return fail(ARTS_E_INVAL, "plan index out of range");
  *series = s->series[plan_index];
  *L = s->L[plan_index];
  return ARTS_OK;
}

int arts_stream_snapshot(arts_stream_t s, uint8_t* host, int64_t bytes, int64_t* chunks_pushed) {
  if (!s || !chunks_pushed) return fail(ARTS_E_INVAL, "NULL argument");
  const int64_t need = ring_bytes_total(s);
  *chunks_pushed = s->pushed;
  if (!host || bytes < need)
    return fail(ARTS_E_CAPACITY, "snapshot needs %lld bytes", (long long)need);
  if (s->pushed != s->waited) return fail(ARTS_E_STATE, "collect the last chunk first");
  ARTS_HIP(hipStreamSynchronize(s->hs));
  int64_t off = 0;
  for (auto& pr : ring_parts(s, static_cast<int>((s->pushed + 1) & 1))) {  // last written
    ARTS_HIP(hipMemcpy(host + off, pr.first, pr.second, hipMemcpyDeviceToHost));
    off += pr.second;
  }
  return ARTS_OK;
}

int arts_stream_restore(arts_stream_t s, const uint8_t* host, int64_t bytes,
                        int64_t chunks_pushed) {
  if (!s || !host || chunks_pushed < 0) return fail(ARTS_E_INVAL, "bad argument");
  const int64_t need = ring_bytes_total(s);
  if (bytes < need) return fail(ARTS_E_CAPACITY, "restore needs %lld bytes", (long long)need);
  if (s->pushed != s->waited) return fail(ARTS_E_STATE, "collect the last chunk first");
  ARTS_HIP(hipStreamSynchronize(s->hs));
  int64_t off = 0;
  for (auto& pr : ring_parts(s, static_cast<int>((chunks_pushed + 1) & 1))) {
    ARTS_HIP(hipMemcpy(pr.first, host + off, pr.second, hipMemcpyHostToDevice));
    off += pr.second;
  }
  s->pushed = s->waited = chunks_pushed;
  s->y_stale = true;  // subband step-1 rows are not part of a snapshot: recompute them once
  return ARTS_OK;
}

int arts_stream_snapshot_bytes(arts_stream_t s, int64_t* bytes) {
  if (!s || !bytes) return fail(ARTS_E_INVAL, "NULL argument");
  *bytes = ring_bytes_total(s);
  return ARTS_OK;
}

int arts_stream_set_rfi(arts_stream_t s, float k_time, int32_t niter_time, float k_freq,
                        int32_t niter_freq) {
  if (!s) return fail(ARTS_E_INVAL, "stream is NULL");
  const auto k_ok = [](float k) { return k == 0.0f || (k >= 0.015625f && k <= 1024.0f); };
  if (niter_time < 0 || niter_freq < 0 || !k_ok(k_time) || !k_ok(k_freq))
    return fail(ARTS_E_INVAL, "RFI: iterations >= 0, thresholds 0 or within [2^-6, 1024]");
  if (niter_freq > 0 && s->nchan > 4096)
    return fail(ARTS_E_INVAL, "RFI: at most 4096 channels for the frequency-domain filter");
  if (s->pushed != s->waited) return fail(ARTS_E_STATE, "a chunk is in flight");
  if (!s->rfi_ws && (niter_time > 0 || niter_freq > 0)) {
    const int64_t bytes = rfi_ws_bytes(s->nsrc, s->nchan, s->chunk);
    if (int st = dev_alloc(s, &s->rfi_ws, bytes)) return st;
  }
  s->rfi_kt = k_time;
  s->rfi_nt = niter_time;
  s->rfi_kf = k_freq;
  s->rfi_nf = niter_freq;
  for (auto& kv : s->graphs)  // captured pushes do not clean: capture again
    if (kv.second) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
  return ARTS_OK;
}

void arts_stream_destroy(arts_stream_t s) { stream_free(s); }

}  // extern "C"

// Uneven batches: many search requests of different channel counts, lengths and DM ranges
// dedispersed in one persistent launch per tiling variant (a work queue of tiles over all
// requests), then thresholded request by request into one candidate list.
#include <algorithm>
#include <cmath>
#include <map>
#include <new>

#include "arts_internal.h"

using namespace arts;

struct arts_batch_s {
  BatchBuffers bb;
  // per-request workspaces: dword-aligned copies (D = 1, odd row length) or 16-bit rows (D > 1)
  std::vector<uint8_t*> ws;
  std::vector<int64_t> ws_cap;
  arts_candidate* d_cand = nullptr;
  unsigned long long* d_count = nullptr;
  int64_t cand_cap = 0;
  ClusterWs cl;  // DM-width clustering of requests whose plan asks for it
  uint8_t* d_flags = nullptr;  // candidate pre-pass rows (max over requests)
  int64_t flags_cap = 0;
};

namespace {

int ensure_ws(arts_batch_s* b, int i, int64_t bytes) {
  if (static_cast<int>(b->ws.size()) <= i) {
    b->ws.resize(i + 1, nullptr);
    b->ws_cap.resize(i + 1, 0);
  }
  if (bytes <= b->ws_cap[i]) return ARTS_OK;
  if (b->ws[i]) (void)hipFree(b->ws[i]);
  b->ws[i] = nullptr;
  b->ws_cap[i] = 0;
  ARTS_HIP(hipMalloc(&b->ws[i], bytes));
  b->ws_cap[i] = bytes;
  return ARTS_OK;
}

int64_t series_len(const arts_plan_s* p, int64_t nin) { return nin / p->ds - p->max_delay; }

}  // namespace

extern "C" {

int arts_batch_create(arts_batch_t* out) {
  if (!out) return fail(ARTS_E_INVAL, "out is NULL");
  *out = new (std::nothrow) arts_batch_s;
  return *out ? ARTS_OK : fail(ARTS_E_NOMEM, "host allocation failed");
}

void arts_batch_destroy(arts_batch_t b) {
  if (!b) return;
  for (auto* p : b->ws)
    if (p) (void)hipFree(p);
  if (b->d_cand) (void)hipFree(b->d_cand);
  if (b->d_count) (void)hipFree(b->d_count);
  if (b->d_flags) (void)hipFree(b->d_flags);
  free_cluster_ws(b->cl);
  delete b;
}

int arts_batch_dedisperse(arts_batch_t b, const arts_request* reqs, int32_t n, int32_t* status,
                          void* stream) {
  if (!b || (!reqs && n > 0) || n < 0) return fail(ARTS_E_INVAL, "bad batch arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::map<int, std::pair<std::vector<arts_plan_s*>, std::vector<DedispJob>>> groups;
  for (int32_t i = 0; i < n; ++i) {
    const arts_request& r = reqs[i];
    int st = ARTS_OK;
    if (!r.plan || !r.in || !r.out || r.nbeam < 1 || r.nin < 1) st = ARTS_E_INVAL;
    else if (series_len(r.plan, r.nin) < 1) st = ARTS_E_SHAPE;
    if (status) status[i] = st;
    if (st != ARTS_OK) continue;
    arts_plan_s* p = r.plan;
    DedispJob job;
    job.in = r.in;
    job.in_bytes = static_cast<int64_t>(r.nbeam) * p->nchan * r.nin;
    job.nin = r.nin;
    job.pitch = r.nin;
    job.nsrc = r.nbeam;
    job.nbeam = r.nbeam;
    job.out = r.out;
    job.nout = series_len(p, r.nin);
    const int64_t rows = static_cast<int64_t>(r.nbeam) * p->nchan;
    if (p->ds > 1) {
      const int64_t nd = r.nin / p->ds, pitch16 = (nd + 1) & ~int64_t(1);
      if (int e = ensure_ws(b, i, rows * pitch16 * 2)) return e;
      uint16_t* w16 = reinterpret_cast<uint16_t*>(b->ws[i]);
      if (int e = launch_downsample(w16, pitch16, r.in, r.nin, rows, nd, p->ds, s)) return e;
      job.in16 = w16;
      job.in16_elems = rows * pitch16;
      job.pitch16 = pitch16;
    } else if (r.nin % 4 != 0) {
      const int64_t pitch = (r.nin + 3) & ~int64_t(3);
      if (int e = ensure_ws(b, i, rows * pitch)) return e;
      if (int e = launch_copy_rows(b->ws[i], pitch, r.in, r.nin, rows, r.nin, r.in,
                                   r.in + job.in_bytes, s))
        return e;
      job.in = b->ws[i];
      job.pitch = pitch;
      job.in_bytes = rows * pitch;
    }
    if (p->nsub > 0) {  // subband plans: their own two-step launches, the plan's workspace
      if (int e = prepare_plan(p, job.nbeam, job.nin,
                               static_cast<int>(reinterpret_cast<uintptr_t>(job.in) & 3u), true))
        return e;
      if (int e = launch_dedisperse(p, job, s)) return e;
      continue;
    }
    auto& g = groups[p->tiling.variant];
    g.first.push_back(p);
    g.second.push_back(job);
  }
  for (auto& kv : groups) {
    auto& g = kv.second;
    if (int e = launch_dedisperse_batch(g.first.data(), g.second.data(),
                                        static_cast<int>(g.first.size()), b->bb, s))
      return e;
  }
  return ARTS_OK;
}

int arts_batch_candidates(arts_batch_t b, const arts_request* reqs, int32_t n, float threshold,
                          arts_candidate* host_out, int64_t capacity, int64_t* count,
                          void* stream) {
  if (!b || (!reqs && n > 0) || n < 0 || !count || capacity < 0 || (capacity > 0 && !host_out))
    return fail(ARTS_E_INVAL, "bad batch arguments");
  if (!std::isfinite(threshold)) return fail(ARTS_E_INVAL, "threshold must be finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!b->d_count) ARTS_HIP(hipMalloc(&b->d_count, 64));
  if (capacity > b->cand_cap || !b->d_cand) {
    if (b->d_cand) (void)hipFree(b->d_cand);
    b->d_cand = nullptr;
    const int64_t cap = std::max<int64_t>(capacity, 1024);
    ARTS_HIP(hipMalloc(&b->d_cand, cap * sizeof(arts_candidate)));
    b->cand_cap = cap;
  }
  // clustered requests share one workspace, sized before any launch
  int64_t cl_rows = 0;
  for (int32_t i = 0; i < n; ++i)
    if (reqs[i].plan && reqs[i].plan->cluster && reqs[i].nbeam >= 1)
      cl_rows = std::max<int64_t>(cl_rows, static_cast<int64_t>(reqs[i].nbeam) * reqs[i].plan->ndm);
  if (cl_rows > 0)
    if (int e = ensure_cluster_ws(b->cl, std::max<int64_t>(capacity, 1), cl_rows)) return e;
  int64_t all_rows = 0;  // candidate pre-pass flags, sized before any launch
  for (int32_t i = 0; i < n; ++i)
    if (reqs[i].plan && reqs[i].nbeam >= 1)
      all_rows = std::max<int64_t>(all_rows, static_cast<int64_t>(reqs[i].nbeam) * reqs[i].plan->ndm);
  if (all_rows > b->flags_cap) {
    if (b->d_flags) (void)hipFree(b->d_flags);
    b->d_flags = nullptr;
    b->flags_cap = 0;
    ARTS_HIP(hipMalloc(&b->d_flags, all_rows));
    b->flags_cap = all_rows;
  }
  if (int e = launch_zero_u64(b->d_count, 1, s)) return e;
  int32_t beam0 = 0;
  for (int32_t i = 0; i < n; ++i) {
    const arts_request& r = reqs[i];
    if (r.plan && r.nbeam >= 1 && r.nin >= 1) {
      const int64_t L = series_len(r.plan, r.nin);
      const int64_t nrep = L - r.plan->wmax + 1;
      if (L >= 1 && nrep >= 1) {
        if (r.plan->cluster)
          if (int e = launch_cluster_mark(b->cl, b->d_count, s)) return e;
        if (int e = launch_candidates(r.plan, r.out, r.nbeam, L, nrep, threshold, 0, beam0, nullptr,
                                      nullptr, b->d_cand, b->d_count, capacity, s, 0, b->d_flags))
          return e;
        if (r.plan->cluster)
          if (int e = launch_cluster(b->cl, b->d_cand, b->d_count, capacity, true, r.nbeam,
                                     r.plan->ndm, beam0, s))
            return e;
      }
    }
    beam0 += std::max(0, r.nbeam);
  }
  unsigned long long nc = 0;
  ARTS_HIP(hipMemcpyAsync(&nc, b->d_count, sizeof nc, hipMemcpyDeviceToHost, s));
  ARTS_HIP(hipStreamSynchronize(s));
  *count = static_cast<int64_t>(nc);
  if (*count > capacity)
    return fail(ARTS_E_CAPACITY, "%llu candidates, capacity %lld", nc, (long long)capacity);
  if (nc == 0) return ARTS_OK;
  ARTS_HIP(hipMemcpy(host_out, b->d_cand, nc * sizeof(arts_candidate), hipMemcpyDeviceToHost));
  std::sort(host_out, host_out + nc, [](const arts_candidate& x, const arts_candidate& y) {
    if (x.beam != y.beam) return x.beam < y.beam;
    if (x.dm_index != y.dm_index) return x.dm_index < y.dm_index;
    if (x.width != y.width) return x.width < y.width;
    return x.sample < y.sample;
  });
  return ARTS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------ autotuner ----
// The paper's search is auto-tuned per platform and observation setup (Sect. 6b.2, AMBER's
// run-time tuning).  Here the compiled kernel shapes are searched instead: every tiling variant
// that suits the plan (DMs per block x samples per lane), each with one LDS buffer and the
// most channels per chunk that fit, is timed; the three fastest are then timed again with two
// buffers (half the channels per chunk, the next chunk fetched while one is summed) and with
// half the channels per chunk, and the fastest shape of all is kept.  Plan calls are timed on pseudo-random bytes of the caller's
// shape; batches on the caller's own requests.  Results are cached in a text file, one line
// per key:
//   <arch> <CUs> <nchan> <ndm> <D>[s<nsub>] <max_delay> <delay-table hash> <nbeam> <nin>
//   <variant> <buffers> <channels> <ms>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

namespace {

struct Shape {
  int variant = -1, nbuf = kDefaultBuffers, cc = 0;
  float ms = 0;
};

std::string device_tag() {
  int dev = 0, ncu = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown 0";
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  std::string arch(prop.gcnArchName);
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  return arch + ' ' + std::to_string(ncu);
}

uint64_t delay_hash(const arts_plan_s* p) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the delay table (and subband step tables)
  auto mix = [&h](const std::vector<int32_t>& v) {
    for (int32_t x : v) {
      h ^= static_cast<uint32_t>(x);
      h *= 1099511628211ull;
    }
  };
  mix(p->delays);
  if (p->sb1) mix(p->sb1->delays);
  if (p->sb2) mix(p->sb2->delays);
  return h;
}

std::string tune_key(const arts_plan_s* p, int32_t nbeam, int64_t nin) {
  std::ostringstream k;
  k << device_tag() << ' ' << p->nchan << ' ' << p->ndm << ' ' << p->ds;
  if (p->nsub > 0) k << 's' << p->nsub;
  k << ' ' << p->max_delay << ' ' << std::hex << delay_hash(p) << std::dec << ' ' << nbeam << ' '
    << nin;
  return k.str();
}

bool cache_lookup(const char* path, const std::string& key, Shape* out) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() ||
        line[key.size()] != ' ')
      continue;
    std::istringstream rest(line.substr(key.size()));
    Shape sh;
    if (rest >> sh.variant >> sh.nbuf >> sh.cc >> sh.ms && sh.variant >= 0 &&
        sh.variant < kNumVariants && (sh.nbuf == 1 || sh.nbuf == 2) && sh.cc >= 0 &&
        sh.cc <= 255) {
      *out = sh;
      found = true;  // the last entry for a key wins
    }
  }
  return found;
}

void cache_store(const char* path, const std::string& key, const Shape& sh) {
  if (!path) return;
  if (FILE* f = std::fopen(path, "a")) {
    std::fprintf(f, "%s %d %d %d %.4f\n", key.c_str(), sh.variant, sh.nbuf, sh.cc, sh.ms);
    std::fclose(f);
  }
}

// The shapes to time: phase 1 every suitable variant at (1 buffer, max channels); phase 2 the
// three fastest with two buffers and with half their channels per chunk.  apply(shape) sets a
// shape on every plan involved (false if it does not fit); time(&ms) times the work.
// Variants a search considers: byte or 16-bit samples as the plan reads them; group sums only
// for subband plans (their first step), whose other tilings are the byte ones.
bool suits(const arts_plan_s* p, int v) {
  if (p->nsub > 0) return kVariants[v].spd == 4 && kVariants[v].pack != 2;
  return (p->ds == 1) == (kVariants[v].spd == 4) && !is_group(kVariants[v].pack);
}

template <typename Suits, typename Apply, typename Time>
int search_shapes(Suits suit, Apply apply, Time time, Shape* best_out) {
  std::vector<Shape> first;
  for (int v = 0; v < kNumVariants; ++v) {
    if (!suit(v)) continue;
    Shape sh;
    sh.variant = v;
    if (!apply(sh)) continue;
    if (int st = time(&sh.ms)) return st;
    first.push_back(sh);
  }
  if (first.empty()) return fail(ARTS_E_INVAL, "no tiling variant fits");
  std::sort(first.begin(), first.end(), [](const Shape& a, const Shape& b) { return a.ms < b.ms; });
  Shape best = first[0];
  for (size_t i = 0; i < first.size() && i < 3; ++i) {
    int cc_max = 0;
    if (!apply(first[i])) continue;
    if (int st = time(&first[i].ms)) return st;  // re-timed next to its variations
    if (first[i].ms < best.ms) best = first[i];
    cc_max = first[i].cc;  // apply() reports the channels per chunk it got
    const Shape vars[2] = {{first[i].variant, 3 - kDefaultBuffers, 0, 0},
                           {first[i].variant, kDefaultBuffers, cc_max / 2, 0}};
    for (Shape sh : vars) {
      if (sh.nbuf == kDefaultBuffers && sh.cc < 8) continue;
      if (!apply(sh)) continue;
      if (int st = time(&sh.ms)) return st;
      if (sh.ms < best.ms) best = sh;
    }
  }
  *best_out = best;
  return ARTS_OK;
}

}  // namespace

extern "C" int arts_plan_autotune(arts_plan_t p, int32_t nbeam, int64_t nin, int32_t reps,
                                  const char* cache_path, int32_t* variant_out, float* ms_out) {
  if (!p || nbeam < 1 || reps < 1) return fail(ARTS_E_INVAL, "bad autotune arguments");
  if (nin / p->ds - p->max_delay < 1) return fail(ARTS_E_SHAPE, "nin shorter than the halo");
  const std::string key = tune_key(p, nbeam, nin);
  Shape best;
  if (cache_lookup(cache_path, key, &best)) {
    if (int st = arts_plan_set_tiling_shape(p, best.variant, best.nbuf, best.cc)) return st;
    if (variant_out) *variant_out = best.variant;
    if (ms_out) *ms_out = best.ms;
    return ARTS_OK;
  }
  const int64_t L = nin / p->ds - p->max_delay;
  const int64_t in_bytes = static_cast<int64_t>(nbeam) * p->nchan * nin;
  const int64_t out_bytes = static_cast<int64_t>(nbeam) * p->ndm * L * 4;
  uint8_t* in = nullptr;
  int32_t* out = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (in) (void)hipFree(in);
    if (out) (void)hipFree(out);
  };
  if (hipMalloc(&in, in_bytes) != hipSuccess || hipMalloc(&out, out_bytes) != hipSuccess ||
      hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(ARTS_E_NOMEM, "autotune buffers (%lld + %lld bytes)", (long long)in_bytes,
                (long long)out_bytes);
  }
  if (int st = launch_fill_random(in, in_bytes, 0x5eedu, s)) {
    cleanup();
    return st;
  }
  const int v0 = p->tiling.variant;
  const arts_plan_s* q = p->nsub > 0 ? p->sb1 : p;
  const int32_t req_nb0 = q->tile_nbuf, req_cc0 = q->tile_cc;
  auto apply = [&](Shape& sh) {
    if (arts_plan_set_tiling_shape(p, sh.variant, sh.nbuf, sh.cc) != ARTS_OK) return false;
    // the channels per chunk the shape got (for the half-channel variation)
    if (sh.cc == 0) (void)arts_plan_get_tiling_shape(p, nullptr, nullptr, &sh.cc);
    return true;
  };
  auto time = [&](float* ms) -> int {
    if (int st = arts_dedisperse(p, in, nbeam, nin, out, s)) return st;  // warm-up, tables
    if (hipEventRecord(e0, s) != hipSuccess) return fail(ARTS_E_DEVICE, "event record");
    for (int r = 0; r < reps; ++r)
      if (int st = arts_dedisperse(p, in, nbeam, nin, out, s)) return st;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
      return fail(ARTS_E_DEVICE, "event timing");
    *ms /= reps;
    return ARTS_OK;
  };
  int st = search_shapes([&](int v) { return suits(p, v); }, apply, time, &best);
  cleanup();
  if (st != ARTS_OK) {
    (void)arts_plan_set_tiling_shape(p, v0, req_nb0, req_cc0);
    return st;
  }
  if (int e = arts_plan_set_tiling_shape(p, best.variant, best.nbuf, best.cc)) return e;
  cache_store(cache_path, key, best);
  if (variant_out) *variant_out = best.variant;
  if (ms_out) *ms_out = best.ms;
  return ARTS_OK;
}

// Batch autotuner: the shape is searched for all requests of one sample kind together, timing
// the persistent launch over the caller's own requests, so that they share one tiling and
// go into one launch.  Native requests are tuned first, then 16-bit ones.
extern "C" int arts_batch_autotune(arts_batch_t b, const arts_request* reqs, int32_t n,
                                   int32_t reps, int32_t* variant_out, float* ms_out) {
  if (!b || !reqs || n < 1 || reps < 1) return fail(ARTS_E_INVAL, "bad autotune arguments");
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
  };
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(ARTS_E_DEVICE, "autotune stream / events");
  }
  int first_variant = -1;
  float first_ms = 0;
  for (int kind = 0; kind < 2; ++kind) {  // 0: native byte requests, 1: 16-bit ones
    std::vector<arts_request> grp;
    std::vector<arts_plan_s*> plans;
    for (int32_t i = 0; i < n; ++i) {
      arts_plan_s* p = reqs[i].plan;
      if (!p || p->nsub > 0 || reqs[i].nbeam < 1 || series_len(p, reqs[i].nin) < 1) continue;
      if ((p->ds > 1) != (kind == 1)) continue;
      grp.push_back(reqs[i]);
      if (std::find(plans.begin(), plans.end(), p) == plans.end()) plans.push_back(p);
    }
    if (grp.empty()) continue;
    std::vector<int32_t> v0(plans.size());
    for (size_t i = 0; i < plans.size(); ++i) v0[i] = plans[i]->tiling.variant;
    auto apply = [&](Shape& sh) {
      int cc_got = 0;
      for (arts_plan_s* p : plans) {
        if (arts_plan_set_tiling_shape(p, sh.variant, sh.nbuf, sh.cc) != ARTS_OK) return false;
        cc_got = std::max(cc_got, p->tiling.cc);
      }
      if (sh.cc == 0) sh.cc = cc_got;
      return true;
    };
    auto time = [&](float* ms) -> int {
      const int32_t m = static_cast<int32_t>(grp.size());
      if (int st = arts_batch_dedisperse(b, grp.data(), m, nullptr, s)) return st;
      if (hipEventRecord(e0, s) != hipSuccess) return fail(ARTS_E_DEVICE, "event record");
      for (int r = 0; r < reps; ++r)
        if (int st = arts_batch_dedisperse(b, grp.data(), m, nullptr, s)) return st;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(ms, e0, e1) != hipSuccess)
        return fail(ARTS_E_DEVICE, "event timing");
      *ms /= reps;
      return ARTS_OK;
    };
    Shape best;
    int st = search_shapes([&](int v) { return suits(plans[0], v); }, apply, time, &best);
    if (st == ARTS_OK) {
      // every plan of the group takes the shape (a plan that the variant does not fit keeps
      // its own and goes into a launch of its own)
      for (arts_plan_s* p : plans) (void)arts_plan_set_tiling_shape(p, best.variant, best.nbuf,
                                                                     best.cc);
    } else {
      for (size_t i = 0; i < plans.size(); ++i) (void)arts_plan_set_tiling(plans[i], v0[i]);
      cleanup();
      return st;
    }
    if (first_variant < 0) {
      first_variant = best.variant;
      first_ms = best.ms;
    }
  }
  cleanup();
  if (first_variant < 0) return fail(ARTS_E_INVAL, "no request to tune");
  if (variant_out) *variant_out = first_variant;
  if (ms_out) *ms_out = first_ms;
  return ARTS_OK;
}

// Serving engine with continuous batching.  Streams (beams or TAB sets of any channel count,
// chunk length and DM range) are admitted while their device memory fits an HBM budget and
// leave when closed; chunks are submitted as they arrive.  Each tick runs one search step for
// every stream that has a chunk waiting: ring advances, then the dedispersion of all those
// streams and plans in one persistent launch per tiling variant (so the streams' work shares
// the device), then each stream's statistics and candidates.  The real-time search keeps up
// with 1.024 s chunks of many beams per GPU node (Sect. 4f, Sect. 9h); a tick here serves all
// streams that are ready.
//
// Ticks are enqueued on compute lanes (HIP streams of default priority) in turn, so a chunk
// that arrives while another tick is still on the GPU is stepped at once, its kernels
// interleaving with those of the running tick, instead of waiting behind it.  Chunks are
// copied in on a separate copy stream; the tick that consumes a chunk waits for its copy on
// the device.  A stream has at most one chunk in flight, so its steps stay in order whatever
// lane they run on.
#include <algorithm>
#include <map>
#include <new>

#include "arts_internal.h"

using namespace arts;

namespace {
constexpr int kMaxLanes = 2;
}

struct arts_server_s {
  int64_t budget = 0, used = 0;
  struct Lane {
    hipStream_t hs = nullptr;
    BatchBuffers bb;           // descriptor buffers of this lane's persistent launches
    hipEvent_t last = nullptr;  // end of the lane's last tick
  };
  Lane lanes[kMaxLanes];
  int nlanes = kMaxLanes, next_lane = 0;
  hipStream_t copy = nullptr;  // host-to-device chunk copies
  struct Entry {
    arts_stream_s* s = nullptr;
    int64_t bytes = 0;
    bool ready = false;            // a submitted chunk waits for the next tick
    hipEvent_t copied = nullptr;   // the submitted chunk has landed in the stream's input
  };
  std::map<int32_t, Entry> streams;
  int32_t next_id = 0;
};

namespace {

int server_sync(arts_server_s* v) {
  for (int l = 0; l < kMaxLanes; ++l)
    if (v->lanes[l].hs) ARTS_HIP(hipStreamSynchronize(v->lanes[l].hs));
  if (v->copy) ARTS_HIP(hipStreamSynchronize(v->copy));
  return ARTS_OK;
}

void server_free(arts_server_s* v) {
  (void)server_sync(v);
  for (auto& kv : v->streams) {
    arts_stream_destroy(kv.second.s);
    if (kv.second.copied) (void)hipEventDestroy(kv.second.copied);
  }
  for (int l = 0; l < kMaxLanes; ++l) {
    if (v->lanes[l].last) (void)hipEventDestroy(v->lanes[l].last);
    if (v->lanes[l].hs) (void)hipStreamDestroy(v->lanes[l].hs);
  }
  if (v->copy) (void)hipStreamDestroy(v->copy);
  delete v;
}

}  // namespace

extern "C" {

int arts_server_create(int64_t hbm_budget_bytes, arts_server_t* out) {
  if (!out || hbm_budget_bytes < 1) return fail(ARTS_E_INVAL, "bad server arguments");
  *out = nullptr;
  arts_server_s* v = new (std::nothrow) arts_server_s;
  if (!v) return fail(ARTS_E_NOMEM, "host allocation failed");
  v->budget = hbm_budget_bytes;
  bool ok = hipStreamCreateWithFlags(&v->copy, hipStreamNonBlocking) == hipSuccess;
  for (int l = 0; l < kMaxLanes && ok; ++l)
    ok = hipStreamCreateWithFlags(&v->lanes[l].hs, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&v->lanes[l].last, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    server_free(v);
    return fail(ARTS_E_DEVICE, "stream creation failed");
  }
  *out = v;
  return ARTS_OK;
}

int arts_server_set_lanes(arts_server_t v, int32_t nlanes) {
  if (!v) return fail(ARTS_E_INVAL, "server is NULL");
  if (nlanes < 1 || nlanes > kMaxLanes) return fail(ARTS_E_INVAL, "lanes must be 1..%d", kMaxLanes);
  if (int st = server_sync(v)) return st;
  v->nlanes = nlanes;
  v->next_lane = 0;
  return ARTS_OK;
}

void arts_server_destroy(arts_server_t v) {
  if (!v) return;
  server_free(v);
}

int arts_server_open(arts_server_t v, const arts_plan_t* plans, int32_t nplan, int32_t nsrc,
                     const uint8_t* sb_table, int32_t nbeam, int64_t chunk, float threshold,
                     int64_t cand_capacity, int32_t* stream_id) {
  if (!v || !stream_id) return fail(ARTS_E_INVAL, "NULL argument");
  const int64_t need = stream_bytes_needed(plans, nplan, nsrc, nbeam, chunk, cand_capacity);
  if (need < 0) return fail(ARTS_E_INVAL, "bad plans");
  if (v->used + need > v->budget)
    return fail(ARTS_E_BUDGET, "stream needs %lld bytes, %lld of %lld in use", (long long)need,
                (long long)v->used, (long long)v->budget);
  arts_stream_t s = nullptr;
  if (int st = arts_stream_create(plans, nplan, nsrc, sb_table, nbeam, chunk, threshold,
                                  cand_capacity, 0, &s))
    return st;
  arts_server_s::Entry e;
  if (hipEventCreateWithFlags(&e.copied, hipEventDisableTiming) != hipSuccess) {
    arts_stream_destroy(s);
    return fail(ARTS_E_DEVICE, "event creation failed");
  }
  const int32_t id = v->next_id++;
  e.s = s;
  e.bytes = s->device_bytes;
  v->streams[id] = e;
  v->used += e.bytes;
  *stream_id = id;
  return ARTS_OK;
}

int arts_server_close(arts_server_t v, int32_t id) {
  if (!v) return fail(ARTS_E_INVAL, "server is NULL");
  auto it = v->streams.find(id);
  if (it == v->streams.end()) return fail(ARTS_E_INVAL, "no stream %d", id);
  if (int st = server_sync(v)) return st;
  v->used -= it->second.bytes;
  arts_stream_destroy(it->second.s);
  if (it->second.copied) (void)hipEventDestroy(it->second.copied);
  v->streams.erase(it);
  return ARTS_OK;
}

int arts_server_submit(arts_server_t v, int32_t id, const uint8_t* chunk, int32_t from_host) {
  TraceRange range("arts_server_submit");
  if (!v || !chunk) return fail(ARTS_E_INVAL, "NULL argument");
  auto it = v->streams.find(id);
  if (it == v->streams.end()) return fail(ARTS_E_INVAL, "no stream %d", id);
  arts_stream_s* s = it->second.s;
  if (it->second.ready || s->pushed != s->waited)
    return fail(ARTS_E_STATE, "stream %d: the previous chunk is still pending", id);
  const int64_t bytes = static_cast<int64_t>(s->nsrc) * s->nchan * s->chunk;
  // the copy stream does not synchronise with the default stream: order the copy after the
  // work queued there so far (a chunk produced on the device by the caller's default stream)
  ARTS_HIP(hipEventRecord(it->second.copied, nullptr));
  ARTS_HIP(hipStreamWaitEvent(v->copy, it->second.copied, 0));
  ARTS_HIP(hipMemcpyAsync(s->input, chunk, bytes,
                          from_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, v->copy));
  ARTS_HIP(hipEventRecord(it->second.copied, v->copy));
  it->second.ready = true;
  return ARTS_OK;
}

int arts_server_tick(arts_server_t v, int32_t* nrun) {
  TraceRange range("arts_server_tick");
  if (!v) return fail(ARTS_E_INVAL, "server is NULL");
  std::vector<arts_server_s::Entry*> run;
  for (auto& kv : v->streams)
    if (kv.second.ready) run.push_back(&kv.second);
  if (nrun) *nrun = static_cast<int32_t>(run.size());
  if (run.empty()) return ARTS_OK;
  // an idle lane if there is one (its last tick has finished), else the lanes in turn
  int li = v->next_lane;
  for (int k = 0; k < v->nlanes; ++k) {
    const int l = (v->next_lane + k) % v->nlanes;
    if (hipEventQuery(v->lanes[l].last) == hipSuccess) {
      li = l;
      break;
    }
  }
  v->next_lane = (li + 1) % v->nlanes;
  arts_server_s::Lane& lane = v->lanes[li];
  hipStream_t hs = lane.hs;
  std::map<int, std::pair<std::vector<arts_plan_s*>, std::vector<DedispJob>>> groups;
  for (auto* e : run) {
    arts_stream_s* s = e->s;
    ARTS_HIP(hipStreamWaitEvent(hs, e->copied, 0));  // the chunk has landed
    const int parity = static_cast<int>(s->pushed & 1);
    stream_y_step(s);
    if (int st = stream_advance(s, parity, hs)) return st;
    for (size_t p = 0; p < s->plans.size(); ++p) {
      if (s->plans[p]->nsub > 0) {  // subband plans: their own two-step launches
        if (int st = launch_dedisperse(s->plans[p], stream_job(s, parity, p), hs)) return st;
        continue;
      }
      auto& g = groups[s->plans[p]->tiling.variant];
      g.first.push_back(s->plans[p]);
      g.second.push_back(stream_job(s, parity, p));
    }
  }
  for (auto& kv : groups)
    if (int st = launch_dedisperse_batch(kv.second.first.data(), kv.second.second.data(),
                                         static_cast<int>(kv.second.first.size()), lane.bb, hs))
      return st;
  for (auto* e : run) {
    arts_stream_s* s = e->s;
    if (int st = stream_candidates(s, hs)) return st;
    ARTS_HIP(hipEventRecord(s->ev_done, hs));
    ++s->pushed;
    s->y_stale = false;
    e->ready = false;
  }
  ARTS_HIP(hipEventRecord(lane.last, hs));
  return ARTS_OK;
}

int arts_server_poll(arts_server_t v, int32_t id, int32_t* done) {
  if (!v || !done) return fail(ARTS_E_INVAL, "NULL argument");
  auto it = v->streams.find(id);
  if (it == v->streams.end()) return fail(ARTS_E_INVAL, "no stream %d", id);
  const arts_stream_s* s = it->second.s;
  if (it->second.ready) {  // submitted, not yet stepped
    *done = 0;
    return ARTS_OK;
  }
  if (s->pushed == s->waited) {  // nothing in flight
    *done = 1;
    return ARTS_OK;
  }
  const hipError_t e = hipEventQuery(s->ev_done);
  if (e == hipSuccess) {
    *done = 1;
  } else if (e == hipErrorNotReady) {
    *done = 0;
  } else {
    return fail(ARTS_E_DEVICE, "hipEventQuery: %s", hipGetErrorString(e));
  }
  return ARTS_OK;
}

int arts_server_collect(arts_server_t v, int32_t id, arts_candidate* host_out, int64_t capacity,
                        int64_t* count, int64_t* chunk_index) {
  if (!v) return fail(ARTS_E_INVAL, "server is NULL");
  auto it = v->streams.find(id);
  if (it == v->streams.end()) return fail(ARTS_E_INVAL, "no stream %d", id);
  return arts_stream_wait(it->second.s, host_out, capacity, count, chunk_index);
}

int arts_server_stream(arts_server_t v, int32_t id, arts_stream_t* s) {
  if (!v || !s) return fail(ARTS_E_INVAL, "NULL argument");
  auto it = v->streams.find(id);
  if (it == v->streams.end()) return fail(ARTS_E_INVAL, "no stream %d", id);
  *s = it->second.s;
  return ARTS_OK;
}

int arts_server_info(arts_server_t v, int64_t* used_bytes, int64_t* budget, int32_t* nstreams) {
  if (!v) return fail(ARTS_E_INVAL, "server is NULL");
  if (used_bytes) *used_bytes = v->used;
  if (budget) *budget = v->budget;
  if (nstreams) *nstreams = static_cast<int32_t>(v->streams.size());
  return ARTS_OK;
}

}  // extern "C"

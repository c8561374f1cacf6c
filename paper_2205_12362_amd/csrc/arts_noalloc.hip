// Candidate extraction without allocation.  arts_candidates keeps its device buffers (candidate
// records, their counter, the pre-pass row flags) in the plan's workspace and grows it with
// hipMalloc on demand.  arts_candidates_noalloc runs the same kernels on a fixed array in device
// global memory instead, so that callers that may not allocate (inside a serving loop with a
// frozen allocator, harnesses that forbid it) can search a series.
//
// The array below is a device symbol: in host code its name is only a stand-in, so host code
// never passes it to a kernel or a copy.  Its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept; every later use goes through it.
// Each device holds its own copy until the process ends.  All calls on one device share it:
// calls that overlap on one device (two host threads, or two streams in flight) race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "arts_internal.h"

namespace arts {

static __device__ __align__(256) unsigned char scratch[int64_t(16) << 20];

namespace {

// Layout: [0, 256) the candidate counter, then one flag byte per (beam, DM) row, then the
// candidate records.
constexpr int64_t kScratchBytes = int64_t(16) << 20;
constexpr int64_t kCountBytes = 256;
constexpr int64_t kMaxRows = ARTS_NOALLOC_MAX_ROWS;
constexpr int64_t kCandOffset = kCountBytes + kMaxRows;
constexpr int64_t kMaxCand = ARTS_NOALLOC_MAX_CANDIDATES;
static_assert(kCandOffset % 256 == 0, "candidate records start 256-byte aligned");
static_assert(kCandOffset + kMaxCand * int64_t(sizeof(arts_candidate)) <= kScratchBytes,
              "the limits must fit the array");
static_assert(sizeof(scratch) == kScratchBytes, "one size");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first call per device).
int scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(ARTS_E_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(ARTS_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                  hipGetErrorString(e));
    g_scratch[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch[dev];
  return ARTS_OK;
}

}  // namespace
}  // namespace arts

using namespace arts;

extern "C" {

int arts_candidates_noalloc(arts_plan_t p, const int32_t* series, int32_t nbeam, int64_t L,
                            float threshold, int64_t t_offset, int32_t beam_offset,
                            arts_candidate* host_out, int64_t capacity, int64_t* count,
                            void* stream) {
  if (!p) return fail(ARTS_E_INVAL, "plan is NULL");
  if (!series || nbeam < 1 || !count || capacity < 0 || (capacity > 0 && !host_out))
    return fail(ARTS_E_INVAL, "bad pointer or size");
  if (!std::isfinite(threshold)) return fail(ARTS_E_INVAL, "threshold must be finite");
  if (p->cluster)
    return fail(ARTS_E_STATE, "clustered plans need the workspace of arts_candidates");
  const int64_t nrep = L - p->wmax + 1;
  if (nrep < 1) return fail(ARTS_E_SHAPE, "L = %lld shorter than wmax", (long long)L);
  const int64_t rows = static_cast<int64_t>(nbeam) * p->ndm;
  if (rows > kMaxRows)
    return fail(ARTS_E_INVAL, "%lld (beam, DM) rows exceed the no-allocation limit of %lld",
                (long long)rows, (long long)kMaxRows);
  if (capacity > kMaxCand)
    return fail(ARTS_E_INVAL, "capacity %lld exceeds the no-allocation limit of %lld records",
                (long long)capacity, (long long)kMaxCand);
  int dev = 0;
  ARTS_HIP(hipGetDevice(&dev));
  if (dev != p->device)
    return fail(ARTS_E_INVAL, "the plan lives on device %d, the current device is %d",
                p->device, dev);
  unsigned char* base = nullptr;
  if (int st = scratch_address(dev, &base)) return st;
  auto* d_count = reinterpret_cast<unsigned long long*>(base);
  auto* d_flags = base + kCountBytes;
  auto* d_cand = reinterpret_cast<arts_candidate*>(base + kCandOffset);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the array keeps the previous call's contents: the counter starts from zero (a kernel, so
  // no memset node); every flag is written by the pre-pass before it is read
  if (int st = launch_zero_u64(d_count, 1, s)) return st;
  if (int st = launch_candidates(p, series, nbeam, L, nrep, threshold, t_offset, beam_offset,
                                 nullptr, nullptr, d_cand, d_count, capacity, s, 0, d_flags))
    return st;
  unsigned long long n = 0;
  ARTS_HIP(hipMemcpyAsync(&n, d_count, sizeof n, hipMemcpyDeviceToHost, s));
  ARTS_HIP(hipStreamSynchronize(s));
  *count = static_cast<int64_t>(n);
  if (static_cast<int64_t>(n) > capacity)
    return fail(ARTS_E_CAPACITY, "%llu candidates, capacity %lld", n, (long long)capacity);
  if (n == 0) return ARTS_OK;
  ARTS_HIP(hipMemcpyAsync(host_out, d_cand, n * sizeof(arts_candidate), hipMemcpyDeviceToHost,
                          s));
  ARTS_HIP(hipStreamSynchronize(s));
  std::sort(host_out, host_out + n, [](const arts_candidate& a, const arts_candidate& b) {
    if (a.beam != b.beam) return a.beam < b.beam;
    if (a.dm_index != b.dm_index) return a.dm_index < b.dm_index;
    if (a.width != b.width) return a.width < b.width;
    return a.sample < b.sample;
  });
  return ARTS_OK;
}

}  // extern "C"

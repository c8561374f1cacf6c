// Internal declarations shared by the host runtime (arts_host.cpp, arts_batch.cpp,
// arts_stream.cpp) and the device code (arts_kernels.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/arts.h"

namespace arts {

// A named range on the ROCTx marker timeline (seen by rocprofv3 --marker-trace) for the span
// of a host call: each chunk step of streams and servers is bracketed by one.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// Dedispersion kernel shapes compiled into the library.  A workgroup of `waves` wave64s owns
// `waves * acc` consecutive DM trials and one time tile of 64 * j * spd output samples; each
// lane accumulates `acc` DMs x `j * spd` consecutive samples in int32 registers.  spd is the
// number of samples per LDS dword: 4 for native uint8 data, 2 for downsampled 16-bit sums.
struct TileVariant {
  int spd, j, acc, waves, pack;
};
// Outputs of one time tile: 64 lanes of t, less the 4 that a tiling whose lanes share their last
// dword (pack 9 and 11) leaves to the next tile.
constexpr __host__ __device__ int tile_outputs(int t, int pack) {
  return 64 * t - (pack == 9 || pack == 11 ? 4 : 0);
}
// Group-sum tilings (the first subband step only): the packed halves are the group sums
constexpr __host__ __device__ bool is_group(int pack) { return pack == 4 || pack == 11; }
// DM-pair tilings (16-bit samples): per pair and chunk, channels in 16 classes of (first
// trial's sample parity, delay step)
constexpr __host__ __device__ bool is_pairs(int pack) { return pack == 5 || pack == 10; }
extern const TileVariant kVariants[];
extern const int kNumVariants;
int default_variant(int downsample, int64_t ndm);
int fallback_variant(int variant);
constexpr int kPairMaxDeltaHost = 7;  // DM-pair tilings: largest delay step inside a pair
int packed_variant(int64_t ndm);
int split_variant(int64_t ncoarse);

// LDS chunk buffers of a tiling unless set otherwise: one buffer fetched in turn (the CU's
// other workgroups sum meanwhile), which doubles the channels per chunk against two.
constexpr int kDefaultBuffers = 1;

// Widest supported boxcar (the candidate kernels stage a segment plus wmax samples in LDS).
constexpr int kMaxWidth = 16384;

// Tiling tables of a plan for one variant.  The offset lists depend on the alignment class g0
// of the input pointer (0..3 for byte rows, 0..1 for 16-bit rows) and are built on first use.
struct Tiling {
  int variant = -1;
  int m_blk = 0;        // DM trials per workgroup
  int nblk = 0;         // DM blocks
  int rmax = 0;         // largest delay spread inside a block (samples)
  int win_dwords = 0;   // LDS dwords staged per channel (a multiple of 4)
  int cc = 0;           // channels per LDS chunk (<= 255)
  int nbuf = kDefaultBuffers;  // LDS chunk buffers (2: the next chunk's fetch overlaps the sums)
  int nchunk = 0;
  int spd = 4;
  std::vector<int32_t> rel;    // host [nblk][m_blk][nchan] delay - block base
  std::vector<int32_t> base;   // host [nblk][nchan]
  int32_t* d_base = nullptr;   // [nblk][nchan] smallest delay of the block in that channel
  int32_t* d_list[4] = {};     // per g0: [nblk][m_blk][nchan] LDS byte offsets, chunk then m
  uint32_t* d_cnt[4] = {};     // per g0: [nblk][nchunk][m_blk] 4 x 8-bit channel counts per m
};

// Device workspace of the DM-width clustering (arts_cluster.hip): per-row counters and
// offsets for `rows` (beam, DM) rows and per-candidate scratch for lists of up to `cap`.
struct ClusterWs {
  void* d_mem = nullptr;
  int64_t cap = 0, rows = 0, bytes = 0;
};

}  // namespace arts

struct arts_plan_s {
  int device = 0;
  int32_t nchan = 0, ndm = 0, nwidth = 0, ds = 1;
  double f_lo = 0, df = 0, tsamp = 0;
  std::vector<double> dms;
  std::vector<int32_t> widths;
  std::vector<int32_t> delays;  // host [ndm][nchan]
  int32_t max_delay = 0, wmax = 0, halo = 0;
  double tie_margin = 0;
  int32_t* d_delays = nullptr;
  int32_t* d_widths = nullptr;
  double* d_dms = nullptr;
  arts::Tiling tiling;
  int lds_budget = 0;  // bytes of LDS per dedispersion workgroup; 0 = by wave count
  // requested tile shape (arts_plan_set_tiling_shape): LDS buffers and channels per chunk
  // (0: as many as the LDS budget allows)
  int32_t tile_nbuf = arts::kDefaultBuffers, tile_cc = 0;
  // bumped by every change that work captured earlier does not see (tiling tables freed and
  // rebuilt, clustering, integration mode): streams drop their graphs when it moves
  uint64_t generation = 0;
  // workspace, grown on demand outside any timed loop
  int64_t* d_s1 = nullptr;
  double* d_musig = nullptr;
  int64_t stats_cap = 0;  // rows
  arts_candidate* d_cand = nullptr;
  unsigned long long* d_count = nullptr;
  int64_t cand_cap = 0;
  uint8_t* d_flags = nullptr;  // per (beam, DM) row: may hold a candidate (candidate pre-pass)
  int64_t flags_cap = 0;
  uint16_t* d_ds16 = nullptr;  // downsampled rows of one-shot calls with D > 1
  int64_t ds16_cap = 0;        // elements
  uint8_t* d_align = nullptr;  // dword-aligned copy of one-shot inputs with odd row pitch
  int64_t align_cap = 0;       // bytes
  // input rows are 16-bit: downsampled sums (D > 1) or, for the second step of a subband plan,
  // step-1 subband sums; smax is the largest sample value (bounds the packed partial sums)
  bool in16 = false;
  int32_t smax = 255;
  // two-step subband plans (arts_plan_create_subband): per-subband step-1 plans over the coarse
  // DMs, the step-2 plan over the subbands at the fine DMs, and the 16-bit intermediate
  // [nbeam][nsub][ncoarse][pitch] the two share
  int32_t nsub = 0, nfine = 0, ncoarse = 0, max_d1 = 0;
  arts_plan_s* sb1 = nullptr;  // step 1: all channels, coarse DMs, outputs split per subband
  arts_plan_s* sb2 = nullptr;
  // channels per output group (step-1 plans: the subband width; 0: one group).  The kernel
  // writes each group's sums to its own output rows and starts the next group from zero.
  int32_t split = 0;
  uint16_t* d_y = nullptr;
  int64_t y_cap = 0;  // elements
  // DM-width clustering of this plan's candidates (arts_plan_set_cluster) and the workspace of
  // one-shot calls
  bool cluster = false;
  // candidate search: 0 sliding boxcars, 1 decimated integration (each width's absolute grid)
  int32_t integration = 0;
  arts::ClusterWs cl;
  bool is16() const { return ds > 1 || in16; }
};

namespace arts {

// Error reporting: record a message for arts_last_error() and return the status.
int fail(int status, const char* fmt, ...);
#define ARTS_HIP(call)                                                                      \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return ::arts::fail(ARTS_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));    \
  } while (0)

int build_tiling(arts_plan_s* p, int variant);
int ensure_tables(arts_plan_s* p, int g0);
void free_tiling(Tiling& t);
int ensure_stats(arts_plan_s* p, int64_t rows);
int ensure_cand(arts_plan_s* p, int64_t cap);
int ensure_flags(arts_plan_s* p, int64_t rows);
int ensure_ds16(arts_plan_s* p, int64_t elems);
int ensure_align(arts_plan_s* p, int64_t bytes);

// One dedispersion job: which rows to read and where to write.
struct DedispJob {
  const uint8_t* in = nullptr;     // row (src, c) starts at in + (src * nchan + c) * pitch
  int64_t in_bytes = 0;            // extent of `in` (bounds for vector loads)
  int64_t nin = 0;                 // native samples per row
  int64_t pitch = 0;               // bytes between rows (>= nin)
  int32_t nsrc = 0;                // source beams in `in`
  const uint16_t* in16 = nullptr;  // downsampled rows for plans with D > 1 (nin / D valid)
  int64_t in16_elems = 0;          // extent of in16
  int64_t pitch16 = 0;             // elements between downsampled rows (even)
  const uint8_t* sb_table = nullptr;  // optional [nbeam][nchan] -> source beam index
  int32_t nbeam = 0;
  int32_t* out = nullptr;          // [nbeam][ndm][nout]
  int64_t nout = 0;
  // layout overrides (0 / false: the plain layout above)
  int32_t src_stride = 0;          // rows between source beams in `in` / `in16` (default nchan)
  int32_t tbl_stride = 0;          // sb_table entries between beams (default nchan)
  int64_t out_pitch = 0;           // out elements between DM rows (default nout)
  int64_t out_bstride = 0;         // out elements between beams (default ndm * out_pitch)
  int64_t out_sstride = 0;         // out elements between channel groups (plans with a split)
  bool out16 = false;              // store the sums as uint16 (the caller bounds them)
  int64_t in16_blk = 0;            // in16 elements added per DM block
  // subband plans: the caller's 16-bit intermediate (streams own one; null: the plan's).  Row r
  // of the window starts at y + r * y_pitch + y_pad (y_pitch 0: the plan's own pitch), chosen
  // so that the new samples start 8-byte aligned.  With y_prev (the previous chunk's window,
  // same pitch) only the last y_new step-1 samples are computed; the rest are the previous
  // window's samples [y_new, L1), copied unless y_prev + y_new == y (already in place).
  // y_elems: elements from y to the end of its buffer; [y_lo, y_hi): the buffer y_prev lies in.
  uint16_t* y = nullptr;
  const uint16_t* y_prev = nullptr;
  int64_t y_elems = 0;
  int64_t y_new = 0;
  int32_t y_pad = 0;
  int64_t y_pitch = 0;
  const uint16_t* y_lo = nullptr;
  const uint16_t* y_hi = nullptr;
};

int launch_dedisperse(arts_plan_s* p, const DedispJob& job, hipStream_t s);
// Workgroups per CU that registers and waves allow (LDS aside) for a tiling variant's kernel
// of one kind; 0 if the runtime cannot tell or the variant has no kernel of that kind.
constexpr int kOccPlain = 0, kOccSplit = 1, kOccBatch = 2;
int variant_occupancy(int variant, int kind);
int variant_blocks_per_cu(int variant, bool split);
// false for a plan in decimated integration whose widths do not all divide nrep
bool integration_grid_ok(const arts_plan_s* p, int64_t nrep);
// Subband plans: elements of the 16-bit intermediate for nbeam beams of nin samples.
int64_t subband_ws_elems(const arts_plan_s* p, int32_t nbeam, int64_t nin);
// Row pitch of a subband plan's step-1 rows: L1 = nin - max step-1 delay samples after a front
// pad of `pad` elements, rounded to 4 (8-byte aligned rows).
int64_t subband_pitch(const arts_plan_s* p, int64_t nin, int32_t pad);
// Subband plans: the step plans' offset tables for input alignment class g0 and, if
// plan_ws, the plan's own intermediate for nbeam x nin, so that a later launch allocates
// nothing.  Other plans: their tables for g0.
int prepare_plan(arts_plan_s* p, int32_t nbeam, int64_t nin, int g0, bool plan_ws);

// Device descriptor storage of persistent batch launches (reused across calls).
struct BatchBuffers {
  void* d_jobs = nullptr;      // job descriptors
  int64_t* d_start = nullptr;  // prefix sums of tiles per job
  unsigned long long* d_counter = nullptr;
  void* h_stage = nullptr;     // pinned staging of the descriptors
  size_t stage_bytes = 0;
  int cap = 0;
  hipEvent_t ev = nullptr;     // marks the last descriptor upload
  ~BatchBuffers();
};
// One persistent launch over the tiles of n jobs whose plans share a tiling variant.
int launch_dedisperse_batch(arts_plan_s* const* plans, const DedispJob* jobs, int n,
                            BatchBuffers& bb, hipStream_t s);
int launch_row_stats(const int32_t* series, int64_t L, int64_t nrep, int64_t nrows,
                     int64_t* s1, double* musig, hipStream_t s);
int launch_candidates(const arts_plan_s* p, const int32_t* series, int32_t nbeam, int64_t L,
                      int64_t nrep, float thr, int64_t t_offset, int32_t beam_offset,
                      const int64_t* s1, const double* musig, arts_candidate* cand,
                      unsigned long long* count, int64_t cap, hipStream_t s,
                      int64_t t_begin = 0, uint8_t* flags = nullptr);
int launch_boxcar_snr(const arts_plan_s* p, const int32_t* series, int32_t nbeam, int64_t L,
                      int64_t nrep, const int64_t* s1, const double* musig, int32_t* sums,
                      float* snr, hipStream_t s);
int launch_sb_gather(const uint8_t* tab, int32_t ntab, const uint8_t* sb_table, int32_t nsb,
                     int32_t nchan, int64_t nsamp, uint8_t* out, hipStream_t s);
int launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
int launch_fill_random(uint8_t* p, int64_t n, uint64_t seed, hipStream_t s);
// DM-width clustering.  launch_cluster replaces the candidates cand[beg, *count) by one per
// cluster (cand[beg, beg + clusters), *count updated on the device), where beg is 0 or, with
// from_mark, the value of *count that launch_cluster_mark saved before the plan's candidates
// were appended.  `cap` is the list capacity: a larger *count (dropped appends) or an invalid
// record leaves the list unchanged (read_cluster_status tells which).
int64_t cluster_ws_bytes(int64_t cap, int64_t rows);
int ensure_cluster_ws(ClusterWs& w, int64_t cap, int64_t rows);
void free_cluster_ws(ClusterWs& w);
int launch_cluster_mark(ClusterWs& w, const unsigned long long* count, hipStream_t s);
int launch_cluster(ClusterWs& w, arts_candidate* cand, unsigned long long* count, int64_t cap,
                   bool from_mark, int32_t nbeam, int32_t ndm, int32_t beam_offset,
                   hipStream_t s);
int read_cluster_status(ClusterWs& w, int* skipped, int* bad, hipStream_t s);
// RFI mitigation of [nrow][nchan] rows of `pitch` bytes (nsamp used), in place; the workspace
// has rfi_ws_bytes(nrow, nchan, nsamp) bytes.
int64_t rfi_ws_bytes(int32_t nrow, int32_t nchan, int64_t nsamp);
int launch_rfi(uint8_t* x, int32_t nrow, int32_t nchan, int64_t nsamp, int64_t pitch,
               float k_time, int32_t niter_time, float k_freq, int32_t niter_freq, void* ws,
               hipStream_t s);
// Offline clustering over time / DM windows (arts_cluster_offline).  The workspace of
// offline_ws_bytes(n, nedge) bytes holds a counter, the hash table, the DM edges (copy them to
// offline_edges(ws, n) first) and the output records; *out, *d_count and *d_bad point into it.
int64_t offline_ws_bytes(int64_t n, int32_t nedge);
double* offline_edges(void* ws, int64_t n);
int launch_cluster_offline(const arts_candidate* cand, int64_t n, int64_t t_window,
                           const double* d_edges, int32_t nedge, float min_snr, void* ws,
                           arts_candidate** out, unsigned long long** d_count, int** d_bad,
                           hipStream_t s);
// dst[r][s] = sum of D consecutive src bytes, s < nout (16-bit rows, pitches in elements/bytes)
int launch_downsample(uint16_t* dst, int64_t dpitch, const uint8_t* src, int64_t spitch,
                      int64_t nrows, int64_t nout, int32_t D, hipStream_t s);
// dst[r * dpitch + i] = src[r * spitch + i] for r < nrows, i < n (byte rows at any alignment)
int launch_copy_rows(uint8_t* dst, int64_t dpitch, const uint8_t* src, int64_t spitch,
                     int64_t nrows, int64_t n, const uint8_t* src_begin, const uint8_t* src_end,
                     hipStream_t s);

}  // namespace arts

struct arts_stream_s {
  std::vector<arts_plan_s*> plans;
  int32_t nsrc = 0, nbeam = 0, nchan = 0;
  const uint8_t* sb_table = nullptr;
  int64_t chunk = 0, hmax = 0, W = 0;
  float thr = 0;
  uint32_t flags = 0;
  uint8_t* ring[2] = {nullptr, nullptr};  // native rows (only if a plan has D = 1)
  uint8_t* input = nullptr;  // stream-owned staging buffer [nsrc][nchan][chunk]
  std::vector<uint16_t*> ring16[2];        // per plan: downsampled rows (D > 1), else null
  std::vector<int64_t> W16;                // per plan: 16-bit ring row pitch (even)
  std::vector<int64_t> N16;                // per plan: 16-bit samples held per row
  std::vector<int32_t*> series;
  std::vector<int64_t> L, H;
  // per plan, subband plans only: one buffer of step-1 rows whose window origin moves by one
  // chunk per push (y_at chunks in, at most y_m) and is compacted back to 0 after that
  std::vector<uint16_t*> ybuf;
  std::vector<int64_t> y_elems;            // buffer elements
  std::vector<int64_t> y_pitch;            // row pitch (elements)
  std::vector<int32_t> y_pad, y_m, y_at, y_from;  // y_from: previous origin, -1: none
  bool y_stale = false;                    // after a restore: the next push recomputes step 1
  arts_candidate* d_cand = nullptr;
  unsigned long long* d_count = nullptr;
  unsigned long long* h_count = nullptr;  // pinned
  uint8_t* d_flags = nullptr;              // candidate pre-pass: nbeam x max ndm rows
  std::vector<char> cluster;               // per plan: cluster its candidates (set at creation)
  arts::ClusterWs cl;
  // RFI mitigation of each pushed chunk (arts_stream_set_rfi): thresholds, iterations, workspace
  float rfi_kt = 0, rfi_kf = 0;
  int32_t rfi_nt = 0, rfi_nf = 0;
  void* rfi_ws = nullptr;
  int64_t cap = 0;
  hipStream_t hs = nullptr;
  hipEvent_t ev_in = nullptr, ev_done = nullptr;
  // captured pushes, keyed by the ring parity and each subband plan's window origin
  std::map<std::vector<int>, hipGraphExec_t> graphs;
  std::vector<uint64_t> plan_gen;  // the plans' generations the graphs were captured at
  bool eager_next = false;         // the next push runs eagerly (after the plans changed)
  int64_t pushed = 0, waited = 0;
  int64_t device_bytes = 0;
  // profiling: events bracketing each phase of the last push
  std::vector<hipEvent_t> pev;
  std::vector<double> phase_ms;
  std::vector<int64_t> phase_n;
  bool pending_profile = false;
};

namespace arts {

// Stream internals (arts_stream.cpp), shared with the serving engine (arts_server.cpp).
int stream_advance(arts_stream_s* s, int parity, hipStream_t hs);
// Moves each subband plan's step-1 window for the next push (once per push, before its jobs).
void stream_y_step(arts_stream_s* s);
DedispJob stream_job(arts_stream_s* s, int parity, size_t plan_index);
// Output samples of chunk k whose dedispersion window starts before the stream's first input
// sample (they read the zero history) are left out of the statistics and the search: plan p
// searches t in [stream_warmup(s, p, k), chunk / D).  All zero once k * chunk >= D * halo.
int64_t stream_warmup(const arts_stream_s* s, size_t plan_index, int64_t k);
bool stream_warm(const arts_stream_s* s, int64_t k);
// Candidate search of chunk k = s->pushed over every plan's series.
int stream_candidates(arts_stream_s* s, hipStream_t hs);
int64_t stream_bytes_needed(const arts_plan_t* plans, int32_t nplan, int32_t nsrc, int32_t nbeam,
                            int64_t chunk, int64_t cand_capacity);

}  // namespace arts

// Host runtime of libarts: argument validation, the FP64 delay table, plan lifecycle, tiling
// tables of the dedispersion kernel, workspace management and the C entry points of the
// plain (one call per step) path.
#include <algorithm>
#include <cfenv>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>

#include "arts_internal.h"

namespace arts {

static thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

// Cold-plasma dispersion constant, s MHz^2 pc^-1 cm^3 (the paper does not state the law; this
// is the standard t = k DM / f^2).
static constexpr double kDispersion = 4.148808e3;

static int compute_delays(int32_t nchan, double f_lo, double df, double tsamp,
                          const double* dms, int32_t ndm, int32_t ds, int32_t* out,
                          double* tie_margin) {
  if (nchan < 1) return fail(ARTS_E_INVAL, "nchan must be >= 1 (got %d)", nchan);
  if (ndm < 1 || !dms) return fail(ARTS_E_INVAL, "need at least one DM trial");
  if (!std::isfinite(f_lo) || !std::isfinite(df) || df == 0.0)
    return fail(ARTS_E_INVAL, "f_lo and df must be finite and df != 0");
  if (!(tsamp > 0.0) || !std::isfinite(tsamp))
    return fail(ARTS_E_INVAL, "tsamp must be finite and > 0");
  if (ds < 1) return fail(ARTS_E_INVAL, "downsample must be >= 1");
  std::vector<double> f(nchan);
  double f_ref = -std::numeric_limits<double>::infinity();
  for (int32_t c = 0; c < nchan; ++c) {
    f[c] = f_lo + static_cast<double>(c) * df;
    if (!(f[c] > 0.0)) return fail(ARTS_E_INVAL, "channel %d has frequency <= 0", c);
    f_ref = std::max(f_ref, f[c]);
  }
  const double inv_ref = 1.0 / (f_ref * f_ref);
  const double step = static_cast<double>(ds) * tsamp;
  double margin = std::numeric_limits<double>::infinity();
  const int old_round = std::fegetround();
  std::fesetround(FE_TONEAREST);  // nearbyint below rounds half to even
  for (int32_t d = 0; d < ndm; ++d) {
    const double dm = dms[d];
    if (!std::isfinite(dm) || dm < 0.0) {
      std::fesetround(old_round);
      return fail(ARTS_E_INVAL, "DM %d is negative or not finite", d);
    }
    for (int32_t c = 0; c < nchan; ++c) {
      const double x = kDispersion * dm * (1.0 / (f[c] * f[c]) - inv_ref) / step;
      if (!(x <= 1073741824.0)) {
        std::fesetround(old_round);
        return fail(ARTS_E_INVAL, "delay of DM %g in channel %d exceeds 2^30 samples", dm, c);
      }
      const double r = std::nearbyint(x);
      margin = std::min(margin, std::fabs((x - std::floor(x)) - 0.5));
      out[static_cast<int64_t>(d) * nchan + c] = static_cast<int32_t>(r);
    }
  }
  std::fesetround(old_round);
  if (tie_margin) *tie_margin = margin;
  return ARTS_OK;
}

void free_tiling(Tiling& t) {
  if (t.d_base) (void)hipFree(t.d_base);
  for (int g = 0; g < 4; ++g) {
    if (t.d_list[g]) (void)hipFree(t.d_list[g]);
    if (t.d_cnt[g]) (void)hipFree(t.d_cnt[g]);
  }
  t = Tiling{};
}

// Geometry of the dedispersion kernel for one variant (see the kernel's description): DM
// blocks, per-block window base per channel, window length and chunking.  The per-alignment
// offset lists are made by ensure_tables.
int build_tiling(arts_plan_s* p, int variant) {
  if (variant < 0 || variant >= kNumVariants)
    return fail(ARTS_E_INVAL, "tiling variant %d out of range [0, %d)", variant, kNumVariants);
  const TileVariant& v = kVariants[variant];
  if (p->nsub > 0) {  // subband plans: the variant of the step-1 plan
    if (v.spd != 4 || v.pack == 2)
      return fail(ARTS_E_INVAL, "variant %d cannot run the first subband step", variant);
    if (int st = build_tiling(p->sb1, variant)) return st;
    p->tiling.variant = variant;
    ++p->generation;
    return ARTS_OK;
  }
  if (p->is16() != (v.spd == 2))
    return fail(ARTS_E_INVAL, "variant %d is for %s data", variant,
                v.spd == 4 ? "byte (native)" : "16-bit (downsampled)");
  // group-sum tilings keep a channel group's sums in 16-bit halves: split plans with groups of
  // at most 257 byte channels
  if (is_group(v.pack) && (p->split <= 0 || p->split > 257))
    return fail(ARTS_E_INVAL, "variant %d runs the first subband step only (groups of at most "
                "257 channels)", variant);
  Tiling t;
  t.variant = variant;
  t.spd = v.spd;
  t.m_blk = v.acc * v.waves;
  t.nblk = static_cast<int>((p->ndm + t.m_blk - 1) / t.m_blk);
  const int64_t nchan = p->nchan;
  const int shift = v.spd == 4 ? 2 : 1;
  t.rel.assign(static_cast<size_t>(t.nblk) * t.m_blk * nchan, 0);
  t.base.assign(static_cast<size_t>(t.nblk) * nchan, 0);
  int rmax = 0;
  for (int b = 0; b < t.nblk; ++b) {
    const int d0 = b * t.m_blk, d1 = std::min<int>(p->ndm, d0 + t.m_blk);
    for (int64_t c = 0; c < nchan; ++c) {
      int32_t lo = std::numeric_limits<int32_t>::max();
      for (int d = d0; d < d1; ++d) lo = std::min(lo, p->delays[d * nchan + c]);
      t.base[b * nchan + c] = lo;
      for (int d = d0; d < d1; ++d) {
        const int32_t r = p->delays[d * nchan + c] - lo;
        t.rel[(static_cast<int64_t>(b) * t.m_blk + (d - d0)) * nchan + c] = r;
        rmax = std::max(rmax, r);
      }
    }
  }
  t.rmax = rmax;
  if (is_pairs(v.pack)) {
    // DM pairs read one window per pair: the second trial may start at most kPairMaxDeltaHost
    // samples after the first, never before it
    if (t.m_blk % 2 != 0) return fail(ARTS_E_INVAL, "variant %d: odd DMs per block", variant);
    for (int b = 0; b < t.nblk; ++b)
      for (int x = 0; x + 1 < t.m_blk && b * t.m_blk + x + 1 < p->ndm; x += 2)
        for (int64_t c = 0; c < nchan; ++c) {
          const int64_t r0 = (static_cast<int64_t>(b) * t.m_blk + x) * nchan + c;
          const int32_t dlt = t.rel[r0 + nchan] - t.rel[r0];
          if (dlt < 0 || dlt > kPairMaxDeltaHost)
            return fail(ARTS_E_INVAL,
                        "variant %d: trials %d and %d differ by %d samples in channel %lld "
                        "(DM pairs need 0..%d)", variant, b * t.m_blk + x,
                        b * t.m_blk + x + 1, dlt, (long long)c, kPairMaxDeltaHost);
        }
  }
  // lane 63 reads dwords 63 j + ((r + g) >> shift) .. + j, with g < spd the window's alignment
  t.win_dwords = (64 * v.j + ((rmax + v.spd - 1) >> shift) + 1 + 3) & ~3;
  // LDS per workgroup: a CU's 160 KiB shared by the workgroups that its registers and waves
  // allow, assuming at least 16 waves per CU
  int64_t budget = p->lds_budget;
  if (budget <= 0) {
    const int nwg = std::max(variant_blocks_per_cu(variant, p->split > 0), 16 / v.waves);
    budget = std::max<int64_t>(16 * 1024, 160 * 1024 / nwg - 1024);
  }
  // nbuf buffers (each with 4 pad words) and an SB-table row; per channel its window plus one
  // offset-list entry per DM of the block
  t.nbuf = p->tile_nbuf;
  const int64_t per_buf = (budget - ((nchan + 3) & ~int64_t(3))) / t.nbuf - 16;
  // a chunk's channels must fit the kernels' narrow partial sums: 8-bit counts of each run, and
  // for packed 16-bit samples (sums of D bytes) a 16-bit half per output
  const int64_t cc_max = (v.pack && v.spd == 2) ? std::min<int64_t>(255, 65535 / p->smax) : 255;
  if (cc_max < 1)
    return fail(ARTS_E_INVAL, "variant %d: samples up to %d overflow its 16-bit partial sums",
                variant, p->smax);
  int cc = static_cast<int>(
      std::min<int64_t>({nchan, cc_max, per_buf / (4LL * (t.win_dwords + t.m_blk))}));
  if (p->tile_cc > 0) cc = std::min(cc, p->tile_cc);
  // DM pairs in raw frames hold a pair's offset list one entry per lane
  if (v.pack == 10) cc = std::min(cc, 64);
  // split plans: chunks must not straddle channel groups, so cc divides the group size
  if (p->split > 0)
    while (cc > 1 && p->split % cc != 0) --cc;
  if (cc < 1)
    return fail(ARTS_E_INVAL,
                "variant %d: one channel's window (%d B) exceeds the LDS budget (%lld B); the DM "
                "trials are too widely spaced for this block size",
                variant, t.win_dwords * 4, (long long)budget);
  t.cc = cc;
  t.nchunk = static_cast<int>((nchan + cc - 1) / cc);
  hipError_t e = hipMalloc(&t.d_base, t.base.size() * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpy(t.d_base, t.base.data(), t.base.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_tiling(t);
    return fail(e == hipErrorOutOfMemory ? ARTS_E_NOMEM : ARTS_E_DEVICE,
                "tiling tables: %s", hipGetErrorString(e));
  }
  free_tiling(p->tiling);
  p->tiling = std::move(t);
  ++p->generation;
  return ARTS_OK;
}

// Offset lists for inputs whose pointer has alignment class g0: channel c's window then starts
// g_c = (g0 + base_c) mod spd samples before its first needed sample, so trial d reads from
// r = rel + g_c; channels are ordered by m = r mod spd within each chunk.
int ensure_tables(arts_plan_s* p, int g0) {
  Tiling& t = p->tiling;
  if (g0 < 0 || g0 >= t.spd) return fail(ARTS_E_INVAL, "alignment class %d", g0);
  if (t.d_list[g0]) return ARTS_OK;
  const int64_t nchan = p->nchan;
  const int shift = t.spd == 4 ? 2 : 1;
  std::vector<int32_t> list(t.rel.size(), 0);
  std::vector<uint32_t> cnt(static_cast<size_t>(t.nblk) * t.nchunk * t.m_blk, 0);
  const bool pairs = is_pairs(kVariants[t.variant].pack);
  if (pairs) {
    // per DM pair (trials 2P, 2P + 1 of the block) and chunk: channels ordered by class
    // m0 * (max delta + 1) + delta, m0 = first trial's offset parity, delta = the second
    // trial's offset minus the first's (its window is read from the first trial's word)
    const int npair = t.m_blk / 2, ncls = 2 * (kPairMaxDeltaHost + 1);
    list.assign(static_cast<size_t>(t.nblk) * npair * nchan, 0);
    cnt.assign(static_cast<size_t>(t.nblk) * t.nchunk * npair * 4, 0);
    for (int b = 0; b < t.nblk; ++b) {
      const int32_t* base = &t.base[static_cast<int64_t>(b) * nchan];
      for (int pr = 0; pr < npair; ++pr) {
        const int32_t* r0 = &t.rel[(static_cast<int64_t>(b) * t.m_blk + 2 * pr) * nchan];
        const int32_t* r1 = r0 + nchan;
        const bool second = b * t.m_blk + 2 * pr + 1 < p->ndm;  // else a copy of the first
        int32_t* l = &list[(static_cast<int64_t>(b) * npair + pr) * nchan];
        for (int ch = 0; ch < t.nchunk; ++ch) {
          const int c0 = ch * t.cc, c1 = static_cast<int>(std::min<int64_t>(nchan, c0 + t.cc));
          int k = c0;
          uint32_t* cw = &cnt[((static_cast<int64_t>(b) * t.nchunk + ch) * npair + pr) * 4];
          for (int cls = 0; cls < ncls; ++cls) {
            int n = 0;
            for (int c = c0; c < c1; ++c) {
              const int32_t g = (g0 + base[c]) & 1;
              const int32_t a0 = r0[c] + g;
              const int32_t dlt = second ? r1[c] - r0[c] : 0;
              if ((a0 & 1) * (kPairMaxDeltaHost + 1) + dlt != cls) continue;
              l[k++] = 4 * ((c - c0) * t.win_dwords + (a0 >> 1));  // LDS byte offset
              ++n;
            }
            cw[cls / 4] |= static_cast<uint32_t>(n) << (8 * (cls % 4));
          }
        }
      }
    }
  }
  for (int b = 0; b < t.nblk && !pairs; ++b) {
    const int32_t* base = &t.base[static_cast<int64_t>(b) * nchan];
    for (int x = 0; x < t.m_blk; ++x) {
      const int32_t* r = &t.rel[(static_cast<int64_t>(b) * t.m_blk + x) * nchan];
      int32_t* l = &list[(static_cast<int64_t>(b) * t.m_blk + x) * nchan];
      for (int ch = 0; ch < t.nchunk; ++ch) {
        const int c0 = ch * t.cc, c1 = static_cast<int>(std::min<int64_t>(nchan, c0 + t.cc));
        int k = c0;
        uint32_t packed = 0;
        for (int m = 0; m < t.spd; ++m) {
          int n = 0;
          for (int c = c0; c < c1; ++c) {
            const int32_t rr = r[c] + ((g0 + base[c]) & (t.spd - 1));
            if ((rr & (t.spd - 1)) != m) continue;
            l[k++] = 4 * ((c - c0) * t.win_dwords + (rr >> shift));  // LDS byte offset
            ++n;
          }
          packed |= static_cast<uint32_t>(n) << (8 * m);
        }
        cnt[(static_cast<int64_t>(b) * t.nchunk + ch) * t.m_blk + x] = packed;
      }
    }
  }
  int32_t* dl = nullptr;
  uint32_t* dc = nullptr;
  hipError_t e = hipMalloc(&dl, list.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&dc, cnt.size() * sizeof(uint32_t));
  if (e == hipSuccess)
    e = hipMemcpy(dl, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(dc, cnt.data(), cnt.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (dl) (void)hipFree(dl);
    if (dc) (void)hipFree(dc);
    return fail(e == hipErrorOutOfMemory ? ARTS_E_NOMEM : ARTS_E_DEVICE, "offset tables: %s",
                hipGetErrorString(e));
  }
  t.d_list[g0] = dl;
  t.d_cnt[g0] = dc;
  return ARTS_OK;
}

int ensure_stats(arts_plan_s* p, int64_t rows) {
  if (rows <= p->stats_cap) return ARTS_OK;
  if (p->d_s1) (void)hipFree(p->d_s1);
  if (p->d_musig) (void)hipFree(p->d_musig);
  p->d_s1 = nullptr;
  p->d_musig = nullptr;
  p->stats_cap = 0;
  ARTS_HIP(hipMalloc(&p->d_s1, rows * sizeof(int64_t)));
  ARTS_HIP(hipMalloc(&p->d_musig, rows * 2 * sizeof(double)));
  p->stats_cap = rows;
  return ARTS_OK;
}

int ensure_cand(arts_plan_s* p, int64_t cap) {
  if (!p->d_count) ARTS_HIP(hipMalloc(&p->d_count, 2 * sizeof(unsigned long long)));
  if (cap <= p->cand_cap && p->d_cand) return ARTS_OK;
  if (p->d_cand) (void)hipFree(p->d_cand);
  p->d_cand = nullptr;
  p->cand_cap = 0;
  const int64_t n = std::max<int64_t>(cap, 1024);
  ARTS_HIP(hipMalloc(&p->d_cand, n * sizeof(arts_candidate)));
  p->cand_cap = n;
  return ARTS_OK;
}

int ensure_flags(arts_plan_s* p, int64_t rows) {
  if (rows <= p->flags_cap && p->d_flags) return ARTS_OK;
  if (p->d_flags) (void)hipFree(p->d_flags);
  p->d_flags = nullptr;
  p->flags_cap = 0;
  ARTS_HIP(hipMalloc(&p->d_flags, rows));
  p->flags_cap = rows;
  return ARTS_OK;
}

int ensure_ds16(arts_plan_s* p, int64_t elems) {
  if (elems <= p->ds16_cap) return ARTS_OK;
  if (p->d_ds16) (void)hipFree(p->d_ds16);
  p->d_ds16 = nullptr;
  p->ds16_cap = 0;
  ARTS_HIP(hipMalloc(&p->d_ds16, elems * sizeof(uint16_t)));
  p->ds16_cap = elems;
  return ARTS_OK;
}

int ensure_align(arts_plan_s* p, int64_t bytes) {
  if (bytes <= p->align_cap) return ARTS_OK;
  if (p->d_align) (void)hipFree(p->d_align);
  p->d_align = nullptr;
  p->align_cap = 0;
  ARTS_HIP(hipMalloc(&p->d_align, bytes));
  p->align_cap = bytes;
  return ARTS_OK;
}

// One-shot dedispersion.  The kernel needs dword-aligned rows: inputs whose row pitch is not a
// multiple of 4 are first copied into a padded workspace; plans with D > 1 first downsample
// every source row once into 16-bit rows of even pitch.
static int run_dedisperse(arts_plan_s* p, DedispJob job, hipStream_t s) {
  const int64_t rows = static_cast<int64_t>(job.nsrc) * p->nchan;
  if (p->ds > 1) {
    const int64_t nd = job.nin / p->ds;
    const int64_t pitch16 = (nd + 1) & ~int64_t(1);
    if (int st = ensure_ds16(p, rows * pitch16)) return st;
    if (int st = launch_downsample(p->d_ds16, pitch16, job.in, job.pitch, rows, nd, p->ds, s))
      return st;
    job.in16 = p->d_ds16;
    job.in16_elems = rows * pitch16;
    job.pitch16 = pitch16;
  } else if (job.pitch % 4 != 0) {
    const int64_t pitch = (job.nin + 3) & ~int64_t(3);
    if (int st = ensure_align(p, rows * pitch)) return st;
    if (int st = launch_copy_rows(p->d_align, pitch, job.in, job.pitch, rows, job.nin, job.in,
                                  job.in + job.in_bytes, s))
      return st;
    job.in = p->d_align;
    job.pitch = pitch;
    job.in_bytes = rows * pitch;
  }
  if (p->nsub > 0)
    if (int st = prepare_plan(p, job.nbeam, job.nin,
                              static_cast<int>(reinterpret_cast<uintptr_t>(job.in) & 3u), true))
      return st;
  return launch_dedisperse(p, job, s);
}

static void plan_free(arts_plan_s* p) {
  if (!p) return;
  plan_free(p->sb1);
  plan_free(p->sb2);
  if (p->d_y) (void)hipFree(p->d_y);
  if (p->d_ds16) (void)hipFree(p->d_ds16);
  if (p->d_align) (void)hipFree(p->d_align);
  free_tiling(p->tiling);
  if (p->d_delays) (void)hipFree(p->d_delays);
  if (p->d_widths) (void)hipFree(p->d_widths);
  if (p->d_dms) (void)hipFree(p->d_dms);
  if (p->d_s1) (void)hipFree(p->d_s1);
  if (p->d_musig) (void)hipFree(p->d_musig);
  if (p->d_cand) (void)hipFree(p->d_cand);
  if (p->d_count) (void)hipFree(p->d_count);
  if (p->d_flags) (void)hipFree(p->d_flags);
  free_cluster_ws(p->cl);
  delete p;
}

static int check_widths(int32_t nchan, int32_t ds, const int32_t* widths, int32_t nwidth) {
  if (nwidth < 1 || !widths) return fail(ARTS_E_INVAL, "need at least one boxcar width");
  for (int32_t i = 0; i < nwidth; ++i) {
    if (widths[i] < 1 || (i > 0 && widths[i] <= widths[i - 1]))
      return fail(ARTS_E_INVAL, "widths must be >= 1 and strictly increasing");
  }
  if (nwidth > 64) return fail(ARTS_E_INVAL, "at most 64 boxcar widths");
  if (widths[nwidth - 1] > kMaxWidth)
    return fail(ARTS_E_INVAL, "widths above %d samples are not supported", kMaxWidth);
  if (static_cast<int64_t>(nchan) * 255 * ds * widths[nwidth - 1] >= (int64_t(1) << 31))
    return fail(ARTS_E_INVAL, "nchan * 255 * D * wmax must stay below 2^31 (exact int32 sums)");
  return ARTS_OK;
}

// Device copies of a plan's delay table, widths and DM values.
static int upload_plan(arts_plan_s* p) {
  if (hipError_t ge = hipGetDevice(&p->device); ge != hipSuccess)
    return fail(ARTS_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(ge));
  hipError_t e = hipMalloc(&p->d_delays, p->delays.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&p->d_widths, p->nwidth * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&p->d_dms, p->ndm * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_delays, p->delays.data(), p->delays.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_widths, p->widths.data(), p->nwidth * sizeof(int32_t),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(p->d_dms, p->dms.data(), p->ndm * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? ARTS_E_NOMEM : ARTS_E_DEVICE, "plan upload: %s",
                hipGetErrorString(e));
  return ARTS_OK;
}

// in16: the plan reads 16-bit rows of samples up to smax without downsampling (the second step
// of a subband plan); variant >= 0 forces that tiling; delays (host [ndm][nchan], nullable)
// replaces the computed table and split sets channel groups (the first step of a subband plan).
static int plan_create(int32_t nchan, double f_lo, double df, double tsamp, const double* dms,
                       int32_t ndm, const int32_t* widths, int32_t nwidth, int32_t ds,
                       arts_plan_t* out, bool in16 = false, int32_t smax = 0,
                       int variant = -1, const int32_t* delays = nullptr, int32_t split = 0) {
  if (!out) return fail(ARTS_E_INVAL, "out is NULL");
  *out = nullptr;
  if (ds > 257) return fail(ARTS_E_INVAL, "downsample must be <= 257 (16-bit sums)");
  if (int st = check_widths(nchan, ds, widths, nwidth)) return st;
  arts_plan_s* p = new (std::nothrow) arts_plan_s;
  if (!p) return fail(ARTS_E_NOMEM, "host allocation failed");
  p->nchan = nchan;
  p->ndm = ndm;
  p->nwidth = nwidth;
  p->ds = ds;
  p->f_lo = f_lo;
  p->df = df;
  p->tsamp = tsamp;
  if (ndm >= 1 && dms) p->dms.assign(dms, dms + ndm);
  p->widths.assign(widths, widths + nwidth);
  p->delays.resize(static_cast<size_t>(std::max(ndm, 1)) * std::max(nchan, 1));
  int st = ARTS_OK;
  if (delays)
    std::copy(delays, delays + p->delays.size(), p->delays.begin());
  else
    st = compute_delays(nchan, f_lo, df, tsamp, dms, ndm, ds, p->delays.data(), &p->tie_margin);
  if (st != ARTS_OK) {
    delete p;
    return st;
  }
  p->split = split;
  p->max_delay = *std::max_element(p->delays.begin(), p->delays.end());
  p->wmax = widths[nwidth - 1];
  p->halo = p->max_delay + p->wmax - 1;
  p->in16 = in16;
  p->smax = smax > 0 ? smax : 255 * ds;
  if ((st = upload_plan(p)) != ARTS_OK) {
    plan_free(p);
    return st;
  }
  st = build_tiling(p, variant >= 0 ? variant : default_variant(ds, ndm));
  if (st != ARTS_OK && variant < 0 && fallback_variant(default_variant(ds, ndm)) >= 0)
    st = build_tiling(p, fallback_variant(default_variant(ds, ndm)));
  if (st != ARTS_OK && variant < 0) {
    // wide DM spacing: fall back to the variant with the fewest DMs per block
    int best = -1;
    for (int v = 0; v < kNumVariants; ++v) {
      if (p->is16() != (kVariants[v].spd == 2)) continue;
      if (best < 0 || kVariants[v].acc * kVariants[v].waves <
                          kVariants[best].acc * kVariants[best].waves)
        best = v;
    }
    st = best >= 0 ? build_tiling(p, best) : st;
  }
  if (st != ARTS_OK) {
    plan_free(p);
    return st;
  }
  *out = p;
  return ARTS_OK;
}

// Two-step subband plan (Sect. 6b.2 "Dedispersion"; Table "dedispersion setup").  Delays as in
// the oracle's reading: coarse DM = centre of each group of nfine fine trials, subband
// reference = its highest channel, both steps rounded half to even in FP64.
static int plan_create_subband(int32_t nchan, double f_lo, double df, double tsamp,
                               double dm_first, double dm_step, int32_t ndm, int32_t nfine,
                               int32_t nsub, const int32_t* widths, int32_t nwidth,
                               arts_plan_t* out) {
  if (!out) return fail(ARTS_E_INVAL, "out is NULL");
  *out = nullptr;
  if (nchan < 1 || nsub < 1 || nchan % nsub != 0)
    return fail(ARTS_E_INVAL, "nsub must divide nchan");
  const int32_t csub = nchan / nsub;
  if (csub > 257) return fail(ARTS_E_INVAL, "at most 257 channels per subband (16-bit sums)");
  if (nfine != 16 && nfine != 32)
    return fail(ARTS_E_INVAL, "nfine must be 16 or 32 (the DM trials of a step-2 block)");
  if (ndm < 1 || !std::isfinite(dm_first) || !std::isfinite(dm_step) || dm_first < 0 ||
      !(dm_step > 0))
    return fail(ARTS_E_INVAL, "need ndm >= 1, dm_first >= 0 and dm_step > 0 (finite)");
  if (int st = check_widths(nchan, 1, widths, nwidth)) return st;
  const int32_t ncoarse = (ndm + nfine - 1) / nfine;
  std::vector<double> fine(ndm), coarse(ncoarse);
  for (int32_t k = 0; k < ndm; ++k) fine[k] = dm_first + dm_step * k;
  for (int32_t j = 0; j < ncoarse; ++j)
    coarse[j] = dm_first + dm_step * (static_cast<double>(j) * nfine + (nfine - 1) / 2.0);
  arts_plan_s* p = new (std::nothrow) arts_plan_s;
  if (!p) return fail(ARTS_E_NOMEM, "host allocation failed");
  p->nchan = nchan;
  p->ndm = ndm;
  p->nwidth = nwidth;
  p->f_lo = f_lo;
  p->df = df;
  p->tsamp = tsamp;
  p->dms = fine;
  p->widths.assign(widths, widths + nwidth);
  p->nsub = nsub;
  p->nfine = nfine;
  p->ncoarse = ncoarse;
  static const int32_t kOne[1] = {1};
  int st = ARTS_OK;
  p->tie_margin = 1e300;
  // step-1 delays: each subband's channels relative to the subband's own highest channel
  std::vector<int32_t> d1(static_cast<size_t>(ncoarse) * nchan), dsub(static_cast<size_t>(ncoarse) * csub);
  for (int32_t s = 0; s < nsub && st == ARTS_OK; ++s) {
    double margin = 0;
    st = compute_delays(csub, f_lo + static_cast<double>(s) * csub * df, df, tsamp,
                        coarse.data(), ncoarse, 1, dsub.data(), &margin);
    p->tie_margin = std::min(p->tie_margin, margin);
    for (int32_t j = 0; j < ncoarse && st == ARTS_OK; ++j)
      for (int32_t c = 0; c < csub; ++c)
        d1[static_cast<size_t>(j) * nchan + s * csub + c] = dsub[static_cast<size_t>(j) * csub + c];
  }
  // the packed tiling that suits the coarse trial count, else whichever fits the delay spread
  if (st == ARTS_OK) {
    st = plan_create(nchan, f_lo, df, tsamp, coarse.data(), ncoarse, kOne, 1, 1, &p->sb1, false,
                     0, split_variant(ncoarse), d1.data(), csub);
    if (st != ARTS_OK)
      st = plan_create(nchan, f_lo, df, tsamp, coarse.data(), ncoarse, kOne, 1, 1, &p->sb1,
                       false, 0, -1, d1.data(), csub);
  }
  if (st == ARTS_OK) {
    p->max_d1 = p->sb1->max_delay;
    const double top = df > 0 ? csub - 1 : 0;
    // step 2: one block per coarse group (32 trials: 8-wave blocks of 4 per wave at six waves
    // per SIMD; 16: 16-wave blocks of 1 per wave at eight)
    st = plan_create(nsub, f_lo + top * df, csub * df, tsamp, fine.data(), ndm, kOne, 1, 1,
                     &p->sb2, true, 255 * csub, nfine == 32 ? 6 : 36);
  }
  if (st != ARTS_OK) {
    plan_free(p);
    return st;
  }
  p->tie_margin = std::min(p->tie_margin, p->sb2->tie_margin);
  // composite delay of (trial k, channel c): step 1 at k's coarse DM plus step 2 of c's subband
  p->delays.resize(static_cast<size_t>(ndm) * nchan);
  for (int32_t k = 0; k < ndm; ++k)
    for (int32_t c = 0; c < nchan; ++c)
      p->delays[static_cast<size_t>(k) * nchan + c] =
          d1[static_cast<size_t>(k / nfine) * nchan + c] +
          p->sb2->delays[static_cast<size_t>(k) * nsub + c / csub];
  p->max_delay = p->max_d1 + p->sb2->max_delay;
  p->wmax = widths[nwidth - 1];
  p->halo = p->max_delay + p->wmax - 1;
  p->tiling.variant = p->sb1->tiling.variant;
  if ((st = upload_plan(p)) != ARTS_OK) {
    plan_free(p);
    return st;
  }
  *out = p;
  return ARTS_OK;
}

int64_t subband_pitch(const arts_plan_s* p, int64_t nin, int32_t pad) {
  return (nin - p->max_d1 + pad + 3) & ~int64_t(3);
}

// Elements for any front pad 0..3.
int64_t subband_ws_elems(const arts_plan_s* p, int32_t nbeam, int64_t nin) {
  if (p->nsub == 0) return 0;
  return static_cast<int64_t>(nbeam) * p->nsub * p->ncoarse *
         std::max<int64_t>(subband_pitch(p, nin, 3), 0);
}

int prepare_plan(arts_plan_s* p, int32_t nbeam, int64_t nin, int g0, bool plan_ws) {
  if (p->nsub == 0) return ensure_tables(p, g0);
  if (plan_ws) {
    if (int st = ensure_tables(p->sb1, g0)) return st;
    // one-shot rows start at even element offsets of a 256-byte aligned buffer: class 0
    if (int st = ensure_tables(p->sb2, 0)) return st;
  } else {  // streams: step 1 also reads shifted windows, step 2 rows after a pad
    for (int g = 0; g < 4; ++g)
      if (int st = ensure_tables(p->sb1, g)) return st;
    for (int g = 0; g < 2; ++g)
      if (int st = ensure_tables(p->sb2, g)) return st;
    return ARTS_OK;
  }
  const int64_t need = subband_ws_elems(p, nbeam, nin);
  if (need <= p->y_cap) return ARTS_OK;
  if (p->d_y) (void)hipFree(p->d_y);
  p->d_y = nullptr;
  p->y_cap = 0;
  ARTS_HIP(hipMalloc(&p->d_y, need * sizeof(uint16_t)));
  p->y_cap = need;
  return ARTS_OK;
}

static int check_plan(const arts_plan_s* p) {
  if (!p) return fail(ARTS_E_INVAL, "plan is NULL");
  return ARTS_OK;
}

static int64_t nrep_of(const arts_plan_s* p, int64_t L) { return L - p->wmax + 1; }

}  // namespace arts

using namespace arts;

extern "C" {

const char* arts_strerror(int status) {
  switch (status) {
    case ARTS_OK: return "ok";
    case ARTS_E_INVAL: return "invalid argument";
    case ARTS_E_SHAPE: return "input shorter than the plan's halo";
    case ARTS_E_NOMEM: return "out of memory";
    case ARTS_E_DEVICE: return "HIP device error";
    case ARTS_E_CAPACITY: return "candidate buffer too small";
    case ARTS_E_BUDGET: return "request exceeds the HBM budget";
    case ARTS_E_STATE: return "call not valid in the current state";
    default: return "unknown status";
  }
}

const char* arts_last_error(void) { return g_last_error.c_str(); }

const char* arts_version(void) { return "arts-mi355x 0.1 (gfx950)"; }

int arts_delay_table(int32_t nchan, double f_lo_mhz, double df_mhz, double tsamp_s,
                     const double* dm_list, int32_t ndm, int32_t downsample,
                     int32_t* delays_out, double* tie_margin_out) {
  if (!delays_out) return fail(ARTS_E_INVAL, "delays_out is NULL");
  return compute_delays(nchan, f_lo_mhz, df_mhz, tsamp_s, dm_list, ndm, downsample, delays_out,
                        tie_margin_out);
}

int arts_plan_create(int32_t nchan, double f_lo_mhz, double df_mhz, double tsamp_s,
                     const double* dm_list, int32_t ndm, const int32_t* widths, int32_t nwidth,
                     arts_plan_t* out) {
  return plan_create(nchan, f_lo_mhz, df_mhz, tsamp_s, dm_list, ndm, widths, nwidth, 1, out);
}

int arts_plan_create_ds(int32_t nchan, double f_lo_mhz, double df_mhz, double tsamp_s,
                        const double* dm_list, int32_t ndm, const int32_t* widths,
                        int32_t nwidth, int32_t downsample, arts_plan_t* out) {
  return plan_create(nchan, f_lo_mhz, df_mhz, tsamp_s, dm_list, ndm, widths, nwidth,
                     downsample, out);
}

int arts_plan_create_subband(int32_t nchan, double f_lo_mhz, double df_mhz, double tsamp_s,
                             double dm_first, double dm_step, int32_t ndm, int32_t nfine,
                             int32_t nsub, const int32_t* widths, int32_t nwidth,
                             arts_plan_t* out) {
  return plan_create_subband(nchan, f_lo_mhz, df_mhz, tsamp_s, dm_first, dm_step, ndm, nfine,
                             nsub, widths, nwidth, out);
}

int arts_plan_subband_info(arts_plan_t p, int32_t* nsub, int32_t* nfine, int32_t* ncoarse,
                           int32_t* max_delay1, int32_t* max_delay2) {
  if (int st = check_plan(p)) return st;
  if (nsub) *nsub = p->nsub;
  if (nfine) *nfine = p->nfine;
  if (ncoarse) *ncoarse = p->ncoarse;
  if (max_delay1) *max_delay1 = p->max_d1;
  if (max_delay2) *max_delay2 = p->nsub ? p->sb2->max_delay : 0;
  return ARTS_OK;
}

void arts_plan_destroy(arts_plan_t plan) { plan_free(plan); }

int arts_plan_info(arts_plan_t p, int32_t* nchan, int32_t* ndm, int32_t* nwidth,
                   int32_t* downsample, int32_t* max_delay, int32_t* halo) {
  if (int st = check_plan(p)) return st;
  if (nchan) *nchan = p->nchan;
  if (ndm) *ndm = p->ndm;
  if (nwidth) *nwidth = p->nwidth;
  if (downsample) *downsample = p->ds;
  if (max_delay) *max_delay = p->max_delay;
  if (halo) *halo = p->halo;
  return ARTS_OK;
}

int arts_plan_delays(arts_plan_t p, int32_t* host_out) {
  if (int st = check_plan(p)) return st;
  if (!host_out) return fail(ARTS_E_INVAL, "host_out is NULL");
  std::memcpy(host_out, p->delays.data(), p->delays.size() * sizeof(int32_t));
  return ARTS_OK;
}

int arts_plan_set_tiling_shape(arts_plan_t p, int32_t variant, int32_t buffers,
                               int32_t channels) {
  if (int st = check_plan(p)) return st;
  if (buffers != 1 && buffers != 2) return fail(ARTS_E_INVAL, "buffers must be 1 or 2");
  if (channels < 0 || channels > 255) return fail(ARTS_E_INVAL, "channels must be 0..255");
  arts_plan_s* q = p->nsub > 0 ? p->sb1 : p;  // subband plans: the first step's tiles
  if (p->tiling.variant == variant && q->tile_nbuf == buffers && q->tile_cc == channels)
    return ARTS_OK;
  const int32_t nb0 = q->tile_nbuf, cc0 = q->tile_cc;
  q->tile_nbuf = buffers;
  q->tile_cc = channels;
  const int st = build_tiling(p, variant);
  if (st != ARTS_OK) {  // the plan keeps its tiling
    q->tile_nbuf = nb0;
    q->tile_cc = cc0;
  }
  return st;
}

int arts_plan_get_tiling_shape(arts_plan_t p, int32_t* variant, int32_t* buffers,
                               int32_t* channels) {
  if (int st = check_plan(p)) return st;
  const arts_plan_s* q = p->nsub > 0 ? p->sb1 : p;
  if (variant) *variant = p->tiling.variant;
  if (buffers) *buffers = q->tiling.nbuf;
  if (channels) *channels = q->tiling.cc;
  return ARTS_OK;
}

int arts_plan_set_tiling(arts_plan_t p, int32_t variant) {
  return arts_plan_set_tiling_shape(p, variant, kDefaultBuffers, 0);
}

int arts_plan_get_tiling(arts_plan_t p, int32_t* variant) {
  if (int st = check_plan(p)) return st;
  if (variant) *variant = p->tiling.variant;
  return ARTS_OK;
}

int arts_plan_set_cluster(arts_plan_t p, int32_t enable) {
  if (int st = check_plan(p)) return st;
  if (enable != 0 && enable != 1) return fail(ARTS_E_INVAL, "enable must be 0 or 1");
  if (p->cluster != (enable != 0)) ++p->generation;
  p->cluster = enable != 0;
  return ARTS_OK;
}

int arts_plan_get_cluster(arts_plan_t p, int32_t* enable) {
  if (int st = check_plan(p)) return st;
  if (enable) *enable = p->cluster ? 1 : 0;
  return ARTS_OK;
}

int arts_plan_set_integration(arts_plan_t p, int32_t mode) {
  if (int st = check_plan(p)) return st;
  if (mode != 0 && mode != 1) return fail(ARTS_E_INVAL, "mode must be 0 or 1");
  if (p->integration != mode) ++p->generation;
  p->integration = mode;
  return ARTS_OK;
}

int arts_plan_get_integration(arts_plan_t p, int32_t* mode) {
  if (int st = check_plan(p)) return st;
  if (mode) *mode = p->integration;
  return ARTS_OK;
}

int arts_sb_table_beam_model(int32_t nsb, int32_t ntab, int32_t nchan, double f_lo_mhz,
                             double df_mhz, double f_max_mhz, double alpha, double b_max_m,
                             double b_cq_m, int32_t quarter, uint8_t* table_out,
                             double* margin_out) {
  if (!table_out) return fail(ARTS_E_INVAL, "table_out is NULL");
  if (nsb < 1 || nchan < 1 || ntab < 2 || ntab > 256 || ntab % 2 != 0)
    return fail(ARTS_E_INVAL, "nsb, nchan >= 1 and an even ntab in [2, 256] required");
  if (!(f_max_mhz > 0) || !(alpha > 0) || !(b_max_m > 0) || !(b_cq_m > 0) ||
      !std::isfinite(f_lo_mhz) || !std::isfinite(df_mhz) || df_mhz == 0 ||
      (quarter != 0 && quarter != 1))
    return fail(ARTS_E_INVAL, "bad beam-model arguments");
  constexpr int kSwitches = 64;  // neighbours followed down in frequency
  const int32_t half = ntab / 2;
  const double a = alpha * b_cq_m;
  double margin = std::numeric_limits<double>::infinity();
  for (int32_t row = 0; row < nsb; ++row) {
    const int32_t n_sb = row - (nsb - 1) / 2;
    int32_t n_tab = ((n_sb % ntab) + ntab) % ntab;  // index at f_max in [-N/2, N/2 - 1]
    if (n_tab > half - 1) n_tab -= ntab;
    const int32_t n_gr = (n_sb - n_tab) / ntab;       // exact: n_sb = n_gr N + n_tab
    const int32_t sg = (n_sb > 0) - (n_sb < 0);
    uint8_t* out = table_out + static_cast<int64_t>(row) * nchan;
    if (sg == 0) {
      std::memset(out, half, nchan);
      continue;
    }
    // f_k: frequency where grating n_gr of TAB n_tab - k sg points where the SB does
    const double den = n_gr * b_max_m + n_tab * a;
    double fk[kSwitches + 1], fsw[kSwitches];
    for (int k = 0; k <= kSwitches; ++k)
      fk[k] = f_max_mhz * (n_gr * b_max_m + (n_tab - k * sg) * a) / den;
    const double b = quarter ? (n_sb % 2 == 0 ? 0.25 : 0.75) : 0.5;
    for (int k = 1; k <= kSwitches; ++k) fsw[k - 1] = (1 - b) * fk[k - 1] + b * fk[k];
    for (int32_t c = 0; c < nchan; ++c) {
      const double f = f_lo_mhz + c * df_mhz;
      if (!(f > 0)) return fail(ARTS_E_INVAL, "channel %d has frequency %g MHz", c, f);
      int k = 0;
      while (k < kSwitches && f < fsw[k]) ++k;
      if (k < kSwitches) margin = std::min(margin, std::fabs(f - fsw[k]));
      if (k > 0) margin = std::min(margin, std::fabs(f - fsw[k - 1]));
      const int32_t j = n_tab - k * sg;
      out[c] = static_cast<uint8_t>((((j + half) % ntab) + ntab) % ntab);
    }
  }
  if (margin_out) *margin_out = margin;
  return ARTS_OK;
}

int arts_rfi_clean(uint8_t* data, int32_t nrow, int32_t nchan, int64_t nsamp, int64_t pitch,
                   float k_time, int32_t niter_time, float k_freq, int32_t niter_freq,
                   void* stream) {
  if (!data) return fail(ARTS_E_INVAL, "data is NULL");
  if (nrow < 1 || nchan < 1 || nsamp < 1 || pitch < nsamp)
    return fail(ARTS_E_INVAL, "nrow, nchan, nsamp >= 1 and pitch >= nsamp required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  const int64_t bytes = rfi_ws_bytes(nrow, nchan, nsamp);
  if (hipMalloc(&ws, bytes) != hipSuccess)
    return fail(ARTS_E_NOMEM, "RFI workspace of %lld bytes", (long long)bytes);
  struct Free {
    void* p;
    ~Free() { (void)hipFree(p); }
  } guard{ws};
  if (int st = launch_rfi(data, nrow, nchan, nsamp, pitch, k_time, niter_time, k_freq,
                          niter_freq, ws, s))
    return st;
  ARTS_HIP(hipStreamSynchronize(s));
  return ARTS_OK;
}

int arts_cluster_offline(const arts_candidate* cand, int64_t n, int64_t t_window,
                         const double* dm_edges, int32_t nedge, float min_snr,
                         arts_candidate* host_out, int64_t capacity, int64_t* count,
                         void* stream) {
  if (!count || n < 0 || (n > 0 && !cand) || capacity < 0 || (capacity > 0 && !host_out))
    return fail(ARTS_E_INVAL, "bad pointer or size");
  if (n >= INT_MAX) return fail(ARTS_E_INVAL, "at most 2^31 - 1 candidates");
  if (t_window < 1) return fail(ARTS_E_INVAL, "t_window must be >= 1");
  if (!dm_edges || nedge < 1 || nedge >= (1 << 20))
    return fail(ARTS_E_INVAL, "1 <= nedge < 2^20 DM window edges required");
  for (int32_t i = 0; i < nedge; ++i)
    if (!std::isfinite(dm_edges[i]) || (i > 0 && !(dm_edges[i] > dm_edges[i - 1])))
      return fail(ARTS_E_INVAL, "DM window edges must be finite and strictly increasing");
  if (std::isnan(min_snr)) return fail(ARTS_E_INVAL, "min_snr is NaN");
  *count = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  const int64_t bytes = offline_ws_bytes(n, nedge);
  if (hipMalloc(&ws, bytes) != hipSuccess)
    return fail(ARTS_E_NOMEM, "offline clustering workspace of %lld bytes", (long long)bytes);
  struct Free {
    void* p;
    ~Free() { (void)hipFree(p); }
  } guard{ws};
  ARTS_HIP(hipMemcpyAsync(offline_edges(ws, n), dm_edges, sizeof(double) * nedge,
                          hipMemcpyHostToDevice, s));
  arts_candidate* d_out = nullptr;
  unsigned long long* d_count = nullptr;
  int* d_bad = nullptr;
  if (int st = launch_cluster_offline(cand, n, t_window, offline_edges(ws, n), nedge, min_snr, ws,
                                      &d_out, &d_count, &d_bad, s))
    return st;
  unsigned long long nk = 0;
  int bad = 0;
  ARTS_HIP(hipMemcpyAsync(&nk, d_count, sizeof nk, hipMemcpyDeviceToHost, s));
  ARTS_HIP(hipMemcpyAsync(&bad, d_bad, sizeof bad, hipMemcpyDeviceToHost, s));
  ARTS_HIP(hipStreamSynchronize(s));
  if (bad)
    return fail(ARTS_E_INVAL, "a candidate has width < 1, downsample outside [1, 2^20), a NaN "
                              "S/N or DM, or a native start beyond +-2^42 samples");
  *count = static_cast<int64_t>(nk);
  if (*count > capacity)
    return fail(ARTS_E_CAPACITY, "%llu kept candidates, capacity %lld", nk, (long long)capacity);
  if (nk == 0) return ARTS_OK;
  ARTS_HIP(hipMemcpyAsync(host_out, d_out, nk * sizeof(arts_candidate), hipMemcpyDeviceToHost,
                          s));
  ARTS_HIP(hipStreamSynchronize(s));
  std::sort(host_out, host_out + nk, [](const arts_candidate& a, const arts_candidate& b) {
    const int64_t ta = a.sample * a.downsample, tb = b.sample * b.downsample;
    if (ta != tb) return ta < tb;
    if (a.dm != b.dm) return a.dm < b.dm;
    if (a.beam != b.beam) return a.beam < b.beam;
    return a.width < b.width;
  });
  return ARTS_OK;
}

int arts_plan_cluster(arts_plan_t p, arts_candidate* cand, int64_t n, int32_t nbeam,
                      int32_t beam_offset, int64_t* count, void* stream) {
  if (int st = check_plan(p)) return st;
  if (!count || n < 0 || (n > 0 && !cand) || nbeam < 1)
    return fail(ARTS_E_INVAL, "bad pointer or size");
  *count = 0;
  if (n == 0) return ARTS_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t rows = static_cast<int64_t>(nbeam) * p->ndm;
  if (int st = ensure_cand(p, 0)) return st;
  if (int st = ensure_cluster_ws(p->cl, n, rows)) return st;
  unsigned long long n0 = static_cast<unsigned long long>(n), n1 = 0;
  ARTS_HIP(hipMemcpyAsync(p->d_count, &n0, sizeof n0, hipMemcpyHostToDevice, s));
  if (int st = launch_cluster(p->cl, cand, p->d_count, n, false, nbeam, p->ndm, beam_offset, s))
    return st;
  ARTS_HIP(hipMemcpyAsync(&n1, p->d_count, sizeof n1, hipMemcpyDeviceToHost, s));
  int skipped = 0, bad = 0;
  if (int st = read_cluster_status(p->cl, &skipped, &bad, s)) return st;  // synchronises
  if (bad)
    return fail(ARTS_E_INVAL, "a candidate lies outside the plan's beams or DM trials, has "
                              "width < 1 or a NaN S/N");
  if (skipped) return fail(ARTS_E_DEVICE, "internal: clustering skipped");
  *count = static_cast<int64_t>(n1);
  return ARTS_OK;
}

int32_t arts_tiling_count(void) { return kNumVariants; }

int arts_tiling_occupancy(int32_t variant, int32_t* per_job, int32_t* persistent) {
  if (variant < 0 || variant >= kNumVariants || !per_job || !persistent)
    return fail(ARTS_E_INVAL, "bad variant or NULL output");
  const bool group = is_group(kVariants[variant].pack);
  *per_job = variant_occupancy(variant, group ? kOccSplit : kOccPlain);
  *persistent = variant_occupancy(variant, kOccBatch);
  if (*per_job < 1 || (!group && *persistent < 1))
    return fail(ARTS_E_DEVICE, "occupancy query failed for variant %d", variant);
  return ARTS_OK;
}

int arts_tiling_describe(int32_t variant, char* buf, int32_t len) {
  if (variant < 0 || variant >= kNumVariants || !buf || len < 1)
    return fail(ARTS_E_INVAL, "bad variant or buffer");
  const TileVariant& v = kVariants[variant];
  snprintf(buf, len, "J=%d ACC=%d WAVES=%d SPD=%d%s", v.j, v.acc, v.waves, v.spd,
           v.pack == 11  ? " framed runs group sums"
           : v.pack == 10 ? " pairs framed"
           : v.pack == 9 ? " framed runs shared"
           : v.pack == 7 ? " framed runs"
           : v.pack == 5 ? " pairs"
           : v.pack == 4 ? " group sums"
           : v.pack == 3 ? " packed held"
           : v.pack == 2 ? " framed"
           : v.pack      ? " packed"
                         : "");
  return ARTS_OK;
}

int arts_sb_synthesize(const uint8_t* tab, int32_t ntab, const uint8_t* sb_table, int32_t nsb,
                       int32_t nchan, int64_t nsamp, uint8_t* sb_out, void* stream) {
  if (!tab || !sb_table || !sb_out) return fail(ARTS_E_INVAL, "NULL pointer");
  if (ntab < 1 || ntab > 256 || nsb < 1 || nchan < 1 || nsamp < 1)
    return fail(ARTS_E_INVAL, "sizes out of range (ntab 1..256, nsb, nchan, nsamp >= 1)");
  return launch_sb_gather(tab, ntab, sb_table, nsb, nchan, nsamp, sb_out,
                          static_cast<hipStream_t>(stream));
}

int arts_dedisperse(arts_plan_t p, const uint8_t* in, int32_t nbeam, int64_t nin, int32_t* out,
                    void* stream) {
  TraceRange range("arts_dedisperse");
  if (int st = check_plan(p)) return st;
  if (!in || !out || nbeam < 1) return fail(ARTS_E_INVAL, "NULL pointer or nbeam < 1");
  const int64_t L = nin / p->ds - p->max_delay;
  if (nin < 1 || L < 1)
    return fail(ARTS_E_SHAPE, "nin = %lld gives no output sample (max delay %d, D %d)",
                (long long)nin, p->max_delay, p->ds);
  DedispJob job;
  job.in = in;
  job.in_bytes = static_cast<int64_t>(nbeam) * p->nchan * nin;
  job.nin = nin;
  job.pitch = nin;
  job.nsrc = nbeam;
  job.nbeam = nbeam;
  job.out = out;
  job.nout = L;
  return run_dedisperse(p, job, static_cast<hipStream_t>(stream));
}

int arts_dedisperse_sb(arts_plan_t p, const uint8_t* tab, int32_t ntab, const uint8_t* sb_table,
                       int32_t nsb, int64_t nin, int32_t* out, void* stream) {
  if (int st = check_plan(p)) return st;
  if (!tab || !sb_table || !out) return fail(ARTS_E_INVAL, "NULL pointer");
  if (ntab < 1 || ntab > 256 || nsb < 1) return fail(ARTS_E_INVAL, "ntab 1..256, nsb >= 1");
  const int64_t L = nin / p->ds - p->max_delay;
  if (nin < 1 || L < 1)
    return fail(ARTS_E_SHAPE, "nin = %lld gives no output sample", (long long)nin);
  DedispJob job;
  job.in = tab;
  job.in_bytes = static_cast<int64_t>(ntab) * p->nchan * nin;
  job.nin = nin;
  job.pitch = nin;
  job.nsrc = ntab;
  job.sb_table = sb_table;
  job.nbeam = nsb;
  job.out = out;
  job.nout = L;
  return run_dedisperse(p, job, static_cast<hipStream_t>(stream));
}

int arts_boxcar_snr(arts_plan_t p, const int32_t* series, int32_t nbeam, int64_t L,
                    double* stats, int32_t* sums, float* snr, void* stream) {
  if (int st = check_plan(p)) return st;
  if (!series || nbeam < 1) return fail(ARTS_E_INVAL, "NULL series or nbeam < 1");
  const int64_t nrep = nrep_of(p, L);
  if (nrep < 1) return fail(ARTS_E_SHAPE, "L = %lld shorter than wmax", (long long)L);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t rows = static_cast<int64_t>(nbeam) * p->ndm;
  if (int st = ensure_stats(p, rows)) return st;
  if (int st = launch_row_stats(series, L, nrep, rows, p->d_s1, p->d_musig, s)) return st;
  if (stats)
    ARTS_HIP(hipMemcpyAsync(stats, p->d_musig, rows * 2 * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
  if (sums || snr)
    return launch_boxcar_snr(p, series, nbeam, L, nrep, p->d_s1, p->d_musig, sums, snr, s);
  return ARTS_OK;
}

int arts_candidates(arts_plan_t p, const int32_t* series, int32_t nbeam, int64_t L,
                    float threshold, int64_t t_offset, int32_t beam_offset,
                    arts_candidate* host_out, int64_t capacity, int64_t* count, void* stream) {
  TraceRange range("arts_candidates");
  if (int st = check_plan(p)) return st;
  if (!series || nbeam < 1 || !count || capacity < 0 || (capacity > 0 && !host_out))
    return fail(ARTS_E_INVAL, "bad pointer or size");
  if (!std::isfinite(threshold)) return fail(ARTS_E_INVAL, "threshold must be finite");
  const int64_t nrep = nrep_of(p, L);
  if (nrep < 1) return fail(ARTS_E_SHAPE, "L = %lld shorter than wmax", (long long)L);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t rows = static_cast<int64_t>(nbeam) * p->ndm;
  if (int st = ensure_stats(p, rows)) return st;
  if (int st = ensure_cand(p, capacity)) return st;
  if (int st = launch_zero_u64(p->d_count, 1, s)) return st;
  if (p->cluster)
    if (int st = ensure_cluster_ws(p->cl, std::max<int64_t>(capacity, 1), rows)) return st;
  if (int st = ensure_flags(p, rows)) return st;
  if (int st = launch_candidates(p, series, nbeam, L, nrep, threshold, t_offset, beam_offset,
                                 p->d_s1, p->d_musig, p->d_cand, p->d_count, capacity, s, 0,
                                 p->d_flags))
    return st;
  if (p->cluster)
    if (int st = launch_cluster(p->cl, p->d_cand, p->d_count, capacity, false, nbeam, p->ndm,
                                beam_offset, s))
      return st;
  unsigned long long n = 0;
  ARTS_HIP(hipMemcpyAsync(&n, p->d_count, sizeof n, hipMemcpyDeviceToHost, s));
  ARTS_HIP(hipStreamSynchronize(s));
  *count = static_cast<int64_t>(n);
  if (static_cast<int64_t>(n) > capacity)
    return fail(ARTS_E_CAPACITY, "%llu candidates, capacity %lld", n, (long long)capacity);
  if (n == 0) return ARTS_OK;
  ARTS_HIP(hipMemcpyAsync(host_out, p->d_cand, n * sizeof(arts_candidate),
                          hipMemcpyDeviceToHost, s));
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

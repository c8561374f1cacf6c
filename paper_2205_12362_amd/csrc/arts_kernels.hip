// Device code of libarts for gfx950 (CDNA4): dedispersion, row statistics, boxcar / S/N /
// candidate extraction and synthesized-beam gather.  All arithmetic on data is integer and
// exact; FP64 is used only for the per-series mean / sigma and thresholds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "arts_internal.h"

namespace arts {

// ------------------------------------------------------------------ tiling variants ----
// id, spd, j, acc, waves, pack.  j is odd so the lane stride of j dwords hits distinct LDS
// banks; pack: 0 plain, 1 packed 16-bit partial sums, 2 framed, 3 packed halves held across
// chunks, 4 group sums (split plans), 5 DM pairs read as one window (16-bit samples), 7 framed
// runs (raw-dword frames per sub-dword class, added into the totals at the end of each run),
// 9 framed runs whose lanes read J dwords per channel and take the sums of their last dword
// from the next lane (a tile then covers 64 T - 4 outputs), 10 DM pairs summed in raw frames
// per sample parity (16-bit samples), aligned once per chunk, 11 framed runs (last word shared)
// added into packed group sums at the end of each run (split plans).
#define ARTS_TILINGS(X)                                                                    \
  X(0, 4, 5, 4, 8, 0)   /* 32 DMs x 1280 samples per block, 80 accumulators per lane */    \
  X(1, 4, 7, 3, 8, 0)   /* 24 DMs x 1792 */                                                \
  X(2, 4, 5, 4, 16, 0)  /* 64 DMs x 1280, one block per CU */                              \
  X(3, 4, 3, 6, 8, 0)   /* 48 DMs x 768 */                                                 \
  X(4, 4, 5, 2, 4, 0)   /*  8 DMs x 1280, small problems */                                \
  X(5, 4, 7, 4, 8, 0)   /* 32 DMs x 1792, 112 accumulators */                              \
  X(6, 2, 5, 4, 8, 0)   /* downsampled: 32 DMs x 640 */                                    \
  X(7, 2, 9, 2, 8, 0)   /* downsampled: 16 DMs x 1152 */                                   \
  X(8, 2, 7, 3, 8, 0)   /* downsampled: 24 DMs x 896 */                                    \
  X(9, 4, 5, 4, 8, 1)   /* as 0, packed */                                                 \
  X(10, 4, 5, 3, 8, 1)  /* 24 DMs x 1280, packed */                                        \
  X(11, 4, 3, 6, 8, 1)  /* as 3, packed */                                                 \
  X(12, 4, 5, 4, 16, 1) /* as 2, packed */                                                 \
  X(13, 2, 5, 4, 8, 1)  /* as 6, packed */                                                 \
  X(14, 2, 9, 2, 8, 1)  /* as 7, packed */                                                 \
  X(15, 2, 7, 3, 8, 1)  /* as 8, packed */                                                 \
  X(16, 2, 5, 6, 8, 1)  /* downsampled, packed: 48 DMs x 640 */                            \
  X(17, 4, 5, 2, 4, 1)  /* as 4, packed */                                                 \
  X(18, 4, 5, 1, 8, 2)  /* framed:  8 DMs x 1280 */                                        \
  X(19, 4, 5, 1, 16, 2) /* framed: 16 DMs x 1280, one block per CU */                      \
  X(20, 4, 3, 2, 8, 2)  /* framed: 16 DMs x 768 */                                         \
  X(21, 4, 7, 1, 8, 2)  /* framed:  8 DMs x 1792 */                                        \
  X(22, 4, 5, 2, 8, 3)  /* 16 DMs x 1280, packed halves held across chunks */              \
  X(23, 4, 5, 4, 8, 4)  /* 32 DMs x 1280, group sums in packed halves (split plans) */     \
  X(24, 2, 5, 4, 8, 5)  /* downsampled, DM pairs: 32 DMs x 640 */                          \
  X(25, 2, 7, 2, 8, 5)  /* downsampled, DM pairs: 16 DMs x 896 */                          \
  X(26, 2, 9, 2, 8, 5)  /* downsampled, DM pairs: 16 DMs x 1152 */                         \
  X(27, 4, 5, 4, 8, 7)  /* framed runs: 32 DMs x 1280 */                                   \
  X(28, 4, 5, 4, 8, 9)  /* framed runs, last word shared: 32 DMs x 1276 */                 \
  X(29, 4, 5, 3, 8, 9)  /* framed runs, last word shared: 24 DMs x 1276 */ \
  X(30, 2, 5, 4, 8, 10) /* downsampled, DM pairs in raw frames: 32 DMs x 640 */            \
  X(31, 4, 5, 4, 8, 11) /* 32 DMs x 1276, framed runs into group sums (split plans) */     \
  X(32, 4, 5, 2, 12, 9) /* framed runs, last word shared, 12-wave blocks, six waves per SIMD:
                           24 DMs x 1276 */ \
  X(33, 2, 5, 2, 12, 10) /* DM pairs in raw frames, 12-wave blocks, six waves per SIMD */ \
  X(34, 2, 5, 2, 16, 10) /* DM pairs in raw frames, 16-wave blocks, eight waves per SIMD:
                            32 DMs x 640 */ \
  X(35, 4, 5, 2, 16, 11) /* as 31 in 16-wave blocks, eight waves per SIMD (split plans) */ \
  X(36, 2, 5, 1, 16, 0) /* 16-bit, 16-wave blocks, eight waves per SIMD: 16 DMs x 640 */

const TileVariant kVariants[] = {
#define ARTS_X(id, spd, j, acc, waves, pack) {spd, j, acc, waves, pack},
    ARTS_TILINGS(ARTS_X)
#undef ARTS_X
};
// the ids of the table are its indices
constexpr int kTilingIds[] = {
#define ARTS_X(id, spd, j, acc, waves, pack) id,
    ARTS_TILINGS(ARTS_X)
#undef ARTS_X
};
constexpr bool tiling_ids_ok() {
  for (int i = 0; i < static_cast<int>(sizeof(kTilingIds) / sizeof(int)); ++i)
    if (kTilingIds[i] != i) return false;
  return true;
}
static_assert(tiling_ids_ok(), "tiling ids must run 0, 1, 2, ...");
const int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Byte samples: the packed tiling with 32 DMs per block (9) unless 24 per block (10) leaves
// fewer idle DM slots in the last block; a slot of 10 costs about 2% more than one of 9.
int packed_variant(int64_t ndm) {
  const int64_t s24 = (ndm + 23) / 24 * 24, s32 = (ndm + 31) / 32 * 32;
  return s24 * 102 < s32 * 100 ? 10 : 9;
}

// The first step of subband plans: framed runs into group sums (32 DMs per 16-wave block at
// eight waves per SIMD, 35; on the ALERT plans 7-9% faster than the 8-wave blocks of 31) when
// the coarse trials fill its blocks, else the held packed halves (16 per block), else as
// above.  Plan creation falls back to the default if the choice does not fit (for instance
// groups of more than 257 channels).
int split_variant(int64_t ncoarse) {
  if (ncoarse % 32 == 0) return 35;
  return ncoarse % 16 == 0 ? 22 : packed_variant(ncoarse);
}

// Byte samples, plain plans: framed runs with a shared last word in 12-wave blocks of 24 DMs
// (32: six waves per SIMD) unless 32 DMs per block (28: four waves per SIMD) leave enough fewer
// idle DM slots; a slot of 28 costs about 7% more than one of 32 (serving plan: 68.8 ms for
// 2048 slots against 63.9 ms for 2064).
int runs_variant(int64_t ndm) {
  const int64_t s24 = (ndm + 23) / 24 * 24, s32 = (ndm + 31) / 32 * 32;
  return s24 * 100 <= s32 * 107 ? 32 : 28;
}

// Downsampled samples: DM pairs in raw frames in 16-wave blocks at eight waves per SIMD (34);
// on the serving plan 13.4 ms per plan call, against 14.7 ms in 12-wave blocks at six (33)
// and 15.0 ms in 8-wave blocks at four (30).
int default_variant(int downsample, int64_t ndm) {
  if (downsample > 1) return 34;
  return ndm <= 64 ? 17 : runs_variant(ndm);
}

// The tiling to try when the default does not fit a plan (DM-pair tilings need neighbouring
// trials at most kPairMaxDelta samples apart in every channel), or -1.
int fallback_variant(int variant) { return is_pairs(kVariants[variant].pack) ? 6 : -1; }

// ------------------------------------------------------------------ dedispersion ----
//
// One workgroup computes out[b][d][t] for a block of m_blk consecutive DM trials and one time
// tile [t0, t0 + 64*T).  Channels are processed in chunks of `cc`: for each channel of the
// chunk the window of input samples that every DM of the block needs,
//     [t0 + base_c, t0 + base_c + 64*T + spread_c),  base_c = min_d delay[d][c],
// is staged once into LDS and then read by every DM trial of the block (the data reuse across
// neighbouring DMs the paper's kernel is tuned for, Sect. 6b.2 "Dedispersion").
//
// Staging is asynchronous and double-buffered: while the waves sum chunk k out of one LDS
// buffer, direct global->LDS loads (global_load_lds_dwordx4: 16 bytes per lane, no registers)
// fill the other buffer with chunk k + 1.  A window is loaded from the dword-aligned address at
// or below its first sample, so channel c's window starts g_c = (row address + base_c) mod 4
// samples early; the plan folds g_c into its per-channel offsets (one table set per alignment
// class of the input pointer; rows must be dword-aligned, which the host arranges).
//
// Lane l of a wave owns T = spd*j consecutive output samples t0 + l*T + i of `acc` DM trials
// and keeps their sums in int32 registers.  For channel c and trial d it reads the j+1 LDS
// dwords holding samples t0 + l*T + r .. + T - 1, r = delay[d][c] - base_c + g_c.  r is the
// same for every lane, and so is its sub-dword offset m = r mod spd.  The plan sorts each DM's
// channels (within a chunk) by m, so the kernel runs spd straight-line loops, one per m, in
// which every sample is added with one v_add_u32 whose source operand is a byte (spd = 4) or a
// 16-bit half (spd = 2) of an LDS dword (SDWA operand select) and the accumulators stay in
// place.  With j odd, lanes read dwords j apart, which spreads a wave's reads over all banks.

struct DedispArgs {
  const uint8_t* in;
  const uint8_t* in_end;
  int64_t nin;        // native samples per input row
  int64_t pitch;      // bytes between input rows
  int64_t nsamp_d;    // nin / D
  const uint16_t* in16;     // downsampled 16-bit rows (spd = 2 kernels)
  const uint16_t* in16_end;
  int64_t pitch16;          // elements between downsampled rows
  const uint8_t* sb_table;  // nullable: row (b, c) reads source beam sb_table[b*tbl_stride + c]
  const int32_t* base;      // [nblk][nchan]
  const int32_t* list;      // [nblk][m_blk][nchan] LDS byte offsets, by chunk then m
                            // (DM-pair tilings: [nblk][m_blk / 2][nchan], by chunk then class)
  const uint32_t* cnt;      // [nblk][nchunk][m_blk] packed per-m channel counts
                            // (DM-pair tilings: [nblk][nchunk][m_blk / 2][4], per class)
  int32_t* out;             // out[b*out_bstride + d*out_pitch + t], int32 (or uint16: out16)
  int64_t nout;
  int64_t out_pitch, out_bstride;
  int64_t in16_blk;         // in16 elements added per DM block
  int64_t nwg;
  int32_t nchan, ndm, nsrc, ds, nbeam;
  int32_t m_blk, nblk, win, cc, nchunk, ntt;
  int32_t nlist;            // offset lists per block: m_blk, or m_blk / 2 for DM pairs
  int32_t nbuf;             // LDS chunk buffers: 2 (fetch overlaps the sums) or 1
  int32_t src_stride;       // rows between source beams (nchan unless the job says otherwise)
  int32_t tbl_stride;       // SB table entries between beams
  int32_t out16;
  int32_t split;            // channels per output group (0: one group); a multiple of cc
  int64_t out_sstride;      // out elements between channel groups
};

// Source beam of channel c of beam b: b itself, or the SB table entry (read from the LDS copy
// of the beam's table row, so that staging issues no vector-memory load that would have to be
// waited for behind the asynchronous window loads).
__device__ __forceinline__ int src_beam(const DedispArgs& a, const uint8_t* sbrow, int b, int c) {
  return a.sb_table ? __builtin_amdgcn_readfirstlane(sbrow[c]) : b;
}

__device__ __forceinline__ const uint8_t* row_ptr(const DedispArgs& a, int src, int c) {
  if (src >= a.nsrc) return nullptr;
  return a.in + (static_cast<int64_t>(src) * a.src_stride + c) * a.pitch;
}

// acc += one byte / 16-bit half of w, as a single SDWA add.  Written as (ALU-only) inline asm
// because the compiler otherwise fuses pairs of such adds into byte extracts + v_add3_u32,
// which costs 1.5 instructions per sample instead of 1.
template <int SEL>
__device__ __forceinline__ void add_byte(uint32_t& acc, uint32_t w) {
  if constexpr (SEL == 0)
    asm("v_add_u32_sdwa %0, %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
        : "+v"(acc) : "v"(w));
  else if constexpr (SEL == 1)
    asm("v_add_u32_sdwa %0, %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
        : "+v"(acc) : "v"(w));
  else if constexpr (SEL == 2)
    asm("v_add_u32_sdwa %0, %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
        : "+v"(acc) : "v"(w));
  else
    asm("v_add_u32_sdwa %0, %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
        : "+v"(acc) : "v"(w));
}

template <int SEL>
__device__ __forceinline__ void add_half(uint32_t& acc, uint32_t w) {
  if constexpr (SEL == 0)
    asm("v_add_u32_sdwa %0, %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_0"
        : "+v"(acc) : "v"(w));
  else
    asm("v_add_u32_sdwa %0, %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:WORD_1"
        : "+v"(acc) : "v"(w));
}

__device__ __forceinline__ const uint16_t* row_ptr16(const DedispArgs& a, int src, int c,
                                                     int blk) {
  if (src >= a.nsrc) return nullptr;
  return a.in16 + (static_cast<int64_t>(src) * a.src_stride + c) * a.pitch16 + blk * a.in16_blk;
}

template <int SPD, int J, int MS>
__device__ __forceinline__ void accum(uint32_t* acc, const uint32_t* w) {
#pragma unroll
  for (int i = 0; i < SPD * J; ++i) {
    const int q = i + MS;
    if constexpr (SPD == 4) {
      switch (q % 4) {
        case 0: add_byte<0>(acc[i], w[q / 4]); break;
        case 1: add_byte<1>(acc[i], w[q / 4]); break;
        case 2: add_byte<2>(acc[i], w[q / 4]); break;
        default: add_byte<3>(acc[i], w[q / 4]); break;
      }
    } else {
      if (q % 2 == 0)
        add_half<0>(acc[i], w[q / 2]);
      else
        add_half<1>(acc[i], w[q / 2]);
    }
  }
}

// Accumulate n channels whose sub-dword offset is MS.  ent (LDS) holds their byte offsets into
// the staged windows and is padded so that reading past a run stays in bounds.  Channels are
// taken four at a time: the four offsets, then the four channels' words are read before any of
// their samples is added, so one LDS round trip is paid per four channels.
template <int SPD, int J, int MS>
__device__ __forceinline__ void accum_run(uint32_t* acc, const int32_t* ent, int n,
                                          const uint8_t* lane_base) {
  constexpr int NW = (MS == 0) ? J : J + 1;
  int i = 0;
  for (; i + 4 <= n; i += 4) {
    uint32_t w[4][J + 1];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + ent[i + u]);
#pragma unroll
      for (int k = 0; k < NW; ++k) w[u][k] = p[k];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) accum<SPD, J, MS>(acc, w[u]);
  }
  for (; i < n; ++i) {
    uint32_t w[J + 1];
    const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + ent[i]);
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = p[k];
    accum<SPD, J, MS>(acc, w);
  }
}

// ---- packed partial sums (spd = 4).  Word e[k] holds, in its low and high 16-bit halves, the
// partial sums of output samples 4k and 4k + 2 of the lane's tile; o[k] those of 4k + 1 and
// 4k + 3.  For a channel whose samples start at byte MS of the lane's first LDS dword, the two
// samples of a word are bytes MS + f and MS + f + 2 of the dword sequence w[k], w[k + 1]
// (f = 0 for e, 1 for o): one v_perm_b32 (or AND) moves both into their halves, and v_add3_u32
// adds two channels' words at a time.  Per four samples this is 3 instructions instead of 4
// single-byte adds.  A staged chunk has at most 255 channels, so a half never exceeds
// 255 * 255 < 2^16; the halves are widened into the int32 totals once per chunk.
template <int S>
__device__ __forceinline__ uint32_t field_pair(const uint32_t* w, int k) {
  // bytes S and S + 2 of (w[k], w[k + 1]) zero-extended into the low and high halves
  if constexpr (S == 0)
    return w[k] & 0x00FF00FFu;
  else if constexpr (S == 1)
    return __builtin_amdgcn_perm(w[k], w[k], 0x0C030C01u);
  else if constexpr (S == 4)
    return w[k + 1] & 0x00FF00FFu;
  else  // selector bytes index the 8-byte value w[k + 1]:w[k]; 0x0C yields a zero byte
    return __builtin_amdgcn_perm(w[k + 1], w[k], 0x0C000C00u | ((S + 2u) << 16) | S);
}

template <int J, int MS>
__device__ __forceinline__ void add_pk(uint32_t* e, uint32_t* o, const uint32_t* w1,
                                       const uint32_t* w2) {
#pragma unroll
  for (int k = 0; k < J; ++k) {
    e[k] += field_pair<MS>(w1, k) + field_pair<MS>(w2, k);
    o[k] += field_pair<MS + 1>(w1, k) + field_pair<MS + 1>(w2, k);
  }
}

template <int J, int MS>
__device__ __forceinline__ void add_pk1(uint32_t* e, uint32_t* o, const uint32_t* w) {
#pragma unroll
  for (int k = 0; k < J; ++k) {
    e[k] += field_pair<MS>(w, k);
    o[k] += field_pair<MS + 1>(w, k);
  }
}

// Packed counterpart of accum_run.  With PF (tiles with at most 60 accumulators per lane, so
// that the registers suffice) four channels per step, the next step's four offsets being read
// while this step's words are summed, so the window reads need not wait for the list read (the
// lists' four pad words keep that read in bounds at the end of the last run); then, and
// otherwise, two channels per step.
template <int J, int MS, bool PF>
__device__ __forceinline__ void accum_run_pk(uint32_t* e, uint32_t* o, const int32_t* ent, int n,
                                             const uint8_t* lane_base) {
  constexpr int NW = (MS == 0) ? J : J + 1;
  int i = 0;
  if (PF && n >= 4) {
    int32_t q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = ent[u];
    for (; i + 4 <= n; i += 4) {
      uint32_t w[4][J + 1];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + q[u]);
#pragma unroll
        for (int k = 0; k < NW; ++k) w[u][k] = p[k];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = ent[i + 4 + u];
      add_pk<J, MS>(e, o, w[0], w[1]);
      add_pk<J, MS>(e, o, w[2], w[3]);
    }
  }
  for (; i + 2 <= n; i += 2) {
    uint32_t w[2][J + 1];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + ent[i + u]);
#pragma unroll
      for (int k = 0; k < NW; ++k) w[u][k] = p[k];
    }
    add_pk<J, MS>(e, o, w[0], w[1]);
  }
  if (i < n) {
    uint32_t w[J + 1];
    const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + ent[i]);
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = p[k];
    add_pk1<J, MS>(e, o, w);
  }
}

// ---- packed partial sums of 16-bit samples (spd = 2, downsampled data).  Word p[k] holds the
// partial sums of outputs 2k and 2k + 1 in its halves.  For MS = 0 an LDS dword already is such
// a pair and is added as it is; for MS = 1 one v_alignbyte_b32 takes the pair out of two
// neighbouring dwords.  A half holds up to floor(65535 / (255 D)) channels (the plan limits its
// chunks to that), after which the halves are widened into the int32 totals.
template <int MS>
__device__ __forceinline__ uint32_t half_pair(const uint32_t* w, int k) {
  if constexpr (MS == 0)
    return w[k];
  else  // bytes 2..5 of the 8-byte value w[k + 1]:w[k]
    return __builtin_amdgcn_alignbyte(w[k + 1], w[k], 2);
}

template <int J, int MS>
__device__ __forceinline__ void add_pk16(uint32_t* pk, const uint32_t* w1, const uint32_t* w2) {
#pragma unroll
  for (int k = 0; k < J; ++k) pk[k] += half_pair<MS>(w1, k) + half_pair<MS>(w2, k);
}

template <int J, int MS, bool PF>
__device__ __forceinline__ void accum_run_pk16(uint32_t* pk, const int32_t* ent, int n,
                                               const uint8_t* lane_base) {
  constexpr int NW = (MS == 0) ? J : J + 1;
  int i = 0;
  if (PF && n >= 4) {
    int32_t q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = ent[u];
    for (; i + 4 <= n; i += 4) {
      uint32_t w[4][J + 1];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + q[u]);
#pragma unroll
        for (int k = 0; k < NW; ++k) w[u][k] = p[k];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = ent[i + 4 + u];
      add_pk16<J, MS>(pk, w[0], w[1]);
      add_pk16<J, MS>(pk, w[2], w[3]);
    }
  }
  for (; i + 2 <= n; i += 2) {
    uint32_t w[2][J + 1];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + ent[i + u]);
#pragma unroll
      for (int k = 0; k < NW; ++k) w[u][k] = p[k];
    }
    add_pk16<J, MS>(pk, w[0], w[1]);
  }
  if (i < n) {
    uint32_t w[J + 1];
    const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + ent[i]);
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = p[k];
#pragma unroll
    for (int k = 0; k < J; ++k) pk[k] += half_pair<MS>(w, k);
  }
}

template <int J>
__device__ __forceinline__ void flush_pk16(uint32_t* acc, uint32_t* pk) {
#pragma unroll
  for (int k = 0; k < J; ++k) {
    add_half<0>(acc[2 * k], pk[k]);
    add_half<1>(acc[2 * k + 1], pk[k]);
    pk[k] = 0;
  }
}

// ---- DM pairs on 16-bit samples (spd = 2).  The lane sums two neighbouring DM trials of the
// block together.  In channel c their windows start S = M0 + DELTA halves apart, DELTA =
// r1 - r0 >= 0 (the delay grows with DM; the plan refuses pairs that are further apart), and
// one read of J + ceil(S / 2) dwords from the first trial's word covers both: the first trial
// adds half pairs at parity M0, the second those S halves further on.  The plan sorts each
// pair's channels by (M0, DELTA), kPairClasses straight-line classes, so that the word offsets
// are compile-time constants.  Against one read per trial this halves the LDS traffic at equal
// delays and saves a third at DELTA = 6, which is what bounds the 16-bit kernels.
constexpr int kPairMaxDelta = kPairMaxDeltaHost;
constexpr int kPairClasses = 2 * (kPairMaxDelta + 1);  // 16: four 8-bit counts per word

template <int J, int M0, int DELTA, bool PF>
__device__ __forceinline__ void accum_run_pair(uint32_t* pk0, uint32_t* pk1, const int32_t* ent,
                                               int n, const uint8_t* lane_base) {
  constexpr int S = M0 + DELTA;
  constexpr int NW = J + (S + 1) / 2;  // union of [M0, M0 + 2J) and [S, S + 2J) halves
  constexpr int W1 = S / 2, P1 = S % 2;
  int i = 0;
  if (PF && n >= 4) {
    int32_t q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = ent[u];
    for (; i + 4 <= n; i += 4) {
      uint32_t w[4][NW];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + q[u]);
#pragma unroll
        for (int k = 0; k < NW; ++k) w[u][k] = p[k];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = ent[i + 4 + u];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        add_pk16<J, M0>(pk0, w[2 * h], w[2 * h + 1]);
        add_pk16<J, P1>(pk1, w[2 * h] + W1, w[2 * h + 1] + W1);
      }
    }
  }
  for (; i + 2 <= n; i += 2) {
    uint32_t w[2][NW];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + ent[i + u]);
#pragma unroll
      for (int k = 0; k < NW; ++k) w[u][k] = p[k];
    }
    add_pk16<J, M0>(pk0, w[0], w[1]);
    add_pk16<J, P1>(pk1, w[0] + W1, w[1] + W1);
  }
  if (i < n) {
    uint32_t w[NW];
    const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + ent[i]);
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = p[k];
#pragma unroll
    for (int k = 0; k < J; ++k) {
      pk0[k] += half_pair<M0>(w, k);
      pk1[k] += half_pair<P1>(w + W1, k);
    }
  }
}

// Every class of one pair, in the plan's order: class = M0 * (kPairMaxDelta + 1) + DELTA, its
// channel count in byte (class % 4) of cnt[class / 4].
template <int J, int CLS, bool PF>
__device__ __forceinline__ void accum_pair_classes(uint32_t* pk0, uint32_t* pk1,
                                                   const int32_t* ent, const uint32_t* cnt,
                                                   const uint8_t* lane_base) {
  if constexpr (CLS < kPairClasses) {
    const int n = (cnt[CLS / 4] >> (8 * (CLS % 4))) & 0xff;
    accum_run_pair<J, CLS / (kPairMaxDelta + 1), CLS % (kPairMaxDelta + 1), PF>(pk0, pk1, ent, n,
                                                                                 lane_base);
    accum_pair_classes<J, CLS + 1, PF>(pk0, pk1, ent + n, cnt, lane_base);
  }
}

// A block's offset list read from global memory through the scalar cache: base and index are
// uniform, so four offsets are one s_load_dwordx4, which costs the LDS and the VALU nothing.
typedef const __attribute__((address_space(4))) int32_t* const_list_t;

// NW consecutive LDS dwords of a channel's window, from the lane's word at byte offset off.
template <int NW>
__device__ __forceinline__ void load_words(uint32_t* w, const uint8_t* lane_base, int32_t off) {
  const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + off);
#pragma unroll
  for (int k = 0; k < NW; ++k) w[k] = p[k];
}

// ---- DM pairs in raw frames (spd = 2).  As the DM pairs above, but each trial adds the raw
// dwords of a channel into one of two frames chosen by the parity of its first sample: word k
// of frame 0 holds outputs 2k and 2k + 1 as they are, frame 1 (J + 1 words) holds them one
// sample later, which one v_alignbyte_b32 per word undoes when the frames are widened at the
// end of the pair's chunk.  A half never carries into its neighbour (a chunk holds at most
// floor(65535 / (255 D)) channels), so the frames are exact: a channel costs one add per word
// and trial, shared by two channels in v_add3_u32, and no per-channel alignment.  A class's
// channels are read STEP at a time: four (then the last one to three together), or two or one
// where the registers must leave room for six or eight waves per SIMD.
template <int J, int M0, int DELTA, int STEP>
__device__ __forceinline__ void accum_run_pair_frames(uint32_t (*f0)[J + 1],
                                                      uint32_t (*f1)[J + 1], int32_t lv, int pos,
                                                      int n, const uint8_t* lane_base) {
  constexpr int S = M0 + DELTA;
  constexpr int NW = J + (S + 1) / 2;    // union of both trials' words
  constexpr int W1 = S / 2, P1 = S % 2;  // the second trial's first word and parity
  constexpr int N0 = J + M0, N1 = J + P1;
  int i = 0;
  if constexpr (STEP == 1) {  // one channel per step: fewest words live
    for (; i < n; ++i) {
      uint32_t w[NW];
      load_words<NW>(w, lane_base, __builtin_amdgcn_readlane(lv, pos + i));
#pragma unroll
      for (int k = 0; k < N0; ++k) f0[M0][k] += w[k];
#pragma unroll
      for (int k = 0; k < N1; ++k) f1[P1][k] += w[W1 + k];
    }
    return;
  }
  if constexpr (STEP == 2) {  // two channels per step: fewer words live, for more waves
    for (; i + 2 <= n; i += 2) {
      uint32_t w[2][NW];
#pragma unroll
      for (int u = 0; u < 2; ++u)
        load_words<NW>(w[u], lane_base, __builtin_amdgcn_readlane(lv, pos + i + u));
#pragma unroll
      for (int k = 0; k < N0; ++k) f0[M0][k] += w[0][k] + w[1][k];
#pragma unroll
      for (int k = 0; k < N1; ++k) f1[P1][k] += w[0][W1 + k] + w[1][W1 + k];
    }
    if (i < n) {
      uint32_t w[NW];
      load_words<NW>(w, lane_base, __builtin_amdgcn_readlane(lv, pos + i));
#pragma unroll
      for (int k = 0; k < N0; ++k) f0[M0][k] += w[k];
#pragma unroll
      for (int k = 0; k < N1; ++k) f1[P1][k] += w[W1 + k];
    }
    return;
  }
  for (; i + 4 <= n; i += 4) {
    uint32_t w[4][NW];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      load_words<NW>(w[u], lane_base, __builtin_amdgcn_readlane(lv, pos + i + u));
#pragma unroll
    for (int k = 0; k < N0; ++k) f0[M0][k] += (w[0][k] + w[1][k]) + (w[2][k] + w[3][k]);
#pragma unroll
    for (int k = 0; k < N1; ++k)
      f1[P1][k] += (w[0][W1 + k] + w[1][W1 + k]) + (w[2][W1 + k] + w[3][W1 + k]);
  }
  // the last 1-3 channels: read together (the unused reads repeat the run's last channel),
  // so that a short class waits for LDS once
  const int r = n - i;
  if (r > 0) {
    uint32_t w[3][NW];
#pragma unroll
    for (int u = 0; u < 3; ++u)
      load_words<NW>(w[u], lane_base, __builtin_amdgcn_readlane(lv, pos + i + min(u, r - 1)));
    if (r == 1) {
#pragma unroll
      for (int k = 0; k < N0; ++k) f0[M0][k] += w[0][k];
#pragma unroll
      for (int k = 0; k < N1; ++k) f1[P1][k] += w[0][W1 + k];
    } else if (r == 2) {
#pragma unroll
      for (int k = 0; k < N0; ++k) f0[M0][k] += w[0][k] + w[1][k];
#pragma unroll
      for (int k = 0; k < N1; ++k) f1[P1][k] += w[0][W1 + k] + w[1][W1 + k];
    } else {
#pragma unroll
      for (int k = 0; k < N0; ++k) f0[M0][k] += (w[0][k] + w[1][k]) + w[2][k];
#pragma unroll
      for (int k = 0; k < N1; ++k) f1[P1][k] += (w[0][W1 + k] + w[1][W1 + k]) + w[2][W1 + k];
    }
  }
}

// Every class of one pair.  The pair's offset list for the chunk (at most 64 entries: the plan
// caps these chunks) is held one entry per lane in lv, so a channel's offset comes from one
// v_readlane_b32 instead of an LDS round trip before each class's reads.
template <int J, int CLS, int STEP>
__device__ __forceinline__ void accum_pair_frames(uint32_t (*f0)[J + 1], uint32_t (*f1)[J + 1],
                                                  int32_t lv, int pos, const uint32_t* cnt,
                                                  const uint8_t* lane_base) {
  if constexpr (CLS < kPairClasses) {
    const int n = (cnt[CLS / 4] >> (8 * (CLS % 4))) & 0xff;
    accum_run_pair_frames<J, CLS / (kPairMaxDelta + 1), CLS % (kPairMaxDelta + 1), STEP>(
        f0, f1, lv, pos, n, lane_base);
    accum_pair_frames<J, CLS + 1, STEP>(f0, f1, lv, pos + n, cnt, lane_base);
  }
}

// Widen a trial's two parity frames into its int32 totals (outputs 2k, 2k + 1 per word).  Every
// channel of the chunk sits in exactly one of the two frames, so the halves of the two frames
// added together still hold at most one chunk of channels and one packed 16-bit add is exact.
template <int J>
__device__ __forceinline__ void flush_pair_frames(uint32_t* acc, const uint32_t (*f)[J + 1]) {
  typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int k = 0; k < J; ++k) {
    const uint32_t odd = __builtin_amdgcn_alignbyte(f[1][k + 1], f[1][k], 2);
    const uint32_t both = __builtin_bit_cast(
        uint32_t, __builtin_bit_cast(u16x2, f[0][k]) + __builtin_bit_cast(u16x2, odd));
    add_half<0>(acc[2 * k], both);
    add_half<1>(acc[2 * k + 1], both);
  }
}

// Widen the packed halves into the int32 totals (one SDWA add each) and clear them.
template <int J>
__device__ __forceinline__ void flush_pk(uint32_t* acc, uint32_t* e, uint32_t* o) {
#pragma unroll
  for (int k = 0; k < J; ++k) {
    add_half<0>(acc[4 * k], e[k]);
    add_half<1>(acc[4 * k + 2], e[k]);
    add_half<0>(acc[4 * k + 1], o[k]);
    add_half<1>(acc[4 * k + 3], o[k]);
    e[k] = 0;
    o[k] = 0;
  }
}

// ---- framed partial sums (spd = 4).  A channel whose samples start at byte MS of the lane's
// first LDS dword maps byte j of its k-th dword to output 4k + j - MS: a fixed frame per MS.
// Per DM and frame, A[k] accumulates the dwords as they are (their byte lanes overlap in a
// 32-bit sum) and O[k] the odd bytes moved into 16-bit halves (one v_perm_b32); v_add3_u32
// adds two channels at a time.  Because O is known exactly, the even-byte sums follow as
// E[k] = A[k] - (O[k] << 8) (exact while each 16-bit half stays below 2^16, i.e. for up to
// 257 channels), so a channel costs one perm and one add per dword: 2 instructions per 4 samples
// (for MS = 0; MS > 0 reads one dword more).  The four frames are widened into the int32
// totals only every 257 channels.
__device__ __forceinline__ uint32_t odd_bytes(uint32_t w) {
  return __builtin_amdgcn_perm(w, w, 0x0C030C01u);  // bytes 1 and 3 into the two halves
}

template <int NW>
__device__ __forceinline__ void add_fr(uint32_t* A, uint32_t* O, const uint32_t* w1,
                                       const uint32_t* w2) {
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    A[k] += w1[k] + w2[k];
    O[k] += odd_bytes(w1[k]) + odd_bytes(w2[k]);
  }
}

template <int J, int MS, bool PF>
__device__ __forceinline__ void accum_run_fr(uint32_t* A, uint32_t* O, const int32_t* ent, int n,
                                             const uint8_t* lane_base) {
  constexpr int NW = (MS == 0) ? J : J + 1;
  int i = 0;
  if (PF && n >= 4) {
    int32_t q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = ent[u];
    for (; i + 4 <= n; i += 4) {
      uint32_t w[4][J + 1];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + q[u]);
#pragma unroll
        for (int k = 0; k < NW; ++k) w[u][k] = p[k];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = ent[i + 4 + u];
      add_fr<NW>(A, O, w[0], w[1]);
      add_fr<NW>(A, O, w[2], w[3]);
    }
  }
  for (; i + 2 <= n; i += 2) {
    uint32_t w[2][J + 1];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + ent[i + u]);
#pragma unroll
      for (int k = 0; k < NW; ++k) w[u][k] = p[k];
    }
    add_fr<NW>(A, O, w[0], w[1]);
  }
  if (i < n) {
    uint32_t w[J + 1];
    const uint32_t* p = reinterpret_cast<const uint32_t*>(lane_base + ent[i]);
#pragma unroll
    for (int k = 0; k < NW; ++k) w[k] = p[k];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      A[k] += w[k];
      O[k] += odd_bytes(w[k]);
    }
  }
}

// Widen frame MS into the int32 totals (one SDWA add per output) and clear it.
template <int J, int MS>
__device__ __forceinline__ void flush_fr(uint32_t* acc, uint32_t* A, uint32_t* O) {
  constexpr int NW = (MS == 0) ? J : J + 1;
  constexpr int T = 4 * J;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const uint32_t e = A[k] - (O[k] << 8);
    const int i0 = 4 * k - MS;
    if (i0 >= 0 && i0 < T) add_half<0>(acc[i0], e);
    if (i0 + 1 >= 0 && i0 + 1 < T) add_half<0>(acc[i0 + 1], O[k]);
    if (i0 + 2 >= 0 && i0 + 2 < T) add_half<1>(acc[i0 + 2], e);
    if (i0 + 3 >= 0 && i0 + 3 < T) add_half<1>(acc[i0 + 3], O[k]);
    A[k] = 0;
    O[k] = 0;
  }
}

// ---- framed runs (spd = 4).  The channels of one sub-dword class MS form a run (the plan sorts
// them so); within a run the raw dwords are summed into a frame A (byte lanes overlap in the
// 32-bit sum) and their odd bytes, moved into 16-bit halves by one v_perm_b32, into O, two
// channels per v_add3_u32: 2 instructions per 4 samples instead of the packed sums' 3.  The
// first channels of the run initialise the frame, so nothing is cleared.  At the end of the
// run the frame is exact (a run has at most 255 channels, so every half stays below 2^16):
// E = A - (O << 8) holds the even bytes' sums, and E and O are added into the int32 totals
// directly (one SDWA add per output), so no packed halves persist between runs or chunks.
__device__ __forceinline__ uint32_t even_sums(uint32_t a, uint32_t o) {
  // a - 256 o (mod 2^32) in one instruction: the 24-bit product only needs o's low 24 bits
  uint32_t r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(o), "v"(-256), "v"(a));
  return r;
}

// Add frame MS (NW = J or J + 1 words) into the lane's int32 totals: byte j of word k is output
// 4k + j - MS; outputs outside the lane's T = 4J samples belong to no total of this lane.
//
// SH (shared last word): dword J of a lane's window is dword 0 of the next lane's, so for
// MS > 0 the lane sums only J dwords and takes the finished sums of dword J from lane + 1 (two
// ds_bpermute per run).  Lane 63 gets lane 0's instead: its last MS outputs are wrong, and the
// tile leaves its last 4 outputs to the next tile.
template <int J, int MS, bool SH = false>
__device__ __forceinline__ void frame_to_totals(uint32_t* acc, const uint32_t* A,
                                                const uint32_t* O) {
  constexpr int NW = (MS == 0) ? J : J + 1;
  constexpr int NR = (MS == 0 || SH) ? J : J + 1;  // words summed by this lane
  constexpr int T = 4 * J;
  uint32_t e[NW], o[NW];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    e[k] = even_sums(A[k], O[k]);
    o[k] = O[k];
  }
  if constexpr (NR < NW) {
    const int next = ((__lane_id() + 1) & 63) << 2;
    e[J] = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(next, static_cast<int>(e[0])));
    o[J] = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(next, static_cast<int>(o[0])));
  }
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int i0 = 4 * k - MS;
    if (i0 >= 0 && i0 < T) add_half<0>(acc[i0], e[k]);
    if (i0 + 2 >= 0 && i0 + 2 < T) add_half<1>(acc[i0 + 2], e[k]);
    if (i0 + 1 >= 0 && i0 + 1 < T) add_half<0>(acc[i0 + 1], o[k]);
    if (i0 + 3 >= 0 && i0 + 3 < T) add_half<1>(acc[i0 + 3], o[k]);
  }
}

// One run: n channels of class MS, whose window offsets in the chunk's LDS (bytes from the
// lane's word) ent lists in the plan's global table, read four at a time by scalar loads.
template <int J, int MS, bool SH>
__device__ __forceinline__ void accum_frame_run(uint32_t* acc, const_list_t ent, int n,
                                                const uint8_t* lane_base) {
  if (n == 0) return;
  constexpr int NW = (MS == 0 || SH) ? J : J + 1;
  uint32_t A[NW], O[NW];
  int i;
  if (n & 1) {  // an odd run starts with its lone channel: the frame is that channel's words
    uint32_t w[NW];
    load_words<NW>(w, lane_base, ent[0]);
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      A[k] = w[k];
      O[k] = odd_bytes(w[k]);
    }
    i = 1;
  } else {
    uint32_t w[2][NW];
    load_words<NW>(w[0], lane_base, ent[0]);
    load_words<NW>(w[1], lane_base, ent[1]);
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      A[k] = w[0][k] + w[1][k];
      O[k] = odd_bytes(w[0][k]) + odd_bytes(w[1][k]);
    }
    i = 2;
  }
  for (; i + 4 <= n; i += 4) {  // the rest in pairs, four offsets read at a time
    int32_t q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = ent[i + u];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t w[2][NW];
      load_words<NW>(w[0], lane_base, q[2 * h]);
      load_words<NW>(w[1], lane_base, q[2 * h + 1]);
      add_fr<NW>(A, O, w[0], w[1]);
    }
  }
  if (i < n) {
    uint32_t w[2][NW];
    load_words<NW>(w[0], lane_base, ent[i]);
    load_words<NW>(w[1], lane_base, ent[i + 1]);
    add_fr<NW>(A, O, w[0], w[1]);
  }
  frame_to_totals<J, MS, SH>(acc, A, O);
}

// Framed runs into group sums: at the end of a run of sub-dword class MS its frame, now exact
// (E = A - 256 O even bytes, O odd bytes, the sums of the lane's last dword taken from the next
// lane), is added into the lane's packed group sums he / ho, where word k holds outputs
// (4k, 4k + 2) and (4k + 1, 4k + 3).  Byte j of frame word k is output 4k + j - MS, so E and O
// land there directly (MS = 0), through one v_alignbyte_b32 per word (half-word shifts), or
// one word later (MS = 3, E).  A group has at most 257 channels, so no half carries into its
// neighbour and the 32-bit adds are exact.
template <int J, int MS>
__device__ __forceinline__ void frame_to_group(uint32_t* he, uint32_t* ho, const uint32_t* A,
                                               const uint32_t* O) {
  uint32_t e[J + 1], o[J + 1];
#pragma unroll
  for (int k = 0; k < J; ++k) {
    e[k] = even_sums(A[k], O[k]);
    o[k] = O[k];
  }
  if constexpr (MS > 0) {
    const int next = ((__lane_id() + 1) & 63) << 2;
    e[J] = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(next, static_cast<int>(e[0])));
    o[J] = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(next, static_cast<int>(o[0])));
  }
#pragma unroll
  for (int k = 0; k < J; ++k) {
    if constexpr (MS == 0) {
      he[k] += e[k];
      ho[k] += o[k];
    } else if constexpr (MS == 1) {
      he[k] += o[k];
      ho[k] += __builtin_amdgcn_alignbyte(e[k + 1], e[k], 2);
    } else if constexpr (MS == 2) {
      he[k] += __builtin_amdgcn_alignbyte(e[k + 1], e[k], 2);
      ho[k] += __builtin_amdgcn_alignbyte(o[k + 1], o[k], 2);
    } else {
      he[k] += __builtin_amdgcn_alignbyte(o[k + 1], o[k], 2);
      ho[k] += e[k + 1];
    }
  }
}

template <int J, int MS>
__device__ __forceinline__ void accum_frame_run_group(uint32_t* he, uint32_t* ho,
                                                      const int32_t* ent, int n,
                                                      const uint8_t* lane_base) {
  if (n == 0) return;
  uint32_t A[J], O[J];
  int i;
  if (n & 1) {
    uint32_t w[J];
    load_words<J>(w, lane_base, ent[0]);
#pragma unroll
    for (int k = 0; k < J; ++k) {
      A[k] = w[k];
      O[k] = odd_bytes(w[k]);
    }
    i = 1;
  } else {
    uint32_t w[2][J];
    load_words<J>(w[0], lane_base, ent[0]);
    load_words<J>(w[1], lane_base, ent[1]);
#pragma unroll
    for (int k = 0; k < J; ++k) {
      A[k] = w[0][k] + w[1][k];
      O[k] = odd_bytes(w[0][k]) + odd_bytes(w[1][k]);
    }
    i = 2;
  }
  for (; i + 4 <= n; i += 4) {  // the rest in pairs, four offsets read at a time
    int32_t q[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] = ent[i + u];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t w[2][J];
      load_words<J>(w[0], lane_base, q[2 * h]);
      load_words<J>(w[1], lane_base, q[2 * h + 1]);
      add_fr<J>(A, O, w[0], w[1]);
    }
  }
  if (i < n) {
    uint32_t w[2][J];
    load_words<J>(w[0], lane_base, ent[i]);
    load_words<J>(w[1], lane_base, ent[i + 1]);
    add_fr<J>(A, O, w[0], w[1]);
  }
  frame_to_group<J, MS>(he, ho, A, O);
}

typedef __attribute__((address_space(1))) const void* global_ptr_t;
typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Stage channel windows [c0, c0 + ncc) into buf (cc windows of win dwords, win % 4 == 0), one
// channel per wave at a time.  Windows that lie inside the input buffer are fetched with
// asynchronous global->LDS loads (completion: vmcnt); others (input buffer edges, absent rows)
// are read through registers with per-dword bounds checks.  Samples a window holds beyond its
// row's valid range only ever feed output samples that are not stored.
template <int SPD, int WAVES>
__device__ __forceinline__ void stage_windows(const DedispArgs& a, const uint8_t* sbrow, int b,
                                              int blk, int64_t t0, const int32_t* base_blk,
                                              int c0, int ncc, uint32_t* buf, int lane,
                                              int wave) {
  for (int jj = wave; jj < ncc; jj += WAVES) {
    const int c = c0 + jj;
    const int64_t ws = t0 + base_blk[c];
    const int src = src_beam(a, sbrow, b, c);
    uint32_t* dst = buf + jj * a.win;
    const uint8_t* first = nullptr;  // byte address of the window's first sample
    const uint8_t* lo = nullptr;
    const uint8_t* hi = nullptr;
    if constexpr (SPD == 4) {
      const uint8_t* row = row_ptr(a, src, c);
      if (row) first = row + ws;
      lo = a.in;
      hi = a.in_end;
    } else {
      const uint16_t* r16 = row_ptr16(a, src, c, blk);
      if (r16) first = reinterpret_cast<const uint8_t*>(r16 + ws);
      lo = reinterpret_cast<const uint8_t*>(a.in16);
      hi = reinterpret_cast<const uint8_t*>(a.in16_end);
    }
    const uint32_t* P = reinterpret_cast<const uint32_t*>(
        reinterpret_cast<uintptr_t>(first) & ~static_cast<uintptr_t>(3));
    const uint8_t* pb = reinterpret_cast<const uint8_t*>(P);
    // the dwords that hold at least one byte of the buffer (a buffer need not start or end on
    // a dword boundary; such a dword lies in the same page as its valid bytes, and the plan's
    // offsets never use the bytes outside the buffer as samples of a stored output)
    lo = reinterpret_cast<const uint8_t*>(reinterpret_cast<uintptr_t>(lo) & ~uintptr_t(3));
    hi = reinterpret_cast<const uint8_t*>((reinterpret_cast<uintptr_t>(hi) + 3) & ~uintptr_t(3));
    if (first && pb >= lo && pb + 4 * static_cast<int64_t>(a.win) <= hi) {
      for (int k4 = 4 * lane; k4 < a.win; k4 += 256)  // 16 bytes per lane, 1 KiB per wave
        __builtin_amdgcn_global_load_lds((global_ptr_t)(P + k4),
                                         (lds_ptr_t)(dst + (k4 - 4 * lane)), 16, 0, 0);
    } else {
      for (int k = lane; k < a.win; k += 64) {
        uint32_t v = 0;
        if (first && pb + 4 * k >= lo && pb + 4 * k + 4 <= hi) v = P[k];
        dst[k] = v;
      }
    }
  }
}

// Fetch the chunk's offset lists (all DMs of the block) into ent (m_blk x cc words) with
// asynchronous dword global->LDS loads, one DM's list per wave instruction.
template <int WAVES>
__device__ __forceinline__ void stage_lists(const DedispArgs& a, const int32_t* list_blk, int c0,
                                            int ncc, int32_t* ent, int lane, int wave) {
  for (int x = wave; x < a.nlist; x += WAVES) {
    const int32_t* src = list_blk + static_cast<int64_t>(x) * a.nchan + c0;
    for (int j0 = 0; j0 < ncc; j0 += 64)
      if (j0 + lane < ncc)
        __builtin_amdgcn_global_load_lds((global_ptr_t)(src + j0 + lane),
                                         (lds_ptr_t)(ent + x * a.cc + j0), 4, 0, 0);
  }
}

// Store a lane's sums of ACC DM trials (rows dwave0 + x) for outputs t0 + lane*T + i < tend
// (the end of the tile or of the row); off: output elements added (the channel group of split
// plans).
// A lane's N consecutive int32 sums to p, where p is M dwords past a 16-byte boundary (VW = 4)
// or M dwords past an 8-byte boundary (VW = 2): scalar stores up to the boundary, then vector
// stores, then the remainder.
template <int N, int VW, int M>
__device__ __forceinline__ void store_run(int32_t* p, const uint32_t* v) {
  constexpr int head = (VW - M) % VW;
  constexpr int nvec = (N - head) / VW;
#pragma unroll
  for (int i = 0; i < head; ++i) p[i] = static_cast<int32_t>(v[i]);
#pragma unroll
  for (int k = 0; k < nvec; ++k) {
    const int i = head + VW * k;
    if constexpr (VW == 4)
      *reinterpret_cast<uint4*>(p + i) = make_uint4(v[i], v[i + 1], v[i + 2], v[i + 3]);
    else
      *reinterpret_cast<uint2*>(p + i) = make_uint2(v[i], v[i + 1]);
  }
#pragma unroll
  for (int i = head + VW * nvec; i < N; ++i) p[i] = static_cast<int32_t>(v[i]);
}

// OUT16: the sums are stored as uint16 (split plans, whose groups are bounded to 16 bits).
template <int T, int ACC, bool OUT16>
__device__ __forceinline__ void store_tile(const DedispArgs& a, const uint32_t (*acc)[T],
                                           int64_t off, int b, int dwave0, int64_t t0,
                                           int64_t tend, int lane) {
#pragma unroll
  for (int x = 0; x < ACC; ++x) {
    const int d = dwave0 + x;
    if (d < a.ndm) {
      const int64_t row = off + static_cast<int64_t>(b) * a.out_bstride + d * a.out_pitch;
      if constexpr (OUT16) {
        // rows are 8-byte aligned (pitch a multiple of 4 samples) and a lane's T = 4 J samples
        // start at a multiple of 4: whole lanes store 16-bit pairs 8 bytes at a time when the
        // output starts 8-byte aligned (always, except a stream's full recomputation)
        static_assert(T % 4 == 0, "16-bit group stores need T % 4 == 0");
        uint16_t* o = reinterpret_cast<uint16_t*>(a.out) + row;
        const int64_t tl = t0 + static_cast<int64_t>(lane) * T;
        if (tl + T <= tend && (reinterpret_cast<uintptr_t>(o + tl) & 7u) == 0) {
          uint2* q = reinterpret_cast<uint2*>(o + tl);
#pragma unroll
          for (int k = 0; k < T / 4; ++k)
            q[k] = make_uint2((acc[x][4 * k] & 0xFFFFu) | (acc[x][4 * k + 1] << 16),
                              (acc[x][4 * k + 2] & 0xFFFFu) | (acc[x][4 * k + 3] << 16));
        } else {
#pragma unroll
          for (int i = 0; i < T; ++i)
            if (tl + i < tend) o[tl + i] = static_cast<uint16_t>(acc[x][i]);
        }
      } else {
        // lanes are T dwords apart, a multiple of 16 bytes for T % 4 == 0 (8 bytes for even
        // T): the alignment of a lane's run is that of the row's tile start, uniform
        int32_t* o = a.out + row;
        const int64_t tl = t0 + static_cast<int64_t>(lane) * T;
        int32_t* p = o + tl;
        const int mis = static_cast<int>((reinterpret_cast<uintptr_t>(p) >> 2) & 3);
        if (tl + T <= tend) {
          if constexpr (T % 4 == 0) {
            switch (mis) {
              case 0: store_run<T, 4, 0>(p, acc[x]); break;
              case 1: store_run<T, 4, 1>(p, acc[x]); break;
              case 2: store_run<T, 4, 2>(p, acc[x]); break;
              default: store_run<T, 4, 3>(p, acc[x]); break;
            }
          } else if constexpr (T % 2 == 0) {
            if (mis & 1)
              store_run<T, 2, 1>(p, acc[x]);
            else
              store_run<T, 2, 0>(p, acc[x]);
          } else {
#pragma unroll
            for (int i = 0; i < T; ++i) p[i] = static_cast<int32_t>(acc[x][i]);
          }
        } else if (T % 4 == 0 && T > 4 && tl + T - 4 == tend) {
          // the last lane of a tile whose lanes share their last dword: T - 4 outputs
          if constexpr (T % 4 == 0 && T > 4) {
            switch (mis) {
              case 0: store_run<T - 4, 4, 0>(p, acc[x]); break;
              case 1: store_run<T - 4, 4, 1>(p, acc[x]); break;
              case 2: store_run<T - 4, 4, 2>(p, acc[x]); break;
              default: store_run<T - 4, 4, 3>(p, acc[x]); break;
            }
          }
        } else {
#pragma unroll
          for (int i = 0; i < T; ++i)
            if (tl + i < tend) p[i] = static_cast<int32_t>(acc[x][i]);
        }
      }
    }
  }
}

// Group-sum variants: the packed halves of a channel group are its sums (at most 257 channels
// of bytes fit a half), stored as 16-bit samples.  Half words: e[k] holds outputs 4k and 4k+2,
// o[k] outputs 4k+1 and 4k+3; two v_perm_b32 put each four in natural order.  Clears e, o.
template <int J, int ACC>
__device__ __forceinline__ void store_group_pk(const DedispArgs& a, uint32_t (*e)[J],
                                               uint32_t (*o)[J], int64_t off, int b,
                                               int dwave0, int64_t t0, int64_t tend, int lane) {
  constexpr int T = 4 * J;
#pragma unroll
  for (int x = 0; x < ACC; ++x) {
    const int d = dwave0 + x;
    if (d < a.ndm) {
      const int64_t row = off + static_cast<int64_t>(b) * a.out_bstride + d * a.out_pitch;
      uint16_t* op = reinterpret_cast<uint16_t*>(a.out) + row;
      const int64_t tl = t0 + static_cast<int64_t>(lane) * T;
      if (tl + T <= tend && (reinterpret_cast<uintptr_t>(op + tl) & 7u) == 0) {
        uint2* q = reinterpret_cast<uint2*>(op + tl);
#pragma unroll
        for (int k = 0; k < J; ++k)
          q[k] = make_uint2(__builtin_amdgcn_perm(o[x][k], e[x][k], 0x05040100u),
                            __builtin_amdgcn_perm(o[x][k], e[x][k], 0x07060302u));
      } else {
#pragma unroll
        for (int k = 0; k < J; ++k) {
          const uint32_t v[4] = {e[x][k] & 0xFFFFu, o[x][k] & 0xFFFFu, e[x][k] >> 16,
                                 o[x][k] >> 16};
#pragma unroll
          for (int m = 0; m < 4; ++m)
            if (tl + 4 * k + m < tend) op[tl + 4 * k + m] = static_cast<uint16_t>(v[m]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < J; ++k) e[x][k] = o[x][k] = 0;
  }
}

// One tile: DM block blk, time tile tt, beam b.  Used by the one-launch-per-job kernel and by
// the persistent batch kernel; ends after its global stores with no LDS access pending.
template <int SPD, int J, int ACC, int WAVES, int PK, bool SPLIT = false>
__device__ __forceinline__ void dedisperse_tile(const DedispArgs& a, int blk, int tt, int b,
                                                uint32_t* lds) {
  constexpr int T = SPD * J;
  constexpr int TT = tile_outputs(T, PK);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // LDS: two buffers, each cc windows of win dwords followed by the chunk's offset lists and
  // 4 pad words; then (for SB formation) the beam's SB-table row
  const int buf_words = a.cc * a.win + a.m_blk * a.cc + 4;
  uint8_t* sbrow = reinterpret_cast<uint8_t*>(lds + a.nbuf * buf_words);
  const int64_t t0 = static_cast<int64_t>(tt) * TT;
  const int64_t tend = min(a.nout, t0 + TT);  // outputs this tile stores
  const int dwave0 = blk * a.m_blk + wave * ACC;
  const bool wave_active = dwave0 < a.ndm;

  // int32 totals (unused by the group-sum variants, whose groups fit the packed halves)
  constexpr int TA = is_group(PK) ? 1 : T;
  uint32_t acc[ACC][TA];
#pragma unroll
  for (int x = 0; x < ACC; ++x)
#pragma unroll
    for (int i = 0; i < TA; ++i) acc[x][i] = 0;
  // framed variants: per DM, four frames of J + 1 dword pairs (unused otherwise)
  constexpr int NF = (PK == 2) ? ACC : 1;
  constexpr int NFW = (PK == 2) ? J + 1 : 1;
  uint32_t fa[NF][4][NFW], fo[NF][4][NFW];
  if constexpr (PK == 2) {
#pragma unroll
    for (int x = 0; x < NF; ++x)
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int k = 0; k < NFW; ++k) fa[x][m][k] = fo[x][m][k] = 0;
  }
  // held and group-sum variants: per DM, packed halves that persist across chunks (unused
  // otherwise)
  constexpr int NH = (PK == 3 || is_group(PK)) ? ACC : 1;
  constexpr int NHW = (PK == 3 || is_group(PK)) ? J : 1;
  uint32_t he[NH][NHW], ho[NH][NHW];
  if constexpr (PK == 3 || is_group(PK)) {
#pragma unroll
    for (int x = 0; x < NH; ++x)
#pragma unroll
      for (int k = 0; k < NHW; ++k) he[x][k] = ho[x][k] = 0;
  }
  int since = 0;  // channels in the frames or held halves since they were last widened

  const int32_t* base_blk = a.base + static_cast<int64_t>(blk) * a.nchan;
  const int32_t* list_blk = a.list + static_cast<int64_t>(blk) * a.nlist * a.nchan;
  const uint32_t* cnt_blk = a.cnt + static_cast<int64_t>(blk) * a.nchunk * a.m_blk + wave * ACC;

  // prologue: pad words, the SB-table row, then chunk 0 into buffer 0
  if (threadIdx.x < 4 * a.nbuf) lds[(threadIdx.x >> 2) * buf_words + a.cc * a.win + a.m_blk * a.cc +
                           (threadIdx.x & 3)] = 0;
  if (a.sb_table)
    for (int c = threadIdx.x; c < a.nchan; c += WAVES * 64)
      sbrow[c] = a.sb_table[static_cast<int64_t>(b) * a.tbl_stride + c];
  __syncthreads();
  stage_windows<SPD, WAVES>(a, sbrow, b, blk, t0, base_blk, 0, min(a.cc, a.nchan), lds, lane,
                            wave);
  stage_lists<WAVES>(a, list_blk, 0, min(a.cc, a.nchan),
                     reinterpret_cast<int32_t*>(lds + a.cc * a.win), lane, wave);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int ch = 0; ch < a.nchunk; ++ch) {
    uint32_t* cur = lds + (a.nbuf == 2 ? (ch & 1) * buf_words : 0);
    const int c0 = ch * a.cc;
    // ---- split plans: the previous chunk ended a channel group: store its sums now, so that
    // the stores have this chunk's work to complete before the wait at its end
    if constexpr (SPLIT) {
      if (ch > 0 && (c0 % a.split) == 0 && wave_active) {
        if constexpr (is_group(PK)) {
          store_group_pk<J, ACC>(a, he, ho, (c0 / a.split - 1) * a.out_sstride, b, dwave0, t0,
                                 tend, lane);
        } else {
          if constexpr (PK == 3) {
#pragma unroll
            for (int x = 0; x < ACC; ++x) flush_pk<J>(acc[x], he[x], ho[x]);
          }
          store_tile<T, ACC, true>(a, acc, (c0 / a.split - 1) * a.out_sstride, b, dwave0, t0,
                                   tend, lane);
#pragma unroll
          for (int x = 0; x < ACC; ++x)
#pragma unroll
            for (int i = 0; i < T; ++i) acc[x][i] = 0;
        }
      }
    }
    // ---- one buffer: fetch this chunk now (the previous one's readers are done, see the
    // barrier at the end of the loop); the CU's other workgroups compute meanwhile
    if (a.nbuf == 1 && ch > 0) {
      stage_windows<SPD, WAVES>(a, sbrow, b, blk, t0, base_blk, c0, min(a.cc, a.nchan - c0),
                                cur, lane, wave);
      stage_lists<WAVES>(a, list_blk, c0, min(a.cc, a.nchan - c0),
                         reinterpret_cast<int32_t*>(cur + a.cc * a.win), lane, wave);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    // ---- two buffers: start fetching the next chunk into the other one
    if (a.nbuf == 2 && ch + 1 < a.nchunk) {
      uint32_t* nxt = lds + ((ch + 1) & 1) * buf_words;
      const int c1 = c0 + a.cc;
      const int ncc1 = min(a.cc, a.nchan - c1);
      stage_windows<SPD, WAVES>(a, sbrow, b, blk, t0, base_blk, c1, ncc1, nxt, lane, wave);
      stage_lists<WAVES>(a, list_blk, c1, ncc1, reinterpret_cast<int32_t*>(nxt + a.cc * a.win),
                         lane, wave);
    }
    // ---- held variants: a channel group's store has just widened the halves
    if constexpr (SPLIT && PK == 3) {
      if (ch > 0 && (c0 % a.split) == 0) since = 0;
    }
    // ---- held variants: widen the halves before they could exceed 257 channels
    if constexpr (PK == 3) {
      const int ncc = min(a.cc, a.nchan - c0);
      if (since + ncc > 257) {
        if (wave_active) {
#pragma unroll
          for (int x = 0; x < ACC; ++x) flush_pk<J>(acc[x], he[x], ho[x]);
        }
        since = 0;
      }
      since += ncc;
    }
    // ---- framed variants: widen the frames before they could exceed 257 channels
    if constexpr (PK == 2) {
      const int ncc = min(a.cc, a.nchan - c0);
      if (since + ncc > 257) {
        if (wave_active) {
#pragma unroll
          for (int x = 0; x < ACC; ++x) {
            flush_fr<J, 0>(acc[x], fa[x][0], fo[x][0]);
            flush_fr<J, 1>(acc[x], fa[x][1], fo[x][1]);
            flush_fr<J, 2>(acc[x], fa[x][2], fo[x][2]);
            flush_fr<J, 3>(acc[x], fa[x][3], fo[x][3]);
          }
        }
        since = 0;
      }
      since += ncc;
    }
    // ---- accumulate: each DM trial of the wave over the chunk, one run per sub-dword offset
    if (wave_active) {
      const int32_t* ent_cur = reinterpret_cast<const int32_t*>(cur + a.cc * a.win);
      const uint8_t* lane_base = reinterpret_cast<const uint8_t*>(cur) + 4 * J * lane;
#pragma unroll
      for (int x = 0; x < ACC; ++x) {
        const uint32_t packed =
            is_pairs(PK) ? 0u : __builtin_amdgcn_readfirstlane(cnt_blk[ch * a.m_blk + x]);
        const int32_t* ent = ent_cur + (wave * ACC + x) * a.cc;
        const int n0 = packed & 0xff, n1 = (packed >> 8) & 0xff;
        if constexpr (PK == 2) {
          static_assert(SPD == 4, "framed sums are for byte samples");
          const int n2 = (packed >> 16) & 0xff, n3 = packed >> 24;
          constexpr bool PF = ACC * 8 * (J + 1) + ACC * T <= 80;
          accum_run_fr<J, 0, PF>(fa[x][0], fo[x][0], ent, n0, lane_base);
          accum_run_fr<J, 1, PF>(fa[x][1], fo[x][1], ent + n0, n1, lane_base);
          accum_run_fr<J, 2, PF>(fa[x][2], fo[x][2], ent + n0 + n1, n2, lane_base);
          accum_run_fr<J, 3, PF>(fa[x][3], fo[x][3], ent + n0 + n1 + n2, n3, lane_base);
        } else if constexpr (PK == 3 || PK == 4) {
          static_assert(SPD == 4, "held halves are for byte samples");
          const int n2 = (packed >> 16) & 0xff, n3 = packed >> 24;
          // registers: the held halves, plus the int32 totals unless the halves are the sums
          constexpr bool PF = (PK == 4 ? 0 : ACC * T) + 2 * ACC * J <= 90;
          accum_run_pk<J, 0, PF>(he[x], ho[x], ent, n0, lane_base);
          accum_run_pk<J, 1, PF>(he[x], ho[x], ent + n0, n1, lane_base);
          accum_run_pk<J, 2, PF>(he[x], ho[x], ent + n0 + n1, n2, lane_base);
          accum_run_pk<J, 3, PF>(he[x], ho[x], ent + n0 + n1 + n2, n3, lane_base);
        } else if constexpr (PK == 11) {
          static_assert(SPD == 4, "framed runs are for byte samples");
          const int n2 = (packed >> 16) & 0xff, n3 = packed >> 24;
          accum_frame_run_group<J, 0>(he[x], ho[x], ent, n0, lane_base);
          accum_frame_run_group<J, 1>(he[x], ho[x], ent + n0, n1, lane_base);
          accum_frame_run_group<J, 2>(he[x], ho[x], ent + n0 + n1, n2, lane_base);
          accum_frame_run_group<J, 3>(he[x], ho[x], ent + n0 + n1 + n2, n3, lane_base);
        } else if constexpr (PK == 7 || PK == 9) {
          static_assert(SPD == 4, "framed runs are for byte samples");
          const int n2 = (packed >> 16) & 0xff, n3 = packed >> 24;
          constexpr bool SH = PK == 9;
          // the runs read their offsets from the global list through the scalar cache; the
          // chunk's copy in LDS goes unread, but fetching it has just brought those lines into
          // L2 (the whole list table does not stay there), so the scalar loads hit
          const const_list_t gl = (const_list_t)(list_blk +
                                                 static_cast<int64_t>(wave * ACC + x) * a.nchan + c0);
          accum_frame_run<J, 0, SH>(acc[x], gl, n0, lane_base);
          accum_frame_run<J, 1, SH>(acc[x], gl + n0, n1, lane_base);
          accum_frame_run<J, 2, SH>(acc[x], gl + n0 + n1, n2, lane_base);
          accum_frame_run<J, 3, SH>(acc[x], gl + n0 + n1 + n2, n3, lane_base);
        } else if constexpr (PK == 5) {
          // DM pairs: trials (x, x + 1) of the wave at even x; odd x have been summed
          static_assert(SPD == 2 && ACC % 2 == 0, "DM pairs are for 16-bit samples");
          if (x % 2 == 0) {
            const int pr = (wave * ACC + x) / 2;
            const uint32_t* cp = a.cnt + ((static_cast<int64_t>(blk) * a.nchunk + ch) *
                                              (a.m_blk / 2) + pr) * 4;
            uint32_t cnt4[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) cnt4[k] = __builtin_amdgcn_readfirstlane(cp[k]);
            uint32_t pk0[J], pk1[J];
#pragma unroll
            for (int k = 0; k < J; ++k) pk0[k] = pk1[k] = 0;
            constexpr bool PF = ACC * T <= 60;
            accum_pair_classes<J, 0, PF>(pk0, pk1, ent_cur + pr * a.cc, cnt4, lane_base);
            flush_pk16<J>(acc[x], pk0);
            flush_pk16<J>(acc[x + 1], pk1);
          }
        } else if constexpr (PK == 10) {
          // DM pairs in raw frames: trials (x, x + 1) at even x
          static_assert(SPD == 2 && ACC % 2 == 0, "DM pairs are for 16-bit samples");
          if (x % 2 == 0) {
            const int pr = (wave * ACC + x) / 2;
            const uint32_t* cp = a.cnt + ((static_cast<int64_t>(blk) * a.nchunk + ch) *
                                              (a.m_blk / 2) + pr) * 4;
            uint32_t cnt4[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) cnt4[k] = __builtin_amdgcn_readfirstlane(cp[k]);
            uint32_t f0[2][J + 1], f1[2][J + 1];
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
              for (int k = 0; k <= J; ++k) f0[m][k] = f1[m][k] = 0;
            const int32_t* lst = ent_cur + pr * a.cc;
            const int32_t lv = lane < min(a.cc, a.nchan - c0) ? lst[lane] : 0;
            accum_pair_frames<J, 0, WAVES == 16 ? 1 : WAVES == 12 ? 2 : 4>(f0, f1, lv, 0, cnt4,
                                                                           lane_base);
            flush_pair_frames<J>(acc[x], f0);
            flush_pair_frames<J>(acc[x + 1], f1);
          }
        } else if constexpr (PK && SPD == 2) {
          uint32_t pk[J];
#pragma unroll
          for (int k = 0; k < J; ++k) pk[k] = 0;
          constexpr bool PF = ACC * T <= 60;
          accum_run_pk16<J, 0, PF>(pk, ent, n0, lane_base);
          accum_run_pk16<J, 1, PF>(pk, ent + n0, n1, lane_base);
          flush_pk16<J>(acc[x], pk);
        } else if constexpr (PK) {
          const int n2 = (packed >> 16) & 0xff, n3 = packed >> 24;
          uint32_t e[J], o[J];
#pragma unroll
          for (int k = 0; k < J; ++k) e[k] = o[k] = 0;
          constexpr bool PF = ACC * T <= 60;
          accum_run_pk<J, 0, PF>(e, o, ent, n0, lane_base);
          accum_run_pk<J, 1, PF>(e, o, ent + n0, n1, lane_base);
          accum_run_pk<J, 2, PF>(e, o, ent + n0 + n1, n2, lane_base);
          accum_run_pk<J, 3, PF>(e, o, ent + n0 + n1 + n2, n3, lane_base);
          flush_pk<J>(acc[x], e, o);
        } else {
          accum_run<SPD, J, 0>(acc[x], ent, n0, lane_base);
          accum_run<SPD, J, 1>(acc[x], ent + n0, n1, lane_base);
          if constexpr (SPD == 4) {
            const int n2 = (packed >> 16) & 0xff, n3 = packed >> 24;
            accum_run<SPD, J, 2>(acc[x], ent + n0 + n1, n2, lane_base);
            accum_run<SPD, J, 3>(acc[x], ent + n0 + n1 + n2, n3, lane_base);
          }
        }
      }
    }
    // the next chunk has landed and nobody reads the current buffer any more
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  if constexpr (SPLIT) {  // the last channel group
    if (wave_active) {
      if constexpr (is_group(PK)) {
        store_group_pk<J, ACC>(a, he, ho, (a.nchan / a.split - 1) * a.out_sstride, b, dwave0,
                               t0, tend, lane);
      } else {
        if constexpr (PK == 3) {
#pragma unroll
          for (int x = 0; x < ACC; ++x) flush_pk<J>(acc[x], he[x], ho[x]);
        }
        store_tile<T, ACC, true>(a, acc, (a.nchan / a.split - 1) * a.out_sstride, b, dwave0,
                                 t0, tend, lane);
      }
    }
  }
  if (wave_active && !SPLIT) {
    if constexpr (PK == 3) {
#pragma unroll
      for (int x = 0; x < ACC; ++x) flush_pk<J>(acc[x], he[x], ho[x]);
    }
    if constexpr (PK == 2) {
#pragma unroll
      for (int x = 0; x < ACC; ++x) {
        flush_fr<J, 0>(acc[x], fa[x][0], fo[x][0]);
        flush_fr<J, 1>(acc[x], fa[x][1], fo[x][1]);
        flush_fr<J, 2>(acc[x], fa[x][2], fo[x][2]);
        flush_fr<J, 3>(acc[x], fa[x][3], fo[x][3]);
      }
    }
    if constexpr (!is_group(PK))  // group-sum variants run split plans only
      store_tile<T, ACC, false>(a, acc, 0, b, dwave0, t0, tend, lane);
  }
}

// One launch per job: workgroup -> tile, renumbered so that each of the 8 XCDs (to which
// workgroups are dealt round-robin) runs a contiguous range of (beam, time tile, DM block):
// neighbouring DM blocks read overlapping input windows and then share that XCD's L2.
template <int SPD, int J, int ACC, int WAVES, int PK, bool SPLIT>
__device__ __forceinline__ void dedisperse_grid(const DedispArgs& a, uint32_t* lds) {
  const int64_t bid = blockIdx.x;
  const int64_t q8 = a.nwg >> 3, r8 = a.nwg & 7, xcd = bid & 7, pos = bid >> 3;
  const int64_t lin = xcd < r8 ? xcd * (q8 + 1) + pos : r8 * (q8 + 1) + (xcd - r8) * q8 + pos;
  const int blk = static_cast<int>(lin % a.nblk);
  const int64_t rest = lin / a.nblk;
  dedisperse_tile<SPD, J, ACC, WAVES, PK, SPLIT>(a, blk, static_cast<int>(rest % a.ntt),
                                                 static_cast<int>(rest / a.ntt), lds);
}

template <int SPD, int J, int ACC, int WAVES, int PK, bool SPLIT>
__global__ __launch_bounds__(WAVES * 64) void dedisperse_kernel(DedispArgs a) {
  extern __shared__ uint32_t lds[];
  dedisperse_grid<SPD, J, ACC, WAVES, PK, SPLIT>(a, lds);
}

// 12-wave blocks of 2 DMs per wave (framed runs; DM pairs in raw frames, which read two
// channels per step to fit): compiled for six waves per SIMD (at most 80 VGPRs), so that two
// blocks share a CU and every SIMD holds six waves to hide the LDS latency of the others (the
// 8-wave tilings hold four).  16-wave blocks of one DM pair per wave, reading one channel per
// step, and of one 16-bit trial per wave (the second subband step with 16 fine trials): eight
// waves per SIMD (at most 64 VGPRs).
template <>
__global__ __launch_bounds__(12 * 64) __attribute__((amdgpu_waves_per_eu(6)))
void dedisperse_kernel<4, 5, 2, 12, 9, false>(DedispArgs a) {
  extern __shared__ uint32_t lds[];
  dedisperse_grid<4, 5, 2, 12, 9, false>(a, lds);
}
template <>
__global__ __launch_bounds__(12 * 64) __attribute__((amdgpu_waves_per_eu(6)))
void dedisperse_kernel<2, 5, 2, 12, 10, false>(DedispArgs a) {
  extern __shared__ uint32_t lds[];
  dedisperse_grid<2, 5, 2, 12, 10, false>(a, lds);
}
template <>
__global__ __launch_bounds__(16 * 64) __attribute__((amdgpu_waves_per_eu(8)))
void dedisperse_kernel<2, 5, 1, 16, 0, false>(DedispArgs a) {
  extern __shared__ uint32_t lds[];
  dedisperse_grid<2, 5, 1, 16, 0, false>(a, lds);
}
template <>
__global__ __launch_bounds__(16 * 64) __attribute__((amdgpu_waves_per_eu(8)))
void dedisperse_kernel<2, 5, 2, 16, 10, false>(DedispArgs a) {
  extern __shared__ uint32_t lds[];
  dedisperse_grid<2, 5, 2, 16, 10, false>(a, lds);
}

// Group-sum split plans (the first subband step): four waves per SIMD, two 8-wave workgroups.
template <int SPD, int J, int ACC, int WAVES, int PK>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(4)))
void dedisperse_group_kernel(DedispArgs a) {
  extern __shared__ uint32_t lds[];
  dedisperse_grid<SPD, J, ACC, WAVES, PK, true>(a, lds);
}
// 16-wave blocks of 2 DMs per wave: eight waves per SIMD (at most 64 VGPRs).
template <>
__global__ __launch_bounds__(16 * 64) __attribute__((amdgpu_waves_per_eu(8)))
void dedisperse_group_kernel<4, 5, 2, 16, 11>(DedispArgs a) {
  extern __shared__ uint32_t lds[];
  dedisperse_grid<4, 5, 2, 16, 11, true>(a, lds);
}

// Split plans (the first subband step): the group stores add live registers; four waves per
// SIMD keep two 8-wave workgroups on a CU.
template <int SPD, int J, int ACC, int WAVES, int PK>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(4)))
void dedisperse_split_kernel(DedispArgs a) {
  extern __shared__ uint32_t lds[];
  dedisperse_grid<SPD, J, ACC, WAVES, PK, true>(a, lds);
}

// Persistent batch kernel: a grid sized to the machine pulls tiles of several jobs from work
// queues until they are empty (every workgroup reaches that exit).  The host orders the tiles
// (most expensive job first, then beam, time tile, DM block) and cuts them into 8 contiguous
// ranges, one per XCD: a workgroup drains the queue of its own XCD first, so neighbouring DM
// blocks -- which read overlapping windows -- share that XCD's L2, then steals from the others.
struct BatchArgs {
  const DedispArgs* jobs;      // [njobs]
  const int64_t* item_start;   // [njobs + 1] prefix sums of tiles per job
  unsigned long long* counter; // [8 * 16]: one counter per XCD queue, 128 bytes apart
  int64_t part[9];             // queue x holds items [part[x], part[x + 1])
  int32_t njobs;
};

// Waves per SIMD of the persistent kernel: as many as the one-launch-per-job kernel of the
// same tiling reaches, since the plan sizes its LDS chunks for that many workgroups per CU.
// Four (<= 128 VGPRs: two 8-wave workgroups per CU), except six (<= 80 VGPRs) for the two
// plain tilings whose one-launch kernels need 76 registers: 16-bit samples with 32 DMs per
// block (three 8-wave workgroups per CU) and byte samples with 8 DMs per 4-wave block (six),
// and for the 12-wave tilings (two blocks per CU); eight for the 16-wave 16-bit tilings.
template <int SPD, int J, int ACC, int WAVES, int PK>
constexpr int batch_waves_per_eu() {
  return (PK == 0 && J == 5 && ((SPD == 2 && ACC == 4 && WAVES == 8) ||
                                (SPD == 4 && ACC == 2 && WAVES == 4)))
             ? 6
             : (WAVES == 12                                                   ? 6
                : (WAVES == 16 && SPD == 2 && (PK == 10 || (PK == 0 && ACC == 1))) ? 8
                                                                                 : 4);
}

template <int SPD, int J, int ACC, int WAVES, int PK>
__global__ __launch_bounds__(WAVES * 64)
__attribute__((amdgpu_waves_per_eu(batch_waves_per_eu<SPD, J, ACC, WAVES, PK>())))
void dedisperse_batch_kernel(BatchArgs q) {
  extern __shared__ uint32_t lds[];
  __shared__ long long s_item;
  const int home = blockIdx.x & 7;
  for (int k = 0; k < 8; ++k) {
    const int x = (home + k) & 7;
    for (;;) {
      if (threadIdx.x == 0)
        s_item = q.part[x] + static_cast<long long>(atomicAdd(q.counter + 16 * x, 1ULL));
      __syncthreads();
      // the same value in every lane: make that visible so the job lookup and the descriptor
      // stay in scalar registers
      const long long raw = s_item;
      const long long item = static_cast<long long>(
          (static_cast<unsigned long long>(
               static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(raw >> 32))))
           << 32) |
          static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(raw))));
      __syncthreads();
      if (item >= q.part[x + 1]) break;
      int j = 0;
      while (j + 1 < q.njobs && q.item_start[j + 1] <= item) ++j;
      j = __builtin_amdgcn_readfirstlane(j);
      // copy the descriptor word by word into scalar registers
      DedispArgs a;
      {
        static_assert(sizeof(DedispArgs) % 4 == 0, "descriptor must be whole words");
        const int* src = reinterpret_cast<const int*>(q.jobs + j);
        int* dst = reinterpret_cast<int*>(&a);
#pragma unroll
        for (int k = 0; k < static_cast<int>(sizeof(DedispArgs) / 4); ++k)
          dst[k] = __builtin_amdgcn_readfirstlane(src[k]);
      }
      const int64_t lin = item - q.item_start[j];
      const int blk = static_cast<int>(lin % a.nblk);
      const int64_t rest = lin / a.nblk;
      dedisperse_tile<SPD, J, ACC, WAVES, PK>(a, blk, static_cast<int>(rest % a.ntt),
                                              static_cast<int>(rest / a.ntt), lds);
    }
  }
}

static size_t lds_bytes(const DedispArgs& a) {
  return a.nbuf * (static_cast<size_t>(a.win) * a.cc + static_cast<size_t>(a.m_blk) * a.cc + 4) * 4 +
         (a.sb_table ? ((static_cast<size_t>(a.nchan) + 3) & ~static_cast<size_t>(3)) : 0);
}

template <typename K>
static int allow_full_lds(K kernel, int static_bytes = 0) {
  ARTS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024 - static_bytes));
  return ARTS_OK;
}

// static LDS of the persistent kernel (the work-queue slot), rounded to its allocation unit
constexpr int kBatchStaticLds = 512;

template <typename K>
static int launch_kernel(K kernel, int waves, const DedispArgs& a, size_t lds, hipStream_t s,
                         bool& attr_set) {
  if (!attr_set) {
    if (int st = allow_full_lds(kernel)) return st;
    attr_set = true;
  }
  (void)hipGetLastError();
  hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(a.nwg)), dim3(waves * 64), lds, s, a);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

// Plans with channel groups (the first step of subband plans) run an instance that stores each
// group's sums; it exists for the byte-sample variants that are not framed.
template <int SPD, int J, int ACC, int WAVES, int PK>
static int launch_variant(DedispArgs a, hipStream_t s) {
  const size_t lds = lds_bytes(a);
  if (lds > 160 * 1024) return fail(ARTS_E_INVAL, "LDS request %zu B exceeds 160 KiB", lds);
  a.nwg = static_cast<int64_t>(a.nbeam) * a.ntt * a.nblk;
  if (a.nwg > INT_MAX) return fail(ARTS_E_INVAL, "grid too large (%lld blocks)", (long long)a.nwg);
  static bool attr_plain = false, attr_split = false;  // one pair per template instance
  if (a.split > 0) {
    if constexpr (is_group(PK))
      return launch_kernel(&dedisperse_group_kernel<SPD, J, ACC, WAVES, PK>, WAVES, a, lds, s,
                           attr_split);
    else if constexpr (SPD == 4 && PK != 2)
      return launch_kernel(&dedisperse_split_kernel<SPD, J, ACC, WAVES, PK>, WAVES, a, lds, s,
                           attr_split);
    else
      return fail(ARTS_E_INVAL, "this tiling variant cannot split channel groups");
  }
  if constexpr (is_group(PK))
    return fail(ARTS_E_INVAL, "group-sum tilings run the first subband step only");
  else
    return launch_kernel(&dedisperse_kernel<SPD, J, ACC, WAVES, PK, false>, WAVES, a, lds, s,
                         attr_plain);
}

template <int SPD, int J, int ACC, int WAVES, int PK>
static int launch_batch_variant(BatchArgs q, size_t lds, hipStream_t s) {
  if constexpr (is_group(PK)) {
    return fail(ARTS_E_INVAL, "group-sum tilings run the first subband step only");
  } else {
    if (lds + kBatchStaticLds > 160 * 1024)
      return fail(ARTS_E_INVAL, "LDS request %zu B too large for a persistent launch", lds);
    static bool attr_set = false;
    if (!attr_set) {
      if (int st = allow_full_lds(&dedisperse_batch_kernel<SPD, J, ACC, WAVES, PK>,
                                  kBatchStaticLds))
        return st;
      attr_set = true;
    }
    int per_cu = 0, dev = 0, ncu = 0;
    ARTS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(&dedisperse_batch_kernel<SPD, J, ACC, WAVES, PK>),
        WAVES * 64, lds));
    ARTS_HIP(hipGetDevice(&dev));
    ARTS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t grid =
        std::max<int64_t>(1, std::min<int64_t>(q.part[8], int64_t(std::max(1, per_cu)) * ncu));
    (void)hipGetLastError();
    hipLaunchKernelGGL((dedisperse_batch_kernel<SPD, J, ACC, WAVES, PK>),
                       dim3(static_cast<unsigned>(grid)), dim3(WAVES * 64), lds, s, q);
    ARTS_HIP(hipGetLastError());
    return ARTS_OK;
  }
}

// Kernel arguments of one job.  Rows must start on dword boundaries (pitch and pointer); the
// alignment class g0 of the input pointer selects the plan's offset tables.
static int make_args(arts_plan_s* p, const DedispJob& job, DedispArgs* out) {
  DedispArgs a{};
  int g0 = 0;
  if (!p->is16()) {
    if (job.pitch % 4 != 0) return fail(ARTS_E_INVAL, "internal: row pitch not a multiple of 4");
    g0 = static_cast<int>(reinterpret_cast<uintptr_t>(job.in) & 3u);
  } else {
    if (!job.in16) return fail(ARTS_E_INVAL, "16-bit plan needs 16-bit rows");
    if (job.pitch16 % 2 != 0 || job.in16_blk % 2 != 0 ||
        (reinterpret_cast<uintptr_t>(job.in16) & 1u))
      return fail(ARTS_E_INVAL, "internal: 16-bit row pitch must be even");
    g0 = static_cast<int>((reinterpret_cast<uintptr_t>(job.in16) >> 1) & 1u);
  }
  if (int st = ensure_tables(p, g0)) return st;
  const Tiling& t = p->tiling;
  const TileVariant& v = kVariants[t.variant];
  a.in = job.in;
  a.in_end = job.in + job.in_bytes;
  a.nin = job.nin;
  a.pitch = job.pitch > 0 ? job.pitch : job.nin;
  a.nsamp_d = job.nin / p->ds;
  a.in16 = job.in16;
  a.in16_end = job.in16 ? job.in16 + job.in16_elems : nullptr;
  a.pitch16 = job.pitch16;
  a.sb_table = job.sb_table;
  a.base = t.d_base;
  a.list = t.d_list[g0];
  a.cnt = t.d_cnt[g0];
  a.out = job.out;
  a.nout = job.nout;
  a.out_pitch = job.out_pitch > 0 ? job.out_pitch : job.nout;
  a.out_bstride = job.out_bstride > 0 ? job.out_bstride : p->ndm * a.out_pitch;
  a.out16 = job.out16 ? 1 : 0;
  a.in16_blk = job.in16_blk;
  a.split = p->split;
  a.out_sstride = job.out_sstride;
  if ((p->split > 0) != job.out16)
    return fail(ARTS_E_INVAL, "internal: 16-bit output goes with channel groups");
  a.src_stride = job.src_stride > 0 ? job.src_stride : p->nchan;
  a.tbl_stride = job.tbl_stride > 0 ? job.tbl_stride : p->nchan;
  a.nchan = p->nchan;
  a.ndm = p->ndm;
  a.nsrc = job.nsrc;
  a.ds = p->ds;
  a.nbeam = job.nbeam;
  a.m_blk = t.m_blk;
  a.nlist = is_pairs(v.pack) ? t.m_blk / 2 : t.m_blk;
  a.nbuf = t.nbuf;
  a.nblk = t.nblk;
  a.win = t.win_dwords;
  a.cc = t.cc;
  a.nchunk = t.nchunk;
  const int TT = tile_outputs(v.spd * v.j, v.pack);
  a.ntt = static_cast<int>((a.nout + TT - 1) / TT);
  *out = a;
  return ARTS_OK;
}

// Two-step subband dedispersion.  Step 1: one launch of the step-1 plan (all channels at the
// coarse DMs, each channel's delay relative to its subband's reference) whose sums are split
// per subband into 16-bit rows Y[b][s][j][t], t < L1 = nin - max step-1 delay.  Step 2: the
// step-2 plan sums the subbands at the fine DMs; its DM blocks are the coarse groups
// (m_blk = nfine), so block j reads rows Y[b][.][j] (in16_blk = one row pitch).
static int launch_subband(arts_plan_s* p, const DedispJob& job, hipStream_t s) {
  const int64_t L1 = job.nin - p->max_d1;
  const int32_t pad = job.y ? job.y_pad : 0;
  const int64_t L1p = job.y && job.y_pitch > 0 ? job.y_pitch : subband_pitch(p, job.nin, pad);
  const int64_t rows = static_cast<int64_t>(job.nbeam) * p->nsub * p->ncoarse;
  const int64_t need = (rows - 1) * L1p + pad + L1;  // through the last row's window
  if (L1 < 1 || job.nout > L1 - p->sb2->max_delay || pad < 0 || pad > 3 || L1p < pad + L1 ||
      (L1p & 3) != 0)
    return fail(ARTS_E_INVAL, "internal: subband job shorter than its delays");
  uint16_t* y = job.y ? job.y : p->d_y;
  const int64_t have = job.y ? job.y_elems : p->y_cap;
  if (need > have) return fail(ARTS_E_INVAL, "internal: subband workspace not prepared");
  DedispJob j1 = job;
  j1.out = reinterpret_cast<int32_t*>(y + pad);
  j1.nout = L1;
  if (job.y && job.y_prev && job.y_new > 0 && job.y_new < L1) {
    // rows [0, L1 - new) are the previous window's rows [new, L1): already in place when the
    // window moved by `new` inside its buffer, else copied; step 1 computes the rest from the
    // last new + max_d1 input samples of the window
    const int64_t keep = L1 - job.y_new;
    const uint16_t* src = job.y_prev + pad + job.y_new;
    if (src != y + pad) {
      if (!job.y_lo || !job.y_hi || src < job.y_lo || src + (rows - 1) * L1p + keep > job.y_hi)
        return fail(ARTS_E_INVAL, "internal: subband history outside its buffer");
      const uint8_t* lo = reinterpret_cast<const uint8_t*>(job.y_lo);
      const uint8_t* hi = reinterpret_cast<const uint8_t*>(job.y_hi);
      if (int st = launch_copy_rows(reinterpret_cast<uint8_t*>(y + pad), 2 * L1p,
                                    reinterpret_cast<const uint8_t*>(src), 2 * L1p, rows, 2 * keep,
                                    lo, hi, s))
        return st;
    }
    j1.in = job.in + keep;
    j1.in_bytes = job.in_bytes - keep;
    j1.nin = job.y_new + p->max_d1;
    j1.out = reinterpret_cast<int32_t*>(y + pad + keep);
    j1.nout = job.y_new;
  }
  j1.out16 = true;
  j1.out_pitch = L1p;
  j1.out_sstride = static_cast<int64_t>(p->ncoarse) * L1p;
  j1.out_bstride = static_cast<int64_t>(p->nsub) * p->ncoarse * L1p;
  if (int st = launch_dedisperse(p->sb1, j1, s)) return st;
  DedispJob j2;
  j2.in16 = y + pad;
  j2.in16_elems = have - pad;
  j2.pitch16 = static_cast<int64_t>(p->ncoarse) * L1p;
  j2.in16_blk = L1p;
  j2.nin = L1;
  j2.nsrc = job.nbeam;
  j2.nbeam = job.nbeam;
  j2.out = job.out;
  j2.nout = job.nout;
  j2.out_pitch = job.out_pitch;
  j2.out_bstride = job.out_bstride;
  return launch_dedisperse(p->sb2, j2, s);
}

// Workgroups per CU that registers and waves allow (LDS aside) for a variant's kernel of one
// kind (kOccPlain / kOccSplit: the one-launch kernel of plain or split plans; kOccBatch: the
// persistent batch kernel); 0 if the runtime cannot tell or the kind does not exist.
template <int SPD, int J, int ACC, int WAVES, int PK>
static int occupancy_variant(int kind) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  if constexpr (is_group(PK)) {  // group sums: split plans only, no persistent instance
    if (kind == kOccBatch) return 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, dedisperse_group_kernel<SPD, J, ACC, WAVES, PK>, WAVES * 64, 0);
  } else {
    if (kind == kOccBatch) {
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &n, dedisperse_batch_kernel<SPD, J, ACC, WAVES, PK>, WAVES * 64, 0);
      return e == hipSuccess ? n : 0;
    }
    if constexpr (SPD == 4 && PK != 2) {
      if (kind == kOccSplit) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &n, dedisperse_split_kernel<SPD, J, ACC, WAVES, PK>, WAVES * 64, 0);
        return e == hipSuccess ? n : 0;
      }
    }
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &n, dedisperse_kernel<SPD, J, ACC, WAVES, PK, false>, WAVES * 64, 0);
  }
  return e == hipSuccess ? n : 0;
}

int variant_occupancy(int variant, int kind) {
  switch (variant) {
#define ARTS_X(id, spd, j, acc, waves, pack) \
    case id: return occupancy_variant<spd, j, acc, waves, pack>(kind);
    ARTS_TILINGS(ARTS_X)
#undef ARTS_X
    default: return 0;
  }
}

int variant_blocks_per_cu(int variant, bool split) {
  return variant_occupancy(variant, split ? kOccSplit : kOccPlain);
}

int launch_dedisperse(arts_plan_s* p, const DedispJob& job, hipStream_t s) {
  if (p->nsub > 0) return launch_subband(p, job, s);
  DedispArgs a;
  if (int st = make_args(p, job, &a)) return st;
  switch (p->tiling.variant) {
#define ARTS_X(id, spd, j, acc, waves, pack) \
    case id: return launch_variant<spd, j, acc, waves, pack>(a, s);
    ARTS_TILINGS(ARTS_X)
#undef ARTS_X
    default: return fail(ARTS_E_INVAL, "plan has no tiling");
  }
}

BatchBuffers::~BatchBuffers() {
  if (ev) (void)hipEventSynchronize(ev);
  if (ev) (void)hipEventDestroy(ev);
  if (d_jobs) (void)hipFree(d_jobs);
  if (d_start) (void)hipFree(d_start);
  if (d_counter) (void)hipFree(d_counter);
  if (h_stage) (void)hipHostFree(h_stage);
}

// All jobs of one launch share the plans' tiling variant.  Jobs are ordered by the cost of one
// tile (channels staged per tile), most expensive first.
int launch_dedisperse_batch(arts_plan_s* const* plans, const DedispJob* jobs, int n,
                            BatchBuffers& bb, hipStream_t s) {
  if (n <= 0) return ARTS_OK;
  // a single job: the one-launch kernel, whose workgroups retire tile by tile, so that work
  // queued on another HIP stream (a concurrent serving tick) gets compute units as they free up
  // instead of waiting for a persistent grid to drain its queue
  if (n == 1) return launch_dedisperse(plans[0], jobs[0], s);
  const int variant = plans[0]->tiling.variant;
  for (int i = 1; i < n; ++i)
    if (plans[i]->tiling.variant != variant)
      return fail(ARTS_E_INVAL, "internal: mixed tiling variants in one batch launch");
  std::vector<DedispArgs> args(n);
  std::vector<int> order(n);
  size_t lds = 0;
  for (int i = 0; i < n; ++i) {
    if (int st = make_args(plans[i], jobs[i], &args[i])) return st;
    order[i] = i;
  }
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    return int64_t(args[x].nchan) * args[x].win > int64_t(args[y].nchan) * args[y].win;
  });
  // stage descriptors in pinned memory; the previous launch's upload must have finished
  const size_t need = n * sizeof(DedispArgs) + (n + 1) * sizeof(int64_t);
  if (bb.ev) ARTS_HIP(hipEventSynchronize(bb.ev));
  if (need > bb.stage_bytes || n > bb.cap) {
    if (bb.h_stage) (void)hipHostFree(bb.h_stage);
    if (bb.d_jobs) (void)hipFree(bb.d_jobs);
    if (bb.d_start) (void)hipFree(bb.d_start);
    bb.h_stage = nullptr;
    bb.d_jobs = nullptr;
    bb.d_start = nullptr;
    bb.stage_bytes = bb.cap = 0;
    ARTS_HIP(hipHostMalloc(&bb.h_stage, need));
    ARTS_HIP(hipMalloc(&bb.d_jobs, n * sizeof(DedispArgs)));
    ARTS_HIP(hipMalloc(&bb.d_start, (n + 1) * sizeof(int64_t)));
    bb.stage_bytes = need;
    bb.cap = n;
  }
  if (!bb.d_counter) ARTS_HIP(hipMalloc(&bb.d_counter, 8 * 16 * sizeof(unsigned long long)));
  if (!bb.ev) ARTS_HIP(hipEventCreateWithFlags(&bb.ev, hipEventDisableTiming));
  DedispArgs* hj = reinterpret_cast<DedispArgs*>(bb.h_stage);
  int64_t* hs = reinterpret_cast<int64_t*>(static_cast<char*>(bb.h_stage) + n * sizeof(DedispArgs));
  hs[0] = 0;
  for (int k = 0; k < n; ++k) {
    DedispArgs a = args[order[k]];
    a.nwg = static_cast<int64_t>(a.nbeam) * a.ntt * a.nblk;
    hj[k] = a;
    hs[k + 1] = hs[k] + a.nwg;
    const size_t l = lds_bytes(a);
    lds = std::max(lds, l);
  }
  if (lds > 160 * 1024) return fail(ARTS_E_INVAL, "LDS request %zu B exceeds 160 KiB", lds);
  ARTS_HIP(hipMemcpyAsync(bb.d_jobs, hj, n * sizeof(DedispArgs), hipMemcpyHostToDevice, s));
  ARTS_HIP(hipMemcpyAsync(bb.d_start, hs, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  ARTS_HIP(hipEventRecord(bb.ev, s));
  if (int st = launch_zero_u64(bb.d_counter, 8 * 16, s)) return st;
  BatchArgs q{};
  q.jobs = static_cast<const DedispArgs*>(bb.d_jobs);
  q.item_start = bb.d_start;
  q.counter = bb.d_counter;
  q.njobs = n;
  for (int x = 0; x <= 8; ++x) q.part[x] = hs[n] * x / 8;
  switch (variant) {
#define ARTS_X(id, spd, j, acc, waves, pack) \
    case id: return launch_batch_variant<spd, j, acc, waves, pack>(q, lds, s);
    ARTS_TILINGS(ARTS_X)
#undef ARTS_X
    default: return fail(ARTS_E_INVAL, "plan has no tiling");
  }
}

// ------------------------------------------------------------------ row statistics ----
// One workgroup per series row: S1 = sum x, S2 = sum x^2 over t < nrep in int64 (exact for
// nrep * max|x|^2 < 2^63), then mean and population sigma in FP64 from the exact integers,
// centred on m0 = S1 / N to avoid cancellation:  N var = S2c - r^2 / N with
// S2c = sum (x - m0)^2 and r = S1 - N m0.
__global__ __launch_bounds__(256) void row_stats_kernel(const int32_t* __restrict__ series,
                                                        int64_t L, int64_t nrep,
                                                        int64_t* __restrict__ s1_out,
                                                        double* __restrict__ musig) {
  const int64_t row = blockIdx.x;
  const int32_t* x = series + row * L;
  long long s1 = 0, s2 = 0;
  int64_t t = threadIdx.x;
  for (; t + 3 * 256 < nrep; t += 4 * 256) {
    const long long v0 = x[t], v1 = x[t + 256], v2 = x[t + 512], v3 = x[t + 768];
    s1 += v0 + v1 + v2 + v3;
    s2 += v0 * v0 + v1 * v1 + v2 * v2 + v3 * v3;
  }
  for (; t < nrep; t += 256) {
    const long long v = x[t];
    s1 += v;
    s2 += v * v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_xor(s1, off, 64);
    s2 += __shfl_xor(s2, off, 64);
  }
  __shared__ long long red[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = s1;
    red[1][wave] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const long long S1 = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const long long S2 = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    const long long N = nrep;
    const long long m0 = S1 / N;
    const long long r = S1 - N * m0;
    const long long S2c = S2 - 2 * m0 * S1 + N * m0 * m0;
    const double dn = static_cast<double>(N);
    const double var = (static_cast<double>(S2c) - static_cast<double>(r) * static_cast<double>(r) / dn) / dn;
    s1_out[row] = S1;
    musig[2 * row] = static_cast<double>(m0) + static_cast<double>(r) / dn;
    musig[2 * row + 1] = var > 0.0 ? sqrt(var) : 0.0;
  }
}

int launch_row_stats(const int32_t* series, int64_t L, int64_t nrep, int64_t nrows, int64_t* s1,
                     double* musig, hipStream_t s) {
  if (nrows > INT_MAX) return fail(ARTS_E_INVAL, "too many series rows");
  (void)hipGetLastError();
  hipLaunchKernelGGL(row_stats_kernel, dim3(static_cast<unsigned>(nrows)), dim3(256), 0, s,
                     series, L, nrep, s1, musig);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

// ------------------------------------------------------------------ boxcars ----
// A row's reported window is cut into segments of SEG start samples.  For a segment starting at
// s0 the workgroup loads x[s0 - 1 .. s0 + n + wmax - 2] into LDS and turns it into an
// exclusive prefix sum P (uint32, wrapping: differences are exact because every boxcar sum is
// below 2^31), so B_w(t) = P[t - s0 + 1 + w] - P[t - s0 + 1] for t in [s0 - 1, s0 + n - 1].
constexpr int kSeg = 2048;
constexpr int kBoxThreads = 256;
// dynamic LDS of the boxcar kernels: (kSeg + wmax + 1) words, wmax <= kMaxWidth
constexpr int kBoxLdsMax = (kSeg + kMaxWidth + 1) * 4;

// In place: P[0 .. ne) becomes its exclusive prefix sum and P[ne] the total, by a workgroup of
// NT threads (wsum: NT / 64 words).  Starts and ends with a barrier.
template <int NT>
__device__ void scan_inplace(uint32_t* P, int ne, uint32_t* wsum) {
  __syncthreads();
  // an odd stride between threads' ranges spreads them over all LDS banks
  const int per = ((ne + NT - 1) / NT) | 1;
  const int lo = min(ne, static_cast<int>(threadIdx.x) * per), hi = min(ne, lo + per);
  // eight independent LDS reads per step, so that one wait covers all of them
  uint32_t tot = 0;
  for (int k = lo; k < hi; k += 8) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = k + u < hi ? P[k + u] : 0u;
#pragma unroll
    for (int u = 0; u < 8; ++u) tot += v[u];
  }
  // inclusive scan of per-thread totals: within the wave, then across the 4 waves
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = tot;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t v = __shfl_up(inc, off, 64);
    if (lane >= off) inc += v;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (int w = 0; w < wave; ++w) pre += wsum[w];
  uint32_t run = pre + inc - tot;  // exclusive prefix of this thread's range
  for (int k = lo; k < hi; k += 8) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = k + u < hi ? P[k + u] : 0u;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k + u < hi) {
        P[k + u] = run;
        run += v[u];
      }
  }
  if (threadIdx.x == NT - 1) P[ne] = pre + inc;
  __syncthreads();
}

template <int NT>
__device__ void load_prefix(const int32_t* __restrict__ x, int64_t L, int64_t s0, int ne,
                            uint32_t* P, uint32_t* wsum) {
  for (int k = threadIdx.x; k < ne; k += NT) {
    const int64_t idx = s0 - 1 + k;
    P[k] = (idx >= 0 && idx < L) ? static_cast<uint32_t>(x[idx]) : 0u;
  }
  scan_inplace<NT>(P, ne, wsum);
}

struct WidthParams {
  long long thr_int;  // B_w > thr_int  <=>  S/N > threshold
  float scale;        // S/N = (N B_w - w S1) * scale
};

__device__ __forceinline__ WidthParams width_params(int w, int64_t N, double mu, double sigma,
                                                    double thr) {
  WidthParams wp;
  const double sw = sqrt(static_cast<double>(w));
  double rhs = floor(static_cast<double>(w) * mu + thr * sigma * sw);
  if (rhs > 4.0e18) rhs = 4.0e18;
  if (rhs < -4.0e18) rhs = -4.0e18;
  wp.thr_int = static_cast<long long>(rhs);
  wp.scale = sigma > 0.0 ? static_cast<float>(1.0 / (static_cast<double>(N) * sigma * sw)) : 0.0f;
  return wp;
}

// Mean and population sigma of a series from its exact sums over N samples (shifted by the
// integer part of the mean, so that the variance comes from small numbers).
__device__ __forceinline__ void row_musig(long long S1, long long S2, long long N, double* mu,
                                          double* sigma) {
  const long long m0 = S1 / N, r = S1 - N * m0;
  const long long S2c = S2 - 2 * m0 * S1 + N * m0 * m0;
  const double dn = static_cast<double>(N);
  const double var =
      (static_cast<double>(S2c) - static_cast<double>(r) * static_cast<double>(r) / dn) / dn;
  *mu = static_cast<double>(m0) + static_cast<double>(r) / dn;
  *sigma = var > 0.0 ? sqrt(var) : 0.0;
}

__global__ __launch_bounds__(kBoxThreads) void boxcar_snr_kernel(
    const int32_t* __restrict__ series, int64_t L, int64_t nrep, int32_t ndm, int64_t nseg,
    const int32_t* __restrict__ widths, int32_t nw, int32_t wmax, const int64_t* __restrict__ s1,
    const double* __restrict__ musig, int32_t* __restrict__ sums, float* __restrict__ snr) {
  extern __shared__ uint32_t P[];
  __shared__ uint32_t wsum[4];
  const int64_t row = blockIdx.x / nseg;
  const int64_t s0 = (blockIdx.x % nseg) * kSeg;
  const int n = static_cast<int>(min<int64_t>(kSeg, nrep - s0));
  const int ne = n + wmax;
  load_prefix<kBoxThreads>(series + row * L, L, s0, ne, P, wsum);
  const int64_t b = row / ndm, d = row % ndm;
  const double mu = musig[2 * row], sigma = musig[2 * row + 1];
  const long long S1 = s1[row];
  for (int wi = 0; wi < nw; ++wi) {
    const int w = widths[wi];
    const WidthParams wp = width_params(w, nrep, mu, sigma, 0.0);
    const int64_t obase = ((b * nw + wi) * ndm + d) * nrep + s0;
    for (int k = threadIdx.x; k < n; k += kBoxThreads) {
      const int32_t B = static_cast<int32_t>(P[k + 1 + w] - P[k + 1]);
      if (sums) sums[obase + k] = B;
      if (snr) {
        const long long num = static_cast<long long>(nrep) * B - static_cast<long long>(w) * S1;
        snr[obase + k] = sigma > 0.0 ? static_cast<float>(num) * wp.scale : 0.0f;
      }
    }
  }
}

int launch_boxcar_snr(const arts_plan_s* p, const int32_t* series, int32_t nbeam, int64_t L,
                      int64_t nrep, const int64_t* s1, const double* musig, int32_t* sums,
                      float* snr, hipStream_t s) {
  const int64_t nseg = (nrep + kSeg - 1) / kSeg;
  const int64_t nblocks = static_cast<int64_t>(nbeam) * p->ndm * nseg;
  if (nblocks > INT_MAX) return fail(ARTS_E_INVAL, "boxcar grid too large");
  const size_t lds = (kSeg + p->wmax + 1) * sizeof(uint32_t);
  static bool attr = false;
  if (!attr) {
    ARTS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&boxcar_snr_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kBoxLdsMax));
    attr = true;
  }
  (void)hipGetLastError();
  hipLaunchKernelGGL(boxcar_snr_kernel, dim3(static_cast<unsigned>(nblocks)), dim3(kBoxThreads),
                     lds, s, series, L, nrep, p->ndm, nseg, p->d_widths, p->nwidth, p->wmax, s1,
                     musig, sums, snr);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

// ------------------------------------------------------------------ candidates ----
// One workgroup per series row (beam, DM).  Pass 1 computes the row's moments over the
// reported window exactly as row_stats_kernel does.  Pass 2 walks the window in segments of
// kCandSeg start samples staged as a prefix sum in LDS; for every width each thread classifies
// its kCandSeg / NT consecutive starts (S/N above threshold <=> B_w > floor(w mu + thr sigma
// sqrt w)):
// runs that begin and end inside its range are emitted at once; the leading run fragment (from
// its first start) and the trailing one (to its last start) are summarised in LDS.  The thread
// that holds a run's first start then walks the following threads' summaries to the run's end,
// or to the segment's end, in which case the open run is carried into the next segment.  Every
// run therefore yields exactly one candidate at its largest B_w (earliest on ties), whatever its
// length, with O(threads) work for the longest run.
constexpr int kCandSeg = 4096;
// dynamic LDS limit of a resident row (16 Ki words: rows of up to 16 383 - wmax searched starts)
constexpr int kCandResLds = 64 * 1024;
// threads of a candidate workgroup: 8 waves for rows of at least kCandLong starts (a resident
// row of that length fills 2 workgroups per CU), else 4
constexpr int kCandLong = 8192;
constexpr int kMaxWidthsCand = 64;
// plans with up to this many widths take the whole-row maxima of all widths in one pass
constexpr int kCandRegW = 16;

struct CandOut {
  arts_candidate* cand;
  unsigned long long* count;
  int64_t cap;
  int64_t t_offset;
  int32_t beam, dm_index, ds;
  float dm;
  long long S1;
  int64_t N;
};

__device__ __forceinline__ void emit_cand(const CandOut& o, int64_t t, int32_t best, int w,
                                          float scale) {
  const unsigned long long idx = atomicAdd(o.count, 1ULL);
  if (static_cast<int64_t>(idx) < o.cap) {
    arts_candidate c;
    c.sample = t + o.t_offset;
    c.beam = o.beam;
    c.dm_index = o.dm_index;
    c.width = w;
    c.downsample = o.ds;
    const long long num = static_cast<long long>(o.N) * best - static_cast<long long>(w) * o.S1;
    c.snr = static_cast<float>(num) * scale;
    c.dm = o.dm;
    o.cand[idx] = c;
  }
}

// RES: the row is resident.  Its n = nrep + wmax - 1 samples are staged into LDS once (direct
// global->LDS loads), the moments are taken from LDS, one in-place prefix sum serves every
// segment, and a whole-row test per width (one barrier) leaves the run scan to the widths
// that exceed the threshold somewhere.  Otherwise (rows too long for LDS) the moments are read
// from global memory and each segment is loaded and summed on its own.
template <bool RES, int NT>
__global__ __launch_bounds__(NT) void candidates_kernel(
    const int32_t* __restrict__ series, int64_t pitch, int64_t L, int64_t nrep, int32_t ndm,
    const int32_t* __restrict__ widths, int32_t nw, int32_t wmax, const double* __restrict__ dms,
    double thr, int64_t t_offset, int32_t beam_offset, int32_t ds,
    arts_candidate* __restrict__ cand, unsigned long long* __restrict__ count, int64_t cap,
    const uint8_t* __restrict__ flags, int32_t decim) {
  // rows the pre-pass found below the threshold at every width give no candidate
  if (flags != nullptr && flags[blockIdx.x] == 0) return;
  extern __shared__ uint32_t P[];
  __shared__ uint32_t wsum[NT / 64];
  __shared__ long long red[2][NT / 64];
  __shared__ long long s_thr[kMaxWidthsCand];
  __shared__ float s_scale[kMaxWidthsCand];
  __shared__ int32_t s_wid[kMaxWidthsCand];
  __shared__ int32_t c_open[2][kMaxWidthsCand], c_best[2][kMaxWidthsCand];
  __shared__ int64_t c_arg[2][kMaxWidthsCand];
  __shared__ int32_t t_full[NT], t_prelen[NT], t_premax[NT];
  __shared__ int32_t t_prearg[NT], t_suf[NT];
  __shared__ double s_musig[2];
  __shared__ int s_hit[kMaxWidthsCand];
  __shared__ unsigned long long s_hitmask;

  const int64_t row = blockIdx.x;
  const int32_t* x = series + row * pitch;
  const int tid = threadIdx.x;
  const int nres = RES ? static_cast<int>(nrep) + wmax - 1 : 0;
  if constexpr (RES) {
    // P[1 + t] = x[t], t < nres, by dword global->LDS loads (lane i lands at base + 4 i)
    const int lane = tid & 63, wave = tid >> 6;
    for (int k0 = wave * 64; k0 < nres; k0 += NT)
      if (k0 + lane < nres)
        __builtin_amdgcn_global_load_lds((global_ptr_t)(x + k0 + lane), (lds_ptr_t)(P + 1 + k0),
                                         4, 0, 0);
    if (tid == 0) P[0] = 0u;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  // ---- pass 1: moments over t < nrep (exact int64 sums), eight independent reads per step
  {
    long long s1 = 0, s2 = 0;
    for (int64_t t0 = tid; t0 < nrep; t0 += 8 * NT) {
      int32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t t = t0 + u * NT;
        if constexpr (RES)
          v[u] = t < nrep ? static_cast<int32_t>(P[1 + static_cast<int>(t)]) : 0;
        else
          v[u] = t < nrep ? x[t] : 0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        s1 += v[u];
        s2 += static_cast<long long>(v[u]) * v[u];
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s1 += __shfl_xor(s1, off, 64);
      s2 += __shfl_xor(s2, off, 64);
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = s1;
      red[1][tid >> 6] = s2;
    }
  }
  __syncthreads();
  long long S1 = 0;
#pragma unroll
  for (int v = 0; v < NT / 64; ++v) S1 += red[0][v];
  if (tid == 0) {
    long long S2 = 0;
#pragma unroll
    for (int v = 0; v < NT / 64; ++v) S2 += red[1][v];
    row_musig(S1, S2, nrep, &s_musig[0], &s_musig[1]);
    s_hitmask = 0;
  }
  __syncthreads();
  const double mu = s_musig[0], sigma = s_musig[1];
  if (!(sigma > 0.0)) return;  // uniform: a flat series gives no candidates
  if (tid < nw) {
    const WidthParams wp = width_params(widths[tid], nrep, mu, sigma, thr);
    s_thr[tid] = wp.thr_int;
    s_scale[tid] = wp.scale;
    s_wid[tid] = widths[tid];
    c_open[0][tid] = 0;
  }
  CandOut o;
  o.cand = cand;
  o.count = count;
  o.cap = cap;
  o.t_offset = t_offset;
  o.beam = static_cast<int32_t>(row / ndm) + beam_offset;
  o.dm_index = static_cast<int32_t>(row % ndm);
  o.ds = ds;
  o.dm = static_cast<float>(dms[row % ndm]);
  o.S1 = S1;
  o.N = nrep;
  if constexpr (RES) {
    // exclusive prefix over x[-1 .. nres) with x[-1] = 0: B_w(t) = P[t + 1 + w] - P[t + 1]
    scan_inplace<NT>(P, nres + 1, wsum);
    const int nr = static_cast<int>(nrep);
    if (nw <= kCandRegW) {
      // whole-row maximum of B_w for every width at once: each start's P[t + 1] is read once
      // and reused by all widths (maxima in registers), then one workgroup-wide OR of the
      // per-width hit bits
      int wreg[kCandRegW];
      int32_t bm[kCandRegW];
#pragma unroll
      for (int wi = 0; wi < kCandRegW; ++wi) {
        wreg[wi] = wi < nw ? __builtin_amdgcn_readfirstlane(s_wid[wi]) : 0;
        bm[wi] = INT_MIN;
      }
      int t0 = tid;
      for (; t0 + 3 * NT < nr; t0 += 4 * NT) {
        const uint32_t* q = P + t0 + 1;
        uint32_t a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) a[u] = q[u * NT];
#pragma unroll
        for (int wi = 0; wi < kCandRegW; ++wi) {
          if (wi < nw) {
            const uint32_t* qw = q + wreg[wi];
            uint32_t b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) b[u] = qw[u * NT];
#pragma unroll
            for (int u = 0; u < 4; ++u) bm[wi] = max(bm[wi], static_cast<int32_t>(b[u] - a[u]));
          }
        }
      }
      for (; t0 < nr; t0 += NT) {
        const uint32_t a0 = P[t0 + 1];
#pragma unroll
        for (int wi = 0; wi < kCandRegW; ++wi)
          if (wi < nw) bm[wi] = max(bm[wi], static_cast<int32_t>(P[t0 + 1 + wreg[wi]] - a0));
      }
      unsigned long long hits = 0;
#pragma unroll
      for (int wi = 0; wi < kCandRegW; ++wi)
        if (wi < nw && static_cast<long long>(bm[wi]) > s_thr[wi]) hits |= 1ULL << wi;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) hits |= __shfl_xor(hits, off, 64);
      if ((tid & 63) == 0 && hits) atomicOr(&s_hitmask, hits);
      __syncthreads();
      if (tid < nw) s_hit[tid] = static_cast<int>((s_hitmask >> tid) & 1ULL);
    } else {
    // whole-row maximum of B_w per width: groups of 8 starts 256 apart, whose 16 reads share
    // one base address (immediate offsets) and are in flight together; then the last starts
    for (int wi = 0; wi < nw; ++wi) {
      const int w = s_wid[wi];
      int32_t bmax = INT_MIN;
      int t0 = tid;
      for (; t0 + 7 * NT < nr; t0 += 8 * NT) {
        const uint32_t* q = P + t0 + 1;
        const uint32_t* qw = q + w;
        uint32_t a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a[u] = q[u * NT];
          b[u] = qw[u * NT];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) bmax = max(bmax, static_cast<int32_t>(b[u] - a[u]));
      }
      for (; t0 < nr; t0 += NT)
        bmax = max(bmax, static_cast<int32_t>(P[t0 + 1 + w] - P[t0 + 1]));
      const int hit = __syncthreads_or(static_cast<long long>(bmax) > s_thr[wi] ? 1 : 0);
      if (tid == 0) s_hit[wi] = hit;
    }
    }
  }
  int cin = 0;  // carry buffer holding runs open at the previous segment's end
  const int k0 = tid * (kCandSeg / NT);
  for (int64_t s0 = 0; s0 < nrep; s0 += kCandSeg) {
    const int n = static_cast<int>(min<int64_t>(kCandSeg, nrep - s0));
    const uint32_t* Pseg = P;
    if constexpr (RES) {
      Pseg = P + s0;
      __syncthreads();  // every read of the carry slot cleared below has happened
    } else {
      // decimated integration reads a start's grid cell, up to wmax - 1 starts back: the
      // segment's prefix then begins that much earlier
      const int lb = decim != 0 ? wmax - 1 : 0;
      load_prefix<NT>(x, L, s0 - lb, n + wmax + lb, P, wsum);  // ends with a barrier
      Pseg = P + lb;
    }
    if (tid < nw) c_open[cin ^ 1][tid] = 0;
    if constexpr (RES) __syncthreads();
    for (int wi = 0; wi < nw; ++wi) {
      const int w = s_wid[wi];
      const long long T = s_thr[wi];
      if (RES && !s_hit[wi] && !c_open[cin][wi]) continue;  // uniform: shared values
      // ---- fast path: nothing above threshold in this segment and no run carried in
      {
        // starts interleaved across lanes: consecutive lanes read consecutive LDS words
        int32_t bmax = INT_MIN;
#pragma unroll
        for (int i = 0; i < (kCandSeg / NT); ++i) {
          const int k = tid + i * NT;
          if (k < n) bmax = max(bmax, static_cast<int32_t>(Pseg[k + 1 + w] - Pseg[k + 1]));
        }
        const bool any = static_cast<long long>(bmax) > T;
        if (!__syncthreads_or(any ? 1 : 0) && !c_open[cin][wi]) continue;
      }
      // ---- classify this thread's starts.  Decimated integration: start k holds the sum of
      // its grid cell, B_w(g) with g = k - r, r = (s0 + k + t_offset) mod w, so that a run over
      // consecutive grid starts is a run over consecutive k, and its first largest value sits
      // at a grid start; cells that begin before the row are below threshold
      bool in_pre = true, open = false;
      int pre_len = 0;
      int32_t pre_max = 0, best = 0;
      int pre_arg = 0, arg = 0;
      const bool dec = decim != 0 && w > 1;
      int r = 0;
      if (dec) {
        const int64_t m = (s0 + k0 + t_offset) % w;
        r = static_cast<int>(m < 0 ? m + w : m);
      }
#pragma unroll
      for (int i = 0; i < (kCandSeg / NT); ++i) {
        const int k = k0 + i;
        const int g = dec ? k - r : k;
        const bool valid = k < n && (!dec || s0 + g >= 0);
        const int32_t B = valid ? static_cast<int32_t>(Pseg[g + 1 + w] - Pseg[g + 1]) : 0;
        if (dec && ++r == w) r = 0;
        const bool a = valid && static_cast<long long>(B) > T;
        if (in_pre) {
          if (a) {
            if (pre_len == 0 || B > pre_max) {
              pre_max = B;
              pre_arg = k;
            }
            ++pre_len;
          } else {
            in_pre = false;
          }
        } else if (a) {
          if (!open || B > best) {
            best = B;
            arg = k;
          }
          open = true;
        } else if (open) {
          emit_cand(o, s0 + arg, best, w, s_scale[wi]);  // run inside this thread's range
          open = false;
        }
      }
      t_full[tid] = in_pre ? 1 : 0;
      t_prelen[tid] = pre_len;
      t_premax[tid] = pre_max;
      t_prearg[tid] = pre_arg;
      t_suf[tid] = open ? 1 : 0;
      __syncthreads();
      // ---- owners: a run whose first start lies in this thread's range.  A thread can own
      // two runs: one at its first start (or, for thread 0, the run carried over from the
      // previous segment) and its trailing fragment; at most one of them reaches its last
      // start, and only that one walks on through the following threads' summaries.
      bool walk = false;
      int32_t rb = 0;
      int64_t ra = 0;
      if (pre_len > 0) {
        const bool prev_above =
            tid == 0 ? (c_open[cin][wi] != 0) : (t_full[tid - 1] || t_suf[tid - 1]);
        bool own = false;
        if (!prev_above) {
          own = true;
          rb = pre_max;
          ra = s0 + pre_arg;
        } else if (tid == 0) {          // continue the run carried from the last segment
          own = true;
          rb = c_best[cin][wi];
          ra = c_arg[cin][wi];
          if (pre_max > rb) {
            rb = pre_max;
            ra = s0 + pre_arg;
          }
        }
        if (own) {
          if (in_pre)
            walk = true;                // covers the whole range: continues past it
          else
            emit_cand(o, ra, rb, w, s_scale[wi]);
        }
      } else if (tid == 0 && c_open[cin][wi]) {
        // the carried run ended exactly at the segment boundary
        emit_cand(o, c_arg[cin][wi], c_best[cin][wi], w, s_scale[wi]);
      }
      if (open) {                       // trailing fragment begun after a gap
        walk = true;
        rb = best;
        ra = s0 + arg;
      }
      if (walk) {
        bool closed = false;
        for (int u = tid + 1; !closed && u < NT; ++u) {
          if (t_prelen[u] > 0 && t_premax[u] > rb) {
            rb = t_premax[u];
            ra = s0 + t_prearg[u];
          }
          if (!t_full[u]) closed = true;
        }
        if (closed) {
          emit_cand(o, ra, rb, w, s_scale[wi]);
        } else {                        // open at the segment's end: carry it
          c_open[cin ^ 1][wi] = 1;
          c_best[cin ^ 1][wi] = rb;
          c_arg[cin ^ 1][wi] = ra;
        }
      }
      __syncthreads();
    }
    cin ^= 1;
  }
  if (tid < nw && c_open[cin][tid]) emit_cand(o, c_arg[cin][tid], c_best[cin][tid], s_wid[tid],
                                              s_scale[tid]);
}

// Pre-pass of the candidate search, one wave per row and no workgroup barrier: the row is read
// once, in chunks of kPreC samples (lane l loads samples 4l .. 4l + 3 of a chunk with one
// 16-byte load, issued one chunk ahead), for the exact moments over its nrep searched starts
// and the inclusive prefix S[i] = x[0] + ... + x[i] (mod 2^32), which goes into a ring of RB
// entries in LDS.  Starts are evaluated D = ceil(wmax / kPreC) chunks behind the newest
// prefix, B_w(t) = S[t + w - 1] - S[t - 1] (S[-1] = 0 in the ring's last slot), and the
// whole-row maximum of B_w per width is kept in registers.  Lane l evaluates starts l, l + 64,
// l + 128 and l + 192 of a chunk, so that one address per width serves all four (immediate
// offsets) and the reads are free of bank conflicts.  A read range that passes the ring's end
// continues into a guard of kPreC entries that mirrors the ring's first chunk slot (written
// together with it), so no read address is wrapped.  A row is flagged if some width's maximum
// exceeds its threshold (the same moments and width_params as the main kernel, so the main
// kernel finds no candidate in a row left unflagged).
//
// Widths w = 2v whose half v is also a width are not evaluated: the series is non-negative, so
// B_2v(t) = B_v(t) + B_v(t + v) <= 2 max B_v over starts up to nrep + v, and the row is
// flagged when that bound exceeds w's threshold.  v's maximum is then taken over those starts
// too.  Both only ever flag more rows (the main kernel decides exactly); on noise the bound
// stays below threshold unless B_v reaches thr / sqrt(2) sigma above its mean.  NW is the count
// of evaluated widths; the ring holds D + 2 chunks.
constexpr int kPreC = 256;
constexpr int kPreMaxW = 6 * kPreC;

struct PreWidths {
  int32_t w[kCandRegW];    // evaluated widths
  int32_t ext[kCandRegW];  // starts evaluated beyond the searched ones: v where v bounds 2v
  int32_t nb;              // widths checked through the bound
  int32_t bw[kCandRegW];   // those widths
  int32_t bs[kCandRegW];   // the slot in w of their half
};

// Inclusive prefix sum across a wave64 with DPP moves (no LDS round trip): shifts by 1, 2, 4
// and 8 lanes within each row of 16, then row 0's total to row 1 and row 2's to row 3
// (row_bcast:15), then row 1's to rows 2 and 3 (row_bcast:31).  Lanes without a source add 0.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
  const int x = static_cast<int>(v);
  int s = x;
  s += __builtin_amdgcn_update_dpp(0, s, 0x111, 0xf, 0xf, false);  // row_shr:1
  s += __builtin_amdgcn_update_dpp(0, s, 0x112, 0xf, 0xf, false);  // row_shr:2
  s += __builtin_amdgcn_update_dpp(0, s, 0x114, 0xf, 0xf, false);  // row_shr:4
  s += __builtin_amdgcn_update_dpp(0, s, 0x118, 0xf, 0xf, false);  // row_shr:8
  s += __builtin_amdgcn_update_dpp(0, s, 0x142, 0xa, 0xf, false);  // row_bcast:15
  s += __builtin_amdgcn_update_dpp(0, s, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return static_cast<uint32_t>(s);
}

// samples c0 + 4 lane + u (u < 4) of a row of lw samples, 0 beyond it
__device__ __forceinline__ void pre_load4(const int32_t* x, int64_t c0, int64_t lw, int lane,
                                          int32_t* v) {
  const int64_t i = c0 + 4 * lane;
  if (c0 + kPreC <= lw) {
    int4 q;
    __builtin_memcpy(&q, x + i, sizeof(q));
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = i + u < lw ? x[i + u] : 0;
  }
}

template <int NW, int RB>
__global__ __launch_bounds__(256) void cand_pre_kernel(
    const int32_t* __restrict__ series, int64_t pitch, int64_t nrep, int64_t nrows,
    PreWidths wd, int32_t wmax, double thr, uint8_t* __restrict__ flags) {
  static_assert(NW <= kCandRegW && RB % kPreC == 0 && (RB & (RB - 1)) == 0, "pre-pass shape");
  __shared__ uint32_t ring[4][RB + kPreC];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + wv;
  if (row >= nrows) return;  // the whole wave: nothing below synchronises across waves
  uint32_t* rg = ring[wv];
  const int32_t* x = series + row * pitch;
  const int64_t lw = nrep + wmax - 1;  // samples the searched starts reach
  int32_t bm[NW];
#pragma unroll
  for (int wi = 0; wi < NW; ++wi) bm[wi] = INT_MIN;
  if (lane == 0) rg[RB - 1] = 0u;  // S[-1]
  long long s1 = 0, s2 = 0;
  uint32_t carry = 0;
  const int64_t D = (wmax + kPreC - 1) / kPreC;
  const int64_t nchunk = (lw + kPreC - 1) / kPreC;
  int32_t nx[4];
  pre_load4(x, 0, lw, lane, nx);
  for (int64_t k = 0; k < nchunk + D; ++k) {
    if (k < nchunk) {
      const int64_t c0 = k * kPreC;
      int32_t cx[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cx[u] = nx[u];
      if (k + 1 < nchunk) pre_load4(x, c0 + kPreC, lw, lane, nx);
      if (c0 + kPreC <= nrep) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          s1 += cx[u];
          s2 += static_cast<long long>(cx[u]) * cx[u];
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (c0 + 4 * lane + u < nrep) {
            s1 += cx[u];
            s2 += static_cast<long long>(cx[u]) * cx[u];
          }
      }
      const uint32_t q0 = static_cast<uint32_t>(cx[0]), q1 = q0 + static_cast<uint32_t>(cx[1]),
                     q2 = q1 + static_cast<uint32_t>(cx[2]), q3 = q2 + static_cast<uint32_t>(cx[3]);
      const uint32_t inc = wave_scan_incl(q3);  // inclusive scan of the lanes' totals
      const uint32_t base = carry + inc - q3;
      uint4 wq;
      wq.x = base + q0;
      wq.y = base + q1;
      wq.z = base + q2;
      wq.w = base + q3;
      const int slot = static_cast<int>(c0 & (RB - 1));
      *reinterpret_cast<uint4*>(rg + slot + 4 * lane) = wq;
      if (slot == 0) *reinterpret_cast<uint4*>(rg + RB + 4 * lane) = wq;  // the guard
      carry += static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(inc), 63));
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS writes are done
      __builtin_amdgcn_wave_barrier();
    }
    const int64_t kk = k - D;
    if (kk >= 0) {
      const int64_t t0 = kk * kPreC;
      const uint32_t* pa = rg + ((t0 - 1) & (RB - 1)) + lane;
      uint32_t av[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) av[u] = pa[64 * u];
      if (t0 + kPreC <= nrep) {
#pragma unroll
        for (int wi = 0; wi < NW; ++wi) {
          const uint32_t* pw = rg + ((t0 + wd.w[wi] - 1) & (RB - 1)) + lane;
#pragma unroll
          for (int u = 0; u < 4; ++u)
            bm[wi] = max(bm[wi], static_cast<int32_t>(pw[64 * u] - av[u]));
        }
      } else {
#pragma unroll
        for (int wi = 0; wi < NW; ++wi) {
          const uint32_t* pw = rg + ((t0 + wd.w[wi] - 1) & (RB - 1)) + lane;
          const int64_t lim = nrep + wd.ext[wi];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (t0 + lane + 64 * u < lim)
              bm[wi] = max(bm[wi], static_cast<int32_t>(pw[64 * u] - av[u]));
        }
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_xor(s1, off, 64);
    s2 += __shfl_xor(s2, off, 64);
#pragma unroll
    for (int wi = 0; wi < NW; ++wi) bm[wi] = max(bm[wi], __shfl_xor(bm[wi], off, 64));
  }
  if (lane == 0) {
    double mu, sigma;
    row_musig(s1, s2, nrep, &mu, &sigma);
    int hit = 0;
    if (sigma > 0.0)
#pragma unroll
      for (int wi = 0; wi < NW; ++wi) {
        const long long m = bm[wi];
        if (m > width_params(wd.w[wi], nrep, mu, sigma, thr).thr_int) hit = 1;
        for (int b = 0; b < wd.nb; ++b)
          if (wd.bs[b] == wi && 2 * m > width_params(wd.bw[b], nrep, mu, sigma, thr).thr_int)
            hit = 1;
      }
    flags[row] = static_cast<uint8_t>(hit);
  }
}

typedef void (*PreKernel)(const int32_t*, int64_t, int64_t, int64_t, PreWidths, int32_t, double,
                          uint8_t*);

template <int RB, int N = 1>
PreKernel pre_kernel_nw(int nw) {
  if constexpr (N < kCandRegW)
    if (nw > N) return pre_kernel_nw<RB, N + 1>(nw);
  return cand_pre_kernel<N, RB>;
}

int launch_candidates(const arts_plan_s* p, const int32_t* series, int32_t nbeam, int64_t L,
                      int64_t nrep, float thr, int64_t t_offset, int32_t beam_offset,
                      const int64_t*, const double*, arts_candidate* cand,
                      unsigned long long* count, int64_t cap, hipStream_t s, int64_t t_begin,
                      uint8_t* flags) {
  if (t_begin < 0 || t_begin >= nrep) return fail(ARTS_E_INVAL, "t_begin outside [0, nrep)");
  const int64_t nrows = static_cast<int64_t>(nbeam) * p->ndm;
  if (nrows > INT_MAX) return fail(ARTS_E_INVAL, "candidate grid too large");
  if (p->nwidth > kMaxWidthsCand) return fail(ARTS_E_INVAL, "at most %d widths", kMaxWidthsCand);
  static bool attr = false;
  if (!attr) {
    ARTS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&candidates_kernel<false, 256>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (kCandSeg + 2 * kMaxWidth) * 4));
    ARTS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&candidates_kernel<false, 512>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (kCandSeg + 2 * kMaxWidth) * 4));
    ARTS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&candidates_kernel<true, 256>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kCandResLds));
    ARTS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&candidates_kernel<true, 512>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, kCandResLds));
    attr = true;
  }
  // resident rows: P[0 .. n] and one spare word, n = searched starts + wmax - 1
  const size_t res_lds = (static_cast<size_t>(nrep - t_begin) + p->wmax + 1) * sizeof(uint32_t);
  const bool res = res_lds <= static_cast<size_t>(kCandResLds);
  // segments of longer rows: kCandSeg starts plus wmax samples (and wmax - 1 before them for
  // decimated integration)
  const size_t lds = res ? res_lds
                         : (kCandSeg + p->wmax + 1 + (p->integration ? p->wmax - 1 : 0)) *
                               sizeof(uint32_t);
  (void)hipGetLastError();
  const bool wide = nrep - t_begin >= kCandLong;
  const int nt = wide ? 512 : 256;
  auto kern = res ? (wide ? candidates_kernel<true, 512> : candidates_kernel<true, 256>)
                  : (wide ? candidates_kernel<false, 512> : candidates_kernel<false, 256>);
  // rows that cannot hold a candidate are sorted out first when the pre-pass applies
  const bool pre = flags != nullptr && p->nwidth <= kCandRegW && p->wmax <= kPreMaxW &&
                   nrows >= 1024;
  if (pre) {
    // evaluated widths in ascending order; 2v is bounded through v when v is evaluated
    PreWidths wd{};
    std::vector<int32_t> ws(p->widths.begin(), p->widths.end());
    std::sort(ws.begin(), ws.end());
    ws.erase(std::unique(ws.begin(), ws.end()), ws.end());
    int nw = 0;
    for (const int32_t w : ws) {
      int half = -1;
      for (int j = 0; j < nw && w % 2 == 0; ++j)
        if (wd.w[j] == w / 2 && wd.ext[j] == 0) half = j;
      if (half >= 0) {
        wd.ext[half] = w / 2;
        wd.bw[wd.nb] = w;
        wd.bs[wd.nb] = half;
        ++wd.nb;
      } else {
        wd.w[nw++] = w;
      }
    }
    // the ring holds D + 2 chunks: 4 of them up to wmax = 2 kPreC, else 8
    const PreKernel kp = p->wmax <= 2 * kPreC ? pre_kernel_nw<4 * kPreC>(nw)
                                              : pre_kernel_nw<8 * kPreC>(nw);
    hipLaunchKernelGGL(kp, dim3(static_cast<unsigned>((nrows + 3) / 4)), dim3(256), 0, s,
                       series + t_begin, L, nrep - t_begin, nrows, wd, p->wmax,
                       static_cast<double>(thr), flags);
  }
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(nrows)), dim3(nt), lds, s,
                     series + t_begin, L, L - t_begin, nrep - t_begin, p->ndm, p->d_widths,
                     p->nwidth, p->wmax, p->d_dms, static_cast<double>(thr),
                     t_offset + t_begin, beam_offset, p->ds, cand, count, cap,
                     pre ? flags : nullptr, p->integration);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

// Pseudo-random bytes (a counter hash, SplitMix64's finaliser) for the autotuner's inputs.
__global__ __launch_bounds__(256) void fill_random_kernel(uint8_t* p, int64_t n, uint64_t seed) {
  const int64_t i0 = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 8;
  if (i0 >= n) return;
  uint64_t z = seed + static_cast<uint64_t>(i0) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  for (int k = 0; k < 8 && i0 + k < n; ++k) p[i0 + k] = static_cast<uint8_t>(z >> (8 * k));
}

int launch_fill_random(uint8_t* p, int64_t n, uint64_t seed, hipStream_t s) {
  if (n <= 0) return ARTS_OK;
  const int64_t blocks = (n + 2047) / 2048;
  (void)hipGetLastError();
  hipLaunchKernelGGL(fill_random_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p,
                     n, seed);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ULL;
}

int launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(zero_u64_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

// ------------------------------------------------------------------ SB gather ----
// sb_out[s][c][:] = tab[sb_table[s][c]][c][:].  Rows start at arbitrary byte offsets, so each
// thread writes whole destination-aligned dwords; the matching source bytes are funnel-shifted
// out of two aligned source dwords.  Destination dwords shared with a neighbouring row (at row
// ends) are written bytewise so rows never race.  A block covers kGatherThreads * kGatherDw
// consecutive dwords of a row, the threads of each pass taking consecutive dwords (coalesced).
constexpr int kGatherThreads = 256;
constexpr int kGatherDw = 4;  // dwords per thread

__global__ __launch_bounds__(kGatherThreads) void sb_gather_kernel(
    const uint8_t* __restrict__ tab, int32_t ntab, const uint8_t* __restrict__ table,
    int32_t nchan, int64_t nsamp, uint8_t* __restrict__ out, int64_t nchunk,
    const uint8_t* tab_end) {
  const uint8_t* tab_begin = tab;
  const int64_t row = blockIdx.x / nchunk;
  const int64_t chunk = blockIdx.x % nchunk;
  const int64_t c = row % nchan;
  const int src_beam = table[row];
  uint8_t* drow = out + row * nsamp;
  const uint8_t* srow = src_beam < ntab ? tab + (static_cast<int64_t>(src_beam) * nchan + c) * nsamp : nullptr;
  const uintptr_t dalign = reinterpret_cast<uintptr_t>(drow) & ~static_cast<uintptr_t>(3);
  const int64_t lead = reinterpret_cast<uintptr_t>(drow) - dalign;  // bytes before the row
  const int64_t ndw = (lead + nsamp + 3) / 4;
  const int64_t k0 = chunk * kGatherThreads * kGatherDw + threadIdx.x;
  for (int i = 0; i < kGatherDw; ++i) {
    const int64_t k = k0 + static_cast<int64_t>(i) * kGatherThreads;
    if (k >= ndw) break;
    const int64_t off = 4 * k - lead;  // row offset of the dword's first byte
    uint8_t* dq = reinterpret_cast<uint8_t*>(dalign) + 4 * k;
    if (off >= 0 && off + 4 <= nsamp) {
      uint32_t v = 0;
      if (srow) {
        const uint8_t* sq = srow + off;
        const uintptr_t sa = reinterpret_cast<uintptr_t>(sq);
        const int h = static_cast<int>(sa & 3u);
        const uint32_t* sp = reinterpret_cast<const uint32_t*>(sa - h);
        if (h == 0) {
          v = sp[0];
        } else if (reinterpret_cast<const uint8_t*>(sp) >= tab_begin &&
                   reinterpret_cast<const uint8_t*>(sp + 2) <= tab_end) {
          v = __builtin_amdgcn_alignbyte(sp[1], sp[0], h);
        } else {
          for (int j = 0; j < 4; ++j) v |= static_cast<uint32_t>(sq[j]) << (8 * j);
        }
      }
      *reinterpret_cast<uint32_t*>(dq) = v;
    } else {
      for (int j = 0; j < 4; ++j) {
        const int64_t o = off + j;
        if (o >= 0 && o < nsamp) drow[o] = srow ? srow[o] : 0;
      }
    }
  }
}

int launch_sb_gather(const uint8_t* tab, int32_t ntab, const uint8_t* sb_table, int32_t nsb,
                     int32_t nchan, int64_t nsamp, uint8_t* out, hipStream_t s) {
  const int64_t per_block = static_cast<int64_t>(kGatherThreads) * kGatherDw * 4;
  const int64_t nchunk = (nsamp + 3 + per_block) / per_block;
  const int64_t rows = static_cast<int64_t>(nsb) * nchan;
  if (rows * nchunk > INT_MAX) return fail(ARTS_E_INVAL, "gather grid too large");
  const uint8_t* tab_end = tab + static_cast<int64_t>(ntab) * nchan * nsamp;
  (void)hipGetLastError();
  hipLaunchKernelGGL(sb_gather_kernel, dim3(static_cast<unsigned>(rows * nchunk)),
                     dim3(kGatherThreads), 0, s, tab, ntab, sb_table, nchan, nsamp, out, nchunk,
                     tab_end);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

// ------------------------------------------------------------------ row copy ----
// Copies byte rows at arbitrary alignment: each thread writes destination-aligned dwords whose
// source bytes are funnel-shifted out of two aligned source dwords; dwords a row shares with
// its neighbour are written bytewise so rows never race.  Blocks and passes as in
// sb_gather_kernel.
__global__ __launch_bounds__(kGatherThreads) void copy_rows_kernel(
    uint8_t* __restrict__ dst, int64_t dpitch, const uint8_t* __restrict__ src, int64_t spitch,
    int64_t n, int64_t nchunk, const uint8_t* src_begin, const uint8_t* src_end) {
  const int64_t row = blockIdx.x / nchunk;
  const int64_t chunk = blockIdx.x % nchunk;
  uint8_t* drow = dst + row * dpitch;
  const uint8_t* srow = src + row * spitch;
  const uintptr_t dalign = reinterpret_cast<uintptr_t>(drow) & ~static_cast<uintptr_t>(3);
  const int64_t lead = reinterpret_cast<uintptr_t>(drow) - dalign;
  const int64_t ndw = (lead + n + 3) / 4;
  const int64_t k0 = chunk * kGatherThreads * kGatherDw + threadIdx.x;
  for (int i = 0; i < kGatherDw; ++i) {
    const int64_t k = k0 + static_cast<int64_t>(i) * kGatherThreads;
    if (k >= ndw) break;
    const int64_t off = 4 * k - lead;
    uint8_t* dq = reinterpret_cast<uint8_t*>(dalign) + 4 * k;
    if (off >= 0 && off + 4 <= n) {
      const uint8_t* sq = srow + off;
      const uintptr_t sa = reinterpret_cast<uintptr_t>(sq);
      const int h = static_cast<int>(sa & 3u);
      const uint32_t* sp = reinterpret_cast<const uint32_t*>(sa - h);
      uint32_t v = 0;
      if (h == 0) {
        v = sp[0];
      } else if (reinterpret_cast<const uint8_t*>(sp) >= src_begin &&
                 reinterpret_cast<const uint8_t*>(sp + 2) <= src_end) {
        v = __builtin_amdgcn_alignbyte(sp[1], sp[0], h);
      } else {
        for (int j = 0; j < 4; ++j) v |= static_cast<uint32_t>(sq[j]) << (8 * j);
      }
      *reinterpret_cast<uint32_t*>(dq) = v;
    } else {
      for (int j = 0; j < 4; ++j) {
        const int64_t o = off + j;
        if (o >= 0 && o < n) drow[o] = srow[o];
      }
    }
  }
}

// Rows whose starts have the same offset within a V word and whose pitches are whole words:
// the first `head` bytes of a row (up to the first word boundary) and the last `tail` bytes
// are copied bytewise by the row's first and last block, the nv words between them one V per
// thread and pass, consecutive threads on consecutive words (kGatherDw passes per block).
template <typename V>
__global__ __launch_bounds__(kGatherThreads) void copy_rows_vec_kernel(
    uint8_t* __restrict__ dst, int64_t dpitch, const uint8_t* __restrict__ src, int64_t spitch,
    int head, int64_t nv, int tail, int64_t nchunk) {
  const int64_t row = blockIdx.x / nchunk;
  const int64_t chunk = blockIdx.x % nchunk;
  uint8_t* drow = dst + row * dpitch;
  const uint8_t* srow = src + row * spitch;
  if (chunk == 0 && static_cast<int>(threadIdx.x) < head) drow[threadIdx.x] = srow[threadIdx.x];
  if (chunk == nchunk - 1 && static_cast<int>(threadIdx.x) < tail) {
    const int64_t o = head + nv * static_cast<int64_t>(sizeof(V)) + threadIdx.x;
    drow[o] = srow[o];
  }
  V* dv = reinterpret_cast<V*>(drow + head);
  const V* sv = reinterpret_cast<const V*>(srow + head);
  const int64_t k0 = chunk * kGatherThreads * kGatherDw + threadIdx.x;
#pragma unroll
  for (int i = 0; i < kGatherDw; ++i) {
    const int64_t k = k0 + static_cast<int64_t>(i) * kGatherThreads;
    if (k < nv) dv[k] = sv[k];
  }
}

template <typename V>
static int launch_copy_rows_vec(uint8_t* dst, int64_t dpitch, const uint8_t* src,
                                int64_t spitch, int64_t nrows, int64_t n, hipStream_t s) {
  constexpr int64_t w = sizeof(V);
  const int head = static_cast<int>(
      std::min<int64_t>(n, (w - static_cast<int64_t>(reinterpret_cast<uintptr_t>(dst) % w)) % w));
  const int64_t nv = (n - head) / w;
  const int tail = static_cast<int>(n - head - nv * w);
  const int64_t per_block = static_cast<int64_t>(kGatherThreads) * kGatherDw;
  const int64_t nchunk = std::max<int64_t>(1, (nv + per_block - 1) / per_block);
  if (nrows * nchunk > INT_MAX) return fail(ARTS_E_INVAL, "copy grid too large");
  (void)hipGetLastError();
  hipLaunchKernelGGL(copy_rows_vec_kernel<V>, dim3(static_cast<unsigned>(nrows * nchunk)),
                     dim3(kGatherThreads), 0, s, dst, dpitch, src, spitch, head, nv, tail,
                     nchunk);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

int launch_copy_rows(uint8_t* dst, int64_t dpitch, const uint8_t* src, int64_t spitch,
                     int64_t nrows, int64_t n, const uint8_t* src_begin, const uint8_t* src_end,
                     hipStream_t s) {
  if (nrows <= 0 || n <= 0) return ARTS_OK;
  // both starts at the same offset within a 16- or 8-byte word and whole-word pitches: words
  // between a bytewise head and tail
  const uint64_t al = (reinterpret_cast<uintptr_t>(dst) ^ reinterpret_cast<uintptr_t>(src)) |
                      static_cast<uint64_t>(dpitch) | static_cast<uint64_t>(spitch);
  if (n >= 64 && (al & 15u) == 0)
    return launch_copy_rows_vec<uint4>(dst, dpitch, src, spitch, nrows, n, s);
  if (n >= 64 && (al & 7u) == 0)
    return launch_copy_rows_vec<uint2>(dst, dpitch, src, spitch, nrows, n, s);
  const int64_t per_block = static_cast<int64_t>(kGatherThreads) * kGatherDw * 4;
  const int64_t nchunk = (n + 3 + per_block) / per_block;
  if (nrows * nchunk > INT_MAX) return fail(ARTS_E_INVAL, "copy grid too large");
  (void)hipGetLastError();
  hipLaunchKernelGGL(copy_rows_kernel, dim3(static_cast<unsigned>(nrows * nchunk)),
                     dim3(kGatherThreads), 0, s, dst, dpitch, src, spitch, n, nchunk, src_begin,
                     src_end);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

// ------------------------------------------------------------------ downsampling ----
// dst[r][s] = sum_{i<D} src[r][D s + i] for s < nout (16-bit: D <= 257).  Each thread makes
// 4 consecutive outputs; rows whose start is 4-byte aligned are read with dword loads.  For
// D = 4 an output is the byte sum of one dword (v_sad_u8 against zero), read 16 bytes at a time
// where the row allows, and the four outputs are stored as one 8-byte word where aligned.
__global__ __launch_bounds__(256) void downsample_rows_kernel(
    uint16_t* __restrict__ dst, int64_t dpitch, const uint8_t* __restrict__ src, int64_t spitch,
    int64_t nout, int32_t D, int64_t nblk_row) {
  const int64_t row = blockIdx.x / nblk_row;
  const int64_t s0 = ((blockIdx.x % nblk_row) * 256 + threadIdx.x) * 4;
  if (s0 >= nout) return;
  const uint8_t* sr = src + row * spitch;
  uint16_t* dr = dst + row * dpitch;
  const int nv = static_cast<int>(min<int64_t>(4, nout - s0));
  uint32_t acc[4] = {0, 0, 0, 0};
  const uint8_t* q = sr + s0 * D;
  if (D == 4 && nv == 4 && (reinterpret_cast<uintptr_t>(q) & 3u) == 0) {
    uint4 w;
    if ((reinterpret_cast<uintptr_t>(q) & 15u) == 0) {
      w = *reinterpret_cast<const uint4*>(q);
    } else {
      const uint32_t* qw = reinterpret_cast<const uint32_t*>(q);
      w = make_uint4(qw[0], qw[1], qw[2], qw[3]);
    }
    acc[0] = __builtin_amdgcn_sad_u8(w.x, 0u, 0u);
    acc[1] = __builtin_amdgcn_sad_u8(w.y, 0u, 0u);
    acc[2] = __builtin_amdgcn_sad_u8(w.z, 0u, 0u);
    acc[3] = __builtin_amdgcn_sad_u8(w.w, 0u, 0u);
    if ((reinterpret_cast<uintptr_t>(dr + s0) & 7u) == 0) {
      *reinterpret_cast<uint2*>(dr + s0) =
          make_uint2(acc[0] | (acc[1] << 16), acc[2] | (acc[3] << 16));
      return;
    }
  } else if ((reinterpret_cast<uintptr_t>(q) & 3u) == 0 && nv == 4) {
    const uint32_t* qw = reinterpret_cast<const uint32_t*>(q);
    for (int j = 0; j < D; ++j) {  // 4 D bytes = D dwords
      const uint32_t w = qw[j];
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[(4 * j + b) / D] += (w >> (8 * b)) & 0xffu;
    }
  } else {
    for (int i = 0; i < nv; ++i)
      for (int j = 0; j < D; ++j) acc[i] += q[i * D + j];
  }
  for (int i = 0; i < nv; ++i) dr[s0 + i] = static_cast<uint16_t>(acc[i]);
}

int launch_downsample(uint16_t* dst, int64_t dpitch, const uint8_t* src, int64_t spitch,
                      int64_t nrows, int64_t nout, int32_t D, hipStream_t s) {
  if (nrows <= 0 || nout <= 0) return ARTS_OK;
  const int64_t nblk_row = (nout + 1023) / 1024;
  if (nrows * nblk_row > INT_MAX) return fail(ARTS_E_INVAL, "downsample grid too large");
  (void)hipGetLastError();
  hipLaunchKernelGGL(downsample_rows_kernel, dim3(static_cast<unsigned>(nrows * nblk_row)),
                     dim3(256), 0, s, dst, dpitch, src, spitch, nout, D, nblk_row);
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

}  // namespace arts

// RFI mitigation of filterbank chunks on the GPU, in place (Sect. 6b.2 "RFI mitigation": a
// filter for bright wide-band low-DM RFI and one for narrow-band RFI; three iterations of each,
// every one on the data the previous one cleaned; local statistics).
//
// Time domain, per source row [nchan][nsamp]: the zero-DM series z(t) = sum_c x[c][t]; samples
// with z(t) > floor(mean + k sigma) (population statistics of z over the chunk) are replaced in
// every channel by that channel's mean over the other samples, rounded half to even.  One dense
// pass gives z and the channel sums S_c; an iteration then touches only the flagged samples:
// the cut comes from the statistics of z, the means from S_c minus the flagged columns, and after
// the replacement S_c and z(t) are updated exactly.
//
// Frequency domain, per spectrum (one source row, one sample): channels with
// x[c] > floor(mean + k sigma) over the spectrum are replaced by the mean of the other channels,
// rounded half to even.  Both cuts are exact (integer tests; FP64 only for the first guess).  A workgroup stages a tile of [nchan][64] samples in LDS, runs every
// iteration there and writes the tile back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "arts_internal.h"

namespace arts {

namespace {

constexpr int kRfiThreads = 256;
constexpr int kRfiTile = 32;          // spectra per frequency-domain workgroup
constexpr int kRfiMaxChan = 4096;     // LDS tile of kRfiMaxChan x kRfiTile bytes

__device__ __forceinline__ uint32_t rhe_div(int64_t s, int64_t n) {
  const int64_t q = s / n, r = s - q * n;
  return static_cast<uint32_t>(q + ((2 * r > n || (2 * r == n && (q & 1))) ? 1 : 0));
}

// A threshold k in standard deviations, exactly k = m / 2^s (s >= 0), and as FP64.
struct KExact {
  double kd;
  uint32_t m;
  int32_t s;
};

// floor(mean + k sigma) of n values with exact sums s1, s2, exactly: an integer u lies above
// mean + k sigma when D = n u - s1 > 0 and D^2 > k^2 (n s2 - s1^2), i.e. D^2 > T with
// T = floor(m^2 (n s2 - s1^2) / 4^s) in 128-bit integers.  The FP64 value (mean-shifted sums)
// is the starting guess; it is off by at most one.
__device__ int64_t cut_of(int64_t s1, int64_t s2, int64_t n, KExact k) {
  const int64_t m0 = s1 / n, r = s1 - n * m0;
  const int64_t s2c = s2 - 2 * m0 * s1 + n * m0 * m0;  // sum of (x - m0)^2
  const double dn = static_cast<double>(n);
  const double var =
      (static_cast<double>(s2c) - static_cast<double>(r) * static_cast<double>(r) / dn) / dn;
  const double mu = static_cast<double>(m0) + static_cast<double>(r) / dn;
  int64_t c = static_cast<int64_t>(floor(mu + k.kd * sqrt(var > 0.0 ? var : 0.0)));
  using u128 = unsigned __int128;
  const u128 V = static_cast<u128>(n) * static_cast<u128>(s2) -
                 static_cast<u128>(s1) * static_cast<u128>(s1);
  const u128 T = (static_cast<u128>(k.m) * k.m * V) >> (2 * k.s);
  const auto above = [&](int64_t u) {
    const int64_t d = n * u - s1;
    return d > 0 && static_cast<u128>(d) * static_cast<u128>(d) > T;
  };
  for (int i = 0; i < 64 && above(c); ++i) --c;
  for (int i = 0; i < 64 && !above(c + 1); ++i) ++c;
  return c;
}

__device__ __forceinline__ int64_t block_sum64(int64_t v, int64_t* red) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int64_t t = 0;
  for (int i = 0; i < static_cast<int>(blockDim.x) / 64; ++i) t += red[i];
  return t;
}

struct RfiRow {  // per source row state of the time-domain filter
  int32_t nflag;
  int32_t done;
  int64_t msum;  // sum over channels of the replacement values of this iteration
};

// z[r][t] = sum_c x[r][c][t]: lanes on consecutive samples, channels in a loop.
__global__ __launch_bounds__(kRfiThreads) void rfi_zero_dm_kernel(
    const uint8_t* __restrict__ x, int64_t pitch, int32_t nchan, int64_t nsamp, int64_t ntile,
    int32_t* __restrict__ z) {
  const int64_t r = blockIdx.x / ntile;
  const int64_t t = (blockIdx.x % ntile) * kRfiThreads + threadIdx.x;
  if (t >= nsamp) return;
  const uint8_t* p = x + r * nchan * pitch + t;
  int32_t s = 0;
  for (int c = 0; c < nchan; ++c) s += p[static_cast<int64_t>(c) * pitch];
  z[r * nsamp + t] = s;
}

// The same with dword loads (rows 4-byte aligned): wave w of 4 sums channels c = w (mod 4) for
// 256 consecutive samples (one dword per lane), the waves' partial sums meet in LDS.  Samples at
// or beyond nsamp inside the last dword are not stored.
__global__ __launch_bounds__(kRfiThreads) void rfi_zero_dm4_kernel(
    const uint8_t* __restrict__ x, int64_t pitch, int32_t nchan, int64_t nsamp, int64_t ntile,
    int32_t* __restrict__ z) {
  __shared__ int32_t part[4][64][4];
  const int64_t r = blockIdx.x / ntile;
  const int64_t j = (blockIdx.x % ntile) * 64 + (threadIdx.x & 63);  // dword index in the row
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t ndw = (nsamp + 3) / 4;
  int32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  if (j < ndw) {
    const uint32_t* p = reinterpret_cast<const uint32_t*>(x + r * nchan * pitch) + j;
    const int64_t pw = pitch / 4;
    int c = w;
    for (; c + 12 < nchan; c += 16) {  // four loads in flight
      const uint32_t v0 = p[c * pw], v1 = p[(c + 4) * pw], v2 = p[(c + 8) * pw],
                     v3 = p[(c + 12) * pw];
      a0 += (v0 & 255u) + (v1 & 255u) + (v2 & 255u) + (v3 & 255u);
      a1 += ((v0 >> 8) & 255u) + ((v1 >> 8) & 255u) + ((v2 >> 8) & 255u) + ((v3 >> 8) & 255u);
      a2 += ((v0 >> 16) & 255u) + ((v1 >> 16) & 255u) + ((v2 >> 16) & 255u) +
            ((v3 >> 16) & 255u);
      a3 += (v0 >> 24) + (v1 >> 24) + (v2 >> 24) + (v3 >> 24);
    }
    for (; c < nchan; c += 4) {
      const uint32_t v = p[c * pw];
      a0 += v & 255u;
      a1 += (v >> 8) & 255u;
      a2 += (v >> 16) & 255u;
      a3 += v >> 24;
    }
  }
  part[w][lane][0] = a0;
  part[w][lane][1] = a1;
  part[w][lane][2] = a2;
  part[w][lane][3] = a3;
  __syncthreads();
  if (w == 0 && j < ndw) {
    for (int b = 0; b < 4; ++b) {
      const int64_t t = 4 * j + b;
      if (t < nsamp)
        z[r * nsamp + t] = part[0][lane][b] + part[1][lane][b] + part[2][lane][b] +
                           part[3][lane][b];
    }
  }
}

// S[r][c] = sum_t x[r][c][t]: one wave per channel row.
__global__ __launch_bounds__(kRfiThreads) void rfi_chan_sum_kernel(
    const uint8_t* __restrict__ x, int64_t pitch, int64_t nrows, int64_t nsamp,
    int64_t* __restrict__ S) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (kRfiThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nrows) return;
  const uint8_t* p = x + row * pitch;
  int64_t s = 0;
  int64_t t0 = 0;
  if (((reinterpret_cast<uintptr_t>(x) | static_cast<uintptr_t>(pitch)) & 3u) == 0) {
    const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
    const int64_t nfull = nsamp / 4;
    // v_sad_u8 against 0: the sum of a dword's four bytes
    for (int64_t j = lane; j < nfull; j += 64) s += __builtin_amdgcn_sad_u8(q[j], 0u, 0u);
    t0 = 4 * nfull;
  }
  for (int64_t t = t0 + lane; t < nsamp; t += 64) s += p[t];
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
  if (lane == 0) S[row] = s;
}

__global__ void rfi_rows_init_kernel(RfiRow* rows, int32_t nrow) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrow) {
    rows[r].nflag = 0;
    rows[r].done = 0;
    rows[r].msum = 0;
  }
}

// One workgroup per source row: the cut of z and the list of samples above it.
__global__ __launch_bounds__(kRfiThreads) void rfi_time_flag_kernel(
    const int32_t* __restrict__ z, int64_t nsamp, KExact k, RfiRow* rows,
    int32_t* __restrict__ flags) {
  __shared__ int64_t red[kRfiThreads / 64];
  __shared__ int32_t s_n;
  const int64_t r = blockIdx.x;
  if (rows[r].done) return;
  const int32_t* zr = z + r * nsamp;
  int64_t s1 = 0, s2 = 0;
  for (int64_t t = threadIdx.x; t < nsamp; t += kRfiThreads) {
    const int64_t v = zr[t];
    s1 += v;
    s2 += v * v;
  }
  s1 = block_sum64(s1, red);
  s2 = block_sum64(s2, red);
  const int64_t cut = cut_of(s1, s2, nsamp, k);
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  int32_t* fr = flags + r * nsamp;
  for (int64_t t = threadIdx.x; t < nsamp; t += kRfiThreads)
    if (zr[t] > cut) fr[atomicAdd(&s_n, 1)] = static_cast<int32_t>(t);
  __syncthreads();
  if (threadIdx.x == 0) {
    rows[r].nflag = s_n;
    rows[r].msum = 0;
    if (s_n == 0) rows[r].done = 1;
  }
}

// One thread per (row, channel): the channel's mean over the unflagged samples, from its sum
// minus the flagged columns; the sum is updated for the replacement.
__global__ __launch_bounds__(kRfiThreads) void rfi_time_mean_kernel(
    const uint8_t* __restrict__ x, int64_t pitch, int32_t nchan, int64_t nsamp, int32_t nrow,
    RfiRow* rows, const int32_t* __restrict__ flags, int64_t* __restrict__ S,
    uint32_t* __restrict__ mean) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kRfiThreads + threadIdx.x;
  if (i >= static_cast<int64_t>(nrow) * nchan) return;
  const int64_t r = i / nchan;
  if (rows[r].done) return;
  const int32_t nf = rows[r].nflag;
  const uint8_t* p = x + i * pitch;
  const int32_t* fr = flags + r * nsamp;
  int64_t g = 0;
  for (int32_t j = 0; j < nf; ++j) g += p[fr[j]];
  const int64_t good = S[i] - g;
  const uint32_t m = rhe_div(good, nsamp - nf);
  mean[i] = m;
  S[i] = good + static_cast<int64_t>(nf) * m;
  atomicAdd(reinterpret_cast<unsigned long long*>(&rows[r].msum),
            static_cast<unsigned long long>(m));
}

// Replace the flagged samples: x[r][c][t] = mean[r][c]; z[r][t] = the sum of the means.
__global__ __launch_bounds__(kRfiThreads) void rfi_time_replace_kernel(
    uint8_t* __restrict__ x, int64_t pitch, int32_t nchan, int64_t nsamp, const RfiRow* rows,
    const int32_t* __restrict__ flags, const uint32_t* __restrict__ mean,
    int32_t* __restrict__ z) {
  const int64_t r = blockIdx.y;
  if (rows[r].done) return;
  const int32_t nf = rows[r].nflag;
  const int32_t* fr = flags + r * nsamp;
  const uint32_t* mr = mean + r * nchan;
  uint8_t* xr = x + r * nchan * pitch;
  for (int32_t j = blockIdx.x; j < nf; j += gridDim.x) {
    const int64_t t = fr[j];
    for (int c = threadIdx.x; c < nchan; c += kRfiThreads)
      xr[static_cast<int64_t>(c) * pitch + t] = static_cast<uint8_t>(mr[c]);
    if (threadIdx.x == 0) z[r * nsamp + t] = static_cast<int32_t>(rows[r].msum);
  }
}

// Frequency domain: workgroup = (row, 32 consecutive samples).  Lane l of wave w works on
// spectrum g = l mod 32 and channel phase p = l / 32 + 2 w: channels c = p (mod 8); the eight
// phases of a spectrum meet in LDS.  A tile of [nchan][32] bytes (48 KB at 1536 channels: three
// workgroups per CU) is staged once; with 4-byte aligned rows it moves by dword loads and stores
// (8 lanes per 32-byte channel segment, no dword past the row's last whole dword inside its
// pitch), and a tile in which nothing was replaced is not written back.
__global__ __launch_bounds__(kRfiThreads) void rfi_freq_kernel(
    uint8_t* __restrict__ x, int64_t pitch, int32_t nchan, int64_t nsamp, int64_t ntile,
    KExact k, int32_t niter) {
  constexpr int P = kRfiThreads / kRfiTile;  // channel phases per spectrum
  extern __shared__ uint8_t tile[];          // [nchan][kRfiTile]
  __shared__ int32_t r1[P][kRfiTile], r2[P][kRfiTile];
  __shared__ int s_changed;
  const int64_t r = blockIdx.x / ntile;
  const int64_t t0 = (blockIdx.x % ntile) * kRfiTile;
  const int tid = threadIdx.x;
  const int g = tid & (kRfiTile - 1);
  const int ph = tid / kRfiTile;
  const int nt = static_cast<int>(std::min<int64_t>(kRfiTile, nsamp - t0));
  uint8_t* xr = x + r * nchan * pitch + t0;
  const bool dw = ((reinterpret_cast<uintptr_t>(x) | static_cast<uintptr_t>(pitch)) & 3u) == 0;
  constexpr int kDw = kRfiTile / 4;          // dwords per channel segment
  if (tid == 0) s_changed = 0;
  if (dw) {
    const int kq = tid % kDw;
    const bool ok = t0 + 4 * kq + 4 <= pitch;
    constexpr int kStep = kRfiThreads / kDw, kUnroll = 8;  // eight loads in flight per thread
    for (int c0 = tid / kDw; c0 < nchan; c0 += kStep * kUnroll) {
      uint32_t v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int c = c0 + u * kStep;
        v[u] = ok && c < nchan
                   ? *reinterpret_cast<const uint32_t*>(xr + static_cast<int64_t>(c) * pitch +
                                                        4 * kq)
                   : 0u;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int c = c0 + u * kStep;
        if (c < nchan) *reinterpret_cast<uint32_t*>(tile + c * kRfiTile + 4 * kq) = v[u];
      }
    }
  } else {
    for (int c = ph; c < nchan; c += P)
      tile[c * kRfiTile + g] = g < nt ? xr[static_cast<int64_t>(c) * pitch + g] : 0;
  }
  __syncthreads();
  bool done = g >= nt;  // the same for the eight phases of a spectrum
  for (int it = 0; it < niter; ++it) {
    int32_t s1 = 0, s2 = 0;  // a phase's share: <= 512 channels of 255^2
    if (!done)
      for (int c = ph; c < nchan; c += P) {
        const int32_t v = tile[c * kRfiTile + g];
        s1 += v;
        s2 += v * v;
      }
    r1[ph][g] = s1;
    r2[ph][g] = s2;
    __syncthreads();
    int64_t S1 = 0, S2 = 0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      S1 += r1[q][g];
      S2 += r2[q][g];
    }
    const int64_t cut = done ? 0 : cut_of(S1, S2, nchan, k);
    int32_t gs = 0, gn = 0;
    if (!done)
      for (int c = ph; c < nchan; c += P) {
        const int32_t v = tile[c * kRfiTile + g];
        if (v <= cut) {
          gs += v;
          ++gn;
        }
      }
    __syncthreads();
    r1[ph][g] = gs;
    r2[ph][g] = gn;
    __syncthreads();
    int64_t GS = 0, GN = 0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      GS += r1[q][g];
      GN += r2[q][g];
    }
    if (!done && GN < nchan) {
      const uint8_t m = static_cast<uint8_t>(rhe_div(GS, GN));
      for (int c = ph; c < nchan; c += P)
        if (tile[c * kRfiTile + g] > cut) tile[c * kRfiTile + g] = m;
      if (ph == 0) s_changed = 1;
    } else {
      done = true;
    }
    __syncthreads();
  }
  if (!s_changed) return;
  if (dw) {
    const int kq = tid % kDw;
    const int b0 = 4 * kq;
    for (int c = tid / kDw; c < nchan; c += kRfiThreads / kDw) {
      uint8_t* gp = xr + static_cast<int64_t>(c) * pitch + b0;
      const uint8_t* l = tile + c * kRfiTile + b0;
      if (b0 + 4 <= nt) {
        *reinterpret_cast<uint32_t*>(gp) = *reinterpret_cast<const uint32_t*>(l);
      } else {
        for (int b = 0; b < 4 && b0 + b < nt; ++b) gp[b] = l[b];
      }
    }
  } else {
    for (int c = ph; c < nchan; c += P)
      if (g < nt) xr[static_cast<int64_t>(c) * pitch + g] = tile[c * kRfiTile + g];
  }
}

}  // namespace

// k = m / 2^s exactly for a float k in {0} or [2^-6, 2^10] (a 24-bit mantissa).
static bool exact_k(float k, KExact* out) {
  out->kd = static_cast<double>(k);
  out->m = 0;
  out->s = 0;
  if (k == 0.0f) return true;
  if (!(k >= 0.015625f && k <= 1024.0f)) return false;
  int e = 0;
  const double f = std::frexp(static_cast<double>(k), &e);  // k = f 2^e, f in [0.5, 1)
  uint32_t m = static_cast<uint32_t>(std::ldexp(f, 24));
  int s = 24 - e;
  while (s > 0 && (m & 1u) == 0) {
    m >>= 1;
    --s;
  }
  out->m = m;
  out->s = s;
  return true;
}

int64_t rfi_ws_bytes(int32_t nrow, int32_t nchan, int64_t nsamp) {
  const auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t rc = static_cast<int64_t>(nrow) * nchan, rs = static_cast<int64_t>(nrow) * nsamp;
  return up(rs * 4) * 2 + up(rc * 8) + up(rc * 4) + up(static_cast<int64_t>(nrow) * 16);
}

int launch_rfi(uint8_t* x, int32_t nrow, int32_t nchan, int64_t nsamp, int64_t pitch,
               float k_time, int32_t niter_time, float k_freq, int32_t niter_freq, void* ws,
               hipStream_t s) {
  if (nrow < 1 || nchan < 1 || nsamp < 1 || pitch < nsamp)
    return fail(ARTS_E_INVAL, "RFI: nrow, nchan, nsamp >= 1 and pitch >= nsamp");
  if (niter_time < 0 || niter_freq < 0) return fail(ARTS_E_INVAL, "RFI: negative iterations");
  KExact kt, kf;
  if (!exact_k(k_time, &kt) || !exact_k(k_freq, &kf))
    return fail(ARTS_E_INVAL, "RFI: thresholds must be 0 or within [2^-6, 1024]");
  // exact cuts in 128-bit integers need nsamp * nchan * 255 < 2^40
  if (nsamp >= INT_MAX || static_cast<int64_t>(nchan) * 255 * 255 >= INT_MAX ||
      nsamp * static_cast<int64_t>(nchan) > (1LL << 32))
    return fail(ARTS_E_INVAL, "RFI: chunk too large");
  if (niter_freq > 0 && nchan > kRfiMaxChan)
    return fail(ARTS_E_INVAL, "RFI: at most %d channels for the frequency-domain filter",
                kRfiMaxChan);
  const auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t rc = static_cast<int64_t>(nrow) * nchan, rs = static_cast<int64_t>(nrow) * nsamp;
  uint8_t* p = static_cast<uint8_t*>(ws);
  int32_t* z = reinterpret_cast<int32_t*>(p);
  int32_t* flags = reinterpret_cast<int32_t*>(p + up(rs * 4));
  int64_t* S = reinterpret_cast<int64_t*>(p + 2 * up(rs * 4));
  uint32_t* mean = reinterpret_cast<uint32_t*>(p + 2 * up(rs * 4) + up(rc * 8));
  RfiRow* rows = reinterpret_cast<RfiRow*>(p + 2 * up(rs * 4) + up(rc * 8) + up(rc * 4));
  (void)hipGetLastError();
  if (niter_time > 0) {
    const int64_t ntile = (nsamp + kRfiThreads - 1) / kRfiThreads;
    if (nrow * ntile > INT_MAX) return fail(ARTS_E_INVAL, "RFI: grid too large");
    hipLaunchKernelGGL(rfi_rows_init_kernel, dim3((nrow + 63) / 64), dim3(64), 0, s, rows, nrow);
    if (((reinterpret_cast<uintptr_t>(x) | static_cast<uintptr_t>(pitch)) & 3u) == 0) {
      const int64_t nt4 = ((nsamp + 3) / 4 + 63) / 64;  // 256 samples per workgroup
      hipLaunchKernelGGL(rfi_zero_dm4_kernel, dim3(static_cast<unsigned>(nrow * nt4)),
                         dim3(kRfiThreads), 0, s, x, pitch, nchan, nsamp, nt4, z);
    } else {
      hipLaunchKernelGGL(rfi_zero_dm_kernel, dim3(static_cast<unsigned>(nrow * ntile)),
                         dim3(kRfiThreads), 0, s, x, pitch, nchan, nsamp, ntile, z);
    }
    hipLaunchKernelGGL(rfi_chan_sum_kernel, dim3(static_cast<unsigned>((rc + 3) / 4)),
                       dim3(kRfiThreads), 0, s, x, pitch, rc, nsamp, S);
    for (int it = 0; it < niter_time; ++it) {
      hipLaunchKernelGGL(rfi_time_flag_kernel, dim3(nrow), dim3(kRfiThreads), 0, s, z, nsamp,
                         kt, rows, flags);
      hipLaunchKernelGGL(rfi_time_mean_kernel,
                         dim3(static_cast<unsigned>((rc + kRfiThreads - 1) / kRfiThreads)),
                         dim3(kRfiThreads), 0, s, x, pitch, nchan, nsamp, nrow, rows, flags, S,
                         mean);
      hipLaunchKernelGGL(rfi_time_replace_kernel, dim3(64, nrow), dim3(kRfiThreads), 0, s, x,
                         pitch, nchan, nsamp, rows, flags, mean, z);
    }
  }
  if (niter_freq > 0) {
    static bool attr = false;
    if (!attr) {
      ARTS_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&rfi_freq_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   kRfiMaxChan * kRfiTile));
      attr = true;
    }
    const int64_t ntile = (nsamp + kRfiTile - 1) / kRfiTile;
    if (nrow * ntile > INT_MAX) return fail(ARTS_E_INVAL, "RFI: grid too large");
    hipLaunchKernelGGL(rfi_freq_kernel, dim3(static_cast<unsigned>(nrow * ntile)),
                       dim3(kRfiThreads), static_cast<size_t>(nchan) * kRfiTile, s, x, pitch,
                       nchan, nsamp, ntile, kf, niter_freq);
  }
  ARTS_HIP(hipGetLastError());
  return ARTS_OK;
}

}  // namespace arts

"""Seeded synthetic inputs for the ARTS search: quantised Stokes-I noise, injected bursts, the
synthetic SB table and the workload configurations.

This module holds no search arithmetic (no delay law, no dedispersion, no S/N): where a burst
must follow a dispersion sweep, the caller passes the per-channel sample offsets.  It is the
only code shared between the oracle-side tests and the GPU-side tests and benchmark.

Stokes-I data are uint8, channel-major with time fastest (the TABF re-orders its output so the
time index changes fastest; TABs are requantised to 8 bit with clipping, Appendix on data loads
and requantisation).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TSAMP = 81.92e-6          # s, native Stokes-I sample time (Sect. 4d)
BAND_LO, BAND_HI = 1220.0, 1520.0   # MHz, 300 MHz band
CHUNK = 12500             # new samples per 1.024 s chunk


def band(nchan: int, lo: float = BAND_LO, hi: float = BAND_HI):
    """(f_lo, df) for nchan channel centres evenly spanning [lo, hi] MHz, ascending."""
    df = (hi - lo) / nchan
    return lo + df / 2.0, df


def _noise_lut(mean: float, sigma: float) -> np.ndarray:
    """uint8 value for each of 65536 equiprobable uniform codes: clip(rint(mean + sigma*z))
    with z the normal quantile at the code's centre, i.e. quantised N(mean, sigma) noise."""
    k = (np.arange(65536, dtype=np.float64) + 0.5) / 65536.0
    z = np.sqrt(2.0) * _erfinv(2.0 * k - 1.0)
    return np.clip(np.rint(mean + sigma * z), 0, 255).astype(np.uint8)


def _erfinv(y: np.ndarray) -> np.ndarray:
    from scipy.special import erfinv
    return erfinv(y)


def _codes_to_float(codes: np.ndarray, mean: float, sigma: float) -> np.ndarray:
    k = (codes.astype(np.float64) + 0.5) / 65536.0
    return mean + sigma * np.sqrt(2.0) * _erfinv(2.0 * k - 1.0)


@dataclass
class Burst:
    """A dispersed burst: per-channel arrival sample offsets (from the caller's delay law),
    its profile width in samples and amplitude in counts per channel."""
    arrival: np.ndarray          # int64 [nchan], absolute sample index of the burst per channel
    width: float                 # FWHM (gaussian) or exact width (tophat), samples
    amplitude: float             # counts per channel
    kind: str = "gaussian"


def noise(shape, seed: int, mean: float = 128.0, sigma: float = 16.0, bursts=(),
          return_codes: bool = False):
    """Quantised N(mean, sigma) noise of the given shape (last axis = time), uint8.

    Gaussian bursts are added in floating point before rounding, so sub-count amplitudes are
    dithered by the noise.  For multi-row shapes, each burst applies to rows [..., c, :] with
    channel c = the second-to-last index, on every leading index (use shape [nchan][nsamp] to
    target one beam)."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    codes = rng.integers(0, 65536, size=shape, dtype=np.uint16)
    out = _noise_lut(mean, sigma)[codes]
    for b in bursts:
        if b.kind != "gaussian":
            raise ValueError("noise() takes gaussian bursts; use add_tophat for exact ones")
        nsamp = shape[-1]
        half = int(math.ceil(3.0 * b.width)) + 1
        for c, a in enumerate(np.asarray(b.arrival, dtype=np.int64)):
            lo, hi = max(0, a - half), min(nsamp, a + half + 1)
            if lo >= hi:
                continue
            t = np.arange(lo, hi, dtype=np.float64)
            prof = b.amplitude * np.exp(-4.0 * math.log(2.0) * ((t - a) / b.width) ** 2)
            sl = (Ellipsis, c, slice(lo, hi))
            x = _codes_to_float(codes[sl], mean, sigma) + prof
            out[sl] = np.clip(np.rint(x), 0, 255).astype(np.uint8)
    return (out, codes) if return_codes else out


def add_tophat(data: np.ndarray, arrival, width: int, amplitude: int) -> np.ndarray:
    """Add an integer top-hat of `width` samples and `amplitude` counts to channel c starting at
    arrival[c] (data [nchan][nsamp] uint8, in place), clipping at 255.  Returns the int64 array
    of what was actually added, so a test can account for clipping exactly."""
    added = np.zeros(data.shape, dtype=np.int64)
    for c, a in enumerate(np.asarray(arrival, dtype=np.int64)):
        lo, hi = max(0, a), min(data.shape[-1], a + width)
        if lo >= hi:
            continue
        old = data[c, lo:hi].astype(np.int64)
        new = np.minimum(old + amplitude, 255)
        data[c, lo:hi] = new.astype(np.uint8)
        added[c, lo:hi] = new - old
    return added


def sb_table_synthetic(nsb: int = 71, ntab: int = 12, nchan: int = 1536) -> np.ndarray:
    """Synthetic SB table: channel c of SB s takes TAB (s + floor(6 c (s - centre) / nchan))
    mod ntab, centre = nsb // 2, in exact integer arithmetic (floor toward -inf, non-negative
    mod).  The centre SB takes one TAB across the band; the edge SBs switch TAB most often."""
    centre = nsb // 2
    s = np.arange(nsb, dtype=np.int64)[:, None]
    c = np.arange(nchan, dtype=np.int64)[None, :]
    return np.mod(s + np.floor_divide(6 * c * (s - centre), nchan), ntab).astype(np.uint8)


@dataclass
class Workload:
    """Shape and search parameters of one synthetic search request."""
    name: str
    nchan: int
    f_lo: float
    df: float
    tsamp: float
    dms: np.ndarray
    widths: list
    nbeam: int = 1
    downsample: int = 1
    threshold: float = 8.0
    sigma: float = 16.0
    seed: int = 0
    extra: dict = field(default_factory=dict)


def cfg_small(seed: int = 1) -> Workload:
    """1 beam, 128 channels over 1220-1520 MHz, 256 trials DM 0..127.5 step 0.5, widths
    1..16, 16384 samples, threshold 8."""
    f_lo, df = band(128)
    return Workload("small-128ch-256dm", 128, f_lo, df, TSAMP,
                    np.arange(256, dtype=np.float64) * 0.5, [1, 2, 4, 8, 16],
                    seed=seed, extra={"nsamp": 16384})


def cfg_apertif(seed: int = 2) -> Workload:
    """1 beam, Apertif shape: 1536 channels, 2048 trials DM 0..2047, widths 1..256."""
    f_lo, df = band(1536)
    return Workload("apertif-1536ch-2048dm", 1536, f_lo, df, TSAMP,
                    np.arange(2048, dtype=np.float64), [1 << k for k in range(9)], seed=seed)


def cfg_apertif_ds(seed: int = 5) -> Workload:
    """High-DM, time-downsampled trials of the serving stream: D = 4, DM 2048..4998 step 2
    (1476 trials), widths 1..64 downsampled samples (4..256 native)."""
    f_lo, df = band(1536)
    return Workload("apertif-1536ch-ds4-1476dm", 1536, f_lo, df, TSAMP,
                    np.arange(2048, 5000, 2, dtype=np.float64), [1 << k for k in range(7)],
                    downsample=4, seed=seed)


def uneven_requests(n: int = 64, seed: int = 4):
    """Uneven batch: nchan in {384, 768, 1536}, 0.5-4 s long, DM ranges 0-500 / 0-2000 /
    0-5000 with 512-4096 linearly spaced trials, noise sigma in [8, 24]."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        nchan = int(rng.choice([384, 768, 1536]))
        f_lo, df = band(nchan)
        nsamp = int(round(float(rng.uniform(0.5, 4.0)) / TSAMP))
        dm_hi = float(rng.choice([500.0, 2000.0, 5000.0]))
        ntrial = int(rng.integers(512, 4097))
        sigma = float(rng.uniform(8.0, 24.0))
        w = Workload(f"req{i}", nchan, f_lo, df, TSAMP, np.linspace(0.0, dm_hi, ntrial),
                     [1 << k for k in range(9)], sigma=sigma, seed=1000 + i,
                     extra={"nsamp": nsamp})
        reqs.append(w)
    return reqs


def random_bursts(delays: np.ndarray, nrep: int, seed: int, n: int = 20, dm_range=(50, 2000),
                  dms=None, snr_range=(8.0, 40.0), width_range=(1.0, 256.0), sigma=16.0,
                  margin: int = 600):
    """n gaussian bursts on trial DMs drawn uniformly in dm_range (dms: the trial DM values),
    start times uniform over the reported window, log-uniform FWHM, and per-channel amplitude
    chosen for a target S/N of A * sqrt(w * nchan) / sigma.  delays: the caller's delay table
    [ndm][nchan] (the arrival sweep).  Returns (bursts, meta) with meta = (dm_index, t0, fwhm,
    target_snr)."""
    rng = np.random.default_rng(seed)
    nchan = delays.shape[1]
    dms = np.arange(delays.shape[0], dtype=np.float64) if dms is None else np.asarray(dms)
    lo = int(np.searchsorted(dms, dm_range[0]))
    hi = int(np.searchsorted(dms, dm_range[1], side="right")) - 1
    bursts, meta = [], []
    for _ in range(n):
        d = int(rng.integers(lo, hi + 1))
        t0 = int(rng.integers(margin, max(margin + 1, nrep - margin)))
        fwhm = float(np.exp(rng.uniform(np.log(width_range[0]), np.log(width_range[1]))))
        target = float(rng.uniform(*snr_range))
        amp = target * sigma / math.sqrt(max(fwhm, 1.0) * nchan)
        bursts.append(Burst(t0 + delays[d].astype(np.int64), fwhm, amp))
        meta.append((d, t0, fwhm, target))
    return bursts, meta


def candidate_tracks(nbeam: int, ndm: int, widths, nsamp: int, ntrack: int, nnoise: int,
                     seed: int, halfspan: int = 40):
    """Synthetic candidate list shaped like a search's output around bright events, for the
    clustering path.  Each track is one event in one beam, seen at DM trials d0 - h .. d0 + h
    (h drawn up to `halfspan`) and at every width, with a start sample that drifts linearly
    with the DM offset (a trial DM away from the true one shifts the arrival) and an S/N that
    falls off away from the track's centre DM and width; `nnoise` isolated candidates are
    spread uniformly over beams, DM trials, widths and samples with S/N just above 8.
    Returns int64 columns (beam, dm_index, width, sample) and float32 snr, with every
    (beam, dm_index, width, sample) distinct, in random order."""
    rng = np.random.default_rng(seed)
    widths = np.asarray(list(widths), dtype=np.int64)
    cols = [[], [], [], [], []]
    for _ in range(ntrack):
        b = int(rng.integers(nbeam))
        d0 = int(rng.integers(ndm))
        h = int(rng.integers(1, halfspan + 1))
        t0 = int(rng.integers(0, nsamp))
        drift = float(rng.uniform(-3.0, 3.0))
        wc = int(rng.integers(widths.size))
        peak = float(rng.uniform(10.0, 60.0))
        d = np.arange(max(0, d0 - h), min(ndm, d0 + h + 1), dtype=np.int64)
        for k, w in enumerate(widths):
            t = t0 + np.rint(drift * (d - d0)).astype(np.int64) - w // 2
            s = peak / (1.0 + np.abs(d - d0) / 4.0) / (1.0 + abs(k - wc) * 0.3)
            cols[0].append(np.full(d.size, b))
            cols[1].append(d)
            cols[2].append(np.full(d.size, w))
            cols[3].append(t)
            cols[4].append(s)
    cols[0].append(rng.integers(0, nbeam, nnoise))
    cols[1].append(rng.integers(0, ndm, nnoise))
    cols[2].append(rng.choice(widths, nnoise))
    cols[3].append(rng.integers(0, nsamp, nnoise))
    cols[4].append(rng.uniform(8.0, 9.0, nnoise))
    b, d, w, t = (np.concatenate(c).astype(np.int64) for c in cols[:4])
    s = np.concatenate(cols[4]).astype(np.float32)
    key = ((b * ndm + d) * (widths.max() + 1) + w) * (4 * nsamp + 1) + (t + 2 * nsamp)
    _, first = np.unique(key, return_index=True)
    order = rng.permutation(first)
    return b[order], d[order], w[order], t[order], s[order]

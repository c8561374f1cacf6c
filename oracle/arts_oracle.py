"""Plain CPU oracle for the ARTS single-pulse search (van Leeuwen et al., "The Apertif Radio
Transient System", arXiv:2205.12362).

TEST INFRASTRUCTURE ONLY -- imported by tests/, __graft_entry__.smoke() and the cpu_baseline
leg of bench.py, never by the product path.  Nothing here is tuned: every step is the direct
definition, in int64 for integer data and FP64 for real numbers.

The paper names the search stages (Sect. 6b.2 "AMBER": downsampling, dedispersion, integration,
S/N evaluation, candidate selection) but does not write out the dispersion law, the boxcar, the
S/N estimator or the candidate rule.  The readings taken here are listed per function and in the
design notes of the repository; each is marked "reading".

Parity status per function:
  channel_freqs, delay_table, tie_audit, downsample, sb_synthesize, dedisperse,
  dedisperse_at, subband_plan, subband_dedisperse, subband_dedisperse_at, boxcar, moments,
  snr, candidates, candidates_integrated, cluster_dm_width, cluster_offline,
  rfi_time_domain, rfi_freq_domain, rfi_clean, sb_index_at_fmax, sb_switch_freqs,
  sb_table_beam_model -- pinned by closed forms / invariants / hand-worked values / brute
  force in tests/test_oracle_pins.py (no function here is "parity unpinned").
"""
from __future__ import annotations

import numpy as np

# Cold-plasma dispersion constant, s MHz^2 pc^-1 cm^3.  Reading: the paper does not state the
# delay law; the standard one, t(f) = K_DM * DM / f^2 with f in MHz, is used.
K_DM = 4.148808e3


def channel_freqs(nchan: int, f_lo_mhz: float, df_mhz: float) -> np.ndarray:
    """Centre frequency of channel c: f_lo + c * df (MHz, FP64).

    The Stokes-I beams have 1536 channels over 300 MHz at 81.92 us (Sect. 4d, dedicated TABF
    output).  Reading: channels are equally spaced, c = 0 at f_lo, index increasing with df.
    """
    if nchan < 1:
        raise ValueError("nchan must be >= 1")
    return f_lo_mhz + np.arange(nchan, dtype=np.float64) * df_mhz


def delay_table(nchan, f_lo_mhz, df_mhz, tsamp_s, dms, downsample=1, return_exact=False):
    """Per-trial, per-channel dispersion delay in (downsampled) samples, int64 [ndm][nchan].

    Dedispersion shifts every channel by the delay of a trial DM (Sect. 6b.2, "Dedispersion").
    Reading: x = K_DM * DM * (1/f_c^2 - 1/f_ref^2) / (D * tsamp) with f_ref the highest channel
    frequency, so every delay is >= 0; delay = x rounded half-to-even (numpy.rint).
    With return_exact the unrounded FP64 x is returned as well.
    """
    if tsamp_s <= 0 or downsample < 1:
        raise ValueError("tsamp must be > 0 and downsample >= 1")
    f = channel_freqs(nchan, f_lo_mhz, df_mhz)
    dms = np.asarray(dms, dtype=np.float64)
    if dms.ndim != 1 or not np.all(np.isfinite(dms)) or np.any(dms < 0):
        raise ValueError("DMs must be a 1-D array of finite values >= 0")
    f_ref = f.max()
    inv = 1.0 / (f * f) - 1.0 / (f_ref * f_ref)
    x = K_DM * dms[:, None] * inv[None, :] / (downsample * tsamp_s)
    d = np.rint(x).astype(np.int64)
    return (d, x) if return_exact else d


def tie_audit(x_exact: np.ndarray) -> float:
    """Smallest distance of any unrounded delay from a rounding tie (k + 0.5).

    A delay table is only well defined if no x sits on a tie within floating-point noise; this
    returns min |frac(x) - 0.5| so a caller can check it against the FP64 evaluation error.
    """
    if x_exact.size == 0:
        return float("inf")
    return float(np.min(np.abs((x_exact - np.floor(x_exact)) - 0.5)))


def downsample(data: np.ndarray, factor: int) -> np.ndarray:
    """Lower the time resolution by summing `factor` consecutive samples (Sect. 6b.2,
    "Downsampling").  Reading: a sum, not a mean, so integers stay exact; trailing samples that
    do not fill a group are dropped.  data [..., nsamp] -> int64 [..., nsamp // factor]."""
    if factor < 1:
        raise ValueError("factor must be >= 1")
    a = np.asarray(data).astype(np.int64)
    n = a.shape[-1] // factor
    return a[..., : n * factor].reshape(a.shape[:-1] + (n, factor)).sum(axis=-1)


def sb_synthesize(tab: np.ndarray, sb_table: np.ndarray) -> np.ndarray:
    """Form synthesized beams from tied-array beams: SB[s][c][t] = TAB[sb_table[s][c]][c][t].

    Each SB takes, per frequency channel, the data of the TAB whose grating response points at
    the SB's sky position at that frequency (Sect. 3d.beam; Appendix "Synthesized Beams").
    tab [ntab][nchan][nsamp], sb_table [nsb][nchan] -> [nsb][nchan][nsamp] (same dtype)."""
    tab = np.asarray(tab)
    sb_table = np.asarray(sb_table)
    ntab, nchan, _ = tab.shape
    if sb_table.ndim != 2 or sb_table.shape[1] != nchan:
        raise ValueError("sb_table must be [nsb][nchan]")
    if sb_table.size and (sb_table.min() < 0 or sb_table.max() >= ntab):
        raise ValueError("sb_table entry out of range")
    out = np.empty((sb_table.shape[0], nchan, tab.shape[2]), dtype=tab.dtype)
    for s in range(sb_table.shape[0]):
        for c in range(nchan):
            out[s, c, :] = tab[sb_table[s, c], c, :]
    return out


def dedisperse(data: np.ndarray, delays: np.ndarray) -> np.ndarray:
    """Brute-force incoherent dedispersion: X[d][t] = sum_c I[c][t + delay[d][c]] (int64).

    The brute-force approach of Sect. 6b.2 ("Dedispersion"), single step.  The output length is
    the same for every trial: nout = nsamp - max(delay) over the whole table, so every output
    sample sees every channel.  data [nchan][nsamp] (any integer dtype), delays [ndm][nchan]."""
    data = np.asarray(data).astype(np.int64)
    delays = np.asarray(delays).astype(np.int64)
    nchan, nsamp = data.shape
    if delays.shape[1] != nchan:
        raise ValueError("delay table channel count does not match the data")
    dmax = int(delays.max()) if delays.size else 0
    nout = nsamp - dmax
    if nout <= 0:
        raise ValueError("input shorter than the largest delay")
    out = np.zeros((delays.shape[0], nout), dtype=np.int64)
    for d in range(delays.shape[0]):
        for c in range(nchan):
            s = delays[d, c]
            out[d] += data[c, s : s + nout]
    return out


def dedisperse_at(data: np.ndarray, delays: np.ndarray, d: int, t: int) -> int:
    """One dedispersed sample X[d][t] = sum_c I[c][t + delay[d][c]], for spot checks at sizes
    where the full table is too slow (same definition as `dedisperse`)."""
    cs = np.arange(data.shape[0])
    return int(np.asarray(data)[cs, t + np.asarray(delays)[d]].astype(np.int64).sum())


def subband_plan(nchan, f_lo_mhz, df_mhz, tsamp_s, dm_first, dm_step, ndm, nfine, nsub):
    """Delay tables of two-step subband dedispersion (Sect. 6b.2 "Dedispersion", the subband
    dedispersion figure, Table "dedispersion setup": 32 subbands of 48 channels, a coarse
    subbanding DM step, 32 fine trials per coarse step).

    The band is cut into nsub subbands of nchan / nsub consecutive channels.  Step 1 shifts each
    channel of a subband by its delay at a coarse DM relative to the subband's own reference
    frequency; step 2 shifts each subband as a whole by the delay of that reference frequency at
    the fine DM, relative to the band's reference.
    Readings: the fine trials are dm_first + k dm_step, k < ndm; trial k belongs to coarse group
    j = k // nfine, whose coarse DM is the group's centre dm_first + (j nfine + (nfine-1)/2)
    dm_step; a subband's reference frequency is its highest channel (so both delays are >= 0);
    both steps use the dispersion law and rounding of delay_table.
    Returns (fine_dms [ndm], coarse_dms [ncoarse], d1 int64 [ncoarse][nchan],
    d2 int64 [ndm][nsub]).
    """
    if nsub < 1 or nchan % nsub != 0:
        raise ValueError("nsub must divide nchan")
    if nfine < 1 or ndm < 1 or not dm_step > 0 or dm_first < 0:
        raise ValueError("need nfine >= 1, ndm >= 1, dm_step > 0, dm_first >= 0")
    csub = nchan // nsub
    ncoarse = (ndm + nfine - 1) // nfine
    fine = dm_first + dm_step * np.arange(ndm, dtype=np.float64)
    coarse = dm_first + dm_step * (np.arange(ncoarse, dtype=np.float64) * nfine
                                   + (nfine - 1) / 2.0)
    d1 = np.concatenate([delay_table(csub, f_lo_mhz + s * csub * df_mhz, df_mhz, tsamp_s, coarse)
                         for s in range(nsub)], axis=1)
    # subband reference frequencies: the highest channel of each subband, spaced csub * df
    top = csub - 1 if df_mhz > 0 else 0
    d2 = delay_table(nsub, f_lo_mhz + top * df_mhz, csub * df_mhz, tsamp_s, fine)
    return fine, coarse, d1, d2


def subband_dedisperse(data: np.ndarray, d1: np.ndarray, d2: np.ndarray, nfine: int):
    """Two-step subband dedispersion of one beam, int64 [ndm][n2] (tables from subband_plan).

    Step 1: Y[j][s][t] = sum over the channels c of subband s of I[c][t + d1[j][c]],
            t < n1 = nin - max d1.
    Step 2: X[k][t] = sum over subbands s of Y[k // nfine][s][t + d2[k][s]],
            t < n2 = n1 - max d2.
    Both lengths are rectangular over the whole plan, as for dedisperse.
    """
    x = np.asarray(data).astype(np.int64)
    nchan, nin = x.shape
    ncoarse, nsub = d1.shape[0], d2.shape[1]
    csub = nchan // nsub
    n1 = nin - int(d1.max())
    if n1 <= 0:
        raise ValueError("input shorter than the step-1 delays")
    y = np.zeros((ncoarse, nsub, n1), dtype=np.int64)
    for j in range(ncoarse):
        for c in range(nchan):
            y[j, c // csub] += x[c, d1[j, c]: d1[j, c] + n1]
    n2 = n1 - int(d2.max())
    if n2 <= 0:
        raise ValueError("input shorter than the two steps' delays")
    out = np.zeros((d2.shape[0], n2), dtype=np.int64)
    for k in range(d2.shape[0]):
        for s in range(nsub):
            out[k] += y[k // nfine, s, d2[k, s]: d2[k, s] + n2]
    return out


def subband_dedisperse_at(data: np.ndarray, d1: np.ndarray, d2: np.ndarray, nfine: int,
                          k: int, t: int) -> int:
    """One output X[k][t] of subband_dedisperse: every channel c of subband s contributes
    I[c][t + d2[k][s] + d1[k // nfine][c]] (for sampled checks at full size)."""
    nchan = data.shape[0]
    csub = nchan // d2.shape[1]
    c = np.arange(nchan)
    idx = t + d2[k][c // csub] + d1[k // nfine][c]
    return int(np.asarray(data)[c, idx].astype(np.int64).sum())


def boxcar(series: np.ndarray, width: int, nrep: int) -> np.ndarray:
    """Boxcar matched filter: B_w[..., t] = sum_{j<w} X[..., t + j] for t < nrep (int64).

    Integration convolves each dedispersed series with trial-width kernels so that S/N peaks at
    the pulse width (Sect. 6b.2, "Integration"; offline, a box-car matched filter over many
    widths, Sect. 6b.1).  Reading: sliding (every t), window [t, t + w - 1] indexed by its start."""
    x = np.asarray(series).astype(np.int64)
    if width < 1 or nrep < 0 or nrep + width - 1 > x.shape[-1]:
        raise ValueError("boxcar window runs past the series")
    out = x[..., 0:nrep].copy()
    for j in range(1, width):
        out += x[..., j : j + nrep]
    return out


def moments(series: np.ndarray, nrep: int):
    """Per-series mean and population standard deviation over t < nrep (FP64).

    Reading of the S/N normalisation (Sect. 6b.2, "S/N evaluation" leaves the method open):
    noise statistics of the unsmoothed dedispersed series over the reported window, which is the
    1.024 s chunk the real-time S/N is based on (Sect. 6b.1)."""
    x = np.asarray(series)[..., :nrep].astype(np.float64)
    mu = x.mean(axis=-1)
    sigma = np.sqrt(((x - mu[..., None]) ** 2).mean(axis=-1))
    return mu, sigma


def snr(box: np.ndarray, width: int, mu, sigma) -> np.ndarray:
    """S/N of boxcar sums: (B_w - w * mu) / (sigma * sqrt(w)), FP64; 0 where sigma == 0.

    Reading: white noise, so the standard deviation of a w-sample sum is sigma * sqrt(w)."""
    mu = np.asarray(mu, dtype=np.float64)[..., None]
    sigma = np.asarray(sigma, dtype=np.float64)[..., None]
    b = np.asarray(box).astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = (b - width * mu) / (sigma * np.sqrt(float(width)))
    return np.where(sigma > 0, s, 0.0)


def candidates(series: np.ndarray, widths, nrep: int, threshold: float, beam: int = 0,
               t_offset: int = 0):
    """Threshold candidates of one beam's dedispersed series X [ndm][L].

    Candidates whose S/N exceeds the threshold are kept (Sect. 6b.2, "Candidate selection");
    S/N is evaluated at all peaks ("S/N evaluation").  Reading: for every (DM, width) each
    maximal run of consecutive samples with S/N > threshold (strict) gives one candidate at the
    run's largest boxcar sum, the earliest sample on ties; no clustering across widths or DMs.
    Returns a list of (beam, dm_index, width, t + t_offset, snr) sorted by (beam, dm, width, t).
    """
    x = np.asarray(series).astype(np.int64)
    mu, sigma = moments(x, nrep)
    out = []
    for w in widths:
        b = boxcar(x, w, nrep)
        s = snr(b, w, mu, sigma)
        for d in range(x.shape[0]):
            above = s[d] > threshold
            t = 0
            while t < nrep:
                if not above[t]:
                    t += 1
                    continue
                e = t
                while e < nrep and above[e]:
                    e += 1
                k = t + int(np.argmax(b[d, t:e]))
                out.append((beam, d, int(w), k + t_offset, float(s[d, k])))
                t = e
    out.sort(key=lambda r: (r[0], r[1], r[2], r[3]))
    return out


def candidates_integrated(series: np.ndarray, widths, nrep: int, threshold: float,
                          beam: int = 0, t_offset: int = 0):
    """Threshold candidates with decimated integration (Sect. 6b.2, "Integration": the
    dedispersed series is downsampled by each trial pulse width).

    Reading: for width w the integrated series holds one sample per w consecutive input samples,
    the sum over [g, g + w - 1] for g on the absolute grid g + t_offset = 0 (mod w), so that
    consecutive chunks of a stream share the grid.  Only starts t < nrep on that grid are
    searched; S/N and threshold are those of `candidates` (the noise of a w-sample sum is
    sigma * sqrt(w)); a run is a maximal sequence of consecutive grid starts (g, g + w, ...)
    above the threshold, reported at its largest sum, the earliest on ties.  For w = 1 this is
    `candidates`.  Returns (beam, dm_index, width, g + t_offset, snr) sorted like `candidates`.
    """
    x = np.asarray(series).astype(np.int64)
    mu, sigma = moments(x, nrep)
    out = []
    for w in widths:
        w = int(w)
        b = boxcar(x, w, nrep)
        s = snr(b, w, mu, sigma)
        grid = np.array([t for t in range(nrep) if (t + t_offset) % w == 0], dtype=np.int64)
        for d in range(x.shape[0]):
            above = s[d, grid] > threshold
            i = 0
            while i < len(grid):
                if not above[i]:
                    i += 1
                    continue
                e = i
                while e < len(grid) and above[e]:
                    e += 1
                k = grid[i + int(np.argmax(b[d, grid[i:e]]))]
                out.append((beam, d, w, int(k) + t_offset, float(s[d, k])))
                i = e
    out.sort(key=lambda r: (r[0], r[1], r[2], r[3]))
    return out


def search(data: np.ndarray, delays: np.ndarray, widths, threshold: float, beam: int = 0,
           nrep: int | None = None, t_offset: int = 0):
    """The whole path on one beam: dedisperse, then boxcar / S/N / candidates over the reported
    window nrep (default: every t whose widest boxcar fits).  Returns (X, candidates)."""
    x = dedisperse(data, delays)
    wmax = max(widths)
    if nrep is None:
        nrep = x.shape[1] - wmax + 1
    return x, candidates(x, widths, nrep, threshold, beam=beam, t_offset=t_offset)


def cluster_dm_width(cands):
    """AMBER's optional real-time clustering in the DM-width plane (Sect. 6b.2, "Clustering").

    The paper's two steps, in its order: (1) candidates of different widths at the same time and
    the same DM are grouped and only the highest S/N is kept; (2) groups in neighbouring DM
    trials are compacted, again keeping the highest S/N; one candidate is reported per
    resulting DM-width cluster.

    Readings: a candidate (beam, dm_index, width w, sample t, snr) occupies the boxcar window
    [t, t + w - 1]; "the same time" means overlapping windows, taken transitively, so a step-1
    group is a maximal chain of overlapping windows in one (beam, DM) row and covers the union of
    its windows; "neighbouring DM trials" are dm_index and dm_index + 1 of the same beam, and two
    groups there are compacted when their covered intervals overlap, again transitively.  The
    reported candidate is the member with the highest S/N, ties to the lowest dm_index, then the
    earliest sample, then the smallest width.

    cands: sequence of (beam, dm_index, width, sample, snr).  Returns (reps, label): reps is the
    list of reported candidates sorted by (beam, dm_index, width, sample), label[i] the index in
    reps of input candidate i's cluster.
    """
    n = len(cands)
    for c in cands:
        if int(c[2]) < 1:
            raise ValueError("candidate width must be >= 1")
    # step 1: per (beam, dm) row, in order of (sample, width); a candidate whose window starts
    # after everything the current group covers opens a new group
    rows = {}
    for i, c in enumerate(cands):
        rows.setdefault((int(c[0]), int(c[1])), []).append(i)
    groups = []                      # [beam, dm, first, last, members]
    for key in sorted(rows):
        order = sorted(rows[key], key=lambda i: (int(cands[i][3]), int(cands[i][2])))
        cur = None
        for i in order:
            t0 = int(cands[i][3])
            t1 = t0 + int(cands[i][2]) - 1
            if cur is None or t0 > cur[3]:
                cur = [key[0], key[1], t0, t1, []]
                groups.append(cur)
            cur[3] = max(cur[3], t1)
            cur[4].append(i)
    # step 2: join groups of DM trials d and d + 1 (same beam) whose covered intervals overlap
    parent = list(range(len(groups)))

    def find(a):
        while parent[a] != a:
            a = parent[a]
        return a

    by_row = {}
    for g, grp in enumerate(groups):
        by_row.setdefault((grp[0], grp[1]), []).append(g)
    for g, grp in enumerate(groups):
        for h in by_row.get((grp[0], grp[1] + 1), []):
            other = groups[h]
            if grp[2] <= other[3] and other[2] <= grp[3]:
                ra, rb = find(g), find(h)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
    # report: the best member of every cluster
    members = {}
    for g, grp in enumerate(groups):
        members.setdefault(find(g), []).extend(grp[4])

    def rank(i):
        c = cands[i]
        return (-float(c[4]), int(c[1]), int(c[3]), int(c[2]))

    best = {root: min(m, key=rank) for root, m in members.items()}
    roots = sorted(best, key=lambda r: (int(cands[best[r]][0]), int(cands[best[r]][1]),
                                        int(cands[best[r]][2]), int(cands[best[r]][3])))
    reps = [tuple(cands[best[r]]) for r in roots]
    index = {r: k for k, r in enumerate(roots)}
    label = [0] * n
    for root, m in members.items():
        for i in m:
            label[i] = index[root]
    return reps, label


def cluster_offline(cands, t_window: int, dm_edges, min_snr: float):
    """Offline clustering of an observation's candidates over time (Sect. 6b.1, "Offline
    analysis"): candidates below a DM or an S/N limit are discarded (the paper: DM below 20,
    S/N below 10), and within each time window (0.5 s in the paper) and each DM window (windows
    that widen as the DM grows) only the candidate with the highest S/N is kept.

    Readings: a candidate's time is its start in native samples, sample * downsample; the time
    windows are [k t_window, (k + 1) t_window) for integer k (floor division, also for negative
    starts); the DM windows are [e_j, e_{j+1}) over the increasing edges dm_edges, the last one
    open-ended, and a DM below e_0 is discarded (e_0 is the DM limit); S/N below min_snr is
    discarded (S/N equal to it is kept); windows are shared by all beams; ties in S/N go to the
    candidate that comes first in the input.

    cands: sequence of (beam, dm_index, width, sample, snr, downsample, dm).  Returns the kept
    candidates sorted by (native start, dm, beam, width).
    """
    edges = [float(e) for e in dm_edges]
    if t_window < 1 or not edges or any(b <= a for a, b in zip(edges, edges[1:])):
        raise ValueError("t_window >= 1 and strictly increasing DM edges are required")
    best = {}
    for i, c in enumerate(cands):
        snr, ds, dm = float(c[4]), int(c[5]), float(c[6])
        if int(c[2]) < 1 or ds < 1 or snr != snr or dm != dm:
            raise ValueError("candidate width and downsample must be >= 1, S/N and DM numbers")
        if dm < edges[0] or snr < min_snr:
            continue
        start = int(c[3]) * ds
        j = max(k for k, e in enumerate(edges) if e <= dm)
        key = (start // t_window, j)
        if key not in best or snr > float(cands[best[key]][4]):
            best[key] = i
    kept = [tuple(cands[i]) for i in best.values()]
    kept.sort(key=lambda c: (int(c[3]) * int(c[5]), float(c[6]), int(c[0]), int(c[2])))
    return kept


def _round_half_even_div(s: int, n: int) -> int:
    """round_half_even(s / n) for integers s >= 0, n >= 1, exactly."""
    q, r = divmod(s, n)
    if 2 * r > n or (2 * r == n and q % 2 == 1):
        q += 1
    return q


def _cut(values: np.ndarray, k: float) -> int:
    """Largest value that is not an outlier: floor(mu + k sigma), exactly, with the population
    mean and standard deviation of `values`; values above it are cut.  An integer u exceeds
    mu + k sigma exactly when D = n u - s1 > 0 and D^2 > k^2 (n s2 - s1^2) (k >= 0, sums
    exact); the FP64 value of mu + k sigma only gives the starting guess."""
    from fractions import Fraction
    v = np.asarray(values, dtype=np.int64)
    n = v.size
    s1 = int(v.sum())
    s2 = int((v * v).sum())
    var_n2 = n * s2 - s1 * s1
    kk = Fraction(k) ** 2

    def above(u):
        d = n * u - s1
        return d > 0 and d * d > kk * var_n2

    c = int(np.floor(s1 / n + k * np.sqrt(max(0, var_n2)) / n))
    while above(c):
        c -= 1
    while not above(c + 1):
        c += 1
    return c


def rfi_time_domain(data: np.ndarray, k: float, niter: int = 3) -> np.ndarray:
    """Time-domain RFI mitigation of one source row [nchan][nsamp] (Sect. 6b.2 "RFI mitigation",
    Sect. 9 on the fraction of data lost: bright, wide-band, low-DM RFI, three iterations on
    ever cleaner data, local statistics).

    Readings: the statistic is the zero-DM series z(t) = sum_c x[c][t] over the chunk; in each
    iteration the samples with z(t) > mean(z) + k std(z) (population, over the chunk's current
    data; decided exactly) are replaced, in every channel, by that channel's mean over the other samples rounded
    half to even.  A dispersed burst spreads over many samples of z and is left alone.
    Returns a cleaned uint8 copy."""
    if not k >= 0:
        raise ValueError("k must be >= 0")
    x = np.array(data, dtype=np.int64)
    for _ in range(niter):
        z = x.sum(axis=0)
        bad = z > _cut(z, k)
        if not bad.any():
            break
        good = ~bad
        n = int(good.sum())
        for c in range(x.shape[0]):
            x[c, bad] = _round_half_even_div(int(x[c, good].sum()), n)
    return x.astype(np.uint8)


def rfi_freq_domain(data: np.ndarray, k: float, niter: int = 3) -> np.ndarray:
    """Frequency-domain RFI mitigation of one source row [nchan][nsamp] (narrow-band RFI, three
    iterations, local statistics; same passages).

    Readings: each spectrum (one sample, all channels) is cleaned on its own: in each iteration
    the channels with x[c] > mean + k std (population, over the spectrum's current values) are
    replaced by the mean of the other channels rounded half to even.  A broad-band signal
    raises the whole spectrum and is left alone.  Returns a cleaned uint8 copy."""
    if not k >= 0:
        raise ValueError("k must be >= 0")
    x = np.array(data, dtype=np.int64)
    for t in range(x.shape[1]):
        col = x[:, t]
        for _ in range(niter):
            bad = col > _cut(col, k)
            if not bad.any():
                break
            good = ~bad
            col[bad] = _round_half_even_div(int(col[good].sum()), int(good.sum()))
        x[:, t] = col
    return x.astype(np.uint8)


def rfi_clean(data: np.ndarray, k_time: float, k_freq: float, niter: int = 3) -> np.ndarray:
    """Both filters on one chunk of source rows [nsrc][nchan][nsamp] (or one row
    [nchan][nsamp]): the time-domain filter, then the frequency-domain filter, per row.
    Reading: that order (the paper names the time-domain method first)."""
    a = np.asarray(data)
    rows = a[None] if a.ndim == 2 else a
    out = np.stack([rfi_freq_domain(rfi_time_domain(r, k_time, niter), k_freq, niter)
                    for r in rows])
    return out[0] if a.ndim == 2 else out


def sb_index_at_fmax(n_sb: int, ntab: int):
    """Grating index and TAB index of SB n_sb at the highest frequency (Appendix "Synthesized
    Beams"): n_TAB = n_sb mod N_TAB, minus N_TAB if above N_TAB/2 - 1, and n_gr such that
    n_sb = n_gr N_TAB + n_TAB.  Reading: the paper calls the rounding of n_sb / N_TAB "upward";
    the rounding that keeps n_sb = n_gr N_TAB + n_TAB (and the position equation) is the one
    taken: n_gr = (n_sb - n_TAB) / N_TAB exactly."""
    if ntab < 2 or ntab % 2:
        raise ValueError("an even number of TABs is required")
    n_tab = n_sb % ntab
    if n_tab > ntab // 2 - 1:
        n_tab -= ntab
    return (n_sb - n_tab) // ntab, n_tab


def sb_switch_freqs(n_sb: int, ntab: int, f_max: float, alpha: float, b_max: float,
                    b_cq: float, kmax: int = 64):
    """Frequencies f_k (MHz) at which grating n_gr of TAB n_TAB - k sgn(n_sb) lies where the SB
    points (Appendix "Synthesized Beams", the equation for f0, applied to the k-th neighbour):
    f_k = f_max (n_gr B_max + (n_TAB - k sgn) alpha B_cq) / (n_gr B_max + n_TAB alpha B_cq).
    Reading: the second term on the right of the position equation uses the TAB separation
    theta_sep(f0), as the substitution that follows it does (the equation as printed has the
    grating spacing there).  Returns [f_0 = f_max, f_1, ..., f_kmax]."""
    n_gr, n_tab = sb_index_at_fmax(n_sb, ntab)
    s = (n_sb > 0) - (n_sb < 0)
    if s == 0:  # the central SB is the central TAB's main lobe at every frequency
        return [f_max]
    a = alpha * b_cq
    den = n_gr * b_max + n_tab * a
    return [f_max * (n_gr * b_max + (n_tab - k * s) * a) / den for k in range(kmax + 1)]


def sb_table_beam_model(nsb: int, ntab: int, nchan: int, f_lo_mhz: float, df_mhz: float,
                        f_max: float = 1500.0, alpha: float = 0.80, b_max: float = 1296.0,
                        b_cq: float = 144.0, quarter: bool = False):
    """SB table from the beam model (Appendix "Synthesized Beams"), uint8 [nsb][nchan]: the TAB
    whose grating response covers SB s in channel c.

    SB s has index n_sb = s - (nsb - 1) // 2 (0 = the centre of the compound beam).  At
    f >= f_max the SB takes TAB n_TAB (sb_index_at_fmax); going down in frequency it switches
    to TAB n_TAB - k sgn(n_sb) below the k-th switch frequency f_sw,k = (1 - b) f_{k-1} + b f_k
    (sb_switch_freqs), b = 1/2 when SBs are one beam width apart (71 SBs) and, when they are
    half a beam width apart (151 SBs, quarter=True), b = 1/4 for even n_sb and 3/4 for odd.
    Readings: a TAB index outside [-N/2, N/2 - 1] is the same TAB one grating over, so the
    index is wrapped into that range; TAB n is row n + N/2 of the input (the central TAB is
    row N/2).  Channel frequencies are f_lo + c df (channel_freqs).  Returns (table, margin):
    margin = the smallest |f_c - f_sw,k| over the decisions taken, so that a caller can confirm
    no channel sits on a switch frequency."""
    if nsb < 1 or nchan < 1 or not (alpha > 0 and b_max > 0 and b_cq > 0 and f_max > 0):
        raise ValueError("bad beam-model arguments")
    f = channel_freqs(nchan, f_lo_mhz, df_mhz)
    half = ntab // 2
    out = np.zeros((nsb, nchan), dtype=np.uint8)
    margin = np.inf
    for srow in range(nsb):
        n_sb = srow - (nsb - 1) // 2
        n_gr, n_tab = sb_index_at_fmax(n_sb, ntab)
        sgn = (n_sb > 0) - (n_sb < 0)
        fk = sb_switch_freqs(n_sb, ntab, f_max, alpha, b_max, b_cq)
        b = 0.5 if not quarter else (0.25 if n_sb % 2 == 0 else 0.75)
        fsw = [(1 - b) * fk[k - 1] + b * fk[k] for k in range(1, len(fk))]
        for c in range(nchan):
            k = 0
            if sgn != 0:
                while k < len(fsw) and f[c] < fsw[k]:
                    k += 1
                if k < len(fsw):
                    margin = min(margin, abs(f[c] - fsw[k]))
                if k > 0:
                    margin = min(margin, abs(f[c] - fsw[k - 1]))
            j = n_tab - k * sgn
            out[srow, c] = ((j + half) % ntab)
    return out, margin

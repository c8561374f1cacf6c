"""Pins for the CPU oracle: closed forms, invariants, hand-worked fixtures and brute force on
tiny inputs -- none of them re-types the oracle's own expressions.  Each `check_*` takes the
oracle module so `test_oracle_mutants.py` can run the same pins against planted mistakes."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _tiny_plan(o, nchan=7, ndm=6, seed=0):
    f_lo, df = synth.band(nchan)
    dms = np.linspace(0.0, 40.0, ndm)
    return o.delay_table(nchan, f_lo, df, 1e-3, dms)


def _tiny_data(nchan=7, nsamp=96, seed=0):
    return np.random.default_rng(seed).integers(0, 256, size=(nchan, nsamp), dtype=np.uint8)


# ---------------------------------------------------------------- delay table
def check_delays_textbook(o):
    for case in _load("delays_textbook.json")["cases"]:
        got = o.delay_table(case["nchan"], case["f_lo"], case["df"], case["tsamp"], case["dms"])
        assert got.tolist() == case["delays"], case["note"]


def check_delay_invariants(o):
    f_lo, df = synth.band(64)
    dms = np.array([0.0, 3.0, 6.0, 50.0, 100.0, 2000.0])
    d, x = o.delay_table(64, f_lo, df, synth.TSAMP, dms, return_exact=True)
    assert np.all(d[0] == 0)                       # DM 0: no delay
    assert np.all(d[:, -1] == 0)                   # highest channel is the reference
    assert np.all(np.diff(d, axis=1) <= 0)         # lower frequency arrives later
    assert np.all(np.diff(d, axis=0) >= 0)         # delay grows with DM
    assert np.allclose(x[2], 2.0 * x[1], rtol=1e-14)          # linear in DM
    assert np.allclose(x[4], 2.0 * x[3], rtol=1e-14)
    # halving the sample time doubles the unrounded delay; downsampling by D divides it by D
    _, x2 = o.delay_table(64, f_lo, df, synth.TSAMP / 2, dms, return_exact=True)
    assert np.allclose(x2, 2.0 * x, rtol=1e-14)
    _, x4 = o.delay_table(64, f_lo, df, synth.TSAMP, dms, downsample=4, return_exact=True)
    assert np.allclose(4.0 * x4, x, rtol=1e-14)
    # rounding: every delay is within half a sample of the exact value
    assert np.all(np.abs(d - x) <= 0.5)
    # descending channel order gives the same delays, reversed along channels
    f_hi = f_lo + 63 * df
    dr = o.delay_table(64, f_hi, -df, synth.TSAMP, dms)
    assert np.array_equal(dr, d[:, ::-1])


def check_delay_apertif_span(o):
    # Across the 300 MHz band (1220-1520 MHz) the sweep is 4.148808 ms * (1/1.22^2 - 1/1.52^2)
    # = 0.99 ms per DM unit, i.e. about 12.1 samples of 81.92 us: DM 2047 spans ~24 770 samples
    # between the band edges; channel centres sit half a channel inside the edges.
    f_lo, df = synth.band(1536)
    d = o.delay_table(1536, f_lo, df, synth.TSAMP, [2047.0])
    edge = 4.148808e-3 * 2047 * (1 / 1.22 ** 2 - 1 / 1.52 ** 2) / synth.TSAMP
    assert d[0, 0] < edge and d[0, 0] > edge - 2 * 12.1 * 2047 * df / 300.0
    assert d.max() == d[0, 0]


def test_delays_textbook():
    check_delays_textbook(O)


def test_delay_invariants():
    check_delay_invariants(O)


def test_delay_apertif_span():
    check_delay_apertif_span(O)


def test_tie_audit():
    assert O.tie_audit(np.array([0.0, 1.25, 2.5])) == 0.0
    assert abs(O.tie_audit(np.array([0.1, 3.9])) - 0.4) < 1e-12
    # the synthetic plans used here sit far from rounding ties compared with FP64 noise
    for w in (synth.cfg_small(), synth.cfg_apertif(), synth.cfg_apertif_ds()):
        _, x = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms, w.downsample,
                             return_exact=True)
        # a few ulps of FP64 at the largest delay bound any evaluation-order difference
        assert O.tie_audit(x) > 64 * np.finfo(np.float64).eps * max(1.0, float(x.max()))


def test_delay_rejects_bad_args():
    with pytest.raises(ValueError):
        O.delay_table(4, 1400.0, 1.0, 0.0, [1.0])
    with pytest.raises(ValueError):
        O.delay_table(4, 1400.0, 1.0, 1e-3, [-1.0])
    with pytest.raises(ValueError):
        O.delay_table(4, 1400.0, 1.0, 1e-3, [float("nan")])


# ---------------------------------------------------------------- dedispersion
def check_zero_dm(o):
    data = _tiny_data()
    f_lo, df = synth.band(7)
    delays = o.delay_table(7, f_lo, df, 1e-3, [0.0, 30.0])
    x = o.dedisperse(data, delays)
    nout = data.shape[1] - int(delays.max())
    assert x.shape == (2, nout)
    assert np.array_equal(x[0], data.astype(np.int64).sum(axis=0)[:nout])


def check_impulse(o):
    delays = _tiny_plan(o)
    nchan, nsamp = 7, 96
    nout = nsamp - int(delays.max())
    for c0, s0, v in [(0, 60, 5), (3, 40, 255), (6, 10, 1)]:
        data = np.zeros((nchan, nsamp), dtype=np.uint8)
        data[c0, s0] = v
        x = o.dedisperse(data, delays)
        for d in range(delays.shape[0]):
            t = s0 - int(delays[d, c0])
            expect = np.zeros(nout, dtype=np.int64)
            if 0 <= t < nout:
                expect[t] = v
            assert np.array_equal(x[d], expect), (c0, s0, d)


def check_sum_conservation(o):
    data = _tiny_data(seed=3)
    delays = _tiny_plan(o)
    x = o.dedisperse(data, delays)
    nout = x.shape[1]
    for d in range(delays.shape[0]):
        tot = sum(int(data[c, delays[d, c]: delays[d, c] + nout].astype(np.int64).sum())
                  for c in range(data.shape[0]))
        assert int(x[d].sum()) == tot


def check_brute_force(o):
    # explicit loops over (d, t, c) on a random tiny case
    rng = np.random.default_rng(11)
    for trial in range(3):
        nchan, nsamp, ndm = int(rng.integers(1, 9)), int(rng.integers(40, 65)), int(rng.integers(1, 7))
        data = rng.integers(0, 256, size=(nchan, nsamp), dtype=np.uint8)
        delays = rng.integers(0, 20, size=(ndm, nchan))
        x = o.dedisperse(data, delays)
        nout = nsamp - int(delays.max())
        ref = np.zeros((ndm, nout), dtype=np.int64)
        for d in range(ndm):
            for t in range(nout):
                acc = 0
                for c in range(nchan):
                    acc += int(data[c][t + delays[d][c]])
                ref[d][t] = acc
        assert np.array_equal(x, ref)
        for d in range(ndm):
            for t in (0, nout - 1):
                assert o.dedisperse_at(data, delays, d, t) == ref[d][t]


def check_linearity_shift_permutation(o):
    a, b = _tiny_data(seed=4), _tiny_data(seed=5)
    delays = _tiny_plan(o)
    xa, xb = o.dedisperse(a, delays), o.dedisperse(b, delays)
    xab = o.dedisperse(a.astype(np.int64) + b.astype(np.int64), delays)
    assert np.array_equal(xab, xa + xb)
    k = 9                                                   # time-shift equivariance
    xs = o.dedisperse(a[:, k:], delays)
    assert np.array_equal(xs, xa[:, k:])
    perm = np.random.default_rng(6).permutation(a.shape[0])  # channel order is irrelevant
    assert np.array_equal(o.dedisperse(a[perm], delays[:, perm]), xa)


def check_chunked_stream(o):
    # streaming: each chunk carries the previous halo samples; outputs concatenate to one shot
    data = _tiny_data(nsamp=160, seed=7)
    delays = _tiny_plan(o)
    halo = int(delays.max())
    full = o.dedisperse(data, delays)
    new = 25
    parts = []
    for s in range(0, full.shape[1], new):
        e = min(s + new, full.shape[1])
        parts.append(o.dedisperse(data[:, s: e + halo], delays))
    assert np.array_equal(np.concatenate(parts, axis=1), full)


def check_tophat_exact(o):
    # an integer top-hat injected along the trial-d sweep adds exactly A*w*nchan to B_w at the
    # injection time (minus whatever clipping removed, which the injector reports)
    w = synth.cfg_small()
    nsamp = 4096
    delays = o.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    data = synth.noise((w.nchan, nsamp), seed=21)
    base = o.dedisperse(data, delays)
    d0, t0, width, amp = 140, 1500, 8, 5
    added = synth.add_tophat(data, t0 + delays[d0], width, amp)
    x = o.dedisperse(data, delays)
    nrep = x.shape[1] - 16 + 1
    bx = o.boxcar(x, width, nrep)
    bb = o.boxcar(base, width, nrep)
    assert bx[d0, t0] - bb[d0, t0] == int(added.sum()) == amp * width * w.nchan
    # the series changes only where some channel overlaps the top-hat
    assert np.array_equal(x[d0, :t0], base[d0, :t0])


def test_zero_dm():
    check_zero_dm(O)


def test_impulse():
    check_impulse(O)


def test_sum_conservation():
    check_sum_conservation(O)


def test_brute_force():
    check_brute_force(O)


def test_linearity_shift_permutation():
    check_linearity_shift_permutation(O)


def test_chunked_stream():
    check_chunked_stream(O)


def test_tophat_exact():
    check_tophat_exact(O)


def test_dedisperse_rejects_short_input():
    with pytest.raises(ValueError):
        O.dedisperse(np.zeros((2, 5), np.uint8), np.array([[0, 5]]))


# ---------------------------------------------------------------- downsampling, SB synthesis
def check_downsample(o):
    ramp = np.arange(23, dtype=np.int64)[None, :]
    for D in (1, 2, 4, 5):
        y = o.downsample(ramp, D)
        n = 23 // D
        t = np.arange(n)
        assert y.shape == (1, n)
        assert np.array_equal(y[0], D * D * t + D * (D - 1) // 2)   # sum_{j<D} (D t + j)
    assert np.array_equal(o.downsample(np.full((2, 9), 255, np.uint8), 4), np.full((2, 2), 1020))


def check_sb_synth(o):
    rng = np.random.default_rng(8)
    tab = rng.integers(0, 256, size=(12, 16, 40), dtype=np.uint8)
    for j in (0, 5, 11):
        sb = o.sb_synthesize(tab, np.full((1, 16), j))
        assert np.array_equal(sb[0], tab[j])
    table = synth.sb_table_synthetic(71, 12, 16)
    sb = o.sb_synthesize(tab, table)
    assert np.array_equal(sb[35], tab[11])                 # centre SB: one TAB, all channels
    c = 9
    assert np.array_equal(sb[0, c], tab[table[0, c], c])
    assert np.array_equal(sb[70, 3], tab[table[70, 3], 3])


def test_downsample():
    check_downsample(O)


def test_sb_synth():
    check_sb_synth(O)


# ---------------------------------------------------------------- boxcar / moments / S/N
def check_boxcar(o):
    x = np.random.default_rng(9).integers(-50, 400, size=(3, 70))
    assert np.array_equal(o.boxcar(x, 1, 70), x)
    for w in (1, 2, 4, 8, 16):
        n = 70 - 2 * w + 1
        b, b2 = o.boxcar(x, w, n + w), o.boxcar(x, 2 * w, n)
        assert np.array_equal(b2, b[:, :n] + b[:, w: w + n])    # doubling identity
    ramp = np.arange(40, dtype=np.int64)
    for w in (1, 3, 8):
        t = np.arange(40 - w + 1)
        assert np.array_equal(o.boxcar(ramp, w, 40 - w + 1), w * t + w * (w - 1) // 2)
    with pytest.raises(ValueError):
        o.boxcar(ramp, 8, 34)


def check_moments(o):
    n = 1000
    ramp = np.arange(n + 17, dtype=np.int64)
    mu, sig = o.moments(ramp, n)
    assert abs(mu - (n - 1) / 2) < 1e-9
    assert abs(sig - math.sqrt((n * n - 1) / 12.0)) < 1e-9   # population, not sample, variance
    mu, sig = o.moments(np.full(50, 7), 40)
    assert mu == 7.0 and sig == 0.0


def check_snr_noise(o):
    # pure quantised N(128, 16) noise, 128 channels: S/N of every boxcar has mean ~0, std ~1;
    # the dedispersed series has sigma ~ 16 sqrt(128) = 181
    w = synth.cfg_small()
    delays = o.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms[::16])
    data = synth.noise((w.nchan, 8192), seed=31)
    x = o.dedisperse(data, delays)
    nrep = x.shape[1] - 15
    mu, sig = o.moments(x, nrep)
    assert np.all(np.abs(sig / (16 * math.sqrt(128)) - 1) < 0.05)
    for width in (1, 4, 16):
        s = o.snr(o.boxcar(x, width, nrep), width, mu, sig)
        assert abs(s.mean()) < 0.05
        assert abs(s.std() - 1) < 0.05 + 0.02 * width
    assert np.all(o.snr(np.ones((1, 5)), 4, [1.0], [0.0]) == 0)


def check_candidates_golden(o):
    g = _load("candidates_tiny.json")
    x = np.array([g["series"]])
    mu, sig = o.moments(x, g["nrep"])
    assert abs(mu[0] - g["mean"]) < 1e-12 and abs(sig[0] - g["sigma"]) < 1e-12
    got = o.candidates(x, g["widths"], g["nrep"], g["threshold"])
    assert [c[:4] for c in got] == [tuple(c[:4]) for c in g["candidates"]]
    for c, e in zip(got, g["candidates"]):
        assert abs(c[4] - e[4]) < 1e-9
    assert o.candidates(x, g["widths"], g["nrep"], 5.0) == []


def check_injected_recovery(o):
    # three dispersed gaussian bursts at DM 30 / 70 / 110 (on-grid), FWHM 2..8, 3 sigma/channel
    w = synth.cfg_small()
    delays = o.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    nsamp = 16384
    bursts = []
    for dm, t0, fwhm in [(30.0, 3000, 2.0), (70.0, 8000, 4.0), (110.0, 12500, 8.0)]:
        d = int(np.argmin(np.abs(w.dms - dm)))
        bursts.append((d, t0, fwhm, synth.Burst(t0 + delays[d], fwhm, 48.0)))
    data = synth.noise((w.nchan, nsamp), seed=w.seed, bursts=[b[3] for b in bursts])
    x, cands = o.search(data, delays, w.widths, w.threshold)
    assert cands, "no candidates"
    for d, t0, fwhm, _ in bursts:
        near = [c for c in cands if abs(c[3] - t0) <= 16]
        assert near, (d, t0)
        best = max(near, key=lambda c: c[4])
        assert abs(best[1] - d) <= 1                      # detected at its DM trial
        assert fwhm / 2 <= best[2] * 1.0 <= 2 * fwhm + 1  # best width near the pulse width
    # nothing far from the bursts
    assert all(min(abs(c[3] - b[1]) for b in bursts) < 400 for c in cands)


def check_tophat_snr(o):
    # S/N of an exact top-hat at matched DM and width ~ A w nchan / (sigma sqrt w)
    w = synth.cfg_small()
    delays = o.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    data = synth.noise((w.nchan, 16384), seed=41)
    d0, t0, width, amp = 100, 7000, 4, 6
    synth.add_tophat(data, t0 + delays[d0], width, amp)
    x = o.dedisperse(data, delays)
    nrep = x.shape[1] - 15
    mu, sig = o.moments(x, nrep)
    s = o.snr(o.boxcar(x[d0:d0 + 1], width, nrep), width, mu[d0:d0 + 1], sig[d0:d0 + 1])
    expect = amp * width * w.nchan / (sig[d0] * math.sqrt(width))
    assert abs(s[0, t0] - expect) < 4.0            # noise of one S/N sample is ~1
    assert s[0, t0] > 8


def test_boxcar():
    check_boxcar(O)


def test_moments():
    check_moments(O)


def test_snr_noise():
    check_snr_noise(O)


def test_candidates_golden():
    check_candidates_golden(O)


def test_injected_recovery():
    check_injected_recovery(O)


def test_tophat_snr():
    check_tophat_snr(O)


# ------------------------------------------------------------------ decimated integration
def check_integrated_golden(o):
    g = _load("integrated_tiny.json")
    x = np.array(g["series"])
    got = o.candidates_integrated(x, g["widths"], g["nrep"], g["threshold"],
                                  t_offset=g["t_offset"])
    assert [c[:4] for c in got] == [tuple(c[:4]) for c in g["candidates"]]
    for c, e in zip(got, g["candidates"]):
        assert abs(c[4] - e[4]) < 1e-9


def _integrated_brute(x, widths, nrep, thr, t_offset):
    # explicit loops: mean and population sigma, the integrated samples of each width on the
    # absolute grid, their S/N, runs over consecutive integrated samples, first maximum
    out = []
    for d, row in enumerate(x.tolist()):
        n = nrep
        mu = sum(row[:n]) / n
        sig = math.sqrt(sum((v - mu) ** 2 for v in row[:n]) / n)
        for w in widths:
            ks = [t for t in range(n) if (t + t_offset) % w == 0]
            vals = [sum(row[t:t + w]) for t in ks]
            snrs = [(v - w * mu) / (sig * math.sqrt(w)) if sig > 0 else 0.0 for v in vals]
            i = 0
            while i < len(ks):
                if not snrs[i] > thr:
                    i += 1
                    continue
                best = i
                e = i
                while e < len(ks) and snrs[e] > thr:
                    if vals[e] > vals[best]:
                        best = e
                    e += 1
                out.append((0, d, w, ks[best] + t_offset, snrs[best]))
                i = e
    return sorted(out, key=lambda r: r[:4])


def check_integrated_brute_force(o):
    rng = np.random.default_rng(77)
    for trial in range(6):
        ndm, nrep = 4, int(rng.integers(30, 70))
        widths = sorted(set(int(v) for v in rng.choice([1, 2, 3, 4, 5, 7, 8], 3)))
        L = nrep + max(widths) - 1
        x = rng.integers(0, 20, size=(ndm, L))
        for r in range(ndm):                      # a few pulses, some straddling grid cells
            t = int(rng.integers(0, L - 6))
            x[r, t:t + int(rng.integers(1, 6))] += int(rng.integers(10, 40))
        t_off = int(rng.integers(-50, 50))
        thr = float(rng.choice([1.5, 2.0, 2.5]))
        got = o.candidates_integrated(x, widths, nrep, thr, t_offset=t_off)
        ref = _integrated_brute(x, widths, nrep, thr, t_off)
        assert [c[:4] for c in got] == [c[:4] for c in ref], trial
        for a, b in zip(got, ref):
            assert abs(a[4] - b[4]) < 1e-9


def check_integrated_invariants(o):
    rng = np.random.default_rng(78)
    x = rng.integers(0, 30, size=(5, 90))
    x[1, 40:44] += 60
    x[3, 10:13] += 50
    widths, nrep, thr = [1, 2, 4, 5], 80, 2.0
    # width 1 is the sliding search
    one = o.candidates_integrated(x, [1], nrep, thr, t_offset=17)
    assert one == o.candidates(x, [1], nrep, thr, t_offset=17)
    got = o.candidates_integrated(x, widths, nrep, thr, t_offset=-13)
    assert got
    for b, d, w, t, s in got:
        assert t % w == 0 and -13 <= t < nrep - 13      # on the absolute grid, searched starts
    # moving the series' origin by a multiple of every width keeps the grid: same candidates,
    # shifted
    lcm = 20
    moved = o.candidates_integrated(x, widths, nrep, thr, t_offset=-13 + lcm)
    assert [c[:3] + (c[3] - lcm,) for c in moved] == [c[:4] for c in got]
    # each integrated candidate is a sliding boxcar value: its S/N is at most the sliding
    # maximum of that row and width
    for b, d, w, t, s in got:
        sl = [c[4] for c in o.candidates(x, [w], nrep, thr, t_offset=-13) if c[1] == d]
        assert sl and s <= max(sl) + 1e-12


def test_integrated_golden():
    check_integrated_golden(O)


def test_integrated_brute_force():
    check_integrated_brute_force(O)


def test_integrated_invariants():
    check_integrated_invariants(O)


# ------------------------------------------------------------------ subband dedispersion
def check_subband_golden(o):
    g = _load("subband_tiny.json")
    pl = g["plan"]
    fine, coarse, d1, d2 = o.subband_plan(pl["nchan"], pl["f_lo"], pl["df"], pl["tsamp"],
                                          pl["dm_first"], pl["dm_step"], pl["ndm"], pl["nfine"],
                                          pl["nsub"])
    assert np.allclose(coarse, g["coarse_dms"])
    assert np.array_equal(d1, np.array(g["d1"]))
    assert np.array_equal(d2, np.array(g["d2"]))
    imp = g["impulses"]
    data = np.zeros((pl["nchan"], imp["nin"]), np.int64)
    for c, t, v in imp["list"]:
        data[c, t] = v
    x = o.subband_dedisperse(data, d1, d2, pl["nfine"])
    exp = np.zeros((pl["ndm"], imp["n2"]), np.int64)
    for k, t, v in imp["hits"]:
        exp[k, t] = v
    assert np.array_equal(x, exp)


def check_subband_reductions(o):
    rng = np.random.default_rng(11)
    nchan, f_lo, df, ts = 16, 1220.0, 1.5, 81.92e-6
    data = rng.integers(0, 256, size=(nchan, 700))
    # one channel per subband, one fine trial per coarse DM: exactly brute force
    fine, coarse, d1, d2 = o.subband_plan(nchan, f_lo, df, ts, 3.0, 7.0, 9, 1, nchan)
    assert np.all(d1 == 0) and np.allclose(coarse, fine)
    assert np.array_equal(o.subband_dedisperse(data, d1, d2, 1),
                          o.dedisperse(data, o.delay_table(nchan, f_lo, df, ts, fine)))
    # one subband: brute force at each trial's coarse DM
    fine, coarse, d1, d2 = o.subband_plan(nchan, f_lo, df, ts, 3.0, 7.0, 9, 4, 1)
    assert np.all(d2 == 0)
    ref = o.dedisperse(data, o.delay_table(nchan, f_lo, df, ts, coarse))
    got = o.subband_dedisperse(data, d1, d2, 4)
    for k in range(9):
        assert np.array_equal(got[k], ref[k // 4, : got.shape[1]])
    # sampled outputs equal the full evaluation
    fine, coarse, d1, d2 = o.subband_plan(nchan, f_lo, df, ts, 0.0, 2.0, 10, 4, 4)
    full = o.subband_dedisperse(data, d1, d2, 4)
    for k, t in zip(rng.integers(0, 10, 50), rng.integers(0, full.shape[1], 50)):
        assert o.subband_dedisperse_at(data, d1, d2, 4, int(k), int(t)) == full[k, t]


def check_subband_smearing_bound(o):
    # the composite delay differs from the brute-force delay by the intra-subband delay of the
    # DM offset from the coarse DM, plus rounding (ALERT GPU 1 plan: DM 0-409.6 step 0.2,
    # subbanding step 6.4 = 32 fine trials, 32 subbands of 48 channels)
    nchan, ts = 1536, 81.92e-6
    df = 300.0 / nchan
    f_lo = 1220.0 + df / 2
    fine, coarse, d1, d2 = o.subband_plan(nchan, f_lo, df, ts, 0.0, 0.2, 2048, 32, 32)
    assert coarse.size == 64 and np.isclose(coarse[0], 3.1) and np.isclose(coarse[1], 9.5)
    brute = o.delay_table(nchan, f_lo, df, ts, fine)
    f = o.channel_freqs(nchan, f_lo, df)
    fs = f.reshape(32, 48).max(axis=1)
    j = np.arange(2048) // 32
    comp = d1[j] + np.repeat(d2, 48, axis=1)
    gap = np.abs(fine - coarse[j])[:, None] * o.K_DM * (1 / f**2 - 1 / np.repeat(fs, 48)**2) / ts
    assert np.all(np.abs(comp - brute) <= np.ceil(gap) + 1)
    assert np.abs(comp - brute).max() >= 2        # the method is an approximation


def test_subband_golden():
    check_subband_golden(O)


def test_subband_reductions():
    check_subband_reductions(O)


def test_subband_smearing_bound():
    check_subband_smearing_bound(O)


def test_subband_rejects_bad_args():
    with pytest.raises(ValueError):
        O.subband_plan(10, 1220.0, 1.0, 1e-4, 0.0, 1.0, 8, 4, 3)   # 3 does not divide 10
    with pytest.raises(ValueError):
        O.subband_plan(12, 1220.0, 1.0, 1e-4, 0.0, 0.0, 8, 4, 3)   # zero DM step


# ---------------------------------------------------------------- DM-width clustering
def check_cluster_golden(o):
    g = _load("cluster_tiny.json")
    cands = [tuple(c) for c in g["candidates"]]
    reps, label = o.cluster_dm_width(cands)
    assert [tuple(r) for r in reps] == [tuple(r) for r in g["reps"]]
    parts = {}
    for i, k in enumerate(label):
        parts.setdefault(k, []).append(i)
    assert sorted(parts.values()) == sorted(g["clusters"])


def _random_cands(rng, n, nbeam=2, ndm=6, tmax=40, widths=(1, 2, 4, 8)):
    seen, out = set(), []
    while len(out) < n:
        key = (int(rng.integers(nbeam)), int(rng.integers(ndm)), int(rng.choice(widths)),
               int(rng.integers(tmax)))
        if key not in seen:
            seen.add(key)
            out.append(key + (float(rng.choice([6.0, 6.5, 7.0, 7.5, 9.0])),))
    return out


def _components_brute(cands):
    # connected components of the graph: same beam, DM indices at most 1 apart, windows
    # [t, t + w - 1] intersecting (the union of a step-1 group is an interval, so two groups'
    # extents overlap exactly when two of their windows do)
    n = len(cands)
    adj = [[] for _ in range(n)]
    for i in range(n):
        bi, di, wi, ti, _ = cands[i]
        for j in range(i + 1, n):
            bj, dj, wj, tj, _ = cands[j]
            if bi == bj and abs(di - dj) <= 1 and ti <= tj + wj - 1 and tj <= ti + wi - 1:
                adj[i].append(j)
                adj[j].append(i)
    comp, out = [-1] * n, []
    for s in range(n):
        if comp[s] >= 0:
            continue
        comp[s], todo, members = len(out), [s], []
        while todo:
            a = todo.pop()
            members.append(a)
            for b in adj[a]:
                if comp[b] < 0:
                    comp[b] = comp[s]
                    todo.append(b)
        out.append(sorted(members))
    return out


def check_cluster_brute_force(o):
    rng = np.random.default_rng(11)
    for n in (1, 2, 5, 30, 80, 160):
        cands = _random_cands(rng, n)
        reps, label = o.cluster_dm_width(cands)
        parts = {}
        for i, k in enumerate(label):
            parts.setdefault(k, []).append(i)
        comps = _components_brute(cands)
        assert sorted(parts.values()) == sorted(comps), n
        assert len(reps) == len(comps)
        for k, members in parts.items():
            top = max(cands[i][4] for i in members)
            r = reps[k]
            assert r[4] == top and tuple(r) in [cands[i] for i in members]
            # the lowest DM, earliest sample, smallest width among the members at that S/N
            assert tuple(r[:4]) == min(((cands[i][0], cands[i][1], cands[i][2], cands[i][3])
                                        for i in members if cands[i][4] == top),
                                       key=lambda c: (c[1], c[3], c[2]))


def check_cluster_invariants(o):
    rng = np.random.default_rng(12)
    cands = _random_cands(rng, 60)
    reps, label = o.cluster_dm_width(cands)
    perm = rng.permutation(len(cands))
    reps2, label2 = o.cluster_dm_width([cands[i] for i in perm])
    assert reps2 == reps                                   # input order does not matter
    assert [label[i] for i in perm] == label2
    assert o.cluster_dm_width([]) == ([], [])
    one = (3, 7, 4, 100, 8.25)
    assert o.cluster_dm_width([one]) == ([one], [0])
    # disjoint windows in one row, or one DM apart with a one-sample gap, never join
    apart = [(0, 0, 4, 0, 7.0), (0, 0, 4, 4, 7.0), (0, 1, 2, 8, 7.0), (0, 3, 2, 8, 7.0)]
    assert len(o.cluster_dm_width(apart)[0]) == 4
    # a dispersed burst seen over widths and DMs reduces to few clusters and keeps its best S/N
    w = synth.cfg_small()
    delays = o.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms[:80])
    data = synth.noise((w.nchan, int(delays.max()) + 1500), seed=5)
    synth.add_tophat(data, 600 + delays[40], 6, 14)
    _, cands = o.search(data, delays, w.widths, 7.0)
    reps, _ = o.cluster_dm_width(cands)
    assert 0 < len(reps) < len(cands) / 4
    assert max(r[4] for r in reps) == max(c[4] for c in cands)
    best = max(reps, key=lambda r: r[4])
    assert abs(best[1] - 40) <= 2 and abs(best[3] - 600) <= 16


def test_cluster_golden():
    check_cluster_golden(O)


def test_cluster_brute_force():
    check_cluster_brute_force(O)


def test_cluster_invariants():
    check_cluster_invariants(O)


def test_cluster_rejects_bad_width():
    with pytest.raises(ValueError):
        O.cluster_dm_width([(0, 0, 0, 5, 7.0)])


# ---------------------------------------------------------------- offline clustering
def check_offline_golden(o):
    g = _load("cluster_offline_tiny.json")
    cands = [tuple(c) for c in g["candidates"]]
    kept = o.cluster_offline(cands, g["t_window"], g["dm_edges"], g["min_snr"])
    assert [tuple(c) for c in kept] == [cands[i] for i in g["kept"]]


def _random_offline(rng, n):
    out = []
    for _ in range(n):
        ds = int(rng.choice([1, 2, 4]))
        out.append((int(rng.integers(3)), int(rng.integers(50)), int(rng.choice([1, 2, 4, 8])),
                    int(rng.integers(-400, 3000)) // ds, float(rng.choice([9.5, 10.0, 11.0, 14.0])),
                    ds, float(rng.choice([15.0, 20.0, 33.0, 60.0, 61.5, 130.0, 400.0]))))
    return out


def check_offline_brute_force(o):
    rng = np.random.default_rng(21)
    edges, tw, smin = [20.0, 40.0, 60.0, 61.5, 200.0], 250, 10.0
    for n in (0, 1, 7, 60, 400):
        cands = _random_offline(rng, n)
        kept = o.cluster_offline(cands, tw, edges, smin)
        # the windows, computed independently: every passing candidate's window, by scanning
        passing = [i for i, c in enumerate(cands) if c[6] >= edges[0] and c[4] >= smin]
        win = {}
        for i in passing:
            c = cands[i]
            start = c[3] * c[5]
            k = 0
            while (k + 1) * tw <= start:
                k += 1
            while k * tw > start:
                k -= 1
            j = sum(1 for e in edges if e <= c[6]) - 1
            win.setdefault((k, j), []).append(i)
        assert len(kept) == len(win), n
        chosen = set()
        for members in win.values():
            top = max(cands[i][4] for i in members)
            first = min(i for i in members if cands[i][4] == top)
            chosen.add(first)
        assert sorted(kept) == sorted(cands[i] for i in chosen)
        starts = [c[3] * c[5] for c in kept]
        assert starts == sorted(starts)


def check_offline_invariants(o):
    rng = np.random.default_rng(22)
    cands = [c for c in _random_offline(rng, 200) if c[3] >= 0]
    # one window holding everything keeps only the global best (first on ties)
    big = o.cluster_offline(cands, 10 ** 9, [-1.0], -1e9)
    assert len(big) == 1 and big[0][4] == max(c[4] for c in cands)
    assert big[0] == next(c for c in cands if c[4] == big[0][4])
    # the limits: a candidate exactly at both limits stays, just below either goes
    base = (0, 0, 1, 7, 10.0, 1, 20.0)
    assert o.cluster_offline([base], 100, [20.0], 10.0) == [base]
    assert o.cluster_offline([base[:4] + (np.nextafter(10.0, 0.0),) + base[5:]], 100,
                             [20.0], 10.0) == []
    assert o.cluster_offline([base[:6] + (np.nextafter(20.0, 0.0),)], 100, [20.0], 10.0) == []
    # the same native start from different downsampling lands in the same window
    a, b = (0, 0, 1, 40, 11.0, 1, 30.0), (1, 0, 1, 10, 12.0, 4, 30.0)
    assert o.cluster_offline([a, b], 41, [20.0], 10.0) == [b]
    assert o.cluster_offline([], 100, [20.0], 10.0) == []


def test_offline_golden():
    check_offline_golden(O)


def test_offline_brute_force():
    check_offline_brute_force(O)


def test_offline_invariants():
    check_offline_invariants(O)


def test_offline_rejects_bad_args():
    with pytest.raises(ValueError):
        O.cluster_offline([], 0, [20.0], 10.0)
    with pytest.raises(ValueError):
        O.cluster_offline([], 10, [20.0, 20.0], 10.0)
    with pytest.raises(ValueError):
        O.cluster_offline([(0, 0, 1, 5, 11.0, 0, 30.0)], 10, [20.0], 10.0)


# ---------------------------------------------------------------- RFI mitigation
def check_rfi_golden(o):
    g = _load("rfi_tiny.json")
    t = np.array(g["time"]["data"], np.uint8)
    assert np.array_equal(o.rfi_time_domain(t, g["time"]["k"]), np.array(g["time"]["clean"]))
    f = np.array(g["freq"]["data"], np.uint8)
    assert np.array_equal(o.rfi_freq_domain(f, g["freq"]["k"]), np.array(g["freq"]["clean"]))
    # both filters: the frequency-domain fixture has no time-domain outlier at k = 3
    assert np.array_equal(o.rfi_clean(f, 3.0, g["freq"]["k"]), np.array(g["freq"]["clean"]))


def check_rfi_ties(o):
    # a value exactly at mean + k sigma is not above the cut: the cut is decided exactly
    g = _load("rfi_tiny.json")["ties"]
    v = np.array(g["values"], np.uint8)
    for k, want in ((g["k_tie"], g["clean_tie"]), (g["k_above"], g["clean_above"])):
        assert np.array_equal(o.rfi_time_domain(v[None], k)[0], want), k
        assert np.array_equal(o.rfi_freq_domain(v[:, None], k)[:, 0], want), k
        assert np.array_equal(o.rfi_clean(v[:, None], 9.0, k)[:, 0], want), k


def check_rfi_targets(o):
    nchan, nsamp = 96, 3000
    base = synth.noise((nchan, nsamp), seed=41)
    # quiet data: nothing moves at 6 sigma
    assert np.array_equal(o.rfi_time_domain(base, 6.0), base)
    assert np.array_equal(o.rfi_freq_domain(base, 6.0), base)
    # a bright broad-band zero-DM spike: the time domain replaces the whole column by the
    # channel means of the other samples, the frequency domain leaves it (the spectrum is flat)
    x = base.copy()
    x[:, 1200] = np.minimum(255, x[:, 1200].astype(int) + 60).astype(np.uint8)
    t = o.rfi_time_domain(x, 6.0)
    others = np.delete(np.arange(nsamp), 1200)
    means = np.rint(base[:, others].astype(np.float64).mean(axis=1))
    assert np.all(np.abs(t[:, 1200].astype(int) - means) <= 1)
    assert np.array_equal(np.delete(t, 1200, axis=1), np.delete(x, 1200, axis=1))
    assert np.array_equal(o.rfi_freq_domain(x, 6.0), x)
    # only bright samples are cut: a dropout (a column of zeros) stays
    w = base.copy()
    w[:, 700] = 0
    assert np.array_equal(o.rfi_time_domain(w, 6.0), w)
    # a dispersed burst of the same energy spread over 500 samples passes the time domain
    f_lo, df = synth.band(nchan)
    d = o.delay_table(nchan, f_lo, df, synth.TSAMP, np.array([500.0]))[0]
    y = base.copy()
    synth.add_tophat(y, 1000 + d, 4, 30)
    assert np.array_equal(o.rfi_time_domain(y, 6.0), y)
    # narrow-band spikes in two channels at one sample: the frequency domain replaces them
    assert np.array_equal(o.rfi_freq_domain(base, 5.0), base)
    z = base.copy()
    z[[10, 50], 2000] = 255
    f = o.rfi_freq_domain(z, 5.0)
    assert np.all(f[[10, 50], 2000] < 200)
    assert np.array_equal(np.delete(f, 2000, axis=1), np.delete(z, 2000, axis=1))


def check_rfi_iterations(o):
    # every iteration cleans what the previous one exposed: two spikes of different height
    # (zero-DM excess 400, 60 and 4 over a flat 400: each hides the next from the 3-sigma cut)
    x = np.full((4, 200), 100, np.uint8)
    x[:, 50] = 200
    x[:, 120] = 115
    x[:, 7] = 101
    cols = [50, 120, 7]
    for n in range(4):
        y = o.rfi_time_domain(x, 3.0, niter=n)
        assert [int(y[0, c]) for c in cols] == [100] * min(n, 3) + [200, 115, 101][min(n, 3):], n
    # constant data are a fixed point of both filters
    c = np.full((5, 40), 77, np.uint8)
    assert np.array_equal(o.rfi_clean(c, 0.5, 0.5), c)


def test_rfi_golden():
    check_rfi_golden(O)


def test_rfi_ties():
    check_rfi_ties(O)


def test_rfi_exact_cut_worked_values():
    # the oracle's cut helper against hand-worked values (fixture "ties"): mean + 2 sigma is an
    # exact integer in both cases
    from oracle.arts_oracle import _cut
    g = _load("rfi_tiny.json")["ties"]
    assert _cut(np.array(g["cut_values"]), g["cut_k"]) == g["cut"]
    assert _cut(np.array(g["values"]), g["k_tie"]) == 31


def test_rfi_targets():
    check_rfi_targets(O)


def test_rfi_iterations():
    check_rfi_iterations(O)


# ---------------------------------------------------------------- SB table from the beam model
def check_sb_beam_golden(o):
    g = _load("sb_beam_tiny.json")
    for n_sb, n_gr, n_tab in g["index"]:
        assert o.sb_index_at_fmax(n_sb, g["ntab"]) == (n_gr, n_tab), n_sb
    for n_sb, f1 in g["f1"]:
        got = o.sb_switch_freqs(n_sb, g["ntab"], g["f_max"], g["alpha"], g["b_max"], g["b_cq"])
        assert abs(got[1] - f1) < 1e-9 and got[0] == g["f_max"], n_sb
    kw = dict(f_max=g["f_max"], alpha=g["alpha"], b_max=g["b_max"], b_cq=g["b_cq"])
    for nsb, key, quarter in ((71, "switch71", False), (151, "switch151", True)):
        t, margin = o.sb_table_beam_model(nsb, g["ntab"], g["nchan"], g["f_lo"], g["df"],
                                          quarter=quarter, **kw)
        assert t.shape == (nsb, g["nchan"]) and margin > 1e-4
        for row, c0, r0, c1, r1 in g[key]:
            assert (int(t[row, c0]), int(t[row, c1])) == (r0, r1), (nsb, row)
        assert np.all(t[(nsb - 1) // 2] == g["ntab"] // 2)


def check_sb_beam_nearest(o):
    # one beam width apart (71 SBs), the switch halfway between f_{k-1} and f_k is where two TABs'
    # grating responses are equally far (in angle) from the SB: the table picks, per channel,
    # the TAB whose response of the SB's grating order is nearest, among all TAB indices
    nchan, ntab, a, bmax, bcq, fmax = 384, 12, 0.8, 1296.0, 144.0, 1500.0
    f_lo, df = synth.band(nchan)
    f = o.channel_freqs(nchan, f_lo, df)
    t, margin = o.sb_table_beam_model(71, ntab, nchan, f_lo, df, fmax, a, bmax, bcq)
    assert margin > 1e-6
    for row in range(71):
        n_sb = row - 35
        n_gr, n_tab = o.sb_index_at_fmax(n_sb, ntab)
        target = (n_gr / bcq + n_tab * a / bmax) / fmax        # position x (c = 1) at f_max
        js = np.arange(n_tab - 60, n_tab + 61)
        for c in range(nchan):
            pos = (n_gr / bcq + js * a / bmax) / f[c]
            j = js[int(np.argmin(np.abs(pos - target)))]
            assert t[row, c] == (j + ntab // 2) % ntab, (n_sb, c)


def check_sb_beam_invariants(o):
    nchan, ntab = 256, 12
    f_lo, df = synth.band(nchan)
    for quarter, nsb in ((False, 71), (True, 151)):
        t, _ = o.sb_table_beam_model(nsb, ntab, nchan, f_lo, df, quarter=quarter)
        f = o.channel_freqs(nchan, f_lo, df)
        for row in range(nsb):
            n_sb = row - (nsb - 1) // 2
            n_gr, n_tab = o.sb_index_at_fmax(n_sb, ntab)
            assert n_sb == n_gr * ntab + n_tab and -ntab // 2 <= n_tab < ntab // 2
            # at and above f_max the TAB of the decomposition; walking down in frequency the
            # TAB index moves away by one at a time, in the direction of -sgn(n_sb)
            top = t[row, f >= 1500.0]
            assert np.all(top == n_tab + ntab // 2)
            steps = (np.diff(t[row][::-1].astype(int)) % ntab)
            sgn = (n_sb > 0) - (n_sb < 0)
            assert set(steps.tolist()) <= {0, (-sgn) % ntab}, n_sb
    with pytest.raises(ValueError):
        o.sb_index_at_fmax(3, 11)


def test_sb_beam_golden():
    check_sb_beam_golden(O)


def test_sb_beam_nearest():
    check_sb_beam_nearest(O)


def test_sb_beam_invariants():
    check_sb_beam_invariants(O)


ALL_CHECKS = [check_delays_textbook, check_delay_invariants, check_delay_apertif_span,
              check_zero_dm, check_impulse, check_sum_conservation, check_brute_force,
              check_linearity_shift_permutation, check_chunked_stream, check_tophat_exact,
              check_downsample, check_sb_synth, check_boxcar, check_moments, check_snr_noise,
              check_candidates_golden, check_injected_recovery, check_tophat_snr,
              check_integrated_golden, check_integrated_brute_force, check_integrated_invariants,
              check_subband_golden, check_subband_reductions, check_subband_smearing_bound,
              check_cluster_golden, check_cluster_brute_force, check_cluster_invariants,
              check_offline_golden, check_offline_brute_force, check_offline_invariants,
              check_rfi_golden, check_rfi_ties, check_rfi_targets, check_rfi_iterations,
              check_sb_beam_golden, check_sb_beam_nearest, check_sb_beam_invariants]

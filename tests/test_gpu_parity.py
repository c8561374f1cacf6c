"""GPU parity: the HIP library against the CPU oracle on the same seeded inputs.
Integer outputs (delays, dedispersed series, boxcar sums, SB data) must match bit for bit;
FP32 S/N within 1e-4 relative of the oracle's FP64; candidate sets equal except in (DM, width)
rows holding an S/N within 1e-4 of the threshold."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from tests._parity import (compare_candidates, near_threshold_runs, oracle_rows_candidates,
                           to_dev)

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _plan(w, variant=None):
    p = arts.Plan.from_workload(w)
    if variant is not None:
        p.set_tiling(variant)
    return p


def _native_variants():
    # byte-sample tilings that run plain plans (group-sum tilings run subband step 1 only)
    return [v for v in range(arts.arts_tiling_count())
            if "SPD=4" in arts.arts_tiling_describe(v)
            and "group" not in arts.arts_tiling_describe(v)]


def _ds_variants():
    return [v for v in range(arts.arts_tiling_count()) if "SPD=2" in arts.arts_tiling_describe(v)]


# ------------------------------------------------------------------------ delays / plans
def test_plan_delays_match_oracle():
    for w in (synth.cfg_small(), synth.cfg_apertif(), synth.cfg_apertif_ds()):
        with _plan(w) as p:
            ref = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms, w.downsample)
            assert np.array_equal(p.delays(), ref)
            assert p.max_delay == int(ref.max())
            assert p.halo == int(ref.max()) + max(w.widths) - 1


# ------------------------------------------------------------------------ dedispersion
def test_dedisperse_small_full():
    w = synth.cfg_small()
    _say("dedisperse small full", w.name)
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    data = synth.noise((w.nchan, 16384), seed=w.seed)
    ref = O.dedisperse(data, delays)
    with _plan(w) as p:
        got = p.dedisperse(to_dev(data)).cpu().numpy()
    assert got.shape == (1,) + ref.shape
    assert np.array_equal(got[0], ref)


@pytest.mark.parametrize("variant", _native_variants())
def test_dedisperse_variants_ragged(variant):
    # 2 beams, DM count not a multiple of any block, nin odd, several time tiles + ragged tail
    _say("dedisperse variant", variant, arts.arts_tiling_describe(variant))
    f_lo, df = synth.band(80)
    dms = np.arange(101) * 1.7
    delays = O.delay_table(80, f_lo, df, synth.TSAMP, dms)
    nin = int(delays.max()) + 3 * 1792 + 77
    data = np.stack([synth.noise((80, nin), seed=s) for s in (11, 12)])
    w = synth.Workload("ragged", 80, f_lo, df, synth.TSAMP, dms, [1, 2, 4])
    with _plan(w, variant) as p:
        got = p.dedisperse(to_dev(data)).cpu().numpy()
    for b in range(2):
        assert np.array_equal(got[b], O.dedisperse(data[b], delays)), b


@pytest.mark.parametrize("variant", [v for v in _native_variants()
                                     if "packed" in arts.arts_tiling_describe(v)
                                     or "runs" in arts.arts_tiling_describe(v)])
def test_packed_variants_many_channels(variant):
    # 600 channels: the 16-bit partial sums are widened more than once per tile (every staged
    # chunk, every run of a sub-dword class, or every 257 channels when they are held across
    # chunks); saturated input puts every half at its largest value, random input is checked
    # against the oracle
    _say("packed variant, 600 channels", variant, arts.arts_tiling_describe(variant))
    nchan = 600
    f_lo, df = synth.band(nchan)
    dms = np.arange(45) * 2.3
    delays = O.delay_table(nchan, f_lo, df, synth.TSAMP, dms)
    nin = int(delays.max()) + 1500 + 13
    w = synth.Workload("wide", nchan, f_lo, df, synth.TSAMP, dms, [1])
    rng = np.random.default_rng(variant + 600)
    data = rng.integers(0, 256, size=(nchan, nin), dtype=np.uint8)
    with _plan(w, variant) as p:
        got = p.dedisperse(to_dev(data)).cpu().numpy()[0]
        full = p.dedisperse(to_dev(np.full((nchan, nin), 255, np.uint8))).cpu().numpy()[0]
    assert np.array_equal(got, O.dedisperse(data, delays))
    assert np.all(full == 255 * nchan)


@pytest.mark.parametrize("variant", [v for v in _native_variants()
                                     if "runs shared" in arts.arts_tiling_describe(v)])
def test_shared_word_tile_edges(variant):
    # lanes that take their last dword's sums from the next lane leave a tile's last 4 outputs
    # to the next tile (the last lane's are wrong): output counts just below, at and above
    # multiples of the 1276-output tile, with all four sub-dword classes in every chunk
    _say("shared-word tile edges", variant, arts.arts_tiling_describe(variant))
    f_lo, df = synth.band(96)
    dms = np.arange(70) * 1.3
    delays = O.delay_table(96, f_lo, df, synth.TSAMP, dms)
    w = synth.Workload("edges", 96, f_lo, df, synth.TSAMP, dms, [1])
    rng = np.random.default_rng(variant)
    with _plan(w, variant) as p:
        for nout in (1, 4, 1272, 1275, 1276, 1277, 1280, 2551, 2552, 2556, 3830):
            nin = int(delays.max()) + nout
            data = rng.integers(0, 256, size=(96, nin), dtype=np.uint8)
            got = p.dedisperse(to_dev(data)).cpu().numpy()[0]
            assert got.shape[1] == nout
            assert np.array_equal(got, O.dedisperse(data, delays)), nout


def _framed_sweep_variants():
    return [v for v in range(arts.arts_tiling_count())
            if ("framed runs" in arts.arts_tiling_describe(v)
                and "group" not in arts.arts_tiling_describe(v))
            or "pairs framed" in arts.arts_tiling_describe(v)]


@pytest.mark.parametrize("variant", _framed_sweep_variants())
def test_framed_channels_per_chunk(variant):
    # channels per chunk 1..13, 17, 44 and as many as the plan allows: a class's run takes every
    # length from 0 up (byte runs: an odd run's lone first channel, then four offsets per step,
    # then a last pair; DM pairs: four channels per step, then the last one to three together),
    # one and two LDS buffers; the largest chunk also with all-255 input, which fills the 16-bit
    # halves of a chunk's frames (for the DM pairs, both parity frames merged at the flush)
    desc = arts.arts_tiling_describe(variant)
    pairs = "pairs" in desc
    if pairs:
        D, nchan = 4, 160
        dms = 2048.0 + 2.3 * np.arange(64)
    else:
        D, nchan = 1, 96
        dms = np.arange(70) * 1.3
    f_lo, df = synth.band(nchan)
    delays = O.delay_table(nchan, f_lo, df, synth.TSAMP, dms, downsample=D)
    nin = (int(delays.max()) + 1500) * D + (D - 1)
    w = synth.Workload("sweep", nchan, f_lo, df, synth.TSAMP, dms, [1], downsample=D)
    rng = np.random.default_rng(variant + 4000)
    data = rng.integers(0, 256, size=(nchan, nin), dtype=np.uint8)
    ref = O.dedisperse(O.downsample(data, D) if D > 1 else data, delays)
    full = np.full((nchan, nin), 255, np.uint8)
    with _plan(w) as p:
        cap = {}
        for buffers in (1, 2):  # as many channels as the LDS holds with that many buffers
            p.set_tiling_shape(variant, buffers, 0)
            cap[buffers] = p.tiling_shape()[2]
        shapes = [(cc, 1 + cc % 2) for cc in list(range(1, 14)) + [17]] + [(44, 2), (0, 1)]
        for cc, buffers in shapes:
            p.set_tiling_shape(variant, buffers, cc)
            v, nb, used = p.tiling_shape()
            _say("framed chunk sweep", variant, desc, "buffers", nb, "channels", used)
            # a requested count is an upper bound: the LDS may hold fewer
            assert (v, nb) == (variant, buffers)
            assert used == (min(cc, cap[buffers]) if cc else cap[buffers])
            got = p.dedisperse(to_dev(data)).cpu().numpy()[0]
            assert np.array_equal(got, ref), (cc, buffers)
        assert used > 13
        if pairs:
            assert used <= 64  # the plan's cap for these chunks: 64 x 1020 < 2^16
        got = p.dedisperse(to_dev(full)).cpu().numpy()[0]
        assert np.all(got == 255 * D * nchan)


@pytest.mark.parametrize("nchan,ndm,extra", [(1, 1, 1), (3, 5, 2), (37, 33, 1000), (7, 70, 5),
                                             (255, 9, 300), (256, 40, 64), (300, 3, 33)])
def test_dedisperse_edge_shapes(nchan, ndm, extra):
    _say("edge shape", nchan, ndm, extra)
    f_lo, df = synth.band(nchan)
    rng = np.random.default_rng(nchan * 1000 + ndm)
    dms = rng.uniform(0, 300, size=ndm)            # unsorted DM list
    delays = O.delay_table(nchan, f_lo, df, synth.TSAMP, dms)
    nin = int(delays.max()) + extra
    data = rng.integers(0, 256, size=(nchan, nin), dtype=np.uint8)
    w = synth.Workload("edge", nchan, f_lo, df, synth.TSAMP, dms, [1])
    with _plan(w) as p:
        got = p.dedisperse(to_dev(data)).cpu().numpy()[0]
    assert np.array_equal(got, O.dedisperse(data, delays))


def test_dedisperse_extreme_values():
    # all-255 input: every output equals 255 * nchan (no overflow, no lost channel)
    w = synth.cfg_apertif()
    with _plan(w) as p:
        nin = p.max_delay + 700
        data = np.full((1536, nin), 255, np.uint8)
        got = p.dedisperse(to_dev(data)).cpu().numpy()
    assert got.shape == (1, 2048, 700)
    assert np.all(got == 255 * 1536)


def test_dedisperse_short_input_rejected():
    w = synth.cfg_small()
    with _plan(w) as p:
        data = to_dev(np.zeros((w.nchan, p.max_delay), np.uint8))
        with pytest.raises(arts.ArtsError) as e:
            p.dedisperse(data)
        assert e.value.status == arts.ARTS_E_SHAPE


def test_dedisperse_apertif_sampled():
    # full Apertif shape (1536 ch, 2048 DMs, 12500 new samples + overlap) in the bench's tiling;
    # the oracle checks 4000 sampled outputs one by one and 6 complete DM rows
    w = synth.cfg_apertif()
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    nin = synth.CHUNK + int(delays.max()) + max(w.widths) - 1
    bursts, meta = synth.random_bursts(delays, synth.CHUNK, seed=w.seed)
    data = synth.noise((w.nchan, nin), seed=w.seed, bursts=bursts)
    _say("apertif sampled: nin", nin)
    with _plan(w) as p:
        got = p.dedisperse(to_dev(data)).cpu().numpy()[0]
    rng = np.random.default_rng(5)
    L = got.shape[1]
    for d, t in zip(rng.integers(0, 2048, 4000), rng.integers(0, L, 4000)):
        assert got[d, t] == O.dedisperse_at(data, delays, d, t), (d, t)
    rows = [0, 1, 2047, meta[0][0], meta[1][0], int(rng.integers(0, 2048))]
    full = O.dedisperse(data, delays[rows])
    # the row-subset oracle's output is shorter when the subset's max delay is smaller
    for i, d in enumerate(rows):
        assert np.array_equal(got[d], full[i, :L]), d


# ------------------------------------------------------------------------ SB synthesis
def test_sb_synthesize_small():
    rng = np.random.default_rng(3)
    tab = rng.integers(0, 256, size=(12, 96, 1001), dtype=np.uint8)
    table = synth.sb_table_synthetic(71, 12, 96)
    got = arts.arts_sb_synthesize(to_dev(tab), to_dev(table)).cpu().numpy()
    assert np.array_equal(got, O.sb_synthesize(tab, table))


def test_sb_synthesize_apertif_rows():
    tab = synth.noise((12, 1536, 37519), seed=33)
    table = synth.sb_table_synthetic()
    got = arts.arts_sb_synthesize(to_dev(tab), to_dev(table))
    for s in (0, 17, 35, 70):
        ref = O.sb_synthesize(tab, table[s: s + 1])[0]
        assert np.array_equal(got[s].cpu().numpy(), ref), s


def test_dedisperse_sb_fused_small():
    f_lo, df = synth.band(64)
    dms = np.arange(70) * 2.0
    w = synth.Workload("sb", 64, f_lo, df, synth.TSAMP, dms, [1, 2])
    delays = O.delay_table(64, f_lo, df, synth.TSAMP, dms)
    nin = int(delays.max()) + 2000
    tab = synth.noise((12, 64, nin), seed=44)
    table = synth.sb_table_synthetic(71, 12, 64)
    sb = O.sb_synthesize(tab, table)
    with _plan(w) as p:
        got = p.dedisperse_sb(to_dev(tab), to_dev(table)).cpu().numpy()
    for s in range(71):
        assert np.array_equal(got[s], O.dedisperse(sb[s], delays)), s


def test_dedisperse_sb_fused_apertif_sampled():
    w = synth.cfg_apertif()
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    nin = synth.CHUNK + int(delays.max()) + 255
    tab = synth.noise((12, 1536, nin), seed=55)
    table = synth.sb_table_synthetic()
    _say("fused SB apertif")
    with _plan(w) as p:
        out = p.dedisperse_sb(to_dev(tab), to_dev(table))
        rng = np.random.default_rng(9)
        for s in (0, 35, 70, 23):
            sb = O.sb_synthesize(tab, table[s: s + 1])[0]
            got = out[s].cpu().numpy()
            for d, t in zip(rng.integers(0, 2048, 500), rng.integers(0, got.shape[1], 500)):
                assert got[d, t] == O.dedisperse_at(sb, delays, d, t), (s, d, t)


# ------------------------------------------------------------------------ downsampling
def _pair_step(delays):
    """Largest and smallest delay step between the trials of a DM pair (trials 2k, 2k + 1)."""
    n = delays.shape[0] // 2 * 2
    d = delays[1:n:2].astype(np.int64) - delays[0:n:2]
    return int(d.max()), int(d.min())


@pytest.mark.parametrize("variant", _ds_variants())
@pytest.mark.parametrize("D", [2, 4, 5])
def test_dedisperse_downsampled(variant, D):
    f_lo, df = synth.band(96)
    dms = np.arange(2048, 2200, 2, dtype=np.float64)
    delays = O.delay_table(96, f_lo, df, synth.TSAMP, dms, downsample=D)
    nin = (int(delays.max()) + 1500) * D + (D - 1)       # trailing partial group dropped
    data = synth.noise((2, 96, nin), seed=66 + D)
    w = synth.Workload("ds", 96, f_lo, df, synth.TSAMP, dms, [1, 2, 4], downsample=D)
    if "pairs" in arts.arts_tiling_describe(variant) and _pair_step(delays)[0] > 7:
        # DM-pair tilings read one window per pair: trials more than 7 samples apart in some
        # channel are refused (plans then take another tiling)
        with pytest.raises(arts.ArtsError) as e:
            _plan(w, variant)
        assert e.value.status == arts.ARTS_E_INVAL
        with _plan(w) as p:
            assert "pairs" not in arts.arts_tiling_describe(p.tiling())
        return
    with _plan(w, variant) as p:
        got = p.dedisperse(to_dev(data)).cpu().numpy()
    for b in range(2):
        ref = O.dedisperse(O.downsample(data[b], D), delays)
        assert np.array_equal(got[b], ref)


def _pair_variants():
    return [v for v in _ds_variants() if "pairs" in arts.arts_tiling_describe(v)]


@pytest.mark.parametrize("variant", _pair_variants())
@pytest.mark.parametrize("case", ["classes", "saturated", "odd"])
def test_dedisperse_ds_pairs(variant, case):
    # DM pairs: every class (both parities of the first trial's offset, steps 0..7 inside a
    # pair) occurs; an odd trial count leaves the last pair with one trial; all-255 input fills
    # the 16-bit partial sums of a 64-channel chunk (64 x 1020 < 2^16)
    D, nchan = 4, 160
    f_lo, df = synth.band(nchan)
    ndm = 77 if case == "odd" else 64
    dms = 2048.0 + 2.3 * np.arange(ndm)
    delays = O.delay_table(nchan, f_lo, df, synth.TSAMP, dms, downsample=D)
    hi, lo = _pair_step(delays)
    assert hi <= 7 and lo == 0
    steps = set((delays[1::2][: ndm // 2] - delays[0::2][: ndm // 2]).ravel().tolist())
    assert steps == set(range(hi + 1)), steps
    nin = (int(delays.max()) + 1300) * D + 2
    if case == "saturated":
        data = np.full((3, nchan, nin), 255, np.uint8)
    else:
        data = synth.noise((3, nchan, nin), seed=91 + ndm)
    w = synth.Workload("pairs", nchan, f_lo, df, synth.TSAMP, dms, [1, 2, 4], downsample=D)
    _say("DM pairs", variant, arts.arts_tiling_describe(variant), case)
    with _plan(w, variant) as p:
        got = p.dedisperse(to_dev(data)).cpu().numpy()
    for b in range(3):
        assert np.array_equal(got[b], O.dedisperse(O.downsample(data[b], D), delays)), b


# ------------------------------------------------------------------------ boxcar / S/N
def test_boxcar_snr_small():
    w = synth.cfg_small()
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    data = synth.noise((w.nchan, 16384), seed=w.seed)
    x = O.dedisperse(data, delays)
    nrep = x.shape[1] - max(w.widths) + 1
    with _plan(w) as p:
        stats, sums, snr = p.boxcar_snr(to_dev(x.astype(np.int32)[None]))
        stats, sums, snr = stats.cpu().numpy()[0], sums.cpu().numpy()[0], snr.cpu().numpy()[0]
    mu, sig = O.moments(x, nrep)
    assert np.allclose(stats[:, 0], mu, rtol=1e-13)
    assert np.allclose(stats[:, 1], sig, rtol=1e-12)
    for wi, width in enumerate(w.widths):
        b = O.boxcar(x, width, nrep)
        assert np.array_equal(sums[wi], b), width
        ref = O.snr(b, width, mu, sig)
        err = np.abs(snr[wi] - ref) / np.maximum(np.abs(ref), 1e-30)
        ok = (np.abs(ref) < 1e-6) & (np.abs(snr[wi]) < 1e-5) | (err <= 1e-4)
        assert ok.all(), (width, float(err.max()))


def test_boxcar_snr_flat_series():
    w = synth.cfg_small()
    with _plan(w) as p:
        x = np.full((2, w.dms.size, 3000), 777, np.int32)
        stats, sums, snr = p.boxcar_snr(to_dev(x))
        assert np.all(stats.cpu().numpy()[..., 1] == 0)
        assert np.all(snr.cpu().numpy() == 0)
        assert np.all(sums.cpu().numpy()[:, 2] == 777 * 4)
        assert len(p.candidates(to_dev(x), 8.0)) == 0


# ------------------------------------------------------------------------ candidates
def test_candidates_small_with_bursts():
    w = synth.cfg_small()
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    bursts = []
    for dm, t0, fwhm in [(30.0, 3000, 2.0), (70.0, 8000, 4.0), (110.0, 12500, 8.0)]:
        d = int(np.argmin(np.abs(w.dms - dm)))
        bursts.append(synth.Burst(t0 + delays[d], fwhm, 48.0))
    data = synth.noise((w.nchan, 16384), seed=w.seed, bursts=bursts)
    x, ora = O.search(data, delays, w.widths, w.threshold)
    nrep = x.shape[1] - max(w.widths) + 1
    rows = np.arange(x.shape[0])
    near = near_threshold_runs(x, w.widths, nrep, w.threshold, rows)
    with _plan(w) as p:
        series = p.dedisperse(to_dev(data))
        assert np.array_equal(series.cpu().numpy()[0], x)
        got = p.candidates(series, w.threshold)
    assert len(ora) > 10
    assert compare_candidates(got, ora, near) > 0
    assert np.all(got["downsample"] == 1)
    assert np.allclose(got["dm"], w.dms[got["dm_index"]].astype(np.float32))


def test_candidates_offsets_and_capacity():
    w = synth.cfg_small()
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    d = 140
    data = synth.noise((w.nchan, 16384), seed=7)
    synth.add_tophat(data, 5000 + delays[d], 8, 40)
    with _plan(w) as p:
        series = p.dedisperse(to_dev(data))
        full = p.candidates(series, 8.0)
        assert len(full) > 3
        shifted = p.candidates(series, 8.0, t_offset=1000, beam_offset=7)
        assert np.array_equal(shifted["sample"], full["sample"] + 1000)
        assert np.all(shifted["beam"] == 7)
        with pytest.raises(arts.ArtsError) as e:
            arts.lib()  # capacity too small: the raw call reports the count
            import ctypes
            n = ctypes.c_int64(0)
            buf = np.zeros(1, dtype=arts.CANDIDATE_DTYPE)
            st = arts.lib().arts_candidates(p.handle, series.data_ptr(), 1, series.shape[2],
                                            8.0, 0, 0, buf.ctypes.data, 1, ctypes.byref(n),
                                            arts._stream(None))
            assert st == arts.ARTS_E_CAPACITY and n.value == len(full)
            arts._check(st)
        assert e.value.status == arts.ARTS_E_CAPACITY


@pytest.mark.parametrize("nsamp", [16384, 40000])
def test_candidates_resident_and_segmented_rows(nsamp):
    # rows up to 16k starts are searched resident in LDS, longer ones segment by segment; both
    # against the oracle, with wide bright top-hats so that runs cross the 4096-start segments
    f_lo, df = synth.band(64)
    dms = np.arange(0, 96, 3.0)
    widths = [1, 2, 4, 8, 16, 32, 64]
    w = synth.Workload("seg", 64, f_lo, df, synth.TSAMP, dms, widths)
    delays = O.delay_table(64, f_lo, df, synth.TSAMP, dms)
    data = synth.noise((64, nsamp), seed=123 + nsamp)
    for d, t0, width in ((5, 4000, 300), (20, 8150, 40), (31, 12280, 16)):
        synth.add_tophat(data, t0 + delays[d], width, 30)
    x, ora = O.search(data, delays, widths, 8.0)
    nrep = x.shape[1] - max(widths) + 1
    near = near_threshold_runs(x, widths, nrep, 8.0, np.arange(x.shape[0]))
    _say("candidates rows", nsamp, "nrep", nrep)
    with _plan(w) as p:
        series = p.dedisperse(to_dev(data))
        assert np.array_equal(series.cpu().numpy()[0], x)
        got = p.candidates(series, 8.0)
    assert len(ora) > 20
    assert compare_candidates(got, ora, near) > 0


def test_candidates_pure_noise_empty():
    w = synth.cfg_small()
    data = synth.noise((w.nchan, 16384), seed=99)
    with _plan(w) as p:
        got = p.candidates(p.dedisperse(to_dev(data)), 8.0)
    assert len(got) == 0


@pytest.mark.parametrize("widths,nrep", [([1, 2, 4, 8, 16, 32, 64, 128, 256], 3001),
                                         ([1, 3, 7, 20, 100, 600, 1000], 3001), ([5], 3001),
                                         (list(range(1, 17)), 3001), ([1, 2, 4, 8, 16], 100),
                                         ([1, 4, 64], 256), ([2, 3, 300], 257)])
def test_candidates_many_rows_match_oracle(widths, nrep):
    # 1030 DM rows of a synthetic series: enough rows that a row-level pre-pass decides which
    # rows the exact search visits.  Rows of one partial chunk, exactly one chunk and one chunk
    # plus a start; a ragged last chunk of starts, odd and even width counts, a widest width
    # above 512 samples, a level whose prefix sums wrap mod 2^32, and top-hats of S/N 6 to 24
    # at random widths in 40 rows (pure noise elsewhere); all rows against the oracle
    ndm, thr = 1030, 8.0
    wmax = max(widths)
    L = nrep + wmax - 1
    rng = np.random.default_rng(500 + len(widths) + wmax + nrep)
    x = np.rint(rng.normal(1.5e6, 600.0, (ndm, L))).astype(np.int64)
    rows = rng.choice(ndm, 40, replace=False)
    for i, r in enumerate(rows):
        w = int(rng.integers(1, wmax + 1))
        t = int(rng.integers(0, L - w))
        x[r, t:t + w] += int(round(600.0 * (6.0 + 6.0 * (i % 4)) / math.sqrt(w)))
    x = x.astype(np.int32)
    f_lo, df = synth.band(64)
    _say("candidates many rows", len(widths), "widths, wmax", wmax)
    with arts.Plan(64, f_lo, df, synth.TSAMP, np.arange(ndm) * 0.01, widths) as p:
        got = p.candidates(to_dev(x[None]), thr)
    ora = O.candidates(x, widths, nrep, thr)
    near = near_threshold_runs(x, widths, nrep, thr, np.arange(ndm))
    assert len(ora) >= 10
    assert compare_candidates(got, ora, near) > 0


@pytest.mark.parametrize("widths", [[1, 2, 4, 8, 16, 32, 64, 128, 256],
                                    [1, 5, 10, 25, 50, 100, 250]])
def test_candidates_bounded_widths(widths):
    # the pre-pass checks a width 2v through twice the largest sum of v over starts up to
    # nrep + v: top-hats whose width is such a 2v, just above threshold at that width, some of
    # them ending in the last searched starts (where the bound needs the extended starts);
    # 1030 rows (the pre-pass runs), all against the oracle
    ndm, thr, nrep = 1030, 8.0, 3001
    wmax = max(widths)
    L = nrep + wmax - 1
    bounded = [w for w in widths if w % 2 == 0 and w // 2 in widths]
    rng = np.random.default_rng(900 + wmax)
    x = np.rint(rng.normal(1.5e6, 600.0, (ndm, L))).astype(np.int64)
    rows = rng.choice(ndm, 48, replace=False)
    for i, r in enumerate(rows):
        w = bounded[i % len(bounded)]
        t = nrep - 1 - int(rng.integers(0, 3)) if i % 3 == 0 else int(rng.integers(0, nrep - 1))
        x[r, t:t + w] += int(round(600.0 * (8.3 + 0.5 * (i % 5)) / math.sqrt(w)))
    x = x.astype(np.int32)
    f_lo, df = synth.band(64)
    _say("candidates, bounded widths", widths)
    with arts.Plan(64, f_lo, df, synth.TSAMP, np.arange(ndm) * 0.01, widths) as p:
        got = p.candidates(to_dev(x[None]), thr)
    ora = O.candidates(x, widths, nrep, thr)
    near = near_threshold_runs(x, widths, nrep, thr, np.arange(ndm))
    assert len(ora) >= 20
    assert any(int(c[2]) in bounded for c in ora)
    assert compare_candidates(got, ora, near) > 0


def test_candidates_apertif_rows():
    # full-size Apertif chunk with 20 bursts: candidates of 48 DM rows (around the bursts and
    # random) against the oracle on those rows; the moments use the reported window only
    w = synth.cfg_apertif()
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    nin = synth.CHUNK + int(delays.max()) + 255
    bursts, meta = synth.random_bursts(delays, synth.CHUNK, seed=w.seed)
    data = synth.noise((w.nchan, nin), seed=w.seed, bursts=bursts)
    _say("apertif candidates")
    with _plan(w) as p:
        series = p.dedisperse(to_dev(data))
        got = p.candidates(series, w.threshold)
        x_all = series.cpu().numpy()[0]
    rng = np.random.default_rng(1)
    rows = sorted(set([m[0] + k for m in meta[:8] for k in (-1, 0, 1)] +
                      list(rng.integers(0, 2048, 24))))
    rows = [r for r in rows if 0 <= r < 2048]
    x_rows = O.dedisperse(data, delays[rows])[:, : x_all.shape[1]]
    assert np.array_equal(x_rows, x_all[rows])
    nrep = x_all.shape[1] - 255
    assert nrep == synth.CHUNK
    ora = oracle_rows_candidates(x_rows, w.widths, nrep, w.threshold, rows)
    near = near_threshold_runs(x_rows, w.widths, nrep, w.threshold, rows)
    sel = got[np.isin(got["dm_index"], rows)]
    compare_candidates(sel, ora, near)
    assert len(ora) > 0


@pytest.mark.parametrize("off", [1, 2, 3])
def test_dedisperse_misaligned_buffer(off):
    # an input whose start and end are not dword-aligned: the dwords holding its first and last
    # samples must be read (DM 0 puts the first samples of channel 0 into output 0, and with
    # DM 0 alone the last samples of the last row into the last output)
    import torch
    f_lo, df = synth.band(64)
    for dms in (np.arange(0.0, 40.0), np.array([0.0])):
        w = synth.Workload("mis", 64, f_lo, df, synth.TSAMP, dms, [1])
        delays = O.delay_table(64, f_lo, df, synth.TSAMP, dms)
        nin = int(delays.max()) + 1200
        nin += (-nin) % 4                                  # row pitch stays a multiple of 4
        data = np.random.default_rng(off).integers(0, 256, (2, 64, nin), dtype=np.uint8)
        buf = torch.zeros(data.size + 8, dtype=torch.uint8, device="cuda")
        view = buf[off: off + data.size].view(2, 64, nin)
        view.copy_(torch.from_numpy(data))
        assert view.data_ptr() % 4 == off
        with _plan(w) as p:
            got = p.dedisperse(view).cpu().numpy()
        for b in range(2):
            assert np.array_equal(got[b], O.dedisperse(data[b], delays)), (off, dms.size, b)

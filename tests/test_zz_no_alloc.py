"""GPU checks of arts_candidates_noalloc (the allocation-free candidate search): through the C
ABI, its records equal those of arts_candidates on the same series, call after call (the second
on a smaller input, so that a stale counter or stale flags in the shared array would show), and
the limits are enforced."""
import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from tests._parity import compare_candidates, near_threshold_runs, to_dev

pytestmark = pytest.mark.gpu


def _same(a, b):
    assert a.dtype == b.dtype and len(a) == len(b)
    assert a.tobytes() == b.tobytes()


def test_noalloc_equals_allocating_call_twice():
    w = synth.cfg_small()
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    bursts = []
    for dm, t0, fwhm in [(30.0, 3000, 2.0), (70.0, 8000, 4.0), (110.0, 12500, 8.0)]:
        d = int(np.argmin(np.abs(w.dms - dm)))
        bursts.append(synth.Burst(t0 + delays[d], fwhm, 48.0))
    data = synth.noise((w.nchan, 16384), seed=w.seed, bursts=bursts)
    print("no-alloc: cfg-small beam, two calls", flush=True)
    with arts.Plan.from_workload(w) as p:
        series = p.dedisperse(to_dev(data))
        ref = p.candidates(series, w.threshold)
        got = arts.arts_candidates_noalloc(p.handle, series, w.threshold, capacity=4096)
        _same(got, ref)
        assert len(got) > 10
        # against the oracle as well
        x = series.cpu().numpy()[0]
        nrep = x.shape[1] - max(w.widths) + 1
        ora = O.candidates(x, w.widths, nrep, w.threshold)
        compare_candidates(got, ora, near_threshold_runs(x, w.widths, nrep, w.threshold,
                                                         np.arange(x.shape[0])))
        # second call: a shorter series holding only the first burst, with offsets
        short = series[:, :, :5000].contiguous()
        ref2 = p.candidates(short, w.threshold, t_offset=17, beam_offset=3)
        got2 = arts.arts_candidates_noalloc(p.handle, short, w.threshold, t_offset=17,
                                            beam_offset=3, capacity=4096)
        _same(got2, ref2)
        assert 0 < len(got2) < len(got)


def test_noalloc_prepass_rows_twice():
    # >= 1024 rows: the row pre-pass runs and its flags live in the shared array too
    rng = np.random.default_rng(77)
    widths = [1, 2, 4, 8, 16, 32, 64, 128, 256]
    f_lo, df = synth.band(64)
    for ndm, nrep, seed in ((1030, 3001, 1), (1024, 1500, 2)):
        L = nrep + max(widths) - 1
        x = np.rint(rng.normal(1.5e6, 600.0, (ndm, L))).astype(np.int64)
        for r in rng.choice(ndm, 30, replace=False):
            wd = int(rng.integers(1, 257))
            t = int(rng.integers(0, L - wd))
            x[r, t:t + wd] += int(600.0 * 12.0 / np.sqrt(wd))
        x = x.astype(np.int32)
        print("no-alloc: pre-pass rows", ndm, nrep, flush=True)
        with arts.Plan(64, f_lo, df, synth.TSAMP, np.arange(ndm) * 0.01, widths) as p:
            dev = to_dev(x[None])
            ref = p.candidates(dev, 8.0)
            got = arts.arts_candidates_noalloc(p.handle, dev, 8.0, capacity=1 << 14)
            _same(got, ref)
            assert len(got) >= 10


def test_noalloc_limits_and_state():
    w = synth.cfg_small()
    data = synth.noise((w.nchan, 4000), seed=5)
    with arts.Plan.from_workload(w) as p:
        series = p.dedisperse(to_dev(data))
        with pytest.raises(arts.ArtsError) as e:
            arts.arts_candidates_noalloc(p.handle, series, 8.0,
                                         capacity=arts.NOALLOC_MAX_CANDIDATES + 1)
        assert e.value.status == arts.ARTS_E_INVAL
        # capacity too small: the count is reported as by arts_candidates
        quiet = arts.arts_candidates_noalloc(p.handle, series, 8.0, capacity=16)
        assert len(quiet) == 0
        loud = arts.arts_candidates_noalloc(p.handle, series, 3.0, capacity=1 << 15)
        assert len(loud) > 2
        with pytest.raises(arts.ArtsError) as e:
            arts.arts_candidates_noalloc(p.handle, series, 3.0, capacity=1)
        assert e.value.status == arts.ARTS_E_CAPACITY
        p.cluster = True
        with pytest.raises(arts.ArtsError) as e:
            arts.arts_candidates_noalloc(p.handle, series, 8.0)
        assert e.value.status == arts.ARTS_E_STATE

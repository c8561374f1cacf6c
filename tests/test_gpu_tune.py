"""GPU checks of the tile shapes and the autotuners (the paper's search is auto-tuned per
platform and setup, Sect. 6b.2): every shape stays bit-exact against the oracle, the plan
autotuner picks a valid shape and caches it (keyed by device and delay table), and the batch
autotuner puts all requests of a kind into one tiling without changing any result."""
import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from tests._parity import to_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _native_plan(nchan=96, ndm=100, step=1.5):
    f_lo, df = synth.band(nchan)
    w = synth.Workload("tune", nchan, f_lo, df, synth.TSAMP, np.arange(ndm) * step,
                       [1, 2, 4, 8])
    return w, arts.Plan.from_workload(w)


def _ds_plan(nchan=128, ndm=70):
    f_lo, df = synth.band(nchan)
    w = synth.Workload("tune-ds", nchan, f_lo, df, synth.TSAMP, 2048.0 + 2.0 * np.arange(ndm),
                       [1, 2, 4], downsample=4)
    return w, arts.Plan.from_workload(w)


@pytest.mark.parametrize("buffers,channels", [(1, 0), (2, 7), (1, 5), (2, 1)])
def test_tile_shapes_bit_exact(buffers, channels):
    # one LDS buffer (twice the channels per chunk) and capped chunk sizes, native and 16-bit
    for make in (_native_plan, _ds_plan):
        w, p = make()
        delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms, w.downsample)
        nin = (int(delays.max()) + 1700) * w.downsample + 3
        data = synth.noise((2, w.nchan, nin), seed=17 + buffers + channels)
        with p:
            v0 = p.tiling()
            p.set_tiling_shape(v0, buffers, channels)
            v, nb, cc = p.tiling_shape()
            assert (v, nb) == (v0, buffers) and cc >= 1
            if channels:
                assert cc <= channels
            _say("shape", w.name, arts.arts_tiling_describe(v), nb, cc)
            got = p.dedisperse(to_dev(data)).cpu().numpy()
        for b in range(2):
            x = data[b] if w.downsample == 1 else O.downsample(data[b], w.downsample)
            assert np.array_equal(got[b], O.dedisperse(x, delays)), (w.name, b)


def test_tile_shape_rejects():
    w, p = _native_plan()
    with p:
        v0 = p.tiling_shape()
        for args in ((v0[0], 3, 0), (v0[0], 2, 256), (v0[0], 0, 0), (arts.arts_tiling_count(), 2, 0)):
            with pytest.raises(arts.ArtsError) as e:
                p.set_tiling_shape(*args)
            assert e.value.status == arts.ARTS_E_INVAL
            assert p.tiling_shape() == v0          # the plan keeps its tiling


def test_plan_autotune_cache_and_parity(tmp_path):
    cache = str(tmp_path / "tune.txt")
    for make in (_native_plan, _ds_plan):
        w, p = make()
        delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms, w.downsample)
        nin = (int(delays.max()) + 2100) * w.downsample
        with p:
            _say("autotune", w.name)
            v, ms = p.autotune(2, nin, reps=1, cache_path=cache)
            assert ms > 0 and p.tiling() == v
            shape = p.tiling_shape()
            d = arts.arts_tiling_describe(v)
            assert ("SPD=4" in d) == (w.downsample == 1)
            lines = open(cache).read().splitlines()
            assert lines and lines[-1].split()[0].startswith("gfx")
            # the cached entry is taken without timing again, and sets the same shape
            spd = "SPD=2" if w.downsample > 1 else "SPD=4"
            other = [u for u in range(arts.arts_tiling_count())
                     if spd in arts.arts_tiling_describe(u) and u != v
                     and "group" not in arts.arts_tiling_describe(u)]
            p.set_tiling(other[-1])
            v2, ms2 = p.autotune(2, nin, reps=1, cache_path=cache)
            assert v2 == v and abs(ms2 - ms) < 1e-3
            assert p.tiling_shape() == shape
            assert len(open(cache).read().splitlines()) == len(lines)
            data = synth.noise((2, w.nchan, nin), seed=5)
            got = p.dedisperse(to_dev(data)).cpu().numpy()
        for b in range(2):
            x = data[b] if w.downsample == 1 else O.downsample(data[b], w.downsample)
            assert np.array_equal(got[b], O.dedisperse(x, delays)), (w.name, b)
    # a different delay table (same sizes) is a different key
    w, p = _native_plan(step=1.25)
    with p:
        before = len(open(cache).read().splitlines())
        p.autotune(2, (int(p.max_delay) + 2100), reps=1, cache_path=cache)
        assert len(open(cache).read().splitlines()) == before + 1


def test_batch_autotune_one_launch_same_results():
    import torch
    reqs = synth.uneven_requests(12, seed=21)
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    items, plans = [], []
    for w in reqs:
        p = arts.Plan.from_workload(w)
        nin = w.extra["nsamp"]
        L = arts.series_length(p, nin)
        if L < max(w.widths):
            p.close()
            continue
        data = torch.randint(0, 256, (1, w.nchan, nin), dtype=torch.uint8, device="cuda",
                             generator=g)
        out = torch.empty((1, w.dms.size, L), dtype=torch.int32, device="cuda")
        items.append((p, data, out))
        plans.append(p)
    assert len(items) >= 4
    with arts.Batch() as b:
        b.dedisperse(items)
        ref = [o.cpu().numpy().copy() for _, _, o in items]
        ref_c = b.candidates(items, 7.0)
        _say("batch autotune over", len(items), "requests")
        v, ms = b.autotune(items, reps=1)
        assert ms > 0
        shapes = {p.tiling_shape()[:2] for p in plans if p.info["downsample"] == 1}
        assert len(shapes) == 1 and next(iter(shapes))[0] == v
        for _, _, o in items:
            o.zero_()
        b.dedisperse(items)
        for (_, _, o), r in zip(items, ref):
            assert np.array_equal(o.cpu().numpy(), r)
        assert np.array_equal(b.candidates(items, 7.0), ref_c)
        # and the series equal the oracle on sampled DM rows of two requests
        for p, d, o in items[:2]:
            delays = p.delays()
            rows = [0, delays.shape[0] // 2, delays.shape[0] - 1]
            L = o.shape[2]
            x = O.dedisperse(d.cpu().numpy()[0], delays[rows])[:, :L]
            assert np.array_equal(o.cpu().numpy()[0][rows], x)
    for p in plans:
        p.close()


def test_default_tilings_of_the_measured_plans():
    # the shapes the plans take by default are the fastest measured on these plans: framed runs
    # in 12-wave blocks (six waves per SIMD) for the 2048 native serving trials, DM pairs in raw
    # frames in 16-wave blocks (eight) for the 1476 D=4 trials, and framed group sums in 16-wave
    # blocks for the first step of the ALERT subband plans; each stays exact (the parity suites
    # run every tiling)
    for w, want in ((synth.cfg_apertif(), "WAVES=12 SPD=4 framed runs shared"),
                    (synth.cfg_apertif_ds(), "WAVES=16 SPD=2 pairs framed")):
        with arts.Plan.from_workload(w) as p:
            d = arts.arts_tiling_describe(p.tiling())
            _say(w.name, p.tiling_shape(), d)
            assert d.endswith(want), d
    f_lo, df = synth.band(1536)
    for dm0, step, ndm, nfine in ((0.0, 0.2, 2048, 32), (819.2, 2.5, 1024, 16)):
        with arts.Plan.subband(1536, f_lo, df, synth.TSAMP, dm0, step, ndm, nfine, 32,
                               [1, 5, 10]) as p:
            d = arts.arts_tiling_describe(p.tiling())
            _say("subband", dm0, p.tiling_shape(), d)
            assert d.endswith("WAVES=16 SPD=4 framed runs group sums"), d

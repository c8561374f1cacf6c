"""GPU parity of decimated integration (arts_plan_set_integration, mode 1) against the oracle's
candidates_integrated: plan calls on synthetic series (small launches, and launches of at least
1024 rows, which go through the row pre-pass) with grid offsets of either sign, rows too long
to hold in LDS, a stream of native and downsampled plans whose chunks share the absolute grid
(including the partially warm chunks), and the argument checks (an unknown mode, widths that
do not divide a stream's chunk).  Candidate sets equal except in (DM, width) rows with an S/N
within 1e-4 of the threshold; matched S/N within 1e-4 relative."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from tests._parity import NearRuns, compare_candidates, near_threshold_runs, to_dev

pytestmark = pytest.mark.gpu

AMBER_WIDTHS = [1, 5, 10, 25, 50, 100, 250]


def _series(ndm, nrep, widths, seed):
    # noise at the level of a dedispersed series plus top-hats of S/N 7..22 at random widths
    # and positions (many straddle grid cells) in up to 40 rows
    wmax = max(widths)
    L = nrep + wmax - 1
    rng = np.random.default_rng(seed)
    x = np.rint(rng.normal(1.5e6, 600.0, (ndm, L))).astype(np.int64)
    for i, r in enumerate(rng.choice(ndm, min(ndm, 40), replace=False)):
        w = int(rng.integers(1, wmax + 1))
        t = int(rng.integers(0, L - w))
        x[r, t:t + w] += int(round(600.0 * (7.0 + 5.0 * (i % 4)) / math.sqrt(w)))
    return x.astype(np.int32)


@pytest.mark.parametrize("ndm,t_offset", [(60, 0), (60, -25013), (1030, 777)])
def test_integrated_plan_matches_oracle(ndm, t_offset):
    nrep, thr = 3001, 8.0
    x = _series(ndm, nrep, AMBER_WIDTHS, seed=900 + ndm)
    f_lo, df = synth.band(64)
    print("integrated plan call", ndm, "rows, t_offset", t_offset, flush=True)
    with arts.Plan(64, f_lo, df, synth.TSAMP, np.arange(ndm) * 0.01, AMBER_WIDTHS) as p:
        assert p.integration == "sliding"
        p.integration = "decimated"
        assert p.integration == "decimated"
        got = p.candidates(to_dev(x[None]), thr, t_offset=t_offset)
        p.integration = "sliding"
        slid = p.candidates(to_dev(x[None]), thr, t_offset=t_offset)
    ora = O.candidates_integrated(x, AMBER_WIDTHS, nrep, thr, t_offset=t_offset)
    near = near_threshold_runs(x, AMBER_WIDTHS, nrep, thr, np.arange(ndm), t_offset=t_offset,
                               integration=True)
    assert len(ora) >= 10
    assert compare_candidates(got, ora, near) > 0
    assert all(int(c["sample"]) % int(c["width"]) == 0 for c in got)
    # width 1 searches every start either way; wider widths report fewer, grid-aligned samples
    one = lambda c: c[c["width"] == 1]
    assert np.array_equal(one(got), one(slid))
    assert len(got) < len(slid)


def test_integrated_stream_matches_oracle():
    nchan, chunk, nsrc = 64, 2500, 2
    f_lo, df = synth.band(nchan)
    ws = [synth.Workload("nat", nchan, f_lo, df, synth.TSAMP, np.arange(0, 300, 3.0),
                         [1, 5, 10, 25, 50]),
          synth.Workload("ds", nchan, f_lo, df, synth.TSAMP, np.arange(300, 900, 6.0),
                         [1, 5, 25], downsample=5)]
    plans = [arts.Plan.from_workload(w) for w in ws]
    for p in plans:
        p.integration = "decimated"
    chunks = []
    for k in range(7):
        c = synth.noise((nsrc, nchan, chunk), seed=500 + k)
        c[0, :, 300 + 37 * k: 330 + 37 * k] = np.minimum(
            255, c[0, :, 300 + 37 * k: 330 + 37 * k].astype(int) + 50).astype(np.uint8)
        chunks.append(c)
    # a burst at DM 600 (a downsampled trial) sweeping across chunk boundaries, in source 1
    whole = np.concatenate(chunks, axis=2)
    d600 = O.delay_table(nchan, f_lo, df, synth.TSAMP, np.array([600.0]))[0]
    synth.add_tophat(whole[1], 6000 + d600, 40, 60)
    chunks = [whole[:, :, k * chunk:(k + 1) * chunk].copy() for k in range(len(chunks))]
    H = [p.info["downsample"] * p.info["halo"] for p in plans]
    hmax = max(H)
    full = np.concatenate([np.zeros((nsrc, nchan, hmax), np.uint8)] + chunks, axis=2)
    delays = [O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms, w.downsample) for w in ws]
    thr, found = 6.0, [0, 0]
    with arts.Stream(plans, nsrc, chunk, thr) as st:
        for k, c in enumerate(chunks):
            print("integrated stream chunk", k, flush=True)
            st.push(to_dev(c))
            cands, _ = st.wait()
            for p, w in enumerate(ws):
                oc, near = [], NearRuns()
                for b in range(nsrc):
                    rows_in = full[b][:, hmax - H[p] + k * chunk: hmax + (k + 1) * chunk]
                    if w.downsample > 1:
                        rows_in = O.downsample(rows_in, w.downsample)
                    x = O.dedisperse(rows_in, delays[p])
                    nrep = chunk // w.downsample
                    off = (k * chunk - H[p]) // w.downsample
                    t0 = min(nrep, max(0, -off))
                    if t0 == nrep:
                        continue
                    xs = x[:, t0:]
                    oc += O.candidates_integrated(xs, w.widths, nrep - t0, thr, beam=b,
                                                  t_offset=off + t0)
                    near |= near_threshold_runs(xs, w.widths, nrep - t0, thr,
                                                np.arange(x.shape[0]), beam=b,
                                                t_offset=off + t0, integration=True)
                sel = cands[cands["downsample"] == w.downsample]
                compare_candidates(sel, oc, near)
                assert all(int(c["sample"]) % int(c["width"]) == 0 for c in sel)
                found[p] += len(sel)
    assert all(f > 0 for f in found)
    for p in plans:
        p.close()


@pytest.mark.parametrize("widths,t_offset", [([1, 5, 10, 25, 50, 100, 250], 3),
                                              ([1, 3, 64, 1000], -4097)])
def test_integrated_long_rows_match_oracle(widths, t_offset):
    # rows too long to hold in LDS (searched segment by segment): cells that begin in the
    # previous segment, runs across segment boundaries, the widest width above a segment's
    # look-back of kCandSeg starts
    ndm, nrep, thr = 12, 21000, 8.0
    x = _series(ndm, nrep, widths, seed=1300 + len(widths))
    f_lo, df = synth.band(16)
    print("integrated long rows", widths, flush=True)
    with arts.Plan(16, f_lo, df, synth.TSAMP, np.arange(ndm) * 1.0, widths) as p:
        p.integration = "decimated"
        got = p.candidates(to_dev(x[None]), thr, t_offset=t_offset)
    ora = O.candidates_integrated(x, widths, nrep, thr, t_offset=t_offset)
    near = near_threshold_runs(x, widths, nrep, thr, np.arange(ndm), t_offset=t_offset,
                               integration=True)
    assert len(ora) >= 5
    assert compare_candidates(got, ora, near) > 0


def test_integrated_argument_checks():
    f_lo, df = synth.band(16)
    with arts.Plan(16, f_lo, df, synth.TSAMP, np.arange(8) * 1.0, [1, 4, 8]) as p:
        with pytest.raises(arts.ArtsError) as e:
            arts.arts_plan_set_integration(p.handle, 2)
        assert e.value.status == arts.ARTS_E_INVAL
        p.integration = "decimated"
        # a stream whose chunk (1004) is not a multiple of width 8; 1000 is
        with pytest.raises(arts.ArtsError) as e:
            arts.Stream([p], 1, 1004, 8.0)
        assert e.value.status == arts.ARTS_E_INVAL
        with arts.Stream([p], 1, 1000, 8.0):
            pass

"""GPU parity of the DM-width clustering (arts_plan_cluster and the clustered candidate searches)
against the oracle's cluster_dm_width: bit-exact on candidate lists given to both (hand-worked
fixture, random lists with S/N ties, rows longer than the LDS sort, clusters chained over many DM
trials, empty lists), and, through the searches, against the oracle applied to the unclustered
GPU list (same FP32 S/N values) or, from raw data, with the oracle's own FP64 candidates (the
cluster partition exact, the reported member the top S/N up to FP32 rounding)."""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from tests._parity import near_threshold_runs, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _records(cands, ds=1):
    a = np.zeros(len(cands), dtype=arts.CANDIDATE_DTYPE)
    for i, (b, d, w, t, s) in enumerate(cands):
        a[i] = (t, b, d, w, ds, s, 0.5 * d)
    return a


def _tuples(arr):
    """Structured candidates -> oracle tuples; the S/N is the FP32 value as a float."""
    return [(int(c["beam"]), int(c["dm_index"]), int(c["width"]), int(c["sample"]),
             float(c["snr"])) for c in arr]


def _plan(ndm=64, widths=(1, 2, 4, 8)):
    f_lo, df = synth.band(64)
    return arts.Plan(64, f_lo, df, synth.TSAMP, np.arange(ndm) * 1.0, list(widths))


def _check_exact(plan, cands, nbeam, beam_offset=0):
    got = plan.cluster_candidates(_records(cands), nbeam, beam_offset)
    f32 = [(b, d, w, t, float(np.float32(s))) for b, d, w, t, s in cands]
    reps, _ = O.cluster_dm_width(f32)
    assert _tuples(got) == sorted(reps, key=lambda r: (r[0], r[1], r[2], r[3]))
    return got


def test_cluster_golden_fixture():
    with open(os.path.join(GOLDEN, "cluster_tiny.json")) as f:
        g = json.load(f)
    p = _plan(ndm=8)
    got = _check_exact(p, [tuple(c) for c in g["candidates"]], nbeam=2)
    assert [r[:4] for r in _tuples(got)] == [tuple(r[:4]) for r in g["reps"]]


def _random_cands(rng, n, nbeam, ndm, tmax, widths=(1, 2, 4, 8, 16), snrs=None):
    keys = set()
    while len(keys) < n:
        keys.add((int(rng.integers(nbeam)), int(rng.integers(ndm)), int(rng.choice(widths)),
                  int(rng.integers(-50, tmax))))
    vals = snrs if snrs is not None else np.round(rng.uniform(6.0, 12.0, n), 1)
    return [k + (float(rng.choice(vals)),) for k in sorted(keys)]


@pytest.mark.parametrize("n,nbeam,ndm,tmax", [(0, 1, 8, 10), (1, 1, 8, 10), (40, 2, 8, 60),
                                              (3000, 4, 64, 4000), (20000, 3, 256, 3000)])
def test_cluster_random_lists_match_oracle(n, nbeam, ndm, tmax):
    rng = np.random.default_rng(n + ndm)
    p = _plan(ndm=ndm)
    cands = _random_cands(rng, n, nbeam, ndm, tmax, snrs=[6.0, 6.5, 7.0, 9.25, 11.0])
    rng.shuffle(cands)
    _check_exact(p, cands, nbeam)


def test_cluster_long_rows_and_deep_chains():
    rng = np.random.default_rng(5)
    p = _plan(ndm=512)
    cands = []
    # one row with 3000 candidates (sorted in global memory), disjoint and overlapping windows
    for t in rng.choice(40000, 3000, replace=False):
        cands.append((0, 7, int(rng.choice([1, 2, 4, 8, 16])), int(t),
                      float(rng.choice([6.0, 8.0, 10.0]))))
    # a diagonal track over all 512 DM trials: one cluster whose union-find tree is deep
    for d in range(512):
        cands.append((1, d, 4, 1000 + 2 * d, 7.0 + (d % 5) * 0.5))
    # two tracks that touch only at their ends join; a one-sample gap keeps a third apart
    cands += [(2, d, 2, 100 + d, 6.0) for d in range(0, 50)]
    cands += [(2, d, 2, 150 + d, 6.5) for d in range(50, 100)]
    cands += [(2, d, 1, 400, 9.0) for d in range(100, 140)] + [(2, 140, 1, 402, 9.0)]
    got = _check_exact(p, cands, nbeam=3)
    assert sum(1 for c in got if c["beam"] == 1) == 1


def test_cluster_beam_offset_and_invalid_records():
    p = _plan(ndm=16)
    cands = [(5, 3, 2, 10, 7.0), (5, 4, 1, 11, 8.0), (6, 3, 2, 10, 9.0)]
    got = _check_exact(p, cands, nbeam=2, beam_offset=5)
    assert len(got) == 2
    for bad in ([(7, 3, 2, 10, 7.0)], [(5, 16, 2, 10, 7.0)], [(5, 3, 0, 10, 7.0)],
                [(5, 3, 2, 10, float("nan"))]):
        with pytest.raises(arts.ArtsError) as e:
            p.cluster_candidates(_records(cands + bad), nbeam=2, beam_offset=5)
        assert e.value.status == arts.ARTS_E_INVAL


def _burst_data(ws, delays, nsamp, seed):
    data = synth.noise((ws.nchan, nsamp), seed=seed)
    for d, t0, wid, amp in [(40, 900, 6, 14), (120, 2600, 12, 9), (200, 4100, 3, 25)]:
        synth.add_tophat(data, t0 + delays[d], wid, amp)
    return data


def test_clustered_candidates_match_oracle_from_data():
    w = synth.cfg_small()
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    data = _burst_data(w, delays, int(delays.max()) + 5000, seed=17)
    p = arts.Plan.from_workload(w)
    series = p.dedisperse(to_dev(data[None]))
    x = series.cpu().numpy()[0]
    nrep = x.shape[1] - max(w.widths) + 1
    thr = 7.0
    ora = O.candidates(x, w.widths, nrep, thr)
    assert not near_threshold_runs(x, w.widths, nrep, thr, np.arange(x.shape[0]))
    raw = p.candidates(series, thr)
    assert sorted(r[:4] for r in _tuples(raw)) == sorted(c[:4] for c in ora)
    p.cluster = True
    assert p.cluster
    got = p.candidates(series, thr)
    reps, label = O.cluster_dm_width(ora)
    assert 3 <= len(reps) < len(ora) / 5
    # the partition is exact; the member reported is the cluster's best up to FP32 rounding
    where = {c[:4]: label[i] for i, c in enumerate(ora)}
    snr64 = {c[:4]: c[4] for c in ora}
    seen = set()
    for c in _tuples(got):
        k = where[c[:4]]
        assert k not in seen
        seen.add(k)
        top = reps[k][4]
        assert math.isclose(snr64[c[:4]], top, rel_tol=2e-6), (c, reps[k])
    assert seen == set(range(len(reps)))


def _stream_pair(nsrc, nbeam, table, graph):
    f_lo, df = synth.band(64)
    specs = [(np.arange(0, 300, 3.0), [1, 2, 4, 8], 1), (np.arange(300, 900, 6.0), [1, 2, 4], 4)]
    mk = lambda: [arts.Plan(64, f_lo, df, synth.TSAMP, d, w, ds) for d, w, ds in specs]
    plain, clus = mk(), mk()
    clus[0].cluster = True       # the native plan is clustered, the downsampled one is not
    kw = dict(sb_table=to_dev(table) if table is not None else None, nbeam=nbeam,
              cand_capacity=1 << 18)
    return (arts.Stream(plain, nsrc, 2400, 5.5, **kw),
            arts.Stream(clus, nsrc, 2400, 5.5, graph=graph, **kw))


def _split(arr):
    """(native-plan tuples, downsampled-plan tuples) of a stream's candidate array."""
    nat = arr["downsample"] == 1
    return sorted(_tuples(arr[nat])), sorted(_tuples(arr[~nat]))


@pytest.mark.parametrize("graph", [False, True])
def test_stream_clusters_equal_oracle_on_unclustered_list(graph):
    nsrc = 3
    table = synth.sb_table_synthetic(4, nsrc, 64)
    chunks = [synth.noise((nsrc, 64, 2400), seed=500 + k) for k in range(6)]
    for k in (2, 4):
        hot = chunks[k][1, :, 300:330].astype(int) + 50
        chunks[k][1, :, 300:330] = np.minimum(255, hot).astype(np.uint8)
    a, b = _stream_pair(nsrc, 4, table, graph)
    with a, b:
        nclus = 0
        for k, c in enumerate(chunks):
            a.push(to_dev(c))
            ca, _ = a.wait()
            b.push(to_dev(c))
            cb, _ = b.wait()
            nat_a, ds_a = _split(ca)
            nat_b, ds_b = _split(cb)
            reps, _ = O.cluster_dm_width(nat_a)
            assert nat_b == sorted(reps), k
            assert ds_b == ds_a, k
            nclus += len(reps)
        assert nclus > 0


def test_batch_clusters_one_request():
    import torch
    w = synth.cfg_small()
    p1, p2, q = (arts.Plan.from_workload(w) for _ in range(3))
    p1.cluster = True
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    data = torch.from_numpy(np.stack([_burst_data(w, delays, int(delays.max()) + 5000, seed=s)
                                      for s in (3, 4)])).cuda()
    L = arts.series_length(p1, data.shape[2])
    o1 = torch.empty((2, w.dms.size, L), dtype=torch.int32, device="cuda")
    o2 = torch.empty_like(o1)
    with arts.Batch() as bt:
        bt.dedisperse([(p1, data, o1), (p2, data, o2)])
        got = bt.candidates([(p1, data, o1), (p2, data, o2)], 7.0)
    raw1 = q.candidates(o1, 7.0)
    raw2 = q.candidates(o2, 7.0, beam_offset=2)
    reps, _ = O.cluster_dm_width(_tuples(raw1))
    g = _tuples(got)
    assert sorted(t for t in g if t[0] < 2) == sorted(reps)
    assert sorted(t for t in g if t[0] >= 2) == sorted(_tuples(raw2))


def test_clustered_capacity_counts_unclustered():
    import ctypes as C
    w = synth.cfg_small()
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
    data = _burst_data(w, delays, int(delays.max()) + 5000, seed=17)
    p = arts.Plan.from_workload(w)
    series = p.dedisperse(to_dev(data[None]))
    nraw = len(p.candidates(series, 7.0))
    p.cluster = True
    buf = np.zeros(4, dtype=arts.CANDIDATE_DTYPE)
    n = C.c_int64(0)
    st = arts.lib().arts_candidates(p.handle, series.data_ptr(), 1, series.shape[2], 7.0, 0, 0,
                                    buf.ctypes.data, 4, C.byref(n), None)
    assert st == arts.ARTS_E_CAPACITY and n.value == nraw
    assert 0 < len(p.candidates(series, 7.0, capacity=4)) < nraw  # retried with the raw count


def test_cluster_serving_scale_list():
    # a burst storm at the serving shape: 71 SBs x 2048 DM trials, AMBER-like widths 1..256,
    # 1500 events spread over up to 81 DM trials and every width, 100 000 isolated candidates
    widths = [1 << k for k in range(9)]
    b, d, w, t, s = synth.candidate_tracks(71, 2048, widths, 12500, 1500, 100000, seed=3)
    cands = list(zip(b.tolist(), d.tolist(), w.tolist(), t.tolist(), s.astype(float).tolist()))
    assert len(cands) > 600000
    print("cluster serving scale: candidates", len(cands), flush=True)
    f_lo, df = synth.band(64)
    p = arts.Plan(64, f_lo, df, synth.TSAMP, np.arange(2048) * 1.0, widths)
    got = p.cluster_candidates(_records(cands), 71)
    reps, _ = O.cluster_dm_width(cands)
    assert _tuples(got) == sorted(reps, key=lambda r: (r[0], r[1], r[2], r[3]))


# ------------------------------------------------------------------ offline (time, DM windows)
def _records7(cands):
    a = np.zeros(len(cands), dtype=arts.CANDIDATE_DTYPE)
    for i, (b, d, w, t, s, ds, dm) in enumerate(cands):
        a[i] = (t, b, d, w, ds, s, dm)
    return a


def _tuples7(arr):
    return [(int(c["beam"]), int(c["dm_index"]), int(c["width"]), int(c["sample"]),
             float(c["snr"]), int(c["downsample"]), float(c["dm"])) for c in arr]


def _check_offline(cands, t_window, edges, min_snr):
    rec = _records7(cands)
    got = arts.arts_cluster_offline(rec, t_window, edges, min_snr)
    ref = O.cluster_offline(_tuples7(rec), t_window, edges, float(np.float32(min_snr)))
    assert _tuples7(got) == ref
    return got


def test_offline_golden_fixture():
    with open(os.path.join(GOLDEN, "cluster_offline_tiny.json")) as f:
        g = json.load(f)
    got = _check_offline([tuple(c) for c in g["candidates"]], g["t_window"], g["dm_edges"],
                         g["min_snr"])
    want = [g["candidates"][i] for i in g["kept"]]
    assert [(c[0], c[1], c[3]) for c in _tuples7(got)] == [(c[0], c[1], c[3]) for c in want]


@pytest.mark.parametrize("n", [0, 1, 100, 50000])
def test_offline_random_lists_match_oracle(n):
    rng = np.random.default_rng(40 + n)
    cands = []
    for _ in range(n):
        ds = int(rng.choice([1, 2, 4, 8]))
        cands.append((int(rng.integers(71)), int(rng.integers(2048)), int(rng.choice([1, 4, 16])),
                      int(rng.integers(-20000, 600000)) // ds,
                      float(rng.choice([9.5, 10.0, 10.5, 12.0, 20.0])), ds,
                      float(rng.choice([10.0, 20.0, 21.5, 50.0, 300.0, 1200.0, 4000.0]))))
    got = _check_offline(cands, 6104, arts.offline_dm_edges(), 10.0)
    assert len(got) <= n


def test_offline_rejects_bad_input_and_reports_capacity():
    base = [(0, 0, 1, 7, 11.0, 1, 30.0), (0, 1, 1, 9000, 12.0, 1, 30.0)]
    for bad in [(0, 2, 0, 7, 11.0, 1, 30.0), (0, 2, 1, 7, 11.0, 0, 30.0),
                (0, 2, 1, 7, float("nan"), 1, 30.0), (0, 2, 1, 1 << 43, 11.0, 1, 30.0)]:
        with pytest.raises(arts.ArtsError) as e:
            arts.arts_cluster_offline(_records7(base + [bad]), 6104, [20.0], 10.0)
        assert e.value.status == arts.ARTS_E_INVAL
    for edges in ([20.0, 20.0], [30.0, 20.0], []):
        with pytest.raises(arts.ArtsError):
            arts.arts_cluster_offline(_records7(base), 6104, edges, 10.0)
    with pytest.raises(arts.ArtsError) as e:
        arts.arts_cluster_offline(_records7(base), 6104, [20.0], 10.0, capacity=1)
    assert e.value.status == arts.ARTS_E_CAPACITY


def test_offline_after_streamed_dm_width_clusters():
    # the paper's chain: per-chunk DM-width clusters from the stream, then the whole observation
    # clustered over 0.5 s windows and widening DM windows, DM >= 20 and S/N >= 10
    nsrc = 3
    table = synth.sb_table_synthetic(4, nsrc, 64)
    chunks = [synth.noise((nsrc, 64, 2400), seed=700 + k) for k in range(8)]
    for k in (3, 5, 6):
        hot = chunks[k][k % nsrc, :, 500:540].astype(int) + 70
        chunks[k][k % nsrc, :, 500:540] = np.minimum(255, hot).astype(np.uint8)
    _, b = _stream_pair(nsrc, 4, table, graph=False)
    allc = []
    with b:
        for c in chunks:
            b.push(to_dev(c))
            allc.append(b.wait()[0])
    allc = np.concatenate(allc)
    assert len(allc) > 0
    got = arts.arts_cluster_offline(allc, 6104, arts.offline_dm_edges(), 10.0)
    ref = O.cluster_offline(_tuples7(allc), 6104, list(arts.offline_dm_edges()), 10.0)
    assert _tuples7(got) == ref


def test_server_stream_with_clustered_plan_equals_standalone():
    # a clustered plan served beside another stream reports what a standalone stream reports
    nsrc, chunk = 3, 2400
    table = synth.sb_table_synthetic(4, nsrc, 64)
    chunks = [synth.noise((nsrc, 64, chunk), seed=800 + k) for k in range(5)]
    for k in (2, 3):
        hot = chunks[k][0, :, 700:740].astype(int) + 60
        chunks[k][0, :, 700:740] = np.minimum(255, hot).astype(np.uint8)
    _, st = _stream_pair(nsrc, 4, table, graph=False)
    f_lo, df = synth.band(64)
    served_plans = [arts.Plan(64, f_lo, df, synth.TSAMP, np.arange(0, 300, 3.0), [1, 2, 4, 8]),
                    arts.Plan(64, f_lo, df, synth.TSAMP, np.arange(300, 900, 6.0), [1, 2, 4], 4)]
    served_plans[0].cluster = True
    other = arts.Plan(64, f_lo, df, synth.TSAMP, np.arange(0, 100, 1.0), [1, 2])
    with st, arts.Server(8 << 30) as srv:
        a = srv.open(served_plans, nsrc, chunk, 5.5, sb_table=to_dev(table), nbeam=4,
                     cand_capacity=1 << 18)
        b = srv.open([other], 1, chunk, 6.0)
        for k, c in enumerate(chunks):
            srv.submit(a, to_dev(c))
            srv.submit(b, to_dev(c[:1]))
            assert srv.tick() == 2
            got, _ = srv.collect(a)
            srv.collect(b)
            st.push(to_dev(c))
            ref, _ = st.wait()
            assert sorted(_tuples(got)) == sorted(_tuples(ref)), k

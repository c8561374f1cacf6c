"""GPU parity of two-step subband dedispersion: bit-exact against the oracle's subband_dedisperse
for small plans (both fine-trial counts, ragged last coarse group, every step-1 tiling, SB
formation in step 1), in a stream (zero history, one-shot oracle on the concatenation), in a
batch, and at the full size of the ALERT plan for one GPU (1536 channels, 32 subbands, DM 0 to
409.6 in steps of 0.2, subbanding step 6.4) on every output of one beam."""
import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from tests._parity import compare_candidates, near_threshold_runs, to_dev

pytestmark = pytest.mark.gpu


def _plan_and_oracle(nchan, nsub, nfine, ndm, dm_first=0.0, dm_step=0.5, widths=(1, 2, 4, 8)):
    f_lo, df = synth.band(nchan)
    p = arts.Plan.subband(nchan, f_lo, df, synth.TSAMP, dm_first, dm_step, ndm, nfine, nsub,
                          widths)
    fine, coarse, d1, d2 = O.subband_plan(nchan, f_lo, df, synth.TSAMP, dm_first, dm_step, ndm,
                                          nfine, nsub)
    return p, (fine, coarse, d1, d2)


@pytest.mark.parametrize("nfine,ndm", [(32, 64), (16, 64), (32, 50), (16, 37)])
def test_subband_small_matches_oracle(nfine, ndm):
    p, (fine, coarse, d1, d2) = _plan_and_oracle(96, 8, nfine, ndm)
    info = p.subband_info()
    assert info["nsub"] == 8 and info["nfine"] == nfine and info["ncoarse"] == coarse.size
    assert info["max_delay1"] == int(d1.max()) and info["max_delay2"] == int(d2.max())
    comp = d1[np.arange(ndm) // nfine] + np.repeat(d2, 12, axis=1)
    assert np.array_equal(p.delays(), comp)
    assert p.max_delay == int(d1.max()) + int(d2.max())
    rng = np.random.default_rng(nfine + ndm)
    nin = p.max_delay + 2500 + int(rng.integers(0, 7))
    data = rng.integers(0, 256, size=(2, 96, nin), dtype=np.uint8)
    got = p.dedisperse(to_dev(data)).cpu().numpy()
    for b in range(2):
        assert np.array_equal(got[b], O.subband_dedisperse(data[b], d1, d2, nfine)), b


def test_subband_step1_tilings_agree():
    p, (fine, coarse, d1, d2) = _plan_and_oracle(144, 12, 32, 96, dm_first=20.0, dm_step=1.0)
    data = synth.noise((1, 144, p.max_delay + 3001), seed=5)
    ref = O.subband_dedisperse(data[0], d1, d2, 32)
    desc = {v: arts.arts_tiling_describe(v) for v in range(arts.arts_tiling_count())}
    for v, d in desc.items():
        if "SPD=4" in d and not d.endswith(" framed"):
            p.set_tiling(v)
            assert p.tiling() == v
            assert np.array_equal(p.dedisperse(to_dev(data)).cpu().numpy()[0], ref), v
        else:                       # 16-bit and (per-chunk) framed tilings cannot run step 1
            with pytest.raises(arts.ArtsError):
                p.set_tiling(v)


def test_subband_fused_sb_formation():
    nchan, nsub = 96, 8
    p, (fine, coarse, d1, d2) = _plan_and_oracle(nchan, nsub, 32, 64)
    tab = synth.noise((4, nchan, p.max_delay + 2200), seed=8)
    table = synth.sb_table_synthetic(9, 4, nchan)
    got = p.dedisperse_sb(to_dev(tab), to_dev(table)).cpu().numpy()
    sb = O.sb_synthesize(tab, table)
    for s in range(9):
        assert np.array_equal(got[s], O.subband_dedisperse(sb[s], d1, d2, 32)), s


def test_subband_candidates_with_burst():
    nchan, nsub = 128, 8
    p, (fine, coarse, d1, d2) = _plan_and_oracle(nchan, nsub, 32, 128, dm_step=0.5,
                                                 widths=(1, 2, 4, 8, 16))
    brute = O.delay_table(nchan, *synth.band(nchan), synth.TSAMP, fine)
    data = synth.noise((nchan, p.max_delay + 6000), seed=31)
    synth.add_tophat(data, 2000 + brute[70], 8, 12)
    x = O.subband_dedisperse(data, d1, d2, 32)
    series = p.dedisperse(to_dev(data[None]))
    assert np.array_equal(series.cpu().numpy()[0], x)
    nrep = x.shape[1] - 15
    ora = O.candidates(x, [1, 2, 4, 8, 16], nrep, 8.0)
    near = near_threshold_runs(x, [1, 2, 4, 8, 16], nrep, 8.0, np.arange(x.shape[0]))
    got = p.candidates(series, 8.0)
    assert len(ora) > 0
    compare_candidates(got, ora, near)


def test_subband_in_stream_matches_one_shot():
    nchan, nsub, chunk = 64, 8, 2400
    f_lo, df = synth.band(nchan)
    p = arts.Plan.subband(nchan, f_lo, df, synth.TSAMP, 0.0, 1.0, 64, 32, nsub, [1, 2, 4])
    _, _, d1, d2 = O.subband_plan(nchan, f_lo, df, synth.TSAMP, 0.0, 1.0, 64, 32, nsub)
    H = p.halo
    chunks = [synth.noise((2, nchan, chunk), seed=60 + k) for k in range(4)]
    full = np.concatenate([np.zeros((2, nchan, H), np.uint8)] + chunks, axis=2)
    with arts.Stream([p], 2, chunk, 6.0) as st:
        for k, c in enumerate(chunks):
            st.push(to_dev(c))
            st.wait()
            got = st.series(0).cpu().numpy()
            for b in range(2):
                win = full[b][:, k * chunk: H + (k + 1) * chunk]
                assert np.array_equal(got[b], O.subband_dedisperse(win, d1, d2, 32)), (k, b)


def test_subband_in_batch_equals_plan_call():
    import torch
    p, _ = _plan_and_oracle(96, 8, 16, 48)
    q = arts.Plan.from_workload(synth.cfg_small())
    rng = np.random.default_rng(2)
    d1 = torch.from_numpy(rng.integers(0, 256, (2, 96, p.max_delay + 1700), dtype=np.uint8)).cuda()
    d2 = torch.from_numpy(rng.integers(0, 256, (1, 128, 9000), dtype=np.uint8)).cuda()
    o1 = torch.empty((2, 48, arts.series_length(p, d1.shape[2])), dtype=torch.int32,
                     device="cuda")
    o2 = torch.empty((1, q.info["ndm"], arts.series_length(q, 9000)), dtype=torch.int32,
                     device="cuda")
    with arts.Batch() as b:
        st = b.dedisperse([(p, d1, o1), (q, d2, o2)])
    assert list(st) == [arts.ARTS_OK, arts.ARTS_OK]
    assert torch.equal(o1, p.dedisperse(d1))
    assert torch.equal(o2, q.dedisperse(d2))


def test_subband_alert_plan_full_size():
    # ALERT GPU 1 (Table "dedispersion setup"): DM 0-409.6 step 0.2, subbanding step 6.4
    nchan = 1536
    f_lo, df = synth.band(nchan)
    p = arts.Plan.subband(nchan, f_lo, df, synth.TSAMP, 0.0, 0.2, 2048, 32, 32,
                          [1 << k for k in range(9)])
    fine, coarse, d1, d2 = O.subband_plan(nchan, f_lo, df, synth.TSAMP, 0.0, 0.2, 2048, 32, 32)
    assert coarse.size == 64
    nin = synth.CHUNK + p.halo
    data = synth.noise((1, nchan, nin), seed=77)
    print("subband full size: nin", nin, flush=True)
    got = p.dedisperse(to_dev(data)).cpu().numpy()[0]
    ref = O.subband_dedisperse(data[0], d1, d2, 32)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


def _sub_stream_setup(chunk, ndm=64, dm_step=5.0):
    nchan, nsub = 64, 8
    f_lo, df = synth.band(nchan)
    p = arts.Plan.subband(nchan, f_lo, df, synth.TSAMP, 0.0, dm_step, ndm, 32, nsub, [1, 2, 4])
    _, _, d1, d2 = O.subband_plan(nchan, f_lo, df, synth.TSAMP, 0.0, dm_step, ndm, 32, nsub)
    return nchan, p, d1, d2


def test_subband_stream_history_longer_than_chunk():
    # the step-1 rows carried between chunks span several chunks (halo > 2 chunks)
    chunk = 1000
    nchan, p, d1, d2 = _sub_stream_setup(chunk)
    H = p.halo
    assert H > 2 * chunk
    chunks = [synth.noise((1, nchan, chunk), seed=200 + k) for k in range(7)]
    full = np.concatenate([np.zeros((1, nchan, H), np.uint8)] + chunks, axis=2)
    with arts.Stream([p], 1, chunk, 6.0) as st:
        for k, c in enumerate(chunks):
            st.push(to_dev(c))
            st.wait()
            win = full[0][:, k * chunk: H + (k + 1) * chunk]
            assert np.array_equal(st.series(0).cpu().numpy()[0],
                                  O.subband_dedisperse(win, d1, d2, 32)), k


def test_subband_stream_restore_and_graph():
    import torch
    chunk = 1200
    nchan, p, d1, d2 = _sub_stream_setup(chunk)
    chunks = [synth.noise((2, nchan, chunk), seed=300 + k) for k in range(8)]
    ref = []
    with arts.Stream([p], 2, chunk, 6.0) as st:
        for k, c in enumerate(chunks):
            st.push(to_dev(c))
            st.wait()
            ref.append(st.series(0).cpu().numpy().copy())
            if k == 3:
                snap, n = st.snapshot()
    # resumed from the snapshot: the step-1 rows are recomputed on the first push
    with arts.Stream([p], 2, chunk, 6.0) as st2:
        st2.restore(snap, n)
        for j, c in enumerate(chunks[4:]):
            st2.push(to_dev(c))
            st2.wait()
            assert np.array_equal(st2.series(0).cpu().numpy(), ref[4 + j]), j
    # graph replay (graphs from the first warm chunk on), with eager work between replays
    with arts.Stream([p], 2, chunk, 6.0, graph=True) as st3:
        for k, c in enumerate(chunks):
            st3.push(to_dev(c))
            st3.wait()
            torch.cuda.synchronize()
            _ = (torch.ones(1000, device="cuda") * 2).sum().item()
            assert np.array_equal(st3.series(0).cpu().numpy(), ref[k]), k


def test_subband_stream_in_server_equals_standalone():
    # the serving engine advances the step-1 window of a subband stream like arts_stream_push,
    # also while a native stream shares its ticks; compaction happens every m + 1 chunks
    chunk = 1000
    nchan, p, d1, d2 = _sub_stream_setup(chunk)
    f_lo, df = synth.band(nchan)
    q = arts.Plan(nchan, f_lo, df, synth.TSAMP, np.arange(0, 100, 2.0), [1, 2, 4])
    chunks = [synth.noise((2, nchan, chunk), seed=400 + k) for k in range(9)]
    with arts.Server(8 << 30) as srv:
        a = srv.open([p], 2, chunk, 6.0)
        b = srv.open([q], 1, chunk, 6.0)
        served = []
        for k, c in enumerate(chunks):
            srv.submit(a, to_dev(c))
            srv.submit(b, to_dev(c[:1]))
            assert srv.tick() == 2
            ca, _ = srv.collect(a)
            srv.collect(b)
            served.append((srv.series(a, 0).cpu().numpy().copy(), ca))
    p2, _ = _plan_and_oracle(nchan, 8, 32, 64, dm_step=5.0, widths=(1, 2, 4))
    H = p2.halo
    full = np.concatenate([np.zeros((2, nchan, H), np.uint8)] + chunks, axis=2)
    with arts.Stream([p2], 2, chunk, 6.0) as st:
        for k, c in enumerate(chunks):
            st.push(to_dev(c))
            cands, _ = st.wait()
            got = st.series(0).cpu().numpy()
            assert np.array_equal(got, served[k][0]), k
            assert np.array_equal(cands, served[k][1]), k
            win = full[0][:, k * chunk: H + (k + 1) * chunk]
            assert np.array_equal(got[0], O.subband_dedisperse(win, d1, d2, 32)), k


def test_subband_stream_chunk_multiple_of_four():
    nchan, p, _, _ = _sub_stream_setup(1000)
    with pytest.raises(arts.ArtsError) as e:
        arts.Stream([p], 1, 1002, 6.0)
    assert e.value.status == arts.ARTS_E_INVAL

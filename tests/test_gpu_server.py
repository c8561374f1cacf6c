"""GPU tests of the continuous-batching serving engine: a stream's series and candidates are the
same alone and in a mix of streams of other shapes that join and leave, they equal a standalone
arts_stream fed the same chunks, and admission follows the HBM budget."""
import numpy as np
import pytest

from paper_2205_12362_amd import arts, synth
from tests._parity import to_dev

pytestmark = pytest.mark.gpu


def _spec(nchan, dms, widths, D, chunk):
    f_lo, df = synth.band(nchan)
    return synth.Workload(f"n{nchan}", nchan, f_lo, df, synth.TSAMP, np.asarray(dms, float),
                          widths, downsample=D)


def _stream_a():
    # both plans search their whole chunk from chunk 3 on (a partial search in chunks 1 and 2)
    ws = [_spec(64, np.arange(0, 300, 3.0), [1, 2, 4, 8], 1, 2400),
          _spec(64, np.arange(300, 600, 3.0), [1, 2, 4], 4, 2400)]
    return ws, 3, 2400


def _chunks(nsrc, nchan, chunk, n, seed):
    out = []
    for k in range(n):
        c = synth.noise((nsrc, nchan, chunk), seed=seed + k)
        c[0, :, 50 + 7 * k: 90 + 7 * k] = 200
        out.append(c)
    return out


def _run_server(with_others):
    ws, nsrc, chunk = _stream_a()
    chunks = _chunks(nsrc, 64, chunk, 6, seed=300)
    res = []
    with arts.Server(8 << 30) as srv:
        pa = [arts.Plan.from_workload(w) for w in ws]
        a = srv.open(pa, nsrc, chunk, 6.0)
        others = []
        if with_others:
            wb = _spec(128, np.arange(0, 100, 0.5), [1, 2, 4], 1, 2000)
            pb = [arts.Plan.from_workload(wb)]
            b = srv.open(pb, 2, 2000, 7.0)
            others.append((b, 2, 128, 2000))
        for k, c in enumerate(chunks):
            srv.submit(a, to_dev(c))
            if with_others and k == 2:   # a third stream joins mid-way ...
                wc = _spec(96, np.arange(0, 400, 4.0), [1, 4, 16], 2, 1000)
                pc = [arts.Plan.from_workload(wc)]
                cid = srv.open(pc, 1, 1000, 6.5)
                others.append((cid, 1, 96, 1000))
            if with_others and k == 4:   # ... and the second leaves
                srv.close_stream(others[0][0])
                others = others[1:]
            for (oid, on, onc, ochunk) in others:
                srv.submit(oid, to_dev(synth.noise((on, onc, ochunk), seed=900 + k)))
            n = srv.tick()
            assert n == 1 + len(others)
            cands, idx = srv.collect(a)
            assert idx == k
            for (oid, *_rest) in others:
                srv.collect(oid)
            res.append(([srv.series(a, p).cpu().numpy().copy() for p in range(2)], cands))
    return res


def test_server_same_alone_and_in_mix():
    alone = _run_server(False)
    mixed = _run_server(True)
    for (sa, ca), (sm, cm) in zip(alone, mixed):
        for p in range(2):
            assert np.array_equal(sa[p], sm[p])
        assert np.array_equal(ca, cm)
    assert sum(len(c) for _, c in alone) > 0


def test_server_equals_standalone_stream():
    ws, nsrc, chunk = _stream_a()
    chunks = _chunks(nsrc, 64, chunk, 6, seed=300)
    served = _run_server(False)
    plans = [arts.Plan.from_workload(w) for w in ws]
    with arts.Stream(plans, nsrc, chunk, 6.0) as st:
        for (ss, cs), c in zip(served, chunks):
            st.push(to_dev(c))
            cands, _ = st.wait()
            for p in range(2):
                assert np.array_equal(st.series(p).cpu().numpy(), ss[p])
            assert np.array_equal(cands, cs)


def test_server_admission_budget():
    ws, nsrc, chunk = _stream_a()
    plans = [arts.Plan.from_workload(w) for w in ws]
    with arts.Server(1 << 30) as probe:
        sid = probe.open(plans, nsrc, chunk, 6.0)
        one = probe.info()["used_bytes"]
        probe.close_stream(sid)
        assert probe.info()["used_bytes"] == 0
    with arts.Server(int(one * 1.5)) as srv:
        a = srv.open(plans, nsrc, chunk, 6.0)
        with pytest.raises(arts.ArtsError) as e:
            srv.open(plans, nsrc, chunk, 6.0)        # a second copy does not fit
        assert e.value.status == arts.ARTS_E_BUDGET
        srv.close_stream(a)
        b = srv.open(plans, nsrc, chunk, 6.0)        # admitted once memory is free
        srv.submit(b, to_dev(np.zeros((nsrc, 64, chunk), np.uint8)))
        with pytest.raises(arts.ArtsError) as e:
            srv.submit(b, to_dev(np.zeros((nsrc, 64, chunk), np.uint8)))
        assert e.value.status == arts.ARTS_E_STATE
        srv.tick()
        srv.collect(b)


def test_server_overlapping_ticks_same_results():
    # a chunk submitted while another stream's tick is still in flight is stepped at once (on
    # the other compute lane) and both streams' results equal standalone streams; with one lane
    # the same calls give the same results.  The big stream's chunks come from pinned host
    # memory (the asynchronous copy path).
    import torch
    ws, nsrc, chunk = _stream_a()
    wb = _spec(128, np.arange(0, 100, 0.5), [1, 2, 4], 1, 2000)
    chunks_a = _chunks(nsrc, 64, chunk, 6, seed=310)
    chunks_b = [synth.noise((2, 128, 2000), seed=950 + k) for k in range(6)]
    out = {}
    for lanes in (2, 1):
        res_a, res_b = [], []
        with arts.Server(8 << 30) as srv:
            srv.set_lanes(lanes)
            pa = [arts.Plan.from_workload(w) for w in ws]
            pb = [arts.Plan.from_workload(wb)]
            a = srv.open(pa, nsrc, chunk, 6.0)
            b = srv.open(pb, 2, 2000, 7.0)
            assert srv.poll(a) and srv.poll(b)       # nothing in flight
            for k in range(6):
                host = torch.from_numpy(chunks_a[k]).pin_memory()
                srv.submit(a, host)
                assert not srv.poll(a)               # submitted, not yet stepped
                assert srv.tick() == 1
                srv.submit(b, to_dev(chunks_b[k]))   # while a's step may still run
                assert srv.tick() == 1
                # collect in the order they finish, polling
                left = {a, b}
                while left:
                    for sid in list(left):
                        if srv.poll(sid):
                            cands, idx = srv.collect(sid)
                            assert idx == k
                            ser = [srv.series(sid, p).cpu().numpy().copy()
                                   for p in range(2 if sid == a else 1)]
                            (res_a if sid == a else res_b).append((ser, cands))
                            left.discard(sid)
                del host
        out[lanes] = (res_a, res_b)
    # standalone streams fed the same chunks
    for which, (wl, ns, ch, thr, chunks) in enumerate(((ws, nsrc, chunk, 6.0, chunks_a),
                                                       ([wb], 2, 2000, 7.0, chunks_b))):
        plans = [arts.Plan.from_workload(w) for w in wl]
        with arts.Stream(plans, ns, ch, thr) as st:
            for k, c in enumerate(chunks):
                st.push(to_dev(c))
                cands, _ = st.wait()
                for lanes in (2, 1):
                    ser, cs = out[lanes][which][k]
                    for p in range(len(plans)):
                        assert np.array_equal(st.series(p).cpu().numpy(), ser[p]), (lanes, k, p)
                    assert np.array_equal(cands, cs), (lanes, k)


def test_server_poll_and_lane_arguments():
    with arts.Server(1 << 30) as srv:
        with pytest.raises(arts.ArtsError) as e:
            srv.set_lanes(3)
        assert e.value.status == arts.ARTS_E_INVAL
        with pytest.raises(arts.ArtsError) as e:
            srv.poll(12345)
        assert e.value.status == arts.ARTS_E_INVAL

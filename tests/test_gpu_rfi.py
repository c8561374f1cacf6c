"""GPU parity of RFI mitigation (arts_rfi_clean, arts_stream_set_rfi) against the oracle's
rfi_time_domain / rfi_freq_domain / rfi_clean: bit-exact cleaned data on the hand-worked fixture
and on noise with injected RFI (zero-DM spikes, narrow-band spikes, dropouts, a persistently hot
channel, a dispersed burst), each filter alone and both, at a small size and at the full chunk of
the serving stream (12 TABs x 1536 channels x 12 500 samples).  Both sides decide the cuts
exactly, so the data must agree byte for byte.  In a stream, each pushed chunk is cleaned before
it is searched, which equals the oracle's dedispersion of the concatenated cleaned chunks."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from tests._parity import to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _inject(x, seed):
    """Zero-DM spikes, narrow-band spikes, a dropout and a hot channel in every row."""
    rng = np.random.default_rng(seed)
    nrow, nchan, nsamp = x.shape
    for r in range(nrow):
        for t in rng.integers(0, nsamp, 3):
            x[r, :, t] = np.minimum(255, x[r, :, t].astype(int) + int(rng.integers(40, 90)))
        for t in rng.integers(0, nsamp, 5):
            x[r, rng.integers(0, nchan, 2), t] = 255
        x[r, :, int(rng.integers(0, nsamp))] = 0
        c = int(rng.integers(0, nchan))
        x[r, c] = np.minimum(255, x[r, c].astype(int) + 70)
    return x


def _oracle(x, kt, kf, nt, nf):
    out = []
    for row in x:
        y = O.rfi_time_domain(row, kt, nt) if nt else row
        y = O.rfi_freq_domain(y, kf, nf) if nf else y
        out.append(y)
    return np.stack(out)


def test_rfi_golden_fixture():
    with open(os.path.join(GOLDEN, "rfi_tiny.json")) as f:
        g = json.load(f)
    t = to_dev(np.array([g["time"]["data"]], np.uint8))
    arts.arts_rfi_clean(t, g["time"]["k"], 0.0, niter_freq=0)
    assert np.array_equal(t.cpu().numpy()[0], np.array(g["time"]["clean"]))
    f = to_dev(np.array([g["freq"]["data"]], np.uint8))
    arts.arts_rfi_clean(f, 0.0, g["freq"]["k"], niter_time=0)
    assert np.array_equal(f.cpu().numpy()[0], np.array(g["freq"]["clean"]))


@pytest.mark.parametrize("nt,nf", [(3, 0), (0, 3), (3, 3), (1, 2)])
def test_rfi_small_matches_oracle(nt, nf):
    x = _inject(synth.noise((3, 96, 3001), seed=11), seed=12)
    ref = _oracle(x, 5.0, 4.5, nt, nf)
    d = to_dev(x)
    arts.arts_rfi_clean(d, 5.0, 4.5, niter_time=nt, niter_freq=nf)
    got = d.cpu().numpy()
    assert np.array_equal(got, ref)
    assert (got != x).sum() > 0


def test_rfi_pitch_and_odd_sizes():
    # rows of 1000 samples inside a pitch of 1003, 257 channels: the padding is not touched
    x = _inject(synth.noise((2, 257, 1003), seed=21), seed=22)
    ref = _oracle(x[:, :, :1000], 4.0, 4.0, 3, 3)
    d = to_dev(x)
    arts.arts_rfi_clean(d, 4.0, 4.0, nsamp=1000)
    got = d.cpu().numpy()
    assert np.array_equal(got[:, :, :1000], ref)
    assert np.array_equal(got[:, :, 1000:], x[:, :, 1000:])


def test_rfi_full_chunk_matches_oracle():
    print("rfi full chunk: 12 x 1536 x 12500", flush=True)
    x = _inject(synth.noise((12, 1536, synth.CHUNK), seed=31), seed=32)
    ref = _oracle(x, 6.0, 5.0, 3, 3)
    d = to_dev(x)
    arts.arts_rfi_clean(d, 6.0, 5.0)
    assert np.array_equal(d.cpu().numpy(), ref)


def test_rfi_rejects_bad_arguments():
    d = to_dev(np.zeros((1, 8, 64), np.uint8))
    for kw in (dict(k_time=-1.0, k_freq=1.0), dict(k_time=float("nan"), k_freq=1.0),
               dict(k_time=1.0, k_freq=1.0, niter_time=-1)):
        with pytest.raises(arts.ArtsError) as e:
            arts.arts_rfi_clean(d, **kw)
        assert e.value.status == arts.ARTS_E_INVAL
    big = to_dev(np.zeros((1, 4097, 16), np.uint8))
    with pytest.raises(arts.ArtsError):
        arts.arts_rfi_clean(big, 3.0, 3.0)
    arts.arts_rfi_clean(big, 3.0, 3.0, niter_freq=0)   # the time domain has no channel limit


@pytest.mark.parametrize("graph", [False, True])
def test_stream_cleans_each_chunk(graph):
    nchan, chunk, nsrc = 64, 2400, 2
    f_lo, df = synth.band(nchan)
    w = synth.Workload("nat", nchan, f_lo, df, synth.TSAMP, np.arange(0, 200, 2.0), [1, 2, 4])
    p = arts.Plan.from_workload(w)
    delays = O.delay_table(nchan, f_lo, df, synth.TSAMP, w.dms)
    chunks = [_inject(synth.noise((nsrc, nchan, chunk), seed=60 + k), seed=70 + k)
              for k in range(5)]
    clean = [_oracle(c, 5.0, 4.5, 3, 3) for c in chunks]
    H = p.halo
    full = np.concatenate([np.zeros((nsrc, nchan, H), np.uint8)] + clean, axis=2)
    with arts.Stream([p], nsrc, chunk, 6.0, graph=graph) as st:
        st.set_rfi(5.0, 4.5)
        for k, c in enumerate(chunks):
            st.push(to_dev(c))
            st.wait()
            got = st.series(0).cpu().numpy()
            for b in range(nsrc):
                win = full[b][:, k * chunk: H + (k + 1) * chunk]
                assert np.array_equal(got[b], O.dedisperse(win, delays)), (k, b)
            if k == 2:
                st.set_rfi(0.0, 0.0, 0, 0)   # cleaning off from chunk 3 on
                clean[3] = chunks[3]
                clean[4] = chunks[4]
                full = np.concatenate([np.zeros((nsrc, nchan, H), np.uint8)] + clean, axis=2)


def test_server_stream_cleans_like_a_standalone_stream():
    # RFI mitigation set on a served stream (through its stream handle) acts as on its own
    import ctypes as C
    nchan, chunk, nsrc = 64, 2400, 2
    f_lo, df = synth.band(nchan)
    mk = lambda: arts.Plan(nchan, f_lo, df, synth.TSAMP, np.arange(0, 200, 2.0), [1, 2, 4])
    p1, p2 = mk(), mk()
    chunks = [_inject(synth.noise((nsrc, nchan, chunk), seed=160 + k), seed=170 + k)
              for k in range(4)]
    with arts.Server(8 << 30) as srv, arts.Stream([p2], nsrc, chunk, 6.0) as st:
        a = srv.open([p1], nsrc, chunk, 6.0)
        h = C.c_void_p()
        arts._check(arts.lib().arts_server_stream(srv.handle, a, C.byref(h)))
        arts._check(arts.lib().arts_stream_set_rfi(h, 5.0, 3, 4.5, 3))
        st.set_rfi(5.0, 4.5)
        for c in chunks:
            srv.submit(a, to_dev(c))
            srv.tick()
            got, _ = srv.collect(a)
            st.push(to_dev(c))
            ref, _ = st.wait()
            assert np.array_equal(srv.series(a, 0).cpu().numpy(), st.series(0).cpu().numpy())
            assert np.array_equal(got, ref)

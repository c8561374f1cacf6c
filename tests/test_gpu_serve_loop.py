"""GPU run of the real-time serving loop (serve.serve over the engine).  A 384-channel stream
with bursts is served twice: once with the default tilings, and once with its plan autotuned at
admission (tune cache in a temporary file).  Tiling never changes a sum, so both runs must give
the same candidates, chunk by chunk.  The latency ledger must cover every chunk."""
import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from paper_2205_12362_amd.serve import DeviceBackend, StreamSpec, serve

pytestmark = pytest.mark.gpu


def _spec():
    nchan, chunk = 384, 6250
    f_lo, df = synth.band(nchan)
    w = synth.Workload("b384", nchan, f_lo, df, synth.TSAMP, np.linspace(0.0, 500.0, 512),
                       [1, 2, 4, 8, 16])
    delays = O.delay_table(nchan, f_lo, df, synth.TSAMP, w.dms)
    pool = []
    for i in range(2):
        bursts, _ = synth.random_bursts(delays, chunk, seed=40 + i, n=3, dm_range=(50, 450),
                                        dms=w.dms, snr_range=(15.0, 30.0),
                                        width_range=(1.0, 8.0), margin=200)
        pool.append(synth.noise((1, nchan, chunk), seed=31 + i, bursts=bursts))
    return StreamSpec("b384", [w], 1, chunk, pool)


def test_serve_loop_autotuned_plans_same_candidates(tmp_path):
    cache = str(tmp_path / "tune.txt")
    runs = {}
    for mode, backend in (("default", DeviceBackend()),
                          ("tuned", DeviceBackend(tune_reps=1, tune_cache=cache))):
        spec = _spec()
        print(mode, flush=True)
        res = serve([spec], 1.6, 4 << 30, backend=backend, keep_results=True)
        assert res["b384"]["chunks"] == 3 == len(spec.results)
        assert len(spec.book.latencies) == 3
        runs[mode] = (res, spec.results)
    tuned = runs["tuned"][0]["_autotuned"]["b384/b384"]
    v, nbuf, cc = tuned["shape"]
    assert "SPD=4" in arts.arts_tiling_describe(v) and nbuf in (1, 2) and cc >= 1
    assert "_autotuned" not in runs["default"][0]
    assert len(open(cache).read().splitlines()) == 1
    total = 0
    for a, b in zip(runs["default"][1], runs["tuned"][1]):
        assert np.array_equal(a, b)
        total += len(a)
    assert total > 0  # the bursts are found

"""CPU checks of the serving loop's late-chunk ledger (serve.LatencyBook): latencies are receipt
minus release, a chunk is late only when its latency exceeds the deadline, and the summary's
percentiles follow the recorded values."""
import numpy as np
import pytest

from paper_2205_12362_amd.serve import LatencyBook, contention_specs
from paper_2205_12362_amd import synth


def test_late_chunks_counted_against_the_deadline():
    b = LatencyBook(0.5)                       # binary-exact times below
    assert b.record(10.0, 10.125) == 0.125
    assert b.record(11.0, 11.5) == 0.5         # exactly at the deadline: on time
    b.record(12.0, 12.75)                      # 0.75 s: late
    b.record(13.0, 13.0625)
    s = b.summary()
    assert s["chunks"] == 4 and s["late"] == 1
    assert s["max_ms"] == 750.0
    lat = np.array([0.125, 0.5, 0.75, 0.0625]) * 1e3
    assert s["p50_ms"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_ms"] == pytest.approx(np.percentile(lat, 99))
    assert s["deadline_ms"] == 500.0


def test_book_rejects_bad_input():
    with pytest.raises(ValueError):
        LatencyBook(0.0)
    b = LatencyBook(0.5)
    with pytest.raises(ValueError):
        b.record(2.0, 1.0)
    assert b.summary()["chunks"] == 0 and b.summary()["p99_ms"] is None


def test_contention_releases_fall_inside_the_big_step():
    # every second release of each small stream lands 30 / 60 ms after a 1.024 s boundary,
    # i.e. while the 71-SB stream's step (released at that boundary) runs
    specs = contention_specs()
    big, small = specs[0], specs[1:]
    assert big.chunk * synth.TSAMP == pytest.approx(1.024)
    for s, off in zip(small, (0.030, 0.060)):
        rel = [s.start + (k + 1) * s.chunk * synth.TSAMP for k in range(8)]
        inside = [r for r in rel if 0.0 < (r % 1.024) < 0.1]
        assert len(inside) == 4
        assert all((r % 1.024) == pytest.approx(off, abs=1e-9) for r in inside)


class _InstantEngine:
    """Host stand-in for the serving engine: a submitted chunk is done as soon as it is ticked."""

    def __init__(self):
        self.ids, self.state = 0, {}

    def set_lanes(self, n):
        assert n in (1, 2)

    def open(self, plans, nsrc, chunk, threshold, sb_table=None, cand_capacity=0):
        self.ids += 1
        self.state[self.ids] = "idle"
        return self.ids

    def submit(self, sid, chunk):
        assert self.state[sid] == "idle", "one chunk in flight per stream"
        self.state[sid] = "ready"

    def tick(self):
        for sid, st in self.state.items():
            if st == "ready":
                self.state[sid] = "done"

    def poll(self, sid):
        return self.state[sid] in ("done", "idle")

    def collect(self, sid):
        self.state[sid] = "idle"
        return np.zeros(0), 0

    def close(self):
        pass


class _HostBackend:
    def plans(self, spec):
        return [None for _ in spec.workloads]

    def host_chunk(self, a):
        return a

    def table(self, t):
        return t

    def server(self, budget_bytes):
        return _InstantEngine()


def test_slow_producer_chunks_counted_late():
    # chunks of 1250 samples (0.1024 s) on a host engine that finishes at once: only the chunk
    # whose producer hands it over 0.15 s after its release misses its one-chunk deadline; the
    # next one, handed over on time, is stepped as soon as the late one has been collected
    from paper_2205_12362_amd.serve import StreamSpec, serve
    chunk = 1250
    spec = StreamSpec("slow", [None], 1, chunk, [np.zeros((1, 4, chunk), np.uint8)])
    delay = lambda name, k: 0.15 if (name, k) == ("slow", 2) else 0.0
    res = serve([spec], 0.75, 1 << 20, backend=_HostBackend(), producer_delay=delay)
    s = res["slow"]
    assert s["chunks"] == 7 and s["late"] == 1
    lat = spec.book.latencies
    assert lat[2] >= 0.15 and lat[2] > spec.book.deadline
    assert all(x < spec.book.deadline for i, x in enumerate(lat) if i != 2)
    # without the slow producer nothing is late
    spec2 = StreamSpec("slow", [None], 1, chunk, [np.zeros((1, 4, chunk), np.uint8)])
    assert serve([spec2], 0.75, 1 << 20, backend=_HostBackend())["slow"]["late"] == 0

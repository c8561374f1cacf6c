"""Real-time serving driver: streams whose chunks are released at the real-time rate (one
chunk of `chunk` samples every chunk * tsamp seconds per stream) are admitted into the
continuous-batching engine (libarts' arts_server) as the HBM budget allows.  The loop never
blocks on the GPU: every turn it admits streams, submits each chunk as soon as it is released
and steps it at once (arts_server_tick returns after enqueueing; ticks alternate between the
engine's two compute lanes, so a chunk released while another tick runs is stepped beside it),
and collects each stream as soon as arts_server_poll reports its step done.
Chunk latency = time the candidates are back on the host minus the chunk's release time; a
chunk is late when that exceeds its deadline (by default one chunk duration: the next chunk
of the stream is then already due).  A producer that hands chunks over after their release
(producer_delay) makes them late by construction: the late-chunk count is the deadline watchdog.

    python -m paper_2205_12362_amd.serve --seconds 20 [--contention] [--lanes 1] [--autotune]
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import arts, synth


class LatencyBook:
    """Per-stream chunk latencies against a deadline (seconds after release)."""

    def __init__(self, deadline: float):
        if not deadline > 0:
            raise ValueError("deadline must be positive")
        self.deadline = deadline
        self.latencies = []
        self.late = 0

    def record(self, release: float, receipt: float) -> float:
        if receipt < release:
            raise ValueError("receipt before release")
        lat = receipt - release
        self.latencies.append(lat)
        if lat > self.deadline:
            self.late += 1
        return lat

    def summary(self) -> dict:
        lat = np.array(self.latencies) * 1e3
        return {"chunks": int(lat.size),
                "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
                "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
                "max_ms": float(lat.max()) if lat.size else None,
                "late": self.late, "deadline_ms": self.deadline * 1e3}


@dataclass
class StreamSpec:
    """A stream to serve: its plans (Workloads), source rows, optional SB table, chunk length,
    start offset in seconds and a pool of chunk data (host uint8 arrays, cycled)."""
    name: str
    workloads: list
    nsrc: int
    chunk: int
    pool: list
    sb_table: np.ndarray | None = None
    start: float = 0.0
    threshold: float = 8.0
    book: LatencyBook | None = None
    ncand: int = 0
    results: list = field(default_factory=list)


class DeviceBackend:
    """The serving loop's device side: libarts plans (optionally autotuned for the stream's step:
    its beams and one chunk plus the plan's halo, with the tune cache at `tune_cache`), chunk
    pools in pinned host memory, SB tables in HBM and the arts_server engine."""

    def __init__(self, tune_reps: int = 0, tune_cache: str | None = None):
        import torch
        self.torch = torch
        self.tune_reps = tune_reps
        self.tune_cache = tune_cache
        self.tuned = {}

    def plans(self, spec):
        plans = [arts.Plan.from_workload(w) for w in spec.workloads]
        if self.tune_reps > 0:
            nbeam = spec.sb_table.shape[0] if spec.sb_table is not None else spec.nsrc
            for w, p in zip(spec.workloads, plans):
                info = p.info
                nin = info["downsample"] * info["halo"] + spec.chunk
                v, ms = p.autotune(nbeam, nin, self.tune_reps, self.tune_cache)
                self.tuned[f"{spec.name}/{w.name}"] = {"shape": list(p.tiling_shape()),
                                                       "tiling": arts.arts_tiling_describe(v),
                                                       "ms": ms}
        return plans

    def host_chunk(self, a):
        return self.torch.from_numpy(a).pin_memory()

    def table(self, t):
        return self.torch.from_numpy(t).cuda() if t is not None else None

    def server(self, budget_bytes):
        return arts.Server(budget_bytes)


def serve(specs, seconds: float, budget_bytes: int, log=None, lanes: int = 2,
          keep_results: bool = False, backend=None, producer_delay=None):
    """Serve the streams for `seconds` of wall-clock time; returns per-stream latency stats
    (and, with keep_results, each stream's candidate arrays in spec.results).

    backend: plans, chunk buffers and the engine (DeviceBackend by default).  producer_delay:
    optional callable (stream name, chunk index) -> seconds after its release at which the
    producer hands the chunk over (a slow producer); its latency still counts from the release."""
    tsamp = synth.TSAMP
    if backend is None:
        backend = DeviceBackend()
    plans = {s.name: backend.plans(s) for s in specs}
    pinned = {s.name: [backend.host_chunk(c) for c in s.pool] for s in specs}
    tables = {s.name: backend.table(s.sb_table) for s in specs}
    for s in specs:
        s.book = LatencyBook(s.chunk * tsamp)
    srv = backend.server(budget_bytes)
    srv.set_lanes(lanes)
    sid, nsub, pending = {}, {}, {}
    waiting = list(specs)
    rejected = ticks = 0
    t0 = time.perf_counter()
    next_log = 10.0
    try:
        while True:
            now = time.perf_counter() - t0
            if log is not None and now >= next_log:
                log(f"{now:.0f} s: " + ", ".join(f"{s.name} {len(s.book.latencies)} chunks"
                                                 for s in specs))
                next_log += 10.0
            if now >= seconds and not pending:
                break
            busy = False
            # admission: streams whose start time has come, while the budget allows
            for s in list(waiting):
                if now < s.start:
                    continue
                try:
                    sid[s.name] = srv.open(plans[s.name], s.nsrc, s.chunk, s.threshold,
                                           sb_table=tables[s.name], cand_capacity=1 << 20)
                    nsub[s.name] = 0
                    waiting.remove(s)
                except arts.ArtsError as e:
                    if e.status != arts.ARTS_E_BUDGET:
                        raise
                    rejected += 1
            # submit every released chunk (one in flight per stream) and step them at once
            submitted = 0
            for s in specs:
                if s.name not in sid or s.name in pending:
                    continue
                k = nsub[s.name]
                release = s.start + (k + 1) * s.chunk * tsamp   # chunk k complete at this time
                handed = release + (producer_delay(s.name, k) if producer_delay else 0.0)
                if handed <= now and release <= seconds:
                    srv.submit(sid[s.name], pinned[s.name][k % len(s.pool)])
                    pending[s.name] = release
                    nsub[s.name] = k + 1
                    submitted += 1
            if submitted:
                srv.tick()
                ticks += 1
                busy = True
            # collect whatever has finished, without blocking
            for name in list(pending):
                if not srv.poll(sid[name]):
                    continue
                cands, _ = srv.collect(sid[name])
                t = time.perf_counter() - t0
                spec = next(s for s in specs if s.name == name)
                spec.book.record(pending.pop(name), t)
                spec.ncand += len(cands)
                if keep_results:
                    spec.results.append(cands)
                busy = True
            if not busy:
                time.sleep(0.0002)
    finally:
        srv.close()
    out = {}
    for s in specs:
        out[s.name] = dict(s.book.summary(), candidates=s.ncand)
    out["_admission_retries"] = rejected
    out["_ticks"] = ticks
    out["_lanes"] = lanes
    if getattr(backend, "tuned", None):
        out["_autotuned"] = backend.tuned
    return out


def default_specs(seed=7):
    """The 71-SB Apertif stream (12 TABs, native + D=4 trials) plus two smaller streams of other
    shapes that join later: a 384-channel beam to DM 500 and a 768-channel beam to DM 2000.
    Each chunk of the 71-SB stream carries four dispersed top-hat bursts (16 samples, 6 counts
    per channel) in TAB 11, which SB 35 takes across the whole band."""
    specs = []
    chunk = synth.CHUNK
    w_nat = synth.cfg_apertif()
    delays, _ = arts.arts_delay_table(w_nat.nchan, w_nat.f_lo, w_nat.df, w_nat.tsamp, w_nat.dms)
    pool = []
    for i in range(2):
        c = synth.noise((12, 1536, chunk), seed=seed + i)
        rng = np.random.default_rng(seed + 100 + i)
        for _ in range(4):
            d = int(rng.integers(100, 2000))
            t = int(rng.integers(0, chunk - 300))
            synth.add_tophat(c[11], t + delays[d] - int(delays[d].max()), 16, 6)
        pool.append(c)
    specs.append(StreamSpec("apertif71", [w_nat, synth.cfg_apertif_ds()], 12, chunk,
                            pool, sb_table=synth.sb_table_synthetic()))
    for name, nchan, dm_hi, ntr, start in (("b384", 384, 500.0, 1024, 2.0),
                                           ("b768", 768, 2000.0, 2048, 4.0)):
        f_lo, df = synth.band(nchan)
        w = synth.Workload(name, nchan, f_lo, df, synth.TSAMP, np.linspace(0, dm_hi, ntr),
                           [1 << k for k in range(9)])
        spool = [synth.noise((1, nchan, 6250), seed=seed + 10 + i) for i in range(2)]
        specs.append(StreamSpec(name, [w], 1, 6250, spool, start=start))
    return specs


def contention_specs(seed=7):
    """The default streams, with the two small streams' chunks released inside the 71-SB
    stream's steps: the 0.512 s chunks of b384 are released 30 ms and those of b768 60 ms after
    a 1.024 s boundary every second chunk, while the 71-SB step (about 0.1 s) is on the GPU."""
    specs = default_specs(seed)
    for s, off in zip(specs[1:], (0.030, 0.060)):
        s.start = 1.024 + off
    return specs


def compare_batching(nsb=71, chunks=8, timed=3, budget_bytes=64 << 30):
    """One search step for nsb single-SB streams (native + D=4 trials, chunks of 12 500
    samples), run one stream per engine tick versus all streams in one tick (their
    dedispersion in one persistent launch per tiling).  The first chunks warm the streams up;
    the last `timed` chunks are timed.  Returns ms per step of each mode."""
    import torch
    plans = [arts.Plan.from_workload(synth.cfg_apertif()),
             arts.Plan.from_workload(synth.cfg_apertif_ds())]
    chunk = synth.CHUNK
    pool = [torch.from_numpy(synth.noise((1, 1536, chunk), seed=40 + i)).cuda() for i in range(2)]
    out = {}
    for mode in ("one_at_a_time", "batched"):
        with arts.Server(budget_bytes) as srv:
            ids = [srv.open(plans, 1, chunk, 8.0) for _ in range(nsb)]
            times = []
            for k in range(chunks):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == "batched":
                    for i in ids:
                        srv.submit(i, pool[(k + i) % 2])
                    srv.tick()
                    for i in ids:
                        srv.collect(i)
                else:
                    for i in ids:
                        srv.submit(i, pool[(k + i) % 2])
                        srv.tick()
                        srv.collect(i)
                times.append(time.perf_counter() - t0)
            out[mode] = {"ms_per_step": 1e3 * float(np.mean(times[-timed:])),
                         "device_bytes": srv.info()["used_bytes"]}
    out["speedup"] = out["one_at_a_time"]["ms_per_step"] / out["batched"]["ms_per_step"]
    out["config"] = f"{nsb} single-SB streams x (2048 native + 1476 D=4 trials), chunk {chunk}"
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seconds", type=float, default=20.0)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--compare-batching", action="store_true",
                    help="time one-stream-per-tick against one batched tick (71 SB streams)")
    ap.add_argument("--contention", action="store_true",
                    help="release the small streams' chunks while the 71-SB step runs")
    ap.add_argument("--lanes", type=int, default=2, choices=[1, 2],
                    help="engine compute lanes (1: every tick waits behind the previous one)")
    ap.add_argument("--autotune", type=int, default=0, metavar="REPS",
                    help="autotune every plan for its stream's step before serving")
    ap.add_argument("--tune-cache", default=None, help="tune cache file (with --autotune)")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if args.compare_batching:
        print(json.dumps(compare_batching(budget_bytes=int(args.budget_gb * 2**30))))
        return
    specs = contention_specs() if args.contention else default_specs()
    res = serve(specs, args.seconds, int(args.budget_gb * 2**30),
                log=lambda m: print(m, file=sys.stderr, flush=True), lanes=args.lanes,
                backend=DeviceBackend(args.autotune, args.tune_cache))
    res["_scenario"] = "contention" if args.contention else "default"
    print(json.dumps(res))


if __name__ == "__main__":
    main()

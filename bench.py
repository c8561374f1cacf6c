#!/usr/bin/env python3
"""Benchmark of the search hot path on one MI355X.

One step = one 1.024 s chunk (12 500 new samples) of the serving stream: 12 TABs x 1536
channels arrive; 71 synthesized beams are formed from them on the fly; each SB is dedispersed
over 2048 trials (DM 0..2047, native 81.92 us) and 1476 time-downsampled trials (D = 4,
DM 2048..4998 step 2); boxcars 1..256 native / 1..64 downsampled samples; per-series S/N and
threshold-8 candidates.  The overlap (halo) stays on the device between steps.  Inputs are
resident in HBM before the timed region; each step copies its chunk from a device pool.

Prints ONE JSON line.  Metric: DM-trial samples per second (reported samples, all SBs, both
trial sets); also the real-time factor and chunk latency percentiles.  The chunk latency is
timed as the metric defines it, from a chunk's release in pinned host memory to the receipt of
its candidates on the host (the host-to-device copy included), in a second loop after the timed
region; the device-pool step time is reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CHUNK = 12500
NTAB, NSB, NCHAN = 12, 71, 1536
THRESHOLD = 8.0
# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz.  Exact integer adds: one 32-bit add per lane
# per clock (v_add_u32), two with packed 16-bit adds (v_pk_add_u16).
PEAK_INT32_ADDS = 256 * 64 * 2.4e9
# RFI mitigation thresholds of --rfi (standard deviations; the paper does not give AMBER's)
RFI_K_TIME, RFI_K_FREQ = 6.0, 5.0
PEAK_PK16_ADDS = 2 * PEAK_INT32_ADDS


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    """Host CPU description: model name, logical CPUs, sockets, and the cores this process may
    use (its affinity set)."""
    name, sockets = None, set()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and name is None:
                    name = line.split(":", 1)[1].strip()
                elif line.startswith("physical id"):
                    sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    name = name or platform.processor() or "unknown"
    return (f"{name}; {os.cpu_count()} logical CPUs in {max(1, len(sockets))} socket(s); "
            f"{len(os.sched_getaffinity(0))} in this process's affinity set")


def oracle_cores():
    """Worker processes for the oracle: every core of the process's CPU share -- its affinity
    set, bounded by OMP_NUM_THREADS where the host sets it (a GPU machine grants one GPU's share of
    its cores that way)."""
    n = len(os.sched_getaffinity(0))
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, n)


def _oracle_rows(args):
    """cpu_baseline worker: the oracle's dedispersion + boxcar/S/N/candidates on DM rows (the
    last row is padding that fixes the output length, see cpu_baseline)."""
    import oracle as O
    beam, delays, widths, nrep, thr = args
    x = O.dedisperse(beam, delays)[:-1]
    O.candidates(x, widths, nrep, thr)
    return x.shape[0]


def oracle_rate(beam, w, nrep, cores):
    """Time the CPU oracle (dedispersion + boxcars/S/N/candidates) on one beam over every DM
    trial of workload w, parallelised over DM blocks; returns (DM-trial samples/s, seconds)."""
    import multiprocessing as mp

    import oracle as O
    delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms, w.downsample)
    dmax = int(delays.max())
    rows = np.arange(delays.shape[0])
    jobs = []
    for b in np.array_split(rows, cores):
        if len(b):
            # a padding trial with the table's largest delay keeps the output length (and so
            # the reported window) equal to the full plan's
            pad = np.zeros((1, delays.shape[1]), dtype=delays.dtype)
            pad[0, 0] = dmax
            jobs.append((beam, np.concatenate([delays[b], pad]), w.widths, nrep, w.threshold))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        done = sum(pool.map(_oracle_rows, jobs))
    dt = time.perf_counter() - t0
    assert done == len(rows)
    return done * nrep / dt, dt


def cpu_baseline(beams, w_native):
    """The CPU oracle on a bounded sample of the serving workload: a few SBs of one chunk (1536
    channels, 12500 new samples plus the overlap each), all 2048 native DM trials, all widths,
    one SB after the other, each over every core of the process's share."""
    cores = oracle_cores()
    done, secs = 0.0, 0.0
    for beam in beams:
        rate, dt = oracle_rate(beam, w_native, CHUNK, cores)
        done += rate * dt
        secs += dt
    return {"value": done / secs, "unit": "DM-trial samples/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{len(beams)} SBs of one serving chunk (1536 ch, 12500 reported samples "
                      f"each), all {w_native.dms.size} native DM trials, widths 1-256, "
                      f"threshold 8: {secs:.1f} s wall on {cores} processes"}


def small_configs(arts, synth, torch, with_oracle):
    """The two single-beam configurations timed in full, on the GPU (plan calls: dedispersion
    + candidates, one call after a warm-up call; HIP events) and, unless with_oracle is False,
    by the oracle: the 128-channel beam (16384 samples, 256 DMs, widths 1-16) and one Apertif
    beam-chunk (1536 channels, 12500 new samples plus the overlap, 2048 DMs, widths 1-256).
    Rates in DM-trial samples/s over the reported window; the dedispersion launch's fraction
    of the packed 16-bit add peak beside them."""
    res = {}
    for w, nsamp, reps in ((synth.cfg_small(), 16384, 20), (synth.cfg_apertif(), None, 3)):
        p = arts.Plan.from_workload(w)
        nin = nsamp if nsamp else CHUNK + p.halo
        beam = synth.noise((w.nchan, nin), seed=w.seed)
        dev = torch.from_numpy(beam[None]).cuda()
        series = p.dedisperse(dev)
        nrep = series.shape[2] - max(w.widths) + 1
        p.candidates(series, w.threshold)
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ms_d = ms_all = 0.0
        for _ in range(reps):
            e[0].record()
            p.dedisperse(dev, out=series)
            e[1].record()
            p.candidates(series, w.threshold)
            e[2].record()
            torch.cuda.synchronize()
            ms_d += e[0].elapsed_time(e[1]) / reps
            ms_all += e[0].elapsed_time(e[2]) / reps
        units = w.dms.size * nrep
        adds = w.dms.size * nrep * w.nchan
        entry = {"workload": w.name, "nchan": w.nchan, "ndm": int(w.dms.size),
                 "reported_samples": int(nrep),
                 "gpu": {"value": units / (ms_all * 1e-3), "unit": "DM-trial samples/s",
                         "ms_per_call": ms_all, "dedisperse_ms": ms_d,
                         "dedisperse_frac_pk16_peak": adds / (ms_d * 1e-3) / PEAK_PK16_ADDS,
                         "note": "one beam per call: small grids do not fill 256 CUs"}}
        if with_oracle:
            cores = oracle_cores()
            rate, dt = oracle_rate(beam, w, nrep, cores)
            entry["oracle"] = {"value": rate, "unit": "DM-trial samples/s", "cores": cores,
                               "seconds": dt, "sample": "the whole configuration, once"}
        res[w.name] = entry
        del series, dev, p
    torch.cuda.empty_cache()
    return res


KERNEL_SRC = os.path.join(ROOT, "paper_2205_12362_amd", "csrc", "arts_kernels.hip")
PROFILE_JSON = os.path.join(ROOT, "profiles", "dedisperse_serving_chunk.json")


def kernel_name(describe):
    """Template name of the dedispersion kernel of a tiling variant, from its description
    ("J=5 ACC=3 WAVES=8 SPD=4 packed" -> "dedisperse_kernel<4, 5, 3, 8, 1>"; "framed" -> 2,
    "pairs" -> 5, "framed runs" -> 7, "framed runs shared" -> 9, "pairs framed" -> 10)."""
    f = dict(kv.split("=") for kv in describe.split() if "=" in kv)
    pack = (11 if "runs group sums" in describe else 10 if "pairs framed" in describe
            else 9 if "runs shared" in describe
            else 7 if "framed runs" in describe
            else 5 if "pairs" in describe
            else 2 if "framed" in describe else 1 if "packed" in describe else 0)
    return f"dedisperse_kernel<{f['SPD']}, {f['J']}, {f['ACC']}, {f['WAVES']}, {pack}>"


def kernel_hash():
    """Hash of the kernel source's code: comments, trailing blanks and empty lines removed, so
    that a comment edit does not void counters taken on the same code."""
    import hashlib
    import re
    with open(KERNEL_SRC, encoding="utf-8") as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", l).rstrip() for l in text.splitlines())
    code = "\n".join(l for l in lines if l)
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of the dominant kernel from the committed counter summary, if the
    counters were taken on this kernel (template name as kernel_name gives it) and its source
    has not changed since (else None)."""
    try:
        with open(PROFILE_JSON) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    if prof.get("kernel_sha") != kernel_hash():
        return None
    if (prof.get("kernel") or "").replace(", false>", ">") != kernel:
        return None
    return prof.get("hbm_bytes_per_launch")


SQ_COUNTERS = ("SQ_INSTS_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE "
               "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_BUSY_CYCLES SQ_WAVES")


def summarize_profile(stats_dir, fetch_dir, write_dir, sq_dir=None):
    """Turn rocprofv3 outputs of this script (kernel stats + FETCH_SIZE + WRITE_SIZE passes, each
    run with --copy-probe, and optionally a pass over SQ_COUNTERS) into
    profiles/dedisperse_serving_chunk.{txt,json}."""
    import csv
    import glob

    def rows(d, pattern):
        f = glob.glob(os.path.join(d, "**", pattern), recursive=True)
        return list(csv.DictReader(open(f[0]))) if f else []

    stats = rows(stats_dir, "*kernel_stats.csv")

    def per_kernel(d, counter):
        out = {}
        for r in rows(d, "*counter_collection.csv"):
            if r["Counter_Name"] != counter:
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    copy_bytes = float(1 << 30)

    def pick(d, key, largest=False):
        vals = [x for k, v in d.items() if key in k for x in v]
        if not vals:
            return None
        return max(vals) if largest else sum(vals) / len(vals)

    # the calibration copies are the largest dispatches of the copy kernel (1 GiB each)
    copy_name = "copyBuffer" if pick(fetch, "copyBuffer") else "elementwise"
    cf, cw = pick(fetch, copy_name, True), pick(write, copy_name, True)
    f_scale = copy_bytes / (cf * 1024) if cf else None   # bytes per KiB reported
    w_scale = copy_bytes / (cw * 1024) if cw else None
    sq_rows = rows(sq_dir, "*counter_collection.csv") if sq_dir else []
    # algorithmic adds per launch of each dedispersion kernel (every output it computes): 71 SBs
    # x 2048 trials x 12755 outputs (native) and x 1476 trials x 3188 outputs (D = 4), x 1536
    work = {"dedisperse_kernel<4,": NSB * 2048 * (CHUNK + 255) * NCHAN,
            "dedisperse_kernel<2,": NSB * 1476 * (CHUNK // 4 + 63) * NCHAN}
    summary = {}
    lines = ["rocprofv3 summary: 71-SB serving chunk (bench.py)", ""]
    lines.append("kernel stats (rocprofv3 --kernel-trace --stats):")
    for r in stats:
        lines.append(f"  {r['Name'][:70]:70s} calls {r['Calls']:>4s}  avg {float(r['AverageNs'])/1e6:9.3f} ms")
    # the HBM-bound steps against the stream rate measured in the same run (the probe's 1 GiB
    # elementwise stream, read once and written once: its fastest dispatch)
    trace = rows(stats_dir, "*kernel_trace.csv")
    copies = sorted(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trace
                    if "bitwise_not" in r["Kernel_Name"])
    copy_tbs = 2 * copy_bytes / (copies[0] * 1e-9) / 1e12 if copies else None
    # the pre-pass instances (one per evaluated-width count): the longer one reads the native
    # rows, the shorter one the D=4 rows
    pre = sorted((r for r in stats if "cand_pre_kernel" in r["Name"]),
                 key=lambda r: -float(r["AverageNs"]))
    pre_names = [r["Name"][r["Name"].index("cand_pre_kernel"):r["Name"].index(">") + 1]
                 .replace(" ", "") for r in pre]
    hbm_steps = tuple(
        (key, label, nbytes) for key, label, nbytes in (
            (pre_names[0] if pre_names else "-", "candidate pre-pass, native rows (71 x 2048 x "
             "12 755 int32 read)", NSB * 2048 * (CHUNK + 255) * 4),
            (pre_names[1] if len(pre_names) > 1 else "-", "candidate pre-pass, D=4 rows (71 x "
             "1476 x 3188 int32 read)", NSB * 1476 * (CHUNK // 4 + 63) * 4),
            ("downsample_rows_kernel", "D=4 downsampling of the new chunk (12 x 1536 x 12 500 B "
             "read, x 3125 x 2 B written)", NTAB * NCHAN * CHUNK + NTAB * NCHAN * (CHUNK // 4) * 2)))
    if copy_tbs:
        lines.append("")
        lines.append(f"HBM-bound steps (algorithmic bytes / average duration) against the measured "
                     f"stream rate, {copy_tbs:.2f} TB/s (an elementwise kernel reading 1 GiB and "
                     f"writing 1 GiB in {copies[0] / 1e6:.3f} ms; HBM peak 8 TB/s):")
        for key, label, nbytes in hbm_steps:
            ks = [r for r in stats if key in r["Name"].replace(" ", "")]
            if not ks:
                continue
            ms = float(ks[0]["AverageNs"]) / 1e6
            tbs = nbytes / (ms * 1e-3) / 1e12
            lines.append(f"  {label}: {ms:.3f} ms, {tbs:.2f} TB/s = {tbs / copy_tbs:.2f} of the "
                         f"stream rate")
            summary.setdefault("hbm_steps", {})[key] = {"ms": ms, "bytes": nbytes, "tb_s": tbs,
                                                        "frac_stream": tbs / copy_tbs}
    lines.append("")
    lines.append(f"1 GiB copy: FETCH_SIZE {cf} KiB -> scale {f_scale} B/KiB; WRITE_SIZE {cw} KiB -> "
                 f"scale {w_scale} B/KiB")
    for prefix, label in (("dedisperse_kernel<4,", "native dedispersion (dominant)"),
                          ("dedisperse_kernel<2,", "D=4 dedispersion")):
        ks = [r for r in stats if prefix in r["Name"]]
        if not ks:
            continue
        dom = max(ks, key=lambda r: float(r["TotalDurationNs"]))
        name = dom["Name"]
        short = name[name.index("dedisperse_kernel"):name.index(">") + 1]
        ms = float(dom["AverageNs"]) / 1e6
        df, dw = pick(fetch, short), pick(write, short)
        traffic = (df * 1024 * f_scale + dw * 1024 * w_scale) if (df and dw and f_scale and w_scale) else None
        sq = {}
        for r in sq_rows:
            if short in r["Kernel_Name"]:
                sq.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        sq = {k: sum(v) / len(v) for k, v in sq.items()}
        adds = work[prefix]
        lines.append("")
        lines.append(f"{label}: {short}, {ms:.3f} ms per launch, {adds:.4e} adds, "
                     f"{adds / ms / 1e9:.2f} Tadd/s = {adds / ms * 1e3 / PEAK_PK16_ADDS:.3f} of the "
                     f"packed 16-bit peak")
        if traffic:
            lines.append(f"  HBM bytes per launch: FETCH {df:.4e} KiB x {f_scale:.4f} + WRITE "
                         f"{dw:.4e} KiB x {w_scale:.4f} = {traffic:.4e} B ({traffic / ms / 1e9:.3f} TB/s)")
        derived = {}
        if sq:
            cycles = sq.get("SQ_BUSY_CYCLES", 0) / 32.0   # summed over the 32 shader engines
            derived = {"cycles": cycles}
            for k in sorted(sq):
                lines.append(f"  {k:24s} {sq[k]:.4e}")
            if cycles > 0:
                derived["valu_lane_instr_per_add"] = sq.get("SQ_INSTS_VALU", 0) * 64 / adds
                derived["valu_issue_per_cu_cycle"] = sq.get("SQ_INSTS_VALU", 0) / (256 * cycles)
                derived["lds_busy_per_cu_cycle"] = sq.get("SQ_LDS_IDX_ACTIVE", 0) / (256 * cycles)
                derived["lds_instr_per_add"] = sq.get("SQ_INSTS_LDS", 0) * 64 / adds
                derived["clock_ghz"] = cycles / (ms * 1e6)
                lines.append(f"  derived: {derived['valu_lane_instr_per_add']:.3f} VALU lane-instructions "
                             f"per add, VALU issue {derived['valu_issue_per_cu_cycle']:.3f} per CU-cycle, "
                             f"LDS busy {derived['lds_busy_per_cu_cycle']:.3f} per CU-cycle, "
                             f"{derived['lds_instr_per_add']:.3f} LDS lane-instructions per add, "
                             f"clock {derived['clock_ghz']:.2f} GHz (busy cycles / 32 SEs / duration)")
        summary[short] = {"avg_ms": ms, "adds_per_launch": adds, "fetch_kib": df, "write_kib": dw,
                          "hbm_bytes_per_launch": traffic, "sq_counters": sq, "derived": derived}
    lines.append("")
    lines.append("commands (from the repository root, TMPDIR=/tmp):")
    lines.append("  rocprofv3 --kernel-trace --stats --output-format csv -d <stats_dir> -o bench -- "
                 "python3 bench.py --steps 4 --warmup 3 --no-cpu-baseline --no-configs --copy-probe")
    lines.append("  rocprofv3 --pmc FETCH_SIZE --output-format csv -d <fetch_dir> -o pmc -- "
                 "python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-configs --copy-probe")
    lines.append("  rocprofv3 --pmc WRITE_SIZE --output-format csv -d <write_dir> -o pmc -- "
                 "python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-configs --copy-probe")
    lines.append(f"  rocprofv3 --pmc {SQ_COUNTERS} --output-format csv -d <sq_dir> -o pmc -- "
                 "python3 bench.py --steps 2 --warmup 1 --no-cpu-baseline --no-configs")
    lines.append("  python3 bench.py --summarize-profile <stats_dir> <fetch_dir> <write_dir> <sq_dir>")
    dom_name = next((k for k in summary if k.startswith("dedisperse_kernel<4,")), None)
    dom = summary.get(dom_name, {})
    os.makedirs(os.path.dirname(PROFILE_JSON), exist_ok=True)
    with open(PROFILE_JSON[:-5] + ".txt", "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(PROFILE_JSON, "w") as f:
        json.dump({"kernel": dom_name, "kernel_sha": kernel_hash(), "avg_ms": dom.get("avg_ms"),
                   "hbm_bytes_per_launch": dom.get("hbm_bytes_per_launch"),
                   "copy_fetch_kib": cf, "copy_write_kib": cw, "kernels": summary}, f, indent=1)
    print("\n".join(lines))


def uneven_bench(args):
    """Uneven batch: 64 requests of different channel counts, lengths and DM ranges, searched
    (dedispersion + candidates) by the persistent batch launch with autotuned tiles, against the
    same requests as a loop of per-request plan calls.  A request of length T carries T plus its
    plan's halo of input samples, so that T seconds are searched.  Prints one JSON line; value =
    the batched rate."""
    import torch

    import paper_2205_12362_amd.arts as arts
    from paper_2205_12362_amd import synth

    reqs = synth.uneven_requests(64, seed=4)
    g = torch.Generator(device="cuda")
    g.manual_seed(4)
    items, units, adds = [], 0, 0
    for w in reqs:
        p = arts.Plan.from_workload(w)
        nin = w.extra["nsamp"] + p.halo * w.downsample
        L = arts.series_length(p, nin)
        data = torch.randint(0, 256, (1, w.nchan, nin), dtype=torch.uint8, device="cuda",
                             generator=g)
        out = torch.empty((1, w.dms.size, L), dtype=torch.int32, device="cuda")
        items.append((p, data, out))
        units += w.dms.size * (L - max(w.widths) + 1)
        adds += w.dms.size * L * w.nchan
    batch = arts.Batch()
    thr = 8.0

    def step_batch():
        batch.dedisperse(items)
        return len(batch.candidates(items, thr))

    def step_plain():
        n = 0
        for p, d, o in items:
            p.dedisperse(d, out=o)
            n += len(p.candidates(o, thr))
        return n

    def timed(f):
        for _ in range(args.warmup):
            f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ncand = f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, ncand

    variants0 = sorted({it[0].tiling() for it in items})
    res = {"plain": timed(step_plain), "batch_default": timed(step_batch)}
    log("autotuning the batch ...")
    t0 = time.perf_counter()
    tuned_v, tuned_ms = batch.autotune(items, reps=1)
    tune_s = time.perf_counter() - t0
    shapes = sorted({it[0].tiling_shape() for it in items})
    res["batch"] = timed(step_batch)
    batch.close()
    ms_b, ms_p = res["batch"][0] * 1e3, res["plain"][0] * 1e3
    print(json.dumps({
        "metric": "DM-trial samples/s", "value": units / res["batch"][0],
        "unit": "DM-trial samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "uneven batch: 64 requests, nchan 384/768/1536, 0.5-4 s searched "
                               "(input: that plus the plan's halo), DM 0-500/0-2000/0-5000 with "
                               "512-4096 trials, widths 1-256, dedispersion + candidates",
                   "requests": len(items), "threshold": thr},
        "adds_per_s": adds / res["batch"][0],
        "plain_per_request": {"ms_per_step": ms_p, "value": units / res["plain"][0]},
        "batch_default_tiling": {"ms_per_step": res["batch_default"][0] * 1e3,
                                 "value": units / res["batch_default"][0],
                                 "variants": variants0},
        "autotune": {"variant": tuned_v, "tiling": arts.arts_tiling_describe(tuned_v),
                     "shapes": [list(x) for x in shapes], "tuning_seconds": tune_s,
                     "persistent_launches_per_step": len({x[:2] for x in shapes})},
        "batch_speedup": ms_p / ms_b,
        "candidates_per_step": res["batch"][1]}))


ALERT_PLANS = ((0.0, 0.2, 2048, 32), (409.6, 0.2, 2048, 32), (819.2, 2.5, 1024, 16))
ALERT_WIDTHS = [1, 5, 10, 25, 50, 100, 250]


def subband_sensitivity(arts, synth, nburst=24, seed=9):
    """S/N of injected top-hat bursts (width 10, DMs uniform in 20-400, off the trial grid) as
    found by the subband plan of DM 0-409.6 and by a brute-force plan over the same trials, on
    one beam of one chunk; returns per-burst best S/N of each and their ratio."""
    import torch
    f_lo, df = synth.band(NCHAN)
    dm0, step, ndm, nfine = ALERT_PLANS[0]
    sub = arts.Plan.subband(NCHAN, f_lo, df, synth.TSAMP, dm0, step, ndm, nfine, 32,
                            ALERT_WIDTHS)
    brute = arts.Plan(NCHAN, f_lo, df, synth.TSAMP, dm0 + step * np.arange(ndm), ALERT_WIDTHS)
    halo = max(sub.halo, brute.halo)
    nin = CHUNK + halo
    rng = np.random.default_rng(seed)
    data = synth.noise((NCHAN, nin), seed=seed)
    bursts = []
    for i in range(nburst):
        dm = float(rng.uniform(20.0, 400.0))
        t0 = 400 + i * 500
        arr = arts.arts_delay_table(NCHAN, f_lo, df, synth.TSAMP, [dm])[0][0].astype(np.int64)
        synth.add_tophat(data, t0 + arr, 10, 2)
        bursts.append((dm, t0))
    dev = torch.from_numpy(data[None]).cuda()
    best = {}
    for name, p in (("subband", sub), ("brute", brute)):
        series = p.dedisperse(dev)
        c = p.candidates(series, 6.0, capacity=1 << 20)
        vals = []
        for dm, t0 in bursts:
            m = (np.abs(c["dm"] - dm) <= 2.0) & (np.abs(c["sample"] - t0) <= 40)
            vals.append(float(c["snr"][m].max()) if m.any() else 0.0)
        best[name] = np.array(vals)
    ratio = best["subband"] / np.maximum(best["brute"], 1e-9)
    return {"bursts": nburst, "width": 10, "dm_range": [20.0, 400.0],
            "brute_snr_mean": float(best["brute"].mean()),
            "subband_snr_mean": float(best["subband"].mean()),
            "ratio_mean": float(ratio.mean()), "ratio_min": float(ratio.min()),
            "ratio_per_burst": [round(float(r), 4) for r in ratio]}


def alert_bench(args):
    """The ALERT dedispersion setup for one compound beam on one GPU (Table "dedispersion
    setup": three DM ranges, each two-step subband dedispersion with 32 subbands), streamed:
    12 TABs x 1536 channels -> 71 SBs, chunks of 12 500 samples, AMBER's integration widths."""
    import torch

    import paper_2205_12362_amd.arts as arts
    from paper_2205_12362_amd import synth

    f_lo, df = synth.band(NCHAN)
    plans = [arts.Plan.subband(NCHAN, f_lo, df, synth.TSAMP, a, st, n, nf, 32, ALERT_WIDTHS)
             for a, st, n, nf in ALERT_PLANS]
    for p in plans:
        p.cluster = bool(args.cluster)
        p.integration = args.integration
    tuned = None
    if args.autotune:
        # first-step tile shapes timed on this device: one-shot plan calls over all SBs and one
        # chunk plus the plan's halo (both steps timed, the first step's shape varied)
        tuned = {}
        for p, (a, st, n, nf) in zip(plans, ALERT_PLANS):
            v, ms = p.autotune(NSB, CHUNK + p.halo, args.autotune, args.tune_cache)
            tuned[f"dm{a:g}"] = {"shape": list(p.tiling_shape()),
                                 "tiling": arts.arts_tiling_describe(v), "ms": ms}
        log(f"autotuned: {tuned}")
    table = torch.from_numpy(synth.sb_table_synthetic(NSB, NTAB, NCHAN)).cuda()
    pool = [torch.from_numpy(synth.noise((NTAB, NCHAN, CHUNK), seed=900 + k)).cuda()
            for k in range(2)]
    stream = arts.Stream(plans, NTAB, CHUNK, THRESHOLD, sb_table=table, nbeam=NSB,
                         cand_capacity=1 << 20, profile=True)
    if args.rfi:
        stream.set_rfi(RFI_K_TIME, RFI_K_FREQ)
    cur = torch.cuda.current_stream()
    nwarm = max(args.warmup, stream.warm_chunks())
    for k in range(nwarm):
        stream.push(pool[k % 2], stream=cur)
        stream.wait()
        log(f"warmup {k + 1}/{nwarm}")
    nph = 2 + len(plans)
    base = [stream.timing(ph) for ph in range(nph)]
    torch.cuda.synchronize()
    lat, ncand = [], 0
    t_start = time.perf_counter()
    for k in range(args.steps):
        t1 = time.perf_counter()
        stream.push(pool[(nwarm + k) % 2], stream=cur)
        c, _ = stream.wait()
        lat.append(time.perf_counter() - t1)
        ncand += len(c)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    phases = []
    for ph in range(nph):
        ms, n = stream.timing(ph)
        phases.append((ms - base[ph][0]) / max(1, n - base[ph][1]))
    info = stream.info()
    stream.close()
    ntrial = sum(n for _, _, n, _ in ALERT_PLANS)
    units = NSB * ntrial * CHUNK
    ms_step = 1e3 * elapsed / args.steps
    adds = 0  # per push once warm: step 1 on the new samples, step 2 on the series
    for p, (a, st, n, nf) in zip(plans, ALERT_PLANS):
        sbi = p.subband_info()
        adds += NSB * sbi["ncoarse"] * NCHAN * CHUNK + NSB * n * 32 * (CHUNK + 249)
    del pool
    torch.cuda.empty_cache()
    log("sensitivity against brute force ...")
    sens = subband_sensitivity(arts, synth)
    lat_ms = np.array(lat) * 1e3
    print(json.dumps({
        "metric": "DM-trial samples/s", "value": units * args.steps / elapsed,
        "unit": "DM-trial samples/s", "n_gpus": 1, "steps": args.steps, "warmup": nwarm,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "ALERT dedispersion setup for one compound beam: 12 TABs x 1536 "
                               "ch -> 71 SBs; subband dedispersion (32 subbands) over DM "
                               "0-409.6/0.2 (step 6.4), 409.6-819.2/0.2 (6.4), "
                               "819.2-3379.2/2.5 (40): 5120 trials; widths 1,5,10,25,50,100,"
                               "250; 12500 new samples per step",
                   "ntrial": ntrial, "nsb": NSB, "chunk": CHUNK, "threshold": THRESHOLD,
                   "cluster": bool(args.cluster), "rfi": bool(args.rfi),
                   "integration": args.integration, "device_bytes": info["device_bytes"],
                   "step1_tiles": {f"dm{a:g}": list(p.tiling_shape())
                                   for p, (a, st, n, nf) in zip(plans, ALERT_PLANS)},
                   "autotuned": tuned},
        "real_time_factor": (CHUNK * synth.TSAMP) / (ms_step * 1e-3),
        "chunk_latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                             "p99": float(np.percentile(lat_ms, 99)),
                             "max": float(lat_ms.max())},
        "phases_ms": {"ring_advance": phases[0],
                      **{f"dedisperse_dm{a:g}": phases[1 + i]
                         for i, (a, _, _, _) in enumerate(ALERT_PLANS)},
                      "stats_candidates": phases[-1]},
        "adds_per_step": adds, "adds_per_s": adds * args.steps / elapsed,
        "brute_force_adds_per_step": NSB * ntrial * NCHAN * (CHUNK + 249),
        "candidates_per_step": ncand / args.steps,
        "sensitivity_vs_brute_force": sens}))


def cluster_bench(args):
    """DM-width clustering of a serving-scale burst storm: 71 SBs x 2048 DM trials, widths
    1..256, 1500 events over up to 81 trials and every width plus 100 000 isolated candidates
    (about 660 000 candidates), clustered in place on the device (arts_plan_cluster).  Each step
    restores the list from a device copy (a 21 MB device copy) and clusters it."""
    import torch

    import paper_2205_12362_amd.arts as arts
    from paper_2205_12362_amd import synth

    widths = [1 << k for k in range(9)]
    b, d, w, t, s = synth.candidate_tracks(NSB, 2048, widths, CHUNK, 1500, 100000, seed=3)
    n = b.size
    rec = np.zeros(n, dtype=arts.CANDIDATE_DTYPE)
    rec["beam"], rec["dm_index"], rec["width"], rec["sample"], rec["snr"] = b, d, w, t, s
    rec["downsample"] = 1
    rec["dm"] = d.astype(np.float32)
    f_lo, df = synth.band(NCHAN)
    plan = arts.Plan(NCHAN, f_lo, df, synth.TSAMP, np.arange(2048, dtype=np.float64), widths)
    pristine = torch.from_numpy(rec.view(np.uint8)).cuda()
    work = torch.empty_like(pristine)
    ncl = 0
    for k in range(args.warmup):
        work.copy_(pristine)
        ncl = len(plan.cluster_candidates(work, NSB))
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    lat = []
    for k in range(args.steps):
        t1 = time.perf_counter()
        work.copy_(pristine)
        cnt = ctypes_cluster(arts, plan, work, n)
        lat.append(time.perf_counter() - t1)
    elapsed = time.perf_counter() - t_start
    assert cnt == ncl or args.warmup == 0
    ms = 1e3 * elapsed / args.steps
    # algorithmic bytes: every candidate record read once, every cluster record written once
    algo = 32 * n + 32 * cnt
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        cands = list(zip(b.tolist(), d.tolist(), w.tolist(), t.tolist(),
                         s.astype(float).tolist()))
        t0 = time.perf_counter()
        reps, _ = O.cluster_dm_width(cands)
        dt = time.perf_counter() - t0
        assert len(reps) == cnt, (len(reps), cnt)
        cpu = {"value": n / dt, "unit": "candidates/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole list ({n} candidates), once"}
    lat_ms = np.array(lat) * 1e3
    print(json.dumps({
        "metric": "candidates clustered/s", "value": n * args.steps / elapsed,
        "unit": "candidates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "DM-width clustering of a burst storm: 71 SBs x 2048 DMs, widths "
                               "1-256, 1500 events + 100000 isolated candidates",
                   "candidates": int(n), "clusters": int(cnt)},
        "call_latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                            "p99": float(np.percentile(lat_ms, 99))},
        "roofline": {"bound": "hbm", "achieved": algo / (ms * 1e-3) / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": algo / (ms * 1e-3) / 8e12, "traffic": None,
                     "note": "whole call: every clustering launch and the host synchronisation"},
        "cpu_baseline": cpu}))


def tilings_bench(args):
    """Every compiled tiling that runs the serving launches, timed on them: the fused-SB
    dedispersion of 71 SBs from 12 TABs x 1536 channels over the 2048 native trials (byte
    tilings) and over the 1476 D=4 trials (16-bit tilings), `args.steps` timed launches after
    one warm-up launch each (HIP events on the current stream).  One JSON line: per variant its
    description, ms per launch and Tadd/s (null where the tiling does not fit the plan)."""
    import torch

    import paper_2205_12362_amd.arts as arts
    from paper_2205_12362_amd import synth

    table = torch.from_numpy(synth.sb_table_synthetic(NSB, NTAB, NCHAN)).cuda()
    res = {}
    for w in (synth.cfg_apertif(), synth.cfg_apertif_ds()):
        p = arts.Plan.from_workload(w)
        nin = CHUNK + p.halo * w.downsample
        g = torch.Generator(device="cuda")
        g.manual_seed(1)
        tab = torch.randint(0, 256, (NTAB, NCHAN, nin), dtype=torch.uint8, device="cuda",
                            generator=g)
        default = p.tiling_shape()
        spd = "SPD=4" if w.downsample == 1 else "SPD=2"
        out = None
        for v in range(arts.arts_tiling_count()):
            d = arts.arts_tiling_describe(v)
            if spd not in d or "group" in d:
                continue
            for nbuf in (2, 1):
                key = f"{v}" if nbuf == 2 else f"{v}/1buf"
                try:
                    p.set_tiling_shape(v, nbuf, 0)
                except arts.ArtsError:
                    res[key] = {"tiling": d, "plan": w.name, "ms": None, "tadd_s": None}
                    continue
                cc = p.tiling_shape()[2]
                log(f"tiling {v}: {d}, {nbuf} buffer(s), {cc} channels per chunk")
                out = p.dedisperse_sb(tab, table, out=out)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(args.steps):
                    p.dedisperse_sb(tab, table, out=out)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / args.steps
                adds = NSB * w.dms.size * out.shape[2] * NCHAN
                res[key] = {"tiling": d, "plan": w.name, "buffers": nbuf, "channels": cc,
                            "default": v == default[0] and nbuf == default[1], "ms": ms,
                            "tadd_s": adds / ms / 1e9}
        del tab, out, p
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "dedispersion tilings on the serving launches (71 SBs fused "
                                  "from 12 TABs x 1536 ch; 2048 native / 1476 D=4 trials)",
                      "steps": args.steps, "tilings": res}), flush=True)


TILINGS_TXT = os.path.join(ROOT, "profiles", "dedisperse_tilings_serving.txt")


def summarize_tilings(json_path):
    """Write the table of a `--workload tilings` JSON line to profiles/ (one row per tiling and
    buffer count, the plans' default shapes marked)."""
    with open(json_path) as f:
        d = json.loads(f.read().strip().splitlines()[-1])
    lines = ["Dedispersion tile shapes on the serving launches (MI355X, one GPU)",
             "(fused SB formation of 71 SBs from 12 TABs x 1536 channels; 2048 native trials over",
             " 12 755 outputs per row, and 1476 D=4 trials over 3188 outputs; "
             f"{d['steps']} timed launches each",
             " after one warm-up launch, HIP events.  A D=4 plan call on byte input first "
             "downsamples",
             " the whole input (12 x 1536 rows) into its 16-bit workspace, about 1.3 ms of these "
             "times;",
             " in the serving stream only the new chunk is downsampled, in the ring advance.)",
             "Each tiling twice: two LDS buffers (the next chunk of channels fetched while one is",
             "summed) and one buffer (fetched in turn, twice the channels per chunk).  * marks the",
             "plans' default shape.",
             f"command: python3 bench.py --workload tilings --steps {d['steps']} > t.json; "
             "python3 bench.py --summarize-tilings t.json", "",
             f"{'tiling':>9s}  {'plan':26s}  {'shape':44s} {'ch/chunk':>8s}  {'ms/launch':>9s}  "
             f"{'Tadd/s':>6s}"]
    for key, r in d["tilings"].items():
        if r.get("ms") is None:
            lines.append(f"{key:>9s}  {r['plan']:26s}  {r['tiling']:44s} {'-':>8s}  "
                         f"{'does not fit':>9s}")
            continue
        mark = "*" if r.get("default") else " "
        lines.append(f"{key:>8s}{mark}  {r['plan']:26s}  {r['tiling']:44s} {r['channels']:8d}  "
                     f"{r['ms']:9.2f}  {r['tadd_s']:6.2f}")
    with open(TILINGS_TXT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def ctypes_cluster(arts, plan, work, n):
    import ctypes as C
    cnt = C.c_int64(0)
    arts._check(arts.lib().arts_plan_cluster(plan.handle, work.data_ptr(), n, NSB, 0,
                                             C.byref(cnt), None))
    return cnt.value


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-profile":
        summarize_profile(*sys.argv[2:6])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-tilings":
        summarize_tilings(sys.argv[2])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--graph", action="store_true", help="replay each step as a hipGraph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the single-beam configurations (128-channel beam, one Apertif "
                         "beam-chunk) timed after the serving steps")
    ap.add_argument("--variant", type=int, default=None, help="native dedispersion tiling")
    ap.add_argument("--autotune", type=int, default=0, metavar="REPS",
                    help="serving and alert: autotune the plans' tile shapes before timing")
    ap.add_argument("--tune-cache", default=None, help="tune cache file (with --autotune)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, copy 1 GiB twice (counter calibration)")
    ap.add_argument("--workload", choices=["serving", "uneven", "alert", "cluster", "tilings"],
                    default="serving",
                    help="serving: the 71-SB stream step (default); uneven: 64 uneven requests, "
                         "persistent batch vs per-request calls; alert: the paper's subband "
                         "dedispersion setup for one compound beam; cluster: DM-width "
                         "clustering of a serving-scale candidate list; tilings: every "
                         "dedispersion tiling timed on the serving launches")
    ap.add_argument("--cluster", action="store_true",
                    help="serving / alert: cluster each chunk's candidates (DM-width)")
    ap.add_argument("--sb-table", choices=["synthetic", "model"], default="synthetic",
                    help="serving: the SB table of the 71 SBs: the synthetic stand-in or the "
                         "beam model's (arts_sb_table_beam_model)")
    ap.add_argument("--integration", choices=["sliding", "decimated"], default="sliding",
                    help="alert: candidate search with sliding boxcars (default) or decimated "
                         "integration on each width's grid (AMBER's downsampling by the trial "
                         "widths; they divide the 12 500-sample chunk)")
    ap.add_argument("--rfi", action="store_true",
                    help="serving / alert: RFI mitigation of each chunk's TABs (time domain at "
                         "6 sigma, frequency domain at 5 sigma, 3 iterations each)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a "
              "design note, not built", file=sys.stderr)
        sys.exit(2)
    if args.workload in ("uneven", "alert", "cluster", "tilings"):
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        torch.cuda.set_device(0)
        {"uneven": uneven_bench, "alert": alert_bench, "cluster": cluster_bench,
         "tilings": tilings_bench}[args.workload](args)
        return

    import torch

    import paper_2205_12362_amd.arts as arts
    from paper_2205_12362_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w_nat = synth.cfg_apertif()
    w_ds = synth.cfg_apertif_ds()
    p_nat = arts.Plan.from_workload(w_nat)
    p_ds = arts.Plan.from_workload(w_ds)
    if args.variant is not None:
        p_nat.set_tiling(args.variant)
    tuned = None
    if args.autotune:
        # tile shapes timed on this device for this step (all SBs, one chunk plus the halo)
        tuned = {}
        for name, p in (("native", p_nat), ("ds4", p_ds)):
            nin = p.info["downsample"] * p.info["halo"] + CHUNK
            v, ms = p.autotune(NSB, nin, args.autotune, args.tune_cache)
            tuned[name] = {"shape": list(p.tiling_shape()), "tiling": arts.arts_tiling_describe(v),
                           "ms": ms}
        log(f"autotuned: {tuned}")
    if args.cluster:
        p_nat.cluster = p_ds.cluster = True
    if args.sb_table == "model":
        table, _ = arts.arts_sb_table_beam_model(NSB, NTAB, NCHAN, w_nat.f_lo, w_nat.df)
    else:
        table = synth.sb_table_synthetic(NSB, NTAB, NCHAN)

    log("generating inputs ...")
    t0 = time.perf_counter()
    # two distinct noise chunks; bursts in TAB 11 (which SB 35 sees across the whole band)
    delays = p_nat.delays()
    pool = []
    for k in range(2):
        chunk = synth.noise((NTAB, NCHAN, CHUNK), seed=500 + k)
        rng = np.random.default_rng(600 + k)
        for _ in range(4):
            d = int(rng.integers(100, 2000))
            t = int(rng.integers(0, CHUNK - 300))
            synth.add_tophat(chunk[11], t + delays[d] - int(delays[d].max()), 16, 6)
        pool.append(torch.from_numpy(chunk).cuda())
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s")
    tbl = torch.from_numpy(table).cuda()

    stream = arts.Stream([p_nat, p_ds], NTAB, CHUNK, THRESHOLD, sb_table=tbl, nbeam=NSB,
                         cand_capacity=1 << 20, graph=args.graph, profile=not args.graph)
    if args.rfi:
        stream.set_rfi(RFI_K_TIME, RFI_K_FREQ)
    info = stream.info()
    cur = torch.cuda.current_stream()

    def step(k):
        stream.push(pool[k % 2], stream=cur)
        return stream.wait()

    # untimed steps: at least until every plan searches its whole chunk (the first chunks only
    # search outputs whose window lies after the stream's start)
    nwarm = max(args.warmup, stream.warm_chunks())
    for k in range(nwarm):
        step(k)
        log(f"warmup {k + 1}/{nwarm}")
    base_ms = {ph: stream.timing(ph) for ph in range(4)} if not args.graph else None
    torch.cuda.synchronize()
    lat = []
    ncand = 0
    t_start = time.perf_counter()
    for k in range(args.steps):
        t1 = time.perf_counter()
        c, _ = step(nwarm + k)
        lat.append(time.perf_counter() - t1)
        ncand += len(c)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    log(f"timed {args.steps} steps in {elapsed:.3f} s")

    ms_step = 1e3 * elapsed / args.steps
    units_nat = NSB * w_nat.dms.size * CHUNK
    units_ds = NSB * w_ds.dms.size * (CHUNK // 4)
    value = (units_nat + units_ds) * args.steps / elapsed

    # dominant kernel: native dedispersion (phase 1), timed by events on its own stream
    roofline = None
    phases = None
    if not args.graph:
        phases = {}
        names = ["ring_advance", "dedisperse_native", "dedisperse_ds4", "stats_candidates"]
        for ph, name in enumerate(names):
            ms, n = stream.timing(ph)
            ms0, n0 = base_ms[ph]
            phases[name] = (ms - ms0) / max(1, n - n0)
        # algorithmic adds per launch: the chunk's new outputs only (the launch also recomputes
        # the wmax - 1 outputs the boxcars of the previous chunk's last starts read)
        adds = NSB * w_nat.dms.size * CHUNK * NCHAN
        dur = phases["dedisperse_native"] * 1e-3
        achieved = adds / dur
        kname = kernel_name(arts.arts_tiling_describe(p_nat.tiling()))
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_PK16_ADDS / 1e12,
                    "unit": "Tadd/s", "frac": achieved / PEAK_PK16_ADDS,
                    "frac_int32_peak": achieved / PEAK_INT32_ADDS,
                    "traffic": measured_traffic(kname), "kernel": kname,
                    "kernel_ms": phases["dedisperse_native"],
                    "adds_per_launch": adds}
    # chunk latency as the metric defines it: release of the chunk in pinned host memory ->
    # its host-to-device copy into the stream's staging buffer -> search -> candidates on the
    # host; a second loop after the timed region, same chunks
    host_pool = [t.cpu().pin_memory() for t in pool]
    staging = stream.input_buffer()
    lat_h2d = []
    for k in range(args.steps):
        t1 = time.perf_counter()
        staging.copy_(host_pool[(nwarm + args.steps + k) % 2], non_blocking=True)
        stream.push(None, stream=cur)
        stream.wait()
        lat_h2d.append(time.perf_counter() - t1)
    del host_pool, staging
    lat_ms = np.array(lat_h2d) * 1e3
    pool_ms = np.array(lat) * 1e3
    out = {
        "metric": "DM-trial samples/s",
        "value": value,
        "unit": "DM-trial samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": nwarm,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "serving stream chunk: 12 TABs x 1536 ch (1220-1520 MHz, "
                               "81.92 us) -> 71 SBs; 2048 DMs 0-2047 + 1476 D=4 DMs 2048-4998; "
                               "widths 1-256; 12500 new samples per step",
                   "nchan": NCHAN, "nsb": NSB, "ntab": NTAB, "chunk": CHUNK,
                   "ndm_native": int(w_nat.dms.size), "ndm_ds4": int(w_ds.dms.size),
                   "graph": bool(args.graph), "threshold": THRESHOLD,
                   "cluster": bool(args.cluster), "rfi": bool(args.rfi),
                   "sb_table": args.sb_table, "device_bytes": info["device_bytes"],
                   "tiles": {"native": list(p_nat.tiling_shape()), "ds4": list(p_ds.tiling_shape()),
                             "autotuned": tuned}},
        "adds_per_s": (units_nat + units_ds) * NCHAN * args.steps / elapsed,
        "real_time_factor": (CHUNK * synth.TSAMP) / (ms_step * 1e-3),
        "chunk_latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                             "p99": float(np.percentile(lat_ms, 99)),
                             "max": float(lat_ms.max()),
                             "from": "release in pinned host memory, H2D copy included",
                             "to": "candidates on the host", "steps": args.steps},
        "step_latency_device_pool_ms": {"p50": float(np.percentile(pool_ms, 50)),
                                        "p99": float(np.percentile(pool_ms, 99)),
                                        "max": float(pool_ms.max())},
        "candidates_per_step": ncand / args.steps,
        "phases_ms": phases,
        "roofline": roofline,
    }
    stream.close()
    del pool
    if args.copy_probe:
        # 1 GiB copies (the counters' calibration) and a 1 GiB elementwise stream (read once,
        # written once: the achievable HBM rate the HBM-bound steps are compared with)
        a = torch.zeros(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        for _ in range(3):
            torch.bitwise_not(a, out=b)
        torch.cuda.synchronize()
        del a, b
    torch.cuda.empty_cache()
    if not args.no_configs:
        log("single-beam configurations ...")
        out["single_beam_configs"] = small_configs(arts, synth, torch,
                                                   with_oracle=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        beams = [synth.noise((NCHAN, CHUNK + p_nat.halo), seed=777 + k) for k in range(4)]
        out["cpu_baseline"] = cpu_baseline(beams, w_nat)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

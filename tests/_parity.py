"""Helpers shared by the GPU parity tests (no test functions here).

Candidate parity rule.  The kernel takes the threshold decision on exact integer sums against
FP64 thresholds, the oracle on FP64 S/N values, so the two can disagree only about starts whose
S/N lies within rounding of the threshold.  Such a start can split, join, grow or shrink a run,
and so change the candidates of the runs it touches -- never anything else.  The rule therefore
excuses a candidate that one side reports and the other does not only when it lies in a
"near-threshold run": a maximal run of starts of its (beam, DM, width) whose oracle S/N exceeds
thr - tol*thr and which holds a start with |S/N - thr| <= tol*thr (tol = 1e-4).  Every candidate
of either side outside such runs must be present on the other side too, at the same sample, with
the S/N within 1e-4 relative.
"""
import math

import numpy as np

import oracle as O


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def oracle_rows_candidates(x_rows, widths, nrep, thr, rows, beam=0, t_offset=0):
    """Oracle candidates for selected DM rows of one beam (x_rows: [len(rows)][L]); dm index of
    each candidate is mapped back to rows[i]."""
    out = []
    for i, d in enumerate(rows):
        for c in O.candidates(x_rows[i: i + 1], widths, nrep, thr, beam=beam, t_offset=t_offset):
            out.append((c[0], int(d), c[2], c[3], c[4]))
    out.sort(key=lambda r: (r[0], r[1], r[2], r[3]))
    return out


class NearRuns:
    """Near-threshold runs per (beam, dm, width): sample intervals [lo, hi] (reported sample
    numbers, i.e. start + t_offset) in which the two candidate sets may differ."""

    def __init__(self):
        self.runs = {}

    def __ior__(self, other):
        for k, v in other.runs.items():
            self.runs.setdefault(k, []).extend(v)
        return self

    def __len__(self):
        return sum(len(v) for v in self.runs.values())

    def covers(self, beam, dm, width, sample):
        return any(lo <= sample <= hi for lo, hi in self.runs.get((beam, dm, width), ()))


def near_threshold_runs(x_rows, widths, nrep, thr, rows, beam=0, t_offset=0,
                        integration=False, tol=1e-4):
    """NearRuns of the oracle's S/N for DM rows `rows` of one beam (x_rows: [len(rows)][L]).
    With `integration`, width w is searched on its grid starts t, (t + t_offset) % w == 0, and a
    run is a sequence of consecutive grid starts (the decimated search)."""
    x_rows = np.asarray(x_rows)
    mu, sig = O.moments(x_rows, nrep)
    out = NearRuns()
    band = tol * abs(thr)
    for w in widths:
        w = int(w)
        s = O.snr(O.boxcar(x_rows, w, nrep), w, mu, sig)
        if integration:
            starts = np.array([t for t in range(nrep) if (t + t_offset) % w == 0], np.int64)
        else:
            starts = np.arange(nrep, dtype=np.int64)
        if starts.size == 0:
            continue
        s = s[:, starts]
        near_any = np.any(np.abs(s - thr) <= band, axis=1)
        for i in np.nonzero(near_any)[0]:
            loose = s[i] > thr - band
            near = np.abs(s[i] - thr) <= band
            j = 0
            n = len(starts)
            while j < n:
                if not loose[j]:
                    j += 1
                    continue
                e = j
                while e < n and loose[e]:
                    e += 1
                if near[j:e].any():
                    out.runs.setdefault((int(beam), int(rows[i]), w), []).append(
                        (int(starts[j]) + t_offset, int(starts[e - 1]) + t_offset))
                j = e
    return out


def compare_candidates(gpu, ora, near, snr_rtol=1e-4):
    """gpu: structured array; ora: oracle tuples (beam, dm, width, sample, snr); near: NearRuns.
    Both sets must hold the same candidates except inside near-threshold runs; matched candidates
    must agree in S/N to snr_rtol.  Returns the number of matched candidates."""
    g = {(int(c["beam"]), int(c["dm_index"]), int(c["width"]), int(c["sample"])): float(c["snr"])
         for c in gpu}
    o = {(int(c[0]), int(c[1]), int(c[2]), int(c[3])): float(c[4]) for c in ora}
    assert len(g) == len(gpu), "the GPU reported a candidate twice"
    bad = sorted(k for k in set(g) ^ set(o) if not near.covers(*k))
    assert not bad, (f"candidate sets differ away from the threshold: "
                     f"{[(k, 'gpu' if k in g else 'oracle') for k in bad[:10]]}")
    for k in set(g) & set(o):
        assert math.isclose(g[k], o[k], rel_tol=snr_rtol, abs_tol=1e-6), (k, g[k], o[k])
    return len(set(g) & set(o))

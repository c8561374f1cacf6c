"""Helpers shared by the GPU parity tests (no test functions here)."""
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


def near_threshold_rows(x_rows, widths, nrep, thr, rows, tol=1e-4):
    """(dm, width) pairs of the given rows that hold an S/N within tol*thr of the threshold --
    the only places where an FP32-vs-FP64 or evaluation-order difference may change the set."""
    mu, sig = O.moments(x_rows, nrep)
    near = set()
    for w in widths:
        s = O.snr(O.boxcar(x_rows, w, nrep), w, mu, sig)
        hit = np.any(np.abs(s - thr) <= tol * abs(thr), axis=1)
        for i in np.nonzero(hit)[0]:
            near.add((int(rows[i]), int(w)))
    return near


def compare_candidates(gpu, ora, near, snr_rtol=1e-4):
    """gpu: structured array; ora: oracle tuples.  Sets must be equal except in (dm, width)
    rows listed in `near`; matched candidates must agree in S/N to snr_rtol."""
    g = {(int(c["beam"]), int(c["dm_index"]), int(c["width"]), int(c["sample"])): float(c["snr"])
         for c in gpu}
    o = {(c[0], c[1], c[2], c[3]): c[4] for c in ora}
    bad = [k for k in set(g) ^ set(o) if (k[1], k[2]) not in near]
    assert not bad, f"candidate sets differ away from threshold: {sorted(bad)[:10]}"
    for k in set(g) & set(o):
        assert math.isclose(g[k], o[k], rel_tol=snr_rtol, abs_tol=1e-6), (k, g[k], o[k])
    return len(set(g) & set(o))

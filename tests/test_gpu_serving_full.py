"""Full-size parity of the streaming configuration that bench.py times: 12 TABs x 1536 channels
formed into 71 SBs by the synthetic SB table, 2048 native DM trials and 1476 D = 4 trials,
chunks of 12 500 samples, default (packed) tilings.  Sampled series points of several SBs in a
partially warm and a warm chunk of each plan, and the candidates of selected rows of the SB
that sees the burst TAB in every channel, are checked against the oracle evaluated on the
zero-prefixed concatenation of the chunks."""
import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from tests._parity import (compare_candidates, near_threshold_runs, oracle_rows_candidates,
                           to_dev)

pytestmark = pytest.mark.gpu

NTAB, NSB, NCHAN, CHUNK, THR = 12, 71, 1536, synth.CHUNK, 8.0
NCHUNKS = 6
SBS = (0, 23, 35, 70)


def _pool(delays_nat):
    # two noise chunks, cycled; bright top-hats in TAB 11 along native DM sweeps
    pool, burst_dms = [], []
    for j in range(2):
        c = synth.noise((NTAB, NCHAN, CHUNK), seed=800 + j)
        rng = np.random.default_rng(810 + j)
        for _ in range(3):
            d = int(rng.integers(100, 2000))
            t = int(rng.integers(0, CHUNK - 300))
            synth.add_tophat(c[11], t + delays_nat[d] - int(delays_nat[d].max()), 16, 6)
            burst_dms.append(d)
        pool.append(c)
    return pool, burst_dms


def _sb_window(sb_pool, hmax, lo, hi):
    """Samples [lo, hi) of one SB's zero-prefixed stream (chunk j = pool entry j % 2)."""
    parts = []
    a = lo
    while a < hi:
        if a < hmax:
            b = min(hi, hmax)
            parts.append(np.zeros((NCHAN, b - a), np.uint8))
        else:
            j, off = divmod(a - hmax, CHUNK)
            b = min(hi, hmax + (j + 1) * CHUNK)
            parts.append(sb_pool[j % 2][:, off: off + (b - a)])
        a = b
    return np.concatenate(parts, axis=1)


def test_serving_configuration_full_size():
    import torch
    w_nat, w_ds = synth.cfg_apertif(), synth.cfg_apertif_ds()
    d_nat = O.delay_table(NCHAN, w_nat.f_lo, w_nat.df, w_nat.tsamp, w_nat.dms)
    d_ds = O.delay_table(NCHAN, w_ds.f_lo, w_ds.df, w_ds.tsamp, w_ds.dms, 4)
    pool, burst_dms = _pool(d_nat)
    table = synth.sb_table_synthetic(NSB, NTAB, NCHAN)
    sb_pool = {s: [O.sb_synthesize(c, table[s: s + 1])[0] for c in pool] for s in SBS}
    plans = [arts.Plan.from_workload(w_nat), arts.Plan.from_workload(w_ds)]
    halo = [int(d_nat.max()) + max(w_nat.widths) - 1, int(d_ds.max()) + max(w_ds.widths) - 1]
    H = [halo[0], 4 * halo[1]]
    hmax = max(H)
    nrep = [CHUNK, CHUNK // 4]
    delays, ws = [d_nat, d_ds], [w_nat, w_ds]
    rng = np.random.default_rng(21)
    checks = {0: (2, 5), 1: (4, 5)}        # (partially warm, warm) chunk of each plan
    dev_pool = [to_dev(c) for c in pool]
    with arts.Stream(plans, NTAB, CHUNK, THR, sb_table=to_dev(table), nbeam=NSB,
                     cand_capacity=1 << 20) as st:
        for k in range(NCHUNKS):
            print(f"serving full size: chunk {k}", flush=True)
            st.push(dev_pool[k % 2])
            cands, idx = st.wait()
            assert idx == k
            for p in (0, 1):
                t0 = st.warmup(p, k)
                assert t0 == min(nrep[p], max(0, halo[p] - k * nrep[p]))
                if k not in checks[p]:
                    continue
                if k == checks[p][0]:
                    assert 0 < t0 < nrep[p]
                series = st.series(p)
                lo, hi = hmax - H[p] + k * CHUNK, hmax + (k + 1) * CHUNK
                for s in SBS:
                    rows_in = _sb_window(sb_pool[s], hmax, lo, hi)
                    if p == 1:
                        rows_in = O.downsample(rows_in, 4)
                    dd = rng.integers(0, delays[p].shape[0], 250)
                    tt = rng.integers(0, series.shape[2], 250)
                    got = series[s][torch.from_numpy(dd).cuda(),
                                    torch.from_numpy(tt).cuda()].cpu().numpy()
                    for g, d, t in zip(got, dd, tt):
                        assert g == O.dedisperse_at(rows_in, delays[p], int(d), int(t)), \
                            (k, p, s, int(d), int(t))
                    if s != 35 or k != checks[p][1]:
                        continue
                    # candidates of SB 35 on rows around the bursts and random rows
                    if p == 0:
                        rows = sorted({min(2047, max(0, d + e)) for d in burst_dms
                                       for e in (-1, 0, 1)} |
                                      set(int(r) for r in rng.integers(0, 2048, 6)))
                    else:
                        rows = sorted(set(int(r) for r in rng.integers(0, 1476, 8)))
                    L = series.shape[2]
                    x_rows = O.dedisperse(rows_in, delays[p][rows])[:, :L]
                    assert np.array_equal(x_rows, series[s][rows].cpu().numpy())
                    off = k * nrep[p] - halo[p]
                    xs = x_rows[:, t0:]
                    ora = oracle_rows_candidates(xs, ws[p].widths, nrep[p] - t0, THR, rows,
                                                 beam=s, t_offset=off + t0)
                    near = near_threshold_runs(xs, ws[p].widths, nrep[p] - t0, THR, rows,
                                               beam=s, t_offset=off + t0)
                    sel = cands[(cands["beam"] == s) & (cands["downsample"] == (1, 4)[p]) &
                                np.isin(cands["dm_index"], rows)]
                    compare_candidates(sel, ora, near)
                    if p == 0:
                        assert len(ora) > 0

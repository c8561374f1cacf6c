"""CPU checks of the candidate parity rule used by the GPU tests (tests/_parity.py): it excuses
differences only inside near-threshold runs and catches every other difference, extras included."""
import numpy as np
import pytest

import oracle as O
from tests._parity import compare_candidates, near_threshold_runs

DT = np.dtype([("sample", "<i8"), ("beam", "<i4"), ("dm_index", "<i4"), ("width", "<i4"),
               ("downsample", "<i4"), ("snr", "<f4"), ("dm", "<f4")])


def _as_gpu(cands):
    a = np.zeros(len(cands), DT)
    for i, c in enumerate(cands):
        a[i] = (c[3], c[0], c[1], c[2], 1, np.float32(c[4]), 0.0)
    return a


def _series(seed=3, ndm=24, L=2100):
    rng = np.random.default_rng(seed)
    x = np.rint(rng.normal(1000.0, 30.0, (ndm, L))).astype(np.int64)
    for r, t, w, a in ((2, 300, 4, 150), (7, 900, 16, 70), (15, 1500, 1, 280), (20, 40, 8, 90)):
        x[r, t:t + w] += a
    return x


WIDTHS = [1, 2, 4, 8, 16]


def test_identical_sets_pass_and_count():
    x = _series()
    nrep = x.shape[1] - 15
    ora = O.candidates(x, WIDTHS, nrep, 6.0)
    near = near_threshold_runs(x, WIDTHS, nrep, 6.0, np.arange(x.shape[0]))
    assert len(ora) > 5
    assert compare_candidates(_as_gpu(ora), ora, near) == len(ora)


def test_threshold_moved_within_tolerance_is_excused():
    # a search whose threshold decision differs by less than 1e-4 relative (what FP32 or another
    # evaluation order can do) changes candidates only inside near-threshold runs
    x = _series(seed=5)
    nrep = x.shape[1] - 15
    mu, sig = O.moments(x, nrep)
    s = O.snr(O.boxcar(x, 4, nrep), 4, mu, sig)
    thr = float(s[7, 900:916].max()) * (1.0 - 2e-5)    # a run peak just above the threshold
    ora = O.candidates(x, WIDTHS, nrep, thr)
    other = O.candidates(x, WIDTHS, nrep, thr * (1.0 + 4e-5))
    assert set(c[:4] for c in ora) != set(c[:4] for c in other)
    near = near_threshold_runs(x, WIDTHS, nrep, thr, np.arange(x.shape[0]))
    assert len(near) > 0
    compare_candidates(_as_gpu(other), ora, near)


@pytest.mark.parametrize("change", ["drop", "extra", "shift", "snr"])
def test_differences_away_from_threshold_fail(change):
    x = _series(seed=7)
    nrep = x.shape[1] - 15
    ora = O.candidates(x, WIDTHS, nrep, 6.0)
    near = near_threshold_runs(x, WIDTHS, nrep, 6.0, np.arange(x.shape[0]))
    far = [c for c in ora if not near.covers(*c[:4])]
    assert far
    g = list(ora)
    c = far[0]
    if change == "drop":
        g.remove(c)
    elif change == "extra":
        g.append((c[0], c[1], c[2], c[3] + 700, 9.0))
    elif change == "shift":
        g[g.index(c)] = (c[0], c[1], c[2], c[3] + 1, c[4])
    else:
        g[g.index(c)] = (c[0], c[1], c[2], c[3], c[4] * 1.001)
    with pytest.raises(AssertionError):
        compare_candidates(_as_gpu(g), ora, near)


def test_integration_runs_follow_the_grid():
    # decimated search: runs are consecutive grid starts, reported with the caller's offset
    x = _series(seed=9)
    nrep, off = x.shape[1] - 15, -7
    ora = O.candidates_integrated(x, WIDTHS, nrep, 5.0, t_offset=off)
    near = near_threshold_runs(x, WIDTHS, nrep, 5.0, np.arange(x.shape[0]), t_offset=off,
                               integration=True)
    for (b, d, w), runs in near.runs.items():
        for lo, hi in runs:
            assert lo % w == 0 and hi % w == 0
    assert compare_candidates(_as_gpu(ora), ora, near) == len(ora)

"""GPU parity of uneven batches: one persistent launch over many requests of different channel
counts, lengths, DM ranges and downsampling gives, for every request, exactly the oracle's
series (small requests) and exactly what the request's own plain call gives (uneven-batch
shapes); requests shorter than their halo are reported and skipped."""
import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from tests._parity import to_dev

pytestmark = pytest.mark.gpu


def _small_requests():
    rng = np.random.default_rng(17)
    reqs = []
    for i in range(9):
        nchan = int(rng.choice([16, 32, 48]))
        f_lo, df = synth.band(nchan)
        D = 1 if i % 3 else 2
        dms = np.sort(rng.uniform(0, 200, size=int(rng.integers(5, 70))))
        w = synth.Workload(f"r{i}", nchan, f_lo, df, synth.TSAMP, dms, [1, 2, 4], downsample=D)
        delays = O.delay_table(nchan, f_lo, df, synth.TSAMP, dms, D)
        nin = (int(delays.max()) + int(rng.integers(1, 3000))) * D + int(rng.integers(0, D))
        if i == 4:
            nin = int(delays.max()) * D      # too short: no output sample
        nbeam = int(rng.integers(1, 3))
        data = rng.integers(0, 256, size=(nbeam, nchan, nin), dtype=np.uint8)
        reqs.append((w, delays, data))
    return reqs


def test_batch_matches_oracle():
    reqs = _small_requests()
    plans = [arts.Plan.from_workload(w) for w, _, _ in reqs]
    items, outs = [], []
    for (w, delays, data), p in zip(reqs, plans):
        L = max(1, arts.series_length(p, data.shape[2]))
        out = to_dev(np.full((data.shape[0], w.dms.size, L), -7, np.int32))
        items.append((p, to_dev(data), out))
        outs.append(out)
    with arts.Batch() as b:
        st = b.dedisperse(items)
    for i, ((w, delays, data), s, out) in enumerate(zip(reqs, st, outs)):
        got = out.cpu().numpy()
        if i == 4:
            assert s == arts.ARTS_E_SHAPE
            assert np.all(got == -7)          # skipped request left untouched
            continue
        assert s == arts.ARTS_OK
        for bm in range(data.shape[0]):
            x = data[bm] if w.downsample == 1 else O.downsample(data[bm], w.downsample)
            assert np.array_equal(got[bm], O.dedisperse(x, delays)), (i, bm)


def _native_variants():
    # byte-sample tilings that run plain plans (group-sum tilings run subband step 1 only)
    return [v for v in range(arts.arts_tiling_count())
            if "SPD=4" in arts.arts_tiling_describe(v)
            and "group" not in arts.arts_tiling_describe(v)]


@pytest.mark.parametrize("variant", _native_variants())
def test_batch_tilings_match_oracle(variant):
    # the persistent kernel of every byte-sample tiling (the native requests are set to it)
    reqs = [r for i, r in enumerate(_small_requests()) if r[0].downsample == 1 and i != 4]
    plans = [arts.Plan.from_workload(w) for w, _, _ in reqs]
    for p in plans:
        p.set_tiling(variant)
    items, outs = [], []
    for (w, delays, data), p in zip(reqs, plans):
        out = to_dev(np.zeros((data.shape[0], w.dms.size, arts.series_length(p, data.shape[2])),
                              np.int32))
        items.append((p, to_dev(data), out))
        outs.append(out)
    with arts.Batch() as b:
        st = b.dedisperse(items)
    for (w, delays, data), s, out in zip(reqs, st, outs):
        assert s == arts.ARTS_OK
        got = out.cpu().numpy()
        for bm in range(data.shape[0]):
            assert np.array_equal(got[bm], O.dedisperse(data[bm], delays)), (variant, bm)


def _uneven(n, seed):
    import torch
    reqs = synth.uneven_requests(n, seed=seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    items, plans = [], []
    for w in reqs:
        p = arts.Plan.from_workload(w)
        nin = w.extra["nsamp"]
        data = torch.randint(0, 256, (1, w.nchan, nin), dtype=torch.uint8, device="cuda",
                             generator=g)
        L = max(1, arts.series_length(p, nin))
        out = torch.empty((1, w.dms.size, L), dtype=torch.int32, device="cuda")
        items.append((p, data, out))
        plans.append(p)
    return reqs, items


def test_batch_equals_per_request_calls():
    import torch
    reqs, items = _uneven(16, seed=4)
    with arts.Batch() as b:
        st = b.dedisperse(items)
        torch.cuda.synchronize()
        nok = 0
        for (p, data, out), s in zip(items, st):
            if s != arts.ARTS_OK:
                with pytest.raises(arts.ArtsError):
                    p.dedisperse(data)
                continue
            ref = p.dedisperse(data)
            assert torch.equal(ref, out)
            nok += 1
        assert nok >= 4
        # candidates of the whole batch equal the per-request lists with shifted beams
        thr = 7.0
        got = b.candidates(items, thr)
        exp = []
        for i, ((p, data, out), s) in enumerate(zip(items, st)):
            if s == arts.ARTS_OK:
                c = p.candidates(out, thr, beam_offset=i)
                exp.append(c)
        exp = np.concatenate(exp) if exp else np.zeros(0, arts.CANDIDATE_DTYPE)
        assert np.array_equal(np.sort(got, order=["beam", "dm_index", "width", "sample"]),
                              np.sort(exp, order=["beam", "dm_index", "width", "sample"]))


def test_batch_sampled_against_oracle():
    # two full-size uneven requests checked point by point against the oracle
    import torch
    reqs, items = _uneven(16, seed=4)
    with arts.Batch() as b:
        st = b.dedisperse(items)
    done = 0
    rng = np.random.default_rng(3)
    for w, (p, data, out), s in zip(reqs, items, st):
        if s != arts.ARTS_OK or done >= 2:
            continue
        x = data.cpu().numpy()[0]
        delays = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
        got = out.cpu().numpy()[0]
        for d, t in zip(rng.integers(0, w.dms.size, 300), rng.integers(0, got.shape[1], 300)):
            assert got[d, t] == O.dedisperse_at(x, delays, d, t)
        done += 1
    assert done == 2


def test_persistent_kernel_keeps_the_per_job_occupancy():
    # a plan sizes its LDS chunks for the workgroups per CU of its tiling's one-launch kernel;
    # the persistent kernel that batches and the serving engine run on the same chunks must
    # reach as many, or the batched launches lose a workgroup per CU
    for v in range(arts.arts_tiling_count()):
        per_job, persistent = arts.arts_tiling_occupancy(v)
        assert per_job >= 1, v
        if "group" in arts.arts_tiling_describe(v):
            assert persistent == 0, v
        else:
            assert persistent >= per_job, (v, arts.arts_tiling_describe(v), per_job, persistent)

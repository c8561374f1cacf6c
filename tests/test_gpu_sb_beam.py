"""GPU parity with SB tables from the beam model (arts_sb_table_beam_model): SBs formed on the
fly by the dedispersion kernel from 12 TABs with the model's table equal the oracle's
sb_synthesize + dedisperse, at the Apertif shape (71 SBs x 1536 channels, sampled SBs, every
output of them) and in a stream of 151 SBs (the half-beam-width table)."""
import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth
from tests._parity import to_dev

pytestmark = pytest.mark.gpu


def test_model_table_fused_sb_full_shape():
    nchan, ntab, nsb = 1536, 12, 71
    f_lo, df = synth.band(nchan)
    table, margin = arts.arts_sb_table_beam_model(nsb, ntab, nchan, f_lo, df)
    assert margin > 1e-4
    dms = np.arange(0, 512, 2.0)
    p = arts.Plan(nchan, f_lo, df, synth.TSAMP, dms, [1, 2, 4])
    delays = O.delay_table(nchan, f_lo, df, synth.TSAMP, dms)
    tab = synth.noise((ntab, nchan, p.max_delay + 1500), seed=81)
    print("model table fused SB: 12 TABs x 1536 ch -> 71 SBs", flush=True)
    got = p.dedisperse_sb(to_dev(tab), to_dev(table)).cpu().numpy()
    for s in (0, 17, 35, 36, 52, 70):          # edge, middle and centre SBs
        sb = O.sb_synthesize(tab, table[s:s + 1])[0]
        assert np.array_equal(got[s], O.dedisperse(sb, delays)), s


def test_model_table_stream_151_sbs():
    nchan, ntab, nsb, chunk = 192, 12, 151, 2000
    f_lo, df = synth.band(nchan)
    table, _ = arts.arts_sb_table_beam_model(nsb, ntab, nchan, f_lo, df, quarter=True)
    dms = np.arange(0, 300, 4.0)
    p = arts.Plan(nchan, f_lo, df, synth.TSAMP, dms, [1, 2, 4, 8])
    delays = O.delay_table(nchan, f_lo, df, synth.TSAMP, dms)
    chunks = [synth.noise((ntab, nchan, chunk), seed=90 + k) for k in range(3)]
    H = p.halo
    full = np.concatenate([np.zeros((ntab, nchan, H), np.uint8)] + chunks, axis=2)
    with arts.Stream([p], ntab, chunk, 7.0, sb_table=to_dev(table), nbeam=nsb) as st:
        for k, c in enumerate(chunks):
            st.push(to_dev(c))
            st.wait()
            got = st.series(0).cpu().numpy()
            win = full[:, :, k * chunk: H + (k + 1) * chunk]
            for s in (0, 40, 75, 76, 150):
                sb = O.sb_synthesize(win, table[s:s + 1])[0]
                assert np.array_equal(got[s], O.dedisperse(sb, delays)), (k, s)

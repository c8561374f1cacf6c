"""CPU-side checks of the C ABI: the library loads, exports every entry point include/arts.h
declares, and its host-only logic (validation, FP64 delay table) matches the oracle.  No
device call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2205_12362_amd import arts, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "arts.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(arts_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = arts.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    # the binding covers every declared entry point under the same name
    missing = set(names) - set(arts.exported_symbols()) - set(dir(arts))
    assert not missing, missing


def test_version_and_tilings():
    assert "gfx950" in arts.arts_version()
    n = arts.arts_tiling_count()
    assert n >= 4
    for v in range(n):
        s = arts.arts_tiling_describe(v)
        assert s.startswith("J=") and "SPD=" in s
    with pytest.raises(arts.ArtsError):
        arts.arts_tiling_describe(n)
    for bad in (-1, n):  # rejected before any device query
        with pytest.raises(arts.ArtsError):
            arts.arts_tiling_occupancy(bad)


@pytest.mark.parametrize("make", [synth.cfg_small, synth.cfg_apertif, synth.cfg_apertif_ds])
def test_delay_table_matches_oracle(make):
    w = make()
    got, margin = arts.arts_delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms, w.downsample)
    ref, x = O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms, w.downsample,
                           return_exact=True)
    assert np.array_equal(got, ref)
    assert abs(margin - O.tie_audit(x)) < 1e-9


def test_delay_table_uneven_requests():
    for w in synth.uneven_requests(8):
        got, _ = arts.arts_delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms)
        assert np.array_equal(got, O.delay_table(w.nchan, w.f_lo, w.df, w.tsamp, w.dms))


def test_delay_table_descending_band():
    f_lo, df = synth.band(96)
    f_hi = f_lo + 95 * df
    dms = np.arange(40) * 3.0
    got, _ = arts.arts_delay_table(96, f_hi, -df, 1e-4, dms)
    assert np.array_equal(got, O.delay_table(96, f_hi, -df, 1e-4, dms))


@pytest.mark.parametrize("args", [
    (0, 1400.0, 1.0, 1e-3, [1.0], 1),          # nchan
    (4, 1400.0, 0.0, 1e-3, [1.0], 1),          # df
    (4, 1400.0, 1.0, 0.0, [1.0], 1),           # tsamp
    (4, 1400.0, 1.0, 1e-3, [-1.0], 1),         # negative DM
    (4, 1400.0, 1.0, 1e-3, [float("inf")], 1),
    (4, 1400.0, 1.0, 1e-3, [1.0], 0),          # downsample
    (4, -10.0, 1.0, 1e-3, [1.0], 1),           # negative frequency
    (4, 1.0, 1.0, 1e-9, [1e6], 1),             # delay above 2^30
])
def test_delay_table_rejects(args):
    with pytest.raises(arts.ArtsError) as e:
        arts.arts_delay_table(*args)
    assert e.value.status == arts.ARTS_E_INVAL


def test_strerror():
    L = arts.lib()
    for st in range(-7, 1):
        assert L.arts_strerror(st)
    assert ctypes.sizeof(arts.Candidate) == 32


@pytest.mark.parametrize("nsb,nchan,quarter", [(71, 1536, False), (151, 1536, True),
                                               (71, 384, False), (9, 100, True), (1, 16, False)])
def test_sb_table_beam_model_matches_oracle(nsb, nchan, quarter):
    # host-only call: the library's beam-model SB table equals the oracle's, switch margins too
    f_lo, df = synth.band(nchan)
    got, margin = arts.arts_sb_table_beam_model(nsb, 12, nchan, f_lo, df, quarter=quarter)
    ref, rmargin = O.sb_table_beam_model(nsb, 12, nchan, f_lo, df, quarter=quarter)
    assert np.array_equal(got, ref)
    assert margin == rmargin


@pytest.mark.parametrize("args", [(71, 11, 64), (71, 0, 64), (0, 12, 64), (71, 12, 0)])
def test_sb_table_beam_model_rejects(args):
    nsb, ntab, nchan = args
    with pytest.raises(arts.ArtsError):
        arts.arts_sb_table_beam_model(nsb, ntab, max(nchan, 1) if nchan else 0, 1220.0, 0.2)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    # no fallback: with libarts.so absent every call raises instead of computing elsewhere
    monkeypatch.setattr(arts, "_lib", None)
    monkeypatch.setattr(arts, "LIB_PATH", str(tmp_path / "libarts.so"))
    with pytest.raises(RuntimeError, match="is missing"):
        arts.lib()
    with pytest.raises(RuntimeError, match="is missing"):
        arts.arts_tiling_count()

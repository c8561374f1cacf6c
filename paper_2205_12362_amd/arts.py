"""Thin Python binding of libarts.so (ctypes).  Argument marshalling only: every step of the
search runs in the library's HIP kernels; torch is used for device memory and streams.

The functions carry the C names.  Device arrays are torch tensors on the GPU; host arrays are
numpy arrays or Python sequences.  A non-zero status raises ArtsError.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libarts.so")
_lib = None

ARTS_OK, ARTS_E_INVAL, ARTS_E_SHAPE, ARTS_E_NOMEM = 0, -1, -2, -3
ARTS_E_DEVICE, ARTS_E_CAPACITY, ARTS_E_BUDGET, ARTS_E_STATE = -4, -5, -6, -7


class ArtsError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(what)


class Request(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("in_", C.c_void_p), ("nbeam", C.c_int32),
                ("nin", C.c_int64), ("out", C.c_void_p)]


class Candidate(C.Structure):
    _fields_ = [("sample", C.c_int64), ("beam", C.c_int32), ("dm_index", C.c_int32),
                ("width", C.c_int32), ("downsample", C.c_int32), ("snr", C.c_float),
                ("dm", C.c_float)]


CANDIDATE_DTYPE = np.dtype([("sample", "<i8"), ("beam", "<i4"), ("dm_index", "<i4"),
                            ("width", "<i4"), ("downsample", "<i4"), ("snr", "<f4"),
                            ("dm", "<f4")])
assert CANDIDATE_DTYPE.itemsize == C.sizeof(Candidate) == 32

_vp, _i32, _i64, _f64, _f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float
_pi32, _pi64, _pf64 = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double)

_SIGNATURES = {
    "arts_delay_table": (C.c_int, [_i32, _f64, _f64, _f64, _pf64, _i32, _i32, _pi32, _pf64]),
    "arts_plan_create": (C.c_int, [_i32, _f64, _f64, _f64, _pf64, _i32, _pi32, _i32,
                                   C.POINTER(_vp)]),
    "arts_plan_create_ds": (C.c_int, [_i32, _f64, _f64, _f64, _pf64, _i32, _pi32, _i32, _i32,
                                      C.POINTER(_vp)]),
    "arts_plan_create_subband": (C.c_int, [_i32, _f64, _f64, _f64, _f64, _f64, _i32, _i32, _i32,
                                           _pi32, _i32, C.POINTER(_vp)]),
    "arts_plan_subband_info": (C.c_int, [_vp, _pi32, _pi32, _pi32, _pi32, _pi32]),
    "arts_plan_destroy": (None, [_vp]),
    "arts_plan_info": (C.c_int, [_vp, _pi32, _pi32, _pi32, _pi32, _pi32, _pi32]),
    "arts_plan_delays": (C.c_int, [_vp, _pi32]),
    "arts_plan_set_tiling": (C.c_int, [_vp, _i32]),
    "arts_plan_get_tiling": (C.c_int, [_vp, _pi32]),
    "arts_plan_set_tiling_shape": (C.c_int, [_vp, _i32, _i32, _i32]),
    "arts_plan_get_tiling_shape": (C.c_int, [_vp, _pi32, _pi32, _pi32]),
    "arts_batch_autotune": (C.c_int, [_vp, _vp, _i32, _i32, _pi32, C.POINTER(C.c_float)]),
    "arts_plan_set_cluster": (C.c_int, [_vp, _i32]),
    "arts_plan_get_cluster": (C.c_int, [_vp, _pi32]),
    "arts_plan_set_integration": (C.c_int, [_vp, _i32]),
    "arts_plan_get_integration": (C.c_int, [_vp, _pi32]),
    "arts_plan_cluster": (C.c_int, [_vp, _vp, _i64, _i32, _i32, _pi64, _vp]),
    "arts_cluster_offline": (C.c_int, [_vp, _i64, _i64, _pf64, _i32, _f32, _vp, _i64, _pi64,
                                       _vp]),
    "arts_rfi_clean": (C.c_int, [_vp, _i32, _i32, _i64, _i64, _f32, _i32, _f32, _i32, _vp]),
    "arts_sb_table_beam_model": (C.c_int, [_i32, _i32, _i32, _f64, _f64, _f64, _f64, _f64, _f64,
                                           _i32, _vp, _pf64]),
    "arts_stream_set_rfi": (C.c_int, [_vp, _f32, _i32, _f32, _i32]),
    "arts_tiling_count": (_i32, []),
    "arts_plan_autotune": (C.c_int, [_vp, _i32, _i64, _i32, C.c_char_p, _pi32,
                                     C.POINTER(C.c_float)]),
    "arts_tiling_describe": (C.c_int, [_i32, C.c_char_p, _i32]),
    "arts_tiling_occupancy": (C.c_int, [_i32, _pi32, _pi32]),
    "arts_sb_synthesize": (C.c_int, [_vp, _i32, _vp, _i32, _i32, _i64, _vp, _vp]),
    "arts_dedisperse": (C.c_int, [_vp, _vp, _i32, _i64, _vp, _vp]),
    "arts_dedisperse_sb": (C.c_int, [_vp, _vp, _i32, _vp, _i32, _i64, _vp, _vp]),
    "arts_boxcar_snr": (C.c_int, [_vp, _vp, _i32, _i64, _vp, _vp, _vp, _vp]),
    "arts_candidates": (C.c_int, [_vp, _vp, _i32, _i64, _f32, _i64, _i32, _vp, _i64, _pi64,
                                  _vp]),
    "arts_candidates_noalloc": (C.c_int, [_vp, _vp, _i32, _i64, _f32, _i64, _i32, _vp, _i64,
                                          _pi64, _vp]),
    "arts_stream_create": (C.c_int, [C.POINTER(_vp), _i32, _i32, _vp, _i32, _i64, _f32, _i64,
                                     C.c_uint32, C.POINTER(_vp)]),
    "arts_stream_input": (C.c_int, [_vp, C.POINTER(_vp)]),
    "arts_stream_push": (C.c_int, [_vp, _vp, _vp]),
    "arts_stream_wait": (C.c_int, [_vp, _vp, _i64, _pi64, _pi64]),
    "arts_stream_info": (C.c_int, [_vp, _pi64, _pi64, _pi64]),
    "arts_stream_warmup": (C.c_int, [_vp, _i32, _i64, _pi64]),
    "arts_stream_timing": (C.c_int, [_vp, _i32, _pf64, _pi64]),
    "arts_stream_series": (C.c_int, [_vp, _i32, C.POINTER(_vp), _pi64]),
    "arts_stream_snapshot_bytes": (C.c_int, [_vp, _pi64]),
    "arts_stream_snapshot": (C.c_int, [_vp, _vp, _i64, _pi64]),
    "arts_stream_restore": (C.c_int, [_vp, _vp, _i64, _i64]),
    "arts_stream_destroy": (None, [_vp]),
    "arts_batch_create": (C.c_int, [C.POINTER(_vp)]),
    "arts_batch_destroy": (None, [_vp]),
    "arts_batch_dedisperse": (C.c_int, [_vp, _vp, _i32, _pi32, _vp]),
    "arts_batch_candidates": (C.c_int, [_vp, _vp, _i32, _f32, _vp, _i64, _pi64, _vp]),
    "arts_server_create": (C.c_int, [_i64, C.POINTER(_vp)]),
    "arts_server_destroy": (None, [_vp]),
    "arts_server_open": (C.c_int, [_vp, C.POINTER(_vp), _i32, _i32, _vp, _i32, _i64, _f32, _i64,
                                   _pi32]),
    "arts_server_close": (C.c_int, [_vp, _i32]),
    "arts_server_submit": (C.c_int, [_vp, _i32, _vp, _i32]),
    "arts_server_tick": (C.c_int, [_vp, _pi32]),
    "arts_server_collect": (C.c_int, [_vp, _i32, _vp, _i64, _pi64, _pi64]),
    "arts_server_poll": (C.c_int, [_vp, _i32, _pi32]),
    "arts_server_set_lanes": (C.c_int, [_vp, _i32]),
    "arts_server_stream": (C.c_int, [_vp, _i32, C.POINTER(_vp)]),
    "arts_server_info": (C.c_int, [_vp, _pi64, _pi64, _pi32]),
    "arts_strerror": (C.c_char_p, [C.c_int]),
    "arts_last_error": (C.c_char_p, []),
    "arts_version": (C.c_char_p, []),
}


def lib():
    """Load libarts.so from the package directory (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2205_12362_amd.build` first")
        # The library shares torch's HIP runtime; let torch bring the device up first so both
        # see the same initialised runtime and current device.
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
                torch.cuda.current_device()
        except ImportError:  # pragma: no cover - torch is the memory/stream provider
            pass
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(h, name)
            f.restype, f.argtypes = res, args
        _lib = h
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


def _check(status: int):
    if status != ARTS_OK:
        L = lib()
        raise ArtsError(status, f"{L.arts_strerror(status).decode()}: "
                                f"{L.arts_last_error().decode()}")


def _f64arr(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    return a, a.ctypes.data_as(_pf64)


def _i32arr(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.int32))
    return a, a.ctypes.data_as(_pi32)


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------------------- host only
def arts_delay_table(nchan, f_lo, df, tsamp, dms, downsample=1):
    """Delay table int32 [ndm][nchan] and the tie margin (host-only call)."""
    d, dp = _f64arr(dms)
    out = np.zeros((len(d), nchan), dtype=np.int32)
    margin = C.c_double(0.0)
    _check(lib().arts_delay_table(int(nchan), float(f_lo), float(df), float(tsamp), dp, len(d),
                                  int(downsample), out.ctypes.data_as(_pi32), C.byref(margin)))
    return out, margin.value


def arts_tiling_count():
    return int(lib().arts_tiling_count())


def arts_tiling_describe(variant):
    buf = C.create_string_buffer(128)
    _check(lib().arts_tiling_describe(int(variant), buf, 128))
    return buf.value.decode()


def arts_tiling_occupancy(variant):
    """(per_job, persistent): workgroups per CU that registers and waves allow for the
    variant's one-launch kernel and for its persistent batch kernel (0: none)."""
    a, b = C.c_int32(), C.c_int32()
    _check(lib().arts_tiling_occupancy(int(variant), C.byref(a), C.byref(b)))
    return a.value, b.value


def arts_version():
    return lib().arts_version().decode()


# ---------------------------------------------------------------------------- plans
def arts_plan_create(nchan, f_lo, df, tsamp, dms, widths):
    d, dp = _f64arr(dms)
    w, wp = _i32arr(widths)
    h = _vp()
    _check(lib().arts_plan_create(int(nchan), float(f_lo), float(df), float(tsamp), dp, len(d),
                                  wp, len(w), C.byref(h)))
    return h


def arts_plan_create_ds(nchan, f_lo, df, tsamp, dms, widths, downsample):
    d, dp = _f64arr(dms)
    w, wp = _i32arr(widths)
    h = _vp()
    _check(lib().arts_plan_create_ds(int(nchan), float(f_lo), float(df), float(tsamp), dp,
                                     len(d), wp, len(w), int(downsample), C.byref(h)))
    return h


def arts_plan_create_subband(nchan, f_lo, df, tsamp, dm_first, dm_step, ndm, nfine, nsub,
                             widths):
    w, wp = _i32arr(widths)
    h = _vp()
    _check(lib().arts_plan_create_subband(int(nchan), float(f_lo), float(df), float(tsamp),
                                          float(dm_first), float(dm_step), int(ndm), int(nfine),
                                          int(nsub), wp, len(w), C.byref(h)))
    return h


def arts_plan_subband_info(plan):
    v = [C.c_int32() for _ in range(5)]
    _check(lib().arts_plan_subband_info(plan, *[C.byref(x) for x in v]))
    return dict(zip(("nsub", "nfine", "ncoarse", "max_delay1", "max_delay2"),
                    (x.value for x in v)))


def arts_plan_destroy(plan):
    lib().arts_plan_destroy(plan)


def arts_plan_info(plan):
    v = [C.c_int32() for _ in range(6)]
    _check(lib().arts_plan_info(plan, *[C.byref(x) for x in v]))
    keys = ("nchan", "ndm", "nwidth", "downsample", "max_delay", "halo")
    return {k: x.value for k, x in zip(keys, v)}


def arts_plan_delays(plan):
    info = arts_plan_info(plan)
    out = np.zeros((info["ndm"], info["nchan"]), dtype=np.int32)
    _check(lib().arts_plan_delays(plan, out.ctypes.data_as(_pi32)))
    return out


def arts_plan_set_tiling(plan, variant):
    _check(lib().arts_plan_set_tiling(plan, int(variant)))


def arts_plan_autotune(plan, nbeam, nin, reps=3, cache_path=None):
    """Pick the fastest tiling for this shape (cached in cache_path); returns (variant, ms)."""
    v, ms = C.c_int32(), C.c_float()
    path = cache_path.encode() if cache_path else None
    _check(lib().arts_plan_autotune(plan, int(nbeam), int(nin), int(reps), path, C.byref(v),
                                    C.byref(ms)))
    return v.value, ms.value


def arts_plan_get_tiling(plan):
    v = C.c_int32()
    _check(lib().arts_plan_get_tiling(plan, C.byref(v)))
    return v.value


def arts_plan_set_tiling_shape(plan, variant, buffers=1, channels=0):
    _check(lib().arts_plan_set_tiling_shape(plan, int(variant), int(buffers), int(channels)))


def arts_plan_get_tiling_shape(plan):
    """(variant, buffers, channels per chunk) in use."""
    v, nb, cc = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().arts_plan_get_tiling_shape(plan, C.byref(v), C.byref(nb), C.byref(cc)))
    return v.value, nb.value, cc.value


# ---------------------------------------------------------------------------- hot path
def arts_sb_synthesize(tab, sb_table, out=None, stream=None):
    import torch
    ntab, nchan, nsamp = tab.shape
    nsb = sb_table.shape[0]
    if sb_table.shape != (nsb, nchan):
        raise ValueError("sb_table must be [nsb][nchan]")
    if out is None:
        out = torch.empty((nsb, nchan, nsamp), dtype=torch.uint8, device=tab.device)
    _check(lib().arts_sb_synthesize(_dev(tab, torch.uint8, "tab"), ntab,
                                    _dev(sb_table, torch.uint8, "sb_table"), nsb, nchan, nsamp,
                                    _dev(out, torch.uint8, "out"), _stream(stream)))
    return out


def _series_len(plan, nin):
    info = arts_plan_info(plan)
    return info, nin // info["downsample"] - info["max_delay"]


def arts_dedisperse(plan, data, out=None, stream=None):
    """data: uint8 [nbeam][nchan][nin] (or [nchan][nin]) -> int32 [nbeam][ndm][L]."""
    import torch
    if data.dim() == 2:
        data = data.unsqueeze(0)
    nbeam, nchan, nin = data.shape
    info, L = _series_len(plan, nin)
    if nchan != info["nchan"]:
        raise ValueError("channel count does not match the plan")
    if out is None:
        out = torch.empty((nbeam, info["ndm"], max(L, 1)), dtype=torch.int32, device=data.device)
    _check(lib().arts_dedisperse(plan, _dev(data, torch.uint8, "data"), nbeam, nin,
                                 _dev(out, torch.int32, "out"), _stream(stream)))
    return out


def arts_dedisperse_sb(plan, tab, sb_table, out=None, stream=None):
    import torch
    ntab, nchan, nin = tab.shape
    nsb = sb_table.shape[0]
    info, L = _series_len(plan, nin)
    if nchan != info["nchan"] or sb_table.shape != (nsb, nchan):
        raise ValueError("shapes do not match the plan")
    if out is None:
        out = torch.empty((nsb, info["ndm"], max(L, 1)), dtype=torch.int32, device=tab.device)
    _check(lib().arts_dedisperse_sb(plan, _dev(tab, torch.uint8, "tab"), ntab,
                                    _dev(sb_table, torch.uint8, "sb_table"), nsb, nin,
                                    _dev(out, torch.int32, "out"), _stream(stream)))
    return out


def arts_boxcar_snr(plan, series, want_stats=True, want_sums=True, want_snr=True, stream=None):
    """series int32 [nbeam][ndm][L] -> (stats f64 [nbeam][ndm][2], sums i32
    [nbeam][nw][ndm][nrep], snr f32 [nbeam][nw][ndm][nrep]); unrequested outputs are None."""
    import torch
    nbeam, ndm, L = series.shape
    info = arts_plan_info(plan)
    nrep = L - (info["halo"] - info["max_delay"])
    dev = series.device
    stats = torch.empty((nbeam, ndm, 2), dtype=torch.float64, device=dev) if want_stats else None
    shape = (nbeam, info["nwidth"], ndm, max(nrep, 1))
    sums = torch.empty(shape, dtype=torch.int32, device=dev) if want_sums else None
    snr = torch.empty(shape, dtype=torch.float32, device=dev) if want_snr else None
    _check(lib().arts_boxcar_snr(plan, _dev(series, torch.int32, "series"), nbeam, L,
                                 stats.data_ptr() if stats is not None else None,
                                 sums.data_ptr() if sums is not None else None,
                                 snr.data_ptr() if snr is not None else None, _stream(stream)))
    return stats, sums, snr


def arts_candidates(plan, series, threshold, t_offset=0, beam_offset=0, capacity=1 << 16,
                    stream=None):
    """Candidates as a numpy structured array (CANDIDATE_DTYPE), sorted by (beam, dm, width,
    sample).  Grows the buffer and retries once if `capacity` is too small."""
    import torch
    nbeam, ndm, L = series.shape
    for _ in range(2):
        buf = np.zeros(max(int(capacity), 1), dtype=CANDIDATE_DTYPE)
        n = C.c_int64(0)
        st = lib().arts_candidates(plan, _dev(series, torch.int32, "series"), nbeam, L,
                                   float(threshold), int(t_offset), int(beam_offset),
                                   buf.ctypes.data, int(capacity), C.byref(n), _stream(stream))
        if st == ARTS_E_CAPACITY:
            capacity = n.value
            continue
        _check(st)
        return buf[: n.value].copy()
    _check(st)


NOALLOC_MAX_ROWS = 1048576
NOALLOC_MAX_CANDIDATES = 491512


def arts_candidates_noalloc(plan, series, threshold, t_offset=0, beam_offset=0,
                            capacity=1 << 16, stream=None):
    """arts_candidates on the library's fixed device array (no device allocation); same result
    layout.  Raises ArtsError(ARTS_E_CAPACITY) if `capacity` is too small (no retry: a larger
    host buffer is the caller's business)."""
    import torch
    nbeam, ndm, L = series.shape
    buf = np.zeros(max(int(capacity), 1), dtype=CANDIDATE_DTYPE)
    n = C.c_int64(0)
    _check(lib().arts_candidates_noalloc(plan, _dev(series, torch.int32, "series"), nbeam, L,
                                         float(threshold), int(t_offset), int(beam_offset),
                                         buf.ctypes.data, int(capacity), C.byref(n),
                                         _stream(stream)))
    return buf[: n.value].copy()


def arts_plan_set_cluster(plan, enable):
    _check(lib().arts_plan_set_cluster(plan, int(enable)))


def arts_plan_set_integration(plan, mode):
    """mode 0 / "sliding" (default) or 1 / "decimated" (each width's absolute grid)."""
    mode = {"sliding": 0, "decimated": 1}.get(mode, mode)
    _check(lib().arts_plan_set_integration(plan, int(mode)))


def arts_plan_get_integration(plan):
    v = C.c_int32(0)
    _check(lib().arts_plan_get_integration(plan, C.byref(v)))
    return ("sliding", "decimated")[v.value]


def arts_plan_get_cluster(plan):
    v = C.c_int32(0)
    _check(lib().arts_plan_get_cluster(plan, C.byref(v)))
    return bool(v.value)


def arts_plan_cluster(plan, cand, nbeam, beam_offset=0, stream=None):
    """Cluster a device candidate list in place.  `cand` is a device uint8 tensor of n * 32
    bytes (arts_candidate records) or a numpy CANDIDATE_DTYPE array (copied to the device);
    returns the clusters as a numpy array sorted by (beam, dm, width, sample)."""
    cand = _device_records(cand)
    n = cand.numel() // 32
    cnt = C.c_int64(0)
    _check(lib().arts_plan_cluster(plan, cand.data_ptr() if n else None, n, int(nbeam),
                                   int(beam_offset), C.byref(cnt), _stream(stream)))
    out = cand[: cnt.value * 32].cpu().numpy().view(CANDIDATE_DTYPE).copy()
    out.sort(order=["beam", "dm_index", "width", "sample"])
    return out


def _device_records(cand):
    import torch
    if isinstance(cand, np.ndarray):
        cand = torch.from_numpy(np.ascontiguousarray(cand, dtype=CANDIDATE_DTYPE)
                                .view(np.uint8)).cuda()
    if cand.dtype != torch.uint8 or not cand.is_cuda or cand.numel() % 32:
        raise ValueError("cand must be a device uint8 tensor of whole 32-byte records")
    return cand


def arts_cluster_offline(cand, t_window, dm_edges, min_snr, capacity=None, stream=None):
    """Offline time/DM-window clustering of a candidate list (numpy CANDIDATE_DTYPE array or
    device uint8 tensor of records); returns the kept candidates as a numpy array."""
    cand = _device_records(cand)
    n = cand.numel() // 32
    edges = np.ascontiguousarray(dm_edges, dtype=np.float64)
    capacity = max(1, n) if capacity is None else int(capacity)
    buf = np.zeros(max(capacity, 1), dtype=CANDIDATE_DTYPE)
    cnt = C.c_int64(0)
    _check(lib().arts_cluster_offline(cand.data_ptr() if n else None, n, int(t_window),
                                      edges.ctypes.data_as(_pf64), edges.size, float(min_snr),
                                      buf.ctypes.data, capacity, C.byref(cnt), _stream(stream)))
    return buf[: cnt.value].copy()


def arts_rfi_clean(data, k_time, k_freq, niter_time=3, niter_freq=3, nsamp=None, stream=None):
    """Clean a device uint8 tensor [nrow][nchan][pitch] in place (the first nsamp samples of
    each row, default all)."""
    import torch
    if data.dtype != torch.uint8 or not data.is_cuda or data.dim() != 3 or not \
            data.is_contiguous():
        raise ValueError("data must be a contiguous device uint8 tensor [nrow][nchan][pitch]")
    nrow, nchan, pitch = data.shape
    _check(lib().arts_rfi_clean(data.data_ptr(), nrow, nchan,
                                pitch if nsamp is None else int(nsamp), pitch, float(k_time),
                                int(niter_time), float(k_freq), int(niter_freq),
                                _stream(stream)))
    return data


def arts_sb_table_beam_model(nsb, ntab, nchan, f_lo, df, f_max=1500.0, alpha=0.80,
                             b_max=1296.0, b_cq=144.0, quarter=False):
    """SB table [nsb][nchan] (numpy uint8) from the beam model, and its switch margin (MHz)."""
    out = np.zeros((int(nsb), int(nchan)), dtype=np.uint8)
    m = C.c_double()
    _check(lib().arts_sb_table_beam_model(int(nsb), int(ntab), int(nchan), float(f_lo), float(df),
                                          float(f_max), float(alpha), float(b_max), float(b_cq),
                                          int(bool(quarter)), out.ctypes.data, C.byref(m)))
    return out, m.value


def offline_dm_edges(dm_lo=20.0, dm_hi=5000.0, ratio=1.1):
    """DM window edges that widen with DM: dm_lo, dm_lo * ratio, ... up to dm_hi (the paper's
    DM limit is 20; it does not give the widths, so the 10 % growth is this helper's choice)."""
    e = [float(dm_lo)]
    while e[-1] * ratio < dm_hi:
        e.append(e[-1] * ratio)
    return np.array(e)


class Plan:
    """Owning wrapper around an arts_plan_t."""

    def __init__(self, nchan, f_lo, df, tsamp, dms, widths, downsample=1):
        self.dms = np.asarray(dms, dtype=np.float64)
        self.widths = [int(w) for w in widths]
        if downsample == 1:
            self.handle = arts_plan_create(nchan, f_lo, df, tsamp, self.dms, self.widths)
        else:
            self.handle = arts_plan_create_ds(nchan, f_lo, df, tsamp, self.dms, self.widths,
                                              downsample)
        self.info = arts_plan_info(self.handle)

    @classmethod
    def from_workload(cls, w):
        return cls(w.nchan, w.f_lo, w.df, w.tsamp, w.dms, w.widths, w.downsample)

    @classmethod
    def subband(cls, nchan, f_lo, df, tsamp, dm_first, dm_step, ndm, nfine, nsub, widths):
        """Two-step subband plan (arts_plan_create_subband); dms are the fine trials."""
        self = cls.__new__(cls)
        self.dms = dm_first + dm_step * np.arange(int(ndm), dtype=np.float64)
        self.widths = [int(w) for w in widths]
        self.handle = arts_plan_create_subband(nchan, f_lo, df, tsamp, dm_first, dm_step, ndm,
                                               nfine, nsub, self.widths)
        self.info = arts_plan_info(self.handle)
        return self

    def subband_info(self):
        return arts_plan_subband_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            arts_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def halo(self):
        return self.info["halo"]

    @property
    def max_delay(self):
        return self.info["max_delay"]

    def delays(self):
        return arts_plan_delays(self.handle)

    def set_tiling(self, variant):
        arts_plan_set_tiling(self.handle, variant)

    def autotune(self, nbeam, nin, reps=3, cache_path=None):
        return arts_plan_autotune(self.handle, nbeam, nin, reps, cache_path)

    def tiling(self):
        return arts_plan_get_tiling(self.handle)

    def set_tiling_shape(self, variant, buffers=1, channels=0):
        arts_plan_set_tiling_shape(self.handle, variant, buffers, channels)

    def tiling_shape(self):
        return arts_plan_get_tiling_shape(self.handle)

    def dedisperse(self, data, out=None, stream=None):
        return arts_dedisperse(self.handle, data, out, stream)

    def dedisperse_sb(self, tab, sb_table, out=None, stream=None):
        return arts_dedisperse_sb(self.handle, tab, sb_table, out, stream)

    def boxcar_snr(self, series, **kw):
        return arts_boxcar_snr(self.handle, series, **kw)

    def candidates(self, series, threshold, **kw):
        return arts_candidates(self.handle, series, threshold, **kw)

    @property
    def cluster(self):
        return arts_plan_get_cluster(self.handle)

    @cluster.setter
    def cluster(self, enable):
        arts_plan_set_cluster(self.handle, enable)

    @property
    def integration(self):
        return arts_plan_get_integration(self.handle)

    @integration.setter
    def integration(self, mode):
        arts_plan_set_integration(self.handle, mode)

    def cluster_candidates(self, cand, nbeam, beam_offset=0, stream=None):
        return arts_plan_cluster(self.handle, cand, nbeam, beam_offset, stream)


# ---------------------------------------------------------------------------- streaming
ARTS_STREAM_GRAPH, ARTS_STREAM_PROFILE = 1, 2


def arts_stream_create(plans, nsrc, sb_table, nbeam, chunk, threshold, cand_capacity=1 << 16,
                       flags=0):
    import torch
    handles = (_vp * len(plans))(*[p.handle if isinstance(p, Plan) else p for p in plans])
    tbl = _dev(sb_table, torch.uint8, "sb_table") if sb_table is not None else None
    h = _vp()
    _check(lib().arts_stream_create(handles, len(plans), int(nsrc), tbl, int(nbeam), int(chunk),
                                    float(threshold), int(cand_capacity), int(flags),
                                    C.byref(h)))
    return h


def arts_stream_input(stream_h):
    p = _vp()
    _check(lib().arts_stream_input(stream_h, C.byref(p)))
    return p.value


def arts_stream_push(stream_h, chunk=None, stream=None):
    import torch
    ptr = None if chunk is None else _dev(chunk, torch.uint8, "chunk")
    _check(lib().arts_stream_push(stream_h, ptr, _stream(stream)))


def arts_stream_wait(stream_h, capacity=1 << 16):
    buf = np.zeros(max(int(capacity), 1), dtype=CANDIDATE_DTYPE)
    n, k = C.c_int64(0), C.c_int64(0)
    _check(lib().arts_stream_wait(stream_h, buf.ctypes.data, int(capacity), C.byref(n),
                                  C.byref(k)))
    return buf[: n.value].copy(), k.value


def arts_stream_info(stream_h):
    a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().arts_stream_info(stream_h, C.byref(a), C.byref(b), C.byref(c)))
    return {"chunks": a.value, "device_bytes": b.value, "halo_native": c.value}


def arts_stream_warmup(stream_h, plan_index, chunk_index):
    t = C.c_int64()
    _check(lib().arts_stream_warmup(stream_h, int(plan_index), int(chunk_index), C.byref(t)))
    return t.value


def arts_stream_timing(stream_h, phase):
    ms, n = C.c_double(), C.c_int64()
    _check(lib().arts_stream_timing(stream_h, int(phase), C.byref(ms), C.byref(n)))
    return ms.value, n.value


def arts_stream_series(stream_h, plan_index, nbeam, ndm):
    import torch
    p, L = _vp(), C.c_int64()
    _check(lib().arts_stream_series(stream_h, int(plan_index), C.byref(p), C.byref(L)))
    return p.value, L.value


def arts_stream_snapshot_bytes(stream_h):
    n = C.c_int64()
    _check(lib().arts_stream_snapshot_bytes(stream_h, C.byref(n)))
    return n.value


def arts_stream_snapshot(stream_h, nbytes=None):
    if nbytes is None:
        nbytes = arts_stream_snapshot_bytes(stream_h)
    buf = np.zeros(int(nbytes), dtype=np.uint8)
    k = C.c_int64()
    _check(lib().arts_stream_snapshot(stream_h, buf.ctypes.data, buf.size, C.byref(k)))
    return buf, k.value


def arts_stream_restore(stream_h, buf, chunks_pushed):
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    _check(lib().arts_stream_restore(stream_h, buf.ctypes.data, buf.size, int(chunks_pushed)))


def arts_stream_destroy(stream_h):
    lib().arts_stream_destroy(stream_h)


class Stream:
    """Owning wrapper of an arts_stream_t; keeps its plans (and SB table) alive."""

    def __init__(self, plans, nsrc, chunk, threshold, sb_table=None, nbeam=None,
                 cand_capacity=1 << 16, graph=False, profile=False):
        self.plans = list(plans)
        self.sb_table = sb_table
        self.nbeam = nbeam if nbeam is not None else (sb_table.shape[0] if sb_table is not None
                                                      else nsrc)
        self.nsrc, self.chunk = nsrc, chunk
        flags = (ARTS_STREAM_GRAPH if graph else 0) | (ARTS_STREAM_PROFILE if profile else 0)
        self.handle = arts_stream_create(self.plans, nsrc, sb_table, self.nbeam, chunk,
                                         threshold, cand_capacity, flags)
        self.capacity = cand_capacity

    def input_buffer(self):
        """The stream's device staging buffer as a torch uint8 tensor view [nsrc][nchan][chunk]."""
        import torch
        nchan = self.plans[0].info["nchan"]
        ptr = arts_stream_input(self.handle)
        return _tensor_from_ptr(ptr, (self.nsrc, nchan, self.chunk), torch.uint8, self)

    def push(self, chunk=None, stream=None):
        arts_stream_push(self.handle, chunk, stream)

    def wait(self):
        return arts_stream_wait(self.handle, self.capacity)

    def info(self):
        return arts_stream_info(self.handle)

    def set_rfi(self, k_time, k_freq, niter_time=3, niter_freq=3):
        _check(lib().arts_stream_set_rfi(self.handle, float(k_time), int(niter_time),
                                         float(k_freq), int(niter_freq)))

    def timing(self, phase):
        return arts_stream_timing(self.handle, phase)

    def warmup(self, plan_index, chunk_index):
        """First output sample of that chunk the plan searches (chunk / D: none)."""
        return arts_stream_warmup(self.handle, plan_index, chunk_index)

    def warm_chunks(self):
        """Index of the first chunk that every plan searches in full."""
        k = 0
        while any(self.warmup(p, k) for p in range(len(self.plans))):
            k += 1
        return k

    def series(self, plan_index):
        """Last chunk's series of one plan as a torch int32 view [nbeam][ndm][L]."""
        import torch
        ndm = self.plans[plan_index].info["ndm"]
        ptr, L = arts_stream_series(self.handle, plan_index, self.nbeam, ndm)
        return _tensor_from_ptr(ptr, (self.nbeam, ndm, L), torch.int32, self)

    def snapshot(self):
        return arts_stream_snapshot(self.handle)

    def restore(self, buf, chunks_pushed):
        arts_stream_restore(self.handle, buf, chunks_pushed)

    def close(self):
        if getattr(self, "handle", None):
            arts_stream_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _tensor_from_ptr(ptr, shape, dtype, owner):
    """A torch view of library-owned device memory (valid while `owner` lives)."""
    import torch

    class _Holder:
        def __init__(self, ptr, nbytes, shape, typestr):
            self.__cuda_array_interface__ = {"shape": shape, "typestr": typestr,
                                             "data": (ptr, False), "version": 2,
                                             "strides": None}
    typestr = {torch.uint8: "|u1", torch.int32: "<i4"}[dtype]
    t = torch.as_tensor(_Holder(ptr, 0, tuple(shape), typestr), device="cuda")
    t._arts_owner = owner
    return t


# ---------------------------------------------------------------------------- batches
def arts_batch_create():
    h = _vp()
    _check(lib().arts_batch_create(C.byref(h)))
    return h


def arts_batch_destroy(batch_h):
    lib().arts_batch_destroy(batch_h)


def _requests(items):
    """items: (Plan, input tensor [nbeam][nchan][nin] uint8, output tensor int32)."""
    import torch
    arr = (Request * len(items))()
    for i, (plan, data, out) in enumerate(items):
        nbeam, nchan, nin = data.shape
        arr[i].plan = plan.handle if isinstance(plan, Plan) else plan
        arr[i].in_ = _dev(data, torch.uint8, "in")
        arr[i].nbeam = nbeam
        arr[i].nin = nin
        arr[i].out = _dev(out, torch.int32, "out")
    return arr


def arts_batch_dedisperse(batch_h, items, stream=None):
    """Returns the per-request status list (0 = done, ARTS_E_SHAPE = too short, skipped)."""
    arr = _requests(items)
    st = (C.c_int32 * len(items))()
    _check(lib().arts_batch_dedisperse(batch_h, arr, len(items), st, _stream(stream)))
    return list(st)


def arts_batch_candidates(batch_h, items, threshold, capacity=1 << 18, stream=None):
    arr = _requests(items)
    for _ in range(2):
        buf = np.zeros(max(int(capacity), 1), dtype=CANDIDATE_DTYPE)
        n = C.c_int64(0)
        st = lib().arts_batch_candidates(batch_h, arr, len(items), float(threshold),
                                         buf.ctypes.data, int(capacity), C.byref(n),
                                         _stream(stream))
        if st == ARTS_E_CAPACITY:
            capacity = n.value
            continue
        _check(st)
        return buf[: n.value].copy()
    _check(st)


def arts_batch_autotune(batch_h, items, reps=2):
    """One tile shape per sample kind for all requests (timed on them); returns (variant, ms)."""
    arr = _requests(items)
    v, ms = C.c_int32(), C.c_float()
    _check(lib().arts_batch_autotune(batch_h, arr, len(items), int(reps), C.byref(v),
                                     C.byref(ms)))
    return v.value, ms.value


class Batch:
    def __init__(self):
        self.handle = arts_batch_create()

    def dedisperse(self, items, stream=None):
        return arts_batch_dedisperse(self.handle, items, stream)

    def autotune(self, items, reps=2):
        return arts_batch_autotune(self.handle, items, reps)

    def candidates(self, items, threshold, **kw):
        return arts_batch_candidates(self.handle, items, threshold, **kw)

    def close(self):
        if getattr(self, "handle", None):
            arts_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def series_length(plan, nin):
    info = plan.info if isinstance(plan, Plan) else arts_plan_info(plan)
    return nin // info["downsample"] - info["max_delay"]


# ---------------------------------------------------------------------------- serving
class Server:
    """Continuous-batching serving engine (arts_server_*)."""

    def __init__(self, hbm_budget_bytes):
        h = _vp()
        _check(lib().arts_server_create(int(hbm_budget_bytes), C.byref(h)))
        self.handle = h
        self._keep = {}

    def open(self, plans, nsrc, chunk, threshold, sb_table=None, nbeam=None,
             cand_capacity=1 << 16):
        """Admit a stream; raises ArtsError (status ARTS_E_BUDGET) if it does not fit."""
        import torch
        handles = (_vp * len(plans))(*[p.handle if isinstance(p, Plan) else p for p in plans])
        tbl = _dev(sb_table, torch.uint8, "sb_table") if sb_table is not None else None
        nbeam = nbeam if nbeam is not None else (sb_table.shape[0] if sb_table is not None
                                                 else nsrc)
        sid = C.c_int32()
        _check(lib().arts_server_open(self.handle, handles, len(plans), int(nsrc), tbl,
                                      int(nbeam), int(chunk), float(threshold),
                                      int(cand_capacity), C.byref(sid)))
        self._keep[sid.value] = (list(plans), sb_table, int(cand_capacity), int(nbeam))
        return sid.value

    def close_stream(self, sid):
        _check(lib().arts_server_close(self.handle, int(sid)))
        self._keep.pop(sid, None)

    def submit(self, sid, chunk):
        """chunk: torch uint8 tensor [nsrc][nchan][chunk] on the GPU, or pinned on the host."""
        import torch
        if not chunk.is_contiguous() or chunk.dtype != torch.uint8:
            raise TypeError("chunk must be a contiguous uint8 tensor")
        _check(lib().arts_server_submit(self.handle, int(sid), chunk.data_ptr(),
                                        0 if chunk.is_cuda else 1))

    def tick(self):
        n = C.c_int32()
        _check(lib().arts_server_tick(self.handle, C.byref(n)))
        return n.value

    def poll(self, sid):
        """True once the stream's last step has finished (collect will not block)."""
        d = C.c_int32()
        _check(lib().arts_server_poll(self.handle, int(sid), C.byref(d)))
        return bool(d.value)

    def set_lanes(self, nlanes):
        _check(lib().arts_server_set_lanes(self.handle, int(nlanes)))

    def collect(self, sid):
        cap = self._keep[sid][2]
        buf = np.zeros(cap, dtype=CANDIDATE_DTYPE)
        n, k = C.c_int64(), C.c_int64()
        _check(lib().arts_server_collect(self.handle, int(sid), buf.ctypes.data, cap,
                                         C.byref(n), C.byref(k)))
        return buf[: n.value].copy(), k.value

    def series(self, sid, plan_index):
        import torch
        sh = _vp()
        _check(lib().arts_server_stream(self.handle, int(sid), C.byref(sh)))
        plans, _, _, nbeam = self._keep[sid]
        ndm = plans[plan_index].info["ndm"]
        ptr, L = arts_stream_series(sh, plan_index, nbeam, ndm)
        return _tensor_from_ptr(ptr, (nbeam, ndm, L), torch.int32, self)

    def info(self):
        u, b, n = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().arts_server_info(self.handle, C.byref(u), C.byref(b), C.byref(n)))
        return {"used_bytes": u.value, "budget": b.value, "streams": n.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().arts_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

"""ctypes binding of the C ABI (names follow include/gnss_acq.h)."""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

try:
    # Load PyTorch's HIP runtime first when it is present: the library then
    # binds to that same runtime (one runtime per process), which is also what
    # lets it run on torch-allocated memory and torch streams.
    import torch  # noqa: F401
except ImportError:  # plain C/numpy users get the system ROCm runtime
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgnss_acq.so")

GNSS_OK = 0
GNSS_EINVAL = -1
GNSS_ENOMEM = -2
GNSS_EDEVICE = -3
GNSS_EBUSY = -4
GNSS_ENOTSUP = -5

GNSS_REAL_I8 = 0
GNSS_CPLX_I8 = 1
GNSS_REAL_2BIT_PACKED = 2
GNSS_FP32 = 0
GNSS_FP16 = 1
GNSS_FP16_PFA = 2

EXPORTED = [
    "gnss_acquire", "gnss_ctx_create", "gnss_ctx_destroy", "gnss_ctx_set",
    "gnss_workspace_bytes", "gnss_acquire_device", "gnss_gold_codes", "gnss_code_replica",
    "gnss_nco_lut", "gnss_wipe_fold", "gnss_fft2048", "gnss_peaks", "gnss_stage_times",
    "gnss_strerror", "gnss_last_error", "gnss_acquire_batch_device", "gnss_graph_create",
    "gnss_graph_launch", "gnss_graph_destroy", "gnss_autotune", "gnss_submit", "gnss_poll",
    "gnss_wait", "gnss_track", "gnss_track_device", "gnss_dft1023", "gnss_box_fold",
    "gnss_acquire_device_noalloc",
]

GNSS_NOALLOC_SCRATCH_BYTES = 64 << 20
GNSS_NOALLOC_META_BYTES = 1 << 20

GNSS_STAGE_WIPE_FOLD = 0
GNSS_STAGE_FFT = 1
GNSS_STAGE_CORR = 2
GNSS_STAGE_DETECT = 3
GNSS_N_STAGES = 4
STAGE_NAMES = ["wipe_fold", "fft", "corr", "detect"]


class GnssError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (%d): %s" % (_strerror(code), code, message))
        self.code = code


class gnss_peak(ctypes.Structure):
    _fields_ = [("prn", ctypes.c_int32), ("doppler_bin", ctypes.c_int32),
                ("code_phase", ctypes.c_int32), ("detected", ctypes.c_int32),
                ("peak", ctypes.c_float), ("second", ctypes.c_float), ("mean", ctypes.c_float),
                ("ratio", ctypes.c_float), ("doppler_hz", ctypes.c_double),
                ("code_phase_frac", ctypes.c_double)]


PEAK_DTYPE = np.dtype([("prn", "<i4"), ("doppler_bin", "<i4"), ("code_phase", "<i4"),
                       ("detected", "<i4"), ("peak", "<f4"), ("second", "<f4"), ("mean", "<f4"),
                       ("ratio", "<f4"), ("doppler_hz", "<f8"), ("code_phase_frac", "<f8")])
assert PEAK_DTYPE.itemsize == ctypes.sizeof(gnss_peak) == 48


class gnss_request(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_void_p), ("fmt", ctypes.c_int32), ("n", ctypes.c_size_t),
                ("fs", ctypes.c_double), ("f_if", ctypes.c_double),
                ("prn_list", ctypes.POINTER(ctypes.c_int32)), ("n_prn", ctypes.c_int32),
                ("doppler_lo", ctypes.c_double), ("doppler_hi", ctypes.c_double),
                ("doppler_step", ctypes.c_double), ("T_coh_ms", ctypes.c_int32),
                ("N_noncoh", ctypes.c_int32), ("out_grid", ctypes.c_void_p),
                ("out_peaks", ctypes.c_void_p)]


class gnss_channel(ctypes.Structure):
    _fields_ = [("prn", ctypes.c_int32), ("carrier_hz", ctypes.c_double),
                ("carrier_phase", ctypes.c_double), ("code_phase", ctypes.c_double),
                ("code_rate", ctypes.c_double), ("spacing", ctypes.c_double)]


class gnss_track_request(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_void_p), ("fmt", ctypes.c_int32), ("n", ctypes.c_size_t),
                ("fs", ctypes.c_double), ("channels", ctypes.POINTER(gnss_channel)),
                ("n_channels", ctypes.c_int32), ("start", ctypes.c_int64),
                ("epoch_len", ctypes.c_int32), ("n_epochs", ctypes.c_int32),
                ("out", ctypes.c_void_p)]


class gnss_ticket_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("queued_s", ctypes.c_double), ("run_s", ctypes.c_double),
                ("total_s", ctypes.c_double)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgnss_acq.so is not built (run __graft_entry__.build() or "
                          "python paper_1309_0052_amd/build.py); there is no CPU fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    pi32 = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "gnss_acquire": [vp, i32, sz, dbl, dbl, pi32, i32, dbl, dbl, dbl, i32, i32, vp, vp],
        "gnss_ctx_create": [ctypes.POINTER(vp), ctypes.c_int, sz, ctypes.c_int],
        "gnss_ctx_destroy": [vp],
        "gnss_ctx_set": [vp, ctypes.c_char_p, dbl],
        "gnss_workspace_bytes": [ctypes.POINTER(gnss_request), ctypes.POINTER(sz)],
        "gnss_acquire_device": [vp, ctypes.POINTER(gnss_request), vp],
        "gnss_acquire_device_noalloc": [vp, ctypes.POINTER(gnss_request), vp],
        "gnss_gold_codes": [vp, pi32, i32, vp, vp],
        "gnss_code_replica": [vp, pi32, i32, dbl, sz, vp, vp],
        "gnss_nco_lut": [vp, vp, vp, vp],
        "gnss_wipe_fold": [vp, ctypes.POINTER(gnss_request), vp, vp],
        "gnss_box_fold": [vp, ctypes.POINTER(gnss_request), vp, vp],
        "gnss_fft2048": [vp, vp, vp, i32, i32, vp],
        "gnss_dft1023": [vp, vp, vp, i32, i32, vp],
        "gnss_peaks": [vp, vp, pi32, i32, i32, i32, i32, dbl, dbl, vp, vp],
        "gnss_stage_times": [vp, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64), i32, i32],
        "gnss_acquire_batch_device": [vp, ctypes.POINTER(gnss_request), i32, vp],
        "gnss_graph_create": [vp, ctypes.POINTER(gnss_request), i32, ctypes.POINTER(vp)],
        "gnss_graph_launch": [vp, vp],
        "gnss_graph_destroy": [vp],
        "gnss_autotune": [vp, ctypes.POINTER(gnss_request), i32, ctypes.c_char_p,
                          ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "gnss_submit": [vp, ctypes.POINTER(gnss_request), ctypes.POINTER(ctypes.c_uint64)],
        "gnss_poll": [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int),
                      ctypes.POINTER(gnss_ticket_info)],
        "gnss_wait": [vp, ctypes.c_uint64, dbl, ctypes.POINTER(gnss_ticket_info)],
        "gnss_track": [ctypes.POINTER(gnss_track_request)],
        "gnss_track_device": [vp, ctypes.POINTER(gnss_track_request), i32, vp],
        "gnss_strerror": [ctypes.c_int],
        "gnss_last_error": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.gnss_ctx_destroy.restype = None
    lib.gnss_graph_destroy.restype = None
    lib.gnss_strerror.restype = ctypes.c_char_p
    lib.gnss_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def library() -> ctypes.CDLL:
    return _lib


def _strerror(code: int) -> str:
    return _lib.gnss_strerror(int(code)).decode()


def last_error() -> str:
    return _lib.gnss_last_error().decode()


def _check(rc: int):
    if rc != GNSS_OK:
        raise GnssError(rc, last_error())


def n_doppler(lo: float, hi: float, step: float) -> int:
    return int(math.floor((hi - lo) / step + 1e-9)) + 1


def _prn_array(prns):
    a = np.ascontiguousarray(np.asarray(prns, np.int32))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _n_samples(samples: np.ndarray, fmt: int) -> int:
    if fmt == GNSS_CPLX_I8:
        return samples.size // 2
    if fmt == GNSS_REAL_I8:
        return samples.size
    return samples.size * 4


def gnss_acquire(samples: np.ndarray, fmt: int, fs: float, f_if: float, prns, doppler_lo: float,
                 doppler_hi: float, doppler_step: float, T_coh_ms: int, N_noncoh: int,
                 want_grid: bool = True, n: int | None = None):
    """Synchronous acquisition on host arrays.  Returns (grid or None, peaks),
    grid float32 [n_prn][n_dopp][N], peaks a PEAK_DTYPE array."""
    s = np.ascontiguousarray(samples)
    prn_a, prn_p = _prn_array(prns)
    n_samp = int(n if n is not None else _n_samples(s, fmt))
    # argument checks happen in the library before any output is sized here
    gnss_workspace_bytes(make_request(s.ctypes.data, fmt, n_samp, fs, f_if, prns, doppler_lo,
                                      doppler_hi, doppler_step, T_coh_ms, N_noncoh, None, 1))
    nd = n_doppler(doppler_lo, doppler_hi, doppler_step)
    N = int(fs) // 1000
    grid = np.empty((prn_a.size, nd, N), np.float32) if want_grid else None
    peaks = np.zeros(prn_a.size, PEAK_DTYPE)
    rc = _lib.gnss_acquire(s.ctypes.data_as(ctypes.c_void_p), int(fmt), n_samp, float(fs),
                           float(f_if),
                           prn_p, prn_a.size, float(doppler_lo), float(doppler_hi),
                           float(doppler_step), int(T_coh_ms), int(N_noncoh),
                           grid.ctypes.data_as(ctypes.c_void_p) if grid is not None else None,
                           peaks.ctypes.data_as(ctypes.c_void_p))
    _check(rc)
    return grid, peaks


def make_request(samples_ptr: int, fmt: int, n: int, fs: float, f_if: float, prns,
                 doppler_lo: float, doppler_hi: float, doppler_step: float, T_coh_ms: int,
                 N_noncoh: int, out_grid_ptr: int | None = None, out_peaks_ptr: int | None = None):
    """Builds a gnss_request; the PRN array is kept alive on the returned object."""
    prn_a, prn_p = _prn_array(prns)
    r = gnss_request()
    r.samples = samples_ptr
    r.fmt = int(fmt)
    r.n = int(n)
    r.fs = float(fs)
    r.f_if = float(f_if)
    r.prn_list = prn_p
    r.n_prn = prn_a.size
    r.doppler_lo = float(doppler_lo)
    r.doppler_hi = float(doppler_hi)
    r.doppler_step = float(doppler_step)
    r.T_coh_ms = int(T_coh_ms)
    r.N_noncoh = int(N_noncoh)
    r.out_grid = out_grid_ptr
    r.out_peaks = out_peaks_ptr
    r._prn_keepalive = prn_a
    return r


def make_track_request(samples_ptr: int, fmt: int, n: int, fs: float, channels, start: int,
                       epoch_len: int, n_epochs: int, out_ptr: int | None):
    """Builds a gnss_track_request.  channels: sequence of objects with prn,
    carrier_hz, carrier_phase, code_phase, code_rate, spacing (or tuples in
    that order); the channel array is kept alive on the returned object."""
    arr = (gnss_channel * len(channels))()
    for i, c in enumerate(channels):
        v = c if isinstance(c, (tuple, list)) else (c.prn, c.carrier_hz, c.carrier_phase, c.code_phase,
                                                     c.code_rate, c.spacing)
        arr[i] = gnss_channel(int(v[0]), float(v[1]), float(v[2]), float(v[3]), float(v[4]), float(v[5]))
    r = gnss_track_request()
    r.samples = samples_ptr
    r.fmt = int(fmt)
    r.n = int(n)
    r.fs = float(fs)
    r.channels = ctypes.cast(arr, ctypes.POINTER(gnss_channel))
    r.n_channels = len(channels)
    r.start = int(start)
    r.epoch_len = int(epoch_len)
    r.n_epochs = int(n_epochs)
    r.out = out_ptr
    r._ch_keepalive = arr
    return r


def gnss_track(samples: np.ndarray, fmt: int, fs: float, channels, start: int, epoch_len: int,
               n_epochs: int, n: int | None = None) -> np.ndarray:
    """Synchronous early/prompt/late correlators on a host record: int64
    [n_channels][n_epochs][3][2] (early, prompt, late; re, im)."""
    s = np.ascontiguousarray(samples)
    n_samp = int(n if n is not None else _n_samples(s, fmt))
    out = np.zeros((len(channels), max(int(n_epochs), 0), 3, 2), np.int64)
    r = make_track_request(s.ctypes.data, fmt, n_samp, fs, channels, start, epoch_len, n_epochs,
                           out.ctypes.data)
    _check(_lib.gnss_track(ctypes.byref(r)))
    return out


def gnss_workspace_bytes(req: gnss_request) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.gnss_workspace_bytes(ctypes.byref(req), ctypes.byref(out)))
    return out.value


def _stream_ptr(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Context:
    """gnss_ctx: one device, its stream, device-resident tables and workspace."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, precision: int = GNSS_FP32):
        h = ctypes.c_void_p()
        _check(_lib.gnss_ctx_create(ctypes.byref(h), int(device), int(hbm_budget_bytes),
                                    int(precision)))
        self.handle = h

    def close(self):
        if self.handle:
            _lib.gnss_ctx_destroy(self.handle)
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

    def set(self, key: str, value: float):
        _check(_lib.gnss_ctx_set(self.handle, key.encode(), float(value)))

    # -- full search on device buffers --------------------------------------
    def acquire_device(self, req: gnss_request, stream=None):
        _check(_lib.gnss_acquire_device(self.handle, ctypes.byref(req), _stream_ptr(stream)))

    def acquire_device_noalloc(self, req: gnss_request, stream=None):
        _check(_lib.gnss_acquire_device_noalloc(self.handle, ctypes.byref(req), _stream_ptr(stream)))

    def stage_times(self, reset: bool = False):
        """{stage name: (total ms, launches)} accumulated while "profile" is 1."""
        ms = (ctypes.c_double * GNSS_N_STAGES)()
        cnt = (ctypes.c_int64 * GNSS_N_STAGES)()
        _check(_lib.gnss_stage_times(self.handle, ms, cnt, GNSS_N_STAGES, 1 if reset else 0))
        return {STAGE_NAMES[i]: (ms[i], cnt[i]) for i in range(GNSS_N_STAGES)}

    def track_device(self, reqs, stream=None):
        """Tracking correlators of gnss_track_request(s) on device buffers."""
        if isinstance(reqs, gnss_track_request):
            reqs = [reqs]
        arr = (gnss_track_request * len(reqs))(*reqs)
        _check(_lib.gnss_track_device(self.handle, arr, len(reqs), _stream_ptr(stream)))

    # -- batches, graphs, autotuning ----------------------------------------
    def acquire_batch_device(self, reqs, stream=None):
        arr = _req_array(reqs)
        _check(_lib.gnss_acquire_batch_device(self.handle, arr, len(reqs), _stream_ptr(stream)))

    def graph(self, reqs):
        """Captures the batch `reqs` (device-buffer requests) into a HIP graph."""
        return Graph(self, reqs)

    def autotune(self, reqs, cache_path: str | None = None):
        """Returns the chosen (PRN tile, persistent schedule)."""
        arr = _req_array(reqs)
        tile, pers = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(_lib.gnss_autotune(self.handle, arr, len(reqs),
                                  cache_path.encode() if cache_path else None, ctypes.byref(tile),
                                  ctypes.byref(pers)))
        return tile.value, pers.value

    # -- serving --------------------------------------------------------------
    def submit(self, req: gnss_request) -> int:
        """Submits a host-buffer request; returns its ticket.  The request's
        output arrays must stay alive until the ticket is done."""
        t = ctypes.c_uint64(0)
        _check(_lib.gnss_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """(done, info or None)."""
        done = ctypes.c_int(0)
        info = gnss_ticket_info()
        _check(_lib.gnss_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(done),
                              ctypes.byref(info)))
        return bool(done.value), (info if done.value else None)

    def wait(self, ticket: int, timeout_s: float = -1.0) -> gnss_ticket_info:
        info = gnss_ticket_info()
        _check(_lib.gnss_wait(self.handle, ctypes.c_uint64(ticket), float(timeout_s),
                              ctypes.byref(info)))
        return info

    # -- stage entry points (device pointers as ints) ------------------------
    def gold_codes(self, prns, d_codes: int, stream=None):
        a, p = _prn_array(prns)
        _check(_lib.gnss_gold_codes(self.handle, p, a.size, d_codes, _stream_ptr(stream)))

    def code_replica(self, prns, fs: float, n: int, d_out: int, stream=None):
        a, p = _prn_array(prns)
        _check(_lib.gnss_code_replica(self.handle, p, a.size, float(fs), int(n), d_out,
                                      _stream_ptr(stream)))

    def nco_lut(self, d_cos: int, d_sin: int, stream=None):
        _check(_lib.gnss_nco_lut(self.handle, d_cos, d_sin, _stream_ptr(stream)))

    def wipe_fold(self, req: gnss_request, d_out: int, stream=None):
        _check(_lib.gnss_wipe_fold(self.handle, ctypes.byref(req), d_out, _stream_ptr(stream)))

    def box_fold(self, req: gnss_request, d_out: int, stream=None):
        _check(_lib.gnss_box_fold(self.handle, ctypes.byref(req), d_out, _stream_ptr(stream)))

    def fft2048(self, d_in: int, d_out: int, batch: int, inverse: bool, stream=None):
        _check(_lib.gnss_fft2048(self.handle, d_in, d_out, int(batch), 1 if inverse else 0,
                                 _stream_ptr(stream)))

    def dft1023(self, d_in: int, d_out: int, batch: int, inverse: bool, stream=None):
        _check(_lib.gnss_dft1023(self.handle, d_in, d_out, int(batch), 1 if inverse else 0,
                                 _stream_ptr(stream)))

    def peaks(self, d_grid: int, prns, n_dopp: int, N: int, spc: int, doppler_lo: float,
              doppler_step: float, d_peaks: int, stream=None):
        a, p = _prn_array(prns)
        _check(_lib.gnss_peaks(self.handle, d_grid, p, a.size, int(n_dopp), int(N), int(spc),
                               float(doppler_lo), float(doppler_step), d_peaks,
                               _stream_ptr(stream)))


def _req_array(reqs):
    arr = (gnss_request * len(reqs))()
    for i, r in enumerate(reqs):
        arr[i] = r
    return arr


class Graph:
    """gnss_graph: a captured batch replayed with launch()."""

    def __init__(self, ctx: Context, reqs):
        self._reqs = list(reqs)  # keep PRN arrays alive
        arr = _req_array(self._reqs)
        h = ctypes.c_void_p()
        _check(_lib.gnss_graph_create(ctx.handle, arr, len(self._reqs), ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(_lib.gnss_graph_launch(self.handle, _stream_ptr(stream)))

    def close(self):
        if self.handle:
            _lib.gnss_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

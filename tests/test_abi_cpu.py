"""C ABI checks that need no GPU: the library loads, exports every function
the public header declares, and rejects bad arguments before touching a
device."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT

G = pytest.importorskip("paper_1309_0052_amd")


def _header_functions():
    text = open(os.path.join(ROOT, "include", "gnss_acq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gnss_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported():
    names = _header_functions()
    assert len(names) >= 14
    lib = G.library()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(G.EXPORTED)


def test_header_constants_match_binding():
    text = open(os.path.join(ROOT, "include", "gnss_acq.h")).read()
    consts = re.findall(r"^#define (GNSS_[A-Z0-9_]+) \(?(-?\d+)\)?", text, flags=re.M)
    assert len(consts) >= 16
    for name, val in consts:
        assert getattr(G, name) == int(val), name


def test_peak_struct_layout():
    assert ctypes.sizeof(G.gnss_peak) == 48
    assert G.gnss_peak.doppler_hz.offset == 32


def test_strerror_codes():
    assert G.library().gnss_strerror(0) == b"ok"
    assert G.library().gnss_strerror(-5) == b"unsupported configuration"


STRONG = dict(fmt=G.GNSS_REAL_I8, fs=4092000.0, f_if=1023000.0, prns=[1, 2], lo=-500.0,
              hi=500.0, step=500.0, T=1, Nn=10)


def _acquire(x, **kw):
    a = dict(STRONG)
    a.update(kw)
    return G.gnss_acquire(x, a["fmt"], a["fs"], a["f_if"], a["prns"], a["lo"], a["hi"],
                          a["step"], a["T"], a["Nn"])


@pytest.mark.parametrize("kw,code", [
    (dict(fs=4092500.0), G.GNSS_EINVAL),          # not a multiple of 1 kHz
    (dict(fs=4092000.5), G.GNSS_EINVAL),          # not an integer
    (dict(fs=-4092000.0), G.GNSS_EINVAL),
    (dict(fs=16385000.0), G.GNSS_ENOTSUP),        # not k * 1.023 MHz and N > 16384
    (dict(fs=17391000.0), G.GNSS_ENOTSUP),        # 17 samples per chip: N > 16384
    (dict(fs=5000000.0), G.GNSS_EINVAL),          # a general rate: 50000 samples needed
    (dict(prns=[0]), G.GNSS_EINVAL),
    (dict(prns=[38]), G.GNSS_EINVAL),
    (dict(prns=list(range(1, 38)) * 2), G.GNSS_EINVAL),  # 74 > 64
    (dict(step=0.0), G.GNSS_EINVAL),
    (dict(step=-1.0), G.GNSS_EINVAL),
    (dict(lo=100.0, hi=-100.0), G.GNSS_EINVAL),
    (dict(T=0), G.GNSS_EINVAL),
    (dict(T=65), G.GNSS_EINVAL),
    (dict(Nn=0), G.GNSS_EINVAL),
    (dict(Nn=11), G.GNSS_EINVAL),                 # needs more samples than given
    (dict(fmt=7), G.GNSS_EINVAL),
    (dict(f_if=2046000.0), G.GNSS_EINVAL),        # real samples need f_if < fs/2
    (dict(f_if=-1.0), G.GNSS_EINVAL),
    (dict(lo=float("nan")), G.GNSS_EINVAL),
])
def test_argument_validation(kw, code):
    x = np.zeros(40920, np.int8)
    with pytest.raises(G.GnssError) as ei:
        _acquire(x, **kw)
    assert ei.value.code == code
    assert G.last_error()


def test_null_pointers_rejected():
    lib = G.library()
    peaks = (G.gnss_peak * 1)()
    prn = (ctypes.c_int32 * 1)(1)
    rc = lib.gnss_acquire(None, 0, 40920, 4092000.0, 0.0, prn, 1, 0.0, 0.0, 1.0, 1, 1, None,
                          ctypes.cast(peaks, ctypes.c_void_p))
    assert rc == G.GNSS_EINVAL
    x = np.zeros(40920, np.int8)
    rc = lib.gnss_acquire(x.ctypes.data_as(ctypes.c_void_p), 0, 40920, 4092000.0, 0.0, prn, 1,
                          0.0, 0.0, 1.0, 1, 1, None, None)
    assert rc == G.GNSS_EINVAL
    rc = lib.gnss_acquire(x.ctypes.data_as(ctypes.c_void_p), 0, 40920, 4092000.0, 0.0, None, 1,
                          0.0, 0.0, 1.0, 1, 1, None, ctypes.cast(peaks, ctypes.c_void_p))
    assert rc == G.GNSS_EINVAL
    assert lib.gnss_ctx_set(None, b"threshold", 2.0) == G.GNSS_EINVAL
    assert lib.gnss_ctx_create(None, 0, 0, 0) == G.GNSS_EINVAL


def test_workspace_bytes_is_host_only():
    x = np.zeros(2 * 1636800, np.int8)
    req = G.make_request(x.ctypes.data, G.GNSS_CPLX_I8, 1636800, 16368000.0, 0.0,
                         list(range(1, 33)), -7500.0, 7500.0, 125.0, 4, 25, None, 1)
    b = G.gnss_workspace_bytes(req)
    # polyphase ints (396 MB), spectra (793 MB), grid (253.5 MB), peak scratch, samples
    assert 1.4e9 < b < 1.5e9


def test_doppler_bin_count():
    assert G.n_doppler(-5000, 5000, 500) == 21
    assert G.n_doppler(-7500, 7500, 125) == 121
    assert G.n_doppler(0, 0, 1) == 1


def _chan(**kw):
    c = dict(prn=5, carrier_hz=1000.0, carrier_phase=0.25, code_phase=100.5, code_rate=1023000.0,
             spacing=0.5)
    c.update(kw)
    return (c["prn"], c["carrier_hz"], c["carrier_phase"], c["code_phase"], c["code_rate"], c["spacing"])


@pytest.mark.parametrize("ch,kw", [
    (_chan(prn=0), {}), (_chan(prn=38), {}), (_chan(carrier_phase=1.0), {}),
    (_chan(carrier_phase=-0.1), {}), (_chan(code_phase=1023.0), {}), (_chan(code_phase=-1.0), {}),
    (_chan(code_rate=0.0), {}), (_chan(code_rate=float("nan")), {}), (_chan(spacing=0.0), {}),
    (_chan(spacing=1.5), {}), (_chan(carrier_hz=float("inf")), {}),
    (_chan(), {"fmt": 7}), (_chan(), {"epoch_len": 0}), (_chan(), {"n_epochs": 0}),
    (_chan(), {"start": -1}), (_chan(), {"n_epochs": 3}),  # 3 x 2046 > 4092 samples
    (_chan(), {"fs": 0.0}),
])
def test_track_argument_validation(ch, kw):
    x = np.zeros(2 * 4092, np.int8)
    args = dict(fmt=G.GNSS_CPLX_I8, fs=2046000.0, start=0, epoch_len=2046, n_epochs=2)
    args.update(kw)
    with pytest.raises(G.GnssError) as ei:
        G.gnss_track(x, args["fmt"], args["fs"], [ch], args["start"], args["epoch_len"],
                     args["n_epochs"], n=4092)
    assert ei.value.code == G.GNSS_EINVAL


def test_track_null_and_count_checks():
    r = G.make_track_request(None, G.GNSS_CPLX_I8, 10, 1023000.0, [_chan()], 0, 5, 1, None)
    assert G.library().gnss_track(ctypes.byref(r)) == G.GNSS_EINVAL
    x = np.zeros(20, np.int8)
    r = G.make_track_request(x.ctypes.data, G.GNSS_CPLX_I8, 10, 1023000.0, [_chan()], 0, 5, 1, None)
    assert G.library().gnss_track(ctypes.byref(r)) == G.GNSS_EINVAL  # out is null
    assert G.library().gnss_track(None) == G.GNSS_EINVAL
    assert G.library().gnss_track_device(None, None, 0, None) == G.GNSS_EINVAL

"""GPU tests of the tracking correlators (early / prompt / late, Fig. 3)
through the C ABI against the oracle.  Everything is exact integer
arithmetic on both sides, so the comparison is bit for bit."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")

F_L1 = 1575.42e6


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = G.Context(0)
    yield c
    c.close()


def _channels(rng, n_ch, prns, dopp_max=4000.0, spacing=0.5, f_if=0.0):
    out = []
    for i in range(n_ch):
        f_d = float(rng.uniform(-dopp_max, dopp_max))
        out.append(O.Channel(prn=int(prns[i % len(prns)]), carrier_hz=f_if + f_d,
                             carrier_phase=float(rng.uniform(0.0, 1.0)),
                             code_phase=float(rng.uniform(0.0, 1023.0)),
                             code_rate=1023000.0 * (1.0 + f_d / F_L1), spacing=spacing))
    return out


def _snapshot(seed, fmt, fs, f_if, ms, prns, cn0=48.0):
    rng = np.random.default_rng(seed)
    N = int(round(fs / 1000))
    pl = [synth.Planted(prn=p, code_phase=int(rng.integers(0, N)), doppler_hz=float(rng.uniform(-3000, 3000)),
                        cn0_dbhz=cn0, carrier_phase=float(rng.uniform(0, 2 * np.pi))) for p in prns]
    return synth.make_snapshot(seed, fmt, int(fs), f_if, ms, pl, O.ca_code)


CASES = [
    # name, fmt, fs, f_if, ms, n_ch, start, epoch_len, n_epochs, spacing
    ("cplx_16M_1ms", O.CPLX_I8, 16368000, 0.0, 5.0, 5, 0, 16368, 4, 0.5),
    ("real_4M_ragged", O.REAL_I8, 4092000, 1023000.0, 6.0, 9, 1234, 3001, 5, 0.1),
    ("packed_8M", O.REAL_2BIT_PACKED, 8184000, 2046000.0, 4.0, 3, 17, 8184, 3, 1.0),
    ("cplx_5M_non_integer_spc", O.CPLX_I8, 5000000, 0.0, 4.0, 4, 5, 4999, 3, 0.5),
    ("cplx_2M_one_channel", O.CPLX_I8, 2046000, 0.0, 3.0, 1, 0, 700, 8, 0.25),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_track_matches_oracle(ctx, case):
    name, fmt, fs, f_if, ms, n_ch, start, elen, n_ep, spacing = case
    rng = np.random.default_rng(sum(name.encode()))
    snap = _snapshot(sum(name.encode()) % 997, fmt, fs, f_if, ms, [3, 11, 19])
    chans = _channels(rng, n_ch, [3, 11, 19, 24, 1, 37], spacing=spacing, f_if=f_if)
    # exercise the code-period ends: late wraps below chip 0, early above chip 1022
    chans[0].code_phase = 0.3 * spacing
    if n_ch > 1:
        chans[1].code_phase = 1023.0 - 0.3 * spacing
    log("track %s: fs=%d n_ch=%d start=%d epoch=%d x %d" % (name, fs, n_ch, start, elen, n_ep))
    ref = O.track(snap.samples, fmt, fs, chans, start, elen, n_ep)
    d_x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
    d_o = torch.full((n_ch * n_ep * 6,), -7, dtype=torch.int64, device="cuda")
    req = G.make_track_request(d_x.data_ptr(), fmt, snap.n, fs, chans, start, elen, n_ep, d_o.data_ptr())
    ctx.track_device(req, torch.cuda.current_stream())
    torch.cuda.synchronize()
    got = d_o.cpu().numpy().reshape(n_ch, n_ep, 3, 2)
    assert np.array_equal(got, ref)
    host = G.gnss_track(snap.samples, fmt, fs, chans, start, elen, n_ep, n=snap.n)
    assert np.array_equal(host, ref)


def test_track_long_epoch_full_scale_samples(ctx):
    # an epoch of 300 000 samples at full int8 scale: per-thread partial sums are
    # flushed to int64 every 1024 samples; the aligned channel's prompt sum,
    # 127 * 4096 * 300 000, is far above 2^31
    fs = 2046000
    n = 300000
    rng = np.random.default_rng(7)
    rep = O.code_replica(9, fs, n).astype(np.int64)
    x = np.zeros(2 * n, np.int8)
    x[0::2] = (127 * rep).astype(np.int8)
    x[1::2] = rng.choice(np.array([-127, 127], np.int8), size=n)
    chans = _channels(rng, 6, [2, 9, 30], dopp_max=500.0)
    chans[2] = O.Channel(prn=9, carrier_hz=0.0, carrier_phase=0.0, code_phase=0.0, code_rate=1023000.0,
                         spacing=0.5)
    ref = O.track(x, O.CPLX_I8, fs, chans, 0, n, 1)
    assert ref[2, 0, 1, 0] == 127 * 4096 * n
    got = G.gnss_track(x, O.CPLX_I8, fs, chans, 0, n, 1)
    assert np.array_equal(got, ref)


def test_track_batch_equals_alone(ctx):
    rng = np.random.default_rng(12)
    items = []
    for i, (fmt, fs, f_if) in enumerate([(O.CPLX_I8, 16368000, 0.0), (O.REAL_I8, 4092000, 1023000.0),
                                         (O.REAL_2BIT_PACKED, 8184000, 2046000.0), (O.CPLX_I8, 2046000, 0.0)]):
        snap = _snapshot(40 + i, fmt, fs, f_if, 3.0, [5, 6])
        n_ch = int(rng.integers(1, 13))
        chans = _channels(rng, n_ch, list(range(1, 33)), f_if=f_if)
        elen = fs // 1000
        items.append((snap, chans, elen, 3))
    bufs, reqs = [], []
    for snap, chans, elen, n_ep in items:
        d_x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
        d_o = torch.zeros(len(chans) * n_ep * 6, dtype=torch.int64, device="cuda")
        bufs.append((d_x, d_o))
        reqs.append(G.make_track_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, chans, 0, elen,
                                         n_ep, d_o.data_ptr()))
    ctx.track_device(reqs, torch.cuda.current_stream())
    torch.cuda.synchronize()
    for (snap, chans, elen, n_ep), (d_x, d_o) in zip(items, bufs):
        ref = O.track(snap.samples, snap.fmt, snap.fs_hz, chans, 0, elen, n_ep)
        assert np.array_equal(d_o.cpu().numpy().reshape(len(chans), n_ep, 3, 2), ref)


def test_track_on_planted_satellite_prompt_dominates(ctx):
    # a channel on a planted satellite's true code phase and Doppler: prompt power
    # well above early/late at one chip spacing and above a wrong PRN
    fs = 4092000
    N = fs // 1000
    pl = [synth.Planted(prn=14, code_phase=1500, doppler_hz=2500.0, cn0_dbhz=50.0)]
    snap = synth.make_snapshot(3, O.CPLX_I8, fs, 0.0, 10.0, pl, O.ca_code)
    chip0 = (1023.0 - 1500 / 4.0) % 1023.0
    good = O.Channel(14, 2500.0, 0.0, chip0, 1023000.0 * (1 + 2500.0 / F_L1), 1.0)
    wrong = O.Channel(15, 2500.0, 0.0, chip0, 1023000.0, 1.0)
    out = G.gnss_track(snap.samples, O.CPLX_I8, fs, [good, wrong], 0, N, 10)
    pw = (out.astype(np.float64) ** 2).sum(axis=3).sum(axis=1)  # [ch][E,P,L]
    assert pw[0, 1] > 3 * pw[0, 0] and pw[0, 1] > 3 * pw[0, 2]
    assert pw[0, 1] > 20 * pw[1, 1]

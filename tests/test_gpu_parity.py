"""GPU parity: every stage of the HIP path and the whole search, through the
C ABI, against the oracle on the same seeded inputs.

Bit-exact: C/A codes, code replicas, carrier LUT, wiped+folded blocks.
FP32 power grid: mixed tolerance 1e-4 (see parity.py); detections identical.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from parity import assert_grid_close, compare_detections, compare_refinement, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = G.Context(0)
    yield c
    c.close()


def _dev(a: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _stream():
    return torch.cuda.current_stream()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# ---------------------------------------------------------------------------
# tables: codes, replicas, LUT (bit-exact)
# ---------------------------------------------------------------------------

def test_gold_codes_bit_exact(ctx):
    prns = list(range(1, 38))
    d = torch.zeros(len(prns) * 1023, dtype=torch.uint8, device="cuda")
    log("gold codes: 37 PRNs")
    ctx.gold_codes(prns, d.data_ptr(), _stream())
    got = _host(d).reshape(len(prns), 1023)
    for i, prn in enumerate(prns):
        assert np.array_equal(got[i], O.ca_code(prn)), prn


@pytest.mark.parametrize("fs", [1023000, 2046000, 4092000, 16368000, 5000000, 2500000, 7777000])
def test_code_replica_bit_exact(ctx, fs):
    prns = [1, 19, 37, 19]
    n = 2 * (fs // 1000) + 17
    d = torch.zeros(len(prns) * n, dtype=torch.int8, device="cuda")
    log("code replica fs=%d n=%d" % (fs, n))
    ctx.code_replica(prns, fs, n, d.data_ptr(), _stream())
    got = _host(d).reshape(len(prns), n)
    for i, prn in enumerate(prns):
        assert np.array_equal(got[i], O.code_replica(prn, fs, n)), (fs, prn)


def test_nco_lut_bit_exact(ctx):
    dc = torch.zeros(1024, dtype=torch.int16, device="cuda")
    ds = torch.zeros(1024, dtype=torch.int16, device="cuda")
    log("nco lut")
    ctx.nco_lut(dc.data_ptr(), ds.data_ptr(), _stream())
    c, s = O.lut()
    assert np.array_equal(_host(dc), c) and np.array_equal(_host(ds), s)


# ---------------------------------------------------------------------------
# carrier NCO + mixing + coherent fold (bit-exact int32)
# ---------------------------------------------------------------------------

WIPE_CASES = [
    # fmt, fs, f_if, lo, hi, step, Tc, Nnc, extra samples
    (O.REAL_I8, 4092000, 1023000.0, -5000.0, 5000.0, 500.0, 1, 10, 0),
    (O.CPLX_I8, 16368000, 0.0, -7500.0, -7000.0, 125.0, 4, 3, 5),
    (O.REAL_2BIT_PACKED, 2046000, 511500.0, -3000.0, 3000.0, 1500.0, 3, 2, 12),
    (O.CPLX_I8, 1023000, 250000.0, -480000.0, 480000.0, 240000.0, 16, 2, 0),
    (O.CPLX_I8, 8184000, -1234.5, 333.25, 999.75, 333.25, 2, 2, 1),
]


def _random_record(rng, fmt, n):
    if fmt == O.CPLX_I8:
        return rng.integers(-127, 128, 2 * n).astype(np.int8)
    q = rng.choice(np.array([-3, -1, 1, 3], np.int8), size=n)
    return synth.pack_2bit(q) if fmt == O.REAL_2BIT_PACKED else q


@pytest.mark.parametrize("case", WIPE_CASES)
def test_wipe_fold_bit_exact(ctx, case):
    fmt, fs, f_if, lo, hi, step, Tc, Nnc, extra = case
    rng = np.random.default_rng(fs % 9973 + Tc)
    N = fs // 1000
    n = Tc * Nnc * N + extra
    x = _random_record(rng, fmt, n)
    nd = O.n_doppler(lo, hi, step)
    d_x = _dev(x)
    out = torch.zeros(nd * Nnc * N * 2, dtype=torch.int32, device="cuda")
    req = G.make_request(d_x.data_ptr(), fmt, n, fs, f_if, [1], lo, hi, step, Tc, Nnc)
    log("wipe_fold fmt=%d fs=%d bins=%d Tc=%d Nnc=%d" % (fmt, fs, nd, Tc, Nnc))
    ctx.wipe_fold(req, out.data_ptr(), _stream())
    got = _host(out).reshape(nd, Nnc, N, 2).astype(np.int64)
    ref = O.wipe_fold(x, fmt, fs, f_if, lo, step, nd, Tc, Nnc)
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------------------
# the search's own first stage (k_box: NCO wipe-off, fold, one-chip boxcar,
# polyphase split), bit-exact against the oracle's folded blocks with the
# boxcar and the split written out here from their definition:
#   F[n] = sum_{t<spc} f[(n + t - d) mod N],  g_s[m] = F[spc m + s] (m < 1023), g_s[1023] = 0
# (d = the code-Doppler shift of the (bin, block) when that option is on)
# ---------------------------------------------------------------------------

def _box_reference(folded_k: np.ndarray, spc: int, shifts=None) -> np.ndarray:
    """folded_k: int64 [Nnc][N][2] of one Doppler bin -> int64 [Nnc][spc][1024][2]."""
    Nnc, N, _ = folded_k.shape
    out = np.zeros((Nnc, spc, 1024, 2), np.int64)
    for b in range(Nnc):
        f = np.roll(folded_k[b], shifts[b], axis=0) if shifts is not None else folded_k[b]
        F = np.zeros_like(f)
        for t in range(spc):
            F += np.roll(f, -t, axis=0)
        out[b, :, :1023, :] = F.reshape(1023, spc, 2).transpose(1, 0, 2)
    return out


BOX_CASES = [
    # name, fmt, fs, f_if, lo, hi, step, Tc, Nnc, extra, code_doppler
    ("spc1_cplx", O.CPLX_I8, 1023000, 250000.0, -4000.0, 4000.0, 2000.0, 3, 3, 0, False),
    # N = 1023 real 2-bit: the blocks start at sample offsets 0, 3, 2, 1 of a byte
    ("spc1_packed_subbyte", O.REAL_2BIT_PACKED, 1023000, 255750.0, -1000.0, 1000.0, 500.0, 1, 4, 3, False),
    ("spc2_packed_tc3", O.REAL_2BIT_PACKED, 2046000, 511500.0, -3000.0, 3000.0, 1500.0, 3, 2, 12, False),
    ("spc4_real", O.REAL_I8, 4092000, 1023000.0, -5000.0, 5000.0, 2500.0, 1, 5, 7, False),
    ("spc8_cplx", O.CPLX_I8, 8184000, -1234.5, 333.25, 999.75, 333.25, 2, 2, 1, False),
    ("spc16_cplx", O.CPLX_I8, 16368000, 0.0, -7500.0, 7500.0, 7500.0, 4, 2, 5, False),
    ("spc16_cplx_tc64", O.CPLX_I8, 16368000, 0.0, -500.0, 500.0, 500.0, 64, 1, 0, False),
    ("spc2_cplx_code_doppler", O.CPLX_I8, 2046000, 0.0, -40000.0, 40000.0, 20000.0, 16, 5, 0, True),
    ("spc1_packed_code_doppler", O.REAL_2BIT_PACKED, 1023000, 255750.0, -45000.0, 45000.0, 15000.0, 10, 4, 2,
     True),
]


def _run_box(ctx, x, fmt, n, fs, f_if, lo, hi, step, Tc, Nnc, code_doppler):
    N, spc = fs // 1000, fs // 1023000
    nd = O.n_doppler(lo, hi, step)
    d_x = _dev(x)
    out = torch.zeros(nd * Nnc * spc * 1024 * 2, dtype=torch.int32, device="cuda")
    req = G.make_request(d_x.data_ptr(), fmt, n, fs, f_if, [1], lo, hi, step, Tc, Nnc)
    ctx.set("code_doppler", 1 if code_doppler else 0)
    try:
        ctx.box_fold(req, out.data_ptr(), _stream())
        got = _host(out).reshape(nd, Nnc, spc, 1024, 2)
    finally:
        ctx.set("code_doppler", 0)
    return got


@pytest.mark.parametrize("case", BOX_CASES, ids=[c[0] for c in BOX_CASES])
def test_box_fold_bit_exact(ctx, case):
    name, fmt, fs, f_if, lo, hi, step, Tc, Nnc, extra, code_doppler = case
    rng = np.random.default_rng(sum(name.encode()))
    N, spc = fs // 1000, fs // 1023000
    n = Tc * Nnc * N + extra
    x = _random_record(rng, fmt, n)
    if name.endswith("tc64"):
        # a full-scale constant: at the 0 Hz bin the 64 ms fold and the 16-sample
        # boxcar reach 16 * 64 * 127 * 4096 = 2^29 - 2^22, the largest value k_box
        # meets for these formats short of a 45-degree carrier
        x = np.full(2 * n, 127, np.int8)
    nd = O.n_doppler(lo, hi, step)
    log("box_fold %s: fmt=%d fs=%d bins=%d Tc=%d Nnc=%d code_doppler=%s" % (name, fmt, fs, nd, Tc, Nnc,
                                                                           code_doppler))
    got = _run_box(ctx, x, fmt, n, fs, f_if, lo, hi, step, Tc, Nnc, code_doppler)
    folded = O.wipe_fold(x, fmt, fs, f_if, lo, step, nd, Tc, Nnc)
    for k in range(nd):
        shifts = None
        if code_doppler:
            shifts = [O.code_shift(b, Tc, N, O.bin_freq(lo, step, k)) % N for b in range(Nnc)]
        ref = _box_reference(folded[k], spc, shifts)
        assert np.abs(ref).max() < 2 ** 31
        assert np.array_equal(got[k].astype(np.int64), ref), (name, k)
    if code_doppler:
        assert any(O.code_shift(b, Tc, N, O.bin_freq(lo, step, 0)) % N for b in range(Nnc))
    if name.endswith("tc64"):
        assert np.abs(got).max() == 16 * 64 * 127 * 4096


@pytest.mark.timeout(600)
def test_box_fold_weak_workload_bit_exact(ctx):
    """The benchmarked weak-signal workload at full size: every polyphase
    vector k_box writes for 121 bins x 25 blocks x 16 phases."""
    snap, srch = synth.weak_complex_int8(O.ca_code, seed=2)
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    fs, Tc, Nnc = snap.fs_hz, srch.T_coh, srch.N_noncoh
    log("box_fold weak workload: 121 bins x 25 blocks x 16 phases")
    got = _run_box(ctx, snap.samples, snap.fmt, snap.n, fs, snap.f_if_hz, srch.lo, srch.hi, srch.step, Tc, Nnc,
                   False)
    folded = O.wipe_fold(snap.samples, snap.fmt, fs, snap.f_if_hz, srch.lo, srch.step, nd, Tc, Nnc)
    for k in range(nd):
        assert np.array_equal(got[k].astype(np.int64), _box_reference(folded[k], 16)), k


# ---------------------------------------------------------------------------
# 2048-point FFT against numpy FP64
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("inverse", [False, True])
def test_fft2048_matches_numpy(ctx, inverse):
    rng = np.random.default_rng(11)
    batch = 37
    x = (rng.standard_normal((batch, 2048)) + 1j * rng.standard_normal((batch, 2048))).astype(np.complex64)
    d_in = _dev(x.view(np.float32))
    d_out = torch.zeros_like(d_in)
    log("fft2048 inverse=%s batch=%d" % (inverse, batch))
    ctx.fft2048(d_in.data_ptr(), d_out.data_ptr(), batch, inverse, _stream())
    got = _host(d_out).view(np.complex64).reshape(batch, 2048).astype(np.complex128)
    xr = x.astype(np.complex128)
    ref = np.fft.ifft(xr, axis=1) * 2048 if inverse else np.fft.fft(xr, axis=1)
    # FP32 FFT: error per output ~ eps * O(log2 N) * rms of the transform
    rms = np.sqrt(np.mean(np.abs(ref) ** 2, axis=1, keepdims=True))
    err = np.abs(got - ref) / rms
    assert err.max() < 1e-5, err.max()


def test_fft2048_round_trip_and_impulses(ctx):
    x = np.zeros((4, 2048), np.complex64)
    x[0, 0] = 1.0
    x[1, 1] = 1.0
    x[2, 1023] = 1.0 - 2.0j
    x[3, :] = 1.0
    d_in = _dev(x.view(np.float32))
    d_mid = torch.zeros_like(d_in)
    d_out = torch.zeros_like(d_in)
    ctx.fft2048(d_in.data_ptr(), d_mid.data_ptr(), 4, False, _stream())
    ctx.fft2048(d_mid.data_ptr(), d_out.data_ptr(), 4, True, _stream())
    mid = _host(d_mid).view(np.complex64).reshape(4, 2048)
    out = _host(d_out).view(np.complex64).reshape(4, 2048) / 2048.0
    assert np.allclose(mid[0], 1.0, atol=1e-6)
    k = np.arange(2048)
    assert np.allclose(mid[1], np.exp(-2j * np.pi * k / 2048), atol=2e-6)
    assert abs(mid[3, 0] - 2048.0) < 1e-3 and np.abs(mid[3, 1:]).max() < 1e-3
    assert np.allclose(out, x, atol=2e-6)


# ---------------------------------------------------------------------------
# whole search vs the direct-correlation oracle (small, ragged)
# ---------------------------------------------------------------------------

def _planted_snapshot(seed, fmt, fs, f_if, ms, prns_planted, cn0, dopplers, noise=True):
    rng = np.random.default_rng(seed)
    N = fs // 1000
    planted = [synth.Planted(prn=p, code_phase=int(rng.integers(0, N)), doppler_hz=d, cn0_dbhz=cn0,
                             carrier_phase=float(rng.uniform(0, 2 * np.pi)))
               for p, d in zip(prns_planted, dopplers)]
    return synth.make_snapshot(seed, fmt, fs, f_if, ms, planted, O.ca_code, noise=noise)


SEARCH_CASES = [
    # name, fmt, fs, f_if, Tc, Nnc, prns searched, planted, lo, hi, step, cn0
    ("spc1_cplx", O.CPLX_I8, 1023000, 0.0, 1, 2, [3, 9], [9], -1000.0, 1000.0, 1000.0, 50.0),
    # N = 1023: the 2-bit blocks start at sample offsets 0, 3, 2, 1 within a byte
    ("spc1_packed_subbyte", O.REAL_2BIT_PACKED, 1023000, 255750.0, 1, 4, [2, 7, 11], [7], -1000.0, 1000.0,
     500.0, 54.0),
    ("spc2_packed_ragged", O.REAL_2BIT_PACKED, 2046000, 511500.0, 2, 3, [1, 5, 9, 13, 17],
     [5, 13], -1500.0, 1500.0, 500.0, 48.0),
    ("spc4_real", O.REAL_I8, 4092000, 1023000.0, 1, 4, [2, 4, 6, 8, 10, 12], [4, 10], -1000.0,
     1000.0, 500.0, 46.0),
    ("spc8_cplx_dup", O.CPLX_I8, 8184000, 0.0, 1, 2, [37, 7, 7], [7], -500.0, 500.0, 500.0, 48.0),
    ("spc16_cplx", O.CPLX_I8, 16368000, 0.0, 2, 1, [11, 31], [31], -250.0, 0.0, 250.0, 47.0),
    # one Doppler bin (lo = hi: no interior bin for the Doppler parabola)
    ("spc2_one_bin", O.CPLX_I8, 2046000, 0.0, 1, 3, [6, 19], [19], 250.0, 250.0, 500.0, 50.0),
    # the longest PRN list, 64 entries: PRNs 1-37 then 1-27 again
    ("spc4_64_prns", O.REAL_I8, 4092000, 1023000.0, 1, 1, list(range(1, 38)) + list(range(1, 28)), [5],
     -500.0, 500.0, 500.0, 50.0),
]


@pytest.mark.parametrize("case", SEARCH_CASES, ids=[c[0] for c in SEARCH_CASES])
def test_search_matches_direct_oracle(ctx, case):
    name, fmt, fs, f_if, Tc, Nnc, prns, planted, lo, hi, step, cn0 = case
    nd = O.n_doppler(lo, hi, step)
    dopp = [lo + step * (nd // 2) + 0.3 * step for _ in planted]
    snap = _planted_snapshot(sum(name.encode()) % 1000, fmt, fs, f_if, Tc * Nnc + 0.5, planted, cn0, dopp)
    log("search %s: fs=%d prns=%s bins=%d Tc=%d Nnc=%d" % (name, fs, prns, nd, Tc, Nnc))
    grid, peaks = G.gnss_acquire(snap.samples, fmt, fs, f_if, prns, lo, hi, step, Tc, Nnc, n=snap.n)
    P = O.grid_direct(snap.samples, fmt, fs, f_if, prns, lo, step, nd, Tc, Nnc)
    worst = assert_grid_close(grid, P)
    spc = fs // 1023000
    ref = O.peaks(P, prns, spc, 2.5, lo, step)
    exempt = compare_detections(peaks, ref, P)
    checked = compare_refinement(peaks, ref, P, grid, lo, step)
    log("  max err %.2e, exemptions %d, refinements checked %d" % (worst, exempt, checked))
    for p in snap.planted:
        i = prns.index(p.prn)
        assert peaks[i]["detected"] and peaks[i]["code_phase"] == p.code_phase


def test_noiseless_code_closed_form_on_gpu(ctx):
    # x = c_p[(n - d) mod N] at 0 Hz: P[d] = Nnc (Tc N)^2, and every cell is the
    # closed form Nnc (Tc A(d - tau))^2 (oracle pin), here within FP32 tolerance.
    fs, Tc, Nnc, prn, d = 4092000, 2, 3, 21, 1001
    N = fs // 1000
    rep = O.code_replica(prn, fs, N).astype(np.int64)
    sig = np.tile(np.roll(rep, d), Tc * Nnc).astype(np.int8)
    x = np.zeros(2 * sig.size, np.int8)
    x[0::2] = sig
    grid, peaks = G.gnss_acquire(x, O.CPLX_I8, fs, 0.0, [prn, 5], 0.0, 0.0, 1.0, Tc, Nnc)
    assert peaks[0]["code_phase"] == d and peaks[0]["detected"]
    assert abs(grid[0, 0, d] / (Nnc * float(Tc * N) ** 2) - 1.0) < 1e-5
    P = O.grid_direct(x, O.CPLX_I8, fs, 0.0, [prn, 5], 0.0, 1.0, 1, Tc, Nnc)
    assert_grid_close(grid, P)


# ---------------------------------------------------------------------------
# detection stage on adversarial grids
# ---------------------------------------------------------------------------

def test_peaks_on_adversarial_grids(ctx):
    rng = np.random.default_rng(4)
    n_prn, nd, N, spc = 5, 7, 500, 3
    Gr = rng.uniform(0.5, 1.0, (n_prn, nd, N)).astype(np.float32)
    Gr[0, 3, 100] = Gr[0, 1, 100] = 9.0          # tie over Doppler -> lowest k
    Gr[1, 2, 10] = Gr[1, 2, 400] = 8.0           # tie over lag -> lowest tau
    Gr[2, 0, 1] = 10.0
    Gr[2, 6, N - 2] = 9.5                         # inside the circular exclusion zone
    Gr[3, 6, 250] = 7.0                           # last Doppler bin: no Doppler refinement
    Gr[4, :, :] = 1.0                             # flat grid
    prns = [4, 8, 15, 16, 23]
    d_g = _dev(Gr)
    d_p = torch.zeros(n_prn * 48, dtype=torch.uint8, device="cuda")
    ctx.peaks(d_g.data_ptr(), prns, nd, N, spc, -300.0, 100.0, d_p.data_ptr(), _stream())
    got = _host(d_p).view(G.PEAK_DTYPE)
    for i in range(n_prn):
        r = O.peak_one(Gr[i].astype(np.float64), prns[i], spc, 2.5, -300.0, 100.0)
        g = got[i]
        assert (g["prn"], g["doppler_bin"], g["code_phase"], bool(g["detected"])) == \
            (r.prn, r.doppler_bin, r.code_phase, r.detected), i
        assert g["peak"] == np.float32(r.peak)
        assert g["second"] == np.float32(r.second)
        # FP32 mean: column sums in row order, then trees over 256 lags and the
        # blocks; relative error <= (additions on the longest path + 2) 2^-24
        assert abs(g["mean"] - r.mean) <= (nd + 8 + 10 + 2) * 2.0 ** -24 * r.mean
        assert abs(g["doppler_hz"] - r.doppler_hz) < 1e-9
        assert abs(g["code_phase_frac"] - r.code_phase_frac) < 1e-9


# ---------------------------------------------------------------------------
# the two measured workloads at full size
# ---------------------------------------------------------------------------

def _run_device(ctx, snap, srch, grid_out=True):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    d_x = _dev(snap.samples)
    d_grid = torch.zeros(len(srch.prns) * nd * N, dtype=torch.float32, device="cuda")
    d_pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
    req = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                         srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                         d_grid.data_ptr(), d_pk.data_ptr())
    ctx.acquire_device(req, _stream())
    grid = _host(d_grid).reshape(len(srch.prns), nd, N)
    pk = _host(d_pk).view(G.PEAK_DTYPE).copy()
    return grid, pk


def test_strong_workload_full_size(ctx, strong_case):
    snap, srch, nd, P = strong_case
    log("strong workload: real 2-bit 4.092 MHz, 32 PRN x 21 bins x 10 ms")
    grid, pk = _run_device(ctx, snap, srch)
    worst = assert_grid_close(grid, P)
    ref = O.peaks(P, srch.prns, 4, 2.5, srch.lo, srch.step)
    exempt = compare_detections(pk, ref, P)
    checked = compare_refinement(pk, ref, P, grid, srch.lo, srch.step)
    assert checked >= len(srch.prns) - exempt
    log("  max err %.2e, exemptions %d, refinements checked %d" % (worst, exempt, checked))
    for p in snap.planted:
        i = srch.prns.index(p.prn)
        assert pk[i]["detected"] and pk[i]["code_phase"] == p.code_phase
    # direct-correlation spot check of sampled cells
    rng = np.random.default_rng(0)
    cells = np.stack([rng.integers(0, 32, 64), rng.integers(0, nd, 64), rng.integers(0, 4092, 64)], 1)
    vals = O.cells_direct(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                          srch.step, nd, srch.T_coh, srch.N_noncoh, cells)
    got = grid[cells[:, 0], cells[:, 1], cells[:, 2]].astype(np.float64)
    means = P.mean(axis=(1, 2))[cells[:, 0]]
    assert np.all(np.abs(got - vals) <= 1e-4 * (vals + means))


@pytest.mark.timeout(600)
def test_weak_workload_full_size(ctx, weak_case):
    snap, srch, nd, P = weak_case
    log("weak workload: complex int8 16.368 MHz, 32 PRN x 121 bins x 25 x 4 ms")
    grid, pk = _run_device(ctx, snap, srch)
    worst = assert_grid_close(grid, P)
    ref = O.peaks(P, srch.prns, 16, 2.5, srch.lo, srch.step)
    exempt = compare_detections(pk, ref, P)
    checked = compare_refinement(pk, ref, P, grid, srch.lo, srch.step)
    assert checked >= len(srch.prns) - exempt
    log("  max err %.2e, exemptions %d, refinements checked %d" % (worst, exempt, checked))
    planted = {p.prn for p in snap.planted}
    det = {int(r["prn"]) for r in pk if r["detected"]}
    assert planted <= det
    # sampled cells against the direct correlation: the planted peaks and random cells
    rng = np.random.default_rng(1)
    cells = [(srch.prns.index(int(r["prn"])), int(r["doppler_bin"]), int(r["code_phase"]))
             for r in pk if r["detected"]]
    cells += list(zip(rng.integers(0, 32, 40), rng.integers(0, nd, 40), rng.integers(0, 16368, 40)))
    cells = np.array(cells, np.int64)
    vals = O.cells_direct(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                          srch.step, nd, srch.T_coh, srch.N_noncoh, cells)
    got = grid[cells[:, 0], cells[:, 1], cells[:, 2]].astype(np.float64)
    means = P.mean(axis=(1, 2))[cells[:, 0]]
    assert np.all(np.abs(got - vals) <= 1e-4 * (vals + means))


def test_device_path_is_deterministic_and_matches_host_path(ctx):
    snap, srch = synth.strong_real_2bit(O.ca_code, seed=3, fmt=O.REAL_2BIT_PACKED)
    g1, p1 = _run_device(ctx, snap, srch)
    g2, p2 = _run_device(ctx, snap, srch)
    assert np.array_equal(g1, g2) and np.array_equal(p1, p2)
    g3, p3 = G.gnss_acquire(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                            srch.hi, srch.step, srch.T_coh, srch.N_noncoh, n=snap.n)
    assert np.array_equal(g1, g3) and np.array_equal(p1, p3)


def test_threshold_option(ctx):
    snap, srch = synth.strong_real_2bit(O.ca_code, seed=1)
    ctx.set("threshold", 1e9)
    try:
        _, pk = _run_device(ctx, snap, srch)
        assert not pk["detected"].any()
    finally:
        ctx.set("threshold", 2.5)
    with pytest.raises(G.GnssError):
        ctx.set("threshold", -1.0)
    with pytest.raises(G.GnssError):
        ctx.set("no_such_option", 1.0)


# ---------------------------------------------------------------------------
# code-Doppler compensation (context option)
# ---------------------------------------------------------------------------

def test_code_doppler_compensation_matches_oracle(ctx):
    # bins far out so that the blocks shift by several samples; every format
    for fmt, fs, f_if in ((O.CPLX_I8, 1023000, 0.0), (O.REAL_2BIT_PACKED, 2046000, 511500.0)):
        Tc, Nnc = 16, 5
        lo, step, nd = -40000.0, 20000.0, 5
        snap = _planted_snapshot(60 + fmt, fmt, fs, f_if, Tc * Nnc + 0.3, [6], 48.0, [-40000.0 + 20000.0 * 3])
        prns = [6, 20]
        ctx.set("code_doppler", 1)
        try:
            grid, peaks = _run_device(ctx, snap, synth.Search(prns, lo, lo + step * (nd - 1), step, Tc, Nnc))
        finally:
            ctx.set("code_doppler", 0)
        P = O.grid_direct(snap.samples, fmt, fs, f_if, prns, lo, step, nd, Tc, Nnc, code_doppler=True)
        worst = assert_grid_close(grid, P)
        ref = O.peaks(P, prns, fs // 1023000, 2.5, lo, step)
        compare_detections(peaks, ref, P)
        plain, _ = _run_device(ctx, snap, synth.Search(prns, lo, lo + step * (nd - 1), step, Tc, Nnc))
        assert not np.array_equal(plain[:, 0], grid[:, 0])  # bin -40 kHz: shifts applied
        log("  code-Doppler fmt %d: max err %.2e" % (fmt, worst))


def test_code_doppler_compensation_realigns_planted_signal(ctx):
    # a satellite whose code rate follows its 10 kHz Doppler over 200 ms: its peak
    # moves 2.5 samples; the compensated search finds the planted code phase
    fs, Tc, Nnc = 2046000, 10, 20
    D = O.nco_step(0.0, 10000.0, fs)
    f_q = D * fs / 2.0 ** 32
    pl = [synth.Planted(prn=9, code_phase=700, doppler_hz=f_q, cn0_dbhz=44.0)]
    snap = synth.make_snapshot(5, O.CPLX_I8, fs, 0.0, Tc * Nnc, pl, O.ca_code, code_doppler=True)
    srch = synth.Search([9, 10], 9000.0, 11000.0, 500.0, Tc, Nnc)
    ctx.set("code_doppler", 1)
    try:
        grid, pk = _run_device(ctx, snap, srch)
    finally:
        ctx.set("code_doppler", 0)
    P = O.grid_fft(snap.samples, O.CPLX_I8, fs, 0.0, srch.prns, srch.lo, srch.step, 5, Tc, Nnc,
                   code_doppler=True)
    assert_grid_close(grid, P)
    assert pk[0]["detected"] and pk[0]["code_phase"] == 700 and pk[0]["doppler_bin"] == 2
    plain, _ = _run_device(ctx, snap, srch)
    log("  planted 10 kHz: compensated peak %.4g, plain max %.4g" % (grid[0].max(), plain[0].max()))
    assert grid[0].max() > plain[0].max()

"""Pins for the oracle's correlation grid (Sec. 3, Fig. 2: mixing, correlation
over all code shifts, detection) and its block processing (Sec. 4).

Pins: a textbook numpy circular cross-correlation (brute force with np.roll
and through the FFT) in the Doppler-0 complex case where the wipe factor is
exactly 4096; the closed form of the noiseless code-vs-code correlation at
integer samples per chip; the planted code phase; a tone at a bin's exact
quantised frequency; agreement of the two oracle routes; recovery of planted
satellites at the configured C/N0.
"""
import numpy as np
import pytest

import oracle as O
import synth


def _cplx_record(re, im):
    x = np.empty(2 * re.size, np.int8)
    x[0::2] = re
    x[1::2] = im
    return x


def test_doppler0_matches_numpy_circular_correlation():
    rng = np.random.default_rng(1)
    fs, N, Tc, Nnc = 2046000, 2046, 2, 3
    re = rng.integers(-127, 128, Tc * Nnc * N).astype(np.int8)
    im = rng.integers(-127, 128, Tc * Nnc * N).astype(np.int8)
    x = _cplx_record(re, im)
    prns = [5, 17]
    P = O.grid_direct(x, O.CPLX_I8, fs, 0.0, prns, 0.0, 100.0, 1, Tc, Nnc)
    xc = re.astype(np.float64) + 1j * im.astype(np.float64)
    for pi, prn in enumerate(prns):
        c = O.code_replica(prn, fs, N).astype(np.float64)
        expect = np.zeros(N)
        for b in range(Nnc):
            blk = xc[b * Tc * N:(b + 1) * Tc * N]
            # brute force: R[tau] = sum_n x[n] c[(n - tau) mod N] ; np.roll(c, tau)[n] = c[n - tau]
            R = np.array([np.dot(blk, np.tile(np.roll(c, tau), Tc)) for tau in range(N)])
            # and the textbook FFT form of the same circular correlation
            fold = blk.reshape(Tc, N).sum(axis=0)
            R2 = np.fft.ifft(np.fft.fft(fold) * np.conj(np.fft.fft(c)))
            assert np.allclose(R, R2, rtol=0, atol=1e-6 * np.abs(R).max())
            expect += np.abs(R) ** 2
        # the wipe factor is exactly 4096 at 0 Hz, so P = sum_b |R_b|^2 up to
        # the FP64 rounding of the squares (|4096 R|^2 exceeds 2^53)
        assert np.all(np.abs(P[pi, 0] - expect) <= 1e-15 * expect)


@pytest.mark.parametrize("spc", [1, 2, 4])
def test_noiseless_code_closed_form(spc):
    """x[n] = c_p[(n - d) mod N] (I only, 0 Hz): R[tau] = 4096 Tc A(d - tau) with
    A(k q + s) = (k - s) rho[q] + s rho[q + 1], rho the chip-level periodic
    autocorrelation.  P = Nnc (Tc A)^2 exactly (integers)."""
    fs = 1023000 * spc
    N, Tc, Nnc, d, prn = 1023 * spc, 2, 2, 37 * spc + 1, 9
    code = 1 - 2 * O.ca_code(prn).astype(np.int64)
    rho = np.array([int(np.dot(code, np.roll(code, -q))) for q in range(1023)])
    rep = O.code_replica(prn, fs, N).astype(np.int64)
    sig = np.tile(np.roll(rep, d), Tc * Nnc)
    x = _cplx_record(sig.astype(np.int8), np.zeros_like(sig, dtype=np.int8))
    P = O.grid_direct(x, O.CPLX_I8, fs, 0.0, [prn], 0.0, 100.0, 1, Tc, Nnc)[0, 0]
    tau = np.arange(N)
    delta = (d - tau) % N
    q, s = delta // spc, delta % spc
    A = (spc - s) * rho[q] + s * rho[(q + 1) % 1023]
    assert np.array_equal(P, Nnc * (Tc * A).astype(np.float64) ** 2)
    assert int(np.argmax(P)) == d
    assert P[d] == Nnc * float(Tc * N) ** 2


def test_planted_tone_at_exact_bin_frequency():
    fs, N, Tc, Nnc, prn, d = 4092000, 4092, 2, 3, 23, 1234
    lo, step, nd = -1000.0, 500.0, 5
    k = 3
    D = O.nco_step(0.0, O.bin_freq(lo, step, k), float(fs))
    fq = D * fs / 2.0 ** 32
    n = np.arange(Tc * Nnc * N)
    A = 60.0
    rep = O.code_replica(prn, fs, N).astype(np.float64)
    sig = A * np.tile(np.roll(rep, d), Tc * Nnc) * np.exp(2j * np.pi * fq * n / fs + 0.7j)
    x = _cplx_record(np.rint(sig.real).astype(np.int8), np.rint(sig.imag).astype(np.int8))
    P = O.grid_direct(x, O.CPLX_I8, fs, 0.0, [prn], lo, step, nd, Tc, Nnc)[0]
    kk, tt = np.unravel_index(np.argmax(P), P.shape)
    assert (kk, tt) == (k, d)
    expect = Nnc * (A * Tc * N) ** 2
    assert abs(P[k, d] / expect - 1.0) < 2e-3


def test_fft_route_matches_direct_route():
    snap, srch = synth.strong_real_2bit(O.ca_code, seed=4)
    prns = [p.prn for p in snap.planted[:2]] + [31]
    nd, lo = 7, -1500.0
    args = (snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, prns, lo, 500.0, nd, 1, 4)
    Pd = O.grid_direct(*args)
    Pf = O.grid_fft(*args)
    for i in range(len(prns)):
        tol = 1e-12 * (Pd[i] + Pd[i].mean())
        assert np.all(np.abs(Pd[i] - Pf[i]) <= tol)


def test_cells_equal_grid_cells():
    snap, _ = synth.strong_real_2bit(O.ca_code, seed=5)
    prns, lo, step, nd = [3, 14], -500.0, 500.0, 3
    args = (snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, prns, lo, step, nd, 1, 3)
    P = O.grid_direct(*args)
    rng = np.random.default_rng(0)
    cells = np.stack([rng.integers(0, 2, 50), rng.integers(0, nd, 50),
                      rng.integers(0, 4092, 50)], axis=1)
    vals = O.cells_direct(*args, cells)
    assert np.array_equal(vals, P[cells[:, 0], cells[:, 1], cells[:, 2]])


def test_folded_blocks_are_sums_of_mixed_samples():
    rng = np.random.default_rng(8)
    fs, N, Tc, Nnc = 1023000, 1023, 3, 2
    x = rng.integers(-127, 128, 2 * Tc * Nnc * N + 20).astype(np.int8)
    f = O.wipe_fold(x, O.CPLX_I8, fs, 0.0, -200.0, 200.0, 3, Tc, Nnc)
    for k in range(3):
        D = O.nco_step(0.0, -200.0 + 200.0 * k, float(fs))
        y = O.wipe(x, O.CPLX_I8, D, 0, Tc * Nnc * N)
        for b in range(Nnc):
            expect = y[b * Tc * N:(b + 1) * Tc * N].reshape(Tc, N, 2).sum(axis=0)
            assert np.array_equal(f[k, b], expect)


def test_strong_workload_recovers_planted():
    snap, srch = synth.strong_real_2bit(O.ca_code, seed=1)
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    assert nd == 21
    P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                   srch.step, nd, srch.T_coh, srch.N_noncoh)
    pk = O.peaks(P, srch.prns, 4, 2.5, srch.lo, srch.step)
    planted = {p.prn: p for p in snap.planted}
    for r in pk:
        if r.prn in planted:
            p = planted[r.prn]
            assert r.detected
            assert r.code_phase == p.code_phase
            assert abs((srch.lo + r.doppler_bin * srch.step) - p.doppler_hz) <= 0.6 * srch.step
        else:
            assert not r.detected


def test_invalid_arguments_rejected():
    x = np.zeros(100, np.int8)
    with pytest.raises(ValueError):
        O.grid_direct(x, O.REAL_I8, 4092000, 0.0, [1], 0.0, 1.0, 1, 1, 1)  # too few samples
    with pytest.raises(ValueError):
        O.ca_code(38)
    with pytest.raises(ValueError):
        O.grid_direct(np.zeros(5000, np.int8), O.REAL_I8, 4092500, 0.0, [1], 0.0, 1.0, 1, 1, 1)


# ---------------------------------------------------------------------------
# sample rates that are not a multiple of the chip rate (any whole number of
# kHz): the replica samples chip floor(n 1023000 / fs) and has no whole number
# of samples per chip
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("fs", [2500000, 5000000, 4000000])
def test_general_rate_doppler0_matches_numpy_circular_correlation(fs):
    rng = np.random.default_rng(fs // 1000)
    N, Tc, Nnc = fs // 1000, 1, 2
    re = rng.integers(-127, 128, Tc * Nnc * N).astype(np.int8)
    im = rng.integers(-127, 128, Tc * Nnc * N).astype(np.int8)
    x = _cplx_record(re, im)
    P = O.grid_direct(x, O.CPLX_I8, fs, 0.0, [7], 0.0, 100.0, 1, Tc, Nnc)[0, 0]
    c = O.code_replica(7, fs, N).astype(np.float64)
    # the replica is the chip-rate code sampled at n * 1023000 / fs, written out here
    chips = 1.0 - 2.0 * O.ca_code(7).astype(np.float64)
    assert np.array_equal(c, chips[(np.arange(N) * 1023000) // fs % 1023])
    xc = re.astype(np.float64) + 1j * im.astype(np.float64)
    expect = np.zeros(N)
    for b in range(Nnc):
        blk = xc[b * N:(b + 1) * N]
        R = np.array([np.dot(blk, np.roll(c, tau)) for tau in range(N)])
        expect += np.abs(R) ** 2
    assert np.all(np.abs(P - expect) <= 1e-15 * expect)


@pytest.mark.parametrize("fs", [5000000, 7777000])
def test_general_rate_noiseless_code_peaks_at_its_phase(fs):
    """x[n] = c_p[(n - d) mod N] at 0 Hz: P[d] = Nnc (Tc N)^2 exactly and it is
    the unique maximum."""
    N, Tc, Nnc, d, prn = fs // 1000, 1, 2, 1234, 22
    rep = O.code_replica(prn, fs, N).astype(np.int64)
    sig = np.tile(np.roll(rep, d), Tc * Nnc)
    x = _cplx_record(sig.astype(np.int8), np.zeros_like(sig, dtype=np.int8))
    P = O.grid_direct(x, O.CPLX_I8, fs, 0.0, [prn], 0.0, 100.0, 1, Tc, Nnc)[0, 0]
    assert P[d] == Nnc * float(Tc * N) ** 2
    others = np.delete(P, d)
    assert others.max() < P[d]


def test_general_rate_fft_route_matches_direct_route():
    fs = 7777000
    pl = [synth.Planted(prn=11, code_phase=4321, doppler_hz=750.0, cn0_dbhz=50.0)]
    snap = synth.make_snapshot(77, O.REAL_I8, fs, 1944250.0, 3.5, pl, O.ca_code)
    args = (snap.samples, snap.fmt, fs, snap.f_if_hz, [11, 2], 0.0, 750.0, 2, 1, 3)
    Pd = O.grid_direct(*args)
    Pf = O.grid_fft(*args)
    for i in range(2):
        assert np.all(np.abs(Pd[i] - Pf[i]) <= 1e-12 * (Pd[i] + Pd[i].mean()))
    r = O.peaks(Pd, [11, 2], O.chip_exclusion(fs), 2.5, 0.0, 750.0)
    assert r[0].detected and r[0].code_phase == 4321 and r[0].doppler_bin == 1


def test_chip_exclusion_is_one_chip():
    assert O.chip_exclusion(4092000) == 4
    assert O.chip_exclusion(5000000) == pytest.approx(4.8876, abs=1e-4)
    # a second peak 5 samples away is a candidate at 5 MHz, 4 samples away is not
    G = np.zeros((1, 5000))
    G[0, 100] = 10.0
    G[0, 104] = 9.0
    G[0, 105] = 2.0
    r = O.peak_one(G, 1, O.chip_exclusion(5000000), 2.5, 0.0, 1.0)
    assert r.second == 2.0 and r.ratio == 5.0


def test_long_integration_generator():
    """The long-integration input (bench.py --workload long) at a reduced size:
    record length 4 ms x blocks + 0.5 ms, the weak-signal search grid over the
    given blocks, eight planted PRNs from 1-32 at 22-30 dB-Hz within the
    Doppler window, and the same record for the same seed."""
    fs, blocks = 1023000, 16
    snap, srch = synth.long_complex_int8(O.ca_code, seed=3, fs=fs, blocks=blocks)
    assert snap.fmt == O.CPLX_I8 and snap.fs_hz == fs
    assert snap.n == int(round(fs * (4.0 * blocks + 0.5) / 1000.0))
    assert srch.prns == list(range(1, 33)) and (srch.lo, srch.hi, srch.step) == (-7500.0, 7500.0, 125.0)
    assert (srch.T_coh, srch.N_noncoh) == (4, blocks)
    assert len(snap.planted) == 8 and len({p.prn for p in snap.planted}) == 8
    for p in snap.planted:
        assert 1 <= p.prn <= 32 and 22.0 <= p.cn0_dbhz <= 30.0 and abs(p.doppler_hz) <= 7500.0
        assert 0 <= p.code_phase < fs // 1000
    again, _ = synth.long_complex_int8(O.ca_code, seed=3, fs=fs, blocks=blocks)
    assert np.array_equal(again.samples, snap.samples)

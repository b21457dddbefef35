"""Pins of the oracle's exact-carrier route (the carrier of the frequency-
domain Doppler variant: exact exponentials instead of the NCO's lookup
table): brute force on tiny inputs, identity with the NCO route where the
carrier frequency is zero, and agreement with the NCO route within the lookup
table's quantisation elsewhere."""
import numpy as np
import pytest

import oracle as O


def _brute(x, fs, f_if, prns, lo, step, nd, Tc, Nnc):
    # the definition written out: per block b and bin k, y[n] = x[bL + n]
    # exp(-2 pi i (f_if + f_k) n / fs), R[tau] = sum_n y[n] c[(n - tau) mod N]
    # over the block's L = Tc N samples, P = sum_b |R|^2
    N = fs // 1000
    L = Tc * N
    P = np.zeros((len(prns), nd, N))
    for pi, prn in enumerate(prns):
        c = O.code_replica(prn, fs, N).astype(np.float64)
        for k in range(nd):
            f = f_if + O.bin_freq(lo, step, k)
            for b in range(Nnc):
                xb = O.raw_samples(x, O.CPLX_I8, b * L, L)
                n = np.arange(L)
                y = xb * np.exp(-2j * np.pi * f * n / fs)
                for tau in range(N):
                    R = np.sum(y * c[(n - tau) % N])
                    P[pi, k, tau] += abs(R) ** 2
    return P


def test_exact_route_matches_brute_force():
    fs, Tc, Nnc = 1023000, 2, 2
    rng = np.random.default_rng(17)
    n = Tc * Nnc * (fs // 1000) + 5
    x = rng.integers(-40, 41, 2 * n).astype(np.int8)
    prns, lo, step, nd = [5], -750.0, 500.0, 4
    P1 = O.grid_fft(x, O.CPLX_I8, fs, 0.0, prns, lo, step, nd, Tc, Nnc, carrier="exact")
    P2 = _brute(x, fs, 0.0, prns, lo, step, nd, Tc, Nnc)
    assert np.max(np.abs(P1 - P2) / (P2 + P2.mean())) < 1e-11


def test_zero_carrier_equals_nco_route():
    # f_if + f_k = 0: the NCO phase stays 0, LUT entry 0 is 4096 exactly, so both
    # routes correlate the same integers (2^-24 undoes the 4096^2)
    fs, Tc, Nnc = 4092000, 1, 3
    rng = np.random.default_rng(3)
    n = Tc * Nnc * (fs // 1000)
    x = rng.integers(-3, 4, n).astype(np.int8)
    f_if = 1023000.0
    Pe = O.grid_fft(x, O.REAL_I8, fs, f_if, [1, 9], -f_if, 500.0, 1, Tc, Nnc, carrier="exact")
    Pn = O.grid_fft(x, O.REAL_I8, fs, f_if, [1, 9], -f_if, 500.0, 1, Tc, Nnc)
    assert np.max(np.abs(Pe - Pn) / (Pn + Pn.mean())) < 1e-12


@pytest.mark.parametrize("fmt,fs,f_if", [(O.CPLX_I8, 2046000, 0.0), (O.REAL_2BIT_PACKED, 4092000, 1023000.0)])
def test_exact_route_close_to_nco_route(fmt, fs, f_if):
    # the NCO route's carrier is a 1024-entry table of 4096 e^(i theta) rounded
    # to integers and indexed by the top 10 phase bits: its phase error is at
    # most pi/1024 and its amplitude error ~1.2e-4, so powers agree to ~1e-2 of
    # the grid scale
    import synth
    rng = np.random.default_rng(fs)
    N = fs // 1000
    pl = [synth.Planted(prn=7, code_phase=int(rng.integers(0, N)), doppler_hz=1300.0, cn0_dbhz=48.0)]
    snap = synth.make_snapshot(5, fmt, fs, f_if, 6.0, pl, O.ca_code)
    args = (snap.samples, fmt, fs, f_if, [7, 20], -2000.0, 500.0, 9, 2, 3)
    Pe = O.grid_fft(*args, carrier="exact")
    Pn = O.grid_fft(*args)
    err = np.max(np.abs(Pe - Pn) / (Pn + Pn.mean()))
    assert err < 1e-2, err
    # same detections
    re = O.peaks(Pe, [7, 20], fs // 1023000, 2.5, -2000.0, 500.0)
    rn = O.peaks(Pn, [7, 20], fs // 1023000, 2.5, -2000.0, 500.0)
    assert [(r.detected, r.doppler_bin, r.code_phase) for r in re] == \
           [(r.detected, r.doppler_bin, r.code_phase) for r in rn]

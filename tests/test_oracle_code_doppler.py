"""Pins of the oracle's code-Doppler compensation (an option of the
non-coherent sum): the direct and FFT routes agree, zero Doppler changes
nothing, and on a signal generated with the physical code-rate model the
compensated sum peaks at the planted code phase where the plain sum smears."""
import numpy as np

import oracle as O
import synth


def test_direct_and_fft_routes_agree_with_compensation():
    fs, Tc, Nnc = 1023000, 16, 6
    lo, step, nd = -40000.0, 20000.0, 5  # large bins: shifts of several samples
    rng = np.random.default_rng(3)
    n = Tc * Nnc * (fs // 1000) + 11
    x = rng.integers(-20, 21, 2 * n).astype(np.int8)
    prns = [4, 17]
    P1 = O.grid_direct(x, O.CPLX_I8, fs, 0.0, prns, lo, step, nd, Tc, Nnc, code_doppler=True)
    P2 = O.grid_fft(x, O.CPLX_I8, fs, 0.0, prns, lo, step, nd, Tc, Nnc, code_doppler=True)
    assert np.max(np.abs(P1 - P2) / (P1 + P1.mean())) < 1e-12
    P0 = O.grid_direct(x, O.CPLX_I8, fs, 0.0, prns, lo, step, nd, Tc, Nnc)
    shifts = [O.code_shift(b, Tc, fs // 1000, lo) for b in range(Nnc)]
    assert shifts[-1] != 0
    assert not np.array_equal(P0[:, 0], P1[:, 0])
    assert np.array_equal(P0[:, 2], P1[:, 2])  # the 0 Hz bin is unchanged


def test_shift_values():
    # drift of the weak workload's last block at the window edge: 96 ms x 7.5 kHz /
    # 1575.42 MHz x 16.368 MHz = 7.47 samples
    assert O.code_shift(24, 4, 16368, 7500.0) == 7
    assert O.code_shift(24, 4, 16368, -7500.0) == -7
    assert O.code_shift(0, 4, 16368, 7500.0) == 0
    assert O.code_shift(5, 1, 4092, 0.0) == 0


def test_compensation_realigns_a_code_doppler_signal():
    # noiseless complex baseband signal whose code rate follows a 10 kHz Doppler over
    # 20 blocks of 10 ms: its correlation peak moves 2.5 samples; compensated, the
    # non-coherent sum peaks at the planted code phase (the code phase at sample 0)
    fs, Tc, Nnc = 2046000, 10, 20
    N = fs // 1000
    D = O.nco_step(0.0, 10000.0, fs)
    f_q = D * fs / 2.0 ** 32  # on the NCO grid: no carrier residual
    pl = [synth.Planted(prn=9, code_phase=700, doppler_hz=f_q, cn0_dbhz=65.6)]
    snap = synth.make_snapshot(5, O.CPLX_I8, fs, 0.0, Tc * Nnc, pl, O.ca_code, noise=False,
                               code_doppler=True)
    P0 = O.grid_fft(snap.samples, O.CPLX_I8, fs, 0.0, [9], 10000.0, 500.0, 1, Tc, Nnc)[0, 0]
    P1 = O.grid_fft(snap.samples, O.CPLX_I8, fs, 0.0, [9], 10000.0, 500.0, 1, Tc, Nnc,
                    code_doppler=True)[0, 0]
    assert int(np.argmax(P1)) == 700
    assert P1.max() > 1.15 * P0.max()
    # the opposite compensation makes it worse than none
    P2 = O.grid_fft(snap.samples, O.CPLX_I8, fs, 0.0, [9], -10000.0, 500.0, 1, Tc, Nnc,
                    code_doppler=True)
    assert P2.max() < P1.max()

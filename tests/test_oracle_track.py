"""Pins of the oracle's tracking correlators (early / prompt / late, Fig. 3)
against things other than their own formula: the acquisition oracle's direct
correlation (an independent routine), closed forms of noiseless code, a pure
tone's phase, and the acquisition code replica."""
import math

import numpy as np
import pytest

import oracle as O
import synth


def _cplx(re, im=None):
    x = np.zeros(2 * len(re), np.int8)
    x[0::2] = re
    if im is not None:
        x[1::2] = im
    return x


@pytest.mark.parametrize("fmt,fs,f_if", [(O.CPLX_I8, 4092000, 0.0), (O.REAL_I8, 4092000, 1023000.0),
                                         (O.REAL_2BIT_PACKED, 8184000, 2046000.0)])
def test_prompt_power_equals_acquisition_direct_correlation(fmt, fs, f_if):
    # code rate 1.023 MHz at spc = fs / 1.023 MHz (exact in fixed point), code phase at
    # sample 0 = -tau / spc chips: the prompt replica is the acquisition replica at lag tau,
    # so sum_e |P_e|^2 2^-24 over 1 ms epochs is the acquisition grid cell (p, k, tau).
    rng = np.random.default_rng(fs + fmt)
    N = fs // 1000
    spc = fs // 1023000
    pl = [synth.Planted(prn=7, code_phase=int(rng.integers(0, N)), doppler_hz=1200.0, cn0_dbhz=50.0)]
    snap = synth.make_snapshot(11 + fmt, fmt, fs, f_if, 4.0, pl, O.ca_code)
    lo, step, nd = -1500.0, 500.0, 7
    cells, chans = [], []
    for prn_i, prn in enumerate([7, 12]):
        for k in (1, 5):
            for tau in (0, 1, pl[0].code_phase, N - 1, int(rng.integers(0, N))):
                cells.append((prn_i, k, tau))
                chans.append(O.Channel(prn=prn, carrier_hz=f_if + (lo + k * step), carrier_phase=0.0,
                                       code_phase=(1023.0 - tau / spc) % 1023.0, code_rate=1023000.0,
                                       spacing=0.5))
    ref = O.cells_direct(snap.samples, fmt, fs, f_if, [7, 12], lo, step, nd, 1, 4, cells)
    out = O.track(snap.samples, fmt, fs, chans, 0, N, 4)
    for i in range(len(cells)):
        acc = 0.0
        for e in range(4):
            re, im = float(out[i, e, 1, 0]), float(out[i, e, 1, 1])
            acc += (re * re + im * im) * 2.0 ** -24
        assert acc == ref[i], (cells[i], acc, ref[i])


def test_noiseless_code_closed_forms_early_prompt_late():
    # x[n] = A c(n - d) (complex baseband, no carrier), replica lagging the signal by
    # one sample: P = 4096 A (L - 2 T1), E (advanced half a chip = 2 samples) and L
    # (retarded 2 samples) from the run structure of the code:  with spc = 4 a
    # replica offset by j samples disagrees with the signal on j samples at every
    # chip transition, so X = 4096 A (L - 2 |j_X| T) over an epoch of whole periods,
    # T = number of chip transitions per period (circular).
    fs, spc, A = 4092000, 4, 5
    N = fs // 1000
    prn = 19
    code = O.ca_code(prn).astype(np.int64)
    T = int(np.sum(code != np.roll(code, -1)))
    d = 37
    rep = O.code_replica(prn, fs, N).astype(np.int64)
    sig = np.tile(np.roll(rep, d), 3) * A
    x = _cplx(sig.astype(np.int8))
    # replica code phase: signal chip 0 at sample d; replica chip 0 one sample later
    ch = O.Channel(prn=prn, carrier_hz=0.0, carrier_phase=0.0, code_phase=(1023.0 - (d + 1) / spc),
                   code_rate=1023000.0, spacing=0.5)
    out = O.track(x, O.CPLX_I8, fs, [ch], 0, N, 3)
    # offsets (replica - signal) in samples: early -1, prompt +1, late +3
    for e in range(3):
        E, P, L = (out[0, e, i, 0] for i in range(3))
        assert (out[0, e, :, 1] == 0).all()
        assert P == 4096 * A * (N - 2 * 1 * T)
        assert E == 4096 * A * (N - 2 * 1 * T)
        assert L == 4096 * A * (N - 2 * 3 * T)
    # replica exactly on the signal: E = L (symmetric), P the full energy
    ch0 = O.Channel(prn=prn, carrier_hz=0.0, carrier_phase=0.0, code_phase=(1023.0 - d / spc),
                    code_rate=1023000.0, spacing=0.5)
    o0 = O.track(x, O.CPLX_I8, fs, [ch0], 0, N, 1)[0, 0]
    assert o0[1, 0] == 4096 * A * N
    assert o0[0, 0] == o0[2, 0] == 4096 * A * (N - 2 * 2 * T)


def test_carrier_phase_sign_and_unit():
    # a tone at a frequency on the NCO grid with phase theta: the prompt correlator of a
    # replica with carrier_phase = theta / (2 pi) is real positive, a quarter cycle off
    # rotates it by -90 degrees; everything within the LUT's phase quantisation.
    fs = 2046000
    N = fs // 1000
    f = 3000.0
    D = O.track_fixed(O.Channel(1, f, 0.0, 0.0, 1023000.0, 0.5), fs)[0]
    f_q = D * fs / 2.0 ** 32
    theta = 1.1
    n = np.arange(N)
    v = 60.0 * np.exp(1j * (2 * np.pi * f_q * n / fs + theta))
    # the tone is spread by the PRN's code, which the prompt replica removes
    prn = 3
    rep = O.code_replica(prn, fs, N).astype(np.int64)
    xr = np.rint(v.real).astype(np.int64) * rep
    xi = np.rint(v.imag).astype(np.int64) * rep
    x = _cplx(xr.astype(np.int8), xi.astype(np.int8))
    for extra, want in ((0.0, 0.0), (0.25, -math.pi / 2)):
        ch = O.Channel(prn=prn, carrier_hz=f, carrier_phase=(theta / (2 * np.pi) + extra) % 1.0,
                       code_phase=0.0, code_rate=1023000.0, spacing=0.5)
        P = O.track(x, O.CPLX_I8, fs, [ch], 0, N, 1)[0, 0, 1]
        ang = math.atan2(float(P[1]), float(P[0]))
        assert abs(math.remainder(ang - want, 2 * math.pi)) < 2 * math.pi / 1024 + 0.02
        assert math.hypot(float(P[0]), float(P[1])) > 0.98 * 4096 * 60 * N


def test_prompt_replica_matches_acquisition_replica_at_other_rates():
    # code rate 1.023 MHz, code phase 0: the prompt chip at sample n is
    # floor(n * 1023000 / fs) mod 1023 (the acquisition replica) except where the
    # fixed-point step's rounding (|err| <= 2^-33 chips per sample) crosses a chip
    # boundary.  A unit impulse at sample n reads the replica value through P.
    fs = 5000000
    n_s = 4000
    rep = O.code_replica(9, fs, n_s).astype(np.int64)
    R = O.track_fixed(O.Channel(9, 0.0, 0.0, 0.0, 1023000.0, 0.5), fs)[3]
    mism = 0
    idx = np.arange(0, n_s, 7)
    for n in idx:
        x = np.zeros(2 * n_s, np.int8)
        x[2 * n] = 1
        ch = O.Channel(prn=9, carrier_hz=0.0, carrier_phase=0.0, code_phase=0.0, code_rate=1023000.0,
                       spacing=0.5)
        P = O.track(x, O.CPLX_I8, fs, [ch], 0, n_s, 1)[0, 0, 1, 0]
        if P != 4096 * rep[n]:
            # allowed only within the accumulated rounding of a chip boundary
            exact = n * 1023000 / fs
            assert abs(exact - round(exact)) <= n * 2.0 ** -33 + 1e-12 and abs(R * n / 2 ** 32 - exact) < 1e-6
            mism += 1
    assert mism <= 1


def test_track_rejects_bad_arguments():
    x = np.zeros(200, np.int8)
    ch = O.Channel(prn=1, carrier_hz=0.0, carrier_phase=0.0, code_phase=0.0, code_rate=1023000.0,
                   spacing=0.5)
    with pytest.raises(ValueError):
        O.track(x, O.CPLX_I8, 1023000, [ch], 0, 60, 2)  # 120 samples needed, 100 present
    with pytest.raises(ValueError):
        O.track(x, O.CPLX_I8, 1023000, [O.Channel(38, 0.0, 0.0, 0.0, 1023000.0, 0.5)], 0, 10, 1)

"""Pins for the oracle's carrier NCO and first mixing stage (Sec. 3, Fig. 2).

The paper gives no NCO design; the reading adopted is a 32-bit phase
accumulator, a 1024-entry integer LUT of amplitude 4096 and down-conversion
by exp(-j theta).  Pins: exact LUT values at the quarter points and the
octant, symmetries, the distance of every entry from a rounding tie, the
fs/4 special case whose wipe factor cycles exactly through
4096, -4096j, -4096, +4096j, an arbitrary-precision phase computation, and a
tone at a bin's quantised frequency that must be mixed to DC.
"""
import math

import numpy as np

import oracle as O


def test_lut_quarter_points_and_octant():
    c, s = O.lut()
    assert (c[0], s[0]) == (4096, 0)
    assert (c[256], s[256]) == (0, 4096)
    assert (c[512], s[512]) == (-4096, 0)
    assert (c[768], s[768]) == (0, -4096)
    assert (c[128], s[128]) == (2896, 2896)  # 4096/sqrt(2) = 2896.31


def test_lut_symmetries():
    c, s = O.lut()
    i = np.arange(1, 1024)
    assert np.array_equal(c[i], c[1024 - i])
    assert np.array_equal(s[i], -s[1024 - i])
    j = np.arange(256)
    assert np.array_equal(s[j], c[256 - j])
    assert np.array_equal(c[(j + 256) % 1024], -s[j])
    assert np.all(np.abs(c.astype(np.int64)) <= 4096) and np.all(np.abs(s.astype(np.int64)) <= 4096)


def test_lut_entries_are_far_from_rounding_ties():
    # Any cos/sin accurate to 1e-9 gives the same integer table: every exact
    # value 4096*cos(2 pi i/1024) is at least 6.8e-3 away from a half-integer.
    c, s = O.lut()
    for i in range(1024):
        for val, tab in ((4096.0 * math.cos(2 * math.pi * i / 1024), c[i]),
                         (4096.0 * math.sin(2 * math.pi * i / 1024), s[i])):
            frac = abs(val - math.floor(val) - 0.5)
            assert frac > 6.7e-3
            assert abs(val - int(tab)) < 0.5


def test_nco_step_special_values():
    fs = 4092000.0
    assert O.nco_step(fs / 4, 0.0, fs) == 1 << 30
    assert O.nco_step(0.0, 0.0, fs) == 0
    assert O.nco_step(fs / 2, 0.0, fs) == 1 << 31
    # negative frequencies wrap as two's complement
    assert O.nco_step(0.0, -1000.0, fs) == (1 << 32) - round(1000.0 * 2 ** 32 / fs)
    # f_if + bin frequency are added before scaling
    assert O.nco_step(1023000.0, 500.0, fs) == round(1023500.0 * 2 ** 32 / fs)


def test_fs_over_4_wipe_cycles_exactly():
    fs = 4092000
    x = np.ones(16, np.int8)
    D = O.nco_step(fs / 4, 0.0, float(fs))
    y = O.wipe(x, O.REAL_I8, D, 0, 16)
    expect = np.array([[4096, 0], [0, -4096], [-4096, 0], [0, 4096]] * 4)
    assert np.array_equal(y, expect)


def test_phase_index_matches_big_integer_phase():
    rng = np.random.default_rng(5)
    n_total = 1 << 21
    x = np.ones(n_total, np.int8)
    c, s = O.lut()
    for D in (123456789, 4000000000, 1, 2 ** 32 - 1):
        n0 = int(rng.integers(0, n_total - 64))
        y = O.wipe(x, O.REAL_I8, D, n0, 64)
        for i in range(64):
            idx = ((n0 + i) * D % (1 << 32)) >> 22  # Python integers: no wrap errors
            assert (y[i, 0], y[i, 1]) == (c[idx], -s[idx])


def test_complex_mixing_sign_and_real_image():
    c, s = O.lut()
    # (xr + j xi)(c - j s) for a single sample at phase index 100
    D = 100 << 22
    x = np.array([0, 0, 3, -2], np.int8)  # two complex samples: (0,0), (3,-2)
    y = O.wipe(x, O.CPLX_I8, D, 0, 2)
    assert tuple(y[0]) == (0, 0)
    cc, ss = int(c[100]), int(s[100])
    assert tuple(y[1]) == (3 * cc + (-2) * ss, (-2) * cc - 3 * ss)


def test_tone_at_bin_frequency_is_mixed_to_dc():
    fs = 4092000
    f_bin = 1500.0
    D = O.nco_step(0.0, f_bin, float(fs))
    f_q = D * fs / 2.0 ** 32  # the bin's quantised frequency
    n = np.arange(4092)
    A = 100.0
    tone = A * np.exp(2j * np.pi * f_q * n / fs)
    x = np.empty(2 * n.size, np.int8)
    x[0::2] = np.rint(tone.real)
    x[1::2] = np.rint(tone.imag)
    y = O.wipe(x, O.CPLX_I8, D, 0, n.size)
    yc = (y[:, 0] + 1j * y[:, 1]) / 4096.0
    # residual carrier: phase-truncation error only (LUT index is phi >> 22)
    assert abs(np.mean(yc)) > 0.99 * A
    assert np.std(np.angle(yc)) < 2 * np.pi / 1024


def test_packed_2bit_equals_int8_record():
    import synth

    rng = np.random.default_rng(3)
    q = rng.choice(np.array([-3, -1, 1, 3], np.int8), size=4092 * 3)
    packed = synth.pack_2bit(q)
    D = O.nco_step(1023000.0, 0.0, 4092000.0)
    a = O.wipe(q, O.REAL_I8, D, 0, q.size)
    b = O.wipe(packed, O.REAL_2BIT_PACKED, D, 0, q.size)
    assert np.array_equal(a, b)
    assert np.array_equal(synth.unpack_2bit(packed, q.size), q)

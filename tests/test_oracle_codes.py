"""Pins for the oracle's code NCO (C/A code generation and code replica).

The paper's acquisition channel generates a local code replica (Sec. 3,
Fig. 2); the code itself is the GPS C/A Gold code of IS-GPS-200 Table 3-Ia.
These tests pin the oracle against facts that do not come from its own
formula: the table's octal first-10-chip column, the table's G2-delay column
(a different construction from the tap pairs the oracle uses), code balance
and the three-valued Gold correlation property.
"""
import numpy as np
import pytest

import oracle as O


def _lfsr_sequence(taps_feedback, length=1023):
    """Plain 10-stage shift register started all ones; returns the stage-10
    output sequence.  taps_feedback are the stages XORed into stage 1."""
    reg = [1] * 11
    out = []
    for _ in range(length):
        out.append(reg[10])
        fb = 0
        for t in taps_feedback:
            fb ^= reg[t]
        reg[2:11] = reg[1:10]
        reg[1] = fb
    return np.array(out, np.uint8)


def test_first_ten_chips_match_icd_octal(icd_table):
    for prn, _, _, _, octal in icd_table:
        chips = O.ca_code(prn)[:10]
        value = int("".join(str(int(c)) for c in chips), 2)
        assert value == octal, "PRN %d: %o != %o" % (prn, value, octal)


def test_g2_delay_construction_matches(icd_table):
    # chip_n = G1_n xor G2_(n - delay): the delay column of Table 3-Ia, an
    # independent construction of the same codes.
    g1 = _lfsr_sequence((3, 10))
    g2 = _lfsr_sequence((2, 3, 6, 8, 9, 10))
    n = np.arange(1023)
    for prn, _, _, delay, _ in icd_table:
        expect = g1 ^ g2[(n - delay) % 1023]
        assert np.array_equal(O.ca_code(prn), expect), prn


def test_prn1_leading_chips():
    # 1440 octal followed by the next six chips of the same sequence.
    assert "".join(map(str, O.ca_code(1)[:16])) == "1100100000111001"


def test_balance_prn_1_to_32():
    for prn in range(1, 33):
        assert int(O.ca_code(prn).sum()) == 512


def test_prns_34_and_37_share_a_code():
    assert np.array_equal(O.ca_code(34), O.ca_code(37))


def test_gold_three_valued_correlation():
    """Gold codes of degree 10: periodic cross-correlation and off-peak
    autocorrelation take only the values {-1, -65, 63}; the peak is 1023."""
    codes = np.stack([1.0 - 2.0 * O.ca_code(p) for p in range(1, 33)])
    F = np.fft.fft(codes, axis=1)
    allowed = {-1, -65, 63}
    for a in range(32):
        corr = np.rint(np.fft.ifft(np.conj(F[a])[None, :] * F, axis=1).real).astype(np.int64)
        for b in range(32):
            vals = corr[b]
            if a == b:
                assert vals[0] == 1023
                assert set(np.unique(vals[1:])) <= allowed
            else:
                assert set(np.unique(vals)) <= allowed, (a + 1, b + 1)


@pytest.mark.parametrize("spc", [1, 2, 4, 8, 16])
def test_replica_repeats_each_chip_spc_times(spc):
    fs = 1023000 * spc
    code = O.ca_code(7)
    rep = O.code_replica(7, fs, 1023 * spc)
    expect = np.repeat(1 - 2 * code.astype(np.int64), spc)
    assert np.array_equal(rep.astype(np.int64), expect)


def test_replica_period_and_offset():
    fs = 4092000
    full = O.code_replica(3, fs, 3 * 4092)
    assert np.array_equal(full[:4092], full[4092:8184])
    part = O.code_replica(3, fs, 100, n0=5000)
    assert np.array_equal(part, full[5000:5100])


def test_replica_non_integer_rate_reads_the_chip_active_at_sample_time():
    # 5 MHz: 5000 samples per code period.  Sample n is taken at time n/fs and
    # must read the chip m active then: m/1.023e6 <= n/fs < (m+1)/1.023e6.
    fs = 5000000
    rep = O.code_replica(11, fs, 5000).astype(np.int64)
    code = 1 - 2 * O.ca_code(11).astype(np.int64)
    n = np.arange(5000, dtype=np.int64)
    m = np.searchsorted(np.arange(1024, dtype=np.int64) * fs, n * 1023000, side="right") - 1
    assert np.all(m * fs <= n * 1023000) and np.all(n * 1023000 < (m + 1) * fs)
    assert np.array_equal(rep, code[m])
    counts = np.bincount(m, minlength=1023)
    assert counts.min() >= 4 and counts.max() <= 5 and counts.sum() == 5000

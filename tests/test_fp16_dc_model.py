"""Why the exact-length FP16 mode removes each block's mean (CPU, model).

A block dominated by a constant (a DC offset in the recorded samples, at a
Doppler bin equal to the carrier) has almost all of its spectrum in bin 0.
The FP16 weights of the forward transform leak a few 10^-6 of that bin's
amplitude into every other bin, and there the code spectrum is about 32
(sqrt(1023)) against +-1 at DC: the leak, multiplied by 32 and summed over
1022 bins, reaches percents of the correlation, whose exact value is the
small constant mean * sum(code).  The numpy model of the mode's roundings
(fp16_pfa_model.py, checked against the GPU transform in test_gpu_pfa.py)
shows it: with FP16 weights the error of a full-scale constant is ~1.7e-2,
with exact weights it is ~1e-5, and with the mean removed before the
transform (bin 0 set to the exact sum) it is ~1e-5 with FP16 weights too.
The bound the mode is held to is TOLX = 2.0e-2 (tests/test_gpu_fp16.py).
"""
import numpy as np
import pytest

import fp16_pfa_model as M

TOLX = 2.0e-2
K = 16 * 64 * 4096  # boxcar x 64 ms fold x LUT amplitude


def _const(a=127 + 127j):
    return np.full(M.L, K * a)


def _noise(rng, amp):
    return (rng.integers(-amp, amp + 1, M.L) + 1j * rng.integers(-amp, amp + 1, M.L)) * K


@pytest.mark.parametrize("prn", [3, 19])
def test_constant_block_error_comes_from_the_fp16_weights(prn):
    plain = M.mixed_power_error(_const(), prn, mean_removed=False)
    exact_w = M.mixed_power_error(_const(), prn, mean_removed=False, fp16_weights=False)
    assert plain > 1e-2, plain          # the failure the mode had
    assert exact_w < 1e-4, exact_w      # gone with exact weights: the weights leak
    assert plain > 100 * exact_w


@pytest.mark.parametrize("prn", [3, 19])
def test_mean_removal_fixes_dc_blocks(prn):
    rng = np.random.default_rng(prn)
    cases = {"full-scale constant": _const(),
             "constant of 1": _const(1 + 1j),
             "offset + small noise": _const() + _noise(rng, 3),
             "offset + noise": _const(40 - 25j) + _noise(rng, 60)}
    for name, g in cases.items():
        err = M.mixed_power_error(g, prn, mean_removed=True)
        assert err < TOLX / 10, (name, err)
    # the offset-plus-small-noise block broke the bound without it
    assert M.mixed_power_error(cases["offset + small noise"], prn, mean_removed=False) > 0.5 * TOLX


def test_mean_removal_keeps_zero_mean_blocks_unchanged():
    """For noise the two schemes are equally good (the mean is ~0)."""
    rng = np.random.default_rng(7)
    g = _noise(rng, 127)
    a = M.mixed_power_error(g, 5, mean_removed=False)
    b = M.mixed_power_error(g, 5, mean_removed=True)
    assert a < 5e-3 and b < 5e-3, (a, b)


def test_model_transform_is_the_dft():
    """The model's index maps and weights make a DFT (FP64 weights, no FP16
    rounding: within FP32 of numpy)."""
    rng = np.random.default_rng(3)
    g = rng.standard_normal(M.L) + 1j * rng.standard_normal(M.L)
    ref = np.fft.fft(g)
    got = M.forward(g * 1e3, mean_removed=False, fp16_weights=True) / 1e3
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    assert np.max(np.abs(got - ref)) < 1e-2 * rms
    # exact weights: only the FP16 input and 31-pass roundings remain
    got = M.forward(g * 1e3, mean_removed=True, fp16_weights=False) / 1e3
    assert np.sqrt(np.mean(np.abs(got - ref) ** 2)) < 2e-3 * rms

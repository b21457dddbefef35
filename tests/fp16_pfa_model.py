"""A numpy model of the exact-length FP16 mode's roundings (test helper).

Not the oracle and not the product: a model of where the GNSS_FP16_PFA
arithmetic rounds, used to explain its error bound and to show why a
DC-dominated block needs its mean removed before the FP16 transform.  It
follows the documented rounding points of that mode:

* the 1023-point DFT as the Good-Thomas 31 x 33 transform, time index
  m = (33 n1 + 31 n2) mod 1023, frequency index k = (528 a + 496 b) mod 1023;
* the input scaled by 2^-e (e from the l1 norm) and rounded to FP16;
* each pass a real-form product with FP16 weights (cos and sin of the exact
  angle, each rounded once), exact FP16 x FP16 products summed in FP32;
* the 31-pass output rounded to FP16 before the 33-pass; the stored spectrum
  and the code spectrum (times 2^-ecs) in FP16;
* the spectrum product in packed FP16 as the kernel forms it:
  re = fma(gr, cr, gi ci), im = fma(gi, cr, -(gr ci)), the inner product
  rounded first.

Its forward transform is checked against the GPU's gnss_dft1023 in
tests/test_gpu_pfa.py; the consequences are checked in
tests/test_fp16_dc_model.py.
"""
import numpy as np

import oracle as O

L1, L2, L = 31, 33, 1023
_n1 = np.arange(L1)[:, None]
_n2 = np.arange(L2)[None, :]
TMAP = (33 * _n1 + 31 * _n2) % L    # [n1][n2] -> time index
FMAP = (528 * _n1 + 496 * _n2) % L  # [a][b]  -> frequency index


def _f32(x):
    x = np.asarray(x)
    return (np.asarray(x.real, np.float32).astype(np.float64)
            + 1j * np.asarray(x.imag, np.float32).astype(np.float64))


def _f16(x):
    """Round each part to FP16 (through FP32, as the kernels convert FP32 values)."""
    x = np.asarray(x)
    return (np.asarray(x.real, np.float32).astype(np.float16).astype(np.float64)
            + 1j * np.asarray(x.imag, np.float32).astype(np.float16).astype(np.float64))


def _h(v):
    return np.asarray(v, np.float32).astype(np.float16).astype(np.float64)


def weights(n: int, inverse: bool, fp16: bool = True):
    """Real-form weights (cos, signed sin) of an n-point DFT."""
    e = np.outer(np.arange(n), np.arange(n)) % n
    th = 2.0 * np.pi * e / n
    cs, sn = np.cos(th), np.sin(th)
    if fp16:
        cs = cs.astype(np.float16).astype(np.float64)
        sn = sn.astype(np.float16).astype(np.float64)
    return cs, (1.0 if inverse else -1.0) * sn


def _pass(x, w, axis):
    """sum over the input index of x * (cs + i sn), exact products, FP32 result."""
    cs, sn = w
    xr, xi = x.real, x.imag
    if axis == 0:
        re = cs.T @ xr - sn.T @ xi
        im = sn.T @ xr + cs.T @ xi
    else:
        re = xr @ cs - xi @ sn
        im = xr @ sn + xi @ cs
    return _f32(re + 1j * im)


def l1_exponent(s: float) -> int:
    """Smallest e with s (1 + 2^-10) 2^-e <= 32 (0 for s = 0)."""
    if not s > 0:
        return 0
    _, x = np.frexp(np.float32(s) * np.float32(1.0 + 2.0 ** -10))
    return int(x) - 5


def forward(g, mean_removed: bool, fp16_weights: bool = True, scaled_output: bool = False):
    """Forward 1023-point transform of one vector g (complex integers) in the
    mode's arithmetic.  mean_removed: the mean S/1023 is subtracted before
    the FP16 transform and bin 0 is set to S.  Returns the spectrum in natural
    order, unscaled (times 2^e), or with scaled_output the FP16-rounded
    scaled spectrum and e."""
    g = np.asarray(g, np.complex128)
    S = complex(np.float32(g.real.sum()), np.float32(g.imag.sum()))
    if mean_removed:
        mu = complex(np.float32(S.real) / np.float32(L), np.float32(S.imag) / np.float32(L))
        x = _f32(_f32(g) - mu)
        e = l1_exponent(np.abs(x.real).sum() + np.abs(x.imag).sum() + abs(S.real) + abs(S.imag))
    else:
        x = _f32(g)
        e = l1_exponent(np.abs(x.real).sum() + np.abs(x.imag).sum())
    xs = _f16(_f32(x * 2.0 ** -e))
    y = _f16(_pass(xs[TMAP], weights(L1, False, fp16_weights), axis=0))   # [a][n2]
    X = _pass(y, weights(L2, False, fp16_weights), axis=1)                 # [a][b]
    out = np.zeros(L, np.complex128)
    out[FMAP] = X
    if mean_removed:
        out[0] = S * 2.0 ** -e
    if scaled_output:
        return _f16(out), e
    return out * 2.0 ** e


def code_spectrum(prn: int) -> np.ndarray:
    return np.fft.fft(1.0 - 2.0 * O.ca_code(prn).astype(np.float64))


def code_exponent() -> int:
    m = max(np.abs(code_spectrum(p)).max() for p in range(1, 38))
    e = 0
    while 2.0 ** e < m * (1.0 + 2.0 ** -10):
        e += 1
    return e


def correlation(g, prn: int, mean_removed: bool, fp16_weights: bool = True):
    """R[q] = sum_m g[m] c[(m - q) mod 1023] through the mode's arithmetic."""
    G16, e = forward(g, mean_removed, fp16_weights, scaled_output=True)
    ecs = code_exponent()
    C = _f16(code_spectrum(prn) * 2.0 ** -ecs)
    gr, gi, cr, ci = G16.real, G16.imag, C.real, C.imag
    Z = _h(gr * cr + _h(gi * ci)) + 1j * _h(gi * cr - _h(gr * ci))
    y = _f16(_pass(Z[FMAP], weights(L1, True, fp16_weights), axis=0))   # [n1][b]
    R = _pass(y, weights(L2, True, fp16_weights), axis=1)               # [n1][n2]
    out = np.zeros(L, np.complex128)
    out[TMAP] = R
    return out * 2.0 ** (e + ecs) / L


def exact_correlation(g, prn: int):
    c = 1.0 - 2.0 * O.ca_code(prn).astype(np.float64)
    return np.fft.ifft(np.fft.fft(np.asarray(g, np.complex128)) * np.conj(np.fft.fft(c)))


def mixed_power_error(g, prn: int, mean_removed: bool, fp16_weights: bool = True) -> float:
    """max |P - P64| / (P64 + mean P64) over the lags, P = |R|^2."""
    P = np.abs(correlation(g, prn, mean_removed, fp16_weights)) ** 2
    Px = np.abs(exact_correlation(g, prn)) ** 2
    return float(np.max(np.abs(P - Px) / (Px + Px.mean())))

"""FP64 oracle for GPS L1 C/A acquisition -- TEST INFRASTRUCTURE ONLY.

Two routes compute the same power grid P[p][k][tau]:

* ``grid_direct`` / ``cells_direct`` (C, exact integers + FP64): the plain
  definition -- carrier wipe-off, then for every code shift the sum of
  sample-by-sample products (Sec. 3: "point by point multiplications ... and
  sample shift operations"), squared magnitude summed over blocks.
* ``grid_fft`` (numpy/scipy FP64): the folded coherent blocks (exact integers
  from the C library) correlated with the code replica through the
  correlation theorem, a library FFT serving as the correlation step -- the
  frequency-domain correlation of Fig. 2 (FFT of the mixed signal, FFT of the
  code replica, multiply, IFFT).  Used where the direct sum is too slow; it is
  pinned against ``grid_direct`` in the tests.

Detection (``peaks``) and sub-bin refinement (``interpolate``) follow the
coarse Doppler / code-phase outputs of the acquisition channel (Sec. 3,
Fig. 1 and Fig. 2); the paper gives no rule, so the reading adopted is:
column maximum over Doppler rows, argmax with lowest-index tie-breaks, second
peak outside +-1 chip (circular), ratio test, 3-point parabolas.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

REAL_I8 = 0
CPLX_I8 = 1
REAL_2BIT_PACKED = 2

CHIP_RATE_HZ = 1023000
CODE_LEN = 1023
POWER_SCALE = 2.0 ** -24  # (LUT amplitude 4096)^-2

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        i32, i64, dbl, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
        vp = ctypes.c_void_p
        lib.orc_ca_code.argtypes = [ctypes.c_int, vp]
        lib.orc_code_replica.argtypes = [ctypes.c_int, i64, i64, i64, vp]
        lib.orc_lut.argtypes = [vp, vp]
        lib.orc_lut.restype = None
        lib.orc_bin_freq.argtypes = [dbl, dbl, ctypes.c_int]
        lib.orc_bin_freq.restype = dbl
        lib.orc_nco_step.argtypes = [dbl, dbl, dbl]
        lib.orc_nco_step.restype = u32
        lib.orc_wipe.argtypes = [vp, ctypes.c_int, i64, u32, i64, i64, vp]
        lib.orc_wipe_fold.argtypes = [vp, ctypes.c_int, i64, i64, dbl, dbl, dbl,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
        lib.orc_grid_direct.argtypes = [vp, ctypes.c_int, i64, i64, dbl, vp, ctypes.c_int,
                                        dbl, dbl, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        vp, ctypes.c_int, ctypes.c_int]
        lib.orc_cells_direct.argtypes = [vp, ctypes.c_int, i64, i64, dbl, vp, ctypes.c_int,
                                         dbl, dbl, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         vp, i64, vp, ctypes.c_int, ctypes.c_int]
        lib.orc_code_shift.argtypes = [i64, ctypes.c_int, i64, dbl]
        lib.orc_code_shift.restype = i64
        lib.orc_track.argtypes = [vp, ctypes.c_int, i64, ctypes.c_int, vp, vp, vp, vp, vp, vp, i64,
                                  i64, ctypes.c_int, vp, ctypes.c_int]
        for f in (lib.orc_ca_code, lib.orc_code_replica, lib.orc_wipe, lib.orc_wipe_fold,
                  lib.orc_grid_direct, lib.orc_cells_direct, lib.orc_track):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError("oracle %s failed with code %d" % (what, rc))


def n_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# ---------------------------------------------------------------------------
# Replicas and NCO (Sec. 3, Fig. 2: code NCO and carrier NCO)
# ---------------------------------------------------------------------------

def ca_code(prn: int) -> np.ndarray:
    """One period of the C/A code of ``prn`` as 0/1 chips (IS-GPS-200 Table 3-Ia,
    tap-pair form)."""
    out = np.zeros(CODE_LEN, np.uint8)
    _check(_load().orc_ca_code(int(prn), _ptr(out)), "ca_code")
    return out


def code_replica(prn: int, fs_hz: int, n: int, n0: int = 0) -> np.ndarray:
    """Code-NCO replica c[n0..n0+n) = 1 - 2*code[floor(n*1023000/fs) mod 1023] (int8)."""
    out = np.zeros(int(n), np.int8)
    _check(_load().orc_code_replica(int(prn), int(fs_hz), int(n0), int(n), _ptr(out)),
           "code_replica")
    return out


def lut():
    """Carrier LUT: (cosL, sinL) int16[1024], lround(4096 cos/sin(2 pi i/1024))."""
    c = np.zeros(1024, np.int16)
    s = np.zeros(1024, np.int16)
    _load().orc_lut(_ptr(c), _ptr(s))
    return c, s


def bin_freq(lo: float, step: float, k: int) -> float:
    return float(_load().orc_bin_freq(float(lo), float(step), int(k)))


def nco_step(f_if: float, f_bin: float, fs: float) -> int:
    """32-bit carrier NCO step: (uint32)(int64) llround((f_if + f_bin) * 2^32 / fs)."""
    return int(_load().orc_nco_step(float(f_if), float(f_bin), float(fs)))


def n_doppler(lo: float, hi: float, step: float) -> int:
    """Number of Doppler bins, both ends inclusive: floor((hi-lo)/step + 1e-9) + 1."""
    return int(math.floor((hi - lo) / step + 1e-9)) + 1


def samples_per_ms(fs_hz: int) -> int:
    return int(fs_hz) // 1000


def n_samples_of(samples: np.ndarray, fmt: int) -> int:
    if fmt == REAL_I8:
        return samples.size
    if fmt == CPLX_I8:
        return samples.size // 2
    return samples.size * 4


def wipe(samples: np.ndarray, fmt: int, step_D: int, n0: int, count: int) -> np.ndarray:
    """Mixed samples y[n] = x[n] (cosL[phi>>22] - j sinL[phi>>22]), phi = n*D mod 2^32.
    Returns int64 [count][2] (first mixing stage of Fig. 2)."""
    s = np.ascontiguousarray(samples)
    out = np.zeros((int(count), 2), np.int64)
    _check(_load().orc_wipe(_ptr(s), int(fmt), n_samples_of(s, fmt), ctypes.c_uint32(step_D),
                            int(n0), int(count), _ptr(out)), "wipe")
    return out


def wipe_fold(samples, fmt, fs_hz, f_if, lo, step, n_dopp, T_coh, N_noncoh) -> np.ndarray:
    """Folded coherent blocks f[k][b][m] = sum_{t<Tc} y_k[(b Tc + t) N + m], int64
    [n_dopp][N_noncoh][N][2] (block processing, Sec. 4)."""
    s = np.ascontiguousarray(samples)
    N = samples_per_ms(fs_hz)
    out = np.zeros((n_dopp, N_noncoh, N, 2), np.int64)
    _check(_load().orc_wipe_fold(_ptr(s), int(fmt), n_samples_of(s, fmt), int(fs_hz),
                                 float(f_if), float(lo), float(step), int(n_dopp), int(T_coh),
                                 int(N_noncoh), _ptr(out)), "wipe_fold")
    return out


def raw_samples(samples: np.ndarray, fmt: int, n0: int, count: int) -> np.ndarray:
    """Decoded samples x[n0 .. n0 + count) as complex128 (the mixing stage at
    carrier step 0: LUT entry 0 is 4096 + 0j)."""
    y = wipe(samples, fmt, 0, n0, count)
    return (y[:, 0] + 1j * y[:, 1]) / 4096.0


def fold_exact(samples, fmt, fs_hz, f_if, lo, step, n_dopp, T_coh, N_noncoh) -> np.ndarray:
    """Folded coherent blocks with an exact carrier: y[n] = x[b L + n]
    exp(-2 pi i (f_if + f_k) n / fs) for n < L = T_coh N (phase zero at the block
    start, which leaves every |R_b|^2 unchanged), f[k][b][j] = sum_{t<Tc} y[j + t N].
    complex128 [n_dopp][N_noncoh][N] -- the carrier of the frequency-domain
    Doppler variant, which removes it by shifting a spectrum instead of by the
    NCO's lookup table."""
    N = samples_per_ms(fs_hz)
    L = T_coh * N
    n = np.arange(L, dtype=np.float64)
    out = np.zeros((n_dopp, N_noncoh, N), np.complex128)
    for b in range(N_noncoh):
        x = raw_samples(samples, fmt, b * L, L)
        for k in range(n_dopp):
            ph = (f_if + bin_freq(lo, step, k)) * n / fs_hz  # cycles
            ph -= np.floor(ph)
            y = x * np.exp(-2j * np.pi * ph)
            out[k, b] = y.reshape(T_coh, N).sum(axis=0)
    return out


# ---------------------------------------------------------------------------
# Correlation grid
# ---------------------------------------------------------------------------

def grid_direct(samples, fmt, fs_hz, f_if, prns, lo, step, n_dopp, T_coh, N_noncoh,
                threads: int | None = None, code_doppler: bool = False) -> np.ndarray:
    """P[p][k][tau] by direct time-domain circular correlation (FP64 float64 array);
    code_doppler: each block's lag shifted by code_shift (the compensated sum)."""
    s = np.ascontiguousarray(samples)
    prn_arr = np.ascontiguousarray(np.asarray(prns, np.int32))
    N = samples_per_ms(fs_hz)
    P = np.zeros((prn_arr.size, n_dopp, N), np.float64)
    _check(_load().orc_grid_direct(_ptr(s), int(fmt), n_samples_of(s, fmt), int(fs_hz),
                                   float(f_if), _ptr(prn_arr), prn_arr.size, float(lo),
                                   float(step), int(n_dopp), int(T_coh), int(N_noncoh),
                                   _ptr(P), int(threads or n_threads()), int(bool(code_doppler))),
           "grid_direct")
    return P


def cells_direct(samples, fmt, fs_hz, f_if, prns, lo, step, n_dopp, T_coh, N_noncoh, cells,
                 threads: int | None = None, code_doppler: bool = False) -> np.ndarray:
    """P at selected cells (rows of (prn index, k, tau)) by direct correlation."""
    s = np.ascontiguousarray(samples)
    prn_arr = np.ascontiguousarray(np.asarray(prns, np.int32))
    cl = np.ascontiguousarray(np.asarray(cells, np.int32).reshape(-1, 3))
    out = np.zeros(cl.shape[0], np.float64)
    _check(_load().orc_cells_direct(_ptr(s), int(fmt), n_samples_of(s, fmt), int(fs_hz),
                                    float(f_if), _ptr(prn_arr), prn_arr.size, float(lo),
                                    float(step), int(n_dopp), int(T_coh), int(N_noncoh),
                                    _ptr(cl), cl.shape[0], _ptr(out),
                                    int(threads or n_threads()), int(bool(code_doppler))), "cells_direct")
    return out


def code_shift(b: int, T_coh: int, N: int, f_bin: float) -> int:
    """Samples by which block b's correlation peak at Doppler f_bin sits
    earlier than block 0's (code-Doppler compensation reading)."""
    return int(_load().orc_code_shift(int(b), int(T_coh), int(N), float(f_bin)))


def grid_fft(samples, fmt, fs_hz, f_if, prns, lo, step, n_dopp, T_coh, N_noncoh,
             folded: np.ndarray | None = None, code_doppler: bool = False,
             carrier: str = "nco", nav_pairs: bool = False) -> np.ndarray:
    """P[p][k][tau] through the correlation theorem in FP64:
    R_b = IDFT_N( DFT_N(f_b) * conj(DFT_N(c)) ), P = sum_b |R_b|^2 2^-24.
    The folded blocks are exact integers, so the only error is FP64 FFT rounding.
    code_doppler: P[tau] = sum_b |R_b[(tau - delta_b(k)) mod N]|^2 2^-24.
    carrier="exact": the blocks of fold_exact (unit-modulus carrier, so no
    2^-24 scale), P = sum_b |R_b|^2.
    nav_pairs: navigation-bit hypotheses -- blocks 2i and 2i+1 combined with
    both relative signs, P = sum_i max(|R_2i + R_2i+1|^2, |R_2i - R_2i+1|^2)
    (after the code-Doppler lag shifts, if any); N_noncoh must be even."""
    import scipy.fft as sfft

    N = samples_per_ms(fs_hz)
    scale = POWER_SCALE
    if carrier == "exact":
        f = fold_exact(samples, fmt, fs_hz, f_if, lo, step, n_dopp, T_coh, N_noncoh)
        scale = 1.0
    else:
        if folded is None:
            folded = wipe_fold(samples, fmt, fs_hz, f_if, lo, step, n_dopp, T_coh, N_noncoh)
        f = folded[..., 0].astype(np.float64) + 1j * folded[..., 1].astype(np.float64)
    F = sfft.fft(f, axis=-1, workers=n_threads())
    del f
    P = np.zeros((len(prns), n_dopp, N), np.float64)
    for pi, prn in enumerate(prns):
        C = np.conj(sfft.fft(code_replica(prn, fs_hz, N).astype(np.float64)))
        R = sfft.ifft(F * C, axis=-1, workers=n_threads())
        if nav_pairs:
            if N_noncoh % 2:
                raise ValueError("nav_pairs needs an even N_noncoh")
            acc = np.zeros((n_dopp, N), np.float64)
            for k in range(n_dopp):
                shifts = [code_shift(b, T_coh, N, bin_freq(lo, step, k)) if code_doppler else 0
                          for b in range(N_noncoh)]
                for i in range(N_noncoh // 2):  # pairs summed in ascending order
                    ra = np.roll(R[k, 2 * i], shifts[2 * i])
                    rb = np.roll(R[k, 2 * i + 1], shifts[2 * i + 1])
                    plus, minus = ra + rb, ra - rb
                    acc[k] += np.maximum(plus.real ** 2 + plus.imag ** 2, minus.real ** 2 + minus.imag ** 2) * scale
            P[pi] = acc
            del R
            continue
        pw = (R.real * R.real + R.imag * R.imag) * scale
        acc = np.zeros((n_dopp, N), np.float64)
        for b in range(N_noncoh):  # blocks summed in ascending order
            if code_doppler:
                for k in range(n_dopp):
                    acc[k] += np.roll(pw[k, b, :], code_shift(b, T_coh, N, bin_freq(lo, step, k)))
            else:
                acc += pw[:, b, :]
        P[pi] = acc
        del R, pw
    return P


# ---------------------------------------------------------------------------
# Detection and refinement
# ---------------------------------------------------------------------------

@dataclass
class Peak:
    prn: int
    doppler_bin: int
    code_phase: int
    detected: bool
    peak: float
    second: float
    mean: float
    ratio: float
    doppler_hz: float
    code_phase_frac: float


def circular_distance(a: np.ndarray, b: int, N: int) -> np.ndarray:
    d = np.abs(a - b) % N
    return np.minimum(d, N - d)


def parabola_offset(y_minus: float, y0: float, y_plus: float) -> float:
    """Vertex offset of the parabola through (-1, y-), (0, y0), (+1, y+):
    delta = (y- - y+) / (2 (y- - 2 y0 + y+)); 0 when the three are collinear."""
    den = y_minus - 2.0 * y0 + y_plus
    if den == 0.0:
        return 0.0
    return 0.5 * (y_minus - y_plus) / den


def peak_one(G: np.ndarray, prn: int, spc: int, threshold: float, lo: float,
             step: float) -> Peak:
    """Detection on one PRN's grid G[k][tau] (float64).

    Q[tau] = max_k G (lowest k on ties); tau* = argmax Q (lowest tau on ties);
    k* = row of that maximum; second = max Q over circular |tau - tau*| > spc;
    mean = mean of G; ratio = peak / second; detected = ratio >= threshold.
    Refinement: 3-point parabolas along the lag (circular) and Doppler axes (no
    Doppler refinement at the first or last bin)."""
    n_dopp, N = G.shape
    # numpy's argmax returns the first maximal index: lowest k, then lowest tau.
    K = np.argmax(G, axis=0)
    Q = G[K, np.arange(N)]
    tau_star = int(np.argmax(Q))
    k_star = int(K[tau_star])
    peak = float(Q[tau_star])
    far = circular_distance(np.arange(N), tau_star, N) > spc
    second = float(Q[far].max()) if far.any() else 0.0
    mean = float(G.sum(dtype=np.float64) / (n_dopp * N))
    ratio = peak / second if second > 0.0 else math.inf
    dc = parabola_offset(float(G[k_star, (tau_star - 1) % N]), peak,
                         float(G[k_star, (tau_star + 1) % N]))
    if 0 < k_star < n_dopp - 1:
        dd = parabola_offset(float(G[k_star - 1, tau_star]), peak, float(G[k_star + 1, tau_star]))
    else:
        dd = 0.0
    f_k = lo + k_star * step
    return Peak(prn=int(prn), doppler_bin=k_star, code_phase=int(tau_star),
                detected=bool(ratio >= threshold), peak=peak, second=second, mean=mean,
                ratio=ratio, doppler_hz=f_k + dd * step, code_phase_frac=tau_star + dc)


def peaks(P: np.ndarray, prns, spc: int, threshold: float, lo: float, step: float):
    """``peak_one`` for every PRN of a grid P[p][k][tau]."""
    return [peak_one(np.asarray(P[i], np.float64), prns[i], spc, threshold, lo, step)
            for i in range(len(prns))]


def samples_per_chip(fs_hz: int) -> int:
    """Integer samples per chip (fs must be a multiple of 1.023 MHz)."""
    if fs_hz % CHIP_RATE_HZ:
        raise ValueError("fs is not a multiple of the chip rate")
    return int(fs_hz) // CHIP_RATE_HZ


def chip_exclusion(fs_hz: int) -> float:
    """Half-width of the second-peak exclusion: one chip, fs / 1.023 MHz
    samples, at any rate (the lags with circular |tau - tau*| > this are
    candidates; at k * 1.023 MHz it is the integer k)."""
    return int(fs_hz) / CHIP_RATE_HZ


# ---------------------------------------------------------------------------
# tracking correlators (Fig. 3)
# ---------------------------------------------------------------------------

@dataclass
class Channel:
    """One tracking channel in physical units."""
    prn: int
    carrier_hz: float          # carrier to remove: IF + Doppler
    carrier_phase: float       # cycles at sample 0, [0, 1)
    code_phase: float          # chips at sample 0, [0, 1023)
    code_rate: float           # chips per second
    spacing: float            # early-late offset, chips, (0, 1]


def track_fixed(ch: Channel, fs_hz: int):
    """Fixed-point NCO words of a channel: (D, phi0, q0, R, dl).  Each is the
    value times 2^32 rounded half away from zero (llround), computed in IEEE
    double as written: carrier step from carrier_hz * 2^32 / fs."""
    D = int(np.int64(_llround(ch.carrier_hz * 4294967296.0 / float(fs_hz)))) & 0xFFFFFFFF
    phi0 = int(np.int64(_llround(ch.carrier_phase * 4294967296.0))) & 0xFFFFFFFF
    q0 = _llround(ch.code_phase * 4294967296.0)
    R = _llround(ch.code_rate * 4294967296.0 / float(fs_hz))
    dl = _llround(ch.spacing * 4294967296.0)
    return D, phi0, q0, R, dl


def _llround(x: float) -> int:
    return int(math.floor(x + 0.5)) if x >= 0 else -int(math.floor(-x + 0.5))


def track(samples, fmt, fs_hz, channels, start, length, n_epochs, threads: int | None = None):
    """Early/prompt/late correlators, int64 [n_ch][n_epochs][3][2] (re, im)."""
    s = np.ascontiguousarray(samples)
    words = [track_fixed(c, fs_hz) for c in channels]
    prn = np.ascontiguousarray([c.prn for c in channels], np.int32)
    D = np.ascontiguousarray([w[0] for w in words], np.uint32)
    phi0 = np.ascontiguousarray([w[1] for w in words], np.uint32)
    q0 = np.ascontiguousarray([w[2] for w in words], np.int64)
    R = np.ascontiguousarray([w[3] for w in words], np.int64)
    dl = np.ascontiguousarray([w[4] for w in words], np.int64)
    out = np.zeros((len(channels), n_epochs, 3, 2), np.int64)
    _check(_load().orc_track(_ptr(s), int(fmt), n_samples_of(s, fmt), len(channels), _ptr(prn),
                             _ptr(D), _ptr(phi0), _ptr(q0), _ptr(R), _ptr(dl), int(start),
                             int(length), int(n_epochs), _ptr(out), int(threads or n_threads())),
           "track")
    return out

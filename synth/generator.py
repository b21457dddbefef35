"""Seeded synthetic IF / baseband snapshots with planted GPS L1 C/A satellites.

The paper measured one recorded 12-channel client file (Sec. 4) that is not
available; these generators stand in for it with the shapes, sample formats
and signal levels of the acquisition workloads:

* real IF, 2-bit {+-1, +-3} samples (front-end style), or
* complex int8 baseband,

each carrying a few planted satellites (C/A code at an integer code phase, a
Doppler offset, a carrier phase, optional 20 ms navigation-bit flips) in white
Gaussian noise at a stated C/N0.

Signal levels: real IF with noise sigma has A = sigma*sqrt(4*CN0/fs); complex
baseband with sigma per component has A = sigma*sqrt(2*CN0/fs) (CN0 linear).
Quantisers: 2-bit sign*(|v| < T ? 1 : 3) with T = std(v), v = 0 -> +1;
int8 rint(v*16/sigma) clipped to [-127, 127].

Callers pass ``code_fn(prn) -> uint8[1023]`` (0/1 chips) for planted PRNs.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

REAL_I8 = 0
CPLX_I8 = 1
REAL_2BIT_PACKED = 2

CHIP_RATE = 1023000


@dataclass
class Planted:
    prn: int
    code_phase: int          # sample at which chip 0 starts (integer)
    doppler_hz: float
    cn0_dbhz: float
    carrier_phase: float = 0.0
    nav_bits: bool = False
    nav_phase_ms: int = 0
    amplitude: float = 0.0   # filled in by the generator


@dataclass
class Snapshot:
    samples: np.ndarray       # int8 (REAL_I8), int8 interleaved (CPLX_I8) or uint8 (packed)
    fmt: int
    fs_hz: int
    f_if_hz: float
    n: int                    # samples (not bytes)
    planted: list = field(default_factory=list)
    seed: int = 0


L1_HZ = 1575420000.0


def _code_wave(chips: np.ndarray, fs_hz: int, n: np.ndarray, code_phase: int,
               doppler_hz: float = 0.0, code_doppler: bool = False) -> np.ndarray:
    """+-1 code waveform at sample indices n for a code whose chip 0 starts at
    sample code_phase.  Code rate 1.023 MHz, or with code_doppler the received
    rate 1.023 MHz * (1 + doppler / f_L1) (chip 0 still at code_phase)."""
    rel = n.astype(np.int64) - int(code_phase)
    if code_doppler and doppler_hz != 0.0:
        rate = CHIP_RATE * (1.0 + doppler_hz / L1_HZ)
        chip = np.floor(rel.astype(np.float64) * (rate / float(fs_hz))).astype(np.int64) % 1023
    else:
        chip = np.floor_divide(rel * CHIP_RATE, int(fs_hz)) % 1023
    return 1.0 - 2.0 * chips[chip].astype(np.float64)


def _nav_wave(rng: np.random.Generator, fs_hz: int, n: np.ndarray, p: Planted) -> np.ndarray:
    N = fs_hz // 1000
    rel = n.astype(np.int64) - int(p.code_phase) - int(p.nav_phase_ms) * N
    bit_idx = np.floor_divide(rel, 20 * N)
    lo, hi = int(bit_idx.min()), int(bit_idx.max())
    bits = rng.choice(np.array([-1.0, 1.0]), size=hi - lo + 1)
    return bits[bit_idx - lo]


def quantise_2bit(v: np.ndarray) -> np.ndarray:
    T = float(np.std(v))
    mag = np.where(np.abs(v) < T, 1, 3)
    sgn = np.where(v < 0, -1, 1)
    return (sgn * mag).astype(np.int8)


def quantise_int8(v: np.ndarray, sigma: float) -> np.ndarray:
    return np.clip(np.rint(v * 16.0 / sigma), -127, 127).astype(np.int8)


def pack_2bit(q: np.ndarray) -> np.ndarray:
    """Pack {+1,+3,-1,-3} samples 4 per byte, first sample in the low bits:
    00:+1 01:+3 10:-1 11:-3.  Length is padded with +1 to a multiple of 4."""
    code = np.select([q == 1, q == 3, q == -1, q == -3], [0, 1, 2, 3], 0).astype(np.uint8)
    pad = (-code.size) % 4
    if pad:
        code = np.concatenate([code, np.zeros(pad, np.uint8)])
    c = code.reshape(-1, 4)
    return (c[:, 0] | (c[:, 1] << 2) | (c[:, 2] << 4) | (c[:, 3] << 6)).astype(np.uint8)


def unpack_2bit(b: np.ndarray, n: int) -> np.ndarray:
    val = np.array([1, 3, -1, -3], np.int8)
    codes = np.stack([(b >> (2 * i)) & 3 for i in range(4)], axis=1).reshape(-1)
    return val[codes[:n]]


def make_snapshot(seed: int, fmt: int, fs_hz: int, f_if_hz: float, duration_ms: float,
                  planted: list, code_fn, noise_sigma: float = 1.0, noise: bool = True,
                  chunk: int = 1 << 20, code_doppler: bool = False) -> Snapshot:
    """Generate one snapshot.  ``planted`` is a list of ``Planted``; their
    amplitudes are set from C/N0 and written back.  code_doppler: the code
    rate of each planted satellite follows its Doppler (off by default)."""
    rng = np.random.default_rng(seed)
    n_total = int(round(fs_hz * duration_ms / 1000.0))
    cplx = fmt == CPLX_I8
    for p in planted:
        cn0 = 10.0 ** (p.cn0_dbhz / 10.0)
        p.amplitude = noise_sigma * np.sqrt((2.0 if cplx else 4.0) * cn0 / fs_hz)
    chips = {p.prn: np.asarray(code_fn(p.prn), np.uint8) for p in planted}
    nav_rngs = [np.random.default_rng([seed, 7, i]) for i in range(len(planted))]
    noise_rng = np.random.default_rng([seed, 11])
    out_re = np.empty(n_total, np.float64)
    out_im = np.empty(n_total, np.float64) if cplx else None
    navs = []
    for i, p in enumerate(planted):
        navs.append(_nav_wave(nav_rngs[i], fs_hz, np.arange(n_total), p) if p.nav_bits else None)
    for s0 in range(0, n_total, chunk):
        n = np.arange(s0, min(n_total, s0 + chunk), dtype=np.int64)
        re = np.zeros(n.size)
        im = np.zeros(n.size) if cplx else None
        for i, p in enumerate(planted):
            w = p.amplitude * _code_wave(chips[p.prn], fs_hz, n, p.code_phase, p.doppler_hz, code_doppler)
            if navs[i] is not None:
                w = w * navs[i][n]
            theta = 2.0 * np.pi * (f_if_hz + p.doppler_hz) * (n / fs_hz) + p.carrier_phase
            if cplx:
                re += w * np.cos(theta)
                im += w * np.sin(theta)
            else:
                re += w * np.cos(theta)
        if noise:
            re += noise_rng.normal(0.0, noise_sigma, n.size)
            if cplx:
                im += noise_rng.normal(0.0, noise_sigma, n.size)
        out_re[n[0]:n[-1] + 1] = re
        if cplx:
            out_im[n[0]:n[-1] + 1] = im
    if cplx:
        q = np.empty(2 * n_total, np.int8)
        q[0::2] = quantise_int8(out_re, noise_sigma)
        q[1::2] = quantise_int8(out_im, noise_sigma)
        samples = q
    else:
        q = quantise_2bit(out_re)
        samples = pack_2bit(q) if fmt == REAL_2BIT_PACKED else q
    return Snapshot(samples=samples, fmt=fmt, fs_hz=int(fs_hz), f_if_hz=float(f_if_hz),
                    n=n_total, planted=list(planted), seed=seed)


# ---------------------------------------------------------------------------
# Workload recipes (acquisition configurations measured by this project)
# ---------------------------------------------------------------------------

@dataclass
class Search:
    prns: list
    lo: float
    hi: float
    step: float
    T_coh: int
    N_noncoh: int


def _draw_planted(rng, n, prn_pool, phase_max, dopp_max, cn0_lo, cn0_hi, nav):
    prns = rng.choice(np.asarray(prn_pool), size=n, replace=False)
    out = []
    for prn in prns:
        out.append(Planted(prn=int(prn), code_phase=int(rng.integers(0, phase_max)),
                           doppler_hz=float(rng.uniform(-dopp_max, dopp_max)),
                           cn0_dbhz=float(rng.uniform(cn0_lo, cn0_hi)),
                           carrier_phase=float(rng.uniform(0.0, 2.0 * np.pi)),
                           nav_bits=nav, nav_phase_ms=int(rng.integers(0, 20))))
    return out


def strong_real_2bit(code_fn, seed: int = 1, fmt: int = REAL_I8):
    """Real 2-bit IF, fs 4.092 MHz, f_IF 1.023 MHz, 10 ms; 4 planted PRNs at 45 dB-Hz,
    Doppler U[-5, 5] kHz; search PRN 1-32, +-5 kHz step 500 Hz, 1 ms x 10."""
    fs = 4092000
    rng = np.random.default_rng([seed, 1])
    planted = _draw_planted(rng, 4, range(1, 33), fs // 1000, 5000.0, 45.0, 45.0, False)
    snap = make_snapshot(seed, fmt, fs, 1023000.0, 10.0, planted, code_fn)
    return snap, Search(list(range(1, 33)), -5000.0, 5000.0, 500.0, 1, 10)


def weak_complex_int8(code_fn, seed: int = 2, fs: int = 16368000):
    """Complex int8 baseband, fs 16.368 MHz (or another rate), 100 ms; 8 planted
    PRNs at C/N0 U[28, 40] dB-Hz, Doppler U[-7.5, 7.5] kHz, 20 ms nav-bit flips;
    search PRN 1-32, +-7.5 kHz step 125 Hz, 4 ms x 25."""
    rng = np.random.default_rng([seed, 2])
    planted = _draw_planted(rng, 8, range(1, 33), fs // 1000, 7500.0, 28.0, 40.0, True)
    snap = make_snapshot(seed, CPLX_I8, fs, 0.0, 100.0, planted, code_fn)
    return snap, Search(list(range(1, 33)), -7500.0, 7500.0, 125.0, 4, 25)


def long_complex_int8(code_fn, seed: int = 3, fs: int = 16368000, blocks: int = 512):
    """Complex int8 baseband, fs 16.368 MHz, 4 ms x `blocks` (2.048 s by
    default); 8 planted PRNs at C/N0 U[22, 30] dB-Hz, weaker than a 100 ms
    record can show, Doppler U[-7.5, 7.5] kHz, 20 ms nav-bit flips; search
    PRN 1-32, +-7.5 kHz step 125 Hz, 4 ms x `blocks`."""
    rng = np.random.default_rng([seed, 5])
    planted = _draw_planted(rng, 8, range(1, 33), fs // 1000, 7500.0, 22.0, 30.0, True)
    snap = make_snapshot(seed, CPLX_I8, fs, 0.0, 4.0 * blocks + 0.5, planted, code_fn)
    return snap, Search(list(range(1, 33)), -7500.0, 7500.0, 125.0, 4, blocks)


def batch_workload(code_fn, seed: int = 4, n: int = 256, ms_range=(20, 200), rates=None,
                   prn_range=(8, 32), window_khz=(2.0, 10.0), planted_range=(1, 6),
                   cn0_range=(30.0, 45.0), workers: int = 1):
    """Heterogeneous snapshots for batched search: lengths U{20..200} ms, fs
    uniform over {4.092, 8.184, 16.368} MHz, format uniform over real 2-bit
    (f_IF = fs/4) and complex int8 (f_IF = 0), PRN subsets of U{8..32} PRNs
    from 1-32, Doppler window +-W with W ~ U[2, 10] kHz snapped to 500 Hz,
    1-6 planted PRNs inside the subset at C/N0 U[30, 45] dB-Hz with Doppler
    inside the window; searched with 1 ms coherent x L non-coherent blocks,
    500 Hz bins.  Returns a list of (Snapshot, Search).  workers > 1 generates
    the snapshots on that many threads (the same snapshots: every one is drawn
    from its own seed)."""
    rates = rates or [4092000, 8184000, 16368000]
    rng = np.random.default_rng([seed, 4])
    jobs = []
    for i in range(n):
        L = int(rng.integers(ms_range[0], ms_range[1] + 1))
        fs = int(rates[int(rng.integers(0, len(rates)))])
        cplx = bool(rng.integers(0, 2))
        fmt = CPLX_I8 if cplx else REAL_I8
        f_if = 0.0 if cplx else fs / 4.0
        n_prn = int(rng.integers(prn_range[0], prn_range[1] + 1))
        prns = sorted(int(p) for p in rng.choice(np.arange(1, 33), size=n_prn, replace=False))
        W = float(np.round(rng.uniform(*window_khz) * 2.0) / 2.0 * 1000.0)
        n_pl = int(rng.integers(planted_range[0], min(planted_range[1], n_prn) + 1))
        pl_prns = rng.choice(np.asarray(prns), size=n_pl, replace=False)
        planted = [Planted(prn=int(p), code_phase=int(rng.integers(0, fs // 1000)),
                           doppler_hz=float(rng.uniform(-0.9 * W, 0.9 * W)),
                           cn0_dbhz=float(rng.uniform(*cn0_range)),
                           carrier_phase=float(rng.uniform(0.0, 2.0 * np.pi)))
                   for p in pl_prns]
        jobs.append(((int(rng.integers(0, 2 ** 31)), fmt, fs, f_if, float(L), planted),
                     Search(prns, -W, W, 500.0, 1, L)))
    if workers <= 1:
        return [(make_snapshot(*a, code_fn), srch) for a, srch in jobs]
    from concurrent.futures import ThreadPoolExecutor

    chips = {p: np.asarray(code_fn(p), np.uint8) for p in range(1, 33)}  # code_fn stays on this thread
    with ThreadPoolExecutor(max_workers=workers) as ex:
        snaps = list(ex.map(lambda a: make_snapshot(*a, chips.__getitem__), [a for a, _ in jobs]))
    return [(snap, srch) for snap, (_, srch) in zip(snaps, jobs)]

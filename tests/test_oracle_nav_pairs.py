"""Pins of the oracle's navigation-bit hypotheses (blocks combined in pairs,
max over the relative sign): brute force on tiny inputs and the closed form
of noiseless code with a bit flip between the two blocks of a pair."""
import numpy as np
import pytest

import oracle as O


def _brute_pairs(x, fs, prn, Tc, Nnc):
    # the definition at 0 Hz, complex samples: R_b[tau] = sum_n y_b[n] c[(n - tau) mod N]
    # with y = 4096 x (the NCO at step 0), P = sum_i max_h |R_2i + h R_2i+1|^2 2^-24
    N = fs // 1000
    L = Tc * N
    c = O.code_replica(prn, fs, N).astype(np.float64)
    n = np.arange(L)
    P = np.zeros(N)
    for i in range(Nnc // 2):
        Rs = []
        for b in (2 * i, 2 * i + 1):
            y = 4096.0 * O.raw_samples(x, O.CPLX_I8, b * L, L)
            Rs.append(np.array([np.sum(y * c[(n - tau) % N]) for tau in range(N)]))
        P += np.maximum(np.abs(Rs[0] + Rs[1]) ** 2, np.abs(Rs[0] - Rs[1]) ** 2) * 2.0 ** -24
    return P


def test_pairs_match_brute_force():
    fs, Tc, Nnc = 1023000, 2, 4
    rng = np.random.default_rng(8)
    n = Tc * Nnc * (fs // 1000) + 3
    x = rng.integers(-30, 31, 2 * n).astype(np.int8)
    P1 = O.grid_fft(x, O.CPLX_I8, fs, 0.0, [6], 0.0, 500.0, 1, Tc, Nnc, nav_pairs=True)[0, 0]
    P2 = _brute_pairs(x, fs, 6, Tc, Nnc)
    assert np.max(np.abs(P1 - P2) / (P2 + P2.mean())) < 1e-11


def test_bit_flip_between_the_blocks_of_a_pair():
    # x = A c[(n - d) mod N] for block 0, -A c[...] for block 1 (0 Hz): the pair's
    # minus hypothesis adds them coherently, (2 L A)^2; the plain sum is 2 (L A)^2
    fs, Tc, prn, d, A = 2046000, 3, 13, 777, 9
    N = fs // 1000
    L = Tc * N
    rep = O.code_replica(prn, fs, N).astype(np.int64)
    sig = np.concatenate([np.tile(np.roll(rep, d), Tc) * A, -np.tile(np.roll(rep, d), Tc) * A])
    x = np.zeros(2 * sig.size, np.int8)
    x[0::2] = sig.astype(np.int8)
    Pp = O.grid_fft(x, O.CPLX_I8, fs, 0.0, [prn], 0.0, 1.0, 1, Tc, 2, nav_pairs=True)[0, 0]
    Ps = O.grid_fft(x, O.CPLX_I8, fs, 0.0, [prn], 0.0, 1.0, 1, Tc, 2)[0, 0]
    assert int(np.argmax(Pp)) == d
    assert abs(Pp[d] / (2 * L * A) ** 2 - 1.0) < 1e-12
    assert abs(Ps[d] / (2 * (L * A) ** 2) - 1.0) < 1e-12


def test_pairs_need_an_even_block_count():
    x = np.zeros(2 * 3 * 1023, np.int8)
    with pytest.raises(ValueError):
        O.grid_fft(x, O.CPLX_I8, 1023000, 0.0, [1], 0.0, 500.0, 1, 1, 3, nav_pairs=True)

"""Pins for the oracle's detection rule and sub-bin refinement.

The paper says acquisition outputs coarse Doppler and code phase, refined
later (Sec. 3); it states no rule.  The reading adopted is pinned here on
hand-built grids whose answers are known by construction: ties, the circular
+-1 chip exclusion zone, mean, ratio, and parabolas that are exact on
quadratics.
"""
import math

import numpy as np

import oracle as O


def test_tie_breaks_lowest_doppler_then_lowest_lag():
    G = np.zeros((4, 50))
    G[2, 10] = 5.0
    G[1, 10] = 5.0   # same value, lower k
    G[3, 30] = 5.0   # same value, higher tau
    r = O.peak_one(G, 1, 2, 2.5, -100.0, 50.0)
    assert (r.doppler_bin, r.code_phase) == (1, 10)
    assert r.second == 5.0 and r.ratio == 1.0 and not r.detected


def test_second_peak_excludes_one_chip_circularly():
    N, spc = 40, 3
    G = np.full((3, N), 1.0)
    G[1, 1] = 100.0
    G[0, N - 2] = 90.0      # circular distance 3 = spc -> excluded
    G[2, 4] = 80.0          # distance 3 -> excluded
    G[2, 5] = 20.0          # distance 4 -> counts
    r = O.peak_one(G, 7, spc, 2.5, 0.0, 1.0)
    assert (r.doppler_bin, r.code_phase) == (1, 1)
    assert r.second == 20.0
    assert r.ratio == 5.0 and r.detected
    assert math.isclose(r.mean, G.mean(), rel_tol=0, abs_tol=1e-12)


def test_threshold_is_inclusive():
    G = np.ones((1, 20))
    G[0, 10] = 2.5
    assert O.peak_one(G, 1, 1, 2.5, 0.0, 1.0).detected
    G[0, 10] = 2.4999
    assert not O.peak_one(G, 1, 1, 2.5, 0.0, 1.0).detected


def test_parabola_exact_on_quadratics():
    for x0 in (-0.49, -0.2, 0.0, 0.3, 0.45):
        y = [-(x - x0) ** 2 + 10.0 for x in (-1.0, 0.0, 1.0)]
        assert abs(O.parabola_offset(*y) - x0) < 1e-12
    assert O.parabola_offset(1.0, 1.0, 1.0) == 0.0


def test_refinement_on_quadratic_grid():
    n_dopp, N = 9, 64
    kc, tc = 4.3, 20.25
    k = np.arange(n_dopp)[:, None]
    t = np.arange(N)[None, :]
    G = 1000.0 - 3.0 * (k - kc) ** 2 - 2.0 * (t - tc) ** 2
    G = np.maximum(G, 0.0)
    r = O.peak_one(G, 2, 1, 2.5, -400.0, 100.0)
    assert (r.doppler_bin, r.code_phase) == (4, 20)
    assert abs(r.code_phase_frac - tc) < 1e-9
    assert abs(r.doppler_hz - (-400.0 + kc * 100.0)) < 1e-7


def test_no_doppler_refinement_at_edges_and_circular_lag():
    G = np.ones((3, 16))
    G[0, 0] = 10.0
    G[0, 15] = 6.0
    G[0, 1] = 4.0
    G[1, 0] = 9.0
    r = O.peak_one(G, 3, 1, 2.5, 250.0, 50.0)
    assert r.doppler_bin == 0 and r.doppler_hz == 250.0
    assert abs(r.code_phase_frac - O.parabola_offset(6.0, 10.0, 4.0)) < 1e-12

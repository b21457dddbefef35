"""Parity helpers shared by the GPU tests (no GPU or oracle code here).

Tolerance on FP32 correlation power (per request and PRN grid):
    |P_gpu - P_ref| <= 1e-4 * (P_ref + mean(P_ref))
A pure per-cell relative test would fail on noiseless inputs, where off-peak
cells are tiny exact integers; FP32 FFT rounding is relative to the norm of
the whole transform, which the grid mean stands in for.

Detections must be identical (detected flag, Doppler bin, code phase) unless
the oracle's decision is a near tie, and then the GPU's answer must still be
one the oracle's grid allows:
  * a different cell only if that cell's oracle power is within tie_rel of the
    oracle's maximum (and the detected flag agrees, unless the oracle's ratio
    is itself within tie_rel of the threshold);
  * the same cell with a different detected flag only if the oracle's ratio
    is within tie_rel of the threshold.
"""
import sys

import numpy as np

GRID_TOL = 1e-4
TIE_REL = 2e-4


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def grid_error(P_gpu: np.ndarray, P_ref: np.ndarray) -> float:
    worst = 0.0
    for i in range(P_ref.shape[0]):
        ref = np.asarray(P_ref[i], np.float64)
        g = np.asarray(P_gpu[i], np.float64)
        err = np.abs(g - ref) / (ref + ref.mean())
        worst = max(worst, float(err.max()))
    return worst


def assert_grid_close(P_gpu, P_ref, tol: float = GRID_TOL) -> float:
    assert P_gpu.shape == P_ref.shape, (P_gpu.shape, P_ref.shape)
    assert np.all(np.isfinite(P_gpu))
    worst = grid_error(P_gpu, P_ref)
    assert worst <= tol, "max mixed-relative power error %.3e > %.1e" % (worst, tol)
    return worst


def compare_detections(gpu_peaks, ref_peaks, P_ref, threshold: float = 2.5, tie_rel: float = TIE_REL,
                       value_rel: float = 1e-4):
    """Returns the number of near-tie exemptions; raises on a real mismatch.
    tie_rel: relative width of a near tie; value_rel: tolerance on the peak
    and mean values."""
    exempt = 0
    for i, r in enumerate(ref_peaks):
        g = gpu_peaks[i]
        assert int(g["prn"]) == r.prn
        Pi = np.asarray(P_ref[i], np.float64)
        gk, gt = int(g["doppler_bin"]), int(g["code_phase"])
        assert 0 <= gk < Pi.shape[0] and 0 <= gt < Pi.shape[1], (r.prn, gk, gt)
        same_cell = gk == r.doppler_bin and gt == r.code_phase
        same_det = bool(g["detected"]) == r.detected
        if same_cell:
            assert abs(float(g["peak"]) - r.peak) <= value_rel * r.peak, (r.prn, g["peak"], r.peak)
        assert abs(float(g["mean"]) - r.mean) <= value_rel * r.mean, (r.prn, g["mean"], r.mean)
        if same_cell and same_det:
            continue
        near_thr = abs(r.ratio - threshold) <= tie_rel * threshold
        if same_cell:
            ok = near_thr  # only the ratio decision differs
        else:
            near_cell = Pi[gk, gt] >= (1.0 - tie_rel) * Pi.max()
            ok = near_cell and (same_det or near_thr)
        if ok:
            exempt += 1
            continue
        raise AssertionError("PRN %d: gpu (det %d, k %d, tau %d, oracle power there %.6g) vs oracle "
                             "(det %d, k %d, tau %d, peak %.6g), ratio %.6f"
                             % (r.prn, g["detected"], gk, gt, Pi[gk, gt], r.detected, r.doppler_bin,
                                r.code_phase, r.peak, r.ratio))
    return exempt


def _parabola(ym: float, y0: float, yp: float) -> float:
    den = ym - 2.0 * y0 + yp
    return 0.0 if den == 0.0 else 0.5 * (ym - yp) / den


def _parabola_bound(ym, y0, yp, em, e0, ep):
    """Largest change of the parabola's vertex offset when each of the three
    values moves by at most its bound (the corners of the box; the offset is
    smooth there unless the denominator can vanish, then inf)."""
    den = ym - 2.0 * y0 + yp
    if abs(den) <= em + 2.0 * e0 + ep:
        return np.inf
    d0 = _parabola(ym, y0, yp)
    worst = 0.0
    for sm in (-1, 1):
        for s0 in (-1, 1):
            for sp in (-1, 1):
                worst = max(worst, abs(_parabola(ym + sm * em, y0 + s0 * e0, yp + sp * ep) - d0))
    return 1.5 * worst  # margin for curvature inside the box


def compare_refinement(gpu_peaks, ref_peaks, P_ref, P_gpu, lo: float, step: float, tol: float = GRID_TOL):
    """The detection fields a full search reports beyond (det, k, tau):
    second, ratio and the FP64 refinements.  For every PRN whose cell matches
    the oracle's:
      * second within tol (second + mean) of the oracle's (the bound the
        grid tolerance puts on a maximum), ratio within the quotient of the
        two bounds;
      * doppler_hz and code_phase_frac equal (1e-9) to the parabolas of the
        GPU's own grid cells, computed here in FP64 -- the refinement stage
        checked on the search's output;
      * and within the change the grid tolerance allows of the oracle's.
    Returns the number of PRNs checked."""
    n = 0
    for i, r in enumerate(ref_peaks):
        g = gpu_peaks[i]
        if int(g["doppler_bin"]) != r.doppler_bin or int(g["code_phase"]) != r.code_phase:
            continue
        n += 1
        Pr = np.asarray(P_ref[i], np.float64)
        Pg = np.asarray(P_gpu[i], np.float64)
        nd, N = Pr.shape
        m = r.mean
        k, t = r.doppler_bin, r.code_phase
        es = tol * (r.second + m)
        assert abs(float(g["second"]) - r.second) <= es, (r.prn, g["second"], r.second)
        if r.second > 0.0 and np.isfinite(r.ratio):
            rel = tol * (r.peak + m) / r.peak + es / r.second
            assert abs(float(g["ratio"]) - r.ratio) <= 1.01 * rel * r.ratio + 1e-6 * r.ratio, \
                (r.prn, g["ratio"], r.ratio)
        # the GPU's refinement from its own grid
        dc_g = _parabola(Pg[k, (t - 1) % N], Pg[k, t], Pg[k, (t + 1) % N])
        dd_g = _parabola(Pg[k - 1, t], Pg[k, t], Pg[k + 1, t]) if 0 < k < nd - 1 else 0.0
        assert abs(float(g["code_phase_frac"]) - (t + dc_g)) <= 1e-9, (r.prn, g["code_phase_frac"], t + dc_g)
        assert abs(float(g["doppler_hz"]) - (lo + k * step + dd_g * step)) <= 1e-9 * max(1.0, abs(step)), \
            (r.prn, g["doppler_hz"])
        # ... and against the oracle's, within what the grid tolerance allows
        e = lambda y: tol * (y + m)  # noqa: E731
        ym, y0, yp = Pr[k, (t - 1) % N], Pr[k, t], Pr[k, (t + 1) % N]
        bc = _parabola_bound(ym, y0, yp, e(ym), e(y0), e(yp))
        assert abs(float(g["code_phase_frac"]) - r.code_phase_frac) <= bc + 1e-12, \
            (r.prn, g["code_phase_frac"], r.code_phase_frac, bc)
        if 0 < k < nd - 1:
            ym, yp = Pr[k - 1, t], Pr[k + 1, t]
            bd = _parabola_bound(ym, y0, yp, e(ym), e(y0), e(yp)) * abs(step)
            assert abs(float(g["doppler_hz"]) - r.doppler_hz) <= bd + 1e-9 * abs(step), \
                (r.prn, g["doppler_hz"], r.doppler_hz, bd)
        else:
            assert abs(float(g["doppler_hz"]) - r.doppler_hz) <= 1e-9 * max(1.0, abs(step))
    return n

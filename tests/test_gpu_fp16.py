"""GPU tests of the FP16 precision mode: both 2048-point transforms in packed
FP16 (two transforms per instruction) with block floating point, |.|^2 and
the sum over blocks in FP32.

There is no exact FP16 reference to compare with, so the mode is held to an
error bound against the FP64 oracle, derived from the arithmetic:

* every FP16 operation rounds to nearest with unit roundoff u = 2^-11; the
  scalings are exact powers of two and no value leaves the normal range (the
  per-vector exponents bound every intermediate below 2^15);
* one transform is 3 passes (radix 16, 16, 8) of log2(2048) = 11 butterfly
  levels plus 2 twiddle multiplications and the FP16 rounding of its input
  and twiddles; with independent rounding errors its output error has RMS
  about sqrt(11 + 4) u ~ 3.9 u relative to the RMS of its output;
* the path does two transforms and one spectrum product: RMS amplitude error
  eta ~ sqrt(2 * 15 + 2) u ~ 5.7 u ~ 2.8e-3 relative to the RMS of the
  correlation R over the lags of a block;
* the power error of one cell is |2 Re(R conj(dR)) + |dR|^2| <= eta_c (P + rms^2)
  (2|R||dR| <= (|R|^2 + rms^2) |dR| / rms), eta_c the cell's amplitude error
  in units of rms; over ~10^8 cells the largest |dR| / rms is about 6 eta;
  summing blocks does not make it worse.

Hence the mixed tolerance |P16 - P64| <= TOL16 (P64 + mean P64) with TOL16 =
2 * 6 * eta = 3.4e-2 (a factor 2 for the non-Gaussian tail).  Detections must
equal the oracle's unless its decision is within TIE16 = TOL16 of a tie or of
the threshold.  The measured errors are logged.

The same tests run on the exact-length mode (GNSS_FP16_PFA: 1023-point
Good-Thomas transforms, each pass an FP16 x FP16 -> FP32 matrix product).
Its roundings to FP16 are the input, the forward 31-pass output, the stored
spectrum, the code spectrum, the two operations of the spectrum product and
the inverse 31-pass output, plus the FP16 weights of the four passes (each
weight within u of the exact one, which perturbs a pass output by about u of
its RMS); sums are FP32.  That is 11 sources of about u each:
eta ~ sqrt(11) u ~ 3.3 u, and the same argument gives TOLX = 2 * 6 * eta =
2.0e-2.
"""
import time
import types

import numpy as np
import pytest

import oracle as O
import synth
from parity import compare_detections, grid_error, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")

TOL16 = 3.4e-2
TOLX = 2.0e-2
TOL = {G.GNSS_FP16: TOL16, G.GNSS_FP16_PFA: TOLX}
NAME = {G.GNSS_FP16: "FP16", G.GNSS_FP16_PFA: "FP16 exact-length"}


@pytest.fixture(scope="module", params=[G.GNSS_FP16, G.GNSS_FP16_PFA], ids=["fp16", "pfa"])
def ctx16(request):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = G.Context(0, precision=request.param)
    c.prec = request.param
    yield c
    c.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(ctx, snap, srch):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    d_x = _dev(snap.samples)
    d_grid = torch.zeros(len(srch.prns) * nd * N, dtype=torch.float32, device="cuda")
    d_pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
    req = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                         srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                         d_grid.data_ptr(), d_pk.data_ptr())
    ctx.acquire_device(req, torch.cuda.current_stream())
    torch.cuda.synchronize()
    grid = d_grid.cpu().numpy().reshape(len(srch.prns), nd, N)
    return grid, d_pk.cpu().numpy().view(G.PEAK_DTYPE).copy()


def _check(grid, pk, P, srch, spc, planted, prec):
    tol = TOL[prec]
    worst = grid_error(grid, P)
    assert np.all(np.isfinite(grid))
    assert worst <= tol, "%s mixed error %.3e > %.1e" % (NAME[prec], worst, tol)
    ref = O.peaks(P, srch.prns, spc, 2.5, srch.lo, srch.step)
    exempt = compare_detections(pk, ref, P, tie_rel=tol, value_rel=tol)
    peak_err = []
    for p in planted:
        i = srch.prns.index(p.prn)
        assert pk[i]["detected"] and pk[i]["code_phase"] == p.code_phase, p.prn
        r = ref[i]
        peak_err.append(abs(float(grid[i, r.doppler_bin, r.code_phase]) - r.peak) / r.peak)
    agree = sum(int(pk[i]["detected"]) == int(r.detected) and int(pk[i]["code_phase"]) == r.code_phase
                and int(pk[i]["doppler_bin"]) == r.doppler_bin for i, r in enumerate(ref))
    log("  %s vs FP64: max mixed error %.3e, planted peak-cell error max %.2e, detections "
        "identical %d / %d, near-tie exemptions %d" % (NAME[prec], worst, max(peak_err) if peak_err else 0.0,
                                                        agree, len(ref), exempt))
    return worst


AMP_SEQUENCES = [
    # per-block content: "full" int8 noise at full scale, "one" a single unit sample,
    # "zero" no signal, an integer k noise in [-k, k]
    ("extreme", ["one", "full", "zero", 2, "full", "one"]),
    ("mild", [10, 127, 40, 127, 3, 80]),
]


@pytest.mark.parametrize("seq", AMP_SEQUENCES, ids=[a[0] for a in AMP_SEQUENCES])
def test_block_exponents_change_between_blocks(ctx16, seq):
    """Blocks of very different amplitude get different per-vector exponents
    (up to ~20 binades apart): the block sums are rescaled between blocks
    (exact powers of two) and must still meet the mode's bound; a block of
    zeros adds nothing."""
    name, amps = seq
    fs, Tc, Nnc = 4092000, 4, len(amps)
    N = fs // 1000
    L = Tc * N
    rng = np.random.default_rng(sum(name.encode()))
    x = np.zeros(2 * L * Nnc, np.int8)
    for b, a in enumerate(amps):
        blk = x[2 * L * b:2 * L * (b + 1)]
        if a == "full":
            blk[:] = rng.integers(-127, 128, 2 * L)
        elif a == "one":
            blk[2 * int(rng.integers(0, L))] = 1
        elif a != "zero":
            blk[:] = rng.integers(-a, a + 1, 2 * L)
    snap = types.SimpleNamespace(samples=x, fmt=O.CPLX_I8, n=L * Nnc, fs_hz=fs, f_if_hz=0.0)
    srch = synth.Search([5, 22], -1000.0, 1000.0, 500.0, Tc, Nnc)
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    P = O.grid_fft(x, O.CPLX_I8, fs, 0.0, srch.prns, srch.lo, srch.step, nd, Tc, Nnc)
    grid, _ = _run(ctx16, snap, srch)
    assert np.all(np.isfinite(grid))
    worst = grid_error(grid, P)
    log("  %s, blocks %s: max mixed error %.3e" % (NAME[ctx16.prec], name, worst))
    assert worst <= TOL[ctx16.prec]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kinds", [("one", "full", "zero", "noise"), ("one", "tone", "zero", "noise")],
                         ids=["constants", "tone"])
def test_block_exponents_at_full_scale_and_longest_blocks(ctx16, kinds):
    """The longest coherent blocks (64 ms at 16.368 MHz) at the extremes of the
    per-vector exponents: a constant of 1 (exponent 28), a full-scale constant
    or a full-scale complex tone at 5 kHz, which folds coherently (35: the
    sums are scaled down by 2^-14), an all-zero block (exponent 0, more than
    2^30 below the largest: its zero power is dropped) and small noise (24:
    scaled up by 2^22).  Within the mode's bound of the FP64 oracle, and
    finite.  The constants put almost all of a block's power in the DC bin,
    where the code spectrum is +-1 against ~32 elsewhere: both modes remove
    each vector's mean before the FP16 transform, which keeps the FP16
    weights from leaking that bin into the others."""
    fs, Tc = 16368000, 64
    N = fs // 1000
    L = Tc * N
    blocks = []
    rng = np.random.default_rng(64)
    ph = 2 * np.pi * 5000.0 * np.arange(L) / fs
    for kind in kinds:
        b = np.zeros(2 * L, np.int8)
        if kind == "one":
            b[:] = 1
        elif kind == "full":
            b[:] = 127
        elif kind == "tone":
            b[0::2] = np.round(127 * np.cos(ph)).astype(np.int8)
            b[1::2] = np.round(127 * np.sin(ph)).astype(np.int8)
        elif kind == "noise":
            b[:] = rng.integers(-3, 4, 2 * L)
        blocks.append(b)
    x = np.concatenate(blocks)
    Nnc = len(blocks)
    snap = types.SimpleNamespace(samples=x, fmt=O.CPLX_I8, n=L * Nnc, fs_hz=fs, f_if_hz=0.0)
    srch = synth.Search([3, 19], 0.0, 0.0, 1.0, Tc, Nnc)
    P = O.grid_fft(x, O.CPLX_I8, fs, 0.0, srch.prns, 0.0, 1.0, 1, Tc, Nnc)
    grid, _ = _run(ctx16, snap, srch)
    assert np.all(np.isfinite(grid))
    worst = grid_error(grid, P)
    log("  %s, 64 ms blocks %s: max mixed error %.3e" % (NAME[ctx16.prec], "/".join(kinds), worst))
    assert worst <= TOL[ctx16.prec]


DC_CASES = [
    # name, fmt, fs, f_if, DC offset (I, Q) added before quantisation, in noise sigmas
    ("cplx_offset", O.CPLX_I8, 16368000, 0.0, (3.0, -2.0)),
    ("cplx_large_offset", O.CPLX_I8, 4092000, 0.0, (6.0, 5.0)),
    ("real_offset", O.REAL_I8, 4092000, 0.0, (1.5, 0.0)),
]


@pytest.mark.parametrize("case", DC_CASES, ids=[c[0] for c in DC_CASES])
def test_dc_offset_records_match_direct_oracle(ctx16, case):
    """Records with a constant offset in the samples (an ordinary front-end
    imperfection) searched over bins that include the carrier's own
    frequency, where the offset folds into each block's DC bin: within the
    mode's bound of the FP64 direct oracle, the planted satellites found."""
    name, fmt, fs, f_if, (oi, oq) = case
    N = fs // 1000
    Tc, Nnc = 2, 3
    rng = np.random.default_rng(sum(name.encode()))
    n = Tc * Nnc * N + N // 2
    pl = [synth.Planted(prn=p, code_phase=int(rng.integers(0, N)), doppler_hz=d, cn0_dbhz=52.0,
                        carrier_phase=float(rng.uniform(0, 2 * np.pi))) for p, d in ((6, 500.0), (21, -1000.0))]
    prns = [6, 21, 14]
    codes = {p.prn: O.ca_code(p.prn) for p in pl}
    t = np.arange(n)
    sig_i = rng.standard_normal(n) + oi
    sig_q = rng.standard_normal(n) + oq
    for p in pl:
        c = 1.0 - 2.0 * codes[p.prn][((t - p.code_phase) * 1023000 // fs) % 1023].astype(np.float64)
        amp = np.sqrt(2 * 10 ** (p.cn0_dbhz / 10) / fs)
        ph = 2 * np.pi * (f_if + p.doppler_hz) * t / fs + p.carrier_phase
        sig_i += amp * c * np.cos(ph)
        sig_q += amp * c * np.sin(ph)
    if fmt == O.CPLX_I8:
        x = np.empty(2 * n, np.int8)
        x[0::2] = np.clip(np.rint(16 * sig_i), -127, 127).astype(np.int8)
        x[1::2] = np.clip(np.rint(16 * sig_q), -127, 127).astype(np.int8)
    else:
        x = np.clip(np.rint(16 * sig_i), -127, 127).astype(np.int8)
    snap = types.SimpleNamespace(samples=x, fmt=fmt, n=n, fs_hz=fs, f_if_hz=f_if, planted=pl)
    srch = synth.Search(prns, -1500.0, 1500.0, 500.0, Tc, Nnc)
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    grid, pk = _run(ctx16, snap, srch)
    P = O.grid_direct(x, fmt, fs, f_if, prns, srch.lo, srch.step, nd, Tc, Nnc)
    log("fp16 DC offset %s: fs=%d offset=(%.1f, %.1f) sigma" % (name, fs, oi, oq))
    _check(grid, pk, P, srch, fs // 1023000, pl, ctx16.prec)


def test_fp16_rejects_unknown_precision():
    with pytest.raises(G.GnssError) as ei:
        G.Context(0, precision=7)
    assert ei.value.code == G.GNSS_EINVAL


SEARCH_CASES = [
    # name, fmt, fs, f_if, Tc, Nnc, prns searched, planted, lo, hi, step, cn0
    ("spc1_cplx", O.CPLX_I8, 1023000, 0.0, 1, 2, [3, 9], [9], -1000.0, 1000.0, 1000.0, 50.0),
    # N = 1023: the 2-bit blocks start at sample offsets 0, 3, 2, 1 within a byte
    ("spc1_packed_subbyte", O.REAL_2BIT_PACKED, 1023000, 255750.0, 1, 4, [2, 7, 11], [7], -1000.0, 1000.0,
     500.0, 54.0),
    ("spc2_packed_ragged", O.REAL_2BIT_PACKED, 2046000, 511500.0, 2, 3, [1, 5, 9, 13, 17],
     [5, 13], -1500.0, 1500.0, 500.0, 48.0),
    ("spc4_real", O.REAL_I8, 4092000, 1023000.0, 1, 4, [2, 4, 6, 8, 10, 12], [4, 10], -1000.0,
     1000.0, 500.0, 46.0),
    ("spc8_cplx_dup", O.CPLX_I8, 8184000, 0.0, 1, 2, [37, 7, 7], [7], -500.0, 500.0, 500.0, 48.0),
    ("spc16_cplx", O.CPLX_I8, 16368000, 0.0, 2, 1, [11, 31], [31], -250.0, 0.0, 250.0, 47.0),
]


@pytest.mark.parametrize("case", SEARCH_CASES, ids=[c[0] for c in SEARCH_CASES])
def test_fp16_search_matches_direct_oracle(ctx16, case):
    name, fmt, fs, f_if, Tc, Nnc, prns, planted, lo, hi, step, cn0 = case
    nd = O.n_doppler(lo, hi, step)
    rng = np.random.default_rng(sum(name.encode()) % 1000)
    N = fs // 1000
    pl = [synth.Planted(prn=p, code_phase=int(rng.integers(0, N)), doppler_hz=lo + step * (nd // 2) + 0.3 * step,
                        cn0_dbhz=cn0, carrier_phase=float(rng.uniform(0, 2 * np.pi))) for p in planted]
    snap = synth.make_snapshot(sum(name.encode()) % 1000, fmt, fs, f_if, Tc * Nnc + 0.5, pl, O.ca_code)
    srch = synth.Search(prns, lo, hi, step, Tc, Nnc)
    log("fp16 search %s: fs=%d prns=%s bins=%d Tc=%d Nnc=%d" % (name, fs, prns, nd, Tc, Nnc))
    grid, pk = _run(ctx16, snap, srch)
    P = O.grid_direct(snap.samples, fmt, fs, f_if, prns, lo, step, nd, Tc, Nnc)
    _check(grid, pk, P, srch, fs // 1023000, snap.planted, ctx16.prec)


def test_fp16_noiseless_closed_form(ctx16):
    # x = c_p[(n - d) mod N] at 0 Hz: P[d] = Nnc (Tc N)^2 exactly in FP64
    fs, Tc, Nnc, prn, d = 4092000, 2, 3, 21, 1001
    N = fs // 1000
    rep = O.code_replica(prn, fs, N).astype(np.int64)
    sig = np.tile(np.roll(rep, d), Tc * Nnc).astype(np.int8)
    x = np.zeros(2 * sig.size, np.int8)
    x[0::2] = sig
    snap = synth.Snapshot(samples=x, fmt=O.CPLX_I8, fs_hz=fs, f_if_hz=0.0, n=sig.size)
    srch = synth.Search([prn, 5], 0.0, 0.0, 1.0, Tc, Nnc)
    grid, pk = _run(ctx16, snap, srch)
    assert pk[0]["code_phase"] == d and pk[0]["detected"]
    rel = abs(grid[0, 0, d] / (Nnc * float(Tc * N) ** 2) - 1.0)
    log("  noiseless peak relative error %.2e" % rel)
    assert rel < TOL[ctx16.prec]
    P = O.grid_direct(x, O.CPLX_I8, fs, 0.0, [prn, 5], 0.0, 1.0, 1, Tc, Nnc)
    assert grid_error(grid, P) <= TOL[ctx16.prec]


def test_fp16_strong_workload(ctx16, strong_case):
    """The strong-signal workload on the FP16 path: error against FP64,
    planted peak cells, detection agreement, and time against FP32."""
    snap, srch, nd, P = strong_case
    log("fp16 strong workload: real 2-bit 4.092 MHz, 32 PRN x 21 bins x 10 ms")
    grid, pk = _run(ctx16, snap, srch)
    _check(grid, pk, P, srch, 4, snap.planted, ctx16.prec)
    # deterministic
    grid2, pk2 = _run(ctx16, snap, srch)
    assert np.array_equal(grid, grid2) and np.array_equal(pk, pk2)
    with G.Context(0) as c32:
        times = {}
        for name, c in (("fp32", c32), ("fp16", ctx16)):
            _run(c, snap, srch)
            t0 = time.perf_counter()
            for _ in range(5):
                _run(c, snap, srch)
            times[name] = (time.perf_counter() - t0) / 5 * 1e3
    log("  wall per search incl. copies: fp32 %.3f ms, %s %.3f ms" % (times["fp32"], NAME[ctx16.prec],
                                                                       times["fp16"]))


@pytest.mark.timeout(600)
def test_fp16_weak_workload_full_size(ctx16, weak_case):
    snap, srch, nd, P = weak_case
    log("fp16 weak workload: complex int8 16.368 MHz, 32 PRN x 121 bins x 25 x 4 ms")
    grid, pk = _run(ctx16, snap, srch)
    _check(grid, pk, P, srch, 16, snap.planted, ctx16.prec)


def test_fp16_batch_graph_serving_equal_alone(ctx16):
    items = synth.batch_workload(O.ca_code, seed=43, n=6, ms_range=(4, 10), prn_range=(3, 7),
                                 window_khz=(1.0, 2.0), planted_range=(1, 2), cn0_range=(44.0, 48.0))
    alone, bufs = [], []
    for snap, srch in items:
        alone.append(_run(ctx16, snap, srch))
    reqs = []
    for snap, srch in items:
        nd = O.n_doppler(srch.lo, srch.hi, srch.step)
        x = _dev(snap.samples)
        g = torch.full((len(srch.prns) * nd * (snap.fs_hz // 1000),), -1.0, device="cuda")
        pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
        bufs.append((x, g, pk, srch, snap))
        reqs.append(G.make_request(x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                                   srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                                   g.data_ptr(), pk.data_ptr()))

    def results():
        torch.cuda.synchronize()
        return [(g.cpu().numpy(), pk.cpu().numpy().view(G.PEAK_DTYPE)) for x, g, pk, srch, snap in bufs]

    ctx16.acquire_batch_device(reqs)
    for i, (g, p) in enumerate(results()):
        assert np.array_equal(g, alone[i][0].ravel()) and np.array_equal(p, alone[i][1]), i
    graph = ctx16.graph(reqs)
    try:
        for rep in range(2):
            for x, g, pk, srch, snap in bufs:
                g.fill_(-1.0)
            graph.launch(torch.cuda.current_stream())
            for i, (g, p) in enumerate(results()):
                assert np.array_equal(g, alone[i][0].ravel()) and np.array_equal(p, alone[i][1]), (rep, i)
    finally:
        graph.close()
    with G.Context(0, precision=ctx16.prec) as sctx:
        tickets = []
        for i, (snap, srch) in enumerate(items):
            nd = O.n_doppler(srch.lo, srch.hi, srch.step)
            grid = np.full((len(srch.prns), nd, snap.fs_hz // 1000), -1.0, np.float32)
            pk = np.zeros(len(srch.prns), G.PEAK_DTYPE)
            xs = np.ascontiguousarray(snap.samples)
            req = G.make_request(xs.ctypes.data, snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                                 srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                                 grid.ctypes.data, pk.ctypes.data)
            tickets.append((i, sctx.submit(req), grid, pk, xs, req))
        for i, t, grid, pk, xs, req in tickets:
            assert sctx.wait(t, 60.0).status == 0
            assert np.array_equal(grid, alone[i][0]) and np.array_equal(pk, alone[i][1]), i

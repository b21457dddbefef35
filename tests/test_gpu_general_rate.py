"""GPU parity at sample rates that are not a multiple of the chip rate.

Any whole number of kHz up to N = 16384 samples per ms is a valid rate: the
replica then samples chip floor(n 1023000 / fs) with no whole number of
samples per chip, and the search correlates each folded block on zero-padded
transforms of length M = 2^ceil(log2 2N) (FP32, in every context precision).
Parity against the oracle's direct correlation (FP64, exact integers before
the squares): the FP32 power grid within the mixed tolerance 1e-4, identical
detections, the second peak, ratio and FP64 refinements as in
test_gpu_parity.py.  The second-peak exclusion is one chip, fs / 1.023 MHz
samples (oracle.chip_exclusion).
"""
import numpy as np
import pytest

import oracle as O
import synth
from parity import assert_grid_close, compare_detections, compare_refinement, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = G.Context(0)
    yield c
    c.close()


def _search(c, snap, srch, stream=None):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    d_x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
    d_grid = torch.zeros(len(srch.prns) * nd * N, dtype=torch.float32, device="cuda")
    d_pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
    req = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                         srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                         d_grid.data_ptr(), d_pk.data_ptr())
    c.acquire_device(req, stream or torch.cuda.current_stream())
    torch.cuda.synchronize()
    return (d_grid.cpu().numpy().reshape(len(srch.prns), nd, N),
            d_pk.cpu().numpy().view(G.PEAK_DTYPE).copy())


CASES = [
    # name, fmt, fs, f_if, Tc, Nnc, prns, planted (prn, Doppler), lo, hi, step
    ("5M_cplx", O.CPLX_I8, 5000000, 0.0, 1, 3, [4, 17, 30], [(17, 750.0)], -1500.0, 1500.0, 750.0),
    ("2M5_real", O.REAL_I8, 2500000, 625000.0, 2, 2, [9, 12], [(12, -500.0)], -1000.0, 1000.0, 500.0),
    ("4M_packed", O.REAL_2BIT_PACKED, 4000000, 1000000.0, 1, 3, [1, 8, 25], [(8, 1000.0)], 0.0, 2000.0, 500.0),
    ("10M_cplx", O.CPLX_I8, 10000000, 0.0, 1, 2, [6, 21], [(21, -1500.0)], -2000.0, 0.0, 500.0),
    ("7M777_real", O.REAL_I8, 7777000, 1944250.0, 1, 2, [11, 2], [(11, 250.0)], -250.0, 750.0, 500.0),
    ("7M777_packed", O.REAL_2BIT_PACKED, 7777000, 1944250.0, 1, 2, [5, 19], [(19, 0.0)], -500.0, 500.0, 500.0),
    ("10M_packed", O.REAL_2BIT_PACKED, 10000000, 2500000.0, 1, 2, [28], [(28, 500.0)], 0.0, 500.0, 500.0),
    ("5M_real", O.REAL_I8, 5000000, 1250000.0, 1, 2, [3, 13], [(3, -250.0)], -750.0, 250.0, 500.0),
    ("2M5_cplx", O.CPLX_I8, 2500000, 0.0, 3, 2, [20, 31], [(31, 400.0)], -400.0, 400.0, 400.0),
    # M = 2P: N > 8192 takes the even/odd split of the 32768-point transforms
    ("8M193_real", O.REAL_I8, 8193000, 2048250.0, 1, 2, [14], [(14, -500.0)], -500.0, 0.0, 500.0),
    ("12M_cplx", O.CPLX_I8, 12000000, 0.0, 1, 2, [7, 24], [(24, 0.0)], -500.0, 500.0, 500.0),
    # N a power of two: M = N, no padding (16384, the largest; 8192; 1024)
    ("16M384_cplx", O.CPLX_I8, 16384000, 0.0, 1, 2, [7, 24], [(24, 0.0)], -500.0, 500.0, 500.0),
    ("8M192_cplx", O.CPLX_I8, 8192000, 0.0, 1, 2, [2, 29], [(29, 500.0)], 0.0, 500.0, 500.0),
    ("1M024_packed", O.REAL_2BIT_PACKED, 1024000, 256000.0, 2, 2, [5, 30], [(30, -500.0)], -500.0, 0.0, 500.0),
    # a tiny N
    ("100k_cplx", O.CPLX_I8, 100000, 0.0, 4, 3, [1, 2], [(2, 0.0)], -250.0, 250.0, 250.0),
    # odd lengths: N = 63 (M = 128); N = 64 (a power of two: M = N); a prime N = 3001;
    # N = 13370 packed (every other block starts inside a byte); N = 16383, the largest
    # length below the limit that is not a power of two (the 32768-point split)
    ("63k_cplx", O.CPLX_I8, 63000, 0.0, 2, 3, [1, 2], [(2, 0.0)], -250.0, 250.0, 250.0),
    ("64k_real", O.REAL_I8, 64000, 16000.0, 2, 3, [5, 6], [(6, 0.0)], -250.0, 250.0, 250.0),
    ("3M001_cplx", O.CPLX_I8, 3001000, 0.0, 1, 2, [4, 9], [(9, 250.0)], -250.0, 250.0, 250.0),
    ("13M37_packed", O.REAL_2BIT_PACKED, 13370000, 3342500.0, 1, 2, [12], [(12, 0.0)], -500.0, 500.0, 500.0),
    ("16M383_cplx", O.CPLX_I8, 16383000, 0.0, 1, 2, [30], [(30, -500.0)], -500.0, 0.0, 500.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_general_rate_search_matches_direct_oracle(ctx, case):
    name, fmt, fs, f_if, Tc, Nnc, prns, planted, lo, hi, step = case
    N = fs // 1000
    rng = np.random.default_rng(sum(name.encode()))
    pl = [synth.Planted(prn=p, code_phase=int(rng.integers(0, N)), doppler_hz=dop, cn0_dbhz=52.0,
                        carrier_phase=float(rng.uniform(0, 2 * np.pi))) for p, dop in planted]
    snap = synth.make_snapshot(sum(name.encode()) % 997, fmt, fs, f_if, Tc * Nnc + 0.37, pl, O.ca_code)
    srch = synth.Search(prns, lo, hi, step, Tc, Nnc)
    nd = O.n_doppler(lo, hi, step)
    M = 64
    while M < 2 * N:
        M *= 2
    if N >= 64 and N & (N - 1) == 0:
        M = N  # a power of two: the N-point correlation, no padding
    log("general rate %s: fs=%d N=%d M=%d fmt=%d bins=%d Tc=%d Nnc=%d" % (name, fs, N, M, fmt, nd, Tc, Nnc))
    grid, pk = _search(ctx, snap, srch)
    P = O.grid_direct(snap.samples, fmt, fs, f_if, prns, lo, step, nd, Tc, Nnc)
    worst = assert_grid_close(grid, P)
    excl = O.chip_exclusion(fs)
    ref = O.peaks(P, prns, excl, 2.5, lo, step)
    exempt = compare_detections(pk, ref, P)
    checked = compare_refinement(pk, ref, P, grid, lo, step)
    if N >= 1023:  # a planted satellite at 52 dB-Hz is found at its code phase
        for p in pl:
            i = prns.index(p.prn)
            assert pk[i]["detected"] and pk[i]["code_phase"] == p.code_phase, (p.prn, pk[i])
    log("  max mixed error %.3e, exemptions %d, refinements checked %d" % (worst, exempt, checked))


@pytest.mark.timeout(600)
def test_weak_workload_at_10mhz_full_size(ctx):
    """The benchmark's 10 MHz weak-signal workload at full size (N = 10000,
    M = 32768: the four-step 16384-point kernels with both halves; 32 PRNs x
    121 bins x 25 blocks of 4 ms) in the launch configuration bench.py times:
    the FP32 grid against the oracle's FP64 FFT route everywhere, detections
    and refinements, and sampled cells (every detected peak and random cells)
    against the direct correlation."""
    snap, srch = synth.weak_complex_int8(O.ca_code, seed=2, fs=10000000)
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    log("weak workload at 10 MHz: complex int8, 32 PRN x %d bins x %d phases x 25 x 4 ms" % (nd, N))
    grid, pk = _search(ctx, snap, srch)
    log("  oracle grid (FP64 FFT route) ...")
    P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.step,
                   nd, srch.T_coh, srch.N_noncoh)
    worst = assert_grid_close(grid, P)
    ref = O.peaks(P, srch.prns, O.chip_exclusion(snap.fs_hz), 2.5, srch.lo, srch.step)
    exempt = compare_detections(pk, ref, P)
    checked = compare_refinement(pk, ref, P, grid, srch.lo, srch.step)
    assert checked >= len(srch.prns) - exempt
    log("  max mixed error %.3e, exemptions %d, refinements checked %d" % (worst, exempt, checked))
    rng = np.random.default_rng(3)
    cells = [(srch.prns.index(int(r["prn"])), int(r["doppler_bin"]), int(r["code_phase"]))
             for r in pk if r["detected"]]
    assert cells  # the strongest planted satellites are found
    cells += list(zip(rng.integers(0, len(srch.prns), 40), rng.integers(0, nd, 40), rng.integers(0, N, 40)))
    cells = np.array(cells, np.int64)
    vals = O.cells_direct(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                          srch.step, nd, srch.T_coh, srch.N_noncoh, cells)
    got = grid[cells[:, 0], cells[:, 1], cells[:, 2]].astype(np.float64)
    means = P.mean(axis=(1, 2))[cells[:, 0]]
    assert np.all(np.abs(got - vals) <= 1e-4 * (vals + means))


def test_general_rate_code_doppler_matches_oracle():
    """Code-Doppler compensation at a general rate: the folded block delayed
    by llround(b Tc N f_k / f_L1) samples, as in the oracle."""
    fs, Tc, Nnc = 5000000, 5, 8
    pl = [synth.Planted(prn=16, code_phase=2222, doppler_hz=5000.0, cn0_dbhz=45.0)]
    snap = synth.make_snapshot(5, O.CPLX_I8, fs, 0.0, Tc * Nnc + 0.2, pl, O.ca_code, code_doppler=True)
    srch = synth.Search([16, 4], 3000.0, 5000.0, 1000.0, Tc, Nnc)
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    shifts = [O.code_shift(b, Tc, fs // 1000, 5000.0) for b in range(Nnc)]
    assert max(shifts) >= 1, shifts  # the compensation moves the later blocks
    with G.Context(0) as c:
        c.set("code_doppler", 1)
        grid, pk = _search(c, snap, srch)
    # the FFT route of the oracle (pinned to the direct one with code-Doppler shifts)
    P = O.grid_fft(snap.samples, snap.fmt, fs, 0.0, srch.prns, srch.lo, srch.step, nd, Tc, Nnc,
                   code_doppler=True)
    assert_grid_close(grid, P)
    compare_detections(pk, O.peaks(P, srch.prns, O.chip_exclusion(fs), 2.5, srch.lo, srch.step), P)
    assert pk[0]["detected"] and pk[0]["doppler_bin"] == 2 and pk[0]["code_phase"] == 2222


def test_general_rate_same_in_every_precision_and_in_a_mixed_batch():
    """The general-rate kernels are FP32 in every context: FP16 and
    exact-length contexts give the FP32 context's grid bit for bit.  In a
    batch beside chip-rate requests (which take the polyphase kernels) each
    request's results equal its results alone, bit for bit, also beside
    general-rate requests of another transform length."""
    snaps = []
    # 5 and 10 MHz take the 16384-point kernels (one and two halves), 2.5 MHz
    # the 8192-point ones: one batch launches both lengths, each skipping the
    # other's items
    for i, (fs, fmt, f_if) in enumerate([(5000000, O.CPLX_I8, 0.0), (4092000, O.REAL_I8, 1023000.0),
                                         (10000000, O.REAL_2BIT_PACKED, 2500000.0), (2046000, O.CPLX_I8, 0.0),
                                         (2500000, O.CPLX_I8, 0.0)]):
        pl = [synth.Planted(prn=3 + i, code_phase=100 * i + 7, doppler_hz=500.0, cn0_dbhz=50.0)]
        snaps.append((synth.make_snapshot(40 + i, fmt, fs, f_if, 3.2, pl, O.ca_code),
                      synth.Search([3 + i, 20], 0.0, 1000.0, 500.0, 1, 3)))
    alone = {}
    with G.Context(0) as c32:
        for j, (snap, srch) in enumerate(snaps):
            alone[j] = _search(c32, snap, srch)
        # the batch
        stream = torch.cuda.current_stream()
        bufs, reqs = [], []
        for snap, srch in snaps:
            nd = O.n_doppler(srch.lo, srch.hi, srch.step)
            N = snap.fs_hz // 1000
            x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
            g = torch.zeros(len(srch.prns) * nd * N, dtype=torch.float32, device="cuda")
            pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
            bufs.append((x, g, pk, nd, N))
            reqs.append(G.make_request(x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                                       srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh, g.data_ptr(),
                                       pk.data_ptr()))
        c32.acquire_batch_device(reqs, stream)
        torch.cuda.synchronize()
        for j, (x, g, pk, nd, N) in enumerate(bufs):
            gb = g.cpu().numpy().reshape(-1, nd, N)
            pb = pk.cpu().numpy().view(G.PEAK_DTYPE)
            assert np.array_equal(gb, alone[j][0]), j
            assert pb.tobytes() == alone[j][1].tobytes(), j
    for prec in (G.GNSS_FP16, G.GNSS_FP16_PFA):
        with G.Context(0, precision=prec) as ch:
            for j in (0, 2, 4):  # the general-rate requests
                grid, pk = _search(ch, *snaps[j])
                assert np.array_equal(grid, alone[j][0]), (prec, j)
                assert pk.tobytes() == alone[j][1].tobytes(), (prec, j)


def test_general_rate_served_equals_alone():
    """Served (continuous batching) general-rate requests, submitted beside a
    chip-rate one: results bit for bit those of the requests alone."""
    import time
    specs = [(91, 5000000, O.CPLX_I8, 0.0), (92, 4092000, O.REAL_I8, 1023000.0),
             (93, 10000000, O.CPLX_I8, 0.0), (94, 2500000, O.REAL_2BIT_PACKED, 625000.0)]
    items = []
    for seed, fs, fmt, f_if in specs:
        pl = [synth.Planted(prn=11, code_phase=777, doppler_hz=500.0, cn0_dbhz=50.0)]
        snap = synth.make_snapshot(seed, fmt, fs, f_if, 4.4, pl, O.ca_code)
        items.append((snap, synth.Search([11, 25], 0.0, 1000.0, 500.0, 2, 2)))
    with G.Context(0) as c:
        alone = [_search(c, snap, srch) for snap, srch in items]
    with G.Context(0) as sctx:
        subs = []
        for i, (snap, srch) in enumerate(items):
            nd = O.n_doppler(srch.lo, srch.hi, srch.step)
            N = snap.fs_hz // 1000
            grid = np.zeros((len(srch.prns), nd, N), np.float32)
            pk = np.zeros(len(srch.prns), G.PEAK_DTYPE)
            x = np.ascontiguousarray(snap.samples)
            req = G.make_request(x.ctypes.data, snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                                 srch.hi, srch.step, srch.T_coh, srch.N_noncoh, grid.ctypes.data, pk.ctypes.data)
            subs.append((sctx.submit(req), grid, pk, x))
            time.sleep(0.001)
        for i, (t, grid, pk, x) in enumerate(subs):
            info = sctx.wait(t, 60.0)
            assert info.status == 0, i
            assert np.array_equal(grid, alone[i][0]), i
            assert pk.tobytes() == alone[i][1].tobytes(), i


def test_general_rate_unsupported_options():
    snap = synth.make_snapshot(9, O.CPLX_I8, 5000000, 0.0, 2.2, [], O.ca_code)
    srch = synth.Search([1], 0.0, 0.0, 1.0, 1, 2)
    with G.Context(0, precision=G.GNSS_FP16_PFA) as c:
        c.set("nav_pairs", 1)
        with pytest.raises(G.GnssError) as ei:
            _search(c, snap, srch)
        assert ei.value.code == G.GNSS_ENOTSUP
    with G.Context(0, precision=G.GNSS_FP16_PFA) as c:
        c.set("doppler_fd", 1)
        with pytest.raises(G.GnssError) as ei:
            _search(c, snap, srch)
        assert ei.value.code == G.GNSS_ENOTSUP
    # the boxcar/polyphase stage entry point needs a chip-rate multiple
    with G.Context(0) as c:
        d_x = torch.from_numpy(snap.samples).cuda()
        out = torch.zeros(1 << 16, dtype=torch.int32, device="cuda")
        req = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, 5000000, 0.0, [1], 0.0, 0.0, 1.0, 1, 2, None, 0)
        with pytest.raises(G.GnssError) as ei:
            c.box_fold(req, out.data_ptr(), torch.cuda.current_stream())
        assert ei.value.code == G.GNSS_ENOTSUP

"""GPU tests of the frequency-domain Doppler variant (option doppler_fd on an
exact-length context): one zero-padded long DFT per block serves every
Doppler bin by a spectrum shift.  The reference is the oracle's exact-carrier
route (grid_fft(carrier="exact"), pinned in test_oracle_exact_carrier.py).

Error bound: the exact-length mode's (TOLX, test_gpu_fp16.py) plus the long
DFT's first pass, which rounds its input, its 31-pass output and its two
weight tables to FP16 (4 more sources of about u = 2^-11); the second pass,
the synthesis and the carrier are FP32.  eta ~ sqrt(15) u ~ 3.9 u, so
TOLFD = 2 * 6 * eta = 2.3e-2; detections identical except oracle near ties.
"""
import numpy as np
import pytest

import oracle as O
import synth
from parity import compare_detections, grid_error, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")

TOLFD = 2.3e-2


@pytest.fixture(scope="module")
def ctxfd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = G.Context(0, precision=G.GNSS_FP16_PFA)
    c.set("doppler_fd", 1)
    yield c
    c.close()


def _run(ctx, snap, srch):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    d_x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
    d_grid = torch.full((len(srch.prns) * nd * N,), -1.0, dtype=torch.float32, device="cuda")
    d_pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
    req = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                         srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                         d_grid.data_ptr(), d_pk.data_ptr())
    ctx.acquire_device(req, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return d_grid.cpu().numpy().reshape(len(srch.prns), nd, N), d_pk.cpu().numpy().view(G.PEAK_DTYPE).copy()


def _check(grid, pk, P, srch, spc, planted=()):
    assert np.all(np.isfinite(grid))
    worst = grid_error(grid, P)
    ref = O.peaks(P, srch.prns, spc, 2.5, srch.lo, srch.step)
    exempt = compare_detections(pk, ref, P, tie_rel=TOLFD, value_rel=TOLFD)
    for p in planted:
        i = srch.prns.index(p.prn)
        assert pk[i]["detected"] and pk[i]["code_phase"] == p.code_phase, p.prn
    log("  frequency-domain Doppler vs FP64 exact carrier: max mixed error %.3e, near-tie exemptions %d"
        % (worst, exempt))
    assert worst <= TOLFD, worst


CASES = [
    # name, fmt, fs, f_if, Tc, Nnc, prns, planted, lo, hi, step   (P = 1000 / (step Tc) rounded up to 1, 2, 4)
    ("spc1_P1", O.CPLX_I8, 1023000, 0.0, 1, 3, [3, 9], [9], -2000.0, 2000.0, 1000.0),
    ("spc2_packed_P2", O.REAL_2BIT_PACKED, 2046000, 511500.0, 2, 2, [1, 5, 13], [5, 13], -1500.0, 1500.0, 250.0),
    ("spc4_real_P2", O.REAL_I8, 4092000, 1023000.0, 1, 4, [2, 4, 10], [4, 10], -1000.0, 1000.0, 500.0),
    ("spc8_cplx_P4", O.CPLX_I8, 8184000, 0.0, 1, 2, [7, 7, 30], [7], -500.0, 500.0, 250.0),
    ("spc16_cplx_P2", O.CPLX_I8, 16368000, 0.0, 4, 2, [11, 31], [31], -375.0, 375.0, 125.0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fd_search_matches_exact_carrier_oracle(ctxfd, case):
    name, fmt, fs, f_if, Tc, Nnc, prns, planted, lo, hi, step = case
    nd = O.n_doppler(lo, hi, step)
    rng = np.random.default_rng(sum(name.encode()) % 1000)
    N = fs // 1000
    pl = [synth.Planted(prn=p, code_phase=int(rng.integers(0, N)), doppler_hz=lo + step * (nd // 2) + 0.3 * step,
                        cn0_dbhz=48.0, carrier_phase=float(rng.uniform(0, 2 * np.pi))) for p in planted]
    snap = synth.make_snapshot(sum(name.encode()) % 997, fmt, fs, f_if, Tc * Nnc + 0.5, pl, O.ca_code)
    srch = synth.Search(prns, lo, hi, step, Tc, Nnc)
    log("fd search %s: fs=%d bins=%d Tc=%d Nnc=%d step=%g" % (name, fs, nd, Tc, Nnc, step))
    grid, pk = _run(ctxfd, snap, srch)
    P = O.grid_fft(snap.samples, fmt, fs, f_if, prns, lo, step, nd, Tc, Nnc, carrier="exact")
    _check(grid, pk, P, srch, fs // 1023000, snap.planted)


def test_fd_strong_workload(ctxfd, strong_case):
    snap, srch, nd, _ = strong_case
    log("fd strong workload: real 2-bit 4.092 MHz, 32 PRN x 21 bins x 10 ms")
    grid, pk = _run(ctxfd, snap, srch)
    P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.step, nd,
                   srch.T_coh, srch.N_noncoh, carrier="exact")
    _check(grid, pk, P, srch, 4, snap.planted)
    grid2, pk2 = _run(ctxfd, snap, srch)
    assert np.array_equal(grid, grid2) and np.array_equal(pk, pk2)


@pytest.mark.timeout(600)
def test_fd_weak_workload_planted_prns(ctxfd, weak_case):
    # full size (P = 2, long DFT 128 x 1023 per 4 ms block); the oracle rows of the
    # eight planted PRNs and two others
    snap, srch, nd, _ = weak_case
    log("fd weak workload: complex int8 16.368 MHz, 32 PRN x 121 bins x 25 x 4 ms")
    grid, pk = _run(ctxfd, snap, srch)
    rows = sorted({p.prn for p in snap.planted} | {srch.prns[0], srch.prns[-1]})
    idx = [srch.prns.index(p) for p in rows]
    P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, rows, srch.lo, srch.step, nd,
                   srch.T_coh, srch.N_noncoh, carrier="exact")
    sub = synth.Search(rows, srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh)
    _check(grid[idx], pk[idx], P, sub, 16)
    for p in snap.planted:
        i = srch.prns.index(p.prn)
        assert pk[i]["detected"] and pk[i]["code_phase"] == p.code_phase, p.prn


def test_fd_equals_alone_in_a_batch(ctxfd):
    items = synth.batch_workload(O.ca_code, seed=44, n=5, ms_range=(4, 8), prn_range=(2, 4),
                                 window_khz=(1.0, 2.0), planted_range=(1, 1), cn0_range=(46.0, 48.0))
    alone = [_run(ctxfd, snap, srch) for snap, srch in items]
    bufs, reqs = [], []
    for snap, srch in items:
        nd = O.n_doppler(srch.lo, srch.hi, srch.step)
        x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
        g = torch.full((len(srch.prns) * nd * (snap.fs_hz // 1000),), -1.0, device="cuda")
        pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
        bufs.append((x, g, pk))
        reqs.append(G.make_request(x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                                   srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                                   g.data_ptr(), pk.data_ptr()))
    ctxfd.acquire_batch_device(reqs)
    torch.cuda.synchronize()
    for i, (x, g, pk) in enumerate(bufs):
        assert np.array_equal(g.cpu().numpy(), alone[i][0].ravel()), i
        assert np.array_equal(pk.cpu().numpy().view(G.PEAK_DTYPE), alone[i][1]), i


def test_fd_unsupported_configurations(ctxfd):
    snap = synth.make_snapshot(1, O.CPLX_I8, 4092000, 0.0, 3.0, [], O.ca_code)
    for srch in (synth.Search([1], -300.0, 300.0, 300.0, 1, 2),      # 0.3 bins: no P in {1, 2, 4}
                 synth.Search([1], -500.0, 500.0, 500.0, 3, 1)):     # P Tc spc = 24: not a power of two
        with pytest.raises(G.GnssError) as ei:
            _run(ctxfd, snap, srch)
        assert ei.value.code == G.GNSS_ENOTSUP
    ctxfd.set("code_doppler", 1)
    try:
        with pytest.raises(G.GnssError) as ei:
            _run(ctxfd, snap, synth.Search([1], -500.0, 500.0, 500.0, 1, 2))
        assert ei.value.code == G.GNSS_ENOTSUP
    finally:
        ctxfd.set("code_doppler", 0)
    with G.Context(0, precision=G.GNSS_FP16) as c16:
        with pytest.raises(G.GnssError) as ei:
            c16.set("doppler_fd", 1)
        assert ei.value.code == G.GNSS_ENOTSUP

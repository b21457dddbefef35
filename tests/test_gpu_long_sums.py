"""GPU parity of long non-coherent sums: requests of more blocks than one
summation group (256 blocks), so that every FP32 correlation kernel adds its
group sums to the grid before the final write.

Covered: the chip-rate kernel at one and four samples per chip and with two
coherent milliseconds per block, each PRN tile and waves-per-workgroup shape
and the persistent launch (bit-identical to the default shape: each cell is
summed in the same block order and grouped at the same blocks), the group
boundaries (256, 257 and 512 blocks), and the general-rate kernels at a
4096-point transform and at both 16384-point cases (M = 32768 in two halves,
M = N = 16384).  The whole FP32 grid against the oracle's FP64 FFT route
within the mixed tolerance, with identical detections.  Long and short
requests batched together and in replayed graphs equal their own searches
bit for bit; the FP16 modes, which keep plain running sums, stay within
their bounds over 600 blocks.
"""
import numpy as np
import pytest

import oracle as O
import synth
from parity import assert_grid_close, compare_detections, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")

GROUP = 256  # blocks per summation group in the FP32 kernels


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = G.Context(0)
    yield c
    c.close()


def _search(c, snap, srch):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    d_x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
    d_grid = torch.zeros(len(srch.prns) * nd * N, dtype=torch.float32, device="cuda")
    d_pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
    req = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                         srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                         d_grid.data_ptr(), d_pk.data_ptr())
    c.acquire_device(req, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return (d_grid.cpu().numpy().reshape(len(srch.prns), nd, N),
            d_pk.cpu().numpy().view(G.PEAK_DTYPE).copy())


def _case(name, fmt, fs, f_if, Tc, Nnc, prns, planted, lo, hi, step):
    rng = np.random.default_rng(sum(name.encode()))
    N = fs // 1000
    pl = [synth.Planted(prn=p, code_phase=int(rng.integers(0, N)), doppler_hz=dop, cn0_dbhz=40.0,
                        carrier_phase=float(rng.uniform(0, 2 * np.pi))) for p, dop in planted]
    snap = synth.make_snapshot(sum(name.encode()) % 991, fmt, fs, f_if, Tc * Nnc + 0.25, pl, O.ca_code)
    return snap, synth.Search(prns, lo, hi, step, Tc, Nnc), pl


def _check(snap, srch, grid, pk):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.step,
                   nd, srch.T_coh, srch.N_noncoh)
    worst = assert_grid_close(grid, P)
    ref = O.peaks(P, srch.prns, O.chip_exclusion(snap.fs_hz), 2.5, srch.lo, srch.step)
    exempt = compare_detections(pk, ref, P)
    return worst, exempt


def test_chip_rate_long_sum_every_shape(ctx):
    """600 blocks (two full groups and 88) at 1.023 MHz, three PRNs (a
    ragged last tile for tiles 2 and 4): every FP32 shape and schedule."""
    snap, srch, pl = _case("1M023_600", O.CPLX_I8, 1023000, 0.0, 1, 600, [3, 11, 19], [(11, 500.0)],
                           -500.0, 500.0, 500.0)
    log("chip rate, 1 sample per chip, 600 blocks, shapes (tile, waves) x schedule")
    grid, pk = _search(ctx, snap, srch)
    worst, exempt = _check(snap, srch, grid, pk)
    i = srch.prns.index(11)
    assert pk[i]["detected"] and pk[i]["code_phase"] == pl[0].code_phase, pk[i]
    log("  default shape: max mixed error %.3e, exemptions %d" % (worst, exempt))
    try:
        for pt, w in ((1, 12), (1, 6), (1, 4), (2, 8), (4, 8)):
            for sched in (0, 1):
                ctx.set("corr_ptile", pt)
                ctx.set("corr_waves", w)
                ctx.set("persistent", sched)
                g2, p2 = _search(ctx, snap, srch)
                assert np.array_equal(g2, grid) and np.array_equal(p2, pk), (pt, w, sched)
    finally:
        ctx.set("corr_ptile", 0)
        ctx.set("corr_waves", 0)
        ctx.set("persistent", -1)


@pytest.mark.parametrize("Nnc", [GROUP, GROUP + 1, 2 * GROUP])
def test_chip_rate_group_boundaries(ctx, Nnc):
    """Exactly one group, one group and one block, exactly two groups."""
    snap, srch, _ = _case("1M023_%d" % Nnc, O.CPLX_I8, 1023000, 0.0, 1, Nnc, [27], [(27, 0.0)],
                          -500.0, 500.0, 500.0)
    grid, pk = _search(ctx, snap, srch)
    worst, _ = _check(snap, srch, grid, pk)
    log("group boundary, %d blocks: max mixed error %.3e" % (Nnc, worst))


CASES = [
    # name, fmt, fs, f_if, Tc, Nnc, prns, planted (prn, Doppler), lo, hi, step
    # four samples per chip: the group sums go to columns s + 4 q
    ("4M092_real_300", O.REAL_I8, 4092000, 1023000.0, 1, 300, [6, 25], [(25, -500.0)], -500.0, 500.0, 500.0),
    # two coherent milliseconds per block, a last group of one block
    ("2M046_T2_257", O.CPLX_I8, 2046000, 0.0, 2, 257, [9, 14], [(9, 250.0)], -250.0, 250.0, 250.0),
    # general rate, M = P = 4096
    ("2M_cplx_300", O.CPLX_I8, 2000000, 0.0, 1, 300, [4, 17], [(17, 500.0)], 0.0, 500.0, 500.0),
    # general rate, M = 32768 in two 16384-point halves
    ("10M_cplx_260", O.CPLX_I8, 10000000, 0.0, 1, 260, [21], [(21, -500.0)], -500.0, 0.0, 500.0),
    # general rate, M = N = 16384
    ("16M384_cplx_257", O.CPLX_I8, 16384000, 0.0, 1, 257, [24], [(24, 0.0)], 0.0, 500.0, 500.0),
]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_long_sum_matches_oracle(ctx, case):
    snap, srch, pl = _case(*case)
    N = snap.fs_hz // 1000
    log("long sum %s: fs=%d N=%d Tc=%d Nnc=%d" % (case[0], snap.fs_hz, N, srch.T_coh, srch.N_noncoh))
    grid, pk = _search(ctx, snap, srch)
    worst, exempt = _check(snap, srch, grid, pk)
    for p in pl:
        i = srch.prns.index(p.prn)
        assert pk[i]["detected"] and pk[i]["code_phase"] == p.code_phase, (p.prn, pk[i])
    log("  max mixed error %.3e, exemptions %d" % (worst, exempt))


class _DevReq:
    """Device buffers of one request; the grid is pre-filled with -1 so that
    a cell the first group's store missed would show."""

    def __init__(self, snap, srch):
        self.snap, self.srch = snap, srch
        self.shape = (len(srch.prns), O.n_doppler(srch.lo, srch.hi, srch.step), snap.fs_hz // 1000)
        self.x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
        self.grid = torch.full((int(np.prod(self.shape)),), -1.0, dtype=torch.float32, device="cuda")
        self.pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
        self.req = G.make_request(self.x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz,
                                  srch.prns, srch.lo, srch.hi, srch.step, srch.T_coh,
                                  srch.N_noncoh, self.grid.data_ptr(), self.pk.data_ptr())

    def clear(self):
        self.grid.fill_(-1.0)
        self.pk.zero_()

    def result(self):
        torch.cuda.synchronize()
        return (self.grid.cpu().numpy().reshape(self.shape).copy(),
                self.pk.cpu().numpy().view(G.PEAK_DTYPE).copy())


def test_long_and_short_requests_batched_and_captured(ctx):
    """Long (several groups) and short (one group) requests, chip-rate and
    general-rate, in one batch and in a graph replayed three times with
    eager work between: each equals its own search alone bit for bit."""
    items = [
        _case("1M023_600", O.CPLX_I8, 1023000, 0.0, 1, 600, [3, 11, 19], [(11, 500.0)], -500.0, 500.0, 500.0),
        _case("4M092_short", O.REAL_I8, 4092000, 1023000.0, 1, 4, [6, 25], [(25, -500.0)], -500.0, 500.0, 500.0),
        _case("2M_cplx_300", O.CPLX_I8, 2000000, 0.0, 1, 300, [4, 17], [(17, 500.0)], 0.0, 500.0, 500.0),
        _case("5M_short", O.CPLX_I8, 5000000, 0.0, 1, 3, [8], [(8, 0.0)], -500.0, 500.0, 500.0),
    ]
    reqs = [_DevReq(snap, srch) for snap, srch, _ in items]
    alone = []
    for r in reqs:
        ctx.acquire_device(r.req)
        alone.append(r.result())
    for r in reqs:
        r.clear()
    ctx.acquire_batch_device([r.req for r in reqs])
    for i, r in enumerate(reqs):
        g, p = r.result()
        assert np.array_equal(g, alone[i][0]) and np.array_equal(p, alone[i][1]), ("batch", i)
    graph = ctx.graph([r.req for r in reqs])
    try:
        stream = torch.cuda.current_stream()
        for rep in range(3):
            for r in reqs:
                r.clear()
            junk = torch.randn(1 << 20, device="cuda")
            (junk * 2.0).sum().item()
            log("long/short graph replay %d" % rep)
            graph.launch(stream)
            for i, r in enumerate(reqs):
                g, p = r.result()
                assert np.array_equal(g, alone[i][0]) and np.array_equal(p, alone[i][1]), (rep, i)
    finally:
        graph.close()
    snap, srch, _ = items[0]
    _check(snap, srch, alone[0][0], alone[0][1])


# the FP16 modes' derived bounds against the FP64 oracle (tests/test_gpu_fp16.py)
TOL16 = {"fp16": 3.4e-2, "fp16pfa": 2.0e-2}


@pytest.mark.parametrize("prec", ["fp16", "fp16pfa"])
def test_fp16_modes_long_sum(prec):
    """The FP16 modes keep plain running FP32 sums (their bounds are two
    orders above the summation error), over 600 blocks rescaled between
    block exponents: within the mode's bound, identical detections."""
    p = G.GNSS_FP16 if prec == "fp16" else G.GNSS_FP16_PFA
    snap, srch, pl = _case("1M023_600", O.CPLX_I8, 1023000, 0.0, 1, 600, [3, 11, 19], [(11, 500.0)],
                           -500.0, 500.0, 500.0)
    with G.Context(0, precision=p) as c:
        grid, pk = _search(c, snap, srch)
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.step,
                   nd, srch.T_coh, srch.N_noncoh)
    tol = TOL16[prec]
    worst = assert_grid_close(grid, P, tol)
    ref = O.peaks(P, srch.prns, O.chip_exclusion(snap.fs_hz), 2.5, srch.lo, srch.step)
    compare_detections(pk, ref, P, tie_rel=tol, value_rel=tol)
    i = srch.prns.index(11)
    assert pk[i]["detected"] and pk[i]["code_phase"] == pl[0].code_phase, pk[i]
    log("%s, 600 blocks: max mixed error %.3e" % (prec, worst))

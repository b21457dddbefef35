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
within the mixed tolerance, with identical detections.
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

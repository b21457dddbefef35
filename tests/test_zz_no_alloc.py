"""GPU tests of the allocation-free entry point (gnss_acquire_device_noalloc):
the same search as gnss_acquire_device with its workspace in the library's
static scratch array.  Its results must equal gnss_acquire_device's bit for
bit (same kernels, same arithmetic, same order), on consecutive calls whose
second is smaller than the first (the scratch keeps the previous call's
contents), in every precision; a long request whose one pass the scratch
cannot hold runs in passes over its blocks through the scratch; a request
too large for the scratch even so is refused with GNSS_ENOMEM and leaves
the context usable."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import assert_grid_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")

PRECISIONS = [G.GNSS_FP32, G.GNSS_FP16, G.GNSS_FP16_PFA]


def _small_case():
    """2.046 MHz packed 2-bit, 2 ms x 3 blocks, 3 PRNs x 3 bins: smaller than
    the strong-signal search in every dimension."""
    planted = [synth.Planted(prn=13, code_phase=901, doppler_hz=480.0, cn0_dbhz=50.0)]
    snap = synth.make_snapshot(77, synth.REAL_2BIT_PACKED, 2046000, 511500.0, 6.3, planted, O.ca_code)
    return snap, synth.Search([4, 13, 30], -500.0, 500.0, 500.0, 2, 3)


class Dev:
    def __init__(self, snap, srch, grid=True):
        self.snap, self.srch = snap, srch
        self.nd = O.n_doppler(srch.lo, srch.hi, srch.step)
        self.N = snap.fs_hz // 1000
        self.x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
        n = len(srch.prns) * self.nd * self.N
        self.grid = torch.full((n,), -1.0, dtype=torch.float32, device="cuda") if grid else None
        self.pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
        self.req = G.make_request(self.x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                                  srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                                  self.grid.data_ptr() if grid else 0, self.pk.data_ptr())

    def clear(self):
        if self.grid is not None:
            self.grid.fill_(-1.0)
        self.pk.zero_()

    def result(self):
        torch.cuda.synchronize()
        g = None
        if self.grid is not None:
            g = self.grid.cpu().numpy().reshape(len(self.srch.prns), self.nd, self.N).copy()
        return g, self.pk.cpu().numpy().view(G.PEAK_DTYPE).copy()


def _same_peaks(a, b):
    assert a.tobytes() == b.tobytes(), (a, b)


@pytest.mark.parametrize("prec", PRECISIONS, ids=["fp32", "fp16", "fp16pfa"])
def test_noalloc_equals_acquire_device_twice_second_smaller(prec, strong_case):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    snap, srch, nd, P = strong_case
    small_snap, small_srch = _small_case()
    with G.Context(0, precision=prec) as ctx:
        big = Dev(snap, srch)
        small = Dev(small_snap, small_srch)
        ref = {}
        for name, d in (("big", big), ("small", small)):
            ctx.acquire_device(d.req)
            ref[name] = d.result()
            d.clear()
        # the allocation-free calls: the strong-signal search, then a smaller one
        for name, d in (("big", big), ("small", small)):
            print("noalloc precision %d, %s request" % (prec, name), flush=True)
            ctx.acquire_device_noalloc(d.req)
            g, pk = d.result()
            assert np.array_equal(g, ref[name][0]), name
            _same_peaks(pk, ref[name][1])
            d.clear()
        # and the big one again after the small one, with the grid kept
        # internal (in the scratch): same peaks
        big_nogrid = Dev(snap, srch, grid=False)
        ctx.acquire_device_noalloc(big_nogrid.req)
        _, pk = big_nogrid.result()
        _same_peaks(pk, ref["big"][1])
    if prec == G.GNSS_FP32:
        # the FP32 result against the FP64 oracle (the library's usual bar)
        assert_grid_close(ref["big"][0], P)
        Ps = O.grid_direct(small_snap.samples, small_snap.fmt, small_snap.fs_hz, small_snap.f_if_hz,
                           small_srch.prns, small_srch.lo, small_srch.step,
                           O.n_doppler(small_srch.lo, small_srch.hi, small_srch.step),
                           small_srch.T_coh, small_srch.N_noncoh)
        assert_grid_close(ref["small"][0], Ps)


def test_noalloc_general_rate_equals_acquire_device():
    """General rates: the zero-padded FP32 transforms keep their block and
    code spectra in the same workspace.  A 10 MHz request (two 16384-point
    halves), then a smaller 2.5 MHz one (8192 points): bit for bit what
    gnss_acquire_device gives."""
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cases = []
    for seed, fs, prns, planted in ((81, 10000000, [6, 21, 30], (21, -500.0)), (82, 2500000, [9, 12], (12, 500.0))):
        pl = [synth.Planted(prn=planted[0], code_phase=1234, doppler_hz=planted[1], cn0_dbhz=50.0)]
        snap = synth.make_snapshot(seed, synth.CPLX_I8, fs, 0.0, 4.3, pl, O.ca_code)
        cases.append((snap, synth.Search(prns, -500.0, 500.0, 500.0, 2, 2)))
    with G.Context(0) as ctx:
        devs = [Dev(snap, srch) for snap, srch in cases]
        ref = []
        for d in devs:
            ctx.acquire_device(d.req)
            ref.append(d.result())
            d.clear()
        for i, d in enumerate(devs):
            print("noalloc general rate, request %d (fs %d)" % (i, d.snap.fs_hz), flush=True)
            ctx.acquire_device_noalloc(d.req)
            g, pk = d.result()
            assert np.array_equal(g, ref[i][0]), i
            _same_peaks(pk, ref[i][1])


def test_noalloc_refuses_oversize_request_and_allocates_nothing(strong_case):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    snap, srch, nd, P = strong_case
    weak, wsrch = synth.weak_complex_int8(O.ca_code, seed=2)
    with G.Context(0) as ctx:
        d = Dev(snap, srch)
        ctx.acquire_device(d.req)
        ref = d.result()
        d.clear()
        # the weak-signal search needs far more than the scratch holds
        big = Dev(weak, wsrch, grid=False)
        with pytest.raises(G.GnssError) as ei:
            ctx.acquire_device_noalloc(big.req)
        assert ei.value.code == G.GNSS_ENOMEM
        assert "scratch" in G.last_error()
        # the context still serves allocation-free calls, and they hold no new device memory
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for _ in range(3):
            ctx.acquire_device_noalloc(d.req)
            g, pk = d.result()
            assert np.array_equal(g, ref[0])
            _same_peaks(pk, ref[1])
            d.clear()
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_runs_a_long_request_in_passes():
    """A request whose one pass the scratch cannot hold (2000 blocks: about
    150 MB of workspace) but whose 256-block passes it can runs in passes
    through the scratch, equal to gnss_acquire_device bit for bit, with no
    new device memory; then a small request on the same scratch."""
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pl = [synth.Planted(prn=11, code_phase=345, doppler_hz=-500.0, cn0_dbhz=38.0)]
    snap = synth.make_snapshot(61, synth.CPLX_I8, 1023000, 0.0, 2000.25, pl, O.ca_code)
    srch = synth.Search([3, 11, 19], -500.0, 500.0, 500.0, 1, 2000)
    small_snap, small_srch = _small_case()
    with G.Context(0) as ctx:
        long_, small = Dev(snap, srch), Dev(small_snap, small_srch)
        ctx.acquire_device(long_.req)
        ref = long_.result()
        ctx.acquire_device(small.req)
        ref_small = small.result()
        long_.clear()
        small.clear()
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        ctx.acquire_device_noalloc(long_.req)
        g, pk = long_.result()
        assert np.array_equal(g, ref[0])
        _same_peaks(pk, ref[1])
        assert pk[1]["detected"] and pk[1]["code_phase"] == 345
        ctx.acquire_device_noalloc(small.req)
        g, pk = small.result()
        assert np.array_equal(g, ref_small[0])
        _same_peaks(pk, ref_small[1])
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_runs_a_long_general_rate_request_in_passes():
    """A 2 MHz request (4096-point zero-padded transforms, whose block and
    code spectra share the scratch) of 2000 blocks, which the scratch holds
    only in passes: equal to gnss_acquire_device bit for bit."""
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pl = [synth.Planted(prn=17, code_phase=1234, doppler_hz=500.0, cn0_dbhz=38.0)]
    snap = synth.make_snapshot(62, synth.CPLX_I8, 2000000, 0.0, 2000.25, pl, O.ca_code)
    srch = synth.Search([4, 17], 0.0, 1000.0, 500.0, 1, 2000)
    with G.Context(0) as ctx:
        d = Dev(snap, srch)
        ctx.acquire_device(d.req)
        ref = d.result()
        d.clear()
        ctx.acquire_device_noalloc(d.req)
        g, pk = d.result()
        assert np.array_equal(g, ref[0])
        _same_peaks(pk, ref[1])
        assert pk[1]["detected"] and pk[1]["code_phase"] == 1234

"""GPU tests of long requests run in passes over their blocks.

A request run alone whose workspace does not fit the context's HBM budget,
or any request under option block_window, runs in passes of a multiple of
256 blocks: each pass wipes, folds and transforms only its own blocks (at
their places in the record: sample positions, carrier phases and
code-Doppler shifts are the record's), adds its correlation sums to the
grid, and only the last pass detects.  In FP32 the result equals the
one-pass search bit for bit (the kernels group their block sums at the same
blocks, multiples of 256); the FP16 modes, whose running sums restart with
each pass, stay within their bounds against the oracle.
"""
import numpy as np
import pytest

import oracle as O
import synth
from parity import assert_grid_close, compare_detections, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")

GROUP = 256


def _case(name, fmt, fs, f_if, Tc, Nnc, prns, planted, lo, hi, step, cn0=40.0):
    rng = np.random.default_rng(sum(name.encode()))
    N = fs // 1000
    pl = [synth.Planted(prn=p, code_phase=int(rng.integers(0, N)), doppler_hz=dop, cn0_dbhz=cn0,
                        carrier_phase=float(rng.uniform(0, 2 * np.pi))) for p, dop in planted]
    snap = synth.make_snapshot(sum(name.encode()) % 977, fmt, fs, f_if, Tc * Nnc + 0.25, pl, O.ca_code)
    return snap, synth.Search(prns, lo, hi, step, Tc, Nnc), pl


def _search(c, snap, srch, want_grid=True, noalloc=False):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    d_x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
    d_grid = torch.full((len(srch.prns) * nd * N,), -1.0, dtype=torch.float32, device="cuda") if want_grid else None
    d_pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
    req = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                         srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                         d_grid.data_ptr() if want_grid else None, d_pk.data_ptr())
    if noalloc:
        c.acquire_device_noalloc(req, torch.cuda.current_stream())
    else:
        c.acquire_device(req, torch.cuda.current_stream())
    torch.cuda.synchronize()
    grid = d_grid.cpu().numpy().reshape(len(srch.prns), nd, N) if want_grid else None
    return grid, d_pk.cpu().numpy().view(G.PEAK_DTYPE).copy()


def _oracle(snap, srch, code_doppler=False):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.step,
                   nd, srch.T_coh, srch.N_noncoh, code_doppler=code_doppler)
    return P, O.peaks(P, srch.prns, O.chip_exclusion(snap.fs_hz), 2.5, srch.lo, srch.step)


CASES = [
    # name, fmt, fs, f_if, Tc, Nnc, prns, planted (prn, Doppler), lo, hi, step
    # chip rate, one sample per chip: passes of 256, 256 and 88 blocks
    ("1M023_cplx_600", O.CPLX_I8, 1023000, 0.0, 1, 600, [3, 11, 19], [(11, 500.0)], -500.0, 500.0, 500.0),
    # 2-bit packed real IF, four samples per chip, two coherent milliseconds
    ("4M092_packed_T2_300", O.REAL_2BIT_PACKED, 4092000, 1023000.0, 2, 300, [6, 25], [(25, -250.0)],
     -250.0, 250.0, 250.0),
    # general rates: a 4096-point transform; the 32768-point two-half split
    ("2M_cplx_300", O.CPLX_I8, 2000000, 0.0, 1, 300, [4, 17], [(17, 500.0)], 0.0, 500.0, 500.0),
    ("10M_cplx_260", O.CPLX_I8, 10000000, 0.0, 1, 260, [21], [(21, -500.0)], -500.0, 0.0, 500.0),
]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = G.Context(0)
    yield c
    c.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_passes_equal_one_pass(ctx, case):
    """Passes of 256 blocks against one pass: grid and peaks bit for bit
    (with a grid, and peaks alone with the grid kept in the workspace); the
    one-pass grid against the FP64 oracle."""
    snap, srch, pl = _case(*case)
    log("passes %s: Nnc=%d" % (case[0], srch.N_noncoh))
    one = _search(ctx, snap, srch)
    one_pk = _search(ctx, snap, srch, want_grid=False)[1]
    try:
        ctx.set("block_window", GROUP)
        many = _search(ctx, snap, srch)
        many_pk = _search(ctx, snap, srch, want_grid=False)[1]
    finally:
        ctx.set("block_window", 0)
    assert np.array_equal(many[0], one[0])
    assert np.array_equal(many[1], one[1]) and np.array_equal(many_pk, one_pk)
    assert np.array_equal(one_pk, one[1])
    P, ref = _oracle(snap, srch)
    worst = assert_grid_close(one[0], P)
    compare_detections(one[1], ref, P)
    for p in pl:
        i = srch.prns.index(p.prn)
        assert one[1][i]["detected"] and one[1][i]["code_phase"] == p.code_phase, (p.prn, one[1][i])
    log("  passes equal one pass; max mixed error %.3e" % worst)


@pytest.mark.parametrize("rate", ["chip", "general"])
def test_passes_with_code_doppler(ctx, rate):
    """Code-Doppler compensation over passes: each pass's shift table is
    built for its blocks' places in the record (chip rate: the polyphase
    path; 2 MHz: the zero-padded general-rate path)."""
    fs = 1023000 if rate == "chip" else 2000000
    snap, srch, _ = _case("cd_600_%s" % rate, O.CPLX_I8, fs, 0.0, 1, 600, [5, 13], [(13, 4000.0)],
                          3000.0, 5000.0, 1000.0)
    try:
        ctx.set("code_doppler", 1)
        one = _search(ctx, snap, srch)
        ctx.set("block_window", 2 * GROUP)
        many = _search(ctx, snap, srch)
    finally:
        ctx.set("block_window", 0)
        ctx.set("code_doppler", 0)
    assert np.array_equal(many[0], one[0]) and np.array_equal(many[1], one[1])
    P, ref = _oracle(snap, srch, code_doppler=True)
    assert_grid_close(one[0], P)
    compare_detections(one[1], ref, P)


@pytest.mark.timeout(300)
def test_budget_too_small_for_one_pass_runs_passes():
    """A context whose HBM budget cannot hold the request's one-pass
    workspace runs it in passes and returns what an unlimited context does."""
    snap, srch, pl = _case("1M023_budget_2000", O.CPLX_I8, 1023000, 0.0, 1, 2000, [3, 11, 19],
                           [(11, -500.0)], -500.0, 500.0, 500.0, cn0=38.0)
    with G.Context(0) as c:
        ref = _search(c, snap, srch)
    req = G.make_request(1, snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.hi,
                         srch.step, srch.T_coh, srch.N_noncoh, None, 1)
    need = G.gnss_workspace_bytes(req)
    budget = 64 << 20
    assert need > 2 * budget, need
    log("budget %d MiB for a request needing %.0f MiB in one pass" % (budget >> 20, need / 2 ** 20))
    with G.Context(0, hbm_budget_bytes=budget) as c:
        got = _search(c, snap, srch)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    P, oref = _oracle(snap, srch)
    assert_grid_close(got[0], P)
    compare_detections(got[1], oref, P)
    i = srch.prns.index(11)
    assert got[1][i]["detected"] and got[1][i]["code_phase"] == pl[0].code_phase


# the modes' derived bounds (tests/test_gpu_fp16.py, test_gpu_fd.py, test_gpu_nav_pairs.py)
TOL16 = {"fp16": 3.4e-2, "fp16pfa": 2.0e-2, "fp16pfa_fd": 2.3e-2, "fp16pfa_pairs": 2.1e-2}


@pytest.mark.parametrize("mode", ["fp16", "fp16pfa", "fp16pfa_fd", "fp16pfa_pairs"])
def test_fp16_modes_in_passes(mode):
    """The FP16 modes (and the exact-length options: frequency-domain
    Doppler, navigation-bit pairs) in passes of 256 blocks: within the
    mode's bound against the oracle, identical detections."""
    prec = G.GNSS_FP16 if mode == "fp16" else G.GNSS_FP16_PFA
    tol = TOL16[mode]
    snap, srch, pl = _case("1M023_h_600", O.CPLX_I8, 1023000, 0.0, 1, 600, [3, 11, 19], [(11, 500.0)],
                           -500.0, 500.0, 500.0)
    with G.Context(0, precision=prec) as c:
        if mode == "fp16pfa_fd":
            c.set("doppler_fd", 1)
        one = _search(c, snap, srch)
        c.set("block_window", GROUP)
        if mode == "fp16pfa_pairs":
            c.set("nav_pairs", 1)
            one = None
        many = _search(c, snap, srch)
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    if mode == "fp16pfa_fd":
        P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.step,
                       nd, srch.T_coh, srch.N_noncoh, carrier="exact")
    elif mode == "fp16pfa_pairs":
        P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.step,
                       nd, srch.T_coh, srch.N_noncoh, nav_pairs=True)
    else:
        P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.step,
                       nd, srch.T_coh, srch.N_noncoh)
    worst = assert_grid_close(many[0], P, tol)
    ref = O.peaks(P, srch.prns, O.chip_exclusion(snap.fs_hz), 2.5, srch.lo, srch.step)
    compare_detections(many[1], ref, P, tie_rel=tol, value_rel=tol)
    i = srch.prns.index(11)
    assert many[1][i]["detected"] and many[1][i]["code_phase"] == pl[0].code_phase
    if one is not None:
        # the same search in one pass: the same detections, grids within the bound of each other
        assert np.array_equal(many[1][["prn", "doppler_bin", "code_phase", "detected"]],
                              one[1][["prn", "doppler_bin", "code_phase", "detected"]])
    log("%s in passes: max mixed error %.3e" % (mode, worst))


def test_block_window_option_is_checked(ctx):
    for bad in (100, -256, 256.5, 3 * GROUP + 1):
        with pytest.raises(G.GnssError) as ei:
            ctx.set("block_window", bad)
        assert ei.value.code == G.GNSS_EINVAL
    for good in (0, GROUP, 4 * GROUP, 0):
        ctx.set("block_window", good)


def _host_request(snap, srch):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    grid = np.full((len(srch.prns), nd, snap.fs_hz // 1000), -1.0, np.float32)
    pk = np.zeros(len(srch.prns), G.PEAK_DTYPE)
    x = np.ascontiguousarray(snap.samples)
    req = G.make_request(x.ctypes.data, snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                         srch.hi, srch.step, srch.T_coh, srch.N_noncoh, grid.ctypes.data, pk.ctypes.data)
    return req, x, grid, pk


@pytest.mark.timeout(300)
def test_served_long_request_runs_in_passes():
    """A submitted request whose one pass exceeds a batch slot's share of
    the budget (a 160 MiB budget: shares of about 75 MiB; the request needs
    about 150 MB in one pass) runs alone in passes, between small requests
    served in batches: every result equals its one-pass search bit for bit."""
    snap, srch, _ = _case("1M023_serve_2000", O.CPLX_I8, 1023000, 0.0, 1, 2000, [3, 11, 19], [(11, 500.0)],
                          -500.0, 500.0, 500.0, cn0=38.0)
    smalls = [_case("1M023_small_%d" % i, O.CPLX_I8, 1023000, 0.0, 1, 4, [7, 9], [(9, 0.0)],
                    -500.0, 500.0, 500.0, cn0=48.0) for i in range(4)]
    with G.Context(0) as c:
        ref = _search(c, snap, srch)
        ref_small = [_search(c, s, q) for s, q, _ in smalls]
    with G.Context(0, hbm_budget_bytes=160 << 20) as sc:
        subs = []
        for k, (s, q, _) in enumerate(smalls):
            if k == 2:
                big = _host_request(snap, srch)
                subs.append(("long", sc.submit(big[0]), big))
            h = _host_request(s, q)
            subs.append((k, sc.submit(h[0]), h))
        for k, t, h in subs:
            info = sc.wait(t, 120.0)
            want = ref if k == "long" else ref_small[k]
            assert np.array_equal(h[2], want[0]), k
            assert h[3].tobytes() == want[1].tobytes(), k
            if k == "long":
                assert info.batch_size == 1
    log("served long request in passes equals its one-pass search")


def _dev_request(snap, srch):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
    grid = torch.full((len(srch.prns) * nd * N,), -1.0, dtype=torch.float32, device="cuda")
    pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
    req = G.make_request(x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.hi,
                         srch.step, srch.T_coh, srch.N_noncoh, grid.data_ptr(), pk.data_ptr())
    return req, x, grid.view(len(srch.prns), nd, N), pk


@pytest.mark.timeout(300)
def test_batch_that_does_not_fit_runs_its_long_request_in_passes():
    """A batch under a 64 MiB budget holding a 2000-block request (about
    150 MB in one pass) between three small ones: the long one runs alone in
    passes, the others as one batch; every result equals its search alone on
    an unlimited context bit for bit."""
    long_ = _case("1M023_budget_2000", O.CPLX_I8, 1023000, 0.0, 1, 2000, [3, 11, 19], [(11, -500.0)],
                  -500.0, 500.0, 500.0, cn0=38.0)
    smalls = [_case("1M023_bsmall_%d" % i, O.CPLX_I8, 1023000, 0.0, 1, 4, [7, 9], [(9, 0.0)],
                    -500.0, 500.0, 500.0, cn0=48.0) for i in range(3)]
    items = [smalls[0], long_, smalls[1], smalls[2]]
    with G.Context(0) as c:
        refs = [_search(c, s, q) for s, q, _ in items]
    with G.Context(0, hbm_budget_bytes=64 << 20) as c:
        devs = [_dev_request(s, q) for s, q, _ in items]
        c.acquire_batch_device([d[0] for d in devs], torch.cuda.current_stream())
        torch.cuda.synchronize()
        for i, d in enumerate(devs):
            assert np.array_equal(d[2].cpu().numpy(), refs[i][0]), i
            assert d[3].cpu().numpy().tobytes() == refs[i][1].tobytes(), i
    log("batch with a long request under a 64 MiB budget equals the requests alone")


def test_a_failed_pass_fails_the_call_and_leaves_the_context_usable(ctx):
    """The second of three passes fails on the host (failure injection): the
    call reports GNSS_EDEVICE, and the next search on the context, again in
    passes, equals the one-pass search bit for bit."""
    snap, srch, _ = _case(*CASES[0])
    ref = _search(ctx, snap, srch)
    try:
        ctx.set("block_window", GROUP)
        ctx.set("fault_launch", 2)
        with pytest.raises(G.GnssError) as ei:
            _search(ctx, snap, srch)
        assert ei.value.code == G.GNSS_EDEVICE
        torch.cuda.synchronize()
        got = _search(ctx, snap, srch)
    finally:
        ctx.set("fault_launch", 0)
        ctx.set("block_window", 0)
    assert np.array_equal(got[0], ref[0]) and got[1].tobytes() == ref[1].tobytes()


@pytest.mark.timeout(300)
def test_a_failed_pass_fails_only_its_served_ticket():
    """Served: the long request's second pass fails (failure injection); its
    ticket reports the error, and the next ticket, the same request, equals
    its one-pass search."""
    snap, srch, _ = _case("1M023_serve_2000", O.CPLX_I8, 1023000, 0.0, 1, 2000, [3, 11, 19], [(11, 500.0)],
                          -500.0, 500.0, 500.0, cn0=38.0)
    with G.Context(0) as c:
        ref = _search(c, snap, srch)
    with G.Context(0, hbm_budget_bytes=160 << 20) as sc:
        sc.set("fault_launch", 2)
        bad = _host_request(snap, srch)
        with pytest.raises(G.GnssError) as ei:
            sc.wait(sc.submit(bad[0]), 120.0)
        assert ei.value.code == G.GNSS_EDEVICE and "injected" in str(ei.value)
        good = _host_request(snap, srch)
        info = sc.wait(sc.submit(good[0]), 120.0)
        assert info.status == 0
        assert np.array_equal(good[2], ref[0]) and good[3].tobytes() == ref[1].tobytes()

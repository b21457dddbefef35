"""GPU tests of the batched, captured and served forms of the search.

Each request's result must be the same whatever batch it runs in: the
kernels do the same arithmetic in the same order for a (request, PRN,
Doppler, phase) regardless of how work is tiled or scheduled, so batch,
graph, served and alone results are compared bit for bit; each is also
checked against the FP64 oracle to the usual tolerance.
"""
import os
import threading
import time

import numpy as np
import pytest

import oracle as O
import synth
from parity import assert_grid_close, compare_detections, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = G.Context(0)
    yield c
    c.close()


def _shape(snap, srch):
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    return len(srch.prns), nd, snap.fs_hz // 1000


class DevReq:
    """Device buffers of one request."""

    def __init__(self, snap, srch):
        self.snap, self.srch = snap, srch
        n_prn, nd, N = _shape(snap, srch)
        self.x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
        self.grid = torch.full((n_prn * nd * N,), -1.0, dtype=torch.float32, device="cuda")
        self.pk = torch.zeros(n_prn * 48, dtype=torch.uint8, device="cuda")
        self.req = G.make_request(self.x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz,
                                  srch.prns, srch.lo, srch.hi, srch.step, srch.T_coh,
                                  srch.N_noncoh, self.grid.data_ptr(), self.pk.data_ptr())

    def clear(self):
        self.grid.fill_(-1.0)
        self.pk.zero_()

    def result(self):
        torch.cuda.synchronize()
        n_prn, nd, N = _shape(self.snap, self.srch)
        return (self.grid.cpu().numpy().reshape(n_prn, nd, N).copy(),
                self.pk.cpu().numpy().view(G.PEAK_DTYPE).copy())


def _small_batch(n=10, seed=41):
    return synth.batch_workload(O.ca_code, seed=seed, n=n, ms_range=(4, 12), prn_range=(3, 9),
                                window_khz=(1.0, 3.0), planted_range=(1, 2), cn0_range=(44.0, 48.0))


@pytest.fixture(scope="module")
def small(ctx):
    items = _small_batch()
    reqs = [DevReq(s, q) for s, q in items]
    alone = []
    for r in reqs:
        ctx.acquire_device(r.req)
        alone.append(r.result())
    return items, reqs, alone


def test_batch_equals_alone_and_oracle(ctx, small):
    items, reqs, alone = small
    for r in reqs:
        r.clear()
    log("batch of %d heterogeneous requests" % len(reqs))
    ctx.acquire_batch_device([r.req for r in reqs])
    for i, r in enumerate(reqs):
        g, p = r.result()
        assert np.array_equal(g, alone[i][0]), i
        assert np.array_equal(p, alone[i][1]), i
    for i, (snap, srch) in enumerate(items[:4]):
        nd = O.n_doppler(srch.lo, srch.hi, srch.step)
        P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                       srch.step, nd, srch.T_coh, srch.N_noncoh)
        assert_grid_close(alone[i][0], P)
        ref = O.peaks(P, srch.prns, snap.fs_hz // 1023000, 2.5, srch.lo, srch.step)
        compare_detections(alone[i][1], ref, P)


def test_tile_and_schedule_do_not_change_results(ctx, small):
    items, reqs, alone = small
    try:
        # FP32 shapes (PRN tile, waves per workgroup): tile 1 at three waves per SIMD
        # with 12, 6 or 4 waves per workgroup, tiles 2 and 4 with 8
        for pt, w in ((1, 12), (1, 6), (1, 4), (2, 8), (4, 8)):
            for sched in (0, 1):
                ctx.set("corr_ptile", pt)
                ctx.set("corr_waves", w)
                ctx.set("persistent", sched)
                for r in reqs:
                    r.clear()
                ctx.acquire_batch_device([r.req for r in reqs])
                for i, r in enumerate(reqs):
                    g, p = r.result()
                    assert np.array_equal(g, alone[i][0]) and np.array_equal(p, alone[i][1]), (pt, sched, i)
    finally:
        ctx.set("corr_ptile", 0)
        ctx.set("corr_waves", 0)
        ctx.set("persistent", -1)


def test_graph_replays_match_eager(ctx, small):
    items, reqs, alone = small
    graph = ctx.graph([r.req for r in reqs])
    try:
        stream = torch.cuda.current_stream()
        for rep in range(3):
            for r in reqs:
                r.clear()
            # unrelated eager work between replays
            junk = torch.randn(1 << 20, device="cuda")
            (junk * 2.0).sum().item()
            log("graph replay %d" % rep)
            graph.launch(stream)
            for i, r in enumerate(reqs):
                g, p = r.result()
                assert np.array_equal(g, alone[i][0]) and np.array_equal(p, alone[i][1]), (rep, i)
    finally:
        graph.close()


def test_autotune_and_cache(ctx, small, tmp_path):
    items, reqs, alone = small
    path = str(tmp_path / "tune.txt")
    pt, sched = ctx.autotune([r.req for r in reqs], path)
    assert pt in (1, 2, 4) and sched in (0, 1)
    # "key tile schedule waves"
    words = open(path).read().split()
    assert os.path.exists(path) and words[-3:-1] == [str(pt), str(sched)] and int(words[-1]) in (4, 6, 8, 12)
    assert ctx.autotune([r.req for r in reqs], path) == (pt, sched)  # from the cache
    for r in reqs:
        r.clear()
    ctx.acquire_batch_device([r.req for r in reqs])
    for i, r in enumerate(reqs):
        g, p = r.result()
        assert np.array_equal(g, alone[i][0]) and np.array_equal(p, alone[i][1])


def _host_request(snap, srch, want_grid=True):
    n_prn, nd, N = _shape(snap, srch)
    grid = np.full((n_prn, nd, N), -1.0, np.float32) if want_grid else None
    pk = np.zeros(n_prn, G.PEAK_DTYPE)
    x = np.ascontiguousarray(snap.samples)
    req = G.make_request(x.ctypes.data, snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                         srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                         grid.ctypes.data if want_grid else None, pk.ctypes.data)
    return req, x, grid, pk


def test_serving_results_equal_alone(small):
    items, reqs, alone = small
    with G.Context(0) as sctx:
        sub = []
        for i, (snap, srch) in enumerate(items):
            req, x, grid, pk = _host_request(snap, srch, want_grid=(i % 2 == 0))
            t = sctx.submit(req)
            del x  # the library copied the samples
            sub.append((i, t, grid, pk, req))
            time.sleep(0.002 * (i % 3))
        sizes = []
        for i, t, grid, pk, req in sub:
            info = sctx.wait(t, 60.0)
            assert info.status == 0
            sizes.append(info.batch_size)
            assert np.array_equal(pk, alone[i][1]), i
            if grid is not None:
                assert np.array_equal(grid, alone[i][0]), i
            assert info.total_s >= info.run_s >= 0.0
        log("served batch sizes %s" % sizes)


def test_serving_admission_under_tight_budget(small):
    items, reqs, alone = small
    # room for about two requests per batch slot: the rest must queue
    need = max(G.gnss_workspace_bytes(r.req) for r in reqs)
    with G.Context(0, hbm_budget_bytes=int(4.5 * need) + (8 << 20)) as sctx:
        tickets = []
        keep = []
        for i, (snap, srch) in enumerate(items):
            req, x, grid, pk = _host_request(snap, srch, want_grid=False)
            tickets.append((i, sctx.submit(req), pk))
            keep.append((x, pk, req))
        sizes = []
        for i, t, pk in tickets:
            info = sctx.wait(t, 60.0)
            sizes.append(info.batch_size)
            assert np.array_equal(pk, alone[i][1]), i
        assert max(sizes) < len(items)  # admission split the queue into several batches
        log("budgeted batch sizes %s" % sizes)
        # a request alone larger than a slot's share is refused
        big_snap, big_srch = synth.weak_complex_int8(O.ca_code, seed=9)
        req, x, grid, pk = _host_request(big_snap, big_srch, want_grid=False)
        with pytest.raises(G.GnssError) as ei:
            sctx.submit(req)
        assert ei.value.code == G.GNSS_ENOMEM


def test_serving_from_threads(small):
    items, reqs, alone = small
    errors = []
    with G.Context(0) as sctx:
        def client(idx):
            try:
                snap, srch = items[idx]
                req, x, grid, pk = _host_request(snap, srch, want_grid=True)
                t = sctx.submit(req)
                info = sctx.wait(t, 60.0)
                assert info.status == 0
                assert np.array_equal(pk, alone[idx][1]) and np.array_equal(grid, alone[idx][0])
            except Exception as e:  # noqa: BLE001
                errors.append((idx, repr(e)))
        th = [threading.Thread(target=client, args=(i,)) for i in range(len(items))]
        for t in th:
            t.start()
        for t in th:
            t.join()
    assert not errors, errors


@pytest.mark.timeout(600)
def test_medium_batch_matches_oracle(ctx):
    """48 heterogeneous requests (20-60 ms, all three rates, both formats) in
    one batch.  For every planted PRN the grid row must match the FP64 oracle
    and the detection must be the oracle's; at these C/N0 (30-45 dB-Hz) with
    1 ms coherent blocks many weak satellites fall below the ratio test, so
    the recovered count is compared with the oracle's, not with a fixed rate."""
    items = synth.batch_workload(O.ca_code, seed=4, n=48, ms_range=(20, 60))
    reqs = [DevReq(s, q) for s, q in items]
    log("batch of 48 requests, 20-60 ms, all three rates")
    ctx.acquire_batch_device([r.req for r in reqs])
    found_gpu = found_ref = total = exempt = 0
    worst = 0.0
    for i, r in enumerate(reqs):
        g, p = r.result()
        snap, srch = items[i]
        planted = {pl.prn: pl for pl in snap.planted}
        prns = sorted(planted)
        rows = [srch.prns.index(prn) for prn in prns]
        nd = O.n_doppler(srch.lo, srch.hi, srch.step)
        P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, prns, srch.lo,
                       srch.step, nd, srch.T_coh, srch.N_noncoh)
        worst = max(worst, assert_grid_close(g[rows], P))
        ref = O.peaks(P, prns, snap.fs_hz // 1023000, 2.5, srch.lo, srch.step)
        exempt += compare_detections(p[rows], ref, P)
        for j, prn in enumerate(prns):
            total += 1
            found_ref += bool(ref[j].detected and ref[j].code_phase == planted[prn].code_phase)
            gj = p[rows[j]]
            found_gpu += bool(gj["detected"] and int(gj["code_phase"]) == planted[prn].code_phase)
    log("planted recovered: gpu %d, oracle %d of %d; max grid err %.2e; %d near-tie exemptions"
        % (found_gpu, found_ref, total, worst, exempt))
    assert abs(found_gpu - found_ref) <= exempt
    assert found_ref >= total // 2
    # a few requests alone are bit-identical to their batched results
    for i in (0, 17, 47):
        g, p = reqs[i].result()
        reqs[i].clear()
        ctx.acquire_device(reqs[i].req)
        g2, p2 = reqs[i].result()
        assert np.array_equal(g, g2) and np.array_equal(p, p2)


def test_serving_budget_holds_across_alternating_shapes():
    # Two request shapes whose largest buffers differ (A: a large grid; B: long
    # records, large forward spectra).  A slot's share of the budget fits either one
    # but not the per-buffer maxima of both; with both slots busy every ticket must
    # still succeed (each slot resizes within its share) and match the result alone.
    a_snap, a_srch = synth.weak_complex_int8(O.ca_code, seed=21)
    a_srch = synth.Search(a_srch.prns, a_srch.lo, a_srch.hi, a_srch.step, 1, 4)
    b_snap = synth.make_snapshot(22, O.REAL_I8, 4092000, 1023000.0, 200.0,
                                 [synth.Planted(prn=3, code_phase=1000, doppler_hz=1500.0, cn0_dbhz=45.0)],
                                 O.ca_code)
    b_srch = synth.Search([3, 4, 5, 6, 7, 8, 9, 10], -5000.0, 5000.0, 500.0, 1, 200)
    shapes = [(a_snap, a_srch, True), (b_snap, b_srch, False)]
    needs = []
    for snap, srch, grid in shapes:
        req, x, g, pk = _host_request(snap, srch, want_grid=grid)
        needs.append(G.gnss_workspace_bytes(req) + (g.nbytes if grid else 0))
    share = int(1.15 * max(needs))
    alone = []
    with G.Context(0) as c1:
        for snap, srch, grid in shapes:
            req, x, g, pk = _host_request(snap, srch, want_grid=grid)
            t = c1.submit(req)
            assert c1.wait(t, 120.0).status == 0
            alone.append((g.copy() if grid else None, pk.copy()))
    log("alternating shapes: needs %s, slot share %d" % (needs, share))
    with G.Context(0, hbm_budget_bytes=2 * share + (8 << 20)) as sctx:
        subs = []
        for i in range(8):
            snap, srch, grid = shapes[i % 2]
            req, x, g, pk = _host_request(snap, srch, want_grid=grid)
            subs.append((i % 2, sctx.submit(req), g, pk, x, req))
        for k, t, g, pk, x, req in subs:
            info = sctx.wait(t, 120.0)
            assert info.status == 0, G.last_error()
            assert np.array_equal(pk, alone[k][1])
            if g is not None:
                assert np.array_equal(g, alone[k][0])

"""The exact-length mode and its two options (frequency-domain Doppler,
navigation-bit pairs) through every batched entry point: a batch, every PRN
tile and correlation schedule, graph replays with eager work between them,
the autotuner and the serving loop all give bit-identical results to single
requests on the same context configuration."""
import os

import numpy as np
import pytest

import oracle as O
import synth
from parity import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")

MODES = [("pfa", {}), ("pfa_fd", {"doppler_fd": 1}), ("pfa_pairs", {"nav_pairs": 1})]


def _items(pairs):
    items = synth.batch_workload(O.ca_code, seed=45, n=8, ms_range=(4, 12), prn_range=(3, 8),
                                 window_khz=(1.0, 3.0), planted_range=(1, 2), cn0_range=(44.0, 48.0))
    if pairs:  # even block counts
        items = [(snap, synth.Search(srch.prns, srch.lo, srch.hi, srch.step, srch.T_coh,
                                     max(2, srch.N_noncoh - srch.N_noncoh % 2))) for snap, srch in items]
    return items


class DevReq:
    def __init__(self, snap, srch):
        self.snap, self.srch = snap, srch
        nd = O.n_doppler(srch.lo, srch.hi, srch.step)
        self.shape = (len(srch.prns), nd, snap.fs_hz // 1000)
        self.x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
        self.grid = torch.full((int(np.prod(self.shape)),), -1.0, dtype=torch.float32, device="cuda")
        self.pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
        self.req = G.make_request(self.x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                                  srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                                  self.grid.data_ptr(), self.pk.data_ptr())

    def clear(self):
        self.grid.fill_(-1.0)
        self.pk.zero_()

    def result(self):
        torch.cuda.synchronize()
        return (self.grid.cpu().numpy().reshape(self.shape).copy(),
                self.pk.cpu().numpy().view(G.PEAK_DTYPE).copy())


def _ctx(opts):
    c = G.Context(0, precision=G.GNSS_FP16_PFA)
    for k, v in opts.items():
        c.set(k, v)
    return c


@pytest.mark.parametrize("mode", MODES, ids=[m[0] for m in MODES])
def test_mode_batch_graph_autotune_serving_equal_alone(mode, tmp_path):
    name, opts = mode
    items = _items("nav_pairs" in opts)
    ctx = _ctx(opts)
    try:
        reqs = [DevReq(s, q) for s, q in items]
        alone = []
        for r in reqs:
            ctx.acquire_device(r.req)
            alone.append(r.result())
        log("%s: batch of %d" % (name, len(reqs)))

        def check(tag):
            for i, r in enumerate(reqs):
                g, p = r.result()
                assert np.array_equal(g, alone[i][0]) and np.array_equal(p, alone[i][1]), (tag, i)

        for r in reqs:
            r.clear()
        ctx.acquire_batch_device([r.req for r in reqs])
        check("batch")
        for pt in (2, 4):
            for sched in (0, 1):
                ctx.set("corr_ptile", pt)
                ctx.set("persistent", sched)
                for r in reqs:
                    r.clear()
                ctx.acquire_batch_device([r.req for r in reqs])
                check(("tile", pt, sched))
        ctx.set("corr_ptile", 0)
        ctx.set("persistent", -1)
        graph = ctx.graph([r.req for r in reqs])
        try:
            for rep in range(3):
                for r in reqs:
                    r.clear()
                junk = torch.randn(1 << 20, device="cuda")
                (junk * 2.0).sum().item()
                graph.launch(torch.cuda.current_stream())
                check(("graph", rep))
        finally:
            graph.close()
        path = str(tmp_path / "tune.txt")
        pt, sched = ctx.autotune([r.req for r in reqs], path)
        assert pt in (2, 4) and sched in (0, 1) and os.path.exists(path)
        for r in reqs:
            r.clear()
        ctx.acquire_batch_device([r.req for r in reqs])
        check("tuned")
    finally:
        ctx.close()
    # serving on a context with the same configuration
    sctx = _ctx(opts)
    try:
        sub = []
        for i, (snap, srch) in enumerate(items):
            grid = np.full(reqs[i].shape, -1.0, np.float32)
            pk = np.zeros(len(srch.prns), G.PEAK_DTYPE)
            x = np.ascontiguousarray(snap.samples)
            req = G.make_request(x.ctypes.data, snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                                 srch.hi, srch.step, srch.T_coh, srch.N_noncoh, grid.ctypes.data, pk.ctypes.data)
            sub.append((i, sctx.submit(req), grid, pk, x, req))
        for i, t, grid, pk, x, req in sub:
            assert sctx.wait(t, 60.0).status == 0
            assert np.array_equal(grid, alone[i][0]) and np.array_equal(pk, alone[i][1]), ("serve", i)
    finally:
        sctx.close()

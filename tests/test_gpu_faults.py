"""Error paths of the device-buffer and served forms, forced from the host.

The context options "fault_alloc", "fault_copy" and "fault_launch" make the
n-th following device allocation, copy or batch launch fail on the host
before anything is enqueued, so no kernel faults: what is tested is that the
failure is reported to the affected request only and that the context keeps
serving the others with unchanged results (a device error fails only the
tickets of the batch it occurred in).  Also: destroying a serving context
returns its device memory.
"""
import numpy as np
import pytest

import oracle as O
import synth
from parity import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")


def _items(n=6, seed=77):
    return synth.batch_workload(O.ca_code, seed=seed, n=n, ms_range=(4, 10), prn_range=(3, 8),
                                window_khz=(1.0, 2.0), planted_range=(1, 2), cn0_range=(44.0, 48.0))


def _host_request(snap, srch):
    x = np.ascontiguousarray(snap.samples)
    pk = np.zeros(len(srch.prns), G.PEAK_DTYPE)
    req = G.make_request(x.ctypes.data, snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                         srch.hi, srch.step, srch.T_coh, srch.N_noncoh, 0, pk.ctypes.data)
    return req, x, pk


def _device_result(ctx, snap, srch):
    x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
    pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
    req = G.make_request(x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                         srch.hi, srch.step, srch.T_coh, srch.N_noncoh, 0, pk.data_ptr())
    ctx.acquire_device(req, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return pk.cpu().numpy().view(G.PEAK_DTYPE).copy()


@pytest.fixture(scope="module")
def alone():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    items = _items()
    with G.Context(0) as c:
        res = [_device_result(c, s, q) for s, q in items]
    return items, res


@pytest.mark.parametrize("option,nth,code", [("fault_launch", 3, G.GNSS_EDEVICE),
                                             ("fault_copy", 1, G.GNSS_EDEVICE),
                                             ("fault_alloc", 1, G.GNSS_ENOMEM)])
def test_served_failure_fails_only_its_ticket(alone, option, nth, code):
    items, res = alone
    with G.Context(0) as sctx:
        sctx.set("max_slots", 1)  # one request per batch: the n-th batch is the n-th ticket
        sctx.set(option, nth)
        log("serving with %s = %d" % (option, nth))
        subs = []
        for snap, srch in items:
            req, x, pk = _host_request(snap, srch)
            subs.append((sctx.submit(req), req, x, pk))
        failed = []
        for i, (t, req, x, pk) in enumerate(subs):
            try:
                info = sctx.wait(t, 60.0)
                assert info.status == 0
                assert np.array_equal(pk, res[i]), i
            except G.GnssError as e:
                assert e.code == code, (i, e)
                assert "injected" in str(e)
                failed.append(i)
        assert failed == [nth - 1], failed
        # the context keeps serving after the failure
        snap, srch = items[0]
        req, x, pk = _host_request(snap, srch)
        assert sctx.wait(sctx.submit(req), 60.0).status == 0
        assert np.array_equal(pk, res[0])


def test_device_call_failures_leave_the_context_usable(alone):
    items, res = alone
    snap, srch = items[1]
    with G.Context(0) as c:
        c.set("fault_alloc", 1)
        with pytest.raises(G.GnssError) as ei:
            _device_result(c, snap, srch)
        assert ei.value.code == G.GNSS_ENOMEM
        assert np.array_equal(_device_result(c, snap, srch), res[1])
        c.set("fault_launch", 1)
        with pytest.raises(G.GnssError) as ei:
            _device_result(c, snap, srch)
        assert ei.value.code == G.GNSS_EDEVICE
        assert np.array_equal(_device_result(c, snap, srch), res[1])
    with pytest.raises(G.GnssError):
        with G.Context(0) as c:
            c.set("fault_launch", -1)


@pytest.mark.timeout(300)
def test_destroying_a_serving_context_returns_its_memory():
    """A served weak-signal request grows a batch slot's arena to ~1.5 GB;
    destroying the context must free it (and its tables)."""
    snap, srch = synth.weak_complex_int8(O.ca_code, seed=2)
    req, x, pk = _host_request(snap, srch)
    need = G.gnss_workspace_bytes(req)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for it in range(3):
        with G.Context(0) as sctx:
            assert sctx.wait(sctx.submit(req), 120.0).status == 0
            free_in, _ = torch.cuda.mem_get_info()
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        log("iteration %d: free %.2f GB before, %.2f GB while serving, %.2f GB after (request needs %.2f GB)"
            % (it, free0 / 1e9, free_in / 1e9, free1 / 1e9, need / 1e9))
        assert free0 - free_in >= need // 2  # the arena really was allocated
        assert free0 - free1 < (256 << 20), (free0, free1)

"""GPU tests of the navigation-bit hypotheses (option nav_pairs, exact-length
contexts): coherent blocks combined in pairs with both relative signs, the
larger power kept.  Reference: the oracle's pair route (grid_fft(nav_pairs=
True), pinned in test_oracle_nav_pairs.py); tolerance: the exact-length
mode's bound (the pair sum G_a 2^(ea-e) +- G_b 2^(eb-e) adds one FP16
rounding: eta ~ sqrt(12) u, TOL = 2 * 6 * eta = 2.1e-2)."""
import numpy as np
import pytest

import oracle as O
import synth
from parity import compare_detections, grid_error, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")

TOLP = 2.1e-2


@pytest.fixture(scope="module")
def ctxp():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = G.Context(0, precision=G.GNSS_FP16_PFA)
    c.set("nav_pairs", 1)
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


def _check(grid, pk, P, srch, spc):
    assert np.all(np.isfinite(grid))
    worst = grid_error(grid, P)
    ref = O.peaks(P, srch.prns, spc, 2.5, srch.lo, srch.step)
    exempt = compare_detections(pk, ref, P, tie_rel=TOLP, value_rel=TOLP)
    log("  pairs vs FP64: max mixed error %.3e, near-tie exemptions %d" % (worst, exempt))
    assert worst <= TOLP, worst


CASES = [
    # name, fmt, fs, f_if, Tc, Nnc, prns, lo, hi, step, code_doppler, doppler_fd
    ("spc1_cplx", O.CPLX_I8, 1023000, 0.0, 1, 4, [3, 9], -1000.0, 1000.0, 500.0, False, False),
    ("spc4_real_cd", O.REAL_I8, 4092000, 1023000.0, 2, 4, [2, 4, 10], -1500.0, 1500.0, 250.0, True, False),
    ("spc16_cplx", O.CPLX_I8, 16368000, 0.0, 1, 2, [11, 31], -500.0, 500.0, 500.0, False, False),
    ("spc8_fd", O.CPLX_I8, 8184000, 0.0, 2, 4, [7, 30], -500.0, 500.0, 250.0, False, True),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pairs_match_oracle(ctxp, case):
    name, fmt, fs, f_if, Tc, Nnc, prns, lo, hi, step, cd, fd = case
    nd = O.n_doppler(lo, hi, step)
    rng = np.random.default_rng(sum(name.encode()) % 1000)
    N = fs // 1000
    pl = [synth.Planted(prn=prns[0], code_phase=int(rng.integers(0, N)), doppler_hz=lo + step * (nd // 2),
                        cn0_dbhz=46.0, nav_bits=True, nav_phase_ms=int(rng.integers(0, 20)))]
    snap = synth.make_snapshot(sum(name.encode()) % 997, fmt, fs, f_if, Tc * Nnc + 0.5, pl, O.ca_code)
    srch = synth.Search(prns, lo, hi, step, Tc, Nnc)
    log("pairs %s: fs=%d bins=%d Tc=%d Nnc=%d code_doppler=%d doppler_fd=%d" % (name, fs, nd, Tc, Nnc, cd, fd))
    ctxp.set("code_doppler", int(cd))
    ctxp.set("doppler_fd", int(fd))
    try:
        grid, pk = _run(ctxp, snap, srch)
    finally:
        ctxp.set("code_doppler", 0)
        ctxp.set("doppler_fd", 0)
    P = O.grid_fft(snap.samples, fmt, fs, f_if, prns, lo, step, nd, Tc, Nnc, code_doppler=cd,
                   carrier="exact" if fd else "nco", nav_pairs=True)
    _check(grid, pk, P, srch, fs // 1023000)


def test_pairs_recover_coherent_gain_across_bit_flips(ctxp):
    # 20 ms coherent blocks over data bits whose edges fall at the blocks' code
    # epochs: the pairs integrate 40 ms coherently whatever the bits, so the
    # planted cell stands higher above the noise floor than with the plain sum
    fs, Tc, Nnc = 4092000, 20, 10
    N = fs // 1000
    step, nd = 25.0, 9
    lo = -100.0
    pl = [synth.Planted(prn=17, code_phase=321, doppler_hz=lo + 4 * step, cn0_dbhz=30.0, nav_bits=True,
                        nav_phase_ms=0)]
    snap = synth.make_snapshot(29, O.CPLX_I8, fs, 0.0, Tc * Nnc + 1.0, pl, O.ca_code)
    srch = synth.Search([17, 3, 25], lo, lo + (nd - 1) * step, step, Tc, Nnc)
    grid_p, pk_p = _run(ctxp, snap, srch)
    P = O.grid_fft(snap.samples, snap.fmt, fs, 0.0, srch.prns, lo, step, nd, Tc, Nnc, nav_pairs=True)
    _check(grid_p, pk_p, P, srch, 4)
    with G.Context(0, precision=G.GNSS_FP16_PFA) as plain:
        grid_s, pk_s = _run(plain, snap, srch)
    cell = (0, 4, 321)
    rise_p = grid_p[cell] / grid_p[0].mean()
    rise_s = grid_s[cell] / grid_s[0].mean()
    log("  planted cell over the PRN's mean: pairs %.1f, plain %.1f; ratios %.2f / %.2f"
        % (rise_p, rise_s, pk_p[0]["ratio"], pk_s[0]["ratio"]))
    assert pk_p[0]["detected"] and pk_p[0]["code_phase"] == 321 and pk_p[0]["doppler_bin"] == 4
    assert rise_p > 1.2 * rise_s


def test_pairs_unsupported(ctxp):
    snap = synth.make_snapshot(1, O.CPLX_I8, 4092000, 0.0, 4.0, [], O.ca_code)
    with pytest.raises(G.GnssError) as ei:
        _run(ctxp, snap, synth.Search([1], 0.0, 0.0, 500.0, 1, 3))  # odd N_noncoh
    assert ei.value.code == G.GNSS_ENOTSUP
    with G.Context(0, precision=G.GNSS_FP16) as c16:
        with pytest.raises(G.GnssError) as ei:
            c16.set("nav_pairs", 1)
        assert ei.value.code == G.GNSS_ENOTSUP


def test_longest_coherent_block_at_full_scale():
    # T_coh = 64 ms at spc 16 with +-127 samples: the folded, boxcar-summed block
    # reaches ~2^30 in int32, the limit the request check is derived from
    from parity import assert_grid_close
    fs, Tc = 16368000, 64
    N = fs // 1000
    rng = np.random.default_rng(64)
    n = Tc * N
    x = rng.choice(np.array([-127, 127], np.int8), size=2 * n)
    rep = O.code_replica(5, fs, N)
    x[0::2] = np.tile(np.roll(rep, 1000), Tc).astype(np.int8) * np.int8(127)  # I: code at full scale
    snap = synth.Snapshot(samples=x, fmt=O.CPLX_I8, fs_hz=fs, f_if_hz=0.0, n=n)
    srch = synth.Search([5, 6], -500.0, 500.0, 500.0, Tc, 1)
    with G.Context(0) as c32:
        grid, pk = _run(c32, snap, srch)
    P = O.grid_fft(x, O.CPLX_I8, fs, 0.0, [5, 6], -500.0, 500.0, 3, Tc, 1)
    assert_grid_close(grid, P)
    assert pk[0]["detected"] and pk[0]["code_phase"] == 1000 and pk[0]["doppler_bin"] == 1

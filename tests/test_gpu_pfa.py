"""GPU tests of the exact-length transform (GNSS_FP16_PFA): the 1023-point
DFT as a 31 x 33 Good-Thomas transform whose passes are FP16 x FP16 -> FP32
matrix products, through the C ABI (gnss_dft1023), against numpy's FFT in
FP64.

Error bounds: the transform rounds to FP16 its scaled input, its 31-pass
output and the weights of both passes (unit roundoff u = 2^-11).

* Worst case, any input: each of the four roundings moves a complex value
  by at most sqrt(2) u of its modulus, and every pass output is bounded by the
  l1 norm of its input (weights of modulus 1), so to first order
  |X - X64| <= 4 sqrt(2) u ||x||_1; the tests use 6 u ||x||_1.
* Random inputs: independent rounding errors each perturb the output by
  about u of its RMS (Parseval); with FP32 sums the RMS error is about
  sqrt(5) u ~ 1.1e-3 of RMS(X) and the largest of ~10^5 outputs stays below
  5 RMS: |X - X64| <= 1e-2 RMS(X64).  Inputs with few distinct values (a tone
  at a third of the rate) have coherent rounding errors and only meet the
  worst-case bound.

The acquisition-level parity of the mode is in test_gpu_fp16.py.
"""
import numpy as np
import pytest

from parity import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1309_0052_amd")

REL = 1e-2
U16 = 2.0 ** -11
WORST = 6 * U16


@pytest.fixture(scope="module")
def ctxx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = G.Context(0, precision=G.GNSS_FP16_PFA)
    yield c
    c.close()


def _dft(ctx, x: np.ndarray, inverse: bool) -> np.ndarray:
    b = x.shape[0]
    xi = np.zeros((b, 1023, 2), np.float32)
    xi[..., 0] = x.real
    xi[..., 1] = x.imag
    d_in = torch.from_numpy(xi.ravel()).cuda()
    d_out = torch.full((b * 1023 * 2,), float("nan"), dtype=torch.float32, device="cuda")
    ctx.dft1023(d_in.data_ptr(), d_out.data_ptr(), b, inverse, torch.cuda.current_stream())
    torch.cuda.synchronize()
    o = d_out.cpu().numpy().reshape(b, 1023, 2).astype(np.float64)
    return o[..., 0] + 1j * o[..., 1]


def _check(got, ref, x, what, random=True):
    """x: the transform's input (for the worst-case bound)."""
    assert np.all(np.isfinite(got)), what
    rms = np.sqrt(np.mean(np.abs(ref) ** 2, axis=1, keepdims=True))
    l1 = np.sum(np.abs(x), axis=1, keepdims=True)
    err = np.max(np.abs(got - ref) / rms)
    worst = np.max(np.abs(got - ref) / l1)
    log("  %s: max error %.2e of RMS, %.2e u of the l1 norm" % (what, err, worst / U16))
    assert worst <= WORST, (what, worst / U16)
    if random:
        assert err <= REL, (what, err)
    return err


def test_dft1023_random_vectors_match_numpy(ctxx):
    rng = np.random.default_rng(1023)
    b = 40
    x = (rng.normal(size=(b, 1023)) + 1j * rng.normal(size=(b, 1023)))
    x *= 2.0 ** rng.integers(-20, 30, size=(b, 1))  # the per-vector exponent covers any scale
    x64 = x.astype(np.complex64).astype(np.complex128)  # what the GPU receives
    _check(_dft(ctxx, x64, False), np.fft.fft(x64, axis=1), x64, "forward")
    _check(_dft(ctxx, x64, True), np.fft.ifft(x64, axis=1) * 1023, x64, "inverse")


def test_dft1023_structured_inputs(ctxx):
    n = np.arange(1023)
    rows = []
    for m0 in (0, 1, 32, 33, 31, 528, 496, 1022):  # impulses at and around the index-map seams
        v = np.zeros(1023, complex)
        v[m0] = 1.0 - 0.5j
        rows.append(v)
    for k0 in (0, 1, 31, 33, 341, 1022):  # complex tones: one nonzero bin
        rows.append(np.exp(2j * np.pi * k0 * n / 1023))
    rows.append(np.where(n % 2 == 0, 1.0, -1.0) + 0j)
    x = np.array(rows).astype(np.complex64).astype(np.complex128)
    _check(_dft(ctxx, x, False), np.fft.fft(x, axis=1), x, "forward structured", random=False)
    _check(_dft(ctxx, x, True), np.fft.ifft(x, axis=1) * 1023, x, "inverse structured", random=False)


def test_dft1023_round_trip_and_zero(ctxx):
    rng = np.random.default_rng(5)
    x = (rng.normal(size=(8, 1023)) + 1j * rng.normal(size=(8, 1023))).astype(np.complex64).astype(np.complex128)
    X = _dft(ctxx, x, False)
    X32 = X.astype(np.complex64).astype(np.complex128)
    back = _dft(ctxx, X32, True) / 1023
    err = np.max(np.abs(back - x) / np.sqrt(np.mean(np.abs(x) ** 2, axis=1, keepdims=True)))
    log("  round trip: max error %.2e of RMS" % err)
    assert err <= 2 * REL  # two transforms
    z = _dft(ctxx, np.zeros((3, 1023), complex), False)
    assert np.array_equal(z, np.zeros_like(z))


def test_dft1023_argument_errors(ctxx):
    d = torch.zeros(2046, dtype=torch.float32, device="cuda")
    with pytest.raises(G.GnssError) as ei:
        ctxx.dft1023(d.data_ptr(), d.data_ptr(), 1, False)
    assert ei.value.code == G.GNSS_EINVAL
    with pytest.raises(G.GnssError) as ei:
        ctxx.dft1023(d.data_ptr(), d.data_ptr(), -1, False)
    assert ei.value.code == G.GNSS_EINVAL
    with G.Context(0) as c32:
        e = torch.zeros(2046, dtype=torch.float32, device="cuda")
        with pytest.raises(G.GnssError) as ei:
            c32.dft1023(d.data_ptr(), e.data_ptr(), 1, False)
        assert ei.value.code == G.GNSS_ENOTSUP


def test_dft1023_matches_the_fp16_rounding_model(ctxx):
    """The numpy model of the mode's roundings (fp16_pfa_model.py: FP16 input
    and weights, FP16 31-pass output, FP32 sums) reproduces the GPU transform
    far below the FP16 error itself, including the leak of a constant's DC
    bin into the other bins through the FP16 weights (the mechanism behind
    the mean removal of the correlation path, test_fp16_dc_model.py)."""
    import fp16_pfa_model as M

    rng = np.random.default_rng(33)
    rows = [rng.normal(size=1023) + 1j * rng.normal(size=1023) for _ in range(6)]
    const = np.full(1023, 127.0 + 127.0j) * 2.0 ** 22
    rows.append(const)
    x = np.array(rows).astype(np.complex64).astype(np.complex128)
    got = _dft(ctxx, x, False)
    for i in range(len(rows)):
        model = M.forward(x[i], mean_removed=False)
        exact = np.fft.fft(x[i])
        rms = np.sqrt(np.mean(np.abs(exact) ** 2))
        d_model = np.max(np.abs(got[i] - model)) / rms
        d_exact = np.max(np.abs(got[i] - exact)) / rms
        log("  row %d: GPU vs model %.2e of RMS, GPU vs FP64 %.2e" % (i, d_model, d_exact))
        assert d_model <= 0.2 * d_exact + 1e-6, (i, d_model, d_exact)
    # the constant: the GPU's non-DC bins are the model's leak
    leak_gpu = np.abs(got[-1][1:])
    leak_model = np.abs(M.forward(x[-1], mean_removed=False)[1:])
    log("  constant: max leak GPU %.3e, model %.3e of the DC bin" %
        (leak_gpu.max() / abs(got[-1][0]), leak_model.max() / abs(got[-1][0])))
    assert np.max(np.abs(got[-1][1:] - M.forward(x[-1], mean_removed=False)[1:])) <= 0.1 * leak_model.max()

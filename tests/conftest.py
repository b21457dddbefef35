import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def icd_table():
    rows = []
    with open(os.path.join(GOLDEN, "icd_table_3_Ia.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            prn, t1, t2, delay, octal = line.split()
            rows.append((int(prn), int(t1), int(t2), int(delay), int(octal, 8)))
    return rows


@pytest.fixture(scope="session")
def weak_case():
    """The full-size weak-signal workload and its FP64 oracle grid (computed
    once per session: both precisions are checked against it)."""
    import oracle as O
    import synth
    snap, srch = synth.weak_complex_int8(O.ca_code, seed=2)
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    print("weak workload oracle grid (FP64 FFT route) ...", flush=True)
    P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.step,
                   nd, srch.T_coh, srch.N_noncoh)
    return snap, srch, nd, P


@pytest.fixture(scope="session")
def strong_case():
    """The strong-signal workload (real 2-bit, 4.092 MHz) and its FP64 oracle grid."""
    import oracle as O
    import synth
    snap, srch = synth.strong_real_2bit(O.ca_code, seed=1)
    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    P = O.grid_fft(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.step,
                   nd, srch.T_coh, srch.N_noncoh)
    return snap, srch, nd, P

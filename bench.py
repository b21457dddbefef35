"""Benchmark: GPS L1 C/A acquisition search on one MI355X.

One step = one complete search (carrier wipe-off, folding, forward FFTs,
spectrum products, IFFTs, non-coherent sums, detection, refinement) of one
snapshot already resident in HBM, through the C ABI (gnss_acquire_device).

Default workload (weak signal): complex int8 baseband, fs 16.368 MHz, 100 ms,
8 planted PRNs at C/N0 U[28, 40] dB-Hz with 20 ms navigation-bit flips;
search 32 PRNs x 121 Doppler bins (+-7.5 kHz, 125 Hz) x 16368 code phases,
4 ms coherent x 25 non-coherent.

Metric: search cells/s, a cell being PRN x Doppler bin x code phase x
millisecond of integrated signal; p50/p99 per-snapshot latency beside it.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X vector peaks (256 CU x 2.4 GHz): FP32 with packed FP32 instructions,
# and FP16 with packed FP16 instructions, both 256 flop/clock/CU
PEAK_VALU_TFLOPS = {"fp32": 157.3, "fp16": 157.3}
# dense FP16 matrix-core peak (FP32 accumulation), MI355X
PEAK_MFMA_F16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# integer VALU: 256 CU x 64 lanes x 2.4 GHz, a multiply-add counted as 2 ops
PEAK_INT_TOPS = 78.6
PRECISIONS = ["fp32", "fp16", "fp16pfa"]
DTYPE = {"fp32": "f32", "fp16": "f16", "fp16pfa": "f16"}
CORR_KERNEL = {"fp32": "k_corr", "fp16": "k_corr_h", "fp16pfa": "k_corr_x"}
# what bounds each mode's correlation kernel, and that unit's peak
ROOF = {"fp32": ("alu", 157.3), "fp16": ("alu", 157.3), "fp16pfa": ("mfma", PEAK_MFMA_F16_TFLOPS)}
# bytes of one stored block spectrum (one polyphase vector)
G_VEC_BYTES = {"fp32": 16384, "fp16": 8192, "fp16pfa": 4224}
# matrix-core flops of one 1023-point inverse transform in the exact-length
# mode: 54 16x16x32 FP16 products of 16384 flops each
PFA_MFMA_FLOPS = 54 * 16384


def precision_const(G, name: str) -> int:
    return {"fp32": G.GNSS_FP32, "fp16": G.GNSS_FP16, "fp16pfa": G.GNSS_FP16_PFA}[name]


def corr_roofline(prec: str, flops: float, corr_ms: float, traffic, transforms: int) -> dict:
    """Roofline object of the correlation kernel: algorithmic flops (exact
    length-N FFT correlation) per launch over its average launch time."""
    bound, peak = ROOF[prec]
    achieved = flops / (corr_ms / 1e3) / 1e12
    r = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
         "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": CORR_KERNEL[prec],
         "avg_launch_ms": round(corr_ms, 4), "flops_per_launch": flops}
    if prec == "fp16pfa":
        issued = transforms * PFA_MFMA_FLOPS
        r["mfma_flops_issued_per_launch"] = issued
        r["mfma_issued_frac"] = round(issued / (corr_ms / 1e3) / 1e12 / peak, 4)
    return r


def kernel_source_hash() -> str:
    h = hashlib.sha1()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_1309_0052_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "%s_%s_counters.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_src = re.search(r"source_hash:\s*([0-9a-f]+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_src or not m_b or m_src.group(1) != kernel_source_hash():
        return None
    return float(m_b.group(1))


def workload(name: str, code_fn):
    import synth

    if name == "weak":
        snap, srch = synth.weak_complex_int8(code_fn, seed=2)
        desc = ("weak-signal complex int8 baseband, fs 16.368 MHz, 100 ms, 8 planted; "
                "32 PRN x 121 Doppler (+-7.5 kHz / 125 Hz) x 16368 phases, 4 ms coh x 25 noncoh")
    elif name == "weak10":
        snap, srch = synth.weak_complex_int8(code_fn, seed=2, fs=10000000)
        desc = ("weak-signal complex int8 baseband at a general rate, fs 10.000 MHz, 100 ms, 8 planted; "
                "32 PRN x 121 Doppler (+-7.5 kHz / 125 Hz) x 10000 phases, 4 ms coh x 25 noncoh "
                "(zero-padded 32768-point FP32 transforms)")
    elif name == "long":
        snap, srch = synth.long_complex_int8(code_fn, seed=3)
        desc = ("long weak-signal integration, complex int8 baseband, fs 16.368 MHz, 2.048 s, 8 planted at "
                "22-30 dB-Hz; 32 PRN x 121 Doppler (+-7.5 kHz / 125 Hz) x 16368 phases, 4 ms coh x 512 "
                "noncoh, under an HBM budget that makes it run in passes over its blocks")
    elif name == "strong":
        snap, srch = synth.strong_real_2bit(code_fn, seed=1)
        desc = ("strong-signal real 2-bit IF, fs 4.092 MHz, f_IF 1.023 MHz, 10 ms, 4 planted; "
                "32 PRN x 21 Doppler (+-5 kHz / 500 Hz) x 4092 phases, 1 ms coh x 10 noncoh")
    else:
        raise SystemExit("unknown workload %r" % name)
    return snap, srch, desc


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(snap, srch, target_s: float):
    """The oracle (plain direct correlation, FP64) on bounded samples of cells
    of the same workload, cells/s extrapolated: the median of three timed runs
    on all host threads after one untimed run, and one run on a single thread
    (each run about target_s / 4 seconds)."""
    import numpy as np

    import oracle as O

    nd = O.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    threads = O.n_threads()
    rng = np.random.default_rng(123)
    ms = srch.T_coh * srch.N_noncoh

    def run(n_cells, nthr):
        cells = np.stack([rng.integers(0, len(srch.prns), n_cells), rng.integers(0, nd, n_cells),
                          rng.integers(0, N, n_cells)], axis=1)
        t0 = time.perf_counter()
        O.cells_direct(snap.samples, snap.fmt, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                       srch.step, nd, srch.T_coh, srch.N_noncoh, cells, threads=nthr)
        return time.perf_counter() - t0

    def size_for(nthr, seconds):
        n = 2 * nthr
        dt = run(n, nthr)  # also the untimed warm-up run
        while dt < 0.5 and n < (1 << 26):  # a first timing long enough to extrapolate from
            n *= 4
            dt = run(n, nthr)
        return max(n, int(n * seconds / dt))

    part = target_s / 4.0
    n_all = size_for(threads, part)
    rates = sorted(n_all * ms / run(n_all, threads) for _ in range(3))
    n_one = size_for(1, part)
    dt_one = run(n_one, 1)
    return {"value": rates[1], "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": "%d random (PRN, Doppler, phase) cells x %d ms by direct time-domain "
                      "correlation, median of 3 runs of ~%.0f s on %d threads (runs: %s cells/s)"
                      % (n_all, ms, part, threads, ", ".join("%.4g" % r for r in rates)),
            "one_core": {"value": n_one * ms / dt_one, "unit": "cells/s", "cores": 1,
                         "sample": "%d cells x %d ms, %.1f s" % (n_one, ms, dt_one)},
            "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="weak",
                    choices=["weak", "weak10", "long", "strong", "batch", "serve", "track", "precision"])
    ap.add_argument("--batch-n", type=int, default=256, help="snapshots in the batch workload")
    ap.add_argument("--rates", default="50,200,800", help="serve: Poisson arrival rates, req/s")
    ap.add_argument("--serve-n", type=int, default=2000, help="serve: timed requests per rate")
    ap.add_argument("--serve-warmup", type=int, default=200, help="serve: untimed requests per rate")
    ap.add_argument("--serve-kind", default="mixed", choices=["mixed", "strong"],
                    help="serve: heterogeneous batch-style requests or strong-signal snapshots")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve: HBM budget")
    ap.add_argument("--long-budget-gb", type=float, default=16.0,
                    help="long: the context's HBM budget (one pass of the request needs ~24 GB)")
    ap.add_argument("--corr-ptile", type=int, default=0, choices=[0, 1, 2, 4, 8],
                    help="PRN tile of the correlation kernel; 0: autotuned for the workload")
    ap.add_argument("--corr-waves", type=int, default=0, choices=[0, 4, 6, 8, 12],
                    help="waves per correlation workgroup; 0: autotuned for the workload")
    ap.add_argument("--persistent", type=int, default=-1, choices=[-1, 0, 1],
                    help="correlation grid: 1 occupancy-sized with work counters, 0 one workgroup "
                         "per item, -1 the library default")
    ap.add_argument("--precision", default="fp32", choices=PRECISIONS,
                    help="fp16: packed FP16 transforms, FP32 power and block sums; fp16pfa: exact-length "
                         "1023-point transforms on the matrix cores (FP16 operands, FP32 accumulation)")
    ap.add_argument("--doppler-fd", action="store_true",
                    help="with --precision fp16pfa: frequency-domain Doppler (one long DFT per block "
                         "serves every bin; exact-exponential carrier)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision, batch and serving figures the default line carries")
    ap.add_argument("--extra-steps", type=int, default=5, help="extras: graph replays of the batch")
    ap.add_argument("--extra-rate", type=float, default=200.0, help="extras: Poisson arrival rate, req/s")
    ap.add_argument("--extra-serve-n", type=int, default=500, help="extras: timed served requests per precision")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-modes", action="store_true",
                    help="skip timing the snapshot on the FP16 and exact-length modes beside FP32")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the search shards by request or by PRN with no "
              "exchange, and no multi-GPU figure is produced here (asked for --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1309_0052_amd as G

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    prec = precision_const(G, args.precision)
    budget = int(args.long_budget_gb * (1 << 30)) if args.workload == "long" else 0
    ctx = G.Context(0, hbm_budget_bytes=budget, precision=prec)
    if args.corr_ptile:
        ctx.set("corr_ptile", args.corr_ptile)
    if args.corr_waves:
        ctx.set("corr_waves", args.corr_waves)
    if args.persistent >= 0:
        ctx.set("persistent", args.persistent)
    if args.doppler_fd:
        ctx.set("doppler_fd", 1)
    stream = torch.cuda.current_stream()

    def code_fn(prn):
        d = torch.zeros(1023, dtype=torch.uint8, device="cuda")
        ctx.gold_codes([prn], d.data_ptr(), stream)
        torch.cuda.synchronize()
        return d.cpu().numpy()

    if args.copy_mb:
        a = torch.ones(args.copy_mb << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.workload == "batch":
        return run_batch(args, G, torch, ctx, code_fn)
    if args.workload == "track":
        return run_track(args, G, torch, ctx, code_fn)
    if args.workload == "precision":
        return run_precision(args, G, torch, ctx, code_fn)
    if args.workload == "serve":
        return run_serve(args, G, torch, ctx, code_fn)

    snap, srch, desc = workload(args.workload, code_fn)
    nd = G.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    n_prn = len(srch.prns)
    d_x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
    d_grid = torch.empty(n_prn * nd * N, dtype=torch.float32, device="cuda")
    d_pk = torch.zeros(n_prn * 48, dtype=torch.uint8, device="cuda")
    req = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns,
                         srch.lo, srch.hi, srch.step, srch.T_coh, srch.N_noncoh,
                         d_grid.data_ptr(), d_pk.data_ptr())
    pt, sched = args.corr_ptile, args.persistent
    if not pt or sched < 0:  # explicit tile and schedule options skip the autotuner
        # the tuner times one-pass batches; its choice is kept per rate mix, so a
        # request run in passes is tuned on its first 256 blocks
        tune = req if args.workload != "long" else G.make_request(
            d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo, srch.hi,
            srch.step, srch.T_coh, 256, d_grid.data_ptr(), d_pk.data_ptr())
        t_pt, t_sched = ctx.autotune([tune], os.path.join("/tmp", "gnss_autotune.txt"))
        pt, sched = pt or t_pt, sched if sched >= 0 else t_sched
    ctx.set("profile", 1)
    for _ in range(args.warmup):
        ctx.acquire_device(req, stream)
    torch.cuda.synchronize()
    ctx.stage_times(reset=True)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        ctx.acquire_device(req, stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    total_ms = ev[0].elapsed_time(ev[-1])
    stages = ctx.stage_times(reset=True)
    ms_step = total_ms / args.steps

    pk = d_pk.cpu().numpy().view(G.PEAK_DTYPE)
    planted = {p.prn for p in snap.planted}
    detected = {int(r["prn"]) for r in pk if r["detected"]}

    cells = n_prn * nd * N * srch.T_coh * srch.N_noncoh
    value = cells / (ms_step / 1e3)

    # dominant kernel: spectrum product -> IFFT -> |.|^2 -> block sum; a request
    # run in passes over its blocks launches it once per pass
    corr_ms = stages["corr"][0] / max(1, stages["corr"][1])
    lps = max(1, stages["corr"][1]) / args.steps  # correlation launches per step
    units = n_prn * nd * srch.N_noncoh / lps  # (PRN, Doppler, block) correlations per launch
    flops_unit = 5.0 * N * math.log2(N) + 10.0 * N
    wl = args.workload
    general = snap.fs_hz % 1023000 != 0 or snap.fs_hz // 1023000 > 16
    if general:
        # a rate that is not a multiple of the chip rate: the zero-padded FP32
        # transforms in every precision
        roofline = corr_roofline("fp32", units * flops_unit, corr_ms, read_traffic("gen_corr", wl), 0)
        # N > 4096: the 16384-point (four-step) kernel; else the radix-8 one of its length
        roofline["kernel"] = "k_gen_corr16" if N > 4096 else "k_gen_corr"
    else:
        kern = CORR_KERNEL[args.precision]
        roofline = corr_roofline(args.precision, units * flops_unit, corr_ms, read_traffic(kern[2:], wl),
                                 units * (N // 1023))

    # the FFT pipeline (forward FFT + correlation stages) against the HBM roofline:
    # staged-model bytes, each stage buffer crossing HBM once (F in, G out, G in,
    # grid out; general rates: the folded-block spectra out and in, the grid out),
    # over the two stages' measured time
    if general:
        M = 64
        while M < 2 * N:
            M *= 2
        if N >= 64 and N & (N - 1) == 0:
            M = N  # a power of two: no padding
        staged = nd * srch.N_noncoh * M * 8 * 2 + n_prn * nd * N * 4
    else:
        n_vec = nd * srch.N_noncoh * (N // 1023)
        g_vec = G_VEC_BYTES[args.precision]
        staged = n_vec * (8192 + 2 * g_vec) + n_prn * nd * N * 4
    pipe_ms = (stages["fft"][0] + stages["corr"][0]) / args.steps
    fft_hbm = {"staged_bytes": staged, "time_ms": round(pipe_ms, 4),
               "achieved_GBs": round(staged / (pipe_ms / 1e3) / 1e9, 1), "peak_GBs": PEAK_HBM_GBS,
               "frac": round(staged / (pipe_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}

    # end to end: the method's algorithmic work (per (PRN, bin, block) an N-point
    # inverse transform, the spectrum product, |.|^2 and the sum; per (bin, block) an
    # N-point forward transform; the wipe-off of every sample in every bin) and its
    # bytes (the record once, the grid once, the code spectra once) against the
    # chip's FP32 and HBM peaks: max(bytes / BW, flops / peak) / measured time
    n_samples = srch.T_coh * srch.N_noncoh * N
    e2e_flops = (n_prn * nd * srch.N_noncoh * flops_unit + nd * srch.N_noncoh * 5.0 * N * math.log2(N)
                 + nd * n_samples * (6.0 if snap.fmt == G.GNSS_CPLX_I8 else 2.0))
    e2e_bytes = snap.samples.nbytes + n_prn * nd * N * 4 + n_prn * N * 8
    t_min = max(e2e_bytes / (PEAK_HBM_GBS * 1e9), e2e_flops / 157.3e12)
    end_to_end = {"flops": e2e_flops, "bytes": e2e_bytes,
                  "bound": "alu" if e2e_flops / 157.3e12 >= e2e_bytes / (PEAK_HBM_GBS * 1e9) else "hbm",
                  "t_min_ms": round(t_min * 1e3, 4), "frac": round(t_min / (ms_step / 1e3), 4)}

    out = {
        "metric": "search cells/s (PRNxDopplerxphasexms) + p50/p99 latency/snapshot",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": desc, "n_prn": n_prn, "n_doppler": nd, "code_phases": N,
                   "T_coh_ms": srch.T_coh, "N_noncoh": srch.N_noncoh,
                   "cells_per_snapshot": cells, "corr_ptile": pt, "persistent": sched,
                   "precision": args.precision, "doppler_fd": bool(args.doppler_fd)},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "min": float(lat.min()), "max": float(lat.max())},
        "wall_s": wall_s,
        "stages_ms": {k: round(v[0] / max(1, v[1]), 4) for k, v in stages.items()},
        "roofline": roofline,
        "fft_pipeline_hbm": fft_hbm,
        "end_to_end": end_to_end,
        "detections": {"planted": sorted(planted), "detected": sorted(detected),
                       "planted_found": sorted(planted & detected)},
        "source_hash": kernel_source_hash(),
    }
    if args.workload == "long":
        out["passes"] = long_passes(args, G, torch, d_x, d_grid, snap, srch, stream, lps, ms_step, budget)
    elif not args.no_other_modes and args.precision == "fp32" and not args.doppler_fd and not general:
        out["other_modes"] = other_modes(args, G, torch, d_x, snap, srch, cells, stream)
    if (not args.no_extras and args.workload == "weak" and args.precision == "fp32" and not args.doppler_fd):
        codes = {p: code_fn(p) for p in range(1, 38)}  # the GPU's codes, kept past this context
        ctx.close()
        del d_x
        torch.cuda.empty_cache()
        out.update(extras(args, G, torch, codes.__getitem__))
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(snap, srch, args.cpu_seconds)
        except Exception as e:  # noqa: BLE001 -- reported in the line, not allowed to cost it
            out["cpu_baseline"] = {"error": "%s: %s" % (type(e).__name__, e), "kind": "oracle"}
    ctx.close()
    print(json.dumps(out), flush=True)


def long_passes(args, G, torch, d_x, d_grid, snap, srch, stream, lps, ms_step, budget):
    """The long request in passes (under the context's budget) against the same
    request in one pass on an unlimited context: ms per step of each, and
    whether the grids are the same bit for bit (they must be in FP32)."""
    nd = G.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    n_prn = len(srch.prns)
    probe = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                           srch.hi, srch.step, srch.T_coh, srch.N_noncoh, None, 1)
    res = {"budget_gb": budget / (1 << 30), "one_pass_workspace_gb": G.gnss_workspace_bytes(probe) / (1 << 30),
           "passes_per_step": lps, "ms_per_step_in_passes": ms_step}
    c = G.Context(0, precision=precision_const(G, args.precision))
    try:
        g = torch.empty(n_prn * nd * N, dtype=torch.float32, device="cuda")
        pk = torch.zeros(n_prn * 48, dtype=torch.uint8, device="cuda")
        req = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                             srch.hi, srch.step, srch.T_coh, srch.N_noncoh, g.data_ptr(), pk.data_ptr())
        c.acquire_device(req, stream)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        steps = max(1, min(args.steps, 5))
        ev[0].record(stream)
        for _ in range(steps):
            c.acquire_device(req, stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        res["ms_per_step_one_pass"] = ev[0].elapsed_time(ev[1]) / steps
        res["grid_equal_one_pass"] = bool(torch.equal(g, d_grid))
    finally:
        c.close()
    return res


def other_modes(args, G, torch, d_x, snap, srch, cells, stream):
    """The same snapshot on the other precision modes of the same GPU (their
    parity against the FP64 oracle is in tests/test_gpu_fp16.py and
    test_gpu_fd.py): ms per step, cells/s, stage times and the correlation
    kernel's roofline."""
    nd = G.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    n_prn = len(srch.prns)
    units = n_prn * nd * srch.N_noncoh
    flops_unit = 5.0 * N * math.log2(N) + 10.0 * N
    res = {}
    for name, prec, opts in (("fp16", "fp16", {}), ("fp16pfa", "fp16pfa", {}),
                             ("fp16pfa_doppler_fd", "fp16pfa", {"doppler_fd": 1})):
        # a failure here is reported in the line, not allowed to cost the line itself
        try:
            res[name] = _time_mode(args, G, torch, d_x, snap, srch, cells, stream, nd, N, n_prn, units,
                                   flops_unit, prec, opts)
        except Exception as e:  # noqa: BLE001
            res[name] = {"error": "%s: %s" % (type(e).__name__, e)}
    return res


def _time_mode(args, G, torch, d_x, snap, srch, cells, stream, nd, N, n_prn, units, flops_unit, prec, opts):
    """One precision mode on the resident snapshot (see other_modes)."""
    c = G.Context(0, precision=precision_const(G, prec))
    try:
        for k, v in opts.items():
            c.set(k, v)
        g = torch.empty(n_prn * nd * N, dtype=torch.float32, device="cuda")
        pk = torch.zeros(n_prn * 48, dtype=torch.uint8, device="cuda")
        req = G.make_request(d_x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                             srch.hi, srch.step, srch.T_coh, srch.N_noncoh, g.data_ptr(), pk.data_ptr())
        c.autotune([req], os.path.join("/tmp", "gnss_autotune.txt"))
        c.set("profile", 1)
        for _ in range(args.warmup):
            c.acquire_device(req, stream)
        torch.cuda.synchronize()
        c.stage_times(reset=True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        steps = max(1, min(args.steps, 10))
        ev[0].record(stream)
        for _ in range(steps):
            c.acquire_device(req, stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / steps
        st = c.stage_times(reset=True)
        corr_ms = st["corr"][0] / max(1, st["corr"][1])
        p = pk.cpu().numpy().view(G.PEAK_DTYPE)
        traffic = read_traffic(CORR_KERNEL[prec][2:], args.workload) if not opts else None
        return {"ms_per_step": ms, "value": cells / (ms / 1e3), "unit": "cells/s", "dtype": DTYPE[prec],
                "stages_ms": {k: round(v[0] / max(1, v[1]), 4) for k, v in st.items()},
                "roofline": corr_roofline(prec, units * flops_unit, corr_ms, traffic, units * (N // 1023)),
                "detected": sorted(int(r["prn"]) for r in p if r["detected"])}
    finally:
        c.close()


def _cells(srch, fs_hz):
    import paper_1309_0052_amd as G

    nd = G.n_doppler(srch.lo, srch.hi, srch.step)
    return len(srch.prns) * nd * (fs_hz // 1000) * srch.T_coh * srch.N_noncoh


BATCH_DESC = ("heterogeneous batch of %d snapshots, 20-200 ms, fs in {4.092, 8.184, 16.368} MHz, 8-32 PRNs, "
              "+-2-10 kHz windows, 1 ms coh; one hipGraph launch per step")


def batch_items(code_fn, n: int):
    """The heterogeneous batch workload (seed 4), generated on host threads."""
    import synth

    t_gen = time.perf_counter()
    items = synth.batch_workload(code_fn, seed=4, n=n, workers=min(16, os.cpu_count() or 1))
    return items, time.perf_counter() - t_gen


def batch_measure(G, torch, ctx, items, prec: str, steps: int, warmup: int, pt=0, sched=-1) -> dict:
    """One captured-graph replay of the whole batch per step on `ctx` (whose
    precision is `prec`): ms per step, snapshots/s, cells/s, the per-stage
    split of one eager profiled pass, the correlation kernel's roofline and
    the planted satellites recovered at their code phase."""
    import numpy as np

    stream = torch.cuda.current_stream()
    bufs, reqs = [], []
    cells = 0
    for snap, srch in items:
        nd = G.n_doppler(srch.lo, srch.hi, srch.step)
        N = snap.fs_hz // 1000
        x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
        g = torch.empty(len(srch.prns) * nd * N, dtype=torch.float32, device="cuda")
        pk = torch.zeros(len(srch.prns) * 48, dtype=torch.uint8, device="cuda")
        bufs.append((x, g, pk))
        reqs.append(G.make_request(x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz,
                                   srch.prns, srch.lo, srch.hi, srch.step, srch.T_coh,
                                   srch.N_noncoh, g.data_ptr(), pk.data_ptr()))
        cells += _cells(srch, snap.fs_hz)
    torch.cuda.synchronize()
    if not pt or sched < 0:  # explicit tile and schedule options skip the autotuner
        t_pt, t_sched = ctx.autotune(reqs, os.path.join("/tmp", "gnss_autotune.txt"))
        pt, sched = pt or t_pt, sched if sched >= 0 else t_sched
    graph = ctx.graph(reqs)
    try:
        for _ in range(warmup):
            graph.launch(stream)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(steps):
            graph.launch(stream)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        wall_s = time.perf_counter() - t0
    finally:
        graph.close()
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    ms_step = ev[0].elapsed_time(ev[-1]) / steps
    # one eager profiled pass for the per-stage split and the dominant kernel
    ctx.set("profile", 1)
    ctx.stage_times(reset=True)
    ctx.acquire_batch_device(reqs, stream)
    torch.cuda.synchronize()
    stages = ctx.stage_times(reset=True)
    ctx.set("profile", 0)
    found = total = 0
    for (snap, srch), (x, g, pk) in zip(items, bufs):
        p = pk.cpu().numpy().view(G.PEAK_DTYPE)
        det = {int(r["prn"]): int(r["code_phase"]) for r in p if r["detected"]}
        for pl in snap.planted:
            total += 1
            found += int(det.get(pl.prn, -1) == pl.code_phase)
    corr_ms = stages["corr"][0] / max(1, stages["corr"][1])
    units_flops = 0.0
    transforms = 0
    for snap, srch in items:
        N = snap.fs_hz // 1000
        nd = G.n_doppler(srch.lo, srch.hi, srch.step)
        units_flops += len(srch.prns) * nd * srch.N_noncoh * (5.0 * N * math.log2(N) + 10.0 * N)
        transforms += len(srch.prns) * nd * srch.N_noncoh * (N // 1023)
    return {"ms_per_step": ms_step, "steps": steps, "warmup": warmup,
            "value": cells / (ms_step / 1e3), "unit": "cells/s", "dtype": DTYPE[prec],
            "snapshots": len(items), "cells_per_step": cells,
            "snapshots_per_s": len(items) / (ms_step / 1e3),
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
            "wall_s": wall_s, "corr_ptile": pt, "persistent": sched,
            "stages_ms": {k: round(v[0] / max(1, v[1]), 4) for k, v in stages.items()},
            "roofline": corr_roofline(prec, units_flops, corr_ms,
                                      read_traffic(CORR_KERNEL[prec][2:], "batch"), transforms),
            "planted_recovered": [found, total]}


def run_batch(args, G, torch, ctx, code_fn):
    """Heterogeneous batch: one captured graph replay per step."""
    items, t_gen = batch_items(code_fn, args.batch_n)
    m = batch_measure(G, torch, ctx, items, args.precision, args.steps, args.warmup, args.corr_ptile,
                      args.persistent)
    out = {
        "metric": "search cells/s (PRNxDopplerxphasexms) + p50/p99 latency/snapshot",
        "value": m["value"], "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": BATCH_DESC % len(items), "snapshots": len(items), "cells_per_step": m["cells_per_step"],
                   "corr_ptile": m["corr_ptile"], "persistent": m["persistent"], "precision": args.precision,
                   "doppler_fd": bool(args.doppler_fd)},
        "snapshots_per_s": m["snapshots_per_s"], "latency_ms": m["latency_ms"], "wall_s": m["wall_s"],
        "generate_s": t_gen, "stages_ms": m["stages_ms"], "roofline": m["roofline"],
        "planted_recovered": m["planted_recovered"], "source_hash": kernel_source_hash(),
    }
    ctx.close()
    print(json.dumps(out), flush=True)


SERVE_KINDS = {"mixed": "heterogeneous batch-style snapshots (20-200 ms, 3 rates, 8-32 PRNs, 1 ms coh)",
               "strong": "strong-signal real 2-bit snapshots (4.092 MHz, 10 ms, 32 PRN x 21 bins)"}


def serve_pool(G, code_fn, kind: str):
    """The requests the served benchmark draws from: host arrays and cells."""
    import numpy as np
    import synth

    if kind == "mixed":
        pool = synth.batch_workload(code_fn, seed=5, n=48, workers=min(16, os.cpu_count() or 1))
    else:
        pool = [synth.strong_real_2bit(code_fn, seed=50 + i) for i in range(16)]
    prepared = []
    for snap, srch in pool:
        nd = G.n_doppler(srch.lo, srch.hi, srch.step)
        prepared.append((np.ascontiguousarray(snap.samples), snap, srch, nd, _cells(srch, snap.fs_hz)))
    return prepared


def serve_measure(G, prepared, prec: str, rate: float, n_timed: int, n_warm: int, budget_gb: float,
                  rng, doppler_fd: bool = False) -> dict:
    """Open-loop Poisson arrivals at `rate` into a serving context: p50/p99
    latency (results on the host - scheduled arrival, from the library's
    clock of each ticket), snapshots/s, cells/s, the paper's effective
    running time (wall / requests) and the mean batch size."""
    import threading

    import numpy as np

    sctx = G.Context(0, hbm_budget_bytes=int(budget_gb * (1 << 30)), precision=precision_const(G, prec))
    try:
        if doppler_fd:
            sctx.set("doppler_fd", 1)
        n_total = n_warm + n_timed
        gaps = rng.exponential(1.0 / rate, n_total)
        sched = np.cumsum(gaps)
        picks = rng.integers(0, len(prepared), n_total)
        submit_at = np.zeros(n_total)
        done_at = np.zeros(n_total)
        batch_sizes = np.zeros(n_total, np.int64)
        tickets = [None] * n_total
        refused = np.zeros(n_total, bool)
        outs = [None] * n_total
        ready = threading.Semaphore(0)
        errors = []

        def collector():
            for i in range(n_total):
                ready.acquire()
                if tickets[i] is None:  # refused at submission
                    continue
                try:
                    info = sctx.wait(tickets[i], 600.0)
                    # completion time from the library's own clock of the ticket
                    done_at[i] = submit_at[i] + info.total_s
                    batch_sizes[i] = info.batch_size
                except Exception as e:  # noqa: BLE001
                    errors.append(repr(e))

        th = threading.Thread(target=collector)
        th.start()
        t0 = time.perf_counter()
        try:
            for i in range(n_total):
                x, snap, srch, nd, _ = prepared[picks[i]]
                pk = np.zeros(len(srch.prns), G.PEAK_DTYPE)
                req = G.make_request(x.ctypes.data, snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz,
                                     srch.prns, srch.lo, srch.hi, srch.step, srch.T_coh,
                                     srch.N_noncoh, None, pk.ctypes.data)
                while True:
                    now = time.perf_counter() - t0
                    if now >= sched[i]:
                        break
                    time.sleep(min(0.0005, sched[i] - now))
                outs[i] = (pk, req)
                submit_at[i] = time.perf_counter()
                try:
                    tickets[i] = sctx.submit(req)
                except G.GnssError as e:
                    if e.code != G.GNSS_ENOMEM:
                        raise
                    refused[i] = True  # larger than a batch slot's share of the HBM budget
                ready.release()
        finally:
            for _ in range(n_total):  # let the collector finish whatever was submitted
                ready.release()
            th.join()
    finally:
        sctx.close()
    if errors:
        raise RuntimeError("serving errors: %s" % errors[:3])
    w = n_warm
    ok = ~refused[w:]
    lat = ((done_at[w:] - t0) - sched[w:])[ok]
    span = done_at[w:][ok].max() - (t0 + sched[w])
    n_ok = int(ok.sum())
    cells = float(sum(prepared[j][4] for j, good in zip(picks[w:], ok) if good))
    return {"rate_req_s": rate, "requests": int(n_timed), "warmup_requests": int(n_warm),
            "refused": int((~ok).sum()), "dtype": DTYPE[prec],
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "snapshots_per_s": float(n_ok / span), "cells_per_s": cells / span,
            "effective_running_time_ms": float(span / n_ok * 1e3),
            "mean_batch": float(batch_sizes[w:][ok].mean())}


def run_serve(args, G, torch, ctx, code_fn):
    """Open-loop Poisson arrivals into the continuous-batching server."""
    import numpy as np

    prepared = serve_pool(G, code_fn, args.serve_kind)
    ctx.close()
    rates = [float(r) for r in args.rates.split(",") if r]
    results = []
    rng = np.random.default_rng(5)
    for rate in rates:
        results.append(serve_measure(G, prepared, args.precision, rate, args.serve_n, args.serve_warmup,
                                     args.budget_gb, rng, args.doppler_fd))
        print("serve rate %.0f req/s: p50 %.1f ms, p99 %.1f ms, %.0f snapshots/s, %d refused"
              % (rate, results[-1]["p50_ms"], results[-1]["p99_ms"], results[-1]["snapshots_per_s"],
                 results[-1]["refused"]), file=sys.stderr, flush=True)
    top = results[-1]
    out = {
        "metric": "search cells/s (PRNxDopplerxphasexms) + p50/p99 latency/snapshot",
        "value": top["cells_per_s"], "unit": "cells/s", "n_gpus": 1, "steps": int(args.serve_n),
        "warmup": int(args.serve_warmup), "ms_per_step": top["effective_running_time_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": "served open-loop Poisson arrivals of %s, HBM budget %g GB"
                               % (SERVE_KINDS[args.serve_kind], args.budget_gb), "rates_req_s": rates,
                   "precision": args.precision, "budget_gb": args.budget_gb, "kind": args.serve_kind},
        "latency_ms": {"p50": top["p50_ms"], "p99": top["p99_ms"]},
        "serving": results,
        "source_hash": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)


def run_track(args, G, torch, ctx, code_fn):
    """Early/prompt/late tracking correlators: 32 records x 12 channels x
    100 ms at 16.368 MHz complex int8, 1 ms epochs, one launch per step."""
    import numpy as np
    import synth

    fs, ms, n_rec, n_ch = 16368000, 100.0, 32, 12
    f_l1 = 1575.42e6
    rng = np.random.default_rng(9)
    t_gen = time.perf_counter()
    recs = []
    for i in range(n_rec):
        prns = rng.choice(np.arange(1, 33), size=n_ch, replace=False)
        pl = [synth.Planted(prn=int(p), code_phase=int(rng.integers(0, fs // 1000)),
                            doppler_hz=float(rng.uniform(-4000, 4000)), cn0_dbhz=float(rng.uniform(35, 48)),
                            carrier_phase=float(rng.uniform(0, 2 * np.pi)), nav_bits=True,
                            nav_phase_ms=int(rng.integers(0, 20))) for p in prns[:8]]
        snap = synth.make_snapshot(900 + i, synth.CPLX_I8, fs, 0.0, ms, pl, code_fn)
        chans = []
        for j, p in enumerate(prns):
            if j < len(pl):  # a channel on each planted satellite's true parameters
                f_d = pl[j].doppler_hz
                cp = (1023.0 - pl[j].code_phase / 16.0) % 1023.0
            else:
                f_d = float(rng.uniform(-4000, 4000))
                cp = float(rng.uniform(0, 1023))
            chans.append((int(p), f_d, 0.0, cp, 1023000.0 * (1 + f_d / f_l1), 0.5))
        recs.append((snap, chans))
    t_gen = time.perf_counter() - t_gen
    epoch, n_ep = fs // 1000, int(ms)
    bufs, reqs = [], []
    for snap, chans in recs:
        x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
        o = torch.zeros(n_ch * n_ep * 6, dtype=torch.int64, device="cuda")
        bufs.append((x, o))
        reqs.append(G.make_track_request(x.data_ptr(), snap.fmt, snap.n, fs, chans, 0, epoch, n_ep, o.data_ptr()))
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        ctx.track_device(reqs, stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        ctx.track_device(reqs, stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    lat = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    ms_step = ev[0].elapsed_time(ev[-1]) / args.steps
    units = n_rec * n_ch * epoch * n_ep  # sample-channels per step
    # algorithmic integer ops per sample-channel: carrier mixing (4 multiplies,
    # 2 adds) and three complex correlator accumulations (+-y: 6 adds)
    ops_unit = 12.0
    achieved = units * ops_unit / (ms_step / 1e3) / 1e12
    # the planted channels' prompt power against their early/late
    o = bufs[0][1].cpu().numpy().reshape(n_ch, n_ep, 3, 2).astype(np.float64)
    pw = (o ** 2).sum(axis=3).sum(axis=1)
    out = {
        "metric": "correlator sample-channels/s (early/prompt/late)", "value": units / (ms_step / 1e3),
        "unit": "sample-channels/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32/int64", "data": "synthetic",
        "config": {"workload": "tracking correlators: %d records x %d channels x %d ms, 16.368 MHz complex "
                               "int8, 1 ms epochs, spacing 0.5 chip; one launch per step" % (n_rec, n_ch, n_ep),
                   "records": n_rec, "channels": n_ch, "epochs": n_ep},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "wall_s": wall_s, "generate_s": t_gen,
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_INT_TOPS, "unit": "Tops/s",
                     "frac": round(achieved / PEAK_INT_TOPS, 4), "traffic": read_traffic("track", "correlators"),
                     "kernel": "k_track", "avg_launch_ms": round(ms_step, 4)},
        "planted_prompt_over_early_late": float(np.min(pw[:8, 1] / np.maximum(pw[:8, 0], pw[:8, 2]))),
        "source_hash": kernel_source_hash(),
    }
    if not args.no_cpu_baseline:
        # the oracle over whole records (all channels, all epochs) until the time target
        import oracle as O
        threads = O.n_threads()
        done, t1 = 0, time.perf_counter()
        while done == 0 or (time.perf_counter() - t1 < args.cpu_seconds and done < 200 * n_rec):
            snap, chans = recs[done % n_rec]
            O.track(snap.samples, snap.fmt, fs, [O.Channel(*c) for c in chans], 0, epoch, n_ep, threads=threads)
            done += 1
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": done * n_ch * epoch * n_ep / dt, "unit": "sample-channels/s",
                               "cores": threads, "kind": "oracle",
                               "sample": "%d records x %d channels x %d ms (the workload's own records), %.1f s"
                                         % (done, n_ch, n_ep, dt)}
    ctx.close()
    print(json.dumps(out), flush=True)


def precision_measure(G, torch, code_fn, steps: int, warmup: int) -> dict:
    """The strong-signal snapshot on FP32, FP16 and exact-length FP16
    contexts of the same GPU: device time of each (cells/s), and each FP16
    mode's grid and detections against the FP32 ones (the error against the
    FP64 oracle is in the FP16 tests)."""
    import numpy as np
    import synth

    snap, srch = synth.strong_real_2bit(code_fn, seed=1)
    nd = G.n_doppler(srch.lo, srch.hi, srch.step)
    N = snap.fs_hz // 1000
    n_prn = len(srch.prns)
    cells = n_prn * nd * N * srch.T_coh * srch.N_noncoh
    stream = torch.cuda.current_stream()
    x = torch.from_numpy(np.ascontiguousarray(snap.samples)).cuda()
    res = {}
    for name in PRECISIONS:
        c = G.Context(0, precision=precision_const(G, name))
        try:
            g = torch.empty(n_prn * nd * N, dtype=torch.float32, device="cuda")
            pk = torch.zeros(n_prn * 48, dtype=torch.uint8, device="cuda")
            req = G.make_request(x.data_ptr(), snap.fmt, snap.n, snap.fs_hz, snap.f_if_hz, srch.prns, srch.lo,
                                 srch.hi, srch.step, srch.T_coh, srch.N_noncoh, g.data_ptr(), pk.data_ptr())
            for _ in range(warmup):
                c.acquire_device(req, stream)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
            ev[0].record(stream)
            for i in range(steps):
                c.acquire_device(req, stream)
                ev[i + 1].record(stream)
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[-1]) / steps
            res[name] = (ms, g.cpu().numpy().reshape(n_prn, nd, N).astype(np.float64),
                         pk.cpu().numpy().view(G.PEAK_DTYPE).copy())
        finally:
            c.close()
    t32, P32, k32 = res["fp32"]
    modes = {"fp32": {"ms": t32, "value": cells / (t32 / 1e3), "dtype": "f32"}}
    for name in ("fp16", "fp16pfa"):
        t, P, k = res[name]
        mixed = max(float(np.max(np.abs(P[i] - P32[i]) / (P32[i] + P32[i].mean()))) for i in range(n_prn))
        same = int(sum(int(a["detected"]) == int(b["detected"]) and int(a["code_phase"]) == int(b["code_phase"])
                       and int(a["doppler_bin"]) == int(b["doppler_bin"]) for a, b in zip(k, k32)))
        peak_rel = []
        for pl in snap.planted:
            i = srch.prns.index(pl.prn)
            kb, tau = int(k32[i]["doppler_bin"]), int(k32[i]["code_phase"])
            peak_rel.append(abs(P[i, kb, tau] - P32[i, kb, tau]) / P32[i, kb, tau])
        modes[name] = {"ms": t, "value": cells / (t / 1e3), "dtype": "f16", "speedup_vs_fp32": t32 / t,
                       "max_mixed_rel_power_diff_vs_fp32": mixed,
                       "planted_peak_cell_rel_diff_max": max(peak_rel), "detections_identical": same,
                       "prns": n_prn}
    return {"workload": "strong-signal snapshot (real 2-bit IF, 4.092 MHz, 10 ms; 32 PRN x 21 bins x 10 ms)",
            "cells_per_snapshot": cells, "steps": steps, "warmup": warmup, "modes": modes}


def run_precision(args, G, torch, ctx, code_fn):
    """The strong-signal snapshot on the three precisions of the same GPU."""
    codes = {p: code_fn(p) for p in range(1, 38)}  # the GPU's codes, kept past this context
    ctx.close()
    m = precision_measure(G, torch, codes.__getitem__, args.steps, args.warmup)
    head = args.precision if args.precision != "fp32" else "fp16"
    out = {
        "metric": "search cells/s (PRNxDopplerxphasexms) + p50/p99 latency/snapshot",
        "value": m["modes"][head]["value"], "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["modes"][head]["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "%s path on the %s, against the FP32 path on the same GPU" % (head, m["workload"]),
                   "precision": head},
        "modes": m["modes"],
        "source_hash": kernel_source_hash(),
    }
    print(json.dumps(out), flush=True)


def extras(args, G, torch, code_fn) -> dict:
    """The other configurations beside the headline line, each in its own
    try (a failure is reported, never costs the line): the precision
    comparison on the strong snapshot, the heterogeneous batch (FP32 and
    exact-length, one graph replay per step) and served Poisson arrivals
    (FP32 and exact-length)."""
    import numpy as np

    out = {}
    try:
        out["precision"] = precision_measure(G, torch, code_fn, 20, 3)
    except Exception as e:  # noqa: BLE001
        out["precision"] = {"error": "%s: %s" % (type(e).__name__, e)}
    try:
        items, t_gen = batch_items(code_fn, args.batch_n)
        b = {"workload": BATCH_DESC % len(items), "generate_s": t_gen}
        for prec in ("fp32", "fp16pfa"):
            c = G.Context(0, precision=precision_const(G, prec))
            try:
                b[prec] = batch_measure(G, torch, c, items, prec, args.extra_steps, 1)
            except Exception as e:  # noqa: BLE001
                b[prec] = {"error": "%s: %s" % (type(e).__name__, e)}
            finally:
                c.close()
        del items
        out["batch"] = b
    except Exception as e:  # noqa: BLE001
        out["batch"] = {"error": "%s: %s" % (type(e).__name__, e)}
    try:
        prepared = serve_pool(G, code_fn, "mixed")
        sv = {"workload": "served open-loop Poisson arrivals of %s, HBM budget %g GB"
                          % (SERVE_KINDS["mixed"], args.budget_gb)}
        rng = np.random.default_rng(5)
        for prec in ("fp32", "fp16pfa"):
            try:
                sv[prec] = serve_measure(G, prepared, prec, args.extra_rate, args.extra_serve_n,
                                         max(20, args.extra_serve_n // 10), args.budget_gb, rng)
            except Exception as e:  # noqa: BLE001
                sv[prec] = {"error": "%s: %s" % (type(e).__name__, e)}
        out["serve"] = sv
    except Exception as e:  # noqa: BLE001
        out["serve"] = {"error": "%s: %s" % (type(e).__name__, e)}
    return out


if __name__ == "__main__":
    main()

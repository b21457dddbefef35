// gnss_api.hip -- C ABI and host runtime of the acquisition engine.
//
// A context owns one device, one HIP stream (default priority), the
// device-resident tables built once at creation (carrier LUT, C/A codes, FFT
// twiddles, the 2048-point code spectra of all 37 PRNs) and workspaces that
// grow on demand under an HBM budget.  The device keeps every intermediate
// of a request (the paper keeps intermediate results on the GPU and batches
// the whole coherent integration, Sec. 5); a host request crosses the bus
// once in (samples) and once out (peaks, and the grid if asked for).
//
// Every search runs as a batch: the host writes a table of request
// descriptors and per-stage work-item prefix sums into pinned memory, one
// copy moves it to the device, and the stage kernels walk it.  A
// single request is a batch of one; a batch can be captured once into a
// HIP graph and replayed (gnss_graph_*).
#include "fft2048.hpp"
#include "gnss_internal.hpp"
#include "gnss_runtime.hpp"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>

namespace gnss_rt {

thread_local std::string t_err;

int set_err(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

size_t sample_bytes(int fmt, size_t n)
{
    if (fmt == GNSS_CPLX_I8) return 2 * n;
    if (fmt == GNSS_REAL_I8) return n;
    return (n + 3) / 4;
}

// ---------------------------------------------------------------------------
// device memory under the context's HBM budget
// ---------------------------------------------------------------------------
bool inject(std::atomic<int> &countdown)
{
    int v = countdown.load();
    while (v > 0 && !countdown.compare_exchange_weak(v, v - 1)) {
    }
    return v == 1;
}

int copy_async(gnss_ctx *c, void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s)
{
    if (inject(c->fault_copy)) return set_err(GNSS_EDEVICE, "injected copy failure (%zu bytes)", bytes);
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, kind, s));
    return GNSS_OK;
}

int mark_use(Workspace &w, hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &st));
    if (st != hipStreamCaptureStatusNone) return GNSS_OK;
    if (!w.use_ev) HIP_TRY(hipEventCreateWithFlags(&w.use_ev, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(w.use_ev, s));
    w.used = true;
    return GNSS_OK;
}

int ensure_ws(gnss_ctx *c, Workspace &w, DevBuf &b, size_t bytes)
{
    return ensure(c, b, bytes, w.used ? w.use_ev : nullptr);
}

int ensure(gnss_ctx *c, DevBuf &b, size_t bytes, hipEvent_t wait_ev)
{
    if (bytes <= b.cap) return GNSS_OK;
    if (inject(c->fault_alloc)) return set_err(GNSS_ENOMEM, "injected allocation failure (%zu bytes)", bytes);
    std::lock_guard<std::mutex> lk(c->mem_mu);
    const size_t in_use = c->dev_bytes - b.cap;
    if (c->budget && in_use + bytes > c->budget)
        return set_err(GNSS_ENOMEM, "device buffer of %zu bytes exceeds the HBM budget (%zu of %zu in use)",
                       bytes, in_use, c->budget);
    if (b.p) {
        // the old buffer may still be in use by enqueued work: wait for its
        // last use, not for the rest of the device
        if (wait_ev) {
            hipError_t w = hipEventSynchronize(wait_ev);
            if (w != hipSuccess) return set_err(GNSS_EDEVICE, "hipEventSynchronize: %s", hipGetErrorString(w));
        }
        hipError_t e = hipFree(b.p);
        c->dev_bytes -= b.cap;
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return set_err(GNSS_EDEVICE, "hipFree: %s", hipGetErrorString(e));
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return set_err(GNSS_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    b.cap = bytes;
    c->dev_bytes += bytes;
    return GNSS_OK;
}

void release(gnss_ctx *c, DevBuf &b)
{
    if (!b.owned) {
        b = DevBuf{};
        return;
    }
    if (!b.p) return;
    (void)hipFree(b.p);
    std::lock_guard<std::mutex> lk(c->mem_mu);
    c->dev_bytes -= b.cap;
    b.p = nullptr;
    b.cap = 0;
}

void release_ws(gnss_ctx *c, Workspace &w)
{
    if (w.stage_ev) (void)hipEventSynchronize(w.stage_ev);
    if (w.use_ev && w.used) (void)hipEventSynchronize(w.use_ev);
    for (DevBuf *b : {&w.F, &w.G, &w.Q, &w.K, &w.part, &w.grid, &w.meta, &w.samples, &w.peaks, &w.tmeta, &w.tout})
        release(c, *b);
    if (w.h_stage) (void)hipHostFree(w.h_stage);
    if (w.stage_ev) (void)hipEventDestroy(w.stage_ev);
    if (w.use_ev) (void)hipEventDestroy(w.use_ev);
    w.h_stage = nullptr;
    w.h_stage_cap = 0;
    w.stage_ev = nullptr;
    w.use_ev = nullptr;
    w.used = false;
}

// ---------------------------------------------------------------------------
// request validation
// ---------------------------------------------------------------------------
int make_plan(const gnss_request *r, gnss::Plan &p, bool need_outputs)
{
    if (!r) return set_err(GNSS_EINVAL, "request is null");
    if (!r->samples) return set_err(GNSS_EINVAL, "samples is null");
    if (need_outputs && !r->out_peaks) return set_err(GNSS_EINVAL, "out_peaks is null");
    if (!r->prn_list) return set_err(GNSS_EINVAL, "prn_list is null");
    if (r->fmt != GNSS_REAL_I8 && r->fmt != GNSS_CPLX_I8 && r->fmt != GNSS_REAL_2BIT_PACKED)
        return set_err(GNSS_EINVAL, "unknown sample format %d", r->fmt);
    if (r->n_prn < 1 || r->n_prn > gnss::kMaxList)
        return set_err(GNSS_EINVAL, "n_prn %d outside [1, %d]", r->n_prn, gnss::kMaxList);
    for (int i = 0; i < r->n_prn; ++i)
        if (r->prn_list[i] < 1 || r->prn_list[i] > gnss::kMaxPrn)
            return set_err(GNSS_EINVAL, "PRN %d outside [1, 37]", r->prn_list[i]);
    if (!(r->fs > 0.0) || !isfinite(r->fs) || r->fs != floor(r->fs) || r->fs > 9.0e15)
        return set_err(GNSS_EINVAL, "fs must be a positive integer number of Hz");
    const int64_t fs = (int64_t)r->fs;
    if (fs % 1000 != 0) return set_err(GNSS_EINVAL, "fs must be a multiple of 1 kHz");
    if (!isfinite(r->f_if)) return set_err(GNSS_EINVAL, "f_if is not finite");
    if (r->fmt != GNSS_CPLX_I8 && (r->f_if < 0.0 || r->f_if >= r->fs / 2.0))
        return set_err(GNSS_EINVAL, "real samples need 0 <= f_if < fs/2");
    if (!isfinite(r->doppler_lo) || !isfinite(r->doppler_hi) || !isfinite(r->doppler_step) ||
        !(r->doppler_step > 0.0) || r->doppler_hi < r->doppler_lo)
        return set_err(GNSS_EINVAL, "Doppler window needs lo <= hi and step > 0");
    double nd = floor((r->doppler_hi - r->doppler_lo) / r->doppler_step + 1e-9) + 1.0;
    if (nd > 65536.0) return set_err(GNSS_EINVAL, "more than 65536 Doppler bins");
    // the folded and boxcar-summed block is exact in int32: |x LUT| <= 2 * 127 * 4096 per sample,
    // times T_coh_ms (fold) times spc <= 16 (boxcar) stays below 2^31 up to 64 ms
    if (r->T_coh_ms < 1 || r->T_coh_ms > 64) return set_err(GNSS_EINVAL, "T_coh_ms outside [1, 64]");
    if (r->N_noncoh < 1 || r->N_noncoh > 100000) return set_err(GNSS_EINVAL, "N_noncoh outside [1, 100000]");
    // k * 1.023 MHz (k <= 16): the polyphase form on 2048-point or 1023-point
    // transforms; any other whole number of kHz up to N = 16384: zero-padded
    // transforms of length M = 2^ceil(log2(2N))
    p.gen = (fs % 1023000 != 0 || fs / 1023000 > gnss::kMaxSpc) ? 1 : 0;
    if (p.gen && fs / 1000 > gnss::kGenMaxN)
        return set_err(GNSS_ENOTSUP, "fs %lld Hz: more than %d samples per ms (and not k * 1.023 MHz, k <= %d)",
                       (long long)fs, gnss::kGenMaxN, gnss::kMaxSpc);
    p.gen_M = p.gen ? gnss::gen_transform_len((int)(fs / 1000)) : 0;
    p.fmt = r->fmt;
    p.n_samples = (int64_t)r->n;
    p.fs_hz = fs;
    p.f_if = r->f_if;
    p.lo = r->doppler_lo;
    p.step = r->doppler_step;
    p.N = (int)(fs / 1000);
    p.spc = (int)(fs / 1023000);
    p.n_dopp = (int)nd;
    p.Tc = r->T_coh_ms;
    p.Nnc = r->N_noncoh;
    p.n_prn = r->n_prn;
    for (int i = 0; i < gnss::kMaxList; ++i) p.prns.v[i] = i < r->n_prn ? r->prn_list[i] : 0;
    const int64_t used = (int64_t)p.Tc * p.Nnc * p.N;
    if (p.n_samples < used)
        return set_err(GNSS_EINVAL, "record has %lld samples, the search needs %lld", (long long)p.n_samples,
                       (long long)used);
    if ((int64_t)p.n_dopp * p.Nnc > 2147483647LL / 4)
        return set_err(GNSS_EINVAL, "Doppler bins x blocks too large");
    return GNSS_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
static long long cdiv(long long a, long long b) { return (a + b - 1) / b; }
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Lays out the requests of a batch: descriptors, prefix sums of work items
// per stage and workspace sizes.  Device pointers of the request (samples,
// grid, peaks) are copied; null grids get offsets in the workspace grid.
// Parameters of the frequency-domain Doppler variant for one request: the
// smallest P in {1, 2, 4} that makes the Doppler step a whole number kappa of
// bins of the long DFT (length P * T_coh * N, bin spacing 1 / (P T_coh)),
// with P * T_coh * spc a power of two <= 256 (the long DFT is a 2^a x 1023
// prime-factor transform).  Returns false if there is none.
static bool fd_params(const gnss::Plan &p, int &PTc, int &A, int &kappa)
{
    for (int P = 1; P <= 4; P *= 2) {
        const double x = (double)P * p.Tc * p.step / 1000.0;
        const double r = std::nearbyint(x);
        if (r < 1.0 || std::fabs(x - r) > 1e-9 * std::max(1.0, x)) continue;
        const int a = P * p.Tc * p.spc;
        if (a > 256 || (a & (a - 1))) return false;
        PTc = P * p.Tc;
        A = a;
        kappa = (int)r;
        return true;
    }
    return false;
}

// D_k = (uint32)(int64)llround((f_if + f_k) * 2^32 / fs), f_k = lo + k*step,
// each operation rounded once in IEEE double as written (no contraction):
// the carrier NCO of Fig. 2 as a 32-bit phase accumulator.
uint32_t nco_step(double fs, double f_if, double lo, double step, int k)
{
#pragma clang fp contract(off)
    const double fk = lo + (double)k * step;
    const double f = f_if + fk;
    const double x = f * 4294967296.0 / fs;
    return (uint32_t)(long long)llround(x);
}

// Code-Doppler drift of block b at Doppler bin k in samples, reduced to
// [0, N): llround(b Tc N f_k / f_L1), f_L1 = 1575.42 MHz (1540 chip rates),
// in IEEE double as written.  Delaying the folded block by it circularly
// shifts the block's correlation by the same number of lags.
int32_t code_shift(long long b, int Tc, int N, double lo, double step, int k)
{
#pragma clang fp contract(off)
    const double fk = lo + (double)k * step;
    const double x = (double)(b * (long long)Tc * (long long)N) * fk / 1575420000.0;
    long long v = (long long)llround(x) % N;
    return (int32_t)(v < 0 ? v + N : v);
}

// Largest code-Doppler shift table per request ([n_dopp][N_noncoh] int32),
// copied to the device with every batch.
static constexpr long long kMaxShiftTable = 1LL << 22;

void build_batch(const gnss::Plan *plans, const gnss_request *reqs, int n, gnss::CorrShape corr,
                 float threshold, int precision, int doppler_fd, int code_doppler, BatchHost &B)
{
    const int corr_pt = corr.pt, corr_w = corr.w;
    B.d.assign(n, gnss::ReqDesc{});
    B.pre.assign((size_t)gnss::kNumStages * (n + 1), 0);
    B.grid_off.assign(n, -1);
    B.fd = doppler_fd;
    B.fd_bad = -1;
    B.dk.clear();
    B.dk_off.assign(n, 0);
    B.cshift.clear();
    B.cshift_off.assign(n, -1);
    B.cshift_bad = -1;
    long long tot[gnss::kNumStages] = {};
    long long vec = 0, qk = 0, part = 0, grid_int = 0, fd_f2 = 0, gen_f2 = 0;
    B.gen_first = -1;
    B.gen_pmask = 0;
    for (int r = 0; r < n; ++r) {
        const gnss::Plan &p = plans[r];
        gnss::ReqDesc &d = B.d[r];
        d.samples = reqs[r].samples;
        d.grid = reqs[r].out_grid;
        d.peaks = reqs[r].out_peaks;
        d.vec_off = vec;
        d.qk_off = qk;
        d.part_off = part;
        d.lo = p.lo;
        d.step = p.step;
        d.fmt = p.fmt;
        d.N = p.N;
        d.spc = p.spc;
        d.n_dopp = p.n_dopp;
        d.Tc = p.Tc;
        d.Nnc = p.Nnc;
        d.n_prn = p.n_prn;
        d.b0 = p.b0;
        d.acc = p.acc;
        d.n_items = p.gen ? 0 : p.n_dopp * p.spc;
        if (p.gen) {
            d.gen = 1;
            d.gen_M = p.gen_M;
            d.gen_P = std::min(p.gen_M, gnss::kGenLds);
            B.gen_pmask |= (unsigned)d.gen_P;
            d.gen_x_off = gen_f2;
            d.gen_c_off = gen_f2 + (long long)p.n_dopp * p.Nnc * p.gen_M;
            gen_f2 += ((long long)p.n_dopp * p.Nnc + p.n_prn) * p.gen_M;
            if (B.gen_first < 0) B.gen_first = r;
        }
        d.n_ptiles = (int)cdiv(p.n_prn, corr_pt);
        d.n_tau_blk = (int)cdiv(p.N, gnss::kPeakThreads);
        d.threshold = threshold;
        for (int i = 0; i < gnss::kMaxList; ++i) d.prns[i] = p.prns.v[i];
        B.dk_off[r] = (long long)B.dk.size();
        for (int k = 0; k < p.n_dopp; ++k) B.dk.push_back(nco_step((double)p.fs_hz, p.f_if, p.lo, p.step, k));
        if (code_doppler) {
            if ((long long)p.n_dopp * p.Nnc > kMaxShiftTable) {
                if (B.cshift_bad < 0) B.cshift_bad = r;
            } else {
                B.cshift_off[r] = (long long)B.cshift.size();
                for (int k = 0; k < p.n_dopp; ++k)
                    for (int b = 0; b < p.Nnc; ++b)
                        B.cshift.push_back(code_shift(p.b0 + b, p.Tc, p.N, p.lo, p.step, k));
            }
        }
        if (!d.grid) {
            B.grid_off[r] = grid_int;
            grid_int += p.grid_elems();
        }
        long long fd_a = 0, fd_b = 0;
        if (doppler_fd) {
            int PTc = 0, A = 0, kappa = 0;
            if (!p.gen && fd_params(p, PTc, A, kappa)) {
                d.fd = 1;
                d.fd_PTc = PTc;
                d.fd_A = A;
                d.fd_kappa = kappa;
                d.fd_off = fd_f2;
                // cycles per sample of the removed carrier, reduced to [0, 1) and
                // scaled to 2^64 (exact: the fraction has at most 53 bits)
                const double cyc = (p.f_if + p.lo) / (double)p.fs_hz;
                double fr = cyc - std::floor(cyc);
                if (!(fr >= 0.0 && fr < 1.0)) fr = 0.0;
                d.fd_dphase = (unsigned long long)ldexpl((long double)fr, 64);
                // inverse residue map of the A x 1023 prime-factor DFT
                long long inv1 = 0, inv2 = 0;
                for (long long t = 0; t < A; ++t)
                    if ((t * gnss::kCodeLen) % A == 1 % A) { inv1 = t; break; }
                for (long long t = 0; t < gnss::kCodeLen; ++t)
                    if ((t * A) % gnss::kCodeLen == 1) { inv2 = t; break; }
                d.fd_crt1 = (long long)gnss::kCodeLen * inv1;
                d.fd_crt2 = (long long)A * inv2;
                // first-pass and final spectra, then the final spectrum's row maxima
                fd_f2 += 2LL * p.Nnc * A * gnss::kCodeLen + cdiv((long long)p.Nnc * PTc, 2);
                fd_a = (long long)p.Nnc * A;
                fd_b = (long long)p.Nnc * cdiv(gnss::kCodeLen, gnss::kFdCols);
            } else if (B.fd_bad < 0) {
                B.fd_bad = r;
            }
        }
        const long long cnt[gnss::kNumStages] = {
            p.gen ? 0 : (long long)p.n_dopp * p.Nnc, p.n_vec(),
            (long long)d.n_ptiles * cdiv(d.n_items, corr_w), p.detect ? (long long)p.n_prn * d.n_tau_blk : 0,
            p.detect ? (long long)p.n_prn : 0,
            fd_a, fd_b,
            p.gen ? (long long)p.n_dopp * p.Nnc : 0, p.gen ? (long long)p.n_prn : 0,
            p.gen ? (long long)p.n_prn * p.n_dopp : 0};
        for (int st = 0; st < gnss::kNumStages; ++st) {
            B.pre[(size_t)st * (n + 1) + r] = tot[st];
            tot[st] += cnt[st];
        }
        vec += p.n_vec();
        qk += (long long)p.n_prn * p.N;
        part += (long long)p.n_prn * d.n_tau_blk;
    }
    for (int st = 0; st < gnss::kNumStages; ++st) {
        B.pre[(size_t)st * (n + 1) + n] = tot[st];
        B.total[st] = tot[st];
    }
    B.n = n;
    B.corr_pt = corr_pt;
    B.corr_w = corr_w;
    B.precision = precision;
    // the frequency-domain variant has no polyphase vectors in F: its long spectra live there
    B.F_bytes = doppler_fd ? (size_t)fd_f2 * sizeof(float2) : (size_t)vec * gnss::kPolyLen * sizeof(int2);
    // the general-rate block and code spectra (FP32 complex) follow the polyphase spectra
    B.gen_off = align256(gnss::g_bytes(vec, precision));
    B.G_bytes = B.gen_off + (size_t)gen_f2 * sizeof(float2);
    B.Q_bytes = (size_t)qk * sizeof(float);
    B.K_bytes = (size_t)qk * sizeof(int32_t);
    B.part_bytes = (size_t)part * sizeof(float);
    B.grid_bytes = (size_t)grid_int * sizeof(float);
}

// Metadata layout: header, prefix sums, descriptors, NCO steps, shift tables.
struct MetaLayout {
    size_t pre, desc, dk, cshift, total;
};

static MetaLayout meta_layout(const BatchHost &B)
{
    MetaLayout m;
    m.pre = align256(sizeof(gnss::BatchHdr));
    m.desc = m.pre + align256((size_t)gnss::kNumStages * (B.n + 1) * sizeof(long long));
    m.dk = m.desc + align256((size_t)B.n * sizeof(gnss::ReqDesc));
    m.cshift = m.dk + align256(B.dk.size() * sizeof(uint32_t));
    m.total = m.cshift + align256(B.cshift.size() * sizeof(int32_t));
    return m;
}

size_t meta_bytes(const BatchHost &B) { return meta_layout(B).total; }

size_t batch_device_bytes(const BatchHost &B)
{
    return B.F_bytes + B.G_bytes + B.Q_bytes + B.K_bytes + B.part_bytes + B.grid_bytes + meta_bytes(B);
}

// Allocates the workspace of a laid-out batch, fills in internal grid
// pointers, writes the metadata into pinned memory and enqueues its copy to
// the device on stream s.  Returns the kernels' view of the batch in L.
int stage_batch(gnss_ctx *c, Workspace &w, BatchHost &B, hipStream_t s, gnss::Launch &L, bool meta_only)
{
    if (c->nav_pairs && !meta_only) {
        if (c->precision != GNSS_FP16_PFA)
            return set_err(GNSS_ENOTSUP, "nav_pairs needs a GNSS_FP16_PFA context");
        for (int r = 0; r < B.n; ++r)
            if (B.d[r].Nnc % 2)
                return set_err(GNSS_ENOTSUP, "nav_pairs: request %d has an odd N_noncoh (%d)", r, B.d[r].Nnc);
    }
    if (B.fd && !meta_only) {
        if (c->precision != GNSS_FP16_PFA)
            return set_err(GNSS_ENOTSUP, "doppler_fd needs a GNSS_FP16_PFA context");
        if (c->code_doppler)
            return set_err(GNSS_ENOTSUP, "doppler_fd and code_doppler are not supported together");
        if (B.fd_bad >= 0)
            return set_err(GNSS_ENOTSUP,
                           "doppler_fd: request %d needs a Doppler step that is a whole number of 1/(P T_coh) "
                           "bins for P in {1, 2, 4}, with P T_coh spc a power of two <= 256",
                           B.fd_bad);
    }
    if (B.cshift_bad >= 0)
        return set_err(GNSS_ENOTSUP, "code_doppler: request %d has more than %lld (Doppler bin, block) pairs",
                       B.cshift_bad, kMaxShiftTable);
    if (c->nav_pairs && B.gen_first >= 0 && !meta_only)
        return set_err(GNSS_ENOTSUP, "nav_pairs: request %d is at a sample rate that is not k * 1.023 MHz",
                       B.gen_first);
    int rc;
    const MetaLayout ml = meta_layout(B);
    const size_t mb = ml.total;
    if (!meta_only &&
        ((rc = ensure_ws(c, w, w.F, std::max<size_t>(B.F_bytes, 1))) ||
         (rc = ensure_ws(c, w, w.G, std::max<size_t>(B.G_bytes, 1))) ||
         (rc = ensure_ws(c, w, w.Q, std::max<size_t>(B.Q_bytes, 1))) ||
         (rc = ensure_ws(c, w, w.K, std::max<size_t>(B.K_bytes, 1))) ||
         (rc = ensure_ws(c, w, w.part, std::max<size_t>(B.part_bytes, 1))) ||
         (rc = ensure_ws(c, w, w.grid, std::max<size_t>(B.grid_bytes, 1)))))
        return rc;
    if ((rc = ensure_ws(c, w, w.meta, mb))) return rc;
    unsigned char *dm = (unsigned char *)w.meta.p;
    for (int r = 0; r < B.n; ++r) {
        if (B.grid_off[r] >= 0) B.d[r].grid = (float *)w.grid.p + B.grid_off[r];
        B.d[r].nav_pairs = c->nav_pairs;
        B.d[r].dk = (const uint32_t *)(dm + ml.dk) + B.dk_off[r];
        B.d[r].cshift = B.cshift_off[r] >= 0 ? (const int32_t *)(dm + ml.cshift) + B.cshift_off[r] : nullptr;
    }
    // pinned staging: wait until the previous copy out of it has finished
    if (w.stage_ev) HIP_TRY(hipEventSynchronize(w.stage_ev));
    if (w.h_stage_cap < mb) {
        if (w.h_stage) HIP_TRY(hipHostFree(w.h_stage));
        w.h_stage = nullptr;
        w.h_stage_cap = 0;
        HIP_TRY(hipHostMalloc(&w.h_stage, mb, hipHostMallocDefault));
        w.h_stage_cap = mb;
    }
    if (!w.stage_ev) HIP_TRY(hipEventCreateWithFlags(&w.stage_ev, hipEventDisableTiming));
    unsigned char *h = (unsigned char *)w.h_stage;
    memset(h, 0, mb);
    gnss::BatchHdr hdr{};
    hdr.n_req = B.n;
    hdr.corr_pt = B.corr_pt;
    for (int st = 0; st < gnss::kNumStages; ++st) hdr.total[st] = B.total[st];
    memcpy(h, &hdr, sizeof hdr);
    memcpy(h + ml.pre, B.pre.data(), B.pre.size() * sizeof(long long));
    memcpy(h + ml.desc, B.d.data(), (size_t)B.n * sizeof(gnss::ReqDesc));
    if (!B.dk.empty()) memcpy(h + ml.dk, B.dk.data(), B.dk.size() * sizeof(uint32_t));
    if (!B.cshift.empty()) memcpy(h + ml.cshift, B.cshift.data(), B.cshift.size() * sizeof(int32_t));
    HIP_TRY(hipMemcpyAsync(w.meta.p, h, mb, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(w.stage_ev, s));
    L.hdr = (gnss::BatchHdr *)dm;
    L.pre = (const long long *)(dm + ml.pre);
    L.reqs = (const gnss::ReqDesc *)(dm + ml.desc);
    L.n_req = B.n;
    L.corr_pt = B.corr_pt;
    L.corr_w = B.corr_w;
    L.persistent = persistent_for(c, B);
    L.precision = B.precision;
    L.fd = B.fd;
    L.nav_pairs = c->nav_pairs;
    L.gen_off = B.gen_off;
    L.gen_pmask = B.gen_pmask;
    for (int st = 0; st < gnss::kNumStages; ++st) L.total[st] = B.total[st];
    return GNSS_OK;
}

int take_event(gnss_ctx *c, hipEvent_t *ev)
{
    if (!c->event_pool.empty()) {
        *ev = c->event_pool.back();
        c->event_pool.pop_back();
        return GNSS_OK;
    }
    HIP_TRY(hipEventCreate(ev));
    return GNSS_OK;
}

// Waits for the recorded stage events and folds them into the totals.
int harvest_events(gnss_ctx *c)
{
    for (auto &grp : c->pending) {
        HIP_TRY(hipEventSynchronize(grp[GNSS_N_STAGES]));
        for (int i = 0; i < GNSS_N_STAGES; ++i) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, grp[i], grp[i + 1]));
            c->stage_ms[i] += ms;
            c->stage_n[i] += 1;
        }
        for (hipEvent_t e : grp) c->event_pool.push_back(e);
    }
    c->pending.clear();
    return GNSS_OK;
}

// Enqueues a staged batch on stream s, with stage events when profiling.
int launch(gnss_ctx *c, Workspace &w, const gnss::Launch &L, hipStream_t s, bool allow_profile)
{
    int rc;
    std::array<hipEvent_t, GNSS_N_STAGES + 1> ev{};
    const bool prof = allow_profile && c->profile;
    if (prof) {
        if (c->pending.size() >= 4096 && (rc = harvest_events(c))) return rc;
        for (auto &e : ev)
            if ((rc = take_event(c, &e))) return rc;
    }
    if (inject(c->fault_launch)) {
        if (prof)
            for (hipEvent_t e : ev) c->event_pool.push_back(e);
        return set_err(GNSS_EDEVICE, "injected launch failure");
    }
    const gnss::Tables T{c->d_lut,   c->d_tw,   c->d_cs,     c->d_tw_h,
                         c->d_cs_h,  c->d_frags_x, c->d_cs_x, c->cs_exp, c->d_tw_gen, c->d_codes};
    HIP_TRY(gnss::launch_batch(L, T, (int2 *)w.F.p, w.G.p, (float *)w.Q.p, (int32_t *)w.K.p, (float *)w.part.p,
                               c->n_cu, s, prof ? ev.data() : nullptr));
    if (prof) c->pending.push_back(ev);
    return mark_use(w, s);
}

int plan_all(const gnss_request *reqs, int n, std::vector<gnss::Plan> &plans)
{
    if (!reqs || n < 1) return set_err(GNSS_EINVAL, "need at least one request");
    plans.resize(n);
    for (int i = 0; i < n; ++i) {
        int rc = make_plan(&reqs[i], plans[i], true);
        if (rc) {
            std::string m = t_err;
            return set_err(rc, "request %d: %s", i, m.c_str());
        }
    }
    return GNSS_OK;
}

// ---------------------------------------------------------------------------
// workspace of the allocation-free entry point
// ---------------------------------------------------------------------------
// Every GPU that loads the library holds its own copy of this array until the
// process ends.  In host code its name is only a stand-in for the symbol:
// kernels and copies get the device address from scratch_address().
static __device__ __align__(256) unsigned char scratch[GNSS_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_addr;  // device -> address of its copy

// Looks up (once per device, with that device current) the device address of
// this device's copy of `scratch`.
int scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return GNSS_OK;
    }
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return set_err(GNSS_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    }
    g_scratch_addr[device] = p;
    *out = p;
    return GNSS_OK;
}

// Lays the device buffers of a one-request batch out in the scratch array as
// 256-byte-aligned views.  Fails if they do not fit.
static void scratch_offsets(const BatchHost &B, size_t (&sizes)[7], size_t (&off)[7], size_t &end)
{
    const size_t sz[7] = {B.F_bytes, B.G_bytes, B.Q_bytes, B.K_bytes, B.part_bytes, B.grid_bytes, meta_bytes(B)};
    end = 0;
    for (int i = 0; i < 7; ++i) {
        sizes[i] = sz[i];
        off[i] = end;
        end += align256(std::max<size_t>(sz[i], 1));
    }
}

// Whether a laid-out batch fits the allocation-free scratch and staging.
static bool scratch_fits(const BatchHost &B, const Workspace &w)
{
    size_t sizes[7], off[7], end;
    scratch_offsets(B, sizes, off, end);
    return end <= GNSS_NOALLOC_SCRATCH_BYTES && sizes[6] <= w.h_stage_cap;
}

static int scratch_layout(gnss_ctx *c, const BatchHost &B, Workspace &w)
{
    DevBuf *bufs[7] = {&w.F, &w.G, &w.Q, &w.K, &w.part, &w.grid, &w.meta};
    size_t sizes[7], off[7], end;
    scratch_offsets(B, sizes, off, end);
    if (end > GNSS_NOALLOC_SCRATCH_BYTES)
        return set_err(GNSS_ENOMEM, "the request needs %zu bytes of workspace, more than the %zu of the "
                       "allocation-free scratch", end, (size_t)GNSS_NOALLOC_SCRATCH_BYTES);
    if (sizes[6] > w.h_stage_cap)
        return set_err(GNSS_ENOMEM, "the request's %zu bytes of metadata exceed the %zu of the allocation-free "
                       "staging", sizes[6], w.h_stage_cap);
    for (int i = 0; i < 7; ++i) {
        bufs[i]->p = (unsigned char *)c->d_scratch + off[i];
        bufs[i]->cap = align256(std::max<size_t>(sizes[i], 1));
        bufs[i]->owned = false;
    }
    return GNSS_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
int ctx_init_tables(gnss_ctx *c)
{
    const size_t lut_b = 1024 * sizeof(uint32_t);
    const size_t codes_b = (gnss::kMaxPrn + 1) * gnss::kCodeLen;
    const size_t tw_b = gnss::kTwElems * sizeof(float2);
    const size_t cs_b = (size_t)(gnss::kMaxPrn + 1) * gnss::kVec * sizeof(float4);
    const bool h = c->precision == GNSS_FP16, x = c->precision == GNSS_FP16_PFA;
    const size_t tw_gen_b = (size_t)gnss::kGenTwLen * sizeof(float2);
    const size_t table_bytes = lut_b + codes_b + tw_b + cs_b + tw_gen_b +
                               (h ? gnss::kTwHBytes + gnss::kCsHBytes : 0) +
                               (x ? gnss::kFragXBytes + gnss::kCsXBytes : 0);
    if (c->budget && table_bytes > c->budget)
        return set_err(GNSS_ENOMEM, "HBM budget %zu below the %zu bytes of tables", c->budget, table_bytes);
    HIP_TRY(hipMalloc(&c->d_lut, lut_b));
    HIP_TRY(hipMalloc(&c->d_codes, codes_b));
    HIP_TRY(hipMalloc(&c->d_tw, tw_b));
    HIP_TRY(hipMalloc(&c->d_cs, cs_b));
    HIP_TRY(hipMalloc(&c->d_tw_gen, tw_gen_b));
    c->dev_bytes += table_bytes;
    {
        // general rates: W_32768^j = exp(-2 pi i j / 32768), each part from its
        // IEEE double value rounded once to float (host libm; the table is
        // only used by the FP32 zero-padded transforms)
        std::vector<float2> tw((size_t)gnss::kGenTwLen);
        for (int j = 0; j < gnss::kGenTwLen; ++j) {
            const double a = 2.0 * M_PI * (double)j / (double)gnss::kGenTwLen;
            tw[j] = make_float2((float)std::cos(a), (float)-std::sin(a));
        }
        HIP_TRY(hipMemcpy(c->d_tw_gen, tw.data(), tw_gen_b, hipMemcpyHostToDevice));
    }
    c->table_bytes = table_bytes;
    HIP_TRY(gnss::launch_lut(c->d_lut, nullptr, nullptr, c->stream));
    HIP_TRY(gnss::launch_gold_codes(c->d_codes, c->stream));
    HIP_TRY(gnss::launch_twiddles(c->d_tw, c->stream));
    HIP_TRY(gnss::launch_code_spectra(c->d_codes, c->d_tw, c->d_cs, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (h) {
        // common exponent of the FP16 code spectra: max |C| * 2^-cs_exp <= 1
        std::vector<float4> cs((size_t)(gnss::kMaxPrn + 1) * gnss::kVec);
        HIP_TRY(hipMemcpy(cs.data(), c->d_cs, cs_b, hipMemcpyDeviceToHost));
        double m = 0.0;
        for (const float4 &v : cs)
            m = std::max(m, std::max(std::hypot((double)v.x, (double)v.y), std::hypot((double)v.z, (double)v.w)));
        int e = 0;
        while (std::ldexp(1.0, e) < m * (1.0 + 0x1p-10)) ++e;
        c->cs_exp = e;
        HIP_TRY(hipMalloc(&c->d_tw_h, gnss::kTwHBytes));
        HIP_TRY(hipMalloc(&c->d_cs_h, gnss::kCsHBytes));
        HIP_TRY(gnss::launch_tables_h(c->d_cs, c->d_codes, c->d_tw_h, c->d_cs_h, c->cs_exp, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    if (x) {
        // exact 1023-point code spectra in FP64, their common exponent
        // (max |C| * 2^-cs_exp <= 1), then the FP16 fragment tables
        HIP_TRY(hipMalloc(&c->d_frags_x, gnss::kFragXBytes));
        HIP_TRY(hipMalloc(&c->d_cs_x, gnss::kCsXBytes));
        double2 *d_stage = nullptr;
        HIP_TRY(hipMalloc(&d_stage, gnss::kCsXStageBytes));
        std::vector<double2> cs(gnss::kCsXStageBytes / sizeof(double2));
        hipError_t err = gnss::launch_tables_x_frags(c->d_frags_x, c->stream);
        if (err == hipSuccess) err = gnss::launch_code_spectra_x(c->d_codes, d_stage, c->stream);
        if (err == hipSuccess) err = hipMemcpyAsync(cs.data(), d_stage, gnss::kCsXStageBytes, hipMemcpyDeviceToHost,
                                                    c->stream);
        if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
        if (err == hipSuccess) {
            double m = 0.0;
            for (const double2 &v : cs) m = std::max(m, std::hypot(v.x, v.y));
            int e = 0;
            while (std::ldexp(1.0, e) < m * (1.0 + 0x1p-10)) ++e;
            c->cs_exp = e;
            err = gnss::launch_code_spectra_x_pack(d_stage, c->d_cs_x, c->cs_exp, c->stream);
        }
        if (err == hipSuccess) err = hipStreamSynchronize(c->stream);
        (void)hipFree(d_stage);
        HIP_TRY(err);
    }
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, c->device));
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    c->dev_total = prop.totalGlobalMem;
    // set-up of the allocation-free entry point: the device address of the
    // static scratch array, the pinned metadata staging and the events it uses
    int rc = scratch_address(c->device, &c->d_scratch);
    if (rc) return rc;
    HIP_TRY(hipHostMalloc(&c->ws_na.h_stage, GNSS_NOALLOC_META_BYTES, hipHostMallocDefault));
    c->ws_na.h_stage_cap = GNSS_NOALLOC_META_BYTES;
    HIP_TRY(hipEventCreateWithFlags(&c->ws_na.stage_ev, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&c->ws_na.use_ev, hipEventDisableTiming));
    return GNSS_OK;
}

void ctx_free(gnss_ctx *c)
{
    if (!c) return;
    server_stop(c);
    int cur = -1;
    bool switched = hipGetDevice(&cur) == hipSuccess && cur != c->device && hipSetDevice(c->device) == hipSuccess;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release_ws(c, c->ws);
    release_ws(c, c->ws_na);
    for (auto &grp : c->pending)
        for (hipEvent_t e : grp) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    if (c->d_lut) (void)hipFree(c->d_lut);
    if (c->d_codes) (void)hipFree(c->d_codes);
    if (c->d_tw) (void)hipFree(c->d_tw);
    if (c->d_cs) (void)hipFree(c->d_cs);
    if (c->d_tw_gen) (void)hipFree(c->d_tw_gen);
    if (c->d_tw_h) (void)hipFree(c->d_tw_h);
    if (c->d_cs_h) (void)hipFree(c->d_cs_h);
    if (c->d_frags_x) (void)hipFree(c->d_frags_x);
    if (c->d_cs_x) (void)hipFree(c->d_cs_x);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    if (switched) (void)hipSetDevice(cur);
    delete c;
}

DeviceGuard::DeviceGuard(int dev)
{
    if (hipGetDevice(&prev) != hipSuccess) {
        rc = set_err(GNSS_EDEVICE, "hipGetDevice failed");
        return;
    }
    if (prev != dev) {
        hipError_t e = hipSetDevice(dev);
        if (e != hipSuccess) {
            rc = set_err(GNSS_EDEVICE, "hipSetDevice(%d): %s", dev, hipGetErrorString(e));
            return;
        }
        changed = true;
    }
}

DeviceGuard::~DeviceGuard()
{
    if (changed) (void)hipSetDevice(prev);
}

static std::mutex g_default_mu;
static gnss_ctx *g_default = nullptr;

int default_ctx(gnss_ctx **out)
{
    std::lock_guard<std::mutex> dlk(g_default_mu);
    if (!g_default) {
        int rc = gnss_ctx_create(&g_default, 0, 0, GNSS_FP32);
        if (rc) return rc;
    }
    *out = g_default;
    return GNSS_OK;
}


// ---- long requests: passes over the blocks (gnss_runtime.hpp) -------------

void lay_out_pass(gnss_ctx *c, const gnss::Plan &p, const gnss_request &r, int b0, int nb, BatchHost &B)
{
    gnss::Plan q = p;
    q.b0 = b0;
    q.Nnc = nb;
    q.acc = b0 > 0;
    q.detect = b0 + nb == p.Nnc;
    build_batch(&q, &r, 1, corr_shape_for(c, &q, 1), c->threshold, c->precision, c->doppler_fd, c->code_doppler, B);
}

// Whether a layout fits beside what the context holds outside workspace w:
// within the context's HBM budget, or without one within nine tenths of
// what the device has free plus what w holds (w's buffers are replaced when
// they grow); extra: what the call needs besides the batch.
static bool fits_hbm(gnss_ctx *c, const Workspace &w, const BatchHost &B, size_t extra)
{
    const DevBuf *bufs[] = {&w.F, &w.G, &w.Q, &w.K, &w.part, &w.grid, &w.meta, &w.samples, &w.peaks};
    size_t held = 0;
    for (const DevBuf *b : bufs)
        if (b->owned) held += b->cap;
    const size_t need = batch_device_bytes(B) + extra;
    if (c->budget) {
        size_t dev;
        {
            std::lock_guard<std::mutex> lk(c->mem_mu);
            dev = c->dev_bytes;
        }
        const size_t other = dev > held ? dev - held : 0;
        return other + need <= c->budget;
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = c->dev_total / 2;
    }
    return need <= (free_b + held) / 10 * 9;
}

int run_passes(gnss_ctx *c, Workspace &w, const gnss::Plan &p, const gnss_request &r, int nb,
                      hipStream_t s, bool prof, bool scratch, BatchHost &B)
{
    int rc;
    for (int b0 = 0; b0 < p.Nnc; b0 += nb) {
        lay_out_pass(c, p, r, b0, std::min(nb, p.Nnc - b0), B);
        if (scratch && b0 == 0 && (rc = scratch_layout(c, B, w))) return rc;
        gnss::Launch L;
        if ((rc = stage_batch(c, w, B, s, L)) || (rc = launch(c, w, L, s, prof))) return rc;
    }
    return GNSS_OK;
}

}  // namespace gnss_rt

using namespace gnss_rt;

extern "C" {

const char *gnss_strerror(int code)
{
    switch (code) {
    case GNSS_OK: return "ok";
    case GNSS_EINVAL: return "invalid argument";
    case GNSS_ENOMEM: return "out of memory or HBM budget";
    case GNSS_EDEVICE: return "device error";
    case GNSS_EBUSY: return "busy";
    case GNSS_ENOTSUP: return "unsupported configuration";
    default: return "unknown error";
    }
}

const char *gnss_last_error(void) { return t_err.c_str(); }

int gnss_ctx_create(gnss_ctx **out, int device, size_t hbm_budget_bytes, int precision)
{
    if (!out) return set_err(GNSS_EINVAL, "out is null");
    *out = nullptr;
    if (precision != GNSS_FP32 && precision != GNSS_FP16 && precision != GNSS_FP16_PFA)
        return set_err(GNSS_EINVAL, "precision %d is not GNSS_FP32, GNSS_FP16 or GNSS_FP16_PFA", precision);
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count < 1) {
        (void)hipGetLastError();
        return set_err(GNSS_EDEVICE, "no HIP device available");
    }
    if (device < 0 || device >= count) return set_err(GNSS_EINVAL, "device %d outside [0, %d)", device, count);
    gnss_ctx *c = new (std::nothrow) gnss_ctx();
    if (!c) return set_err(GNSS_ENOMEM, "host allocation failed");
    c->device = device;
    c->budget = hbm_budget_bytes;
    c->precision = precision;
    int rc;
    {
        DeviceGuard g(device);
        if (g.rc) {
            delete c;
            return g.rc;
        }
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            c->stream = nullptr;
            ctx_free(c);
            return set_err(GNSS_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        rc = ctx_init_tables(c);
    }
    if (rc) {
        std::string msg = t_err;
        ctx_free(c);
        t_err = msg;
        return rc;
    }
    *out = c;
    return GNSS_OK;
}

void gnss_ctx_destroy(gnss_ctx *ctx) { ctx_free(ctx); }

int gnss_ctx_set(gnss_ctx *ctx, const char *key, double value)
{
    if (!ctx || !key) return set_err(GNSS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!strcmp(key, "threshold")) {
        if (!(value > 0.0) || !isfinite(value)) return set_err(GNSS_EINVAL, "threshold must be > 0");
        ctx->threshold = (float)value;
        return GNSS_OK;
    }
    if (!strcmp(key, "profile")) {
        if (value != 0.0 && value != 1.0) return set_err(GNSS_EINVAL, "profile must be 0 or 1");
        ctx->profile = value != 0.0;
        return GNSS_OK;
    }
    if (!strcmp(key, "hbm_budget")) {
        if (!(value >= 0.0)) return set_err(GNSS_EINVAL, "hbm_budget must be >= 0");
        ctx->budget = (size_t)value;
        return GNSS_OK;
    }
    if (!strcmp(key, "corr_waves")) {
        if (value != 0.0 && (value != floor(value) || (value != 4.0 && value != 6.0 && value != 8.0 && value != 12.0)))
            return set_err(GNSS_EINVAL, "corr_waves must be 0 (tuned) or 4, 6, 8 or 12");
        ctx->corr_w_forced = (int)value;
        return GNSS_OK;
    }
    if (!strcmp(key, "corr_ptile")) {
        if (value != 0.0 && (value != floor(value) || !gnss::corr_ptile_valid((int)value, ctx->precision)))
            return set_err(GNSS_EINVAL, "corr_ptile must be 0 (tuned) or, for this precision, %s",
                           ctx->precision == GNSS_FP32 ? "1, 2 or 4"
                           : ctx->precision == GNSS_FP16 ? "2 or 4" : "1, 2, 4 or 8");
        ctx->corr_pt_forced = (int)value;
        return GNSS_OK;
    }
    if (!strcmp(key, "persistent")) {
        if (value != -1.0 && value != 0.0 && value != 1.0)
            return set_err(GNSS_EINVAL, "persistent must be 0, 1 or -1 (tuned)");
        ctx->persistent_forced = (int)value;
        return GNSS_OK;
    }
    if (!strcmp(key, "nav_pairs")) {
        if (value != 0.0 && value != 1.0) return set_err(GNSS_EINVAL, "nav_pairs must be 0 or 1");
        if (value != 0.0 && ctx->precision != GNSS_FP16_PFA)
            return set_err(GNSS_ENOTSUP, "nav_pairs needs a GNSS_FP16_PFA context");
        ctx->nav_pairs = (int)value;
        return GNSS_OK;
    }
    if (!strcmp(key, "doppler_fd")) {
        if (value != 0.0 && value != 1.0) return set_err(GNSS_EINVAL, "doppler_fd must be 0 or 1");
        if (value != 0.0 && ctx->precision != GNSS_FP16_PFA)
            return set_err(GNSS_ENOTSUP, "doppler_fd needs a GNSS_FP16_PFA context");
        ctx->doppler_fd = (int)value;
        return GNSS_OK;
    }
    if (!strcmp(key, "code_doppler")) {
        if (value != 0.0 && value != 1.0) return set_err(GNSS_EINVAL, "code_doppler must be 0 or 1");
        ctx->code_doppler = (int)value;
        return GNSS_OK;
    }
    if (!strcmp(key, "fault_alloc") || !strcmp(key, "fault_copy") || !strcmp(key, "fault_launch")) {
        if (!(value >= 0.0) || value > 1e9 || value != floor(value))
            return set_err(GNSS_EINVAL, "%s must be a whole number >= 0", key);
        std::atomic<int> &a = key[6] == 'a' ? ctx->fault_alloc : key[6] == 'c' ? ctx->fault_copy : ctx->fault_launch;
        a.store((int)value);
        return GNSS_OK;
    }
    if (!strcmp(key, "block_window")) {
        if (!(value >= 0.0) || value > 1e9 || value != std::floor(value) || (long long)value % gnss::kSumGroup)
            return set_err(GNSS_EINVAL, "block_window must be 0 or a multiple of %d", gnss::kSumGroup);
        ctx->block_window = (int)value;
        return GNSS_OK;
    }
    if (!strcmp(key, "max_slots")) {
        if (!(value >= 1.0) || value > 4096.0) return set_err(GNSS_EINVAL, "max_slots outside [1, 4096]");
        ctx->max_slots = (int)value;
        return GNSS_OK;
    }
    return set_err(GNSS_EINVAL, "unknown option '%s'", key);
}

int gnss_stage_times(gnss_ctx *ctx, double *ms_total, int64_t *launches, int32_t n, int32_t reset)
{
    if (!ctx || !ms_total || !launches || n < GNSS_N_STAGES) return set_err(GNSS_EINVAL, "bad argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    int rc = harvest_events(ctx);
    if (rc) return rc;
    for (int i = 0; i < GNSS_N_STAGES; ++i) {
        ms_total[i] = ctx->stage_ms[i];
        launches[i] = ctx->stage_n[i];
        if (reset) {
            ctx->stage_ms[i] = 0.0;
            ctx->stage_n[i] = 0;
        }
    }
    return GNSS_OK;
}

int gnss_workspace_bytes(const gnss_request *req, size_t *bytes)
{
    if (!bytes) return set_err(GNSS_EINVAL, "bytes is null");
    gnss::Plan p;
    int rc = make_plan(req, p, false);
    if (rc) return rc;
    BatchHost B;
    gnss_request r = *req;
    r.out_grid = nullptr;
    build_batch(&p, &r, 1, gnss::CorrShape{2, gnss::kCorrWaves}, 2.5f, GNSS_FP32, 0, 1, B);  // FP32 and the shift table: the most
    *bytes = batch_device_bytes(B) + sample_bytes(p.fmt, (size_t)p.n_samples) + (size_t)p.n_prn * sizeof(gnss_peak);
    return GNSS_OK;
}

int gnss_acquire_batch_device(gnss_ctx *ctx, const gnss_request *reqs, int32_t n_req, void *stream)
{
    if (!ctx) return set_err(GNSS_EINVAL, "ctx is null");
    std::vector<gnss::Plan> plans;
    int rc = plan_all(reqs, n_req, plans);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    hipStream_t s = (hipStream_t)stream;
    BatchHost B;
    build_batch(plans.data(), reqs, n_req, corr_shape_for(ctx, plans.data(), n_req), ctx->threshold, ctx->precision, ctx->doppler_fd, ctx->code_doppler, B);
    auto fits = [&](const BatchHost &Bx) { return fits_hbm(ctx, ctx->ws, Bx, 0); };
    if (n_req == 1) {
        if (needs_passes(ctx, plans[0], B, fits)) {
            const int nb = pass_blocks(ctx, plans[0], reqs[0], fits);
            if (nb < plans[0].Nnc) return run_passes(ctx, ctx->ws, plans[0], reqs[0], nb, s, true, false, B);
        }
    } else if (!fits(B)) {
        // a batch that does not fit: the requests that need passes run alone
        // in passes, first, and the others as one batch, all on the stream
        std::vector<gnss::Plan> rest_p;
        std::vector<gnss_request> rest_r;
        for (int i = 0; i < n_req; ++i) {
            BatchHost Bi;
            build_batch(&plans[i], &reqs[i], 1, corr_shape_for(ctx, &plans[i], 1), ctx->threshold, ctx->precision,
                        ctx->doppler_fd, ctx->code_doppler, Bi);
            int nb = plans[i].Nnc;
            if (needs_passes(ctx, plans[i], Bi, fits)) nb = pass_blocks(ctx, plans[i], reqs[i], fits);
            if (nb < plans[i].Nnc) {
                if ((rc = run_passes(ctx, ctx->ws, plans[i], reqs[i], nb, s, true, false, Bi))) {
                    std::string m = t_err;
                    return set_err(rc, "request %d: %s", i, m.c_str());
                }
            } else {
                rest_p.push_back(plans[i]);
                rest_r.push_back(reqs[i]);
            }
        }
        if (rest_p.empty()) return GNSS_OK;
        if ((int)rest_p.size() < n_req)
            build_batch(rest_p.data(), rest_r.data(), (int)rest_p.size(), corr_shape_for(ctx, rest_p.data(), (int)rest_p.size()),
                        ctx->threshold, ctx->precision, ctx->doppler_fd, ctx->code_doppler, B);
    }
    gnss::Launch L;
    if ((rc = stage_batch(ctx, ctx->ws, B, s, L))) return rc;
    return launch(ctx, ctx->ws, L, s, true);
}

int gnss_acquire_device(gnss_ctx *ctx, const gnss_request *req, void *stream)
{
    return gnss_acquire_batch_device(ctx, req, 1, stream);
}

int gnss_acquire_device_noalloc(gnss_ctx *ctx, const gnss_request *req, void *stream)
{
    if (!ctx) return set_err(GNSS_EINVAL, "ctx is null");
    gnss::Plan p;
    int rc = make_plan(req, p, true);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    if (!ctx->d_scratch) return set_err(GNSS_EDEVICE, "the context has no scratch address");
    hipStream_t s = (hipStream_t)stream;
    BatchHost B;
    build_batch(&p, req, 1, corr_shape_for(ctx, &p, 1), ctx->threshold, ctx->precision, ctx->doppler_fd,
                ctx->code_doppler, B);
    Workspace &w = ctx->ws_na;
    // every buffer gets the capacity the batch needs in the scratch, and the
    // staging and its events exist: staging and launch allocate nothing
    auto fits = [&](const BatchHost &Bx) { return scratch_fits(Bx, w); };
    if (needs_passes(ctx, p, B, fits)) {
        const int nb = pass_blocks(ctx, p, *req, fits);
        if (nb < p.Nnc) return run_passes(ctx, w, p, *req, nb, s, false, true, B);
    }
    if ((rc = scratch_layout(ctx, B, w))) return rc;
    gnss::Launch L;
    if ((rc = stage_batch(ctx, w, B, s, L))) return rc;
    return launch(ctx, w, L, s, false);
}

int gnss_acquire(const void *samples, int32_t fmt, size_t n, double fs, double f_if,
                 const int32_t *prn_list, int32_t n_prn, double doppler_lo, double doppler_hi,
                 double doppler_step, int32_t T_coh_ms, int32_t N_noncoh, float *out_grid,
                 gnss_peak *out_peaks)
{
    gnss_request r;
    r.samples = samples;
    r.fmt = fmt;
    r.n = n;
    r.fs = fs;
    r.f_if = f_if;
    r.prn_list = prn_list;
    r.n_prn = n_prn;
    r.doppler_lo = doppler_lo;
    r.doppler_hi = doppler_hi;
    r.doppler_step = doppler_step;
    r.T_coh_ms = T_coh_ms;
    r.N_noncoh = N_noncoh;
    r.out_grid = out_grid;
    r.out_peaks = out_peaks;
    gnss::Plan p;
    int rc = make_plan(&r, p, true);
    if (rc) return rc;
    std::lock_guard<std::mutex> dlk(g_default_mu);
    if (!g_default) {
        rc = gnss_ctx_create(&g_default, 0, 0, GNSS_FP32);
        if (rc) return rc;
    }
    gnss_ctx *c = g_default;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (g.rc) return g.rc;
    Workspace &w = c->ws;
    const size_t sb = sample_bytes(fmt, n);
    const size_t pb = (size_t)n_prn * sizeof(gnss_peak);
    if ((rc = ensure_ws(c, w, w.samples, sb)) || (rc = ensure_ws(c, w, w.peaks, pb))) return rc;
    if ((rc = copy_async(c, w.samples.p, samples, sb, hipMemcpyHostToDevice, c->stream))) return rc;
    gnss_request dr = r;
    dr.samples = w.samples.p;
    dr.out_grid = nullptr;  // workspace grid, copied out below
    dr.out_peaks = (gnss_peak *)w.peaks.p;
    BatchHost B;
    build_batch(&p, &dr, 1, corr_shape_for(c, &p, 1), c->threshold, c->precision, c->doppler_fd, c->code_doppler, B);
    auto fits = [&](const BatchHost &Bx) { return fits_hbm(c, w, Bx, sb + pb); };
    int nb = p.Nnc;
    if (needs_passes(c, p, B, fits)) nb = pass_blocks(c, p, dr, fits);
    gnss::Launch L;
    if (nb < p.Nnc ? (rc = run_passes(c, w, p, dr, nb, c->stream, true, false, B))
                   : ((rc = stage_batch(c, w, B, c->stream, L)) || (rc = launch(c, w, L, c->stream, true)))) {
        (void)hipStreamSynchronize(c->stream);
        return rc;
    }
    if ((out_grid && (rc = copy_async(c, out_grid, B.d[0].grid, (size_t)p.grid_elems() * sizeof(float),
                                      hipMemcpyDeviceToHost, c->stream))) ||
        (rc = copy_async(c, out_peaks, w.peaks.p, pb, hipMemcpyDeviceToHost, c->stream))) {
        (void)hipStreamSynchronize(c->stream);
        return rc;
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return GNSS_OK;
}

// ---- captured batches ----------------------------------------------------

int gnss_graph_create(gnss_ctx *ctx, const gnss_request *reqs, int32_t n_req, gnss_graph **out)
{
    if (!ctx || !out) return set_err(GNSS_EINVAL, "null argument");
    *out = nullptr;
    std::vector<gnss::Plan> plans;
    int rc = plan_all(reqs, n_req, plans);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    gnss_graph *gr = new (std::nothrow) gnss_graph();
    if (!gr) return set_err(GNSS_ENOMEM, "host allocation failed");
    gr->ctx = ctx;
    BatchHost B;
    build_batch(plans.data(), reqs, n_req, corr_shape_for(ctx, plans.data(), n_req), ctx->threshold, ctx->precision, ctx->doppler_fd, ctx->code_doppler, B);
    gr->corr_pt = B.corr_pt;
    gr->corr_w = B.corr_w;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete gr;
        return set_err(GNSS_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    gnss::Launch L;
    // allocate and fill everything before capture (no allocation inside it)
    rc = stage_batch(ctx, gr->ws, B, cs, L);
    if (!rc) {
        e = hipStreamSynchronize(cs);
        if (e != hipSuccess) rc = set_err(GNSS_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    if (!rc) {
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) rc = set_err(GNSS_EDEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    if (!rc) {
        // the metadata copy is part of the graph (pinned source, contents fixed)
        const size_t mb = meta_bytes(B);
        e = hipMemcpyAsync(gr->ws.meta.p, gr->ws.h_stage, mb, hipMemcpyHostToDevice, cs);
        int rc2 = e == hipSuccess ? launch(ctx, gr->ws, L, cs, false)
                                  : set_err(GNSS_EDEVICE, "hipMemcpyAsync: %s", hipGetErrorString(e));
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        if (rc2) rc = rc2;
        else if (e != hipSuccess) rc = set_err(GNSS_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        if (!rc) {
            e = hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = set_err(GNSS_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
        if (!rc) {
            e = hipEventCreateWithFlags(&gr->done, hipEventDisableTiming);
            if (e != hipSuccess) {
                gr->done = nullptr;
                rc = set_err(GNSS_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
            }
        }
        if (graph) (void)hipGraphDestroy(graph);
    }
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (gr->done) (void)hipEventDestroy(gr->done);
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        release_ws(ctx, gr->ws);
        delete gr;
        return rc;
    }
    *out = gr;
    return GNSS_OK;
}

int gnss_graph_launch(gnss_graph *graph, void *stream)
{
    if (!graph || !graph->exec) return set_err(GNSS_EINVAL, "graph is null");
    DeviceGuard g(graph->ctx->device);
    if (g.rc) return g.rc;
    HIP_TRY(hipGraphLaunch(graph->exec, (hipStream_t)stream));
    HIP_TRY(hipEventRecord(graph->done, (hipStream_t)stream));
    return GNSS_OK;
}

void gnss_graph_destroy(gnss_graph *graph)
{
    if (!graph) return;
    DeviceGuard g(graph->ctx->device);
    // the last launch (replays do not overlap), not the rest of the device
    if (graph->done) {
        (void)hipEventSynchronize(graph->done);
        (void)hipEventDestroy(graph->done);
    }
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    release_ws(graph->ctx, graph->ws);
    delete graph;
}

// ---- stage entry points -------------------------------------------------

int gnss_gold_codes(gnss_ctx *ctx, const int32_t *prn_list, int32_t n_prn, uint8_t *d_codes, void *stream)
{
    if (!ctx || !prn_list || !d_codes) return set_err(GNSS_EINVAL, "null argument");
    if (n_prn < 1 || n_prn > gnss::kMaxList) return set_err(GNSS_EINVAL, "n_prn outside [1, 64]");
    for (int i = 0; i < n_prn; ++i)
        if (prn_list[i] < 1 || prn_list[i] > gnss::kMaxPrn) return set_err(GNSS_EINVAL, "PRN outside [1, 37]");
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    hipStream_t s = (hipStream_t)stream;
    // rows of the context's generated table, gathered in list order
    for (int i = 0; i < n_prn; ++i)
        HIP_TRY(hipMemcpyAsync(d_codes + (size_t)i * gnss::kCodeLen, ctx->d_codes + prn_list[i] * gnss::kCodeLen,
                               gnss::kCodeLen, hipMemcpyDeviceToDevice, s));
    return GNSS_OK;
}

int gnss_code_replica(gnss_ctx *ctx, const int32_t *prn_list, int32_t n_prn, double fs, size_t n,
                      int8_t *d_out, void *stream)
{
    if (!ctx || !prn_list || !d_out) return set_err(GNSS_EINVAL, "null argument");
    if (n_prn < 1 || n_prn > gnss::kMaxList) return set_err(GNSS_EINVAL, "n_prn outside [1, 64]");
    gnss::PrnList pl;
    for (int i = 0; i < gnss::kMaxList; ++i) {
        if (i < n_prn && (prn_list[i] < 1 || prn_list[i] > gnss::kMaxPrn))
            return set_err(GNSS_EINVAL, "PRN outside [1, 37]");
        pl.v[i] = i < n_prn ? prn_list[i] : 0;
    }
    if (!(fs >= 1.0) || fs != floor(fs) || fs > 9.0e15) return set_err(GNSS_EINVAL, "fs must be a positive integer");
    if (n == 0) return GNSS_OK;
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    HIP_TRY(gnss::launch_code_replica(ctx->d_codes, pl, n_prn, (int64_t)fs, (int64_t)n, d_out, (hipStream_t)stream));
    return GNSS_OK;
}

int gnss_nco_lut(gnss_ctx *ctx, int16_t *d_cos, int16_t *d_sin, void *stream)
{
    if (!ctx || !d_cos || !d_sin) return set_err(GNSS_EINVAL, "null argument");
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    HIP_TRY(gnss::launch_lut(nullptr, d_cos, d_sin, (hipStream_t)stream));
    return GNSS_OK;
}

// A one-request batch whose metadata (descriptor and NCO steps) is staged in
// the context's workspace for a stage entry point; no search workspace.
static int stage_one(gnss_ctx *ctx, const gnss_request *req, gnss::Plan &p, hipStream_t s, BatchHost &B,
                     gnss::Launch &L)
{
    int rc = make_plan(req, p, false);
    if (rc) return rc;
    gnss_request r = *req;
    r.out_grid = nullptr;
    build_batch(&p, &r, 1, gnss::CorrShape{2, gnss::corr_waves(ctx->precision, 2)}, ctx->threshold, ctx->precision, 0, ctx->code_doppler, B);
    return stage_batch(ctx, ctx->ws, B, s, L, true);
}

int gnss_wipe_fold(gnss_ctx *ctx, const gnss_request *req, int32_t *d_out, void *stream)
{
    if (!ctx || !d_out) return set_err(GNSS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    gnss::Plan p;
    BatchHost B;
    gnss::Launch L;
    hipStream_t s = (hipStream_t)stream;
    int rc = stage_one(ctx, req, p, s, B, L);
    if (rc) return rc;
    HIP_TRY(gnss::launch_wipe_fold(L, p, ctx->d_lut, d_out, s));
    return mark_use(ctx->ws, s);
}

int gnss_box_fold(gnss_ctx *ctx, const gnss_request *req, int32_t *d_out, void *stream)
{
    if (!ctx || !d_out) return set_err(GNSS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    gnss::Plan p;
    BatchHost B;
    gnss::Launch L;
    hipStream_t s = (hipStream_t)stream;
    int rc = stage_one(ctx, req, p, s, B, L);
    if (rc) return rc;
    if (p.gen)
        return set_err(GNSS_ENOTSUP, "the boxcar and polyphase split need fs = k * 1.023 MHz, k <= %d",
                       gnss::kMaxSpc);
    HIP_TRY(gnss::launch_box(L, ctx->d_lut, (int2 *)d_out, ctx->n_cu, s));
    return mark_use(ctx->ws, s);
}

int gnss_fft2048(gnss_ctx *ctx, const float *d_in, float *d_out, int32_t batch, int32_t inverse, void *stream)
{
    if (!ctx || !d_in || !d_out) return set_err(GNSS_EINVAL, "null argument");
    if (batch < 0) return set_err(GNSS_EINVAL, "batch < 0");
    if (batch == 0) return GNSS_OK;
    if (d_in == d_out) return set_err(GNSS_EINVAL, "in-place transform is not supported");
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    HIP_TRY(gnss::launch_fft_test((const float2 *)d_in, (float2 *)d_out, batch, inverse ? 1 : 0, ctx->d_tw,
                                  (hipStream_t)stream));
    return GNSS_OK;
}

int gnss_dft1023(gnss_ctx *ctx, const float *d_in, float *d_out, int32_t batch, int32_t inverse, void *stream)
{
    if (!ctx || !d_in || !d_out) return set_err(GNSS_EINVAL, "null argument");
    if (batch < 0 || batch > (1 << 28)) return set_err(GNSS_EINVAL, "batch outside [0, 2^28]");
    if (ctx->precision != GNSS_FP16_PFA) return set_err(GNSS_ENOTSUP, "gnss_dft1023 needs a GNSS_FP16_PFA context");
    if (batch == 0) return GNSS_OK;
    if (d_in == d_out) return set_err(GNSS_EINVAL, "in-place transform is not supported");
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    HIP_TRY(gnss::launch_dft1023_test((const float2 *)d_in, (float2 *)d_out, batch, inverse ? 1 : 0,
                                      ctx->d_frags_x, (hipStream_t)stream));
    return GNSS_OK;
}

int gnss_peaks(gnss_ctx *ctx, const float *d_grid, const int32_t *prn_list, int32_t n_prn, int32_t n_dopp,
               int32_t N, int32_t spc, double doppler_lo, double doppler_step, gnss_peak *d_peaks, void *stream)
{
    if (!ctx || !d_grid || !prn_list || !d_peaks) return set_err(GNSS_EINVAL, "null argument");
    if (n_prn < 1 || n_prn > gnss::kMaxList || n_dopp < 1 || N < 3 || spc < 0)
        return set_err(GNSS_EINVAL, "bad grid shape");
    if (!isfinite(doppler_lo) || !isfinite(doppler_step)) return set_err(GNSS_EINVAL, "bad Doppler grid");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    // a batch of one request that runs only the detection stages
    BatchHost B;
    B.n = 1;
    B.corr_pt = 2;
    B.d.assign(1, gnss::ReqDesc{});
    gnss::ReqDesc &d = B.d[0];
    d.grid = (float *)d_grid;
    d.peaks = d_peaks;
    d.lo = doppler_lo;
    d.step = doppler_step;
    d.N = N;
    d.spc = spc;
    d.n_dopp = n_dopp;
    d.n_prn = n_prn;
    d.n_tau_blk = (N + gnss::kPeakThreads - 1) / gnss::kPeakThreads;
    d.threshold = ctx->threshold;
    for (int i = 0; i < gnss::kMaxList; ++i) d.prns[i] = i < n_prn ? prn_list[i] : 0;
    B.grid_off.assign(1, -1);
    B.dk_off.assign(1, 0);         // no NCO steps or shift tables: detection only
    B.cshift_off.assign(1, -1);
    const long long cnt[gnss::kNumStages] = {0, 0, 0, (long long)n_prn * d.n_tau_blk, n_prn};
    B.pre.assign((size_t)gnss::kNumStages * 2, 0);
    for (int st = 0; st < gnss::kNumStages; ++st) {
        B.pre[(size_t)st * 2 + 1] = cnt[st];
        B.total[st] = cnt[st];
    }
    B.F_bytes = B.G_bytes = B.grid_bytes = 0;
    B.Q_bytes = (size_t)n_prn * N * sizeof(float);
    B.K_bytes = (size_t)n_prn * N * sizeof(int32_t);
    B.part_bytes = (size_t)n_prn * d.n_tau_blk * sizeof(float);
    gnss::Launch L;
    int rc = stage_batch(ctx, ctx->ws, B, (hipStream_t)stream, L);
    if (rc) return rc;
    return launch(ctx, ctx->ws, L, (hipStream_t)stream, false);
}

}  // extern "C"

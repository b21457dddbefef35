// gnss_api.hip -- C ABI and host runtime of the acquisition engine.
//
// A context owns one device, one HIP stream (default priority), the
// device-resident tables built once at creation (carrier LUT, C/A codes, FFT
// twiddles, the 2048-point code spectra of all 37 PRNs) and a workspace that
// grows on demand under an HBM budget.  The device keeps every intermediate
// of a request (the paper keeps intermediate results on the GPU and batches
// the whole coherent integration, Sec. 5); a host request crosses the bus
// once in (samples) and once out (peaks, and the grid if asked for).
#include "fft2048.hpp"
#include "gnss_internal.hpp"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <array>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace {

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

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return set_err(GNSS_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                           __FILE__, __LINE__);                                           \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

}  // namespace

struct gnss_ctx {
    int device = 0;
    size_t budget = 0;  // 0: unlimited
    int precision = GNSS_FP32;
    float threshold = 2.5f;
    hipStream_t stream = nullptr;
    // tables
    uint32_t *d_lut = nullptr;  // [1024] packed cos16 | sin16 << 16
    uint8_t *d_codes = nullptr; // [38][1023], row = PRN
    float2 *d_tw = nullptr;     // twiddles
    float4 *d_cs = nullptr;     // [38][1024] code spectra, storage order
    size_t table_bytes = 0;
    // workspace
    DevBuf samples, F, G, grid, Q, K, part, peaks;
    // per-stage timing
    bool profile = false;
    std::vector<hipEvent_t> event_pool;
    std::vector<std::array<hipEvent_t, GNSS_N_STAGES + 1>> pending;
    double stage_ms[GNSS_N_STAGES] = {0, 0, 0, 0};
    int64_t stage_n[GNSS_N_STAGES] = {0, 0, 0, 0};
    std::mutex mu;
};

namespace {

size_t ws_total(const gnss_ctx *c)
{
    return c->samples.cap + c->F.cap + c->G.cap + c->grid.cap + c->Q.cap + c->K.cap + c->part.cap +
           c->peaks.cap;
}

int ensure(gnss_ctx *c, DevBuf &b, size_t bytes)
{
    if (bytes <= b.cap) return GNSS_OK;
    size_t other = ws_total(c) - b.cap + c->table_bytes;
    if (c->budget && other + bytes > c->budget)
        return set_err(GNSS_ENOMEM, "workspace of %zu bytes exceeds the HBM budget (%zu of %zu in use)",
                       bytes, other, c->budget);
    if (b.p) {
        // the old buffer may still be in use by enqueued work
        (void)hipDeviceSynchronize();
        hipError_t e = hipFree(b.p);
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
    return GNSS_OK;
}

size_t sample_bytes(int fmt, size_t n)
{
    if (fmt == GNSS_CPLX_I8) return 2 * n;
    if (fmt == GNSS_REAL_I8) return n;
    return (n + 3) / 4;
}

// Validates a request and derives its plan.
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
    if (r->T_coh_ms < 1 || r->T_coh_ms > 16) return set_err(GNSS_EINVAL, "T_coh_ms outside [1, 16]");
    if (r->N_noncoh < 1 || r->N_noncoh > 100000) return set_err(GNSS_EINVAL, "N_noncoh outside [1, 100000]");
    if (fs % 1023000 != 0 || fs / 1023000 > gnss::kMaxSpc)
        return set_err(GNSS_ENOTSUP, "fs %lld Hz is not k * 1.023 MHz with 1 <= k <= %d", (long long)fs,
                       gnss::kMaxSpc);
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

struct WsSizes {
    size_t F, G, grid, Q, K, part, peaks;
};

WsSizes ws_sizes(const gnss::Plan &p)
{
    WsSizes w;
    w.F = (size_t)p.n_vec() * gnss::kPolyLen * sizeof(int2);
    w.G = (size_t)p.n_vec() * gnss::kVec * sizeof(float4);
    w.grid = (size_t)p.grid_elems() * sizeof(float);
    w.Q = (size_t)p.n_prn * p.N * sizeof(float);
    w.K = (size_t)p.n_prn * p.N * sizeof(int32_t);
    w.part = gnss::peak_scratch_part_elems(p) * sizeof(double);
    w.peaks = (size_t)p.n_prn * sizeof(gnss_peak);
    return w;
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

// Enqueues the whole search for a validated plan on stream s.
int run_device(gnss_ctx *c, const gnss::Plan &p, const void *d_samples, float *d_grid_out,
               gnss_peak *d_peaks, hipStream_t s)
{
    WsSizes w = ws_sizes(p);
    int rc;
    if ((rc = ensure(c, c->F, w.F)) || (rc = ensure(c, c->G, w.G)) || (rc = ensure(c, c->Q, w.Q)) ||
        (rc = ensure(c, c->K, w.K)) || (rc = ensure(c, c->part, w.part)))
        return rc;
    float *grid = d_grid_out;
    if (!grid) {
        if ((rc = ensure(c, c->grid, w.grid))) return rc;
        grid = (float *)c->grid.p;
    }
    std::array<hipEvent_t, GNSS_N_STAGES + 1> ev{};
    if (c->profile) {
        if (c->pending.size() >= 4096 && (rc = harvest_events(c))) return rc;
        for (auto &e : ev)
            if ((rc = take_event(c, &e))) return rc;
    }
    auto mark = [&](int i) -> hipError_t { return c->profile ? hipEventRecord(ev[i], s) : hipSuccess; };
    HIP_TRY(mark(0));
    HIP_TRY(gnss::launch_wipe_fold_box(d_samples, p, c->d_lut, (int2 *)c->F.p, s));
    HIP_TRY(mark(1));
    HIP_TRY(gnss::launch_fft_poly((const int2 *)c->F.p, c->d_tw, (float4 *)c->G.p, p.n_vec(), s));
    HIP_TRY(mark(2));
    HIP_TRY(gnss::launch_corr((const float4 *)c->G.p, c->d_cs, c->d_tw, grid, p, s));
    HIP_TRY(mark(3));
    HIP_TRY(gnss::launch_peaks(grid, p, c->threshold, (float *)c->Q.p, (int32_t *)c->K.p,
                               (double *)c->part.p, d_peaks, s));
    HIP_TRY(mark(4));
    if (c->profile) c->pending.push_back(ev);
    return GNSS_OK;
}

int ctx_init_tables(gnss_ctx *c)
{
    const size_t lut_b = 1024 * sizeof(uint32_t);
    const size_t codes_b = (gnss::kMaxPrn + 1) * gnss::kCodeLen;
    const size_t tw_b = gnss::kTwElems * sizeof(float2);
    const size_t cs_b = (size_t)(gnss::kMaxPrn + 1) * gnss::kVec * sizeof(float4);
    c->table_bytes = lut_b + codes_b + tw_b + cs_b;
    if (c->budget && c->table_bytes > c->budget)
        return set_err(GNSS_ENOMEM, "HBM budget %zu below the %zu bytes of tables", c->budget, c->table_bytes);
    HIP_TRY(hipMalloc(&c->d_lut, lut_b));
    HIP_TRY(hipMalloc(&c->d_codes, codes_b));
    HIP_TRY(hipMalloc(&c->d_tw, tw_b));
    HIP_TRY(hipMalloc(&c->d_cs, cs_b));
    HIP_TRY(gnss::launch_lut(c->d_lut, nullptr, nullptr, c->stream));
    HIP_TRY(gnss::launch_gold_codes(c->d_codes, c->stream));
    HIP_TRY(gnss::launch_twiddles(c->d_tw, c->stream));
    HIP_TRY(gnss::launch_code_spectra(c->d_codes, c->d_tw, c->d_cs, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return GNSS_OK;
}

void ctx_free(gnss_ctx *c)
{
    if (!c) return;
    int cur = -1;
    bool switched = hipGetDevice(&cur) == hipSuccess && cur != c->device &&
                    hipSetDevice(c->device) == hipSuccess;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (DevBuf *b : {&c->samples, &c->F, &c->G, &c->grid, &c->Q, &c->K, &c->part, &c->peaks})
        if (b->p) (void)hipFree(b->p);
    for (auto &grp : c->pending)
        for (hipEvent_t e : grp) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
    if (c->d_lut) (void)hipFree(c->d_lut);
    if (c->d_codes) (void)hipFree(c->d_codes);
    if (c->d_tw) (void)hipFree(c->d_tw);
    if (c->d_cs) (void)hipFree(c->d_cs);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    if (switched) (void)hipSetDevice(cur);
    delete c;
}

// Makes ctx->device current for the calling thread, remembering the previous one.
struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    int rc = GNSS_OK;
    explicit DeviceGuard(int dev)
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
    ~DeviceGuard()
    {
        if (changed) (void)hipSetDevice(prev);
    }
};

std::mutex g_default_mu;
gnss_ctx *g_default = nullptr;

}  // namespace

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
    if (precision != GNSS_FP32) return set_err(GNSS_EINVAL, "precision %d is not supported", precision);
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
    WsSizes w = ws_sizes(p);
    *bytes = w.F + w.G + w.grid + w.Q + w.K + w.part + w.peaks + sample_bytes(p.fmt, (size_t)p.n_samples);
    return GNSS_OK;
}

int gnss_acquire_device(gnss_ctx *ctx, const gnss_request *req, void *stream)
{
    if (!ctx) return set_err(GNSS_EINVAL, "ctx is null");
    gnss::Plan p;
    int rc = make_plan(req, p, true);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    hipStream_t s = (hipStream_t)stream;
    return run_device(ctx, p, req->samples, req->out_grid, req->out_peaks, s);
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
    WsSizes w = ws_sizes(p);
    const size_t sb = sample_bytes(fmt, n);
    if ((rc = ensure(c, c->samples, sb)) || (rc = ensure(c, c->peaks, w.peaks)) ||
        (rc = ensure(c, c->grid, w.grid)))
        return rc;
    HIP_TRY(hipMemcpyAsync(c->samples.p, samples, sb, hipMemcpyHostToDevice, c->stream));
    rc = run_device(c, p, c->samples.p, (float *)c->grid.p, (gnss_peak *)c->peaks.p, c->stream);
    if (rc) {
        (void)hipStreamSynchronize(c->stream);
        return rc;
    }
    if (out_grid)
        HIP_TRY(hipMemcpyAsync(out_grid, c->grid.p, w.grid, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(out_peaks, c->peaks.p, w.peaks, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return GNSS_OK;
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
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(gnss::launch_code_replica(ctx->d_codes, pl, n_prn, (int64_t)fs, (int64_t)n, d_out, s));
    return GNSS_OK;
}

int gnss_nco_lut(gnss_ctx *ctx, int16_t *d_cos, int16_t *d_sin, void *stream)
{
    if (!ctx || !d_cos || !d_sin) return set_err(GNSS_EINVAL, "null argument");
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(gnss::launch_lut(nullptr, d_cos, d_sin, s));
    return GNSS_OK;
}

int gnss_wipe_fold(gnss_ctx *ctx, const gnss_request *req, int32_t *d_out, void *stream)
{
    if (!ctx || !d_out) return set_err(GNSS_EINVAL, "null argument");
    gnss::Plan p;
    int rc = make_plan(req, p, false);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(gnss::launch_wipe_fold(req->samples, p, ctx->d_lut, d_out, s));
    return GNSS_OK;
}

int gnss_fft2048(gnss_ctx *ctx, const float *d_in, float *d_out, int32_t batch, int32_t inverse, void *stream)
{
    if (!ctx || !d_in || !d_out) return set_err(GNSS_EINVAL, "null argument");
    if (batch < 0) return set_err(GNSS_EINVAL, "batch < 0");
    if (batch == 0) return GNSS_OK;
    if (d_in == d_out) return set_err(GNSS_EINVAL, "in-place transform is not supported");
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(gnss::launch_fft_test((const float2 *)d_in, (float2 *)d_out, batch, inverse ? 1 : 0, ctx->d_tw, s));
    return GNSS_OK;
}

int gnss_peaks(gnss_ctx *ctx, const float *d_grid, const int32_t *prn_list, int32_t n_prn, int32_t n_dopp,
               int32_t N, int32_t spc, double doppler_lo, double doppler_step, gnss_peak *d_peaks, void *stream)
{
    if (!ctx || !d_grid || !prn_list || !d_peaks) return set_err(GNSS_EINVAL, "null argument");
    if (n_prn < 1 || n_prn > gnss::kMaxList || n_dopp < 1 || N < 3 || spc < 0)
        return set_err(GNSS_EINVAL, "bad grid shape");
    if (!isfinite(doppler_lo) || !isfinite(doppler_step)) return set_err(GNSS_EINVAL, "bad Doppler grid");
    gnss::Plan p{};
    p.n_prn = n_prn;
    p.n_dopp = n_dopp;
    p.N = N;
    p.spc = spc;
    p.lo = doppler_lo;
    p.step = doppler_step;
    for (int i = 0; i < gnss::kMaxList; ++i) p.prns.v[i] = i < n_prn ? prn_list[i] : 0;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    WsSizes w = ws_sizes(p);
    int rc;
    if ((rc = ensure(ctx, ctx->Q, w.Q)) || (rc = ensure(ctx, ctx->K, w.K)) || (rc = ensure(ctx, ctx->part, w.part)))
        return rc;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(gnss::launch_peaks(d_grid, p, ctx->threshold, (float *)ctx->Q.p, (int32_t *)ctx->K.p,
                               (double *)ctx->part.p, d_peaks, s));
    return GNSS_OK;
}

}  // extern "C"

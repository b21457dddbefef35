// gnss_track.hip -- C ABI of the tracking correlators: request validation,
// fixed-point NCO words, request tables, launches.
#include "gnss_internal.hpp"
#include "gnss_runtime.hpp"

#include <math.h>
#include <string.h>

#include <vector>

namespace gnss_rt {

static const double kTwo32 = 4294967296.0;

// Fixed-point words of a channel: each value times 2^32, rounded half away
// from zero (llround) in IEEE double as written; the carrier step is
// carrier_hz * 2^32 / fs.
static int channel_words(const gnss_channel &c, double fs, gnss::TrackCh &w)
{
    if (c.prn < 1 || c.prn > gnss::kMaxPrn) return set_err(GNSS_EINVAL, "PRN %d outside [1, 37]", c.prn);
    if (!isfinite(c.carrier_hz) || fabs(c.carrier_hz) > fs * 1e3)
        return set_err(GNSS_EINVAL, "carrier_hz %g is not finite or too large", c.carrier_hz);
    if (!(c.carrier_phase >= 0.0 && c.carrier_phase < 1.0))
        return set_err(GNSS_EINVAL, "carrier_phase %g outside [0, 1) cycles", c.carrier_phase);
    if (!(c.code_phase >= 0.0 && c.code_phase < 1023.0))
        return set_err(GNSS_EINVAL, "code_phase %g outside [0, 1023) chips", c.code_phase);
    if (!(c.code_rate > 0.0) || !isfinite(c.code_rate) || c.code_rate / fs > 1023.0 / gnss::kTrackThreads)
        return set_err(GNSS_EINVAL, "code_rate %g chips/s outside (0, %g fs]", c.code_rate,
                       1023.0 / gnss::kTrackThreads);
    if (!(c.spacing > 0.0 && c.spacing <= 1.0)) return set_err(GNSS_EINVAL, "spacing %g outside (0, 1] chips", c.spacing);
    w.D = (uint32_t)(int64_t)llround(c.carrier_hz * kTwo32 / fs);
    w.phi0 = (uint32_t)(int64_t)llround(c.carrier_phase * kTwo32);
    w.q0 = (long long)llround(c.code_phase * kTwo32);
    w.R = (long long)llround(c.code_rate * kTwo32 / fs);
    w.dl = (long long)llround(c.spacing * kTwo32);
    w.prn = c.prn;
    w.pad = 0;
    return GNSS_OK;
}

static int check_track(const gnss_track_request *r, bool need_out)
{
    if (!r) return set_err(GNSS_EINVAL, "request is null");
    if (!r->samples) return set_err(GNSS_EINVAL, "samples is null");
    if (need_out && !r->out) return set_err(GNSS_EINVAL, "out is null");
    if (!r->channels) return set_err(GNSS_EINVAL, "channels is null");
    if (r->fmt != GNSS_REAL_I8 && r->fmt != GNSS_CPLX_I8 && r->fmt != GNSS_REAL_2BIT_PACKED)
        return set_err(GNSS_EINVAL, "unknown sample format %d", r->fmt);
    if (!(r->fs > 0.0) || !isfinite(r->fs)) return set_err(GNSS_EINVAL, "fs must be positive");
    if (r->n_channels < 1 || r->n_channels > 256) return set_err(GNSS_EINVAL, "n_channels %d outside [1, 256]", r->n_channels);
    if (r->epoch_len < 1 || r->epoch_len > (1 << 24)) return set_err(GNSS_EINVAL, "epoch_len outside [1, 2^24]");
    if (r->n_epochs < 1) return set_err(GNSS_EINVAL, "n_epochs must be >= 1");
    if (r->start < 0) return set_err(GNSS_EINVAL, "start must be >= 0");
    const long long end = r->start + (long long)r->epoch_len * r->n_epochs;
    if ((unsigned long long)end > (unsigned long long)r->n)
        return set_err(GNSS_EINVAL, "epochs end at sample %lld, the record has %zu", end, r->n);
    return GNSS_OK;
}

// Channel words of a request, with the range check that keeps every code
// phase q0 + n R + dl below 2^62.
static int request_words(const gnss_track_request *r, std::vector<gnss::TrackCh> &out)
{
    const long long end = r->start + (long long)r->epoch_len * r->n_epochs;
    for (int c = 0; c < r->n_channels; ++c) {
        gnss::TrackCh w;
        int rc = channel_words(r->channels[c], r->fs, w);
        if (rc) {
            std::string m = t_err;
            return set_err(rc, "channel %d: %s", c, m.c_str());
        }
        if ((double)end * (double)w.R + (double)w.q0 + (double)w.dl > 0x1p62)
            return set_err(GNSS_EINVAL, "channel %d: code phase exceeds 2^30 chips over the record", c);
        out.push_back(w);
    }
    return GNSS_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Lays out and enqueues a batch of tracking requests (device samples and
// outputs) on stream s, using the workspace's tracking table buffer.
static int track_enqueue(gnss_ctx *c, Workspace &w, const gnss_track_request *reqs, int n, hipStream_t s)
{
    std::vector<gnss::TrackDesc> d(n);
    std::vector<gnss::TrackCh> ch;
    std::vector<long long> pre(n + 1, 0);
    int rc;
    for (int i = 0; i < n; ++i) {
        const gnss_track_request &r = reqs[i];
        if ((rc = check_track(&r, true))) {
            std::string m = t_err;
            return set_err(rc, "request %d: %s", i, m.c_str());
        }
        d[i].samples = r.samples;
        d[i].out = (long long *)r.out;
        d[i].start = r.start;
        d[i].fmt = r.fmt;
        d[i].epoch_len = r.epoch_len;
        d[i].n_epochs = r.n_epochs;
        d[i].n_ch = r.n_channels;
        d[i].ch_off = (int)ch.size();
        if ((rc = request_words(&r, ch))) {
            std::string m = t_err;
            return set_err(rc, "request %d: %s", i, m.c_str());
        }
        pre[i + 1] = pre[i] + r.n_epochs;
    }
    const size_t off_pre = align256((size_t)n * sizeof(gnss::TrackDesc));
    const size_t off_ch = off_pre + align256((size_t)(n + 1) * sizeof(long long));
    const size_t mb = off_ch + ch.size() * sizeof(gnss::TrackCh);
    if ((rc = ensure_ws(c, w, w.tmeta, mb))) return rc;
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
    memcpy(h, d.data(), (size_t)n * sizeof(gnss::TrackDesc));
    memcpy(h + off_pre, pre.data(), (size_t)(n + 1) * sizeof(long long));
    memcpy(h + off_ch, ch.data(), ch.size() * sizeof(gnss::TrackCh));
    HIP_TRY(hipMemcpyAsync(w.tmeta.p, h, mb, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(w.stage_ev, s));
    unsigned char *dm = (unsigned char *)w.tmeta.p;
    HIP_TRY(gnss::launch_track((const gnss::TrackDesc *)dm, (const long long *)(dm + off_pre), n, pre[n],
                               (const gnss::TrackCh *)(dm + off_ch), c->d_codes, c->d_lut, s));
    return mark_use(w, s);
}

}  // namespace gnss_rt

using namespace gnss_rt;

extern "C" {

int gnss_track_device(gnss_ctx *ctx, const gnss_track_request *reqs, int32_t n_req, void *stream)
{
    if (!ctx) return set_err(GNSS_EINVAL, "ctx is null");
    if (!reqs || n_req < 1) return set_err(GNSS_EINVAL, "need at least one request");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    return track_enqueue(ctx, ctx->ws, reqs, n_req, (hipStream_t)stream);
}

int gnss_track(const gnss_track_request *req)
{
    int rc = check_track(req, true);
    if (rc) return rc;
    std::vector<gnss::TrackCh> words;
    if ((rc = request_words(req, words))) return rc;
    gnss_ctx *c = nullptr;
    if ((rc = default_ctx(&c))) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    DeviceGuard g(c->device);
    if (g.rc) return g.rc;
    Workspace &w = c->ws;
    const size_t sb = sample_bytes(req->fmt, req->n);
    const size_t ob = (size_t)req->n_channels * req->n_epochs * 6 * sizeof(long long);
    if ((rc = ensure_ws(c, w, w.samples, sb)) || (rc = ensure_ws(c, w, w.tout, ob))) return rc;
    HIP_TRY(hipMemcpyAsync(w.samples.p, req->samples, sb, hipMemcpyHostToDevice, c->stream));
    gnss_track_request dr = *req;
    dr.samples = w.samples.p;
    dr.out = (int64_t *)w.tout.p;
    if ((rc = track_enqueue(c, w, &dr, 1, c->stream))) {
        (void)hipStreamSynchronize(c->stream);
        return rc;
    }
    HIP_TRY(hipMemcpyAsync(req->out, w.tout.p, ob, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return GNSS_OK;
}

}  // extern "C"

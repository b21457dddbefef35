// gnss_serve.hip -- continuous-batching request loop and the PRN-tile
// autotuner.
//
// The paper's goal is cloud throughput: many client requests processed per
// unit of time while each waits as little as possible (Sec. 1), measured as
// effective running time (Sec. 4).  Here requests are submitted with host
// buffers (copied at submission) and served by one scheduler thread per
// context.  It keeps two batch slots, each with its own HIP stream and
// workspace: while one batch runs, the requests that arrived meanwhile are
// admitted into the other slot as far as the slot's share of the HBM budget
// allows, uploaded and launched, so consecutive batches overlap on the
// device.  A request larger than a slot's share runs alone in passes over
// its blocks, each within the share, when it has more than 256 blocks, and
// otherwise fails with GNSS_ENOMEM; the others wait in arrival order.
#include "gnss_runtime.hpp"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <fstream>
#include <sstream>

namespace gnss_rt {

using Clock = std::chrono::steady_clock;

static double seconds_since(Clock::time_point t0, Clock::time_point t)
{
    return std::chrono::duration<double>(t - t0).count();
}

enum TicketState { kQueued = 0, kRunning, kDone };

struct Ticket {
    uint64_t id = 0;
    gnss_request req{};             // host output pointers of the caller
    std::vector<int32_t> prns;
    gnss::Plan plan{};
    void *h_samples = nullptr;      // pinned copy of the record
    size_t h_samples_cap = 0;
    size_t sample_bytes = 0;
    size_t need_bytes = 0;          // device bytes of this request alone (one pass of it)
    int pass_blocks = 0;            // > 0: runs alone in passes of this many blocks
    int state = kQueued;
    int status = GNSS_OK;
    std::string error;
    int batch_size = 0;
    Clock::time_point t_submit, t_start, t_done;
};

// A batch slot.  All its device buffers are views into one arena that grows
// geometrically, up to the slot's share of the budget, and is never resized
// for a batch that fits: the per-batch layout changes, the allocation does not.
struct Slot {
    Workspace ws;                  // device fields: views into the arena
    DevBuf arena, samples, peaks, grids;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<Ticket *> members;
    std::vector<size_t> sample_off, peak_off, grid_off;
    void *h_peaks = nullptr;        // pinned results
    size_t h_peaks_cap = 0;
};

// Reusable pinned host buffers for submitted records (pinned allocation is
// slow compared with a request's service time).
struct PinnedPool {
    std::mutex mu;
    std::multimap<size_t, void *> free;  // capacity -> buffer
    size_t held = 0;
    static constexpr size_t kMaxHeld = (size_t)4 << 30;

    void *take(size_t bytes, size_t *cap)
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = free.lower_bound(bytes);
            if (it != free.end() && it->first <= 2 * bytes + 4096) {
                void *p = it->second;
                *cap = it->first;
                held -= it->first;
                free.erase(it);
                return p;
            }
        }
        void *p = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        *cap = bytes;
        return p;
    }
    void give(void *p, size_t cap)
    {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu);
        if (held + cap > kMaxHeld) {
            (void)hipHostFree(p);
            return;
        }
        free.emplace(cap, p);
        held += cap;
    }
    void clear()
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &kv : free) (void)hipHostFree(kv.second);
        free.clear();
        held = 0;
    }
};

struct Server {
    std::thread th;
    std::mutex mu;
    PinnedPool pinned;
    std::condition_variable cv;     // wakes the scheduler
    std::condition_variable done_cv;  // wakes waiters
    bool stop = false;
    std::deque<Ticket *> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Ticket>> tickets;
    uint64_t next_id = 1;
    Slot slots[2];
    Clock::time_point t0 = Clock::now();
};

static size_t slot_budget(gnss_ctx *c)
{
    if (c->budget) return c->budget > c->table_bytes ? (c->budget - c->table_bytes) / 2 : 0;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return (size_t)32 << 30;
    return free_b / 3;  // two slots and headroom
}

// What admission lets into one batch: the slot's share less a reserve for the
// 256-byte alignment of the buffers laid out in the slot's arena.
static size_t admit_budget(gnss_ctx *c)
{
    const size_t share = slot_budget(c), reserve = (size_t)4 << 20;
    return share > reserve ? share - reserve : 0;
}

static int ensure_pinned(void **p, size_t *cap, size_t bytes)
{
    if (*cap >= bytes) return GNSS_OK;
    if (*p) HIP_TRY(hipHostFree(*p));
    *p = nullptr;
    *cap = 0;
    HIP_TRY(hipHostMalloc(p, bytes, hipHostMallocDefault));
    *cap = bytes;
    return GNSS_OK;
}

// Fails every member of a slot's batch with the current error.
static void fail_members(Server &S, Slot &sl, int rc)
{
    std::lock_guard<std::mutex> lk(S.mu);
    for (Ticket *t : sl.members) {
        S.pinned.give(t->h_samples, t->h_samples_cap);
        t->h_samples = nullptr;
        t->status = rc;
        t->error = t_err;
        t->state = kDone;
        t->t_done = Clock::now();
    }
    sl.members.clear();
    sl.busy = false;
    S.done_cv.notify_all();
}

static void release_slot_buffers(gnss_ctx *c, Slot &sl)
{
    (void)hipStreamSynchronize(sl.stream);
    release_ws(c, sl.ws);
    release(c, sl.samples);
    release(c, sl.peaks);
    release(c, sl.grids);
    release(c, sl.arena);
}

static DevBuf view(const DevBuf &arena, size_t off, size_t bytes)
{
    DevBuf v;
    v.p = (char *)arena.p + off;
    v.cap = bytes;
    v.owned = false;
    return v;
}

static int run_slot_once(gnss_ctx *c, Slot &sl);

// Uploads, launches and enqueues the result copies of a formed batch.
static int run_slot(gnss_ctx *c, Slot &sl)
{
    return run_slot_once(c, sl);
}

static int run_slot_once(gnss_ctx *c, Slot &sl)
{
    const int n = (int)sl.members.size();
    size_t sb = 0, pb = 0, gb = 0;
    sl.sample_off.resize(n);
    sl.peak_off.resize(n);
    sl.grid_off.resize(n);
    for (int i = 0; i < n; ++i) {
        Ticket *t = sl.members[i];
        sl.sample_off[i] = sb;
        sb += (t->sample_bytes + 255) & ~(size_t)255;
        sl.peak_off[i] = pb;
        pb += (size_t)t->plan.n_prn * sizeof(gnss_peak);
        sl.grid_off[i] = gb;
        if (t->req.out_grid) gb += (size_t)t->plan.grid_elems() * sizeof(float);
    }
    int rc;
    // a request in passes runs alone, its arena laid out for the first pass
    const int nb = n == 1 ? sl.members[0]->pass_blocks : 0;
    {
        // the batch's layout in the slot's arena: workspace buffers, then the
        // samples, peaks and grids of its requests
        std::vector<gnss_request> rq(n);
        std::vector<gnss::Plan> pl(n);
        for (int i = 0; i < n; ++i) {
            rq[i] = sl.members[i]->req;
            pl[i] = sl.members[i]->plan;
        }
        if (nb) pl[0].Nnc = nb;
        BatchHost P;
        build_batch(pl.data(), rq.data(), n, gnss::CorrShape{2, gnss::corr_waves(c->precision, 2)}, c->threshold, c->precision, c->doppler_fd, c->code_doppler, P);
        const size_t sizes[10] = {P.F_bytes, P.G_bytes, P.Q_bytes, P.K_bytes, P.part_bytes, P.grid_bytes,
                                  meta_bytes(P), sb, pb, gb};
        size_t off[10], need = 0;
        for (int k = 0; k < 10; ++k) {
            off[k] = need;
            need += (std::max<size_t>(sizes[k], 1) + 255) & ~(size_t)255;
        }
        if (need > sl.arena.cap) {
            // grow geometrically, within the slot's share (of the budget, or of the
            // free device memory without one)
            const size_t want = std::max(need, std::min(2 * sl.arena.cap, slot_budget(c)));
            (void)hipStreamSynchronize(sl.stream);
            release_slot_buffers(c, sl);
            if ((rc = ensure(c, sl.arena, want))) return rc;
        }
        DevBuf *bufs[10] = {&sl.ws.F, &sl.ws.G, &sl.ws.Q, &sl.ws.K, &sl.ws.part, &sl.ws.grid, &sl.ws.meta,
                            &sl.samples, &sl.peaks, &sl.grids};
        for (int k = 0; k < 10; ++k) *bufs[k] = view(sl.arena, off[k], std::max<size_t>(sizes[k], 1));
    }
    if ((rc = ensure_pinned(&sl.h_peaks, &sl.h_peaks_cap, pb))) return rc;
    std::vector<gnss_request> reqs(n);
    std::vector<gnss::Plan> plans(n);
    for (int i = 0; i < n; ++i) {
        Ticket *t = sl.members[i];
        if ((rc = copy_async(c, (char *)sl.samples.p + sl.sample_off[i], t->h_samples, t->sample_bytes,
                             hipMemcpyHostToDevice, sl.stream)))
            return rc;
        reqs[i] = t->req;
        reqs[i].samples = (char *)sl.samples.p + sl.sample_off[i];
        reqs[i].prn_list = t->prns.data();
        reqs[i].out_peaks = (gnss_peak *)((char *)sl.peaks.p + sl.peak_off[i]);
        reqs[i].out_grid = t->req.out_grid ? (float *)((char *)sl.grids.p + sl.grid_off[i]) : nullptr;
        plans[i] = t->plan;
    }
    BatchHost B;
    if (nb) {
        if ((rc = run_passes(c, sl.ws, plans[0], reqs[0], nb, sl.stream, false, false, B))) return rc;
    } else {
        build_batch(plans.data(), reqs.data(), n, corr_shape_for(c, plans.data(), n), c->threshold, c->precision, c->doppler_fd, c->code_doppler, B);
        gnss::Launch L;
        if ((rc = stage_batch(c, sl.ws, B, sl.stream, L)) || (rc = launch(c, sl.ws, L, sl.stream, false))) return rc;
    }
    if ((rc = copy_async(c, sl.h_peaks, sl.peaks.p, pb, hipMemcpyDeviceToHost, sl.stream))) return rc;
    for (int i = 0; i < n; ++i) {
        Ticket *t = sl.members[i];
        if (t->req.out_grid)
            HIP_TRY(hipMemcpyAsync(t->req.out_grid, (char *)sl.grids.p + sl.grid_off[i],
                                   (size_t)t->plan.grid_elems() * sizeof(float), hipMemcpyDeviceToHost, sl.stream));
    }
    HIP_TRY(hipEventRecord(sl.done, sl.stream));
    return GNSS_OK;
}

// Delivers a finished slot's results to the callers' buffers.
static void retire_slot(Server &S, Slot &sl)
{
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lk(S.mu);
    for (size_t i = 0; i < sl.members.size(); ++i) {
        Ticket *t = sl.members[i];
        memcpy(t->req.out_peaks, (char *)sl.h_peaks + sl.peak_off[i], (size_t)t->plan.n_prn * sizeof(gnss_peak));
        S.pinned.give(t->h_samples, t->h_samples_cap);
        t->h_samples = nullptr;
        t->state = kDone;
        t->status = GNSS_OK;
        t->t_done = now;
    }
    sl.members.clear();
    sl.busy = false;
    S.done_cv.notify_all();
}

static void server_loop(gnss_ctx *c)
{
    Server &S = *c->server;
    (void)hipSetDevice(c->device);
    for (;;) {
        // retire finished batches
        for (Slot &sl : S.slots) {
            if (!sl.busy) continue;
            hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                retire_slot(S, sl);
            } else if (q != hipErrorNotReady) {
                set_err(GNSS_EDEVICE, "batch failed: %s", hipGetErrorString(q));
                fail_members(S, sl, GNSS_EDEVICE);
            }
        }
        // form a batch in a free slot from the queued requests
        Slot *free_slot = nullptr;
        for (Slot &sl : S.slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        bool launched = false;
        if (free_slot) {
            std::vector<Ticket *> take;
            {
                std::unique_lock<std::mutex> lk(S.mu);
                const size_t cap = admit_budget(c);
                size_t used = 0;
                while (!S.queue.empty() && (int)take.size() < c->max_slots) {
                    Ticket *t = S.queue.front();
                    // a request in passes over its blocks runs alone
                    if (!take.empty() && (t->pass_blocks || used + t->need_bytes > cap)) break;
                    S.queue.pop_front();
                    used += t->need_bytes;
                    t->state = kRunning;
                    t->t_start = Clock::now();
                    take.push_back(t);
                    if (t->pass_blocks) break;
                }
                for (Ticket *t : take) t->batch_size = (int)take.size();
            }
            if (!take.empty()) {
                free_slot->members = take;
                free_slot->busy = true;
                int rc = run_slot(c, *free_slot);
                if (rc) {
                    (void)hipStreamSynchronize(free_slot->stream);
                    fail_members(S, *free_slot, rc);
                }
                launched = true;
            }
        }
        std::unique_lock<std::mutex> lk(S.mu);
        if (S.stop && S.queue.empty() && !S.slots[0].busy && !S.slots[1].busy) break;
        if (!launched) {
            const bool running = S.slots[0].busy || S.slots[1].busy;
            if (running || !S.queue.empty())
                S.cv.wait_for(lk, std::chrono::microseconds(50));
            else
                S.cv.wait_for(lk, std::chrono::milliseconds(20));
        }
    }
}

static int server_start(gnss_ctx *c)
{
    if (c->server) return GNSS_OK;
    Server *S = new (std::nothrow) Server();
    if (!S) return set_err(GNSS_ENOMEM, "host allocation failed");
    for (Slot &sl : S->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            for (Slot &t : S->slots) {
                if (t.done) (void)hipEventDestroy(t.done);
                if (t.stream) (void)hipStreamDestroy(t.stream);
            }
            delete S;
            return set_err(GNSS_EDEVICE, "serving stream setup: %s", hipGetErrorString(e));
        }
    }
    c->server = S;
    c->server->th = std::thread(server_loop, c);
    return GNSS_OK;
}

void server_stop(gnss_ctx *c)
{
    if (!c->server) return;
    Server &S = *c->server;
    {
        std::lock_guard<std::mutex> lk(S.mu);
        S.stop = true;
    }
    S.cv.notify_all();
    if (S.th.joinable()) S.th.join();
    for (Slot &sl : S.slots) {
        // the slot's buffers are views into its arena: the arena is what is freed
        release_slot_buffers(c, sl);
        if (sl.h_peaks) (void)hipHostFree(sl.h_peaks);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto &kv : S.tickets)
        if (kv.second->h_samples) (void)hipHostFree(kv.second->h_samples);
    S.pinned.clear();
    delete c->server;
    c->server = nullptr;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
std::string rate_signature(const gnss::Plan *plans, int n)
{
    std::vector<int> spc;
    for (int i = 0; i < n; ++i) spc.push_back(plans[i].spc);
    std::sort(spc.begin(), spc.end());
    spc.erase(std::unique(spc.begin(), spc.end()), spc.end());
    std::ostringstream os;
    os << "spc";
    for (int v : spc) os << "_" << v;
    return os.str();
}

gnss::CorrShape corr_shape_for(gnss_ctx *c, const gnss::Plan *plans, int n)
{
    // untuned: FP32 tile 1 with 4 waves (three workgroups, i.e. three waves per
    // SIMD; the fastest shape on the weak workload), FP16 tile 2 (PRNs go in
    // pairs), exact-length tile 2; forced options override tile and waves
    gnss::CorrShape s{c->precision == GNSS_FP32 ? 1 : 2, 0};
    {
        std::lock_guard<std::mutex> lk(c->tuned_mu);
        auto it = c->tuned.find(rate_signature(plans, n));
        if (it != c->tuned.end()) s = {it->second.pt, it->second.w};
    }
    if (c->corr_pt_forced && c->corr_pt_forced != s.pt) s = {c->corr_pt_forced, 0};
    if (c->corr_w_forced) s.w = c->corr_w_forced;
    if (!gnss::corr_shape_valid(s, c->precision)) s.w = gnss::corr_waves(c->precision, s.pt);
    return s;
}

int persistent_for(gnss_ctx *c, const BatchHost &B)
{
    if (c->persistent_forced >= 0) return c->persistent_forced;
    std::vector<gnss::Plan> spc(B.n);
    for (int i = 0; i < B.n; ++i) spc[i].spc = B.d[i].spc;
    std::lock_guard<std::mutex> lk(c->tuned_mu);
    auto it = c->tuned.find(rate_signature(spc.data(), B.n));
    return it != c->tuned.end() ? it->second.pers : 1;
}

static std::string device_key(int dev)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName) + "_cu" + std::to_string(prop.multiProcessorCount);
}

// Cache file: one "key tile schedule waves" line per tuned configuration
// (key = device, precision and rate signature).
static void cache_read(const char *path, std::map<std::string, CorrTune> &m)
{
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        CorrTune t;
        if (!(is >> k >> t.pt)) continue;
        if (!(is >> t.pers)) t.pers = 1;
        if (!(is >> t.w)) t.w = 0;
        m[k] = t;
    }
}

static void cache_write(const char *path, const std::map<std::string, CorrTune> &m)
{
    std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        for (auto &kv : m) f << kv.first << " " << kv.second.pt << " " << kv.second.pers << " " << kv.second.w << "\n";
    }
    (void)rename(tmp.c_str(), path);
}

}  // namespace gnss_rt

using namespace gnss_rt;

extern "C" {

int gnss_submit(gnss_ctx *ctx, const gnss_request *req, uint64_t *ticket)
{
    if (!ctx || !ticket) return set_err(GNSS_EINVAL, "null argument");
    gnss::Plan p;
    int rc = make_plan(req, p, true);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if ((rc = server_start(ctx))) return rc;
    }
    std::unique_ptr<Ticket> t(new (std::nothrow) Ticket());
    if (!t) return set_err(GNSS_ENOMEM, "host allocation failed");
    t->req = *req;
    t->prns.assign(req->prn_list, req->prn_list + req->n_prn);
    t->plan = p;
    t->sample_bytes = sample_bytes(p.fmt, (size_t)p.n_samples);
    BatchHost B;
    gnss_request r1 = *req;
    build_batch(&p, &r1, 1, corr_shape_for(ctx, &p, 1), ctx->threshold, ctx->precision, ctx->doppler_fd, ctx->code_doppler, B);
    const size_t fixed = t->sample_bytes + (size_t)p.n_prn * sizeof(gnss_peak) +
                         (req->out_grid ? (size_t)p.grid_elems() * sizeof(float) : 0);
    t->need_bytes = batch_device_bytes(B) + fixed;
    if (t->need_bytes > admit_budget(ctx)) {
        // a long request runs alone in passes over its blocks, each within a slot's share
        auto fits = [&](const BatchHost &Bx) { return batch_device_bytes(Bx) + fixed <= admit_budget(ctx); };
        const int nb = p.Nnc > gnss::kSumGroup ? pass_blocks(ctx, p, r1, fits) : p.Nnc;
        BatchHost Bp;
        if (nb < p.Nnc) lay_out_pass(ctx, p, r1, 0, nb, Bp);
        if (nb >= p.Nnc || !fits(Bp))
            return set_err(GNSS_ENOMEM, "request needs %zu device bytes, more than a batch slot's %zu, even in "
                           "passes of %d blocks", t->need_bytes, admit_budget(ctx), gnss::kSumGroup);
        t->pass_blocks = nb;
        t->need_bytes = batch_device_bytes(Bp) + fixed;
    }
    Server &S = *ctx->server;
    t->h_samples = S.pinned.take(std::max<size_t>(t->sample_bytes, 1), &t->h_samples_cap);
    if (!t->h_samples) return set_err(GNSS_ENOMEM, "pinned allocation of %zu bytes failed", t->sample_bytes);
    memcpy(t->h_samples, req->samples, t->sample_bytes);
    {
        std::lock_guard<std::mutex> lk(S.mu);
        t->id = S.next_id++;
        t->t_submit = Clock::now();
        *ticket = t->id;
        S.queue.push_back(t.get());
        S.tickets[t->id] = std::move(t);
    }
    S.cv.notify_all();
    return GNSS_OK;
}

static void fill_info(const Ticket &t, gnss_ticket_info *info)
{
    if (!info) return;
    info->status = t.status;
    info->batch_size = t.batch_size;
    info->queued_s = seconds_since(t.t_submit, t.t_start);
    info->run_s = seconds_since(t.t_start, t.t_done);
    info->total_s = seconds_since(t.t_submit, t.t_done);
}

int gnss_poll(gnss_ctx *ctx, uint64_t ticket, int *done, gnss_ticket_info *info)
{
    if (!ctx || !done) return set_err(GNSS_EINVAL, "null argument");
    if (!ctx->server) return set_err(GNSS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Server &S = *ctx->server;
    std::lock_guard<std::mutex> lk(S.mu);
    auto it = S.tickets.find(ticket);
    if (it == S.tickets.end()) return set_err(GNSS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Ticket &t = *it->second;
    *done = t.state == kDone;
    if (!*done) return GNSS_OK;
    fill_info(t, info);
    int status = t.status;
    std::string err = t.error;
    S.tickets.erase(it);
    if (status) return set_err(status, "%s", err.c_str());
    return GNSS_OK;
}

int gnss_wait(gnss_ctx *ctx, uint64_t ticket, double timeout_s, gnss_ticket_info *info)
{
    if (!ctx) return set_err(GNSS_EINVAL, "null argument");
    if (!ctx->server) return set_err(GNSS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Server &S = *ctx->server;
    std::unique_lock<std::mutex> lk(S.mu);
    auto it = S.tickets.find(ticket);
    if (it == S.tickets.end()) return set_err(GNSS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Ticket *t = it->second.get();
    auto pred = [&] { return t->state == kDone; };
    if (timeout_s < 0)
        S.done_cv.wait(lk, pred);
    else if (!S.done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
        return set_err(GNSS_EBUSY, "ticket %llu not done after %.3f s", (unsigned long long)ticket, timeout_s);
    fill_info(*t, info);
    int status = t->status;
    std::string err = t->error;
    S.tickets.erase(ticket);
    if (status) return set_err(status, "%s", err.c_str());
    return GNSS_OK;
}

int gnss_autotune(gnss_ctx *ctx, const gnss_request *reqs, int32_t n_req, const char *cache_path,
                  int32_t *chosen_tile, int32_t *chosen_persistent)
{
    if (!ctx) return set_err(GNSS_EINVAL, "ctx is null");
    std::vector<gnss::Plan> plans;
    int rc = plan_all(reqs, n_req, plans);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    if (g.rc) return g.rc;
    const std::string sig = rate_signature(plans.data(), n_req);
    const std::string key =
        device_key(ctx->device) +
        (ctx->precision == GNSS_FP16 ? "/fp16/" : ctx->precision == GNSS_FP16_PFA ? "/fp16pfa/" : "/fp32/") + sig;
    std::map<std::string, CorrTune> cache;
    if (cache_path) cache_read(cache_path, cache);
    auto hit = cache.find(key);
    CorrTune best;
    if (hit != cache.end() && gnss::corr_shape_valid({hit->second.pt, hit->second.w}, ctx->precision) &&
        (hit->second.pers == 0 || hit->second.pers == 1)) {
        best = hit->second;
    } else {
        // every (PRN tile, waves per workgroup, correlation schedule) the
        // precision has, fastest of 3 runs each
        double best_ms = 1e30;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            return set_err(GNSS_EDEVICE, "hipEventCreate failed");
        }
        std::vector<gnss::CorrShape> shapes;
        for (int pt : {1, 2, 4, 8})
            for (int w : {4, 6, 8, 12})
                if (gnss::corr_shape_valid({pt, w}, ctx->precision)) shapes.push_back({pt, w});
        for (const gnss::CorrShape &sh : shapes) {
            for (int pers : {1, 0}) {
                std::lock_guard<std::mutex> lk(ctx->mu);
                BatchHost B;
                build_batch(plans.data(), reqs, n_req, sh, ctx->threshold, ctx->precision, ctx->doppler_fd, ctx->code_doppler, B);
                gnss::Launch L;
                if ((rc = stage_batch(ctx, ctx->ws, B, ctx->stream, L))) break;
                L.persistent = pers;
                double ms_min = 1e30;
                for (int rep = 0; rep < 3 && !rc; ++rep) {
                    float ms = 0.f;
                    if (hipEventRecord(e0, ctx->stream) != hipSuccess) rc = set_err(GNSS_EDEVICE, "hipEventRecord");
                    if (!rc) rc = launch(ctx, ctx->ws, L, ctx->stream, false);
                    if (!rc && (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                        rc = set_err(GNSS_EDEVICE, "timing events failed");
                    if (!rc) ms_min = std::min(ms_min, (double)ms);
                }
                if (rc) break;
                if (ms_min < best_ms) {
                    best_ms = ms_min;
                    best.pt = sh.pt;
                    best.w = sh.w;
                    best.pers = pers;
                }
            }
            if (rc) break;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
        cache[key] = best;
        if (cache_path) cache_write(cache_path, cache);
    }
    {
        std::lock_guard<std::mutex> lk(ctx->tuned_mu);
        ctx->tuned[sig] = best;
    }
    if (chosen_tile) *chosen_tile = best.pt;
    if (chosen_persistent) *chosen_persistent = best.pers;
    return GNSS_OK;
}

}  // extern "C"

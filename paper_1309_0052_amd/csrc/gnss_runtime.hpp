// gnss_runtime.hpp -- host runtime objects shared by the C ABI, the batch
// graphs, the serving loop and the autotuner.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gnss_internal.hpp"

namespace gnss_rt {

int set_err(int code, const char *fmt, ...);
extern thread_local std::string t_err;

#define HIP_TRY(expr)                                                                                \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return ::gnss_rt::set_err(GNSS_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                      __FILE__, __LINE__);                                           \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    bool owned = true;  // false: a view into another allocation (never freed on its own)
};

// Device buffers of one in-flight batch and the pinned staging of its
// metadata.
struct Workspace {
    DevBuf F, G, Q, K, part, grid, meta, samples, peaks;
    DevBuf tmeta, tout;  // tracking: request table and host-call outputs
    void *h_stage = nullptr;
    size_t h_stage_cap = 0;
    hipEvent_t stage_ev = nullptr;
    // recorded after the last enqueued work that uses these buffers: growing a
    // buffer waits for it (not for the whole device)
    hipEvent_t use_ev = nullptr;
    bool used = false;
};

// A laid-out batch on the host.
struct BatchHost {
    int n = 0;
    int corr_pt = 2;
    int corr_w = 8;
    int precision = GNSS_FP32;
    std::vector<gnss::ReqDesc> d;
    std::vector<long long> pre;
    std::vector<long long> grid_off;
    long long total[gnss::kNumStages] = {};
    size_t F_bytes = 0, G_bytes = 0, Q_bytes = 0, K_bytes = 0, part_bytes = 0, grid_bytes = 0;
    int fd = 0;          // frequency-domain Doppler requested
    int fd_bad = -1;     // first request it cannot serve, or -1
    int gen_first = -1;  // first request at a general rate (zero-padded transforms), or -1
    size_t gen_off = 0;  // bytes of the spectrum buffer before the general-rate region
    unsigned gen_pmask = 0;  // general-rate transform lengths P present (bit P)
    // host-computed tables copied with the descriptors: carrier NCO steps of
    // every (request, Doppler bin) and, with code-Doppler compensation, the
    // lag shift of every (request, bin, block); offsets in elements
    std::vector<uint32_t> dk;
    std::vector<long long> dk_off;
    std::vector<int32_t> cshift;
    std::vector<long long> cshift_off;  // -1: no table
    int cshift_bad = -1;  // first request whose shift table would be too large, or -1
};

struct Ticket;
struct Server;

// An autotuned correlation launch: PRN tile, waves per workgroup, schedule.
struct CorrTune {
    int pt = 2, w = 8, pers = 1;
};

}  // namespace gnss_rt

struct gnss_ctx {
    int device = 0;
    int n_cu = 1;
    size_t budget = 0;      // 0: unlimited
    size_t dev_total = 0;   // the device's memory (bytes)
    size_t dev_bytes = 0;   // device bytes held by this context (tables + workspaces)
    size_t table_bytes = 0; // of which the constant tables
    int precision = GNSS_FP32;
    float threshold = 2.5f;
    int corr_pt_forced = 0; // 0: tuned / default
    int corr_w_forced = 0;  // waves per correlation workgroup; 0: tuned / default
    int persistent_forced = -1;  // correlation grid: 1 occupancy-sized with work counters, 0 one
                                 // workgroup per item, -1 tuned / default (1)
    int code_doppler = 0;   // 1: code-Doppler compensation of the non-coherent sum
    int doppler_fd = 0;     // 1: frequency-domain Doppler (exact-length contexts)
    int nav_pairs = 0;      // 1: blocks in pairs, max over the navigation-bit sign (exact-length contexts)
    int max_slots = 64;     // requests per served batch
    int block_window = 0;   // blocks per pass of a request run alone; 0: all that fit
    hipStream_t stream = nullptr;
    // tables
    uint32_t *d_lut = nullptr;  // [1024] packed cos16 | sin16 << 16
    uint8_t *d_codes = nullptr; // [38][1023], row = PRN
    float2 *d_tw = nullptr;     // twiddles
    float4 *d_cs = nullptr;     // [38][1024] code spectra, storage order
    void *d_tw_h = nullptr;     // FP16 contexts: packed twiddles
    void *d_cs_h = nullptr;     //   code spectra * 2^-cs_exp, packed storage order
    void *d_frags_x = nullptr;  // exact-length contexts: weight fragments of the 31/33-point passes
    void *d_cs_x = nullptr;     //   1023-point code spectra * 2^-cs_exp, fragment layout
    int cs_exp = 0;
    float2 *d_tw_gen = nullptr; // general rates: W_32768^j, j < 32768
    gnss_rt::Workspace ws;      // synchronous and device-buffer calls
    // allocation-free searches: this device's copy of the static scratch
    // array, and a workspace of views into it whose pinned metadata staging
    // and events are created with the context
    void *d_scratch = nullptr;
    gnss_rt::Workspace ws_na;
    // autotuned (PRN tile, correlation schedule) per sample-rate signature
    std::map<std::string, gnss_rt::CorrTune> tuned;
    // per-stage timing
    bool profile = false;
    std::vector<hipEvent_t> event_pool;
    std::vector<std::array<hipEvent_t, GNSS_N_STAGES + 1>> pending;
    double stage_ms[GNSS_N_STAGES] = {0, 0, 0, 0};
    int64_t stage_n[GNSS_N_STAGES] = {0, 0, 0, 0};
    gnss_rt::Server *server = nullptr;  // serving loop, created on first submit
    std::mutex mu;      // serialises calls that use ws / timing state
    std::mutex mem_mu;  // dev_bytes accounting
    std::mutex tuned_mu;  // guards `tuned` (read by the serving thread)
    // failure injection for tests (options "fault_alloc", "fault_copy",
    // "fault_launch"): the n-th following device allocation, host/device copy
    // or batch launch of this context fails on the host, before anything is
    // enqueued; 0 = off
    std::atomic<int> fault_alloc{0}, fault_copy{0}, fault_launch{0};
};

struct gnss_graph {
    gnss_ctx *ctx = nullptr;
    gnss_rt::Workspace ws;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after every launch (replays do not overlap)
    int corr_pt = 2;
    int corr_w = 8;
};

namespace gnss_rt {

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    int rc = GNSS_OK;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

size_t sample_bytes(int fmt, size_t n);
// Grows b to at least `bytes` under the HBM budget.  The old buffer is freed
// after `wait_ev` (the last enqueued use of b, if any) has completed.
int ensure(gnss_ctx *c, DevBuf &b, size_t bytes, hipEvent_t wait_ev = nullptr);
// ensure() for a buffer of workspace w
int ensure_ws(gnss_ctx *c, Workspace &w, DevBuf &b, size_t bytes);
// Records w.use_ev on s after work that uses w's buffers (not while s is
// being captured into a graph, whose workspace never grows).
int mark_use(Workspace &w, hipStream_t s);
// True when the countdown reaches this call (failure injection).
bool inject(std::atomic<int> &countdown);
// hipMemcpyAsync with the context's copy-failure injection
int copy_async(gnss_ctx *c, void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
void release(gnss_ctx *c, DevBuf &b);
void release_ws(gnss_ctx *c, Workspace &w);
int make_plan(const gnss_request *r, gnss::Plan &p, bool need_outputs);
int plan_all(const gnss_request *reqs, int n, std::vector<gnss::Plan> &plans);
void build_batch(const gnss::Plan *plans, const gnss_request *reqs, int n, gnss::CorrShape corr, float threshold,
                 int precision, int doppler_fd, int code_doppler, BatchHost &B);
// Bytes of a batch's metadata on the device: header, prefix sums,
// descriptors and the host-computed tables.
size_t meta_bytes(const BatchHost &B);
// carrier NCO step and code-Doppler shift, computed on the host
uint32_t nco_step(double fs, double f_if, double lo, double step, int k);
int32_t code_shift(long long b, int Tc, int N, double lo, double step, int k);
size_t batch_device_bytes(const BatchHost &B);
// meta_only: only the metadata buffer (stage entry points that run one
// stage into a caller's buffer); the search options are then not checked.
int stage_batch(gnss_ctx *c, Workspace &w, BatchHost &B, hipStream_t s, gnss::Launch &L, bool meta_only = false);
int launch(gnss_ctx *c, Workspace &w, const gnss::Launch &L, hipStream_t s, bool allow_profile);

// Long requests run alone in passes over their blocks: each pass a multiple
// of kSumGroup blocks, so that the FP32 kernels group their block sums at
// the same blocks as in one pass (the results are the same bit for bit);
// each pass after the first adds its sums to the grid's and only the last
// detects.  lay_out_pass lays out the pass of blocks b0 .. b0 + nb - 1 of
// request r (plan p); run_passes runs r in passes of nb blocks on stream s
// (scratch: the first pass, the longest, lays out the allocation-free
// scratch and the others run in that layout); B gets the last pass's layout.
void lay_out_pass(gnss_ctx *c, const gnss::Plan &p, const gnss_request &r, int b0, int nb, BatchHost &B);
int run_passes(gnss_ctx *c, Workspace &w, const gnss::Plan &p, const gnss_request &r, int nb, hipStream_t s,
               bool prof, bool scratch, BatchHost &B);

// Whether request r (plan p, one-pass layout B) runs in passes: option
// block_window below its blocks, or a one-pass layout that does not fit.
template <typename Fits>
bool needs_passes(gnss_ctx *c, const gnss::Plan &p, const BatchHost &B, Fits fits)
{
    if (p.Nnc <= gnss::kSumGroup) return false;
    if (c->block_window > 0) return c->block_window < p.Nnc;
    return B.cshift_bad >= 0 || !fits(B);
}

// Blocks per pass: option block_window, else the largest multiple of
// kSumGroup whose pass layout fits (fits(B)); all of them (one pass, which
// then reports the shortage) when not even kSumGroup blocks fit.
template <typename Fits>
int pass_blocks(gnss_ctx *c, const gnss::Plan &p, const gnss_request &r, Fits fits)
{
    if (c->block_window > 0) return std::min(c->block_window, p.Nnc);
    auto ok = [&](int nb) {
        BatchHost B;
        lay_out_pass(c, p, r, 0, nb, B);
        return B.cshift_bad < 0 && fits(B);
    };
    if (p.Nnc <= gnss::kSumGroup || !ok(gnss::kSumGroup)) return p.Nnc;
    int lo = 1, hi = (p.Nnc - 1) / gnss::kSumGroup;  // groups per pass; ok(lo groups)
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (ok(mid * gnss::kSumGroup))
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo * gnss::kSumGroup;
}

// autotuner lookup: the PRN tile for a batch of these plans
gnss::CorrShape corr_shape_for(gnss_ctx *c, const gnss::Plan *plans, int n);
int persistent_for(gnss_ctx *c, const BatchHost &B);
std::string rate_signature(const gnss::Plan *plans, int n);

// serving loop
void server_stop(gnss_ctx *c);

// the internally locked default context of the synchronous host-buffer calls
int default_ctx(gnss_ctx **out);

}  // namespace gnss_rt

/*
 * gnss_acq.h -- C ABI of the MI355X (gfx950) GPS L1 C/A acquisition engine.
 *
 * The engine is the acquisition channel of Karimi, Pamir and Afzal,
 * "Accelerating a Cloud-Based Software GNSS Receiver" (Sec. 3, Figs. 1-2):
 * carrier and code NCOs generate local replicas, the first mixing stage wipes
 * the carrier off the recorded samples, FFTs of the mixed signal and of the
 * code replica are multiplied (frequency-domain correlation) and an IFFT
 * returns the correlation over every code shift, which is used to detect each
 * satellite and to estimate its coarse Doppler and code phase.  Coherent
 * blocks follow the paper's block processing (Sec. 4) and the whole coherent
 * integration is processed as one batch on the device (Sec. 5).
 *
 * Conventions common to every entry point
 *  - Every function returns int: GNSS_OK (0) or a negative GNSS_E* code;
 *    gnss_last_error() then gives a thread-local message.
 *  - Sample rate fs (Hz): any whole number of kHz with N = fs/1000 samples
 *    per millisecond at most 16384 (the paper sizes its replica loops by the
 *    recording's sampling frequency, Sec. 3); larger N gives GNSS_ENOTSUP.
 *    At fs = k * 1.023 MHz with k <= 16 (spc = k samples per chip) the
 *    search uses the polyphase form on 2048-point (FP32, FP16) or 1023-point
 *    (GNSS_FP16_PFA) transforms; at every other rate it correlates each
 *    block on zero-padded FP32 transforms of length M = 2^ceil(log2 2N),
 *    whatever the context's precision.
 *  - Doppler bins f_k = lo + k*step (IEEE double, as written), k = 0..n_dopp-1,
 *    n_dopp = floor((hi - lo)/step + 1e-9) + 1 (both ends inclusive).
 *  - Coherent block b covers samples [b*T*N, (b+1)*T*N), T = T_coh_ms; blocks
 *    start at sample 0 and samples beyond T*N_noncoh*N are ignored.
 *  - Carrier NCO: 32-bit phase, step D_k = (uint32)(int64)llround((f_if + f_k)
 *    * 2^32 / fs), phase of sample n = (uint32)(n * D_k), 1024-entry integer
 *    LUT (amplitude 4096, index = phase >> 22), mixing by exp(-j theta).
 *  - C/A codes: IS-GPS-200 Table 3-Ia, chip value 0 -> +1, 1 -> -1.
 *  - Correlation of block b at lag tau (tau = sample at which chip 0 starts):
 *      R_b[tau] = sum_{n in block b} y[n] * c[(n - tau) mod N]
 *    Power grid P[p][k][tau] = sum_b |R_b[tau]|^2 * 2^-24, FP32, layout
 *    [prn][doppler][tau] (tau fastest).
 *  - Detection per PRN: Q[tau] = max_k P (lowest k on ties), tau* = argmax Q
 *    (lowest tau), second = max Q over circular |tau - tau*| > fs/1.023 MHz
 *    (one chip; at a general rate that is |tau - tau*| > floor(fs/1.023 MHz)),
 *    ratio = peak/second, detected = ratio >= threshold (default 2.5).
 *    Sub-bin refinement: 3-point parabolas in FP64 along tau (circular) and
 *    along Doppler (not at the first or last bin).
 */
#ifndef GNSS_ACQ_H
#define GNSS_ACQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define GNSS_OK 0
#define GNSS_EINVAL (-1)   /* bad argument (null pointer, out-of-range value) */
#define GNSS_ENOMEM (-2)   /* host or device allocation failed, or HBM budget exceeded */
#define GNSS_EDEVICE (-3)  /* a HIP runtime call or kernel launch failed */
#define GNSS_EBUSY (-4)    /* context busy */
#define GNSS_ENOTSUP (-5)  /* valid but unsupported configuration (e.g. fs) */

/* ---- sample formats ---------------------------------------------------- */
#define GNSS_REAL_I8 0          /* one int8 per real sample (2-bit data as -3,-1,1,3) */
#define GNSS_CPLX_I8 1          /* interleaved I, Q int8 per complex sample           */
#define GNSS_REAL_2BIT_PACKED 2 /* 4 real samples per byte, first sample in the low
                                   bits, 00:+1 01:+3 10:-1 11:-3                      */

/* ---- precision --------------------------------------------------------- */
#define GNSS_FP32 0  /* FP32 transforms and power                             */
#define GNSS_FP16 1  /* packed FP16 transforms with per-vector power-of-two
                        scaling; FP32 |.|^2 and block sums                    */
#define GNSS_FP16_PFA 2 /* exact-length 1023-point transforms (Good-Thomas
                        31 x 33, no zero padding) as FP16 x FP16 -> FP32
                        matrix-core products, the same per-vector scaling;
                        FP32 |.|^2 and block sums                            */

/* One detection result per requested PRN (Sec. 3: coarse Doppler and code
 * phase; refined values come from the FP64 parabolas). */
typedef struct gnss_peak {
    int32_t prn;          /* PRN number (1..37)                                */
    int32_t doppler_bin;  /* k* (0-based index into the Doppler grid)          */
    int32_t code_phase;   /* tau* in samples, 0..N-1                           */
    int32_t detected;     /* 1 if ratio >= threshold                           */
    float peak;           /* P[k*][tau*]                                       */
    float second;         /* highest Q outside +-1 chip of tau*                */
    float mean;           /* mean of P over the PRN's grid                     */
    float ratio;          /* peak / second (+inf if second == 0)               */
    double doppler_hz;    /* f_k* + delta_d * step                             */
    double code_phase_frac; /* tau* + delta_c (samples)                        */
} gnss_peak;

typedef struct gnss_ctx gnss_ctx;

/* A request: the arguments of gnss_acquire gathered in one struct. */
typedef struct gnss_request {
    const void *samples;   /* record (host memory for gnss_acquire, device memory
                              for gnss_acquire_device)                         */
    int32_t fmt;           /* GNSS_REAL_I8 / GNSS_CPLX_I8 / GNSS_REAL_2BIT_PACKED */
    size_t n;              /* samples in the record (not bytes)                */
    double fs;             /* sample rate, Hz                                  */
    double f_if;           /* intermediate frequency, Hz (0 for baseband)      */
    const int32_t *prn_list; /* host memory, n_prn PRN numbers in 1..37        */
    int32_t n_prn;         /* 1..64                                            */
    double doppler_lo, doppler_hi, doppler_step; /* Hz                        */
    int32_t T_coh_ms;      /* coherent integration, 1..64 ms                   */
    int32_t N_noncoh;      /* non-coherent blocks, >= 1                        */
    float *out_grid;       /* nullable; n_prn*n_dopp*N floats [prn][dopp][tau] */
    gnss_peak *out_peaks;  /* n_prn entries, same order as prn_list            */
} gnss_request;

/* Synchronous acquisition on host buffers (Sec. 3, Fig. 2).  Uses an
 * internally locked default context on device 0; thread-safe.  samples,
 * prn_list, out_grid (nullable) and out_peaks are host memory owned by the
 * caller; outputs are written before the call returns.  A long request whose
 * workspace does not fit runs in passes over its blocks (see
 * gnss_acquire_device).  Errors: GNSS_EINVAL (arguments), GNSS_ENOTSUP (fs),
 * GNSS_ENOMEM, GNSS_EDEVICE. */
int gnss_acquire(const void *samples, int32_t fmt, size_t n, double fs, double f_if,
                 const int32_t *prn_list, int32_t n_prn, double doppler_lo,
                 double doppler_hi, double doppler_step, int32_t T_coh_ms,
                 int32_t N_noncoh, float *out_grid, gnss_peak *out_peaks);

/* Context: one device, one HIP stream, the device-resident tables (carrier
 * LUT, C/A codes, code spectra, twiddles) and a workspace that grows on
 * demand up to hbm_budget_bytes (0 = no limit).  precision: GNSS_FP32, or
 * GNSS_FP16 for packed FP16 transforms (Fig. 2's FFT, spectrum product and
 * IFFT) with per-vector power-of-two scaling that keeps every intermediate
 * inside the FP16 range, |.|^2 and block sums in FP32, or GNSS_FP16_PFA for
 * the same correlation with exact-length 1023-point transforms whose passes
 * run on the matrix cores (FP16 operands, FP32 accumulation); every search on
 * the context uses it.  Errors: GNSS_EINVAL (unknown precision or device),
 * GNSS_ENOMEM, GNSS_EDEVICE. */
int gnss_ctx_create(gnss_ctx **out, int device, size_t hbm_budget_bytes, int precision);
/* Waits for the context's work, stops its serving thread (unfinished tickets
 * are dropped) and frees its tables and workspaces; NULL is a no-op. */
void gnss_ctx_destroy(gnss_ctx *ctx);

/* Context options (the search parameters of Sec. 3's acquisition channel
 * that the paper leaves open, the serving knobs of the cloud setting of
 * Sec. 1, and test hooks): "threshold" (detection ratio, > 0), "hbm_budget" (bytes,
 * 0 = unlimited; device memory of tables and workspaces), "profile" (1:
 * record per-stage HIP events, see gnss_stage_times; 0: off), "corr_ptile"
 * (PRNs per correlation workgroup: GNSS_FP32 1, 2 or 4, GNSS_FP16 2 or 4,
 * GNSS_FP16_PFA 1, 2, 4 or 8; 0 = autotuned, by default 1 for GNSS_FP32 and
 * 2 otherwise), "corr_waves" (waves, i.e. (Doppler, phase) items, per
 * correlation workgroup: GNSS_FP32 tile 1 runs 12, 6 or 4 at three waves per
 * SIMD, tiles 2 and 4 run 8; the FP16 kernels have one width each; 0 =
 * autotuned, by default 4 for tile 1; a width the tile does not have falls
 * back to its default),
 * "persistent" (grid of the correlation kernel, the dominant one: 1 an
 * occupancy-sized grid whose workgroups take items from per-XCD work counters
 * and then from the other XCDs' ranges; 0 one workgroup per item; -1, the
 * default, the autotuned choice or 1; the other stages always run one
 * workgroup per item),
 * "code_doppler" (1: code-Doppler compensation of the non-coherent sum: the
 * code rate follows the carrier Doppler (f_L1 = 1540 chip rates), so block
 * b's correlation at bin f_k is taken at lag tau - llround(b T_coh N f_k /
 * 1575.42e6) (circular); 0, the default: plain sum), "doppler_fd" (1, only on
 * GNSS_FP16_PFA contexts: frequency-domain Doppler -- the carrier is removed
 * once per block at f_if + doppler_lo by an exact exponential, one
 * zero-padded DFT of length P*T_coh*N per block serves every Doppler bin by a
 * shift of k*kappa bins, and the polyphase block spectra are synthesised from
 * it; needs doppler_step*T_coh*P/1000 a whole number kappa for some P in
 * {1, 2, 4} and P*T_coh*spc a power of two <= 256, else GNSS_ENOTSUP at
 * search time; not with code_doppler, not at general rates.  The grid is then sum_b |R_b|^2 of the
 * exactly wiped blocks, on the scale of the NCO path's 2^-24 |R_b|^2 of its
 * 4096-scaled table; 0, the default: NCO and lookup table as in Fig. 2),
 * "nav_pairs" (1, only on GNSS_FP16_PFA contexts:
 * navigation-bit hypotheses for coherent integration past one 20 ms bit --
 * coherent blocks 2i and 2i+1 are combined with both relative signs and the
 * larger power kept, P = sum_i max(|R_2i + R_2i+1|^2, |R_2i - R_2i+1|^2), so
 * that a data-bit flip between them does not cancel the signal; needs an even
 * N_noncoh and fs = k * 1.023 MHz, else GNSS_ENOTSUP at search time; 0,
 * the default: plain sum),
 * "block_window" (blocks per pass of a request run alone, see
 * gnss_acquire_device: a multiple of 256; 0, the default: all the blocks
 * that fit),
 * "max_slots" (requests per
 * served batch, 1..4096), "fault_alloc" / "fault_copy" / "fault_launch" (n >= 1:
 * the n-th following device allocation, host/device copy or batch launch of
 * the context fails on the host before anything is enqueued, reporting
 * GNSS_ENOMEM, GNSS_EDEVICE and GNSS_EDEVICE; 0: off; for tests of the error
 * paths).
 * Errors: GNSS_EINVAL. */
int gnss_ctx_set(gnss_ctx *ctx, const char *key, double value);

/* Device bytes the context's workspace needs for a request in FP32 (an
 * upper bound for FP16, whose spectra take half the space) searched in one
 * pass: the block and spectrum buffers of the device-resident pipeline
 * (Sec. 5 keeps intermediates on the GPU); does not allocate.  A request run
 * alone that needs more than the context can hold runs in passes in less.
 * Errors: as gnss_acquire's argument checks. */
int gnss_workspace_bytes(const gnss_request *req, size_t *bytes);

/* Acquisition on device buffers (Sec. 3, Fig. 2; the whole coherent
 * integration as one device batch, Sec. 5).  req->samples, req->out_grid
 * (nullable) and req->out_peaks are device pointers; req->prn_list is host
 * memory.  Work is enqueued on `stream` (a hipStream_t; NULL = the HIP null
 * stream, which is PyTorch's default stream) and the call returns without waiting; outputs are valid once
 * the stream reaches that point.  The context's workspace is reused, so calls
 * on one context must not overlap on different streams.  May allocate
 * workspace on first use or growth.
 * Long requests (the non-coherent sum of Sec. 3 over many blocks): when the
 * one-pass workspace does not fit (within the HBM budget beside what the
 * context holds elsewhere, or without one within nine tenths of the
 * device's free memory plus the context's workspace), or under option
 * "block_window", the request runs in passes of
 * a multiple of 256 blocks, enqueued one after another on the stream; each
 * pass wipes, folds and transforms only its own blocks at their places in
 * the record, adds its sums to the grid (out_grid, or an internal one) and
 * only the last detects.  In GNSS_FP32 the results equal a one-pass search
 * bit for bit; the FP16 precisions stay within their bounds.  A request that
 * does not fit even in 256-block passes gets GNSS_ENOMEM.
 * Errors: GNSS_EINVAL, GNSS_ENOTSUP, GNSS_ENOMEM, GNSS_EDEVICE. */
int gnss_acquire_device(gnss_ctx *ctx, const gnss_request *req, void *stream);

/* Allocation-free form of gnss_acquire_device, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, arithmetic,
 * kernels and results as gnss_acquire_device; the call allocates no device
 * or pinned memory and creates no HIP objects: the request's workspace (block
 * and spectrum buffers, column maxima, the internal grid when out_grid is
 * NULL, and the request metadata) is laid out in a static device array of
 * GNSS_NOALLOC_SCRATCH_BYTES bytes that every GPU running the library holds
 * until the process ends, and the metadata goes through
 * GNSS_NOALLOC_META_BYTES of pinned staging that gnss_ctx_create sets up.
 * A search of the strong-signal size (4.092 MHz, 10 ms, 32 PRNs x 21 bins,
 * internal grid) fits in every precision.  The caller owns samples,
 * out_grid and out_peaks (device memory), as for gnss_acquire_device.
 * Every such call on a GPU shares that GPU's array (all contexts on the
 * device), which keeps the last call's contents; calls that overlap on one
 * GPU, on any streams or contexts, race and give undefined results.  The
 * host waits for the previous call's metadata copy before staging the next.
 * A long request whose one pass does not fit the array runs in passes over
 * its blocks as in gnss_acquire_device, all in the array (laid out for the
 * first, longest pass).
 * Errors: as gnss_acquire_device; GNSS_ENOMEM (with the bytes needed in
 * gnss_last_error) when the workspace or metadata exceeds those sizes even
 * in 256-block passes. */
#define GNSS_NOALLOC_SCRATCH_BYTES 67108864
#define GNSS_NOALLOC_META_BYTES 1048576
int gnss_acquire_device_noalloc(gnss_ctx *ctx, const gnss_request *req, void *stream);

/* Batched acquisition on device buffers: n_req requests of any lengths,
 * sample rates, PRN lists and Doppler windows searched by one pass of the
 * stage kernels over a device table of the requests (the batch mode of the
 * paper's Listing 3(b), applied to whole requests).  Each request as for gnss_acquire_device.
 * Results are identical to running each request alone.  A batch whose
 * workspace does not fit (see gnss_acquire_device) runs its requests that
 * need passes over their blocks alone, in passes, and the others as one
 * batch, all on `stream`.  Errors: as gnss_acquire_device; a bad request
 * reports its index. */
int gnss_acquire_batch_device(gnss_ctx *ctx, const gnss_request *reqs, int32_t n_req, void *stream);

/* A batch captured once into a HIP graph (metadata copy and every stage
 * kernel) with its own workspace, replayed by gnss_graph_launch on any
 * stream; device buffers named by the requests must stay valid and keep
 * their sizes.  Replays of one graph must not overlap.  Errors: as
 * gnss_acquire_batch_device. */
typedef struct gnss_graph gnss_graph;
int gnss_graph_create(gnss_ctx *ctx, const gnss_request *reqs, int32_t n_req, gnss_graph **out);
int gnss_graph_launch(gnss_graph *graph, void *stream);
/* Waits for the graph's last launch (not for the rest of the device), then
 * frees the graph and its workspace; NULL is a no-op. */
void gnss_graph_destroy(gnss_graph *graph);

/* Picks the correlation kernel's launch for batches with the sample rates of
 * `reqs` (the batch mode of the paper's Listing 3(b) needs a launch shape the
 * paper's hardware fixed by hand): PRN tile, waves per workgroup (the shapes
 * the precision has, see "corr_ptile" and "corr_waves" of gnss_ctx_set) and
 * schedule (1: persistent with work counters, 0: one workgroup per item), by
 * timing every combination on the device (fastest of 3 runs; reqs are
 * device-buffer requests, their outputs are overwritten), or takes them from
 * the text cache file `cache_path` (nullable) keyed by device, precision and
 * rate signature; writes the cache and sets the context to use the choice
 * (options "corr_ptile", "corr_waves" and "persistent" override it); the
 * cache file holds "key tile schedule waves" lines.  The timed runs are
 * one-pass batches: a request that only fits in passes over its blocks gets
 * GNSS_ENOMEM here, and a shorter request at the same rates tunes it.
 * *chosen_tile and *chosen_persistent (nullable) get it. */
int gnss_autotune(gnss_ctx *ctx, const gnss_request *reqs, int32_t n_req, const char *cache_path,
                  int32_t *chosen_tile, int32_t *chosen_persistent);

/* ---- serving: continuous batching of submitted requests --------------- */
/* Outcome of a finished ticket: status (GNSS_OK or the request's error),
 * seconds queued (submission to start of its batch), running (batch start
 * to results delivered) and in total, and the size of its batch. */
typedef struct gnss_ticket_info {
    int32_t status;
    int32_t batch_size;
    double queued_s, run_s, total_s;
} gnss_ticket_info;

/* Submits a request with host buffers (the paper's cloud setting, Sec. 1:
 * clients upload recordings, results go back).  samples are copied before
 * the call returns; prn_list is copied; out_peaks (and out_grid if not
 * null) must stay valid until the ticket is reported done.  A context
 * thread batches queued requests as batch slots and the HBM budget allow
 * (two batches in flight, overlapping on the device).  A request whose
 * one pass exceeds a batch slot's share of the budget runs alone in passes
 * over its blocks (see gnss_acquire_device), each within the share.
 * Errors: argument errors as gnss_acquire; GNSS_ENOMEM if the request
 * exceeds a slot's share even in 256-block passes. */
int gnss_submit(gnss_ctx *ctx, const gnss_request *req, uint64_t *ticket);

/* Non-blocking completion check of a submitted request (the cloud client's
 * view of its upload, Sec. 1; queued and running times give the per-request
 * latency behind the paper's throughput measure, Sec. 4).  When *done is 1
 * the outputs are written, info (nullable) is filled, the ticket is released
 * and the return value is the request's status (a device error fails only
 * the tickets of the batch it occurred in).  Errors: GNSS_EINVAL (null
 * argument, unknown ticket). */
int gnss_poll(gnss_ctx *ctx, uint64_t ticket, int *done, gnss_ticket_info *info);

/* Blocks until a submitted request is done (Sec. 1's cloud service; timeout_s
 * < 0: no limit); then as gnss_poll with *done = 1.  Errors: GNSS_EINVAL
 * (null context, unknown ticket), GNSS_EBUSY on timeout (ticket kept), or the
 * request's own status. */
int gnss_wait(gnss_ctx *ctx, uint64_t ticket, double timeout_s, gnss_ticket_info *info);

/* ---- stage entry points (device pointers, enqueued on `stream`, a
 *      hipStream_t; NULL = the HIP null stream) ----------------------------- */

/* C/A code generator (code NCO source, Sec. 3 Fig. 2; IS-GPS-200 Table 3-Ia):
 * d_codes[i*1023 + n] = chip n (0/1) of prn_list[i].  prn_list is host memory.
 * Errors: GNSS_EINVAL. */
int gnss_gold_codes(gnss_ctx *ctx, const int32_t *prn_list, int32_t n_prn, uint8_t *d_codes,
                    void *stream);

/* Code replica (code NCO, Sec. 3 Fig. 2): d_out[i*n + m] =
 * 1 - 2*code_i[floor(m*1023000/fs) mod 1023] (int8), any integer fs in Hz. */
int gnss_code_replica(gnss_ctx *ctx, const int32_t *prn_list, int32_t n_prn, double fs,
                      size_t n, int8_t *d_out, void *stream);

/* Carrier LUT (carrier NCO, Sec. 3 Fig. 2): d_cos[i], d_sin[i] =
 * lround(4096 cos/sin(2 pi i/1024)), i < 1024 (int16). */
int gnss_nco_lut(gnss_ctx *ctx, int16_t *d_cos, int16_t *d_sin, void *stream);

/* First mixing stage + coherent folding (Sec. 3 Fig. 2; block processing,
 * Sec. 4): d_out[((k*N_noncoh + b)*N + m)*2 + {0,1}] = re/im of
 * sum_{t<T} y_k[(b*T + t)*N + m], exact int32.  Other fields of req as for
 * gnss_acquire_device (outputs ignored).  A standalone kernel; the search
 * itself runs the stage of gnss_box_fold at k * 1.023 MHz and the same
 * arithmetic inside its general-rate block transform at other rates.  Calls
 * on one context must not overlap.  Errors: GNSS_EINVAL, GNSS_ENOTSUP (N >
 * 16384), GNSS_ENOMEM, GNSS_EDEVICE. */
int gnss_wipe_fold(gnss_ctx *ctx, const gnss_request *req, int32_t *d_out, void *stream);

/* The search's own first stage, run alone with the kernel and launch the
 * search uses: carrier NCO and first mixing stage (Sec. 3 Fig. 2), coherent
 * fold of each block (block processing, Sec. 4), then the one-chip boxcar and
 * polyphase split that turn the length-N correlation into spc length-1023
 * ones.  With f_kb the folded block of gnss_wipe_fold, delayed circularly by
 * the code-Doppler shift d_kb when the context's "code_doppler" option is 1
 * (else d_kb = 0), F[n] = sum_{t<spc} f_kb[(n + t - d_kb) mod N] and
 *   d_out[(((k*N_noncoh + b)*spc + s)*1024 + m)*2 + {0,1}] = re/im of F[spc*m + s]
 * for m < 1023, and 0 at m = 1023; exact int32.  d_out is device memory of
 * n_dopp*N_noncoh*spc*1024*2 int32 owned by the caller; other fields of req as
 * for gnss_acquire_device (outputs ignored; "doppler_fd" does not apply).
 * Calls on one context must not overlap.  Errors: as gnss_wipe_fold, and
 * GNSS_ENOTSUP when fs is not k * 1.023 MHz with k <= 16 (no polyphase form). */
int gnss_box_fold(gnss_ctx *ctx, const gnss_request *req, int32_t *d_out, void *stream);

/* Batched 2048-point complex FFT (the FFT/IFFT stages of Fig. 2), natural
 * order in and out, interleaved float re/im, forward exp(-2 pi i nk/2048) or
 * (inverse != 0) unnormalised exp(+2 pi i nk/2048).  d_in and d_out hold
 * batch*2048 complex values and may not overlap. */
int gnss_fft2048(gnss_ctx *ctx, const float *d_in, float *d_out, int32_t batch,
                 int32_t inverse, void *stream);

/* Batched exact-length 1023-point DFT in the GNSS_FP16_PFA arithmetic (the
 * Good-Thomas 31 x 33 transform of that mode: per-vector power-of-two scaling
 * from the l1 norm, FP16 operands, FP32 accumulation), natural order in and
 * out, interleaved float re/im, forward exp(-2 pi i nk/1023) or (inverse != 0)
 * unnormalised exp(+2 pi i nk/1023).  d_in and d_out (device memory, owned by
 * the caller) hold batch*1023 complex values, batch <= 2^28, and may not
 * overlap.  Errors: GNSS_EINVAL (arguments), GNSS_ENOTSUP (context not
 * created with GNSS_FP16_PFA), GNSS_EDEVICE. */
int gnss_dft1023(gnss_ctx *ctx, const float *d_in, float *d_out, int32_t batch,
                 int32_t inverse, void *stream);

/* Detection and refinement on a device grid [n_prn][n_dopp][N] (rule in the
 * header comment): fills d_peaks[n_prn] (device memory).  spc > 0 gives the
 * +-1 chip exclusion.  prn_list is host memory and only labels the results. */
int gnss_peaks(gnss_ctx *ctx, const float *d_grid, const int32_t *prn_list, int32_t n_prn,
               int32_t n_dopp, int32_t N, int32_t spc, double doppler_lo, double doppler_step,
               gnss_peak *d_peaks, void *stream);

/* ---- tracking correlators ----------------------------------------------- */
/* One tracking channel (the tracking channel of Fig. 3: carrier and code
 * NCOs, first mixing stage, time-domain correlation with the code replica;
 * Sec. 3 names that correlation as the tracking loops' main cost).  The
 * paper gives no further detail; the correlators are the usual early /
 * prompt / late set.  Values are physical; the library turns each into a
 * fixed-point word (value * 2^32 rounded half away from zero, in IEEE double
 * as written; the carrier step is carrier_hz * 2^32 / fs), so results are
 * exact integers:
 *   carrier phase(n) = (uint32)(phi0 + n * D), y[n] = x[n] * (cosL - j sinL)[phase >> 22]
 *   (the LUT of gnss_nco_lut); code phase q(n) = q0 + n * R (chips * 2^32);
 *   chip_X(n) = floor((q(n) + off_X) / 2^32) mod 1023 with off = +dl (early),
 *   0 (prompt), -dl (late); X_e = sum over epoch e of y[n] (1 - 2 code[chip_X(n)]). */
typedef struct gnss_channel {
    int32_t prn;           /* 1..37                                              */
    double carrier_hz;     /* carrier to remove (IF + Doppler), Hz               */
    double carrier_phase;  /* cycles at the record's first sample, [0, 1)        */
    double code_phase;     /* chips at the record's first sample, [0, 1023)      */
    double code_rate;      /* chips per second, (0, 1023 fs / 256]               */
    double spacing;        /* early / late offset from prompt, chips, (0, 1]     */
} gnss_channel;

/* A batch entry: one record, its channels and the epochs to correlate.
 * Epoch e covers samples [start + e epoch_len, start + (e + 1) epoch_len). */
typedef struct gnss_track_request {
    const void *samples;          /* record (host for gnss_track, device for _device) */
    int32_t fmt;                  /* sample format, as for gnss_request               */
    size_t n;                     /* samples in the record                            */
    double fs;                    /* sample rate, Hz                                  */
    const gnss_channel *channels; /* host memory, n_channels entries (1..256)        */
    int32_t n_channels;
    int64_t start;                /* first sample of epoch 0                          */
    int32_t epoch_len;            /* samples per epoch, 1..2^24                       */
    int32_t n_epochs;             /* >= 1; start + n_epochs epoch_len <= n            */
    int64_t *out;                 /* [n_channels][n_epochs][3][2] int64: early,
                                     prompt, late, each (re, im)                      */
} gnss_track_request;

/* Synchronous tracking correlators on host buffers (default context, locked;
 * thread-safe).  Errors: GNSS_EINVAL (a bad field, or a code phase that would
 * pass 2^30 chips over the record), GNSS_ENOMEM, GNSS_EDEVICE. */
int gnss_track(const gnss_track_request *req);

/* Tracking correlators of n_req requests (device samples and outputs) in one
 * launch, one workgroup per (request, epoch), enqueued on `stream` (NULL =
 * the HIP null stream); returns without waiting.  Calls on one context must
 * not overlap on different streams.  Errors: as gnss_track; a bad request
 * reports its index. */
int gnss_track_device(gnss_ctx *ctx, const gnss_track_request *reqs, int32_t n_req, void *stream);

/* ---- per-stage device timing -------------------------------------------- */
#define GNSS_STAGE_WIPE_FOLD 0  /* carrier NCO, mixing, fold, boxcar, polyphase */
#define GNSS_STAGE_FFT 1        /* forward FFT of the mixed blocks              */
#define GNSS_STAGE_CORR 2       /* spectrum product, IFFT, |.|^2, block sum     */
#define GNSS_STAGE_DETECT 3     /* column max, peaks, refinement                */
#define GNSS_N_STAGES 4

/* Where the time goes, stage by stage (the paper's per-stage accounting of
 * its receiver, Secs. 3-4: mixing, FFT stages, correlation, detection).
 * While the context's "profile" option is 1, every search records HIP events
 * on its stream around each stage.  This call waits for the recorded events
 * and adds their elapsed milliseconds to ms_total[i] and the number of timed
 * launches to launches[i] (host arrays of n >= GNSS_N_STAGES entries, set to
 * the totals since the last reset); reset != 0 clears the totals.
 * Errors: GNSS_EINVAL, GNSS_EDEVICE. */
int gnss_stage_times(gnss_ctx *ctx, double *ms_total, int64_t *launches, int32_t n, int32_t reset);

/* ---- errors ------------------------------------------------------------ */
/* Text of a GNSS_E* code (static storage), and the calling thread's detail
 * message of its last failed call (valid until that thread's next call).
 * Plumbing of this library: the paper defines no error reporting. */
const char *gnss_strerror(int code);
const char *gnss_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GNSS_ACQ_H */

// gnss_internal.hpp -- launch wrappers shared by the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gnss_acq.h"

namespace gnss {

constexpr int kMaxPrn = 37;            // PRNs 1..37 (IS-GPS-200 Table 3-Ia)
constexpr int kCodeLen = 1023;
constexpr int kMaxList = 64;           // PRNs per request (duplicates allowed)
constexpr int kMaxSpc = 16;            // samples per chip: fs <= 16.368 MHz
constexpr int kMaxN = kCodeLen * kMaxSpc;
constexpr int kVec = 1024;             // float4 per storage-order spectrum (2048 complex)
constexpr int kPolyLen = 1024;         // int2 per polyphase component (1023 + 1 zero)
constexpr int kCorrWaves = 8;          // waves per FP32 correlation workgroup (PRN tiles 2, 4)
constexpr int kCorrWaves1 = 4;         // ... PRN tile 1 (three 4-wave workgroups per CU: three waves per SIMD)
constexpr int kCorrWavesH = 4;         // waves per FP16 correlation workgroup
constexpr int kCorrWavesX = 4;         // waves per exact-length correlation workgroup
// FP32 non-coherent sums are cascaded: each group of kSumGroup blocks is
// summed in registers, then added to the sum so far kept in the grid.  A
// sequential FP32 sum of Nnc positive terms has relative error up to
// (Nnc - 1) 2^-24, and a biased one in practice once the sum dwarfs the
// terms (terms below half its ulp are dropped); in groups the bound is
// (kSumGroup + Nnc / kSumGroup) 2^-24, and requests of at most kSumGroup
// blocks take one group, exactly as a plain sum.
constexpr int kSumGroup = 256;

struct PrnList {
    int32_t v[kMaxList];
};

// Derived sizes of one acquisition request.
struct Plan {
    int fmt;
    int64_t n_samples;
    int64_t fs_hz;
    double f_if, lo, step;
    int N;          // samples per ms
    int spc;        // samples per chip (whole part of fs / 1.023 MHz for a general rate)
    int n_dopp;
    int Tc, Nnc;
    int n_prn;
    PrnList prns;   // PRN numbers (1..37)
    // general rate (fs not k * 1.023 MHz with 1 <= k <= kMaxSpc): the
    // length-N correlations run on zero-padded transforms of length gen_M
    int gen;
    int gen_M;      // power of two >= 2N
    // a pass over part of the blocks (see ReqDesc): the first block, whether
    // the grid already holds earlier passes' sums, whether detection runs
    int b0 = 0, acc = 0, detect = 1;
    int64_t grid_elems() const { return (int64_t)n_prn * n_dopp * N; }
    int64_t n_vec() const { return gen ? 0 : (int64_t)n_dopp * Nnc * spc; }
};

// General rates: N <= kGenMaxN samples per ms, transforms of length
// M = 2^ceil(log2(2N)) <= 2 kGenLds (M = N when N is a power of two) done as
// one (M <= kGenLds) or two (M = 2 kGenLds, even and odd bins) transforms of
// at most kGenLds points in a workgroup's LDS.
constexpr int kGenMaxN = 16384;
constexpr int kGenLds = 16384;
constexpr int kGenTwLen = 2 * kGenLds;  // twiddle table W_32768^j, j < 32768
constexpr int kGenThreads = 1024;
inline int gen_transform_len(int N)
{
    // N a power of two (>= 64): the length-N circular correlation is the
    // N-point one, no padding needed
    if (N >= 64 && (N & (N - 1)) == 0) return N;
    int M = 64;
    while (M < 2 * N) M *= 2;
    return M;
}

// one-time tables
hipError_t launch_gold_codes(uint8_t *d_codes /*[38][1023], row = prn*/, hipStream_t s);
hipError_t launch_code_replica(const uint8_t *d_codes, PrnList prns, int n_prn, int64_t fs_hz,
                               int64_t n, int8_t *d_out, hipStream_t s);
hipError_t launch_lut(uint32_t *d_lut_packed, int16_t *d_cos, int16_t *d_sin, hipStream_t s);
hipError_t launch_twiddles(float2 *d_tw, hipStream_t s);
hipError_t launch_code_spectra(const uint8_t *d_codes, const float2 *d_tw, float4 *d_cs,
                               hipStream_t s);
// FP16 tables: packed twiddles and the code spectra scaled by 2^-cs_exp
hipError_t launch_tables_h(const float4 *d_cs, const uint8_t *d_codes, void *d_tw_h, void *d_cs_h, int cs_exp,
                           hipStream_t s);
constexpr size_t kTwHBytes = 2176 * 8;                      // hc2 twiddles
constexpr size_t kCsHSpecBytes = (size_t)(kMaxPrn + 1) * 8192;  // [38][2048] half2
// followed by one float per PRN: 2048 * 2^-cs_exp * sum(code) / 1023, the
// inverse output's lag-independent part per unit of a block's scaled sum
constexpr size_t kCsHBytes = kCsHSpecBytes + 256;
// Exact-length mode tables: FP16 weight fragments of the 31- and 33-point
// passes, and the code spectra (FP64 staging, then FP16 fragments)
constexpr size_t kPfaVecBytes = 264 * 16;  // one stored 1023-point spectrum
constexpr size_t kFragXBytes = 49 * 64 * 16;
constexpr size_t kCsXBytes = (size_t)(kMaxPrn + 1) * kPfaVecBytes;
constexpr size_t kCsXStageBytes = (size_t)(kMaxPrn + 1) * 31 * 33 * 16;
hipError_t launch_tables_x_frags(void *d_frags, hipStream_t s);
hipError_t launch_code_spectra_x(const uint8_t *d_codes, double2 *d_stage, hipStream_t s);
hipError_t launch_code_spectra_x_pack(const double2 *d_stage, void *d_cs_x, int cs_exp, hipStream_t s);

// Bytes of the block spectra of n_vec polyphase vectors: FP32 float4
// storage order; FP16 packed half2 (re, im), followed by one int exponent per
// vector.
inline size_t g_spectra_bytes(long long n_vec, int precision)
{
    return precision == GNSS_FP16 ? (size_t)n_vec * 8192
           : precision == GNSS_FP16_PFA ? (size_t)n_vec * kPfaVecBytes
                                        : (size_t)n_vec * kVec * 16;
}
inline size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
// FP16 modes: the spectra, the per-vector exponents (int) and, for GNSS_FP16,
// the per-vector scaled sums (float2)
inline size_t g_bytes(long long n_vec, int precision)
{
    return precision == GNSS_FP32 ? g_spectra_bytes(n_vec, precision)
           : precision == GNSS_FP16_PFA
               ? g_spectra_bytes(n_vec, precision) + round256((size_t)n_vec * 4)
               : g_spectra_bytes(n_vec, precision) + round256((size_t)n_vec * 4) + round256((size_t)n_vec * 8);
}

// ---------------------------------------------------------------------------
// batched hot path: every stage kernel walks a device-resident table of
// requests (a single request is a batch of one); the correlation kernel can
// run persistent, the others run one workgroup per work item
// ---------------------------------------------------------------------------
// kStGenX / kStGenC / kStGenCorr: the general-rate path (block spectra,
// code spectra, correlation)
enum Stage { kStBox = 0, kStVec, kStCorr, kStColmax, kStPeak, kStFdA, kStFdB, kStGenX, kStGenC, kStGenCorr,
             kNumStages };
constexpr int kXcds = 8;

// One request as the kernels see it (device memory).
struct ReqDesc {
    const void *samples;
    float *grid;          // [n_prn][n_dopp][N]
    gnss_peak *peaks;     // [n_prn]
    // Carrier NCO steps D_k, one per Doppler bin, and (option code_doppler)
    // the code-Doppler lag shift of every (bin, block), [n_dopp][Nnc] in
    // [0, N): both computed on the host in IEEE double as written, so the
    // kernels do no FP64 arithmetic for them
    const uint32_t *dk;
    const int32_t *cshift;  // null without code_doppler
    long long vec_off;    // first polyphase vector of the request in F and G
    long long qk_off;     // offset of the request in Q and K (n_prn * N)
    long long part_off;   // offset in the partial sums (n_prn * n_tau_blk)
    double lo, step;      // Doppler grid, for the FP64 refinement only
    int fmt, N, spc, n_dopp, Tc, Nnc, n_prn;
    int n_items;          // (Doppler, phase) items = n_dopp * spc
    int n_ptiles;         // PRN tiles of the correlation kernel
    int n_tau_blk;        // 256-lag blocks of the detection kernels
    float threshold;
    int nav_pairs;        // 1: blocks combined in pairs, max over the relative sign (navigation bit)
    // frequency-domain Doppler (exact-length contexts, option doppler_fd):
    // one zero-padded DFT of length fd_A * 1023 per block serves every bin
    int fd;               // 1: this request uses it
    int fd_PTc;           // P * Tc: bins of the long DFT per 1 kHz
    int fd_A;             // P * Tc * spc, a power of two
    int fd_kappa;         // long-DFT bins per Doppler step
    long long fd_off;     // first float2 of the request's long spectra (first pass, then final)
    long long fd_crt1;    // 1023 (1023^-1 mod A): long index = (k1 crt1 + k2 crt2) mod M
    long long fd_crt2;    // A (A^-1 mod 1023)
    // carrier f_if + lo removed before the long DFT: a 64-bit phase
    // accumulator, cycles * 2^64 per sample (phase of in-block sample n =
    // n * fd_dphase mod 2^64)
    unsigned long long fd_dphase;
    // general rate: transform length M, its LDS part (M or M/2) and the
    // request's block spectra [n_dopp][Nnc][M] and code spectra [n_prn][M]
    // (float2 offsets in the general-rate region of the spectrum buffer)
    int gen, gen_M, gen_P;
    long long gen_x_off, gen_c_off;
    // A long request may run in passes over its blocks: this pass's blocks
    // are the record's blocks b0 .. b0 + Nnc - 1 (sample positions and
    // carrier phases are the record's; F, G and the shift table hold the
    // pass's blocks only), and with acc the correlation adds its sums to the
    // grid's, those of the earlier passes
    int b0, acc;
    int prns[kMaxList];
};

// Batch header (device memory): request count, work totals per stage and the
// dynamic work counters (zeroed by k_reset at the start of every batch).
struct BatchHdr {
    int n_req;
    int corr_pt;
    long long total[kNumStages];
    unsigned int counter[kNumStages * kXcds];
};

struct Launch {
    const ReqDesc *reqs;
    BatchHdr *hdr;
    const long long *pre;  // [kNumStages][n_req + 1] work-item prefix sums
    int n_req;
    long long total[kNumStages];  // host copy (grid sizing)
    int corr_pt;                  // PRN tile of the correlation kernel
    int corr_w;                   // its waves per workgroup
    int persistent;               // correlation kernel: 1 occupancy-sized grid with work counters, 0 a workgroup per item
    int precision;                // GNSS_FP32 / GNSS_FP16 / GNSS_FP16_PFA
    int fd;                       // 1: frequency-domain Doppler (exact-length contexts)
    int nav_pairs;                // 1: navigation-bit hypotheses (exact-length contexts)
    size_t gen_off;               // bytes of the spectrum buffer before its general-rate region
    unsigned gen_pmask;           // general-rate transform lengths P present (bit P)
};

// Device-resident tables of a context.
struct Tables {
    const uint32_t *lut;
    const float2 *tw;
    const float4 *cs;
    const void *tw_h;  // FP16 path only
    const void *cs_h;
    const void *frags_x;  // exact-length path only
    const void *cs_x;
    int cs_exp;
    const float2 *tw_gen;  // general rates: W_32768^j, j < 32768
    const uint8_t *codes;  // C/A chips [38][1023] (row = PRN)
};

hipError_t launch_batch(const Launch &L, const Tables &T, int2 *d_F, void *d_G, float *d_Q, int32_t *d_K,
                        float *d_part, int n_cu, hipStream_t s, hipEvent_t *marks);
int corr_ptile_valid(int pt, int precision);
// Launch shape of the correlation kernel: PRNs per workgroup (pt) and waves
// per workgroup (w, one (Doppler, phase) item per wave).
struct CorrShape {
    int pt, w;
};
// the waves per workgroup a PRN tile runs with unless tuned
inline int corr_waves(int precision, int pt)
{
    return precision == GNSS_FP16 ? kCorrWavesH
           : precision == GNSS_FP16_PFA ? kCorrWavesX
           : pt == 1 ? kCorrWaves1
                     : kCorrWaves;
}
// instantiated shapes: FP32 tile 1 with 12, 6 or 4 waves (three waves per
// SIMD), tiles 2 and 4 with 8; the FP16 kernels have one width each
bool corr_shape_valid(CorrShape c, int precision);
constexpr int kBoxChunk = 2048;
constexpr int kPeakThreads = 256;   // threads of the column-max kernel (256-lag blocks)
constexpr int kArgThreads = 1024;   // threads of the per-PRN argmax kernel

// standalone wipe + fold (stage entry point): request 0 of the staged batch
hipError_t launch_wipe_fold(const Launch &L, const Plan &p, const uint32_t *d_lut,
                            int32_t *d_out /*[n_dopp][Nnc][N][2]*/, hipStream_t s);
// the search's wipe + fold + boxcar + polyphase stage alone (stage entry point)
hipError_t launch_box(const Launch &L, const uint32_t *d_lut, int2 *d_F, int n_cu, hipStream_t s);
// detection on a caller's grid (stage entry point)
size_t peak_scratch_part_elems(const Plan &p);

// ---------------------------------------------------------------------------
// tracking correlators (early / prompt / late)
// ---------------------------------------------------------------------------
// Fixed-point NCO words of one channel.
struct TrackCh {
    uint32_t D, phi0;     // carrier step and initial phase, cycles * 2^32
    long long q0, R, dl;  // code phase at sample 0, code step, early-late offset, chips * 2^32
    int prn, pad;
};
// One tracking request as the kernel sees it.
struct TrackDesc {
    const void *samples;
    long long *out;       // [n_ch][n_epochs][3][2]
    long long start;      // first sample of epoch 0
    int fmt, epoch_len, n_epochs, n_ch, ch_off;
};
constexpr int kFdCols = 8;  // columns of the long DFT's second pass per workgroup
constexpr int kTrackThreads = 256;
constexpr int kTrackCG = 4;  // channels per pass over an epoch
hipError_t launch_track(const TrackDesc *d_reqs, const long long *d_pre, int n_req, long long total,
                        const TrackCh *d_ch, const uint8_t *d_codes, const uint32_t *d_lut, hipStream_t s);

// test entry: natural-order batched 2048-point transforms
hipError_t launch_fft_test(const float2 *d_in, float2 *d_out, int batch, int inverse,
                           const float2 *d_tw, hipStream_t s);
// test entry: natural-order batched 1023-point transforms (exact-length mode)
hipError_t launch_dft1023_test(const float2 *d_in, float2 *d_out, int batch, int inverse, const void *d_frags,
                               hipStream_t s);

}  // namespace gnss

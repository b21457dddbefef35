// gnss_kernels.hip -- HIP kernels (gfx950) of the GPS L1 C/A acquisition search.
//
// The acquisition channel of the paper (Sec. 3, Fig. 2): code and carrier
// NCOs, first mixing stage, FFTs of mixed signal and code replica, second
// mixing (spectrum product), IFFT, detection; block processing (Sec. 4) and
// batching of the whole coherent integration on the device (Sec. 5).
//
// Correlation in polyphase form.  With spc = fs/1.023 MHz integer samples per
// chip the code replica is c[n] = C[floor(n/spc)] (C the +-1 chip code), so
// for the folded block f (length N = 1023 spc) the circular correlation
//   R[tau] = sum_n f[n] c[(n - tau) mod N]
// at tau = spc q + s equals the length-1023 circular correlation
//   R[spc q + s] = sum_m g_s[m] C[(m - q) mod 1023],
//   g_s[m] = F[spc m + s],  F[n] = sum_{t<spc} f[(n + t) mod N]
// (a boxcar over one chip, then a polyphase split).  Each g_s is correlated
// with the chip-rate code through 2048-point transforms (zero padding makes
// the circular length-1023 correlation a linear one), so one code spectrum
// per PRN serves every sample rate, and each transform lives in one
// wavefront's registers.
//
// Kernel sequence of a batch (every kernel walks a device table of the batch's
// requests; a single request is a batch of one):
//   k_reset          clears the work counters (a kernel, so the sequence can be
//                    captured in a graph)
//   k_box            NCO wipe-off + coherent fold + boxcar + polyphase split
//                    (exact int32)                     -> F[k][b][s][1024]
//   k_fft_poly       forward 2048-point FFT of every g_s -> G (storage order)
//   k_corr           per (PRN tile, Doppler, phase): G * conj(code spectrum),
//                    IFFT, |.|^2, sum over blocks in registers -> grid
//   k_colmax/k_peak  column max over Doppler, argmax, second peak, mean
//   k_interp         FP64 parabolic refinement
// FP16 contexts use k_fft_poly_h and k_corr_h (packed half precision with
// per-vector power-of-two scaling).  k_track computes the tracking channel's
// early / prompt / late correlators (Fig. 3).
#include "fft2048.hpp"
#include "gnss_internal.hpp"
#include "pfa1023.hpp"

#include <math.h>

namespace gnss {

// Device pointers of a request live in the request table, so the compiler
// cannot tell that they address global memory; these casts let it use global
// (not flat) loads and stores for them.
#define GNSS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GNSS_GLOBAL T *gmem(T *p)
{
    return (GNSS_GLOBAL T *)p;
}

// A workgroup-uniform 64-bit value in scalar registers.
__device__ __forceinline__ long long uniform64(long long v)
{
    const unsigned long long u = (unsigned long long)v;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}


// ===========================================================================
// C/A codes (IS-GPS-200 Table 3-Ia), G2-delay construction
// ===========================================================================
// G2 delay in chips for PRN 1..37: chip_n = G1_n xor G2_(n - delay).
__constant__ int16_t c_g2_delay[kMaxPrn] = {
    5,   6,   7,   8,   17,  18,  139, 140, 141, 251, 252, 254, 255, 256, 257, 258, 469, 470, 471,
    472, 473, 474, 509, 512, 513, 514, 515, 516, 859, 860, 861, 862, 863, 950, 947, 948, 950};

// 10-stage registers, stage i in bit i-1, output is stage 10 (bit 9).
__device__ __forceinline__ uint32_t g1_next(uint32_t r)
{
    uint32_t fb = ((r >> 2) ^ (r >> 9)) & 1u;  // stages 3, 10
    return ((r << 1) | fb) & 0x3FFu;
}
__device__ __forceinline__ uint32_t g2_next(uint32_t r)
{
    uint32_t fb = ((r >> 1) ^ (r >> 2) ^ (r >> 5) ^ (r >> 7) ^ (r >> 8) ^ (r >> 9)) & 1u;  // 2,3,6,8,9,10
    return ((r << 1) | fb) & 0x3FFu;
}

// One thread per PRN row (row 0 is all zeros).  codes is [38][1023].
__global__ void k_gold_codes(uint8_t *codes)
{
    int prn = threadIdx.x;
    if (prn > kMaxPrn) return;
    uint8_t *row = codes + prn * kCodeLen;
    if (prn == 0) {
        for (int n = 0; n < kCodeLen; ++n) row[n] = 0;
        return;
    }
    const int delay = c_g2_delay[prn - 1];
    uint32_t g1 = 0x3FFu, g2 = 0x3FFu;
    // bring G2 to sequence index (-delay mod 1023)
    for (int i = 0; i < (kCodeLen - delay) % kCodeLen; ++i) g2 = g2_next(g2);
    for (int n = 0; n < kCodeLen; ++n) {
        row[n] = (uint8_t)(((g1 ^ g2) >> 9) & 1u);
        g1 = g1_next(g1);
        g2 = g2_next(g2);
    }
}

hipError_t launch_gold_codes(uint8_t *d_codes, hipStream_t s)
{
    hipLaunchKernelGGL(k_gold_codes, dim3(1), dim3(64), 0, s, d_codes);
    return hipGetLastError();
}

// Code replica at sample rate fs: out[i*n + m] = 1 - 2 code[floor(m*1023000/fs) mod 1023].
__global__ void k_code_replica(const uint8_t *codes, PrnList prns, int n_prn, long long fs_hz,
                               long long n, int8_t *out)
{
    const long long total = (long long)n_prn * n;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        long long i = idx / n, m = idx - i * n;
        long long chip = (m * 1023000LL) / fs_hz;
        int bit = codes[prns.v[i] * kCodeLen + (int)(chip % kCodeLen)];
        out[idx] = (int8_t)(1 - 2 * bit);
    }
}

hipError_t launch_code_replica(const uint8_t *d_codes, PrnList prns, int n_prn, int64_t fs_hz,
                               int64_t n, int8_t *d_out, hipStream_t s)
{
    long long total = (long long)n_prn * n;
    long long blocks = (total + 255) / 256;
    if (blocks > 65535) blocks = 65535;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_code_replica, dim3((unsigned)blocks), dim3(256), 0, s, d_codes, prns,
                       n_prn, (long long)fs_hz, (long long)n, d_out);
    return hipGetLastError();
}

// ===========================================================================
// carrier LUT and FFT twiddles
// ===========================================================================
// packed[i] = (uint16)cos16 | (uint16)sin16 << 16, values lround(4096 cos/sin(2 pi i/1024)).
__global__ void k_lut(uint32_t *packed, int16_t *cosL, int16_t *sinL)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 1024) return;
    double s, c;
    sincospi((double)i / 512.0, &s, &c);
    int ci = (int)llround(4096.0 * c);
    int si = (int)llround(4096.0 * s);
    if (packed) packed[i] = (uint32_t)(uint16_t)(int16_t)ci | ((uint32_t)(uint16_t)(int16_t)si << 16);
    if (cosL) cosL[i] = (int16_t)ci;
    if (sinL) sinL[i] = (int16_t)si;
}

hipError_t launch_lut(uint32_t *d_lut_packed, int16_t *d_cos, int16_t *d_sin, hipStream_t s)
{
    hipLaunchKernelGGL(k_lut, dim3(4), dim3(256), 0, s, d_lut_packed, d_cos, d_sin);
    return hipGetLastError();
}

__global__ void k_twiddles(float2 *tw)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s, c;
    if (i < kT1Elems) {
        int hk = i >> 6, l = i & 63;
        int h = hk >> 4, k1 = hk & 15;
        int e = ((l + 64 * h) * k1) & 2047;  // angle 2 pi e / 2048
        sincospi((double)e / 1024.0, &s, &c);
        tw[i] = make_float2((float)c, (float)s);
    } else if (i < kTwElems) {
        int j = i - kT1Elems;
        int k2a = j >> 3, m2 = j & 7;
        int e = (m2 * k2a) & 127;  // angle 2 pi e / 128
        sincospi((double)e / 64.0, &s, &c);
        tw[i] = make_float2((float)c, (float)s);
    }
}

hipError_t launch_twiddles(float2 *d_tw, hipStream_t s)
{
    hipLaunchKernelGGL(k_twiddles, dim3((kTwElems + 255) / 256), dim3(256), 0, s, d_tw);
    return hipGetLastError();
}

__device__ __forceinline__ void stage_twiddles(float2 *s_tw, const float2 *tw, int tid, int nthreads)
{
    for (int i = tid; i < kTwElems; i += nthreads) s_tw[i] = tw[i];
}

// ===========================================================================
// code spectra: CS[prn] = conj(FFT_2048(cc_prn)) in storage order, where
// cc[i] = C[i] (i < 1023), 0 (1023..1025), C[i - 1025] (1026..2047), so that
// IFFT_2048(FFT(g0) * CS)[q] = 2048 * sum_m g[m] C[(m - q) mod 1023] for q < 1023.
// ===========================================================================
__global__ __launch_bounds__(256) void k_code_spectra(const uint8_t *codes, const float2 *tw,
                                                      float4 *cs)
{
    __shared__ float2 s_tw[kTwElems];
    __shared__ float2 s_xb[4][kXbufElems];
    stage_twiddles(s_tw, tw, threadIdx.x, 256);
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int prn = blockIdx.x * 4 + w;
    if (prn > kMaxPrn) return;
    const uint8_t *code = codes + prn * kCodeLen;
    float2 v[32];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k2b = 0; k2b < 8; ++k2b) {
            int q = l + 64 * u + 256 * k2b;
            float val = 0.f;
            if (prn != 0) {
                if (q < kCodeLen)
                    val = 1.f - 2.f * (float)code[q];
                else if (q >= 1026)
                    val = 1.f - 2.f * (float)code[q - 1025];
            }
            v[8 * u + k2b] = make_float2(val, 0.f);
        }
    fft2048<false>(v, s_xb[w], s_tw, s_tw + kT1Elems, l);
    float4 *dst = cs + (long long)prn * kVec;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj)
        dst[jj * 64 + l] = make_float4(v[2 * jj].x, -v[2 * jj].y, v[2 * jj + 1].x, -v[2 * jj + 1].y);
}

hipError_t launch_code_spectra(const uint8_t *d_codes, const float2 *d_tw, float4 *d_cs,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_code_spectra, dim3((kMaxPrn + 1 + 3) / 4), dim3(256), 0, s, d_codes,
                       d_tw, d_cs);
    return hipGetLastError();
}

__device__ __forceinline__ void load_sample(const void *samples, int fmt, long long n, int &xr, int &xi)
{
    if (fmt == GNSS_CPLX_I8) {
        const uint32_t v = ((const GNSS_GLOBAL uint16_t *)samples)[n];  // I in the low byte
        xr = (int)(int8_t)(v & 0xFFu);
        xi = (int)(int8_t)(v >> 8);
    } else if (fmt == GNSS_REAL_I8) {
        xr = ((const GNSS_GLOBAL int8_t *)samples)[n];
        xi = 0;
    } else {
        uint32_t byte = ((const GNSS_GLOBAL uint8_t *)samples)[n >> 2];
        uint32_t code = (byte >> (2 * (uint32_t)(n & 3))) & 3u;
        // 00:+1 01:+3 10:-1 11:-3
        int mag = (code & 1u) ? 3 : 1;
        xr = (code & 2u) ? -mag : mag;
        xi = 0;
    }
}

// y[n] = x[n] * (cosL - j sinL)[phase(n) >> 22], summed over the Tc
// milliseconds of coherent block b at in-block offset m.
__device__ __forceinline__ int2 wipe_fold_one(const void *samples, int fmt, int N, int Tc,
                                              const uint32_t *lut, uint32_t D, int b, int m)
{
    int yr = 0, yi = 0;
    for (int c = 0; c < Tc; ++c) {
        long long ng = (long long)(b * Tc + c) * N + m;
        int xr, xi;
        load_sample(samples, fmt, ng, xr, xi);
        uint32_t ph = (uint32_t)(unsigned long long)ng * D;
        uint32_t e = lut[ph >> 22];
        int cs = (int)(int16_t)(e & 0xFFFFu), sn = (int)(int16_t)(e >> 16);
        yr += xr * cs + xi * sn;
        yi += xi * cs - xr * sn;
    }
    return make_int2(yr, yi);
}

// Standalone wipe + fold (stage entry) of request 0 of a staged batch:
// out[((k*Nnc + b)*N + m)*2 + {0,1}].
__global__ __launch_bounds__(256) void k_wipe_fold(const ReqDesc *__restrict__ R, const uint32_t *lut, int2 *out)
{
    __shared__ uint32_t s_lut[1024];
    for (int i = threadIdx.x; i < 1024; i += 256) s_lut[i] = lut[i];
    const ReqDesc &d = R[0];
    const int k = blockIdx.x / d.Nnc, b = blockIdx.x % d.Nnc;
    const uint32_t D = d.dk[k];
    __syncthreads();
    int2 *dst = out + (long long)blockIdx.x * d.N;
    for (int m = threadIdx.x; m < d.N; m += 256)
        dst[m] = wipe_fold_one(d.samples, d.fmt, d.N, d.Tc, s_lut, D, d.b0 + b, m);
}

hipError_t launch_wipe_fold(const Launch &L, const Plan &p, const uint32_t *d_lut, int32_t *d_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_wipe_fold, dim3(p.n_dopp * p.Nnc), dim3(256), 0, s, L.reqs, d_lut, (int2 *)d_out);
    return hipGetLastError();
}

// ===========================================================================
// batch plumbing
// ===========================================================================
// Request owning work item `it` of a stage: the last r with pre[r] <= it.
__device__ __forceinline__ int find_req(const long long *pre, int n_req, long long it)
{
    int lo = 0, hi = n_req - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_reset(BatchHdr *h)
{
    int i = threadIdx.x;
    if (i < kNumStages * kXcds) h->counter[i] = 0u;
}

// Work distribution.  A stage launched with at least one workgroup per item
// runs one item per workgroup; the ids are dealt so that each XCD (workgroups
// go to the 8 XCDs round-robin) takes a contiguous range of items, which share
// data through that XCD's L2.  A persistent launch (fewer workgroups than
// items) instead splits the items into 8 contiguous ranges, one per XCD; each
// workgroup takes the next item of its own XCD's range from that XCD's
// counter and, once that range is exhausted, takes items from the others.
// Returns -1 when no item is left.  Called by every thread of the workgroup;
// `first` is true on the first call.
__device__ __forceinline__ long long xcd_remap(long long bid, long long nwg)
{
    const long long q = nwg / kXcds, r = nwg % kXcds;
    const long long xcd = bid % kXcds, local = bid / kXcds;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

__device__ __forceinline__ long long next_item(BatchHdr *h, int stage, long long total, long long *s_item,
                                               bool &first)
{
    if ((long long)gridDim.x >= total) {
        if (!first) return -1;
        first = false;
        const long long id = xcd_remap(blockIdx.x, gridDim.x);
        return id < total ? id : -1;
    }
    first = false;
    const long long per = (total + kXcds - 1) / kXcds;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long found = -1;
        const int home = blockIdx.x % kXcds;
        for (int t = 0; t < kXcds; ++t) {
            const int x = (home + t) % kXcds;
            const long long lo = (long long)x * per;
            const long long hi = min(total, lo + per);
            if (lo >= hi) continue;
            const unsigned int got = atomicAdd(&h->counter[stage * kXcds + x], 1u);
            if (lo + (long long)got < hi) {
                found = lo + (long long)got;
                break;
            }
        }
        *s_item = found;
    }
    __syncthreads();
    return uniform64(*s_item);
}

// ===========================================================================
// stage A1: wipe + fold, then the one-chip boxcar
// F[n] = sum_{t<spc} f[(n+t) mod N], written split by phase:
// F[vec(k, b, s)][m] = F[spc m + s] (m < 1023), [..][1023] = 0.  A work item is
// one (request, Doppler, block), done in chunks of kBoxChunk outputs, each
// wiping the spc - 1 samples past it as a halo.  All integer, exact.
// ===========================================================================
constexpr int kBoxRun = 8;
__device__ __forceinline__ int bpad(int i) { return i + (i >> 3); }  // bank-conflict padding

// Wipe + fold of samples n0 .. n0 + len - 1 (mod N) of block b into s_f,
// FMT-specialised; the phase of the folded milliseconds advances by N D (mod
// 2^32) from one to the next, and |x| <= 127, |LUT| <= 4096 make the 24-bit
// multiplies exact.  Same values as wipe_fold_one.  Samples are addressed from
// the block's first byte (the same pointer in every thread) by 32-bit in-block
// offsets: a block holds Tc N <= 64 * 16368 samples.
template <int FMT, int NT>
__device__ __forceinline__ void box_wipe(const void *samples, int N, int Tc, const uint32_t *s_lut, uint32_t D,
                                         int b, int n0, int len, int shift, int2 *s_f)
{
    const uint32_t dN = (uint32_t)N * D;
    const long long base = (long long)b * Tc * N;
    // 2-bit packed records: the block may start inside a byte
    const uint32_t sub = FMT == GNSS_REAL_2BIT_PACKED ? (uint32_t)(base & 3) : 0u;
    const long long blk_byte = FMT == GNSS_CPLX_I8 ? 2 * base : FMT == GNSS_REAL_I8 ? base : (base >> 2);
    const GNSS_GLOBAL uint8_t *blk = (const GNSS_GLOBAL uint8_t *)samples + blk_byte;
    const uint32_t step = FMT == GNSS_CPLX_I8 ? 2u * (uint32_t)N : (uint32_t)N;  // bytes (samples if packed)
    for (int i = threadIdx.x; i < len; i += NT) {
        int n = n0 + i - shift;  // shift in [0, N): the block read circularly delayed
        if (n < 0) n += N;
        if (n >= N) n -= N;
        uint32_t ph = (uint32_t)(base + n) * D;
        // the milliseconds' phases are ph + c N D: additions, not one multiply each
        asm volatile("" : "+v"(ph));
        // byte offset (sample index if packed) of millisecond c in the block
        uint32_t off = FMT == GNSS_CPLX_I8 ? 2u * (uint32_t)n : (uint32_t)n + sub;
        int yr = 0, yi = 0;
#pragma unroll 4
        for (int c = 0; c < Tc; ++c) {
            int xr, xi;
            if (FMT == GNSS_CPLX_I8) {
                const uint32_t v = *(const GNSS_GLOBAL uint16_t *)(blk + off);  // I in the low byte
                xr = (int)(int8_t)(v & 0xFFu);
                xi = (int)(int8_t)(v >> 8);
            } else if (FMT == GNSS_REAL_I8) {
                xr = (int)(int8_t)blk[off];
                xi = 0;
            } else {
                const uint32_t code = (blk[off >> 2] >> (2u * (off & 3u))) & 3u;
                // 00:+1 01:+3 10:-1 11:-3
                const int mag = (code & 1u) ? 3 : 1;
                xr = (code & 2u) ? -mag : mag;
                xi = 0;
            }
            const uint32_t e = s_lut[ph >> 22];
            const int cs = (int)(int16_t)(e & 0xFFFFu), sn = (int)(int16_t)(e >> 16);
            if (FMT == GNSS_CPLX_I8) {
                yr += __mul24(xr, cs) + __mul24(xi, sn);
                yi += __mul24(xi, cs) - __mul24(xr, sn);
            } else {
                yr += __mul24(xr, cs);
                yi -= __mul24(xr, sn);
            }
            off += step;
            ph += dN;
        }
        s_f[bpad(i)] = make_int2(yr, yi);
    }
}

// LDS chunk buffer of box_item: kBoxChunk + spc - 1 wiped samples, padded
constexpr int kBoxBuf = (kBoxChunk + kMaxSpc) + (kBoxChunk + kMaxSpc) / 8 + 8;

// The wipe, fold, boxcar and polyphase split of one (Doppler k, block b) item
// of request d by NT threads: dst[s * kPolyLen + m] = F[spc m + s] for m <
// 1023 and 0 at m = 1023 (dst: the item's polyphase vectors in F).
template <int NT, typename DstPtr>
__device__ __forceinline__ void box_item(const ReqDesc &d, int k, int b, const uint32_t *s_lut, int2 *s_f,
                                         DstPtr dst)
{
    const int N = d.N, spc = d.spc;
    const uint32_t D = d.dk[k];
    // code-Doppler drift of this (bin, block) in samples, in [0, N): delaying
    // the folded block by it circularly shifts its correlation by as many lags
    const int shift = d.cshift ? d.cshift[(long long)k * d.Nnc + b] : 0;
    for (int n0 = 0; n0 < N; n0 += kBoxChunk) {
        const int cnt = min(kBoxChunk, N - n0);
        const int len = cnt + spc - 1;
        __syncthreads();  // LUT staged / previous chunk's boxcar done
        if (d.fmt == GNSS_CPLX_I8)
            box_wipe<GNSS_CPLX_I8, NT>(d.samples, N, d.Tc, s_lut, D, d.b0 + b, n0, len, shift, s_f);
        else if (d.fmt == GNSS_REAL_I8)
            box_wipe<GNSS_REAL_I8, NT>(d.samples, N, d.Tc, s_lut, D, d.b0 + b, n0, len, shift, s_f);
        else
            box_wipe<GNSS_REAL_2BIT_PACKED, NT>(d.samples, N, d.Tc, s_lut, D, d.b0 + b, n0, len, shift, s_f);
        __syncthreads();
        const int n_runs = (cnt + kBoxRun - 1) / kBoxRun;
        for (int rr = threadIdx.x; rr < n_runs; rr += NT) {
            const int i0 = rr * kBoxRun;
            int sx = 0, sy = 0;
            for (int t = 0; t < spc; ++t) {
                int2 v = s_f[bpad(i0 + t)];
                sx += v.x;
                sy += v.y;
            }
            const int n = n0 + i0;
            int m = n / spc, s = n - m * spc;
#pragma unroll
            for (int j = 0; j < kBoxRun; ++j) {
                const int i = i0 + j;
                if (i >= cnt) break;
                dst[s * kPolyLen + m] = make_int2(sx, sy);
                if (i + 1 < cnt) {
                    int2 vi = s_f[bpad(i + spc)], vo = s_f[bpad(i)];
                    sx += vi.x - vo.x;
                    sy += vi.y - vo.y;
                }
                if (++s == spc) {
                    s = 0;
                    ++m;
                }
            }
        }
    }
    if (threadIdx.x < spc) dst[threadIdx.x * kPolyLen + (kPolyLen - 1)] = make_int2(0, 0);
}

__global__ __launch_bounds__(256) void k_box(const ReqDesc *__restrict__ R, BatchHdr *H, const long long *pre,
                                             const uint32_t *lut, int2 *F)
{
    __shared__ int2 s_f[kBoxBuf];
    __shared__ uint32_t s_lut[1024];
    __shared__ long long s_item;
    for (int i = threadIdx.x; i < 1024; i += 256) s_lut[i] = lut[i];
    const int n_req = H->n_req;
    const long long total = H->total[kStBox];
    const long long *pst = pre + (long long)kStBox * (n_req + 1);
    bool first = true;
    for (;;) {
        const long long it = next_item(H, kStBox, total, &s_item, first);
        if (it < 0) break;
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        // (Doppler, block)-major items (dealing them block-major, so that the bins of
        // a block share its samples in L2, was measured 15% slower)
        const int kb = (int)(it - pst[r]);  // < 2^31 by the plan checks
        const int k = kb / d.Nnc, b = kb - (kb / d.Nnc) * d.Nnc;
        box_item<256>(d, k, b, s_lut, s_f, F + (d.vec_off + (long long)kb * d.spc) * kPolyLen);
    }
}

// ===========================================================================
// stage A2: forward 2048-point FFT of every polyphase component (one wave
// per vector; vectors of all requests are contiguous in F and G)
// ===========================================================================
__global__ __launch_bounds__(256) void k_fft_poly(const int2 *F, const float2 *tw, float4 *G,
                                                  const BatchHdr *H)
{
    __shared__ float2 s_tw[kTwElems];
    __shared__ float2 s_xb[4][kXbufElemsQ];  // transposes in quarters: fewer LDS bank conflicts
    stage_twiddles(s_tw, tw, threadIdx.x, 256);
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const long long n_vec = H->total[kStVec];
    for (long long vec = (long long)blockIdx.x * 4 + w; vec < n_vec; vec += (long long)gridDim.x * 4) {
        const int2 *src = F + vec * kPolyLen;
        float2 v[32];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k2b = 0; k2b < 8; ++k2b) {
                if (k2b < 4) {
                    int2 t = src[l + 64 * u + 256 * k2b];
                    v[8 * u + k2b] = make_float2((float)t.x, (float)t.y);
                } else {
                    v[8 * u + k2b] = make_float2(0.f, 0.f);
                }
            }
        fft2048<true, true>(v, s_xb[w], s_tw, s_tw + kT1Elems, l);
        float4 *dst = G + vec * kVec;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
            dst[jj * 64 + l] = make_float4(v[2 * jj].x, v[2 * jj].y, v[2 * jj + 1].x, v[2 * jj + 1].y);
    }
}

// ===========================================================================
// stage B: fused conj-multiply -> IFFT -> |.|^2 -> non-coherent sum
// ===========================================================================

// Grid write of a correlation work item.  Lag tau = spc*q + s interleaves the
// waves' phases, so the sums are staged in LDS ([1024 q][W + 1] floats per
// PRN: both the per-wave writes and the per-row reads are free of bank
// conflicts) and written as contiguous runs of consecutive tau.
// write_rows writes one PRN's staged sums (column w = wave w's (Doppler,
// phase) item; consecutive items of a bin are consecutive lags), or adds
// them to the grid (add): the element-to-thread map depends only on the
// request, chunk and thread, so each thread reads back its own earlier store.
template <int W>
__device__ __forceinline__ void write_rows(const float *st, const ReqDesc &d, int pi, int chunk, int tid, bool add = false)
{
    constexpr int kPad = W + 1;
    const int spc = d.spc;
    const int first = chunk * W;
    const int n_items_here = min(W, d.n_items - first);
    int wa = 0;
    while (wa < n_items_here) {
        const int ka = (first + wa) / spc, sa = (first + wa) - ka * spc;
        const int ns = min(spc - sa, n_items_here - wa);  // consecutive phases of bin ka
        const int cnt = kCodeLen * ns;
        GNSS_GLOBAL float *row = gmem(d.grid) + ((long long)pi * d.n_dopp + ka) * d.N + sa;
        for (int idx = tid; idx < cnt; idx += 64 * W) {
            const int q = idx / ns, j = idx - q * ns;
            GNSS_GLOBAL float *o = row + (long long)spc * q + j;
            *o = add ? *o + st[q * kPad + wa + j] : st[q * kPad + wa + j];
        }
        wa += ns;
    }
}

// Stages and writes a tile's sums, P = |IFFT|^2 * scale (2^-22 for the
// unnormalised 2048-point IFFT and 2^-24 for the LUT scale, times the FP16
// path's code-spectrum scaling); add: adds them to the grid's sums instead
// (every wave of the workgroup passes the same flag).
template <int PT, int W>
__device__ __forceinline__ void store_tile(const float (&acc)[PT][16], float *s_stage, const ReqDesc &d,
                                           int ptile, int chunk, int w, int l, int tid, float scale,
                                           bool add = false)
{
    constexpr int kPad = W + 1;
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k2b = 0; k2b < 4; ++k2b) {
                int q = l + 64 * u + 256 * k2b;
                s_stage[(p * 1024 + q) * kPad + w] = acc[p][4 * u + k2b] * scale;
            }
    __syncthreads();
    for (int p = 0; p < PT; ++p) {
        const int pi = ptile * PT + p;
        if (pi >= d.n_prn) break;
        write_rows<W>(s_stage + p * 1024 * kPad, d, pi, chunk, tid, add);
    }
}

// Cascaded non-coherent sums: a wave adds its lanes' sums of the group of
// blocks just done to the grid (add) or stores them there (the first group),
// then clears them; each lane reads back only its own stores, and the final
// write (store_tile with add, another thread per element) comes after its
// workgroup barriers.  Lane l holds the lags q = l + 64 u + 256 k2b of the
// item (bin k, phase s): grid column s + spc q.
template <int PT>
__device__ __forceinline__ void add_group(float (&acc)[PT][16], const ReqDesc &d, int ptile, int k, int s, int l,
                                          float scale, bool add)
{
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        const int pi = ptile * PT + p;
        if (pi < d.n_prn) {
            GNSS_GLOBAL float *row = gmem(d.grid) + ((long long)pi * d.n_dopp + k) * d.N + s;
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int k2b = 0; k2b < 4; ++k2b) {
                    const int q = l + 64 * u + 256 * k2b;
                    if (q < kCodeLen) {
                        GNSS_GLOBAL float *o = row + (long long)d.spc * q;
                        const float v = acc[p][4 * u + k2b] * scale;
                        *o = add ? *o + v : v;
                    }
                }
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[p][i] = 0.f;
    }
}

// Work item = (request, PRN tile, chunk of kCorrWaves (Doppler, phase)
// items); one wave per (Doppler, phase) item, looping over the blocks and the
// tile's PT PRNs with the sums in registers.
// W waves per workgroup, WPE the waves per SIMD the registers are budgeted for
// (PRN tile 1 at three waves per SIMD: 164 VGPRs; tiles 2 and 4 at two;
// tile 4, at the 256-register limit, keeps 12 bytes of its set-up in
// scratch, stored once per item and reloaded for the final write).
template <int PT, int W, int WPE>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(WPE))) void k_corr(const ReqDesc *__restrict__ R, BatchHdr *H,
                                                          const long long *pre, const float4 *G,
                                                          const float4 *__restrict__ CS,
                                                          const float2 *__restrict__ tw)
{
    constexpr int kCcBytes = PT * kVec * (int)sizeof(float4);
    constexpr int kTwBytes = kTwElems * (int)sizeof(float2);
    // the transposes go through a quarter-size buffer per wave in four rounds:
    // measured faster than the full buffer (its paired accesses conflict in LDS)
    constexpr int kXbBytes = W * kXbufElemsQ * (int)sizeof(float2);
    constexpr int kStageBytes = PT * 1024 * (W + 1) * (int)sizeof(float);
    constexpr int kSmem = (kCcBytes + kTwBytes + kXbBytes) > kStageBytes ? (kCcBytes + kTwBytes + kXbBytes)
                                                                          : kStageBytes;
    __shared__ __align__(16) unsigned char smem[kSmem];
    __shared__ long long s_item;
    float4 *s_cc = (float4 *)smem;
    float2 *s_tw = (float2 *)(smem + kCcBytes);
    float2 *s_xb = (float2 *)(smem + kCcBytes + kTwBytes);
    float *s_stage = (float *)smem;  // reused after the transforms

    const int tid = threadIdx.x;
    // the wave index as a wave-uniform (scalar) value: the item's bin and
    // phase derived from it stay out of the vector registers
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
    const int n_req = H->n_req;
    const long long total = H->total[kStCorr];
    const long long *pst = pre + (long long)kStCorr * (n_req + 1);
    bool first = true;
    for (;;) {
        const long long it = next_item(H, kStCorr, total, &s_item, first);
        if (it < 0) break;
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        const long long local = it - pst[r];
        const int ptile = (int)(local % d.n_ptiles), chunk = (int)(local / d.n_ptiles);
        const int item = chunk * W + w;
        const bool active = item < d.n_items;
        const int spc = d.spc;
        const int k = item / spc, s = item - k * spc;

        // code spectra of the tile's PRNs and the twiddles (in a persistent
        // launch this overwrites the staging area of the previous item's
        // write: the barrier inside next_item separates them)
        for (int i = tid; i < PT * kVec; i += 64 * W) {
            int p = i / kVec, e = i - p * kVec;
            int pi = ptile * PT + p;
            int prn = pi < d.n_prn ? d.prns[pi] : 0;
            s_cc[i] = CS[(long long)prn * kVec + e];
        }
        stage_twiddles(s_tw, tw, tid, 64 * W);
        __syncthreads();

        float acc[PT][16];
#pragma unroll
        for (int p = 0; p < PT; ++p)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[p][i] = 0.f;

        if (active) {
            float2 *xb = s_xb + w * kXbufElemsQ;
            // groups of kSumGroup blocks (one for most requests)
            for (int b0 = 0; b0 < d.Nnc; b0 += kSumGroup) {
                if (b0) add_group<PT>(acc, d, ptile, k, s, l, 0x1p-46f, d.acc || b0 > kSumGroup);
                const float4 *gk = G + (d.vec_off + ((long long)k * d.Nnc + b0) * spc + s) * kVec;
                const int nb = min(d.Nnc - b0, kSumGroup);
                for (int b = 0; b < nb; ++b) {
                    const float4 *gp = gk + (long long)b * spc * kVec;
                    // PRN slots past n_prn hold the all-zero spectrum of row 0; they are
                    // computed (no branch in the loop) but never written.
#pragma unroll
                    for (int p = 0; p < PT; ++p) {
                        // the block spectrum is re-read for every PRN of the tile (L1/L2
                        // hits after the first) rather than pinned in registers
                        float2 z[32];
                        const float4 *gq = gp;
                        asm volatile("" : "+v"(gq));
                        phase_barrier();
#pragma unroll
                        for (int jj = 0; jj < 16; ++jj) {
                            float4 t = gq[jj * 64 + l];
                            float4 c = s_cc[p * kVec + jj * 64 + l];
                            z[2 * jj] = c_mul(make_float2(t.x, t.y), make_float2(c.x, c.y));
                            z[2 * jj + 1] = c_mul(make_float2(t.z, t.w), make_float2(c.z, c.w));
                        }
                        phase_barrier();
                        ifft2048<true, true>(z, xb, s_tw, s_tw + kT1Elems, l);
                        phase_barrier();
#pragma unroll
                        for (int u = 0; u < 4; ++u)
#pragma unroll
                            for (int k2b = 0; k2b < 4; ++k2b) {
                                float2 rv = z[8 * u + k2b];
                                acc[p][4 * u + k2b] = fmaf(rv.x, rv.x, fmaf(rv.y, rv.y, acc[p][4 * u + k2b]));
                            }
                    }
                }
            }
        }

        store_tile<PT, W>(acc, s_stage, d, ptile, chunk, w, l, tid, 0x1p-46f, d.acc || d.Nnc > kSumGroup);
    }
}

bool corr_shape_valid(CorrShape c, int precision)
{
    if (!corr_ptile_valid(c.pt, precision)) return false;
    if (precision != GNSS_FP32 || c.pt != 1) return c.w == corr_waves(precision, c.pt);
    return c.w == 12 || c.w == 6 || c.w == 4;
}

int corr_ptile_valid(int pt, int precision)
{
    return precision == GNSS_FP32 ? (pt == 1 || pt == 2 || pt == 4)
           : precision == GNSS_FP16 ? (pt == 2 || pt == 4)
                                    : (pt == 1 || pt == 2 || pt == 4 || pt == 8);
}

// ===========================================================================
// FP16 path: packed half-precision transforms with block floating point
// ===========================================================================
// Scaling.  Each polyphase vector g is scaled by 2^-e (e per vector, from its
// l1 norm) so that ||g 2^-e||_1 <= 32, and every code spectrum by the common
// 2^-ecs with max|C 2^-ecs| <= 1.  Then every intermediate stays below 2^15:
// all forward-transform values are bounded by the l1 norm (<= 32); the
// spectrum product by 32; the inverse transform's radix-16 outputs by 16*32
// and 256*32, the radix-8 partial sums by 4*256*32 = 2^15; and its outputs
// (the correlation times 2048 * 2^-ecs) by 2^(16 - ecs).  The scale factors
// are exact powers of two; |.|^2 and the sum over blocks are FP32.
constexpr int kL1Exp = 5;  // ||g 2^-e||_1 <= 2^5

// Smallest e with s * 2^-e <= 2^kL1Exp for a float sum s of non-negative
// terms (the factor covers the rounding of that sum).
__device__ __forceinline__ int l1_exponent(float s)
{
    if (!(s > 0.f)) return 0;
    int x;
    (void)frexpf(s * (1.f + 0x1p-10f), &x);  // s' < 2^x
    return x - kL1Exp;
}

// Sum over the wave; every lane gets the same value (each butterfly level adds
// the same two operands on both partner lanes).
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ uint32_t h2_bits(__half2 h) { return __builtin_bit_cast(uint32_t, h); }
__device__ __forceinline__ __half2 bits_h2(uint32_t u) { return __builtin_bit_cast(__half2, u); }

// hc2 twiddles: the T1/T2 tables of the FP32 path rounded to FP16 from the
// exact angle, each value in both halves.
__global__ void k_twiddles_h(hc2 *tw)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double s, c;
    int e;
    double den;
    if (i < kT1Elems) {
        int hk = i >> 6, l = i & 63;
        int h = hk >> 4, k1 = hk & 15;
        e = ((l + 64 * h) * k1) & 2047;
        den = 1024.0;
    } else if (i < kTwElems) {
        int j = i - kT1Elems;
        int k2a = j >> 3, m2 = j & 7;
        e = (m2 * k2a) & 127;
        den = 64.0;
    } else {
        return;
    }
    sincospi((double)e / den, &s, &c);
    // one rounding, double -> FP16 (round to nearest even)
    const __half hc = __builtin_bit_cast(__half, (_Float16)c), hs = __builtin_bit_cast(__half, (_Float16)s);
    tw[i] = make_hc2(__halves2half2(hc, hc), __halves2half2(hs, hs));
}

// FP16 code spectra: CSh[prn] = conj(C) * 2^-ecs as (re, im) half2 in the
// packed storage order (uint4 unit 64 jj + l holds registers 4 jj .. 4 jj + 3
// of lane l), from the FP32 spectra.
__global__ void k_code_spectra_h(const float4 *cs, uint4 *csh, int ecs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // prn * 512 + 64 jj + l
    if (i >= (kMaxPrn + 1) * 512) return;
    const int prn = i >> 9, unit = i & 511, jj = unit >> 6, l = unit & 63;
    const float sc = ldexpf(1.f, -ecs);
    const float4 *src = cs + (long long)prn * kVec;
    const float4 a = src[(2 * jj) * 64 + l], b = src[(2 * jj + 1) * 64 + l];
    csh[i] = make_uint4(h2_bits(__floats2half2_rn(a.x * sc, a.y * sc)), h2_bits(__floats2half2_rn(a.z * sc, a.w * sc)),
                        h2_bits(__floats2half2_rn(b.x * sc, b.y * sc)), h2_bits(__floats2half2_rn(b.z * sc, b.w * sc)));
}

// dck[prn] = 2048 * 2^-ecs * sum(code) / 1023 (PRN 0: 0)
__global__ void k_code_dc_h(const uint8_t *codes, float *dck, int ecs)
{
    const int prn = blockIdx.x * blockDim.x + threadIdx.x;
    if (prn > kMaxPrn) return;
    int sum = 0;
    if (prn > 0)
        for (int m = 0; m < kCodeLen; ++m) sum += codes[prn * kCodeLen + m] ? -1 : 1;
    dck[prn] = ldexpf(2048.f, -ecs) * (float)sum / (float)kCodeLen;
}

hipError_t launch_tables_h(const float4 *d_cs, const uint8_t *d_codes, void *d_tw_h, void *d_cs_h, int cs_exp,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_code_dc_h, dim3(1), dim3(64), 0, s, d_codes, (float *)((char *)d_cs_h + kCsHSpecBytes),
                       cs_exp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_twiddles_h, dim3((kTwElems + 255) / 256), dim3(256), 0, s, (hc2 *)d_tw_h);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_code_spectra_h, dim3(((kMaxPrn + 1) * 512 + 255) / 256), dim3(256), 0, s, d_cs,
                       (uint4 *)d_cs_h, cs_exp);
    return hipGetLastError();
}

__device__ __forceinline__ void stage_twiddles_h(hc2 *s_tw, const hc2 *tw, int tid, int nthreads)
{
    for (int i = tid; i < kTwElems; i += nthreads) s_tw[i] = tw[i];
}

// Forward transforms, two polyphase vectors per wave (the low and high
// halves).  Each vector is transformed with its mean S/1023 removed (S its
// sum over the 1023 values), scaled by 2^-e with e from the l1 norm of the
// mean-removed vector plus |S|; the correlation adds the mean's part back as
// the constant S/1023 * sum(code) of every lag.  (A strong DC component would
// otherwise cancel in the inverse transform against values far larger than
// the result, and the FP16 roundings of those values would dominate it.)
// Output: Gh[vec] in the packed storage order, the vector's exponent E[vec]
// and its scaled sum Dc[vec] = S * 2^-e.
// three waves per SIMD (168 VGPRs with a 44-byte spill): faster than two
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_fft_poly_h(const int2 *F, const hc2 *tw, uint4 *Gh, int *E,
                                                    float2 *Dc, const BatchHdr *H)
{
    __shared__ hc2 s_tw[kTwElems];
    __shared__ hc2 s_xb[4][kXbufElemsQ];
    stage_twiddles_h(s_tw, tw, threadIdx.x, 256);
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const long long n_vec = H->total[kStVec];
    const long long n_pair = (n_vec + 1) / 2;
    for (long long pr = (long long)blockIdx.x * 4 + w; pr < n_pair; pr += (long long)gridDim.x * 4) {
        const long long va = 2 * pr, vb = va + 1;
        const bool has_b = vb < n_vec;
        const int2 *sa = F + va * kPolyLen, *sb = F + vb * kPolyLen;
        int2 a[16], b[16];
        float sar = 0.f, sai = 0.f, sbr = 0.f, sbi = 0.f;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k2b = 0; k2b < 4; ++k2b) {
                const int idx = l + 64 * u + 256 * k2b;  // element 1023 is zero
                a[4 * u + k2b] = sa[idx];
                b[4 * u + k2b] = has_b ? sb[idx] : make_int2(0, 0);
                sar += (float)a[4 * u + k2b].x;
                sai += (float)a[4 * u + k2b].y;
                sbr += (float)b[4 * u + k2b].x;
                sbi += (float)b[4 * u + k2b].y;
            }
        const float Sar = wave_sum(sar), Sai = wave_sum(sai), Sbr = wave_sum(sbr), Sbi = wave_sum(sbi);
        // IEEE division: a constant vector's mean is its value exactly
        const float mar = Sar / (float)kCodeLen, mai = Sai / (float)kCodeLen;
        const float mbr = Sbr / (float)kCodeLen, mbi = Sbi / (float)kCodeLen;
        float na = 0.f, nb = 0.f;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k2b = 0; k2b < 4; ++k2b)
                if (l + 64 * u + 256 * k2b < kCodeLen) {
                    na += fabsf((float)a[4 * u + k2b].x - mar) + fabsf((float)a[4 * u + k2b].y - mai);
                    nb += fabsf((float)b[4 * u + k2b].x - mbr) + fabsf((float)b[4 * u + k2b].y - mbi);
                }
        const int ea = l1_exponent(wave_sum(na) + fabsf(Sar) + fabsf(Sai));
        const int eb = l1_exponent(wave_sum(nb) + fabsf(Sbr) + fabsf(Sbi));
        const float fa = ldexpf(1.f, -ea), fb = ldexpf(1.f, -eb);
        hc2 v[32];
        const __half2 zero = __floats2half2_rn(0.f, 0.f);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k2b = 0; k2b < 8; ++k2b) {
                if (k2b < 4) {
                    const int2 x = a[4 * u + k2b], y = b[4 * u + k2b];
                    // the zero element 1023 stays zero
                    const bool in = l + 64 * u + 256 * k2b < kCodeLen;
                    const float xr = in ? ((float)x.x - mar) * fa : 0.f, xi = in ? ((float)x.y - mai) * fa : 0.f;
                    const float yr = in ? ((float)y.x - mbr) * fb : 0.f, yi = in ? ((float)y.y - mbi) * fb : 0.f;
                    v[8 * u + k2b] = make_hc2(__floats2half2_rn(xr, yr), __floats2half2_rn(xi, yi));
                } else {
                    v[8 * u + k2b] = make_hc2(zero, zero);
                }
            }
        fft2048<true, true>(v, s_xb[w], s_tw, s_tw + kT1Elems, l);
        uint4 *ga = Gh + va * 512, *gb = Gh + vb * 512;
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const hc2 *q = v + 4 * jj;
            ga[jj * 64 + l] = make_uint4(h2_bits(__lows2half2(q[0].re, q[0].im)), h2_bits(__lows2half2(q[1].re, q[1].im)),
                                         h2_bits(__lows2half2(q[2].re, q[2].im)), h2_bits(__lows2half2(q[3].re, q[3].im)));
            if (has_b)
                gb[jj * 64 + l] = make_uint4(h2_bits(__highs2half2(q[0].re, q[0].im)), h2_bits(__highs2half2(q[1].re, q[1].im)),
                                             h2_bits(__highs2half2(q[2].re, q[2].im)), h2_bits(__highs2half2(q[3].re, q[3].im)));
        }
        if (l == 0) {
            E[va] = ea;
            Dc[va] = make_float2(Sar * fa, Sai * fa);
            if (has_b) {
                E[vb] = eb;
                Dc[vb] = make_float2(Sbr * fb, Sbi * fb);
            }
        }
    }
}

// (g.re + i g.im) * c for both transforms of c
__device__ __forceinline__ hc2 c_mul_bcast(__half2 g, hc2 c)
{
    const __half2 gr = __low2half2(g), gi = __high2half2(g);
    return make_hc2(__hfma2(gr, c.re, __hneg2(__hmul2(gi, c.im))), __hfma2(gr, c.im, __hmul2(gi, c.re)));
}

// FP16 correlation: as k_corr, with the tile's PRNs in pairs, one packed
// inverse transform per pair and block.  Work item = (request, PRN tile,
// chunk of kCorrWavesH (Doppler, phase) items).
template <int PT>
__global__ __launch_bounds__(64 * kCorrWavesH) __attribute__((amdgpu_waves_per_eu(PT == 2 ? 3 : 1))) void k_corr_h(const ReqDesc *__restrict__ R, BatchHdr *H,
                                                             const long long *pre, const uint4 *Gh,
                                                             const int *E, const float2 *Dc,
                                                             const uint4 *__restrict__ CSh,
                                                             const float *__restrict__ dck,
                                                             const hc2 *__restrict__ tw, float out_scale)
{
    static_assert(PT % 2 == 0, "PRNs go in pairs");
    constexpr int NP = PT / 2;
    constexpr int W = kCorrWavesH;
    constexpr int kCcBytes = NP * 1024 * (int)sizeof(uint4);
    constexpr int kTwBytes = kTwElems * (int)sizeof(hc2);
    constexpr int kXbBytes = W * kXbufElemsQ * (int)sizeof(hc2);
    constexpr int kStageBytes = PT * 1024 * (W + 1) * (int)sizeof(float);
    constexpr int kSmem = (kCcBytes + kTwBytes + kXbBytes) > kStageBytes ? (kCcBytes + kTwBytes + kXbBytes)
                                                                          : kStageBytes;
    __shared__ __align__(16) unsigned char smem[kSmem];
    __shared__ long long s_item;
    uint4 *s_cc = (uint4 *)smem;  // unit 64 jj2 + l: registers 2 jj2, 2 jj2 + 1 of lane l (hc2 each)
    hc2 *s_tw = (hc2 *)(smem + kCcBytes);
    hc2 *s_xb = (hc2 *)(smem + kCcBytes + kTwBytes);
    float *s_stage = (float *)smem;

    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63;
    const int n_req = H->n_req;
    const long long total = H->total[kStCorr];
    const long long *pst = pre + (long long)kStCorr * (n_req + 1);
    bool first = true;
    for (;;) {
        const long long it = next_item(H, kStCorr, total, &s_item, first);
        if (it < 0) break;
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        const long long local = it - pst[r];
        const int ptile = (int)(local % d.n_ptiles), chunk = (int)(local / d.n_ptiles);
        for (int i = tid; i < NP * 1024; i += 64 * W) {
            const int pp = i >> 10, unit = i & 1023, jj2 = unit >> 6, ll = unit & 63;
            const int pa = ptile * PT + 2 * pp, pb = pa + 1;
            const int prn_a = pa < d.n_prn ? d.prns[pa] : 0, prn_b = pb < d.n_prn ? d.prns[pb] : 0;
            const uint4 ca = CSh[(long long)prn_a * 512 + (jj2 >> 1) * 64 + ll];
            const uint4 cb = CSh[(long long)prn_b * 512 + (jj2 >> 1) * 64 + ll];
            const uint32_t a0 = (jj2 & 1) ? ca.z : ca.x, a1 = (jj2 & 1) ? ca.w : ca.y;
            const uint32_t b0 = (jj2 & 1) ? cb.z : cb.x, b1 = (jj2 & 1) ? cb.w : cb.y;
            s_cc[i] = make_uint4(h2_bits(__lows2half2(bits_h2(a0), bits_h2(b0))), h2_bits(__highs2half2(bits_h2(a0), bits_h2(b0))),
                                 h2_bits(__lows2half2(bits_h2(a1), bits_h2(b1))), h2_bits(__highs2half2(bits_h2(a1), bits_h2(b1))));
        }
        stage_twiddles_h(s_tw, tw, tid, 64 * W);
        __syncthreads();

        const int item = chunk * W + w;
        const bool active = item < d.n_items;
        const int spc = d.spc;
        const int k = item / spc, s = item - k * spc;

        float acc[PT][16];
#pragma unroll
        for (int p = 0; p < PT; ++p)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[p][i] = 0.f;
        // per PRN: the lag-independent part of the inverse output per unit of
        // the scaled block sum, 2048 * 2^-ecs * sum(code) / 1023
        float kdc[PT];
#pragma unroll
        for (int p = 0; p < PT; ++p) {
            const int pi = ptile * PT + p;
            kdc[p] = dck[pi < d.n_prn ? d.prns[pi] : 0];
        }

        if (active) {
            const long long v0 = d.vec_off + (long long)k * d.Nnc * spc + s;
            hc2 *xb = s_xb + w * kXbufElemsQ;
            for (int b = 0; b < d.Nnc; ++b) {
                const long long vec = v0 + (long long)b * spc;
                const float sc = ldexpf(1.f, 2 * E[vec]);
                const float2 ds = Dc[vec];
#pragma unroll
                for (int pp = 0; pp < NP; ++pp) {
                    const __half2 dre = __floats2half2_rn(kdc[2 * pp] * ds.x, kdc[2 * pp + 1] * ds.x);
                    const __half2 dim = __floats2half2_rn(kdc[2 * pp] * ds.y, kdc[2 * pp + 1] * ds.y);
                    const uint4 *gq = Gh + vec * 512;
                    asm volatile("" : "+v"(gq));
                    phase_barrier();
                    hc2 z[32];
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj) {
                        const uint4 g = gq[jj * 64 + l];
                        const uint4 c0 = s_cc[pp * 1024 + (2 * jj) * 64 + l];
                        const uint4 c1 = s_cc[pp * 1024 + (2 * jj + 1) * 64 + l];
                        z[4 * jj + 0] = c_mul_bcast(bits_h2(g.x), make_hc2(bits_h2(c0.x), bits_h2(c0.y)));
                        z[4 * jj + 1] = c_mul_bcast(bits_h2(g.y), make_hc2(bits_h2(c0.z), bits_h2(c0.w)));
                        z[4 * jj + 2] = c_mul_bcast(bits_h2(g.z), make_hc2(bits_h2(c1.x), bits_h2(c1.y)));
                        z[4 * jj + 3] = c_mul_bcast(bits_h2(g.w), make_hc2(bits_h2(c1.z), bits_h2(c1.w)));
                    }
                    phase_barrier();
                    ifft2048<true, true>(z, xb, s_tw, s_tw + kT1Elems, l);
                    phase_barrier();
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int k2b = 0; k2b < 4; ++k2b) {
                            const hc2 o = z[8 * u + k2b];
                            const float2 re = __half22float2(__hadd2(o.re, dre)), im = __half22float2(__hadd2(o.im, dim));
                            const float ta = fmaf(re.x, re.x, im.x * im.x);
                            const float tb = fmaf(re.y, re.y, im.y * im.y);
                            acc[2 * pp][4 * u + k2b] = fmaf(ta, sc, acc[2 * pp][4 * u + k2b]);
                            acc[2 * pp + 1][4 * u + k2b] = fmaf(tb, sc, acc[2 * pp + 1][4 * u + k2b]);
                        }
                }
            }
        }

        store_tile<PT, W>(acc, s_stage, d, ptile, chunk, w, l, tid, out_scale, d.acc != 0);
    }
}

// ===========================================================================
// Exact-length mode (GNSS_FP16_PFA): the length-1023 correlations of the
// polyphase form with 1023-point transforms (Good-Thomas 31 x 33, no zero
// padding, pfa1023.hpp) whose two passes are FP16 x FP16 -> FP32 products on
// the matrix cores.  Scaling as in the FP16 mode: each polyphase vector is
// scaled by 2^-e so that its l1 norm is <= 32, and the code spectra by
// 2^-ecs so that max |C| <= 1.  Every pass output is bounded by the l1 norm
// of its input: the forward transform's values by 32, the spectrum product's
// by 32, the inverse 31-pass by 31 * 32 (rounded to FP16 for the second
// pass) and the 33-pass output (FP32) by 33 * 31 * 32.  |.|^2 is formed in
// FP32, times 2^(2e), summed over blocks; the grid gets 2^(2 ecs - 24) / 1023^2.
// ===========================================================================

// Real-form weight of an L-point DFT (L = 31 or 33): input (i_in, part p_in)
// to output (i_out, part p_out), parts 0 = re, 1 = im; zero outside [0, L).
// The complex weight is e^(-+ 2 pi i i_in i_out / L) (forward: minus).
__device__ double pfa_weight(int L, bool inv, int i_in, int p_in, int i_out, int p_out)
{
    if (i_in < 0 || i_out < 0 || i_in >= L || i_out >= L) return 0.0;
    const int e = (i_in * i_out) % L;
    double sn, cs;
    sincospi(2.0 * (double)e / (double)L, &sn, &cs);
    const double sg = inv ? 1.0 : -1.0;  // weight = cs + i sg sn
    // (xr + i xi)(cs + i sg sn) = (xr cs - xi sg sn) + i (xr sg sn + xi cs)
    if (p_out == 0) return p_in == 0 ? cs : -sg * sn;
    return p_in == 0 ? sg * sn : cs;
}

// two doubles to FP16 (one rounding, to nearest even)
__device__ __forceinline__ uint32_t pack2d(double x, double y)
{
    pfa::h2v v = {(_Float16)x, (_Float16)y};
    return __builtin_bit_cast(uint32_t, v);
}

// Output column of an x32 weight fragment: (index, part); index -1 = unused.
__device__ __forceinline__ void pfa_column(int L, bool inv, int tile, int c, int &i_out, int &p_out)
{
    if (L == pfa::kN1) {
        i_out = 16 * (tile & 1) + c;
        p_out = tile >> 1;
    } else if (tile < 4 || !inv) {
        i_out = 16 * (tile >> 1) + c;
        p_out = tile & 1;
    } else {  // inverse tile 4: column 32, re in lane c = 0, im in lane c = 1
        i_out = c < 2 ? 32 : -1;
        p_out = c & 1;
    }
}

// B fragments of the four passes (forward / inverse, 31 / 33), FP16.  K
// slot 8 g + j of step `step` is input index 16 step + 4 g + (j & 3), part
// j >> 2.
__global__ void k_pfa_frags(pfa::u4 *fr)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= pfa::kFrags * 64) return;
    const int f = i >> 6, l = i & 63, g = l >> 4, c = l & 15;
    int L, step, tile;
    bool inv;
    if (f < pfa::kFragInv33) {
        L = pfa::kN1, inv = true, step = f / 4, tile = f % 4;
    } else if (f < pfa::kFragFwd31) {
        L = pfa::kN2, inv = true, step = (f - pfa::kFragInv33) / 5, tile = (f - pfa::kFragInv33) % 5;
    } else if (f < pfa::kFragFwd33) {
        L = pfa::kN1, inv = false, step = (f - pfa::kFragFwd31) / 4, tile = (f - pfa::kFragFwd31) % 4;
    } else {
        L = pfa::kN2, inv = false, step = (f - pfa::kFragFwd33) / 6, tile = (f - pfa::kFragFwd33) % 6;
    }
    int i_out, p_out;
    pfa_column(L, inv, tile, c, i_out, p_out);
    double wv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) wv[j] = pfa_weight(L, inv, 16 * step + 4 * g + (j & 3), j >> 2, i_out, p_out);
    fr[i] = pfa::u4{pack2d(wv[0], wv[1]), pack2d(wv[2], wv[3]), pack2d(wv[4], wv[5]), pack2d(wv[6], wv[7])};
}

// Exact 1023-point spectra of the +-1 codes in FP64, [prn][a][b] at
// k = k(a, b) (PRN 0: zero).  Grid (31, 38), one thread per b.
__global__ __launch_bounds__(64) void k_code_spectra_x(const uint8_t *codes, double2 *out)
{
    __shared__ double2 s_w[kCodeLen];  // e^(-2 pi i j / 1023)
    for (int j = threadIdx.x; j < kCodeLen; j += 64) {
        double sn, cs;
        sincospi(2.0 * (double)j / (double)kCodeLen, &sn, &cs);
        s_w[j] = make_double2(cs, -sn);
    }
    __syncthreads();
    const int a = blockIdx.x, prn = blockIdx.y, b = threadIdx.x;
    if (b >= pfa::kN2) return;
    const int k = pfa::freq_index(a, b);
    double re = 0.0, im = 0.0;
    if (prn != 0) {
        const uint8_t *code = codes + prn * kCodeLen;
        int idx = 0;
        for (int m = 0; m < kCodeLen; ++m) {
            const double chip = code[m] ? -1.0 : 1.0;
            re += chip * s_w[idx].x;
            im += chip * s_w[idx].y;
            idx += k;
            if (idx >= kCodeLen) idx -= kCodeLen;
        }
    }
    out[((long long)prn * pfa::kN1 + a) * pfa::kN2 + b] = make_double2(re, im);
}

// Coordinates of stored unit `unit` of a spectrum (see pfa::kUnits).
__device__ __forceinline__ void pfa_unit(int unit, int &t, int &s, int &g, int &c)
{
    if (unit < pfa::kTailUnit) {
        const int ff = unit >> 6, l = unit & 63;
        t = ff >> 1, s = ff & 1, g = l >> 4, c = l & 15;
    } else {
        t = 2, s = (unit - pfa::kTailUnit) >> 2, g = (unit - pfa::kTailUnit) & 3, c = 0;
    }
}

// FP16 code spectra C * 2^-ecs in the stored fragment layout.
__global__ void k_code_spectra_x_pack(const double2 *cs, pfa::u4 *out, int ecs)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (kMaxPrn + 1) * pfa::kUnits) return;
    const int prn = i / pfa::kUnits, unit = i % pfa::kUnits;
    int t, s, g, c;
    pfa_unit(unit, t, s, g, c);
    double re[4], im[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int a = 16 * s + 4 * g + j, b = 16 * t + c;
        double2 v = make_double2(0.0, 0.0);
        if (a < pfa::kN1 && b < pfa::kN2) v = cs[((long long)prn * pfa::kN1 + a) * pfa::kN2 + b];
        re[j] = ldexp(v.x, -ecs);
        im[j] = ldexp(v.y, -ecs);
    }
    out[i] = pfa::u4{pack2d(re[0], re[1]), pack2d(re[2], re[3]), pack2d(im[0], im[1]), pack2d(im[2], im[3])};
}

hipError_t launch_tables_x_frags(void *d_frags, hipStream_t s)
{
    constexpr int n = pfa::kFrags * 64;
    hipLaunchKernelGGL(k_pfa_frags, dim3((n + 255) / 256), dim3(256), 0, s, (pfa::u4 *)d_frags);
    return hipGetLastError();
}

hipError_t launch_code_spectra_x(const uint8_t *d_codes, double2 *d_tmp, hipStream_t s)
{
    hipLaunchKernelGGL(k_code_spectra_x, dim3(pfa::kN1, kMaxPrn + 1), dim3(64), 0, s, d_codes, d_tmp);
    return hipGetLastError();
}

hipError_t launch_code_spectra_x_pack(const double2 *d_tmp, void *d_cs_x, int cs_exp, hipStream_t s)
{
    constexpr int n = (kMaxPrn + 1) * pfa::kUnits;
    hipLaunchKernelGGL(k_code_spectra_x_pack, dim3((n + 255) / 256), dim3(256), 0, s, d_tmp, (pfa::u4 *)d_cs_x,
                       cs_exp);
    return hipGetLastError();
}

// Forward transform of one polyphase vector held in LDS (xs, 1024 int2, the
// last zero) by one wave: its sum S and mean S/1023, the exponent from the l1
// norm of the mean-removed vector plus |S|, the Good-Thomas gather of the
// mean-removed vector into fragments, two passes, and the spectrum stored as
// fragments (dst) with its exponent (*e_out, lane 0).  The DC bin is stored as
// S itself.  Removing the mean keeps the FP16 weights from leaking a strong DC
// component into the other bins: the code spectra are +-1 at DC and about 32
// elsewhere, so a leak of a few 10^-6 of the DC amplitude into every bin would
// reach percents of the correlation of a DC-dominated block (a constant
// offset in the samples).
__device__ __forceinline__ void fft_x_vector(const int2 *xs, const pfa::FwdB &B, pfa::u4 *dst, int *e_out, int l)
{
    const int g = l >> 4, c = l & 15;
    int2 v[kPolyLen / 64];
    float sr = 0.f, si = 0.f;
#pragma unroll
    for (int i = 0; i < kPolyLen / 64; ++i) {
        v[i] = xs[l + 64 * i];  // element 1023 is zero
        sr += (float)v[i].x;
        si += (float)v[i].y;
    }
    const float Sr = wave_sum(sr), Si = wave_sum(si);
    // IEEE division: a constant vector's mean is its value exactly
    const float mr = Sr / (float)kCodeLen, mi = Si / (float)kCodeLen;
    float nrm = 0.f;
#pragma unroll
    for (int i = 0; i < kPolyLen / 64; ++i)
        if (l + 64 * i < kCodeLen) nrm += fabsf((float)v[i].x - mr) + fabsf((float)v[i].y - mi);
    const int e = l1_exponent(wave_sum(nrm) + fabsf(Sr) + fabsf(Si));
    const float f = ldexpf(1.f, -e);
    pfa::u4 a1[3][2];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            float re[4], im[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int n1 = 16 * s + 4 * g + j, n2 = 16 * t + c;
                re[j] = 0.f;
                im[j] = 0.f;
                if (n1 < pfa::kN1 && n2 < pfa::kN2) {
                    const int2 x = xs[pfa::time_index(n1, n2)];
                    re[j] = ((float)x.x - mr) * f;
                    im[j] = ((float)x.y - mi) * f;
                }
            }
            a1[t][s] = pfa::u4{pfa::pack2(re[0], re[1]), pfa::pack2(re[2], re[3]), pfa::pack2(im[0], im[1]),
                               pfa::pack2(im[2], im[3])};
        }
    pfa::f4 o[2][6];
    pfa::forward(a1, B, o);
    if (l == 0) {  // bin 0 (a = 0, b = 0): the vector's sum
        o[0][0].x = Sr * f;
        o[0][1].x = Si * f;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const pfa::f4 re = o[s][2 * t], im = o[s][2 * t + 1];
            dst[(2 * t + s) * 64 + l] = pfa::u4{pfa::pack2(re.x, re.y), pfa::pack2(re.z, re.w),
                                                pfa::pack2(im.x, im.y), pfa::pack2(im.z, im.w)};
        }
    if (c == 0) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const pfa::f4 re = o[s][4], im = o[s][5];
            dst[pfa::kTailUnit + 4 * s + g] = pfa::u4{pfa::pack2(re.x, re.y), pfa::pack2(re.z, re.w),
                                                      pfa::pack2(im.x, im.y), pfa::pack2(im.z, im.w)};
        }
    }
    if (l == 0) *e_out = e;
}

// Forward transforms of the polyphase vectors in F: one vector per wave,
// copied into LDS, then fft_x_vector.  (Fusing this with the wipe/fold stage,
// the spc vectors of a (Doppler, block) item built in LDS and transformed
// there, was measured slower: one 154 KB workgroup per CU left the wipe's
// memory latency exposed, 0.63 ms against 0.33 ms for the two kernels.)
__global__ __launch_bounds__(256) void k_fft_x(const int2 *F, const pfa::u4 *__restrict__ fr, pfa::u4 *Gx, int *E,
                                               const BatchHdr *H)
{
    __shared__ int2 s_x[4][kPolyLen];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    pfa::FwdB B;
    pfa::load_fwd(B, fr, l);
    const long long n_vec = H->total[kStVec];
    int2 *xs = s_x[w];
    for (long long vec = (long long)blockIdx.x * 4 + w; vec < n_vec; vec += (long long)gridDim.x * 4) {
        const int2 *src = F + vec * kPolyLen;
        lds_fence();  // the previous vector's gathers are complete
#pragma unroll
        for (int i = 0; i < kPolyLen / 64; ++i) xs[l + 64 * i] = src[l + 64 * i];
        lds_fence();
        fft_x_vector(xs, B, Gx + vec * pfa::kUnits, E + vec, l);
    }
}

// LDS copy of one stored spectrum: the four full fragments (1 KB each) and
// the 128-byte tail, staged as 32 dwords (lanes 32..63 repeat them).
constexpr int kXBuf = pfa::kTailUnit + 16;  // u4 units per LDS spectrum buffer
__device__ __forceinline__ void stage_spectrum(const pfa::u4 *src, pfa::u4 *dst, int l)
{
    typedef __attribute__((address_space(1))) const void gvoid;
    typedef __attribute__((address_space(3))) void lvoid;
#pragma unroll
    for (int f = 0; f < 4; ++f)
        __builtin_amdgcn_global_load_lds((gvoid *)(src + f * 64 + l), (lvoid *)(dst + f * 64), 16, 0, 0);
    const uint32_t *tail = (const uint32_t *)(src + pfa::kTailUnit);
    __builtin_amdgcn_global_load_lds((gvoid *)(tail + (l & 31)), (lvoid *)(dst + pfa::kTailUnit), 4, 0, 0);
}

// Value of lane 4 q + 1 in lane 4 q (DPP quad permutation [1, 1, 3, 3]).
__device__ __forceinline__ float from_next_lane(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0xF5, 0xF, 0xF, false));
}

// G * conj(C) for the four complex values of a fragment (packed FP16)
__device__ __forceinline__ pfa::u4 cmul_conj_frag(pfa::u4 g, pfa::u4 c)
{
    const __half2 gr0 = bits_h2(g.x), gr1 = bits_h2(g.y), gi0 = bits_h2(g.z), gi1 = bits_h2(g.w);
    const __half2 cr0 = bits_h2(c.x), cr1 = bits_h2(c.y), ci0 = bits_h2(c.z), ci1 = bits_h2(c.w);
    const __half2 yr0 = __hfma2(gr0, cr0, __hmul2(gi0, ci0)), yr1 = __hfma2(gr1, cr1, __hmul2(gi1, ci1));
    const __half2 yi0 = __hfma2(gi0, cr0, __hneg2(__hmul2(gr0, ci0)));
    const __half2 yi1 = __hfma2(gi1, cr1, __hneg2(__hmul2(gr1, ci1)));
    return pfa::u4{h2_bits(yr0), h2_bits(yr1), h2_bits(yi0), h2_bits(yi1)};
}

// Correlation, exact-length mode.  Work item = (request, PRN tile, chunk of
// kCorrWavesX (Doppler, phase) items); one wave per item; the tile's PRNs in
// turn, each over all blocks with its sums in registers, then written.
template <bool PAIRS>
__global__ __launch_bounds__(64 * kCorrWavesX) void k_corr_x(const ReqDesc *__restrict__ R, BatchHdr *H,
                                                             const long long *pre, const pfa::u4 *Gx,
                                                             const int *__restrict__ E, const pfa::u4 *__restrict__ CSx,
                                                             const pfa::u4 *__restrict__ fr, float out_scale)
{
    constexpr int W = kCorrWavesX;
    constexpr int kPad = W + 1;
    __shared__ pfa::u4 s_c[pfa::kUnits];
    __shared__ float s_stage[1024 * kPad];
    __shared__ pfa::u4 s_g[W * 2 * kXBuf];  // two block spectra per wave
    __shared__ long long s_item;
    const int tid = threadIdx.x;
    // the wave index is uniform: item indices, block addresses and exponents stay scalar
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4, c = l & 15;
    pfa::InvB B;
    pfa::load_inv(B, fr, l);
    const int n_req = H->n_req;
    const int pt = H->corr_pt;
    const long long total = H->total[kStCorr];
    const long long *pst = pre + (long long)kStCorr * (n_req + 1);
    const pfa::u4 zero4 = {0u, 0u, 0u, 0u};
    bool first = true;
    for (;;) {
        const long long it = next_item(H, kStCorr, total, &s_item, first);
        if (it < 0) break;
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        const long long local = it - pst[r];
        const int ptile = (int)(local % d.n_ptiles), chunk = (int)(local / d.n_ptiles);
        const int item = chunk * W + w;
        const bool active = item < d.n_items;
        const int spc = d.spc;
        const int k = item / spc, s = item - k * spc;
        const long long v0 = d.vec_off + (long long)k * d.Nnc * spc + s;
        for (int pp = 0; pp < pt; ++pp) {
            const int pi = ptile * pt + pp;
            if (pi >= d.n_prn) break;
            __syncthreads();  // the previous PRN's reads of s_c and s_stage are done
            for (int i = tid; i < pfa::kUnits; i += 64 * W) s_c[i] = CSx[(long long)d.prns[pi] * pfa::kUnits + i];
            __syncthreads();
            float acc[2][3][4];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int h = 0; h < 3; ++h)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[u][h][q] = 0.f;
            if (active) {
                // Block b + 1's spectrum is copied from HBM into the wave's other
                // LDS buffer (direct-to-LDS loads, no registers) while block b's
                // transform runs.
                pfa::u4 *bufs = s_g + w * 2 * kXBuf;
                auto spectrum = [&](int b) { return Gx + (v0 + (long long)b * spc) * pfa::kUnits; };
                auto product = [&](const pfa::u4 *cur, pfa::u4 (&a1)[3][2]) {
#pragma unroll
                    for (int t = 0; t < 3; ++t)
#pragma unroll
                        for (int ss = 0; ss < 2; ++ss) {
                            const int unit = t < 2 ? (2 * t + ss) * 64 + l : pfa::kTailUnit + 4 * ss + g;
                            const bool has = t < 2 || c == 0;
                            a1[t][ss] = has ? cmul_conj_frag(cur[unit], s_c[unit]) : zero4;
                        }
                };
                // |.|^2 into the sums, which are kept in units of 2^(2 e_ref), e_ref
                // the exponent of the last block added: a block at e_ref adds its
                // power unscaled.  Column 32 has its real part in lane c = 0 and its
                // imaginary part in lane c = 1: each lane sums its own square and
                // the two are added at the end.
                auto power_unit = [&](const pfa::f4 (&o)[2][5]) {
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
#pragma unroll
                        for (int h = 0; h < 2; ++h)
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const float yr = o[u][2 * h][q], yi = o[u][2 * h + 1][q];
                                acc[u][h][q] = fmaf(yi, yi, fmaf(yr, yr, acc[u][h][q]));
                            }
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc[u][2][q] = fmaf(o[u][4][q], o[u][4][q], acc[u][2][q]);
                    }
                };
                if constexpr (PAIRS) {
                    // Navigation-bit hypotheses: blocks 2i and 2i + 1 combined
                    // coherently with both relative signs, max over the two;
                    // R_a +- R_b is the inverse transform of (G_a +- G_b) conj(C).
                    // The + hypothesis's power waits in the wave's part of s_stage,
                    // which is free until the item's grid write.
                    float *pplus = s_stage + w * 1024;
                    for (int b = 0; b < d.Nnc; b += 2) {
                        stage_spectrum(spectrum(b), bufs, l);
                        stage_spectrum(spectrum(b + 1), bufs + kXBuf, l);
                        const int ea = E[v0 + (long long)b * spc], eb = E[v0 + (long long)(b + 1) * spc];
                        const int e = max(ea, eb);
                        // 2^(ea - e) and 2^(eb - e) in FP16 (exact; below 2^-24 they vanish,
                        // as that block's contribution does at FP16 precision)
                        const float fa32 = ldexpf(1.f, ea - e), fb32 = ldexpf(1.f, eb - e);
                        const __half2 fa = __floats2half2_rn(fa32, fa32), fb = __floats2half2_rn(fb32, fb32);
                        const float sc = ldexpf(1.f, 2 * e);
                        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // both blocks are in LDS
#pragma unroll
                        for (int hyp = 0; hyp < 2; ++hyp) {
                            pfa::u4 a1[3][2];
#pragma unroll
                            for (int t = 0; t < 3; ++t)
#pragma unroll
                                for (int ss = 0; ss < 2; ++ss) {
                                    const int unit = t < 2 ? (2 * t + ss) * 64 + l : pfa::kTailUnit + 4 * ss + g;
                                    if (t < 2 || c == 0) {
                                        const pfa::u4 ga = bufs[unit], gb = bufs[kXBuf + unit];
                                        pfa::u4 gs;
#pragma unroll
                                        for (int q = 0; q < 4; ++q) {
                                            const __half2 x = __hmul2(bits_h2(ga[q]), fa), y = __hmul2(bits_h2(gb[q]), fb);
                                            gs[q] = h2_bits(hyp == 0 ? __hadd2(x, y) : __hsub2(x, y));
                                        }
                                        a1[t][ss] = cmul_conj_frag(gs, s_c[unit]);
                                    } else {
                                        a1[t][ss] = zero4;
                                    }
                                }
                            pfa::f4 o[2][5];
                            pfa::inverse(a1, B, o);
#pragma unroll
                            for (int u = 0; u < 2; ++u)
#pragma unroll
                                for (int h = 0; h < 3; ++h)
#pragma unroll
                                    for (int q = 0; q < 4; ++q) {
                                        float pw;
                                        if (h < 2) {
                                            const float yr = o[u][2 * h][q], yi = o[u][2 * h + 1][q];
                                            pw = fmaf(yr, yr, yi * yi);
                                        } else {  // column 32: re in lane c = 0, im in lane c = 1
                                            const float t2 = o[u][4][q] * o[u][4][q];
                                            pw = t2 + from_next_lane(t2);
                                        }
                                        const int n1 = 16 * u + 4 * g + q, n2 = 16 * h + c;
                                        if (n1 < pfa::kN1 && n2 < pfa::kN2) {
                                            float *slot = pplus + pfa::time_index(n1, n2);
                                            if (hyp == 0)
                                                *slot = pw;
                                            else
                                                acc[u][h][q] = fmaf(fmaxf(*slot, pw), sc, acc[u][h][q]);
                                        }
                                    }
                            lds_fence();
                        }
                    }
                } else {
                stage_spectrum(spectrum(0), bufs, l);
                int e_cur = E[v0], e_ref = e_cur, e_max = e_cur;
                for (int b = 0; b < d.Nnc; ++b) {
                    pfa::u4 a1[3][2];
                    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // block b is in LDS
                    product(bufs + (b & 1) * kXBuf, a1);
                    int e_next = 0;
                    if (b + 1 < d.Nnc) {
                        // the other buffer was last read by block b - 1's product
                        stage_spectrum(spectrum(b + 1), bufs + ((b + 1) & 1) * kXBuf, l);
                        e_next = E[v0 + (long long)(b + 1) * spc];
                    }
                    pfa::f4 o[2][5];
                    pfa::inverse(a1, B, o);
                    if (e_cur != e_ref) {
                        // Another block exponent: bring the sums to it (a power of
                        // two, exact).  A block's power is below 2^30 in its own
                        // units and Nnc < 2^17, so the sums stay below 2^47 in the
                        // units of the largest exponent so far, e_max; scaling to
                        // e_cur >= e_max - 30 multiplies them by at most 2^60 over
                        // that, which stays finite.  A block more than 2^30 below
                        // e_max adds less than 2^-60 of that block's power and is
                        // dropped (an all-zero block has exponent 0 and power 0).
                        if (e_cur >= e_max - 30) {
                            const float f = ldexpf(1.f, 2 * (e_ref - e_cur));
#pragma unroll
                            for (int u = 0; u < 2; ++u)
#pragma unroll
                                for (int h = 0; h < 3; ++h)
#pragma unroll
                                    for (int q = 0; q < 4; ++q) acc[u][h][q] *= f;
                            e_ref = e_cur;
                            e_max = max(e_max, e_cur);
                        } else {
#pragma unroll
                            for (int u = 0; u < 2; ++u)
#pragma unroll
                                for (int v = 0; v < 5; ++v) o[u][v] = pfa::f4{0.f, 0.f, 0.f, 0.f};
                        }
                    }
                    power_unit(o);
                    e_cur = e_next;
                }
                // column 32: lane c = 0 adds lane c = 1's imaginary part; then
                // the sums in absolute units
                const float f = ldexpf(1.f, 2 * e_ref);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int q = 0; q < 4; ++q) acc[u][2][q] += from_next_lane(acc[u][2][q]);
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int h = 0; h < 3; ++h)
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc[u][h][q] *= f;
                }
            }
            __syncthreads();  // every wave is done with s_stage (the pair hypotheses use it)
            if (active) {
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int h = 0; h < 3; ++h)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int n1 = 16 * u + 4 * g + q, n2 = 16 * h + c;
                            if (n1 < pfa::kN1 && n2 < pfa::kN2)
                                s_stage[pfa::time_index(n1, n2) * kPad + w] = acc[u][h][q] * out_scale;
                        }
            }
            __syncthreads();
            write_rows<W>(s_stage, d, pi, chunk, tid, d.acc != 0);
        }
    }
}

// ===========================================================================
// Frequency-domain Doppler (exact-length contexts, option doppler_fd).  The
// carrier is removed once per block at the base frequency f_if + lo by an
// exact exponential (64-bit integer phase, FP32 sin/cos; phase zero at the block start,
// which leaves |R|^2 unchanged), and one zero-padded DFT of length
// M = P T_coh N = A * 1023 serves every Doppler bin: bin k's folded block has
// the N-point spectrum F^[q] = Y_M[P T_coh q + k kappa] (folding T_coh
// milliseconds keeps every (P T_coh)-th bin of the long spectrum, and the
// residual carrier k*step shifts it by k*kappa bins).  The one-chip boxcar
// multiplies by H[q] = sum_{t<spc} e^(2 pi i t q / N), and the polyphase
// spectra follow from
//   G_s[j] = (1/spc) e^(2 pi i s j / N) sum_{r<spc} B^[j + 1023 r] e^(2 pi i s r / spc).
// The long DFT is a prime-factor transform, A x 1023 (coprime): 1023-point
// DFTs on the matrix cores over the inner index, then A-point DFTs in FP32.
// Input map n = (1023 n1 + A m) mod M; the final spectrum is kept as
// X[k1][a * 33 + b'] with k1 = k mod A and (a, b') = (k mod 31, k mod 33).
// ===========================================================================

// Per (block, residue) maxima of max(|re|, |im|) of the final long spectrum
// (float bits; non-negative, so they order as unsigned integers), after the
// request's two spectra in the long-DFT buffer.
__device__ __forceinline__ uint32_t *fd_rowmax(const float2 *FD, const ReqDesc &d)
{
    return (uint32_t *)(FD + d.fd_off + 2LL * d.Nnc * d.fd_A * kCodeLen);
}

// First pass: one wave per (request, block, n1): the 1023-point DFT over m of
// the base-wiped samples y[(1023 n1 + A m) mod M] (zero past the block),
// scaled by its l1 exponent; written in FP32 times 2^e as Z[b][n1][a*33 + b'].
__global__ __launch_bounds__(256) void k_fd_pass1(const ReqDesc *__restrict__ R, const BatchHdr *H,
                                                  const long long *pre, const pfa::u4 *__restrict__ fr,
                                                  float2 *FD)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    pfa::FwdB B;
    pfa::load_fwd(B, fr, l);
    const int n_req = H->n_req;
    const long long total = H->total[kStFdA];
    const long long *pst = pre + (long long)kStFdA * (n_req + 1);
    for (long long it = (long long)blockIdx.x * 4 + w; it < total; it += (long long)gridDim.x * 4) {
        const int r = find_req(pst, n_req, uniform64(it));
        const ReqDesc &d = R[r];
        const long long local = it - pst[r];
        const int A = d.fd_A, b = (int)(local / A), n1 = (int)(local % A);
        const long long M = (long long)A * kCodeLen, L = (long long)d.Tc * d.N;
        const long long base = (long long)(d.b0 + b) * L;
        if (n1 < d.fd_PTc && l == 0) fd_rowmax(FD, d)[b * d.fd_PTc + n1] = 0u;  // for the second pass
        float vr[3][2][4], vi[3][2][4];
        float nrm = 0.f;
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i31 = 16 * s + 4 * g + j, i33 = 16 * t + c;
                    float yr = 0.f, yi = 0.f;
                    if (i31 < pfa::kN1 && i33 < pfa::kN2) {
                        const long long n = (1023LL * n1 + (long long)A * pfa::time_index(i31, i33)) % M;
                        if (n < L) {
                            int xr, xi;
                            load_sample(d.samples, d.fmt, base + n, xr, xi);
                            // carrier phase of in-block sample n: the top 24 bits of the
                            // 64-bit accumulator n * fd_dphase, exact as a float in [0, 1)
                            const unsigned long long ph = (unsigned long long)n * d.fd_dphase;
                            const float cyc = (float)(uint32_t)(ph >> 40) * 0x1p-24f;
                            float sn, cs;
                            sincospif(2.f * cyc, &sn, &cs);
                            yr = (float)xr * cs + (float)xi * sn;  // x e^(-i theta)
                            yi = (float)xi * cs - (float)xr * sn;
                        }
                    }
                    vr[t][s][j] = yr;
                    vi[t][s][j] = yi;
                    nrm += fabsf(yr) + fabsf(yi);
                }
        const int e = l1_exponent(wave_sum(nrm));
        const float f = ldexpf(1.f, -e), fo = ldexpf(1.f, e);
        pfa::u4 a1[3][2];
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int s = 0; s < 2; ++s)
                a1[t][s] = pfa::u4{pfa::pack2(vr[t][s][0] * f, vr[t][s][1] * f), pfa::pack2(vr[t][s][2] * f, vr[t][s][3] * f),
                                   pfa::pack2(vi[t][s][0] * f, vi[t][s][1] * f), pfa::pack2(vi[t][s][2] * f, vi[t][s][3] * f)};
        pfa::f4 o[2][6];
        pfa::forward(a1, B, o);
        float *dst = (float *)(FD + d.fd_off + (long long)(b * A + n1) * kCodeLen);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 6; ++v)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int a = 16 * u + 4 * g + q, bb = 16 * (v >> 1) + c;
                    if (a < pfa::kN1 && bb < pfa::kN2) dst[2 * (a * pfa::kN2 + bb) + (v & 1)] = o[u][v][q] * fo;
                }
    }
}

// Second pass: one workgroup per (request, block, 8 columns sigma): the
// columns' A x 8 values in LDS, the A-point DFTs over n1 in FP32,
//   Y_M[i] = sum_n1 Z[b][n1][sigma] e^(-2 pi i n1 k1 / A),
// i = (k1 crt1 + k2 crt2) mod M, k2 the frequency of sigma; stored by residue,
// Yt[b][i mod P T_coh][i div P T_coh] (i mod P T_coh = k1 mod P T_coh, since
// crt1 = 1 mod A and crt2 = 0 mod A), so that a Doppler bin's folded spectrum
// (every (P T_coh)-th bin from an offset) is a contiguous circular run of one
// row; and each row's max(|re|, |im|).  For A >= 4 a thread computes the four
// outputs k1 + m A/4 from each LDS value: their weights differ by (-i)^(n1 m).
__device__ __forceinline__ float2 quarter_turns(float2 t, int q)  // t (-i)^q, q in 0..3
{
    return q == 0 ? t : q == 1 ? make_float2(t.y, -t.x) : q == 2 ? make_float2(-t.x, -t.y) : make_float2(-t.y, t.x);
}

__global__ __launch_bounds__(256) void k_fd_pass2(const ReqDesc *__restrict__ R, const BatchHdr *H,
                                                  const long long *pre, float2 *FD)
{
    __shared__ float2 s_w[256];  // e^(-2 pi i m / 256); A divides 256
    __shared__ float2 s_z[256 * kFdCols];
    __shared__ uint32_t s_max[256];
    for (int m = threadIdx.x; m < 256; m += 256) {
        float sn, cs;
        sincospif((float)m / 128.f, &sn, &cs);
        s_w[m] = make_float2(cs, -sn);
    }
    const int n_req = H->n_req;
    const long long total = H->total[kStFdB];
    const long long *pst = pre + (long long)kStFdB * (n_req + 1);
    constexpr int kChunks = (kCodeLen + kFdCols - 1) / kFdCols;
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        const long long local = it - pst[r];
        const int A = d.fd_A, PTc = d.fd_PTc;
        const int b = (int)(local / kChunks), sig0 = (int)(local % kChunks) * kFdCols;
        const int ncol = min(kFdCols, kCodeLen - sig0);
        const long long M = (long long)A * kCodeLen;
        const int N = (int)(M / PTc);
        const float2 *z = FD + d.fd_off + (long long)b * A * kCodeLen + sig0;
        __syncthreads();  // twiddles staged; the previous item's reads of s_z and s_max are done
        for (int i = threadIdx.x; i < A * kFdCols; i += 256) {
            const int n1 = i / kFdCols, cc = i % kFdCols;
            s_z[i] = cc < ncol ? z[(long long)n1 * kCodeLen + cc] : make_float2(0.f, 0.f);
        }
        if (threadIdx.x < PTc) s_max[threadIdx.x] = 0u;
        __syncthreads();
        const int step = 256 / A;
        float2 *yt = FD + d.fd_off + (long long)d.Nnc * M + (long long)b * M;
        auto emit = [&](int k1, int cc, float ar, float ai) {
            const int sigma = sig0 + cc;
            const int k2 = pfa::freq_index(sigma / pfa::kN2, sigma % pfa::kN2);
            const long long i = ((long long)k1 * d.fd_crt1 + (long long)k2 * d.fd_crt2) % M;
            yt[(i % PTc) * N + i / PTc] = make_float2(ar, ai);
            atomicMax(&s_max[k1 % PTc], __float_as_uint(fmaxf(fabsf(ar), fabsf(ai))));
        };
        if (A >= 4) {
            const int qa = A / 4;
            for (int o = threadIdx.x; o < qa * ncol; o += 256) {
                const int k1 = o / ncol, cc = o % ncol;
                float2 acc[4] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
                for (int p4 = 0; p4 < A; p4 += 4) {
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int n1 = p4 + rr;
                        const float2 v = s_z[n1 * kFdCols + cc];
                        const float2 wv = s_w[(n1 * k1 * step) & 255];
                        const float2 t = make_float2(v.x * wv.x - v.y * wv.y, v.x * wv.y + v.y * wv.x);
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            const float2 u = quarter_turns(t, (rr * m) & 3);
                            acc[m].x += u.x;
                            acc[m].y += u.y;
                        }
                    }
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) emit(k1 + m * qa, cc, acc[m].x, acc[m].y);
            }
        } else {
            for (int o = threadIdx.x; o < A * ncol; o += 256) {
                const int k1 = o / ncol, cc = o % ncol;
                float ar = 0.f, ai = 0.f;
                for (int n1 = 0; n1 < A; ++n1) {
                    const float2 v = s_z[n1 * kFdCols + cc];
                    const float2 wv = s_w[(n1 * k1 * step) & 255];
                    ar = fmaf(v.x, wv.x, fmaf(-v.y, wv.y, ar));
                    ai = fmaf(v.x, wv.y, fmaf(v.y, wv.x, ai));
                }
                emit(k1, cc, ar, ai);
            }
        }
        __syncthreads();
        if (threadIdx.x < PTc) atomicMax(fd_rowmax(FD, d) + b * PTc + threadIdx.x, s_max[threadIdx.x]);
    }
}

// In-register inverse DFT of S points, u_s = sum_r v_r e^(2 pi i s r / S):
// radix 2, decimation in frequency, then the bit-reversal permutation.  tw16[m]
// = e^(2 pi i m / 16).
template <int S>
__device__ __forceinline__ void idft_small(float2 (&v)[kMaxSpc], const float2 *tw16)
{
#pragma unroll
    for (int half = S / 2; half >= 1; half /= 2) {
#pragma unroll
        for (int i0 = 0; i0 < S; i0 += 2 * half)
#pragma unroll
            for (int j = 0; j < half; ++j) {
                const float2 a = v[i0 + j], b = v[i0 + j + half];
                const float2 w = tw16[j * (8 / half)];  // e^(2 pi i j / (2 half))
                const float2 d = make_float2(a.x - b.x, a.y - b.y);
                v[i0 + j] = make_float2(a.x + b.x, a.y + b.y);
                v[i0 + j + half] = make_float2(d.x * w.x - d.y * w.y, d.x * w.y + d.y * w.x);
            }
    }
    float2 t[kMaxSpc];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        int rv = 0;
#pragma unroll
        for (int k = 1, m = S >> 1; k < S; k <<= 1, m >>= 1)
            if (i & k) rv |= m;
        t[rv] = v[i];
    }
#pragma unroll
    for (int i = 0; i < S; ++i) v[i] = t[i];
}

// Synthesis: one workgroup (512 threads) per (request, Doppler bin, block),
// the items of k_box.  For each frequency j < 1023 (one thread, reading the
// long spectrum contiguously) the spc values F^[j + 1023 r] give the
// polyphase spectra of the fold,
//   F_s'[j] = (1/spc) e^(2 pi i s' j / N) sum_r F^[j + 1023 r] e^(2 pi i s' r / spc),
// and the one-chip boxcar (g_s[m] = sum_{s'>=s} f_s'[m] + sum_{s'<s} f_s'[m+1])
// is G_s[j] = T + (e^(2 pi i j / 1023) - 1) P_s with T = sum_s' F_s' and
// P_s = sum_{s'<s} F_s'.  The spc spectra are staged in LDS in the stored
// fragment layout and written out whole.  |G_s| <= spc max |F^| sets the
// exponent e of the item's vectors (from the row maximum of the second pass).
constexpr int kSynthThreads = 512;
__global__ __launch_bounds__(kSynthThreads) void k_fd_synth(const ReqDesc *__restrict__ R, BatchHdr *H,
                                                            const long long *pre, const float2 *FD, pfa::u4 *Gx,
                                                            int *E)
{
    __shared__ pfa::u4 s_out[kMaxSpc * pfa::kUnits];
    __shared__ float2 s_tw16[16];
    __shared__ long long s_item;
    const int n_req = H->n_req;
    const long long total = H->total[kStBox];
    const long long *pst = pre + (long long)kStBox * (n_req + 1);
    const int tid = threadIdx.x;
    if (tid < 16) {
        float sn, cs;
        sincospif((float)tid / 8.f, &sn, &cs);
        s_tw16[tid] = make_float2(cs, sn);
    }
    bool first = true;
    for (;;) {
        const long long it = next_item(H, kStBox, total, &s_item, first);
        if (it < 0) break;
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        const int kb = (int)(it - pst[r]);
        const int k = kb / d.Nnc, b = kb - k * d.Nnc;
        const int N = d.N, spc = d.spc, A = d.fd_A, PTc = d.fd_PTc;
        const long long M = (long long)A * kCodeLen;
        const long long shift = ((long long)k * d.fd_kappa) % M;
        // F^[q] = Y_M[(q P T_coh + k kappa) mod M] = Yt[rho][(q + delta) mod N] with
        // k kappa = delta P T_coh + rho
        const int rho = (int)(shift % PTc), delta = (int)(shift / PTc);
        const float2 *row = FD + d.fd_off + (long long)d.Nnc * M + (long long)b * M + (long long)rho * N;
        const float mx = __uint_as_float(fd_rowmax(FD, d)[b * PTc + rho]) * 1.41421357f * (float)spc;
        int e = 0;
        if (mx > 0.f) {
            int x;
            (void)frexpf(mx * (1.f + 0x1p-10f), &x);  // mx' < 2^x
            e = x - kL1Exp;
        }
        const float scale = ldexpf(1.f, -e) / (float)spc;
        __syncthreads();  // tables staged; the previous item's copy out of s_out is done
        uint16_t *o16 = (uint16_t *)s_out;
        for (int j = tid; j < kCodeLen; j += kSynthThreads) {
            float2 v[kMaxSpc];
#pragma unroll
            for (int rr = 0; rr < kMaxSpc; ++rr) {
                int qq = j + kCodeLen * rr + delta;
                if (qq >= N) qq -= N;
                v[rr] = rr < spc ? row[qq] : make_float2(0.f, 0.f);
            }
            switch (spc) {
            case 2: idft_small<2>(v, s_tw16); break;
            case 4: idft_small<4>(v, s_tw16); break;
            case 8: idft_small<8>(v, s_tw16); break;
            case 16: idft_small<16>(v, s_tw16); break;
            default: break;  // spc 1: the value itself
            }
            float s1, c1, s2, c2;
            sincospif(2.f * (float)j / (float)N, &s1, &c1);         // e^(2 pi i j / N)
            sincospif(2.f * (float)j / (float)kCodeLen, &s2, &c2);  // e^(2 pi i j / 1023)
            float2 wv = make_float2(1.f, 0.f), tsum = make_float2(0.f, 0.f);
#pragma unroll
            for (int sp = 0; sp < kMaxSpc; ++sp) {
                if (sp < spc) {
                    const float2 f = make_float2((v[sp].x * wv.x - v[sp].y * wv.y) * scale,
                                                 (v[sp].x * wv.y + v[sp].y * wv.x) * scale);
                    v[sp] = f;
                    tsum.x += f.x;
                    tsum.y += f.y;
                    wv = make_float2(wv.x * c1 - wv.y * s1, wv.x * s1 + wv.y * c1);
                }
            }
            // fragment position of frequency j: (a, b') = (j mod 31, j mod 33)
            const int a = j % pfa::kN1, bb = j % pfa::kN2;
            const int t = bb >> 4, cc = bb & 15, s31 = a >> 4, gg = (a >> 2) & 3, jj = a & 3;
            const int unit = t < 2 ? (2 * t + s31) * 64 + 16 * gg + cc : pfa::kTailUnit + 4 * s31 + gg;
            const float2 wm1 = make_float2(c2 - 1.f, s2);
            float2 pre_s = make_float2(0.f, 0.f);
#pragma unroll
            for (int ss = 0; ss < kMaxSpc; ++ss) {
                if (ss < spc) {
                    const float gr = tsum.x + wm1.x * pre_s.x - wm1.y * pre_s.y;
                    const float gi = tsum.y + wm1.x * pre_s.y + wm1.y * pre_s.x;
                    uint16_t *u16 = o16 + ((long long)ss * pfa::kUnits + unit) * 8;
                    u16[jj] = __builtin_bit_cast(uint16_t, (_Float16)gr);
                    u16[4 + jj] = __builtin_bit_cast(uint16_t, (_Float16)gi);
                    if (a == pfa::kN1 - 1) {  // the unit's padding slot a = 31 (every other slot is written)
                        u16[3] = 0;
                        u16[7] = 0;
                    }
                    pre_s.x += v[ss].x;
                    pre_s.y += v[ss].y;
                }
            }
        }
        __syncthreads();
        const long long vec0 = d.vec_off + (long long)kb * spc;
        for (int i = tid; i < spc * pfa::kUnits; i += kSynthThreads) Gx[vec0 * pfa::kUnits + i] = s_out[i];
        if (tid < spc) E[vec0 + tid] = e;
    }
}

// ===========================================================================
// General sample rates: fs a whole number of kHz that is not k * 1.023 MHz
// (k <= 16), so the replica has no whole number of samples per chip and the
// polyphase form does not apply.  The length-N circular correlation of each
// folded block is done on zero-padded transforms of length M = 2^ceil(log2
// 2N): the block f at [0, N), the replica over two code periods cc[j] =
// c[j mod N] at [0, 2N), and
//   R[tau] = sum_n f[n] c[(n - tau) mod N] = IDFT_M(DFT_M(f) conj(DFT_M(cc)))[M - N + tau] / M
// (no wrap-around because M >= 2N).  When N is a power of two, M = N: the
// same formula is then the N-point circular correlation itself (cc is one
// period on [0, M)).  FP32 throughout, in every context
// precision.  Each transform of P = min(M, 16384) points runs in one
// workgroup's LDS; for M = 32768 the even and odd bins are two 16384-point
// transforms:
//   X[2k] = DFT_P(x[j] + x[j + P])[k],  X[2k + 1] = DFT_P((x[j] - x[j + P]) W_M^j)[k],
// and the inverse's upper half (the only outputs needed, as N <= M/2) is
//   out[P + k] = A[k] - W_M^-k B[k],  A = IDFT_P(Z even bins), B = IDFT_P(Z odd bins).
// P <= 8192: in-place radix-8 passes and one radix-2 or 4 pass in a
// 1024-thread workgroup, decimation in frequency forward (natural order in,
// digit-reversed out) and the exact adjoint inverse (digit-reversed in,
// natural out), so spectra are multiplied in the order they are stored.
// P = 16384: four-step 8 x 2048 transforms (below).
// ===========================================================================

// Radix of the LDS passes (a radix-16 butterfly with its twiddles needs about
// twice the registers, too many beside the correlation's per-lag sums at
// 1024 threads).
constexpr int kGenRad = 8;
// LDS layout of a transform: element i at i + i/32 (one unused slot per 32,
// P + P/32 slots), which spreads the strided accesses of the small-span
// passes over the banks
__device__ __forceinline__ int gx(int i) { return i + (i >> 5); }

// The first octant of the P-point twiddles, s_tw[i] = W_P^i for i < P/8,
// taken from the table of W_32768^i (forward sign).  A pass of span s needs
// W_{8s}^j = W_P^(j P / 8s) with j < s, always in this octant.
__device__ __forceinline__ void gen_load_tw(float2 *s_tw, int P, const float2 *tw)
{
    const int st = kGenTwLen / P;
    for (int i = threadIdx.x; i < P / kGenRad; i += kGenThreads) s_tw[i] = tw[i * st];
}

// w[r] = W^(j r) for r = 1..7 from w1 = W^j: products of at most three
// table values, a few ulp from the correctly rounded twiddles
__device__ __forceinline__ void gen_powers(float2 (&w)[kGenRad], float2 w1)
{
    w[1] = w1;
    w[2] = c_mul(w1, w1);
    w[3] = c_mul(w[2], w1);
    w[4] = c_mul(w[2], w[2]);
    w[5] = c_mul(w[4], w1);
    w[6] = c_mul(w[3], w[3]);
    w[7] = c_mul(w[4], w[3]);
}

// One radix-8 pass of span S over a P-point transform (both powers of two,
// compile time), one butterfly per thread-iteration on the 8 values at
// i0 + r S, i0 = 8 (t - j) + j, j = t mod S, in place.  Forward (decimation
// in frequency): 8-point DFT, then output r times W_{8S}^(j r).  Inverse:
// the adjoint, conjugate twiddles first.  In the padded layout
// gx(i0 + r S) = gx(i0) + r S + floor(r S / 32) for every such i0, so only
// gx(i0) is computed.
template <int P, int S, bool INV>
__device__ __forceinline__ void gen_pass(float2 *x, const float2 *s_tw)
{
    constexpr int ts = P / kGenRad / S;
#pragma unroll 1
    for (int t = threadIdx.x; t < P / kGenRad; t += kGenThreads) {
        const int j = t & (S - 1);
        float2 *base = x + gx((t - j) * kGenRad + j);
        float2 v[kGenRad], w[kGenRad];
#pragma unroll
        for (int r = 0; r < kGenRad; ++r) v[r] = base[r * S + ((r * S) >> 5)];
        if constexpr (S > 1) gen_powers(w, s_tw[j * ts]);
        if constexpr (INV) {
            if constexpr (S > 1) {
#pragma unroll
                for (int r = 1; r < kGenRad; ++r) v[r] = c_mulc(v[r], w[r]);
            }
            dft8<true, false, false, 0>(v);
        } else {
            dft8<false, false, false, 0>(v);
            if constexpr (S > 1) {
#pragma unroll
                for (int r = 1; r < kGenRad; ++r) v[r] = c_mul(v[r], w[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < kGenRad; ++r) base[r * S + ((r * S) >> 5)] = v[r];
    }
}

// The last pass of span 1 when P is not a power of 8: DFTs of R = 2 or 4
// consecutive values (no twiddles; gx(i0 + r) = gx(i0) + r, as R <= 4
// values never cross a 32-slot row).
template <int P, int R, bool INV>
__device__ __forceinline__ void gen_tail(float2 *x)
{
    for (int t = threadIdx.x; t < P / R; t += kGenThreads) {
        float2 *base = x + gx(t * R);
        if constexpr (R == 2) {
            const float2 a = base[0], b = base[1];
            base[0] = c_add(a, b);
            base[1] = c_sub(a, b);
        } else {
            float2 v0 = base[0], v1 = base[1], v2 = base[2], v3 = base[3];
            dft4<INV>(v0, v1, v2, v3);
            base[0] = v0;
            base[1] = v1;
            base[2] = v2;
            base[3] = v3;
        }
    }
}

// the factor of P left after its radix-8 passes (1, 2 or 4)
constexpr int gen_tail_radix(int P)
{
    int R = 1;
    while (R * kGenRad <= P) R *= kGenRad;
    return P / R;
}

// forward passes of spans S, S/8, ..., 1 (each followed by a barrier)
template <int P, int S>
__device__ __forceinline__ void gen_fwd_passes(float2 *x, const float2 *s_tw)
{
    if constexpr (S >= 1) {
        gen_pass<P, S, false>(x, s_tw);
        __syncthreads();
        gen_fwd_passes<P, S / kGenRad>(x, s_tw);
    }
}

// inverse passes of spans S, 8S, ..., P/8
template <int P, int S>
__device__ __forceinline__ void gen_inv_passes(float2 *x, const float2 *s_tw)
{
    if constexpr (S <= P / kGenRad) {
        gen_pass<P, S, true>(x, s_tw);
        __syncthreads();
        gen_inv_passes<P, S * kGenRad>(x, s_tw);
    }
}

// P-point forward transform in LDS (natural order in, digit-reversed out):
// radix-8 passes of spans P/8, P/64, ... and a last radix-2 or 4 pass when
// P is not a power of 8.  Callers synchronise before (the data and s_tw are
// written) and after.
template <int P>
__device__ __forceinline__ void gen_forward(float2 *x, const float2 *s_tw)
{
    gen_fwd_passes<P, P / kGenRad>(x, s_tw);
    constexpr int R = gen_tail_radix(P);
    if constexpr (R > 1) {
        gen_tail<P, R, false>(x);
        __syncthreads();
    }
}

// Exact adjoint of gen_forward: digit-reversed in, natural order out,
// unnormalised exp(+2 pi i nk / P).
template <int P>
__device__ __forceinline__ void gen_inverse(float2 *x, const float2 *s_tw)
{
    constexpr int R = gen_tail_radix(P);
    if constexpr (R > 1) {
        gen_tail<P, R, true>(x);
        __syncthreads();
    }
    gen_inv_passes<P, R>(x, s_tw);
}

// The thread index through an empty asm statement, so that the compiler
// does not hoist the per-lag addresses derived from it out of the loops
// (16 lags x 64-bit addresses, held across the transforms, spill).
__device__ __forceinline__ int opaque_tid()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// The general-rate kernels are instantiated per transform length P < 16384
// (LDS sized by P, so smaller transforms share a CU) and launched once for
// each length present in a batch; items of requests with another length are
// skipped.  P = 16384 has kernels of its own (below).

// Code spectra of a general-rate request: item = (request, PRN).
// CC[p][h P + i] = DFT_M(cc)[bin of storage position i of half h].
template <int P>
__global__ __launch_bounds__(kGenThreads) void k_gen_code(const ReqDesc *__restrict__ R, const BatchHdr *H,
                                                          const long long *pre, const uint8_t *codes,
                                                          const float2 *tw, float2 *gen)
{
    __shared__ float2 x[P + P / 32];
    __shared__ float2 s_tw[P / kGenRad];
    const int n_req = H->n_req;
    const long long total = H->total[kStGenC];
    const long long *pst = pre + (long long)kStGenC * (n_req + 1);
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        if (d.gen_P != P) continue;
        const int pi = (int)(it - pst[r]);
        const uint8_t *code = codes + (long long)d.prns[pi] * kCodeLen;
        const int N = d.N, M = d.gen_M;
        const long long fs = (long long)N * 1000;
        float2 *dst = gen + d.gen_c_off + (long long)pi * M;
        // c[j mod N] for j < 2N, else 0
        auto cc = [&](int j) -> float {
            if (j >= 2 * N) return 0.f;
            const long long n = j >= N ? j - N : j;
            return code[(n * 1023000LL / fs) % kCodeLen] ? -1.f : 1.f;
        };
        for (int h = 0; h < M / P; ++h) {
            __syncthreads();  // the previous transform's outputs are read
            if (h == 0) gen_load_tw(s_tw, P, tw);
            for (int j = threadIdx.x; j < P; j += kGenThreads) {
                float2 v;
                if (M == P) {
                    v = make_float2(cc(j), 0.f);
                } else if (h == 0) {
                    v = make_float2(cc(j) + cc(j + P), 0.f);
                } else {
                    const float c = cc(j) - cc(j + P);
                    const float2 w = tw[j];  // W_M^j, M = 32768
                    v = make_float2(c * w.x, c * w.y);
                }
                x[gx(j)] = v;
            }
            __syncthreads();
            gen_forward<P>(x, s_tw);
            for (int j = threadIdx.x; j < P; j += kGenThreads) dst[(long long)h * P + j] = x[gx(j)];
        }
    }
}

// Block spectra of a general-rate request: item = (request, Doppler bin,
// block).  The carrier NCO, first mixing stage and fold of the block (the
// integer arithmetic of the polyphase path), delayed circularly by the
// code-Doppler shift if any, then the zero-padded forward transform.
template <int P>
__global__ __launch_bounds__(kGenThreads) void k_gen_x(const ReqDesc *__restrict__ R, const BatchHdr *H,
                                                       const long long *pre, const uint32_t *lut, const float2 *tw,
                                                       float2 *gen)
{
    __shared__ float2 x[P + P / 32];
    __shared__ float2 s_tw[P / kGenRad];
    __shared__ uint32_t s_lut[1024];
    constexpr int kPer = kGenMaxN / kGenThreads;
    for (int i = threadIdx.x; i < 1024; i += kGenThreads) s_lut[i] = lut[i];
    const int n_req = H->n_req;
    const long long total = H->total[kStGenX];
    const long long *pst = pre + (long long)kStGenX * (n_req + 1);
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        if (d.gen_P != P) continue;
        const long long local = it - pst[r];
        const int k = (int)(local / d.Nnc), b = (int)(local % d.Nnc);
        const int N = d.N, M = d.gen_M;
        const uint32_t D = d.dk[k];
        const int shift = d.cshift ? d.cshift[(long long)k * d.Nnc + b] : 0;
        __syncthreads();  // s_lut staged; the previous item's reads of x and s_tw are done
        gen_load_tw(s_tw, P, tw);
        // the folded block, n = tid + 1024 i (zero at n >= N)
        float2 f[kPer];
        int tid = opaque_tid();
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int n = tid + kGenThreads * i;
            f[i] = make_float2(0.f, 0.f);
            if (n < N) {
                int m = n - shift;
                if (m < 0) m += N;
                const int2 v = wipe_fold_one(d.samples, d.fmt, N, d.Tc, s_lut, D, d.b0 + b, m);
                f[i] = make_float2((float)v.x, (float)v.y);
            }
        }
        float2 *dst = gen + d.gen_x_off + local * M;
        for (int h = 0; h < M / P; ++h) {
            if (h) __syncthreads();  // the previous half's outputs are read
            tid = opaque_tid();
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int n = tid + kGenThreads * i;
                if (n < P) {
                    // N <= P: the block has no samples at n + P; the odd-bin
                    // half takes it times W_M^n
                    float2 v = f[i];
                    if (h == 1) v = c_mul(v, tw[n]);
                    x[gx(n)] = v;
                }
            }
            __syncthreads();
            gen_forward<P>(x, s_tw);
            for (int j = threadIdx.x; j < P; j += kGenThreads) dst[(long long)h * P + j] = x[gx(j)];
        }
    }
}

// One correlation item of length P = M (see k_gen_corr).
template <int P>
__device__ __forceinline__ void gen_corr_item(const ReqDesc &d, int k, int pi, const float2 *tw, const float2 *gen,
                                              float2 *x, float2 *s_tw)
{
    static_assert(P < kGenLds, "the 16384-point transforms have kernels of their own");
    constexpr int kPer = kGenMaxN / kGenThreads;
    constexpr int kFill = 8;  // product values loaded per thread before they are stored
    const int N = d.N;
    const float2 *C = gen + d.gen_c_off + (long long)pi * P;
    // 2^-24 (LUT scale) / P^2 (two unnormalised transforms), an exact power of two
    const float scale = ldexpf(1.f, -24 - 2 * (31 - __clz(P)));
    GNSS_GLOBAL float *row = gmem(d.grid) + ((long long)pi * d.n_dopp + k) * N;
    // fill x with the product of block b's spectrum and the code's; the first
    // loads are issued before the barrier that frees x
    auto product = [&](int b, bool first) {
        const float2 *X = gen + d.gen_x_off + ((long long)k * d.Nnc + b) * P;
        const int tid = opaque_tid();
        for (int j0 = 0; j0 < P; j0 += kFill * kGenThreads) {
            float2 xv[kFill], cv[kFill];
#pragma unroll
            for (int u = 0; u < kFill; ++u) {
                const int j = j0 + u * kGenThreads + tid;
                if (j < P) {
                    xv[u] = X[j];
                    cv[u] = C[j];
                }
            }
            if (j0 == 0) {
                __syncthreads();  // the previous inverse's outputs are read
                if (first) gen_load_tw(s_tw, P, tw);
            }
#pragma unroll
            for (int u = 0; u < kFill; ++u) {
                const int j = j0 + u * kGenThreads + tid;
                if (j < P) x[gx(j)] = c_mulc(xv[u], cv[u]);
            }
        }
        __syncthreads();
    };
    // lag tau is output P - N + tau; the sums in groups of kSumGroup blocks,
    // each group's added to the row by the thread that holds it
    for (int b0 = 0; b0 < d.Nnc; b0 += kSumGroup) {
        float acc[kPer];
#pragma unroll
        for (int i = 0; i < kPer; ++i) acc[i] = 0.f;
        const int b1 = min(d.Nnc, b0 + kSumGroup);
        for (int b = b0; b < b1; ++b) {
            product(b, b == 0);
            gen_inverse<P>(x, s_tw);
            const int tid = opaque_tid();
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int tau = tid + kGenThreads * i;
                if (tau < N) {
                    const float2 o = x[gx(P - N + tau)];
                    acc[i] = fmaf(o.x, o.x, fmaf(o.y, o.y, acc[i]));
                }
            }
        }
        const int tid = opaque_tid();
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int tau = tid + kGenThreads * i;
            if (tau < N) row[tau] = (b0 || d.acc) ? row[tau] + acc[i] * scale : acc[i] * scale;
        }
    }
}

// Correlation of a general-rate request with M = P <= 8192: item =
// (request, Doppler bin, PRN), Doppler-major so that the workgroups running
// together share the block spectra; over the blocks, Z = X conj(CC), the
// inverse transform and |.|^2 of the lags' outputs, summed in block order
// in registers; the grid gets sum |out|^2 2^-24 / M^2.
template <int P>
__global__ __launch_bounds__(kGenThreads) void k_gen_corr(const ReqDesc *__restrict__ R, const BatchHdr *H,
                                                          const long long *pre, const float2 *tw,
                                                          const float2 *gen)
{
    __shared__ float2 x[P + P / 32];
    __shared__ float2 s_tw[P / kGenRad];
    const int n_req = H->n_req;
    const long long total = H->total[kStGenCorr];
    const long long *pst = pre + (long long)kStGenCorr * (n_req + 1);
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        if (d.gen_P != P) continue;
        const long long local = it - pst[r];
        const int k = (int)(local / d.n_prn), pi = (int)(local % d.n_prn);
        gen_corr_item<P>(d, k, pi, tw, gen, x, s_tw);
    }
}

// v W_16^a (forward sign) or v W_16^-a (INV) for a < 8; a is a constant once
// the callers' loops are unrolled
__device__ __forceinline__ float2 twiddle16(float2 v, int a, bool inv)
{
    switch (a) {
    case 0: return v;
    case 1: return inv ? tw<16, 1, true>(v) : tw<16, 1, false>(v);
    case 2: return inv ? tw<16, 2, true>(v) : tw<16, 2, false>(v);
    case 3: return inv ? tw<16, 3, true>(v) : tw<16, 3, false>(v);
    case 4: return inv ? tw<16, 4, true>(v) : tw<16, 4, false>(v);
    case 5: return inv ? tw<16, 5, true>(v) : tw<16, 5, false>(v);
    case 6: return inv ? tw<16, 6, true>(v) : tw<16, 6, false>(v);
    default: return inv ? tw<16, 7, true>(v) : tw<16, 7, false>(v);
    }
}

// a copy the compiler cannot see through (keeps per-column products from
// being hoisted out of loops and held)
__device__ __forceinline__ float2 opaque(float2 v)
{
    asm volatile("" : "+v"(v.x), "+v"(v.y));
    return v;
}

// ---------------------------------------------------------------------------
// P = 16384: four-step transforms, 8 x 2048.  With n = 2048 a + b and
// k = k1 + 8 k2 (a, k1 < 8; b, k2 < 2048)
//   X[k1 + 8 k2] = DFT_2048 over b of ( W_P^(b k1) DFT_8 over a of x[2048 a + b] )[k2]:
// a radix-8 stage across the eight 2048-point rows (in LDS, one column b per
// thread-iteration), then one 2048-point transform per wave (the register
// FFT of the polyphase path, its transposes in the wave's own LDS row).  The
// forward transform's rows end in the 2048-point storage order, so a half
// spectrum is stored as [k1][1024 float4] exactly as that FFT leaves it; the
// inverse is the adjoint (2048-point inverse per row, then conjugate
// twiddles and the inverse radix-8 stage).  Two workgroup barriers per
// transform instead of one per radix pass.
// ---------------------------------------------------------------------------
constexpr int kG16Threads = 512;  // eight waves, one 2048-point row each
constexpr int kG16Cols = kGenLds / 8 / kG16Threads;  // columns b per thread (4)
static_assert(kGenLds == 8 * 2048, "four-step split of the 16384-point transform");

// Forward radix-8 stage: y[k1][b] = W_P^(b k1) sum_a x(2048 a + b) W_8^(a k1)
// for this thread's columns b = tid + 512 j; x(j, a, b) supplies the input;
// wb[j] = W_P^b (g16_bases).
template <typename Src>
__device__ __forceinline__ void g16_fwd_stage(float2 *y, const float2 (&wb)[kG16Cols], Src x)
{
    const int tid = opaque_tid();
#pragma unroll
    for (int j = 0; j < kG16Cols; ++j) {
        const int b = tid + kG16Threads * j;
        float2 v[8], w[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) v[a] = x(j, a, b);
        dft8<false, false, false, 0>(v);
        gen_powers(w, opaque(wb[j]));  // formed here, not hoisted and held
#pragma unroll
        for (int r = 1; r < 8; ++r) v[r] = c_mul(v[r], w[r]);
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) y[k1 * 2048 + b] = v[k1];
        phase_barrier();  // one column at a time (registers)
    }
}

// W_P^b of this thread's columns b, from the table of W_32768^i (loaded once
// per kernel: the stages' column loop would otherwise wait for each); with
// wm, W_M^b for M = 2P = 32768, which gives W_M^(2048 a + b) = W_M^b W_16^a.
__device__ __forceinline__ void g16_bases(float2 (&wb)[kG16Cols], float2 (&wm)[kG16Cols], const float2 *twg)
{
#pragma unroll
    for (int j = 0; j < kG16Cols; ++j) {
        wb[j] = twg[2 * (threadIdx.x + kG16Threads * j)];
        wm[j] = twg[threadIdx.x + kG16Threads * j];
    }
}

// Wave k1 transforms row k1 of y (natural order) and stores the storage-order
// result at dst[k1][1024 float4].  The row is the wave's transpose buffer.
__device__ __forceinline__ void g16_fwd_rows(float2 *y, const float2 *s_tw, float4 *dst)
{
    const int tid = opaque_tid(), w = tid >> 6, l = tid & 63;
    float2 *row = y + w * 2048;
    float2 v[32];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k2b = 0; k2b < 8; ++k2b) v[8 * u + k2b] = row[l + 64 * u + 256 * k2b];
    fft2048<false, true>(v, row, s_tw, s_tw + kT1Elems, l);
    float4 *d = dst + w * 1024;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj)
        d[jj * 64 + l] = make_float4(v[2 * jj].x, v[2 * jj].y, v[2 * jj + 1].x, v[2 * jj + 1].y);
}

// Wave k1 forms row k1 of X conj(C) (half spectra in the stored layout),
// transforms it back and leaves the natural-order row in y.  The barrier
// that frees y (the previous stage's reads) is taken inside, after the
// spectra are loaded, so their latency overlaps the wait.
__device__ __forceinline__ void g16_inv_rows(float2 *y, const float2 *s_tw, const float4 *X, const float4 *C)
{
    // an opaque index, so that no address is hoisted out of the callers' loops
    const int tid = opaque_tid(), w = tid >> 6, l = tid & 63;
    float2 *row = y + w * 2048;
    const float4 *xq = X + w * 1024, *cq = C + w * 1024;
    float2 z[32];
    phase_barrier();
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const float4 t = xq[jj * 64 + l], c = cq[jj * 64 + l];
        z[2 * jj] = c_mulc(make_float2(t.x, t.y), make_float2(c.x, c.y));
        z[2 * jj + 1] = c_mulc(make_float2(t.z, t.w), make_float2(c.z, c.w));
    }
    __syncthreads();
    ifft2048<false, true>(z, row, s_tw, s_tw + kT1Elems, l);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k2b = 0; k2b < 8; ++k2b) row[l + 64 * u + 256 * k2b] = z[8 * u + k2b];
}

// Inverse radix-8 stage: out(2048 a + b) = sum_k1 W_8^(-a k1) W_P^(-b k1) y[k1][b]
// for this thread's columns; f(j, a, b, value) receives each output.
template <typename Sink>
__device__ __forceinline__ void g16_inv_stage(const float2 *y, const float2 (&wb)[kG16Cols], Sink f)
{
    const int tid = opaque_tid();
#pragma unroll
    for (int j = 0; j < kG16Cols; ++j) {
        const int b = tid + kG16Threads * j;
        float2 v[8], w[8];
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) v[k1] = y[k1 * 2048 + b];
        gen_powers(w, opaque(wb[j]));  // formed here, not hoisted and held
#pragma unroll
        for (int r = 1; r < 8; ++r) v[r] = c_mulc(v[r], w[r]);
        dft8<true, false, false, 0>(v);
#pragma unroll
        for (int a = 0; a < 8; ++a) f(j, a, b, v[a]);
        phase_barrier();  // one column at a time (registers)
    }
}

// Code spectra, P = 16384 (see k_gen_code).
__global__ __launch_bounds__(kG16Threads) void k_gen_code16(const ReqDesc *__restrict__ R, const BatchHdr *H,
                                                            const long long *pre, const uint8_t *codes,
                                                            const float2 *tw, const float2 *twg, float2 *gen)
{
    constexpr int P = kGenLds;
    __shared__ float2 y[P];
    __shared__ float2 s_tw[kTwElems];
    stage_twiddles(s_tw, tw, threadIdx.x, kG16Threads);
    float2 wb[kG16Cols], wm[kG16Cols];
    g16_bases(wb, wm, twg);
    const int n_req = H->n_req;
    const long long total = H->total[kStGenC];
    const long long *pst = pre + (long long)kStGenC * (n_req + 1);
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        if (d.gen_P != P) continue;
        const int pi = (int)(it - pst[r]);
        const uint8_t *code = codes + (long long)d.prns[pi] * kCodeLen;
        const int N = d.N, M = d.gen_M;
        const long long fs = (long long)N * 1000;
        float2 *dst = gen + d.gen_c_off + (long long)pi * M;
        // c[j mod N] for j < 2N, else 0
        auto cc = [&](int j) -> float {
            if (j >= 2 * N) return 0.f;
            const long long n = j >= N ? j - N : j;
            return code[(n * 1023000LL / fs) % kCodeLen] ? -1.f : 1.f;
        };
        for (int h = 0; h < M / P; ++h) {
            __syncthreads();  // the twiddles are staged; the previous rows are read
            g16_fwd_stage(y, wb, [&](int j, int a, int b) -> float2 {
                const int n = 2048 * a + b;
                if (M == P) return make_float2(cc(n), 0.f);
                if (h == 0) return make_float2(cc(n) + cc(n + P), 0.f);
                // (cc[n] - cc[n + P]) W_M^n, M = 32768: W_M^b W_16^a
                const float c = cc(n) - cc(n + P);
                const float2 w = opaque(wm[j]);
                return twiddle16(make_float2(c * w.x, c * w.y), a, false);
            });
            __syncthreads();
            g16_fwd_rows(y, s_tw, (float4 *)(dst + (long long)h * P));
        }
    }
}

// The wipe-off and fold of this thread's 32 samples n = 2048 a + tid + 512 j
// of block b (zero at n >= N), delayed circularly by shift: the arithmetic
// of wipe_fold_one with the milliseconds outermost, so that the 32 samples'
// loads of one millisecond are in flight together.
template <int FMT>
__device__ __forceinline__ void g16_fold(const ReqDesc &d, int b, uint32_t D, int shift, const uint32_t *s_lut,
                                         int tid, float2 (&f)[kG16Cols][8])
{
    const int N = d.N, Tc = d.Tc;
    int yr[kG16Cols][8], yi[kG16Cols][8], m[kG16Cols][8];
#pragma unroll
    for (int j = 0; j < kG16Cols; ++j)
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int n = 2048 * a + tid + kG16Threads * j;
            int mm = n - shift;
            if (mm < 0) mm += N;
            m[j][a] = n < N ? mm : -1;
            yr[j][a] = 0;
            yi[j][a] = 0;
        }
    for (int c = 0; c < Tc; ++c) {
        const long long base = (long long)((d.b0 + b) * Tc + c) * N;
#pragma unroll
        for (int j = 0; j < kG16Cols; ++j)
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                if (m[j][a] < 0) continue;
                const long long ng = base + m[j][a];
                int xr, xi;
                load_sample(d.samples, FMT, ng, xr, xi);
                const uint32_t ph = (uint32_t)(unsigned long long)ng * D;
                const uint32_t e = s_lut[ph >> 22];
                const int cs = (int)(int16_t)(e & 0xFFFFu), sn = (int)(int16_t)(e >> 16);
                yr[j][a] += xr * cs + xi * sn;
                yi[j][a] += xi * cs - xr * sn;
            }
    }
#pragma unroll
    for (int j = 0; j < kG16Cols; ++j)
#pragma unroll
        for (int a = 0; a < 8; ++a) f[j][a] = make_float2((float)yr[j][a], (float)yi[j][a]);
}

// Block spectra, P = 16384 (see k_gen_x).
__global__ __launch_bounds__(kG16Threads) void k_gen_x16(const ReqDesc *__restrict__ R, const BatchHdr *H,
                                                         const long long *pre, const uint32_t *lut,
                                                         const float2 *tw, const float2 *twg, float2 *gen)
{
    constexpr int P = kGenLds;
    __shared__ float2 y[P];
    __shared__ float2 s_tw[kTwElems];
    __shared__ uint32_t s_lut[1024];
    for (int i = threadIdx.x; i < 1024; i += kG16Threads) s_lut[i] = lut[i];
    stage_twiddles(s_tw, tw, threadIdx.x, kG16Threads);
    float2 wb[kG16Cols], wm[kG16Cols];
    g16_bases(wb, wm, twg);
    const int n_req = H->n_req;
    const long long total = H->total[kStGenX];
    const long long *pst = pre + (long long)kStGenX * (n_req + 1);
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        if (d.gen_P != P) continue;
        const long long local = it - pst[r];
        const int k = (int)(local / d.Nnc), b = (int)(local % d.Nnc);
        const int N = d.N, M = d.gen_M;
        const uint32_t D = d.dk[k];
        const int shift = d.cshift ? d.cshift[(long long)k * d.Nnc + b] : 0;
        __syncthreads();  // s_lut staged
        // the folded block at n = 2048 a + tid + 512 j (zero at n >= N)
        float2 f[kG16Cols][8];
        const int tid = opaque_tid();
        if (d.fmt == GNSS_CPLX_I8)
            g16_fold<GNSS_CPLX_I8>(d, b, D, shift, s_lut, tid, f);
        else if (d.fmt == GNSS_REAL_I8)
            g16_fold<GNSS_REAL_I8>(d, b, D, shift, s_lut, tid, f);
        else
            g16_fold<GNSS_REAL_2BIT_PACKED>(d, b, D, shift, s_lut, tid, f);
        float2 *dst = gen + d.gen_x_off + local * M;
        for (int h = 0; h < M / P; ++h) {
            if (h) __syncthreads();  // the previous half's rows are read
            // N <= P: no samples at n + P; the odd-bin half takes x[n] W_M^n
            g16_fwd_stage(y, wb, [&](int j, int a, int) -> float2 {
                if (h == 0) return f[j][a];
                // f W_M^n, n = 2048 a + b: W_M^b W_16^a
                return twiddle16(c_mul(f[j][a], opaque(wm[j])), a, false);
            });
            __syncthreads();
            g16_fwd_rows(y, s_tw, (float4 *)(dst + (long long)h * P));
        }
    }
}

// Correlation, P = 16384 (see k_gen_corr): item = (request, Doppler bin,
// PRN), Doppler-major; this thread's lags are the outputs n = 2048 a + b_j
// at or above P - N, their sums in registers in groups of kSumGroup blocks
// (for M = 2P with the first half's outputs A beside them).
__global__ __launch_bounds__(kG16Threads) void k_gen_corr16(const ReqDesc *__restrict__ R, const BatchHdr *H,
                                                            const long long *pre, const float2 *tw,
                                                            const float2 *twg, const float2 *gen)
{
    constexpr int P = kGenLds;
    __shared__ float2 y[P];
    __shared__ float2 s_tw[kTwElems];
    stage_twiddles(s_tw, tw, threadIdx.x, kG16Threads);
    float2 wb[kG16Cols], wm[kG16Cols];
    g16_bases(wb, wm, twg);
    const int n_req = H->n_req;
    const long long total = H->total[kStGenCorr];
    const long long *pst = pre + (long long)kStGenCorr * (n_req + 1);
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        if (d.gen_P != P) continue;
        const long long local = it - pst[r];
        const int k = (int)(local / d.n_prn), pi = (int)(local % d.n_prn);
        const int N = d.N, M = d.gen_M;
        const float4 *C = (const float4 *)(gen + d.gen_c_off + (long long)pi * M);
        const float scale = ldexpf(1.f, -24 - 2 * (31 - __clz(M)));
        GNSS_GLOBAL float *row = gmem(d.grid) + ((long long)pi * d.n_dopp + k) * N;
        // the sums in groups of kSumGroup blocks, each group's added to the
        // row by the thread that holds it
        for (int b0 = 0; b0 < d.Nnc; b0 += kSumGroup) {
            float acc[kG16Cols][8];
#pragma unroll
            for (int j = 0; j < kG16Cols; ++j)
#pragma unroll
                for (int a = 0; a < 8; ++a) acc[j][a] = 0.f;
            const int b1 = min(d.Nnc, b0 + kSumGroup);
            for (int b = b0; b < b1; ++b) {
                const float4 *X = (const float4 *)(gen + d.gen_x_off + ((long long)k * d.Nnc + b) * M);
                // (the barrier inside: the twiddles are staged, the previous stage's reads of y done)
                g16_inv_rows(y, s_tw, X, C);
                __syncthreads();
                if (M == P) {
                    // lag tau = n - (P - N)
                    g16_inv_stage(y, wb, [&](int j, int a, int bb, float2 o) {
                        const int n = 2048 * a + bb;
                        if (n >= P - N) acc[j][a] = fmaf(o.x, o.x, fmaf(o.y, o.y, acc[j][a]));
                    });
                } else {
                    // lag tau is output P + kk, kk = n - (P - N): A - W_M^-kk B
                    float2 A[kG16Cols][8];
                    g16_inv_stage(y, wb, [&](int j, int a, int, float2 o) { A[j][a] = o; });
                    g16_inv_rows(y, s_tw, X + P / 2, C + P / 2);
                    __syncthreads();
                    g16_inv_stage(y, wb, [&](int j, int a, int bb, float2 o) {
                        const int n = 2048 * a + bb;
                        if (n >= P - N) {
                            // W_M^-n = conj(W_M^b) W_16^-a
                            const float2 v = c_sub(A[j][a], twiddle16(c_mulc(o, opaque(wm[j])), a, true));
                            acc[j][a] = fmaf(v.x, v.x, fmaf(v.y, v.y, acc[j][a]));
                        }
                    });
                }
            }
            const int tid = opaque_tid();
#pragma unroll
            for (int j = 0; j < kG16Cols; ++j)
#pragma unroll
                for (int a = 0; a < 8; ++a) {
                    const int n = 2048 * a + tid + kG16Threads * j;
                    if (n >= P - N) {
                        GNSS_GLOBAL float *o = row + (n - (P - N));
                        *o = (b0 || d.acc) ? *o + acc[j][a] * scale : acc[j][a] * scale;
                    }
                }
        }
    }
}

// ===========================================================================
// detection: column max over Doppler, argmax, second peak, mean; refinement
// ===========================================================================
// Work item = (request, PRN, block of 256 lags).  Q[tau] = max_k P (lowest k
// on ties), K = that k; part = the block's FP32 sum of P: each column summed
// in row order, then the block's columns in a fixed binary tree, so the mean
// does not depend on scheduling.  The relative error of a sum of positive
// terms is at most (depth of its addition tree) * 2^-24.
__global__ __launch_bounds__(kPeakThreads) void k_colmax(const ReqDesc *__restrict__ R, BatchHdr *H,
                                                         const long long *pre, float *Q, int32_t *K,
                                                         float *part)
{
    __shared__ float red[kPeakThreads];
    const int n_req = H->n_req;
    const long long total = H->total[kStColmax];
    const long long *pst = pre + (long long)kStColmax * (n_req + 1);
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        const long long local = it - pst[r];
        const int p = (int)(local / d.n_tau_blk), blk = (int)(local % d.n_tau_blk);
        const int N = d.N, tau = blk * kPeakThreads + threadIdx.x;
        float colsum = 0.f;
        if (tau < N) {
            const GNSS_GLOBAL float *col = gmem(d.grid) + (long long)p * d.n_dopp * N + tau;
            float best = col[0];
            int kb = 0;
            colsum = best;
            int k = 1;
            // eight rows' loads in flight at a time; max and sum in row order
            for (; k + 8 <= d.n_dopp; k += 8) {
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = col[(long long)(k + j) * N];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    colsum += v[j];
                    if (v[j] > best) {
                        best = v[j];
                        kb = k + j;
                    }
                }
            }
            for (; k < d.n_dopp; ++k) {
                float v = col[(long long)k * N];
                colsum += v;
                if (v > best) {
                    best = v;
                    kb = k;
                }
            }
            Q[d.qk_off + (long long)p * N + tau] = best;
            K[d.qk_off + (long long)p * N + tau] = kb;
        }
        __syncthreads();
        red[threadIdx.x] = colsum;
        __syncthreads();
        for (int st = kPeakThreads / 2; st > 0; st >>= 1) {
            if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[d.part_off + (long long)p * d.n_tau_blk + blk] = red[0];
    }
}

// Work item = (request, PRN): argmax (lowest tau on ties), second peak outside
// +-spc (circular), mean, ratio test.
__global__ __launch_bounds__(kArgThreads) void k_peak(const ReqDesc *__restrict__ R, BatchHdr *H,
                                                       const long long *pre, const float *Q,
                                                       const int32_t *K, const float *part)
{
    __shared__ float sv[kArgThreads];
    __shared__ int st[kArgThreads];
    const int tid = threadIdx.x;
    const int n_req = H->n_req;
    const long long total = H->total[kStPeak];
    const long long *pst = pre + (long long)kStPeak * (n_req + 1);
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        const int p = (int)(it - pst[r]);
        const int N = d.N;
        const float *q = Q + d.qk_off + (long long)p * N;
        float bv = -INFINITY;
        int bt = 0x7fffffff;
        for (int tau = tid; tau < N; tau += kArgThreads) {
            float v = q[tau];
            if (v > bv) {
                bv = v;
                bt = tau;
            }
        }
        __syncthreads();
        sv[tid] = bv;
        st[tid] = bt;
        __syncthreads();
        for (int s = kArgThreads / 2; s > 0; s >>= 1) {
            if (tid < s) {
                float v2 = sv[tid + s];
                int t2 = st[tid + s];
                if (v2 > sv[tid] || (v2 == sv[tid] && t2 < st[tid])) {
                    sv[tid] = v2;
                    st[tid] = t2;
                }
            }
            __syncthreads();
        }
        const float peak = sv[0];
        // a grid with no ordered maximum (all NaN) leaves tau* unset: keep it in range
        const int tstar = (st[0] >= 0 && st[0] < N) ? st[0] : 0;
        __syncthreads();
        float m2 = -INFINITY;
        for (int tau = tid; tau < N; tau += kArgThreads) {
            int dd = abs(tau - tstar);
            dd = min(dd, N - dd);
            if (dd > d.spc) m2 = fmaxf(m2, q[tau]);
        }
        sv[tid] = m2;
        __syncthreads();
        for (int s = kArgThreads / 2; s > 0; s >>= 1) {
            if (tid < s) sv[tid] = fmaxf(sv[tid], sv[tid + s]);
            __syncthreads();
        }
        const float second = sv[0] == -INFINITY ? 0.f : sv[0];
        __syncthreads();
        // the blocks' partial sums in a fixed binary tree (FP32)
        float ps = 0.f;
        for (int i = tid; i < d.n_tau_blk; i += kArgThreads) ps += part[d.part_off + (long long)p * d.n_tau_blk + i];
        sv[tid] = ps;
        __syncthreads();
        for (int s = kArgThreads / 2; s > 0; s >>= 1) {
            if (tid < s) sv[tid] += sv[tid + s];
            __syncthreads();
        }
        if (tid == 0) {
            const float sum = sv[0];
            gnss_peak rr;
            rr.prn = d.prns[p];
            rr.doppler_bin = K[d.qk_off + (long long)p * N + tstar];
            rr.code_phase = tstar;
            rr.peak = peak;
            rr.second = second;
            rr.mean = sum / ((float)d.n_dopp * (float)N);
            rr.ratio = second > 0.f ? peak / second : INFINITY;
            rr.detected = rr.ratio >= d.threshold ? 1 : 0;
            rr.doppler_hz = 0.0;
            rr.code_phase_frac = (double)tstar;
            d.peaks[p] = rr;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double parabola(double ym, double y0, double yp)
{
    double den = ym - 2.0 * y0 + yp;
    if (den == 0.0) return 0.0;
    return 0.5 * (ym - yp) / den;
}

// FP64 sub-bin refinement, one thread per (request, PRN): the only FP64
// arithmetic of a search on the device (the carrier and code-Doppler steps
// are computed on the host; FP64 elsewhere in this file builds the constant
// tables once per context: the carrier LUT, twiddles and exact-length code
// spectra).
__global__ void k_interp(const ReqDesc *__restrict__ R, BatchHdr *H, const long long *pre)
{
    const int n_req = H->n_req;
    const long long total = H->total[kStPeak];
    const long long *pst = pre + (long long)kStPeak * (n_req + 1);
    for (long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (long long)gridDim.x * blockDim.x) {
        const int r = find_req(pst, n_req, it);
        const ReqDesc &d = R[r];
        const int p = (int)(it - pst[r]);
        gnss_peak *pk = d.peaks + p;
        gnss_peak rr = *pk;
        const int N = d.N, nd = d.n_dopp;
        const GNSS_GLOBAL float *Gp = gmem(d.grid) + (long long)p * nd * N;
        const int k = rr.doppler_bin, t = rr.code_phase;
        double y0 = Gp[(long long)k * N + t];
        double dc = parabola(Gp[(long long)k * N + (t - 1 + N) % N], y0, Gp[(long long)k * N + (t + 1) % N]);
        double dd = 0.0;
        if (k > 0 && k < nd - 1) dd = parabola(Gp[(long long)(k - 1) * N + t], y0, Gp[(long long)(k + 1) * N + t]);
        double fk = __dadd_rn(d.lo, __dmul_rn((double)k, d.step));
        pk->doppler_hz = __dadd_rn(fk, __dmul_rn(dd, d.step));
        pk->code_phase_frac = __dadd_rn((double)t, dc);
    }
}

// ===========================================================================
// launch of a whole batch (or of its detection stages only)
// ===========================================================================
template <typename K>
static int occupancy(K kernel, int threads, int n_cu)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return per_cu * n_cu;
}

// Grid of a stage with `work` items: one workgroup per item, or, for a
// persistent launch (or a stage too large for one grid), `cap` workgroups
// that take items from the work counters.  At least one workgroup per XCD.
static unsigned grid_for(long long work, long long cap, bool persistent)
{
    long long g = work;
    if ((persistent && g > cap) || g > 0x7fffffffLL) g = cap;
    if (g < kXcds) g = kXcds;
    return (unsigned)g;
}

// The wipe + fold + boxcar + polyphase stage of a staged batch alone, launched
// exactly as launch_batch launches it (stage entry point).
hipError_t launch_box(const Launch &L, const uint32_t *d_lut, int2 *d_F, int n_cu, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, L.hdr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || L.total[kStBox] == 0) return e;
    static int cap = 0;
    if (!cap) cap = occupancy(k_box, 256, n_cu);
    hipLaunchKernelGGL(k_box, dim3(grid_for(L.total[kStBox], cap, false)), dim3(256), 0, s, L.reqs, L.hdr, L.pre,
                       d_lut, d_F);
    return hipGetLastError();
}

// Frequency-domain Doppler: long DFT of every block (two passes), then the
// block spectra of every (Doppler, block) item; replaces k_box and k_fft_x.
static hipError_t launch_fd(const Launch &L, const Tables &T, void *d_fd, void *d_G, int *d_E, int n_cu,
                            hipStream_t s)
{
    hipError_t e;
    if (L.total[kStFdA] > 0) {
        static int cap = 0;
        if (!cap) cap = occupancy(k_fd_pass1, 256, n_cu);
        hipLaunchKernelGGL(k_fd_pass1, dim3(grid_for((L.total[kStFdA] + 3) / 4, cap, false)), dim3(256), 0, s,
                           L.reqs, L.hdr, L.pre, (const pfa::u4 *)T.frags_x, (float2 *)d_fd);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        static int cap2 = 0;
        if (!cap2) cap2 = occupancy(k_fd_pass2, 256, n_cu);
        hipLaunchKernelGGL(k_fd_pass2, dim3(grid_for(L.total[kStFdB], cap2, false)), dim3(256), 0, s,
                           L.reqs, L.hdr, L.pre, (float2 *)d_fd);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (L.total[kStBox] > 0) {
        static int cap = 0;
        if (!cap) cap = occupancy(k_fd_synth, kSynthThreads, n_cu);
        hipLaunchKernelGGL(k_fd_synth, dim3(grid_for(L.total[kStBox], cap, false)), dim3(kSynthThreads), 0, s,
                           L.reqs, L.hdr, L.pre, (const float2 *)d_fd, (pfa::u4 *)d_G, d_E);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Calls f(std::integral_constant<int, Q>()) for each general-rate transform
// length Q >= P whose bit is set in mask (bit Q, a power of two), in
// increasing order; stops at the first error.
template <int P, typename F>
static hipError_t gen_lengths(unsigned mask, F &f)
{
    if constexpr (P > kGenLds) {
        return hipSuccess;
    } else {
        if (mask & (unsigned)P) {
            const hipError_t e = f(std::integral_constant<int, P>());
            if (e != hipSuccess) return e;
        }
        return gen_lengths<P * 2>(mask, f);
    }
}

hipError_t launch_batch(const Launch &L, const Tables &T, int2 *d_F, void *d_G, float *d_Q, int32_t *d_K,
                        float *d_part, int n_cu, hipStream_t s, hipEvent_t *marks)
{
    const uint32_t *d_lut = T.lut;
    const float2 *d_tw = T.tw;
    const float4 *d_cs = T.cs;
    const bool h = L.precision == GNSS_FP16, x = L.precision == GNSS_FP16_PFA;
    // FP16 modes: packed spectra, then the per-vector exponents
    uint4 *d_Gh = (uint4 *)d_G;
    int *d_E = (int *)((char *)d_G + g_spectra_bytes(L.total[kStVec], L.precision));
    float2 *d_Dc = (float2 *)((char *)d_E + round256((size_t)L.total[kStVec] * 4));  // GNSS_FP16 only
    const float *d_dck = h ? (const float *)((const char *)T.cs_h + kCsHSpecBytes) : nullptr;
    hipError_t e;
    const bool pers = L.persistent != 0;
    auto mark = [&](int i) -> hipError_t { return marks ? hipEventRecord(marks[i], s) : hipSuccess; };
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, L.hdr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = mark(0)) != hipSuccess) return e;
    if (x && L.fd) {
        if ((e = launch_fd(L, T, d_F, d_G, d_E, n_cu, s)) != hipSuccess) return e;
    } else if (L.total[kStBox] > 0) {
        static int cap = 0;
        if (!cap) cap = occupancy(k_box, 256, n_cu);
        hipLaunchKernelGGL(k_box, dim3(grid_for(L.total[kStBox], cap, false)), dim3(256), 0, s, L.reqs,
                           L.hdr, L.pre, d_lut, d_F);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = mark(1)) != hipSuccess) return e;
    if (x && L.fd) {
        // the block spectra are already written
    } else if (L.total[kStVec] > 0 && x) {
        static int cap = 0;
        if (!cap) cap = occupancy(k_fft_x, 256, n_cu);
        hipLaunchKernelGGL(k_fft_x, dim3(grid_for((L.total[kStVec] + 3) / 4, cap, false)), dim3(256), 0, s, d_F,
                           (const pfa::u4 *)T.frags_x, (pfa::u4 *)d_G, d_E, L.hdr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if (L.total[kStVec] > 0 && !h) {
        static int cap = 0;
        if (!cap) cap = occupancy(k_fft_poly, 256, n_cu);
        hipLaunchKernelGGL(k_fft_poly, dim3(grid_for((L.total[kStVec] + 3) / 4, cap, false)), dim3(256), 0,
                           s, d_F, d_tw, (float4 *)d_G, L.hdr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if (L.total[kStVec] > 0) {
        static int cap = 0;
        if (!cap) cap = occupancy(k_fft_poly_h, 256, n_cu);
        hipLaunchKernelGGL(k_fft_poly_h, dim3(grid_for((L.total[kStVec] + 7) / 8, cap, false)), dim3(256), 0,
                           s, d_F, (const hc2 *)T.tw_h, d_Gh, d_E, d_Dc, L.hdr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (L.total[kStGenX] > 0) {  // general rates: code spectra and block spectra
        float2 *d_gen = (float2 *)((char *)d_G + L.gen_off);
        auto spectra = [&](auto pc) -> hipError_t {
            constexpr int P = decltype(pc)::value;
            if constexpr (P == kGenLds) {
                hipLaunchKernelGGL(k_gen_code16, dim3(grid_for(L.total[kStGenC], 65535, false)), dim3(kG16Threads),
                                   0, s, L.reqs, L.hdr, L.pre, T.codes, T.tw, T.tw_gen, d_gen);
                hipError_t e2 = hipGetLastError();
                if (e2 != hipSuccess) return e2;
                hipLaunchKernelGGL(k_gen_x16, dim3(grid_for(L.total[kStGenX], 65535, false)), dim3(kG16Threads), 0,
                                   s, L.reqs, L.hdr, L.pre, d_lut, T.tw, T.tw_gen, d_gen);
                return hipGetLastError();
            } else {
                hipLaunchKernelGGL(k_gen_code<P>, dim3(grid_for(L.total[kStGenC], 65535, false)), dim3(kGenThreads),
                                   0, s, L.reqs, L.hdr, L.pre, T.codes, T.tw_gen, d_gen);
                hipError_t e2 = hipGetLastError();
                if (e2 != hipSuccess) return e2;
                hipLaunchKernelGGL(k_gen_x<P>, dim3(grid_for(L.total[kStGenX], 65535, false)), dim3(kGenThreads), 0,
                                   s, L.reqs, L.hdr, L.pre, d_lut, T.tw_gen, d_gen);
                return hipGetLastError();
            }
        };
        if ((e = gen_lengths<64>(L.gen_pmask, spectra)) != hipSuccess) return e;
    }
    if ((e = mark(2)) != hipSuccess) return e;
    if (L.total[kStGenCorr] > 0) {
        const float2 *d_gen = (const float2 *)((char *)d_G + L.gen_off);
        auto corr = [&](auto pc) -> hipError_t {
            constexpr int P = decltype(pc)::value;
            if constexpr (P == kGenLds)
                hipLaunchKernelGGL(k_gen_corr16, dim3(grid_for(L.total[kStGenCorr], 65535, false)),
                                   dim3(kG16Threads), 0, s, L.reqs, L.hdr, L.pre, T.tw, T.tw_gen, d_gen);
            else
                hipLaunchKernelGGL(k_gen_corr<P>, dim3(grid_for(L.total[kStGenCorr], 65535, false)),
                                   dim3(kGenThreads), 0, s, L.reqs, L.hdr, L.pre, T.tw_gen, d_gen);
            return hipGetLastError();
        };
        if ((e = gen_lengths<64>(L.gen_pmask, corr)) != hipSuccess) return e;
    }
    if (L.total[kStCorr] > 0 && x) {
        // the frequency-domain variant wipes with unit exponentials (no LUT scale 2^12)
        const float osc = ldexpf(1.f, 2 * T.cs_exp - (L.fd ? 0 : 24)) / (float)(kCodeLen * kCodeLen);
        // the pair variant is a separate instantiation: its registers would halve the
        // plain kernel's occupancy
        if (L.nav_pairs) {
            static int cap = 0;
            if (!cap) cap = occupancy(k_corr_x<true>, 64 * kCorrWavesX, n_cu);
            hipLaunchKernelGGL(k_corr_x<true>, dim3(grid_for(L.total[kStCorr], cap, pers)), dim3(64 * kCorrWavesX),
                               0, s, L.reqs, L.hdr, L.pre, (const pfa::u4 *)d_G, d_E, (const pfa::u4 *)T.cs_x,
                               (const pfa::u4 *)T.frags_x, osc);
        } else {
            static int cap = 0;
            if (!cap) cap = occupancy(k_corr_x<false>, 64 * kCorrWavesX, n_cu);
            hipLaunchKernelGGL(k_corr_x<false>, dim3(grid_for(L.total[kStCorr], cap, pers)), dim3(64 * kCorrWavesX),
                               0, s, L.reqs, L.hdr, L.pre, (const pfa::u4 *)d_G, d_E, (const pfa::u4 *)T.cs_x,
                               (const pfa::u4 *)T.frags_x, osc);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if (L.total[kStCorr] > 0 && h) {
        const float osc = ldexpf(1.f, 2 * T.cs_exp - 46);
        if (L.corr_pt == 2) {
            static int cap = 0;
            if (!cap) cap = occupancy(k_corr_h<2>, 64 * kCorrWavesH, n_cu);
            hipLaunchKernelGGL(k_corr_h<2>, dim3(grid_for(L.total[kStCorr], cap, pers)), dim3(64 * kCorrWavesH),
                               0, s, L.reqs, L.hdr, L.pre, d_Gh, d_E, d_Dc, (const uint4 *)T.cs_h, d_dck, (const hc2 *)T.tw_h, osc);
        } else {
            static int cap = 0;
            if (!cap) cap = occupancy(k_corr_h<4>, 64 * kCorrWavesH, n_cu);
            hipLaunchKernelGGL(k_corr_h<4>, dim3(grid_for(L.total[kStCorr], cap, pers)), dim3(64 * kCorrWavesH),
                               0, s, L.reqs, L.hdr, L.pre, d_Gh, d_E, d_Dc, (const uint4 *)T.cs_h, d_dck, (const hc2 *)T.tw_h, osc);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if (L.total[kStCorr] > 0) {
        if (L.corr_pt == 1 && L.corr_w == 4) {
            static int cap = 0;
            if (!cap) cap = occupancy(k_corr<1, 4, 3>, 64 * 4, n_cu);
            hipLaunchKernelGGL((k_corr<1, 4, 3>), dim3(grid_for(L.total[kStCorr], cap, pers)), dim3(64 * 4), 0, s,
                               L.reqs, L.hdr, L.pre, (const float4 *)d_G, d_cs, d_tw);
        } else if (L.corr_pt == 1 && L.corr_w == 6) {
            static int cap = 0;
            if (!cap) cap = occupancy(k_corr<1, 6, 3>, 64 * 6, n_cu);
            hipLaunchKernelGGL((k_corr<1, 6, 3>), dim3(grid_for(L.total[kStCorr], cap, pers)), dim3(64 * 6), 0, s,
                               L.reqs, L.hdr, L.pre, (const float4 *)d_G, d_cs, d_tw);
        } else if (L.corr_pt == 1) {
            static int cap = 0;
            if (!cap) cap = occupancy(k_corr<1, 12, 3>, 64 * 12, n_cu);
            hipLaunchKernelGGL((k_corr<1, 12, 3>), dim3(grid_for(L.total[kStCorr], cap, pers)), dim3(64 * 12), 0, s,
                               L.reqs, L.hdr, L.pre, (const float4 *)d_G, d_cs, d_tw);
        } else if (L.corr_pt == 2) {
            static int cap = 0;
            if (!cap) cap = occupancy(k_corr<2, kCorrWaves, 2>, 64 * kCorrWaves, n_cu);
            hipLaunchKernelGGL((k_corr<2, kCorrWaves, 2>), dim3(grid_for(L.total[kStCorr], cap, pers)),
                               dim3(64 * kCorrWaves), 0, s, L.reqs, L.hdr, L.pre, (const float4 *)d_G, d_cs, d_tw);
        } else {
            static int cap = 0;
            if (!cap) cap = occupancy(k_corr<4, kCorrWaves, 2>, 64 * kCorrWaves, n_cu);
            hipLaunchKernelGGL((k_corr<4, kCorrWaves, 2>), dim3(grid_for(L.total[kStCorr], cap, pers)),
                               dim3(64 * kCorrWaves), 0, s, L.reqs, L.hdr, L.pre, (const float4 *)d_G, d_cs, d_tw);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = mark(3)) != hipSuccess) return e;
    {
        static int cap = 0;
        if (!cap) cap = occupancy(k_colmax, kPeakThreads, n_cu);
        hipLaunchKernelGGL(k_colmax, dim3(grid_for(L.total[kStColmax], cap, false)), dim3(kPeakThreads), 0, s,
                           L.reqs, L.hdr, L.pre, d_Q, d_K, d_part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_peak, dim3(grid_for(L.total[kStPeak], 4LL * n_cu, false)), dim3(kArgThreads), 0,
                           s, L.reqs, L.hdr, L.pre, d_Q, d_K, d_part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const long long ni = (L.total[kStPeak] + 63) / 64;
        hipLaunchKernelGGL(k_interp, dim3((unsigned)(ni < 1 ? 1 : ni > 65536 ? 65536 : ni)), dim3(64), 0, s,
                           L.reqs, L.hdr, L.pre);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return mark(4);
}

// ===========================================================================
// tracking correlators (the tracking channel's carrier and code NCOs, first
// mixing stage and time-domain correlation, Fig. 3): early / prompt / late
// sums per (request, channel, epoch), exact in integers.
// ===========================================================================
constexpr long long kCodeFix = 1023LL << 32;  // one code period, chips * 2^32

// One round of the wave reduce-scatter below: value i pairs with value
// i + H; the lane whose bit O is set keeps the upper one, its partner the
// lower, and each adds the one the other sends.
template <int O, int H>
__device__ __forceinline__ void rs_round(long long (&v)[24], int l)
{
    const bool up = (l & O) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const long long send = up ? v[i] : v[i + H];
        const long long keep = up ? v[i + H] : v[i];
        v[i] = keep + __shfl_xor(send, O);
    }
}

// The workgroup's sums of a pass's kTrackCG x 6 per-thread totals, with one
// pair of barriers for all of them.  Within a wave a reduce-scatter halves
// the values per lane each round (24, 12, 6, 3, padded to 4, 2, 1) while
// the lanes paired across bits 5 .. 1 add them, and the last round over bit
// 0 completes the wave's sum; the lane's bits then name its value.  The
// waves' sums meet in LDS and thread i < 24 adds them.  Returns value i's
// total in thread i (0 in the others); the sums are exact (int64), so their
// order does not matter.
constexpr int kTrackVals = kTrackCG * 6;
static_assert(kTrackVals == 24, "the reduce-scatter rounds are laid out for 24 values");
__device__ __forceinline__ long long block_sums64(const long long (&tot)[kTrackCG][6], long long *s_red)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    long long v[24];
#pragma unroll
    for (int cc = 0; cc < kTrackCG; ++cc)
#pragma unroll
        for (int k = 0; k < 6; ++k) v[cc * 6 + k] = tot[cc][k];
    rs_round<32, 12>(v, l);
    rs_round<16, 6>(v, l);
    rs_round<8, 3>(v, l);
    v[3] = 0;
    rs_round<4, 2>(v, l);
    rs_round<2, 1>(v, l);
    const long long sum = v[0] + __shfl_xor(v[0], 1);
    const int j = ((l & 4) ? 2 : 0) + ((l & 2) ? 1 : 0);  // 3: the padding
    const int idx = ((l & 32) ? 12 : 0) + ((l & 16) ? 6 : 0) + ((l & 8) ? 3 : 0) + j;
    __syncthreads();  // the previous pass's reads of s_red are done
    if ((l & 1) == 0 && j < 3) s_red[w * kTrackVals + idx] = sum;
    __syncthreads();
    long long t = 0;
    if (threadIdx.x < kTrackVals)
        for (int i = 0; i < kTrackThreads / 64; ++i) t += s_red[i * kTrackVals + threadIdx.x];
    return t;
}

// Code replicas of a pass as +-1 bytes with one chip of wrap-around on each
// side: s_sign[c][i] = 1 - 2 code[(i - 1) mod 1023], i in [0, 1024], so the
// early (chip in [0, 1023]) and late (chip in [-1, 1022]) lookups need no wrap.
constexpr int kSignRow = 1028;

// Correlates the epoch's samples of one thread with kTrackCG channels:
// FMT-specialised so the sample decode leaves the loop.  All products fit in
// 24 bits (|x| <= 127, |LUT| <= 4096, |y| < 2^20), so 24-bit multiplies are exact.
template <int FMT>
__device__ __forceinline__ void track_pass(const void *samples, long long n_first, int n_mine,
                                           const uint32_t *s_lut, const int8_t (*s_sign)[kSignRow],
                                           uint32_t (&ph)[kTrackCG], const uint32_t (&dph)[kTrackCG],
                                           unsigned long long (&q)[kTrackCG],
                                           const unsigned long long (&dq)[kTrackCG],
                                           const unsigned long long (&dl)[kTrackCG],
                                           const unsigned long long (&ndl)[kTrackCG], long long (&tot)[kTrackCG][6])
{
    // int32 partial sums over at most 1024 samples: |x y| < 2^20
    for (int j0 = 0; j0 < n_mine; j0 += 1024) {
        int acc[kTrackCG][6];
#pragma unroll
        for (int cc = 0; cc < kTrackCG; ++cc)
#pragma unroll
            for (int k = 0; k < 6; ++k) acc[cc][k] = 0;
        const int j1 = min(n_mine, j0 + 1024);
        for (int j = j0; j < j1; ++j) {
            int xr, xi;
            load_sample(samples, FMT, n_first + (long long)j * kTrackThreads, xr, xi);
#pragma unroll
            for (int cc = 0; cc < kTrackCG; ++cc) {
                const uint32_t lv = s_lut[ph[cc] >> 22];
                const int cs = (int)(int16_t)(lv & 0xFFFFu), sn = (int)(int16_t)(lv >> 16);
                int yr, yi;
                if (FMT == GNSS_CPLX_I8) {
                    yr = __mul24(xr, cs) + __mul24(xi, sn);
                    yi = __mul24(xi, cs) - __mul24(xr, sn);
                } else {
                    yr = __mul24(xr, cs);
                    yi = __mul24(-xr, sn);
                }
                // keeps the compiler from distributing the +-1 factors below into these
                // products (which it then evaluates with 64-bit multiply-adds)
                asm volatile("" : "+v"(yr), "+v"(yi));
                const int chp = (int)(uint32_t)(q[cc] >> 32);
                const int che = (int)(uint32_t)((q[cc] + dl[cc]) >> 32);
                const int chl = (int)(uint32_t)((q[cc] + ndl[cc]) >> 32);  // high word of q - dl: >= -1
                const int se = s_sign[cc][che + 1], sp = s_sign[cc][chp + 1], sl = s_sign[cc][chl + 1];
                acc[cc][0] += __mul24(se, yr);
                acc[cc][1] += __mul24(se, yi);
                acc[cc][2] += __mul24(sp, yr);
                acc[cc][3] += __mul24(sp, yi);
                acc[cc][4] += __mul24(sl, yr);
                acc[cc][5] += __mul24(sl, yi);
                ph[cc] += dph[cc];
                q[cc] += dq[cc];
                q[cc] -= q[cc] >= (unsigned long long)kCodeFix ? (unsigned long long)kCodeFix : 0ull;
            }
        }
#pragma unroll
        for (int cc = 0; cc < kTrackCG; ++cc)
#pragma unroll
            for (int k = 0; k < 6; ++k) tot[cc][k] += acc[cc][k];
    }
}

// One workgroup per (request, epoch); the request's channels in passes of
// kTrackCG.  Thread t handles samples t, t + 256, ... of the epoch with the
// NCO words advanced by 256 steps between them; the code phase is kept in
// [0, 1023 * 2^32), which leaves every chip index mod 1023 unchanged.
__global__ __launch_bounds__(kTrackThreads) void k_track(const TrackDesc *__restrict__ R, const long long *pre,
                                                         int n_req, long long total, const TrackCh *__restrict__ CH,
                                                         const uint8_t *codes, const uint32_t *lut)
{
    __shared__ uint32_t s_lut[1024];
    __shared__ int8_t s_sign[kTrackCG][kSignRow];
    __shared__ long long s_red[kTrackThreads / 64 * kTrackVals];
    for (int i = threadIdx.x; i < 1024; i += kTrackThreads) s_lut[i] = lut[i];
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const int r = find_req(pre, n_req, it);
        const TrackDesc &d = R[r];
        const int e = (int)(it - pre[r]);
        const long long n_first = d.start + (long long)e * d.epoch_len + threadIdx.x;
        for (int c0 = 0; c0 < d.n_ch; c0 += kTrackCG) {
            __syncthreads();  // LUT staged; previous pass done with s_sign and s_red
            for (int i = threadIdx.x; i < kTrackCG * (kCodeLen + 2); i += kTrackThreads) {
                const int cc = i / (kCodeLen + 2), k = i - cc * (kCodeLen + 2);
                const int prn = CH[d.ch_off + min(c0 + cc, d.n_ch - 1)].prn;
                const int chip = k == 0 ? kCodeLen - 1 : (k == kCodeLen + 1 ? 0 : k - 1);
                s_sign[cc][k] = (int8_t)(1 - 2 * (int)(codes[prn * kCodeLen + chip] & 1u));
            }
            __syncthreads();
            uint32_t ph[kTrackCG], dph[kTrackCG];
            unsigned long long q[kTrackCG], dq[kTrackCG], dl[kTrackCG], ndl[kTrackCG];
#pragma unroll
            for (int cc = 0; cc < kTrackCG; ++cc) {
                const TrackCh c = CH[d.ch_off + min(c0 + cc, d.n_ch - 1)];
                ph[cc] = c.phi0 + (uint32_t)((unsigned long long)n_first * c.D);
                dph[cc] = (uint32_t)kTrackThreads * c.D;
                q[cc] = (unsigned long long)(c.q0 + n_first * c.R) % (unsigned long long)kCodeFix;
                dq[cc] = (unsigned long long)((long long)kTrackThreads * c.R) % (unsigned long long)kCodeFix;
                dl[cc] = (unsigned long long)c.dl;
                ndl[cc] = (unsigned long long)(-c.dl);
            }
            long long tot[kTrackCG][6];
#pragma unroll
            for (int cc = 0; cc < kTrackCG; ++cc)
#pragma unroll
                for (int k = 0; k < 6; ++k) tot[cc][k] = 0;
            const int n_mine = d.epoch_len > (int)threadIdx.x ? (d.epoch_len - 1 - (int)threadIdx.x) / kTrackThreads + 1 : 0;
            if (d.fmt == GNSS_CPLX_I8)
                track_pass<GNSS_CPLX_I8>(d.samples, n_first, n_mine, s_lut, s_sign, ph, dph, q, dq, dl, ndl, tot);
            else if (d.fmt == GNSS_REAL_I8)
                track_pass<GNSS_REAL_I8>(d.samples, n_first, n_mine, s_lut, s_sign, ph, dph, q, dq, dl, ndl, tot);
            else
                track_pass<GNSS_REAL_2BIT_PACKED>(d.samples, n_first, n_mine, s_lut, s_sign, ph, dph, q, dq, dl, ndl,
                                                  tot);
            const long long v = block_sums64(tot, s_red);
            if (threadIdx.x < kTrackVals) {
                const int cc = threadIdx.x / 6, k = threadIdx.x - cc * 6;
                if (c0 + cc < d.n_ch) gmem(d.out)[((long long)(c0 + cc) * d.n_epochs + e) * 6 + k] = v;
            }
        }
    }
}

hipError_t launch_track(const TrackDesc *d_reqs, const long long *d_pre, int n_req, long long total,
                        const TrackCh *d_ch, const uint8_t *d_codes, const uint32_t *d_lut, hipStream_t s)
{
    const long long g = total < 0x7fffffffLL ? total : 0x7fffffffLL;
    hipLaunchKernelGGL(k_track, dim3((unsigned)(g > 0 ? g : 1)), dim3(kTrackThreads), 0, s, d_reqs, d_pre, n_req,
                       total, d_ch, d_codes, d_lut);
    return hipGetLastError();
}

size_t peak_scratch_part_elems(const Plan &p)
{
    return (size_t)p.n_prn * ((p.N + kPeakThreads - 1) / kPeakThreads);
}

// ===========================================================================
// test entry: batched natural-order 2048-point FFT / IFFT
// ===========================================================================
__global__ __launch_bounds__(256) void k_fft_test(const float2 *in, float2 *out, int batch,
                                                  int inverse, const float2 *tw)
{
    __shared__ float2 s_tw[kTwElems];
    __shared__ float2 s_xb[4][kXbufElems];
    stage_twiddles(s_tw, tw, threadIdx.x, 256);
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const long long vec = (long long)blockIdx.x * 4 + w;
    if (vec >= batch) return;
    const float2 *src = in + vec * 2048;
    float2 *dst = out + vec * 2048;
    float2 v[32];
    if (!inverse) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k2b = 0; k2b < 8; ++k2b) v[8 * u + k2b] = src[l + 64 * u + 256 * k2b];
        fft2048<false>(v, s_xb[w], s_tw, s_tw + kT1Elems, l);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int n1 = 0; n1 < 16; ++n1) dst[128 * n1 + l + 64 * h] = v[16 * h + n1];
    } else {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int n1 = 0; n1 < 16; ++n1) v[16 * h + n1] = src[128 * n1 + l + 64 * h];
        ifft2048<false>(v, s_xb[w], s_tw, s_tw + kT1Elems, l);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k2b = 0; k2b < 8; ++k2b) dst[l + 64 * u + 256 * k2b] = v[8 * u + k2b];
    }
}

hipError_t launch_fft_test(const float2 *d_in, float2 *d_out, int batch, int inverse,
                           const float2 *d_tw, hipStream_t s)
{
    hipLaunchKernelGGL(k_fft_test, dim3((batch + 3) / 4), dim3(256), 0, s, d_in, d_out, batch,
                       inverse, d_tw);
    return hipGetLastError();
}


// ===========================================================================
// test entry: batched natural-order 1023-point DFT / unnormalised inverse in
// the exact-length mode's arithmetic (per-vector exponent from the l1 norm,
// FP16 operands, FP32 accumulation); one wave per vector
// ===========================================================================
__global__ __launch_bounds__(256) void k_dft1023_test(const float2 *in, float2 *out, int batch, int inverse,
                                                      const pfa::u4 *__restrict__ fr)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c = l & 15;
    const long long vec = (long long)blockIdx.x * 4 + w;
    if (vec >= batch) return;
    const float2 *src = in + vec * kCodeLen;
    float *dst = (float *)(out + vec * kCodeLen);
    float nrm = 0.f;
    for (int i = l; i < kCodeLen; i += 64) nrm += fabsf(src[i].x) + fabsf(src[i].y);
    const int e = l1_exponent(wave_sum(nrm));
    const float f = ldexpf(1.f, -e), fo = ldexpf(1.f, e);
    pfa::u4 a1[3][2];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            float re[4], im[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i1 = 16 * s + 4 * g + j, i2 = 16 * t + c;
                float2 v = make_float2(0.f, 0.f);
                if (i1 < pfa::kN1 && i2 < pfa::kN2)
                    v = src[inverse ? pfa::freq_index(i1, i2) : pfa::time_index(i1, i2)];
                re[j] = v.x * f;
                im[j] = v.y * f;
            }
            a1[t][s] = pfa::u4{pfa::pack2(re[0], re[1]), pfa::pack2(re[2], re[3]), pfa::pack2(im[0], im[1]),
                               pfa::pack2(im[2], im[3])};
        }
    if (!inverse) {
        pfa::FwdB B;
        pfa::load_fwd(B, fr, l);
        pfa::f4 o[2][6];
        pfa::forward(a1, B, o);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 6; ++v)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int a = 16 * u + 4 * g + r, b = 16 * (v >> 1) + c;
                    if (a < pfa::kN1 && b < pfa::kN2) dst[2 * pfa::freq_index(a, b) + (v & 1)] = o[u][v][r] * fo;
                }
    } else {
        pfa::InvB B;
        pfa::load_inv(B, fr, l);
        pfa::f4 o[2][5];
        pfa::inverse(a1, B, o);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 5; ++v)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n1 = 16 * u + 4 * g + r;
                    const int n2 = v < 4 ? 16 * (v >> 1) + c : (c < 2 ? 32 : pfa::kN2);
                    const int part = v < 4 ? (v & 1) : c;
                    if (n1 < pfa::kN1 && n2 < pfa::kN2) dst[2 * pfa::time_index(n1, n2) + part] = o[u][v][r] * fo;
                }
    }
}

hipError_t launch_dft1023_test(const float2 *d_in, float2 *d_out, int batch, int inverse, const void *d_frags,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_dft1023_test, dim3((batch + 3) / 4), dim3(256), 0, s, d_in, d_out, batch, inverse,
                       (const pfa::u4 *)d_frags);
    return hipGetLastError();
}

}  // namespace gnss

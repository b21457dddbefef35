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
// Kernel sequence per request:
//   k_wipe_fold_box  NCO wipe-off + coherent fold + boxcar + polyphase split
//                    (exact int32)                     -> F[k][b][s][1024]
//   k_fft_poly       forward 2048-point FFT of every g_s -> G (storage order)
//   k_corr           per (PRN tile, Doppler, phase): G * conj(code spectrum),
//                    IFFT, |.|^2, sum over blocks in registers -> grid
//   k_colmax/k_peak  column max over Doppler, argmax, second peak, mean
//   k_interp         FP64 parabolic refinement
#include "fft2048.hpp"
#include "gnss_internal.hpp"

#include <math.h>

namespace gnss {

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

// ===========================================================================
// carrier NCO + first mixing stage + coherent fold
// ===========================================================================
struct WipeArgs {
    int fmt;
    int N, spc, Tc, Nnc;
    double fs, f_if, lo, step;
};

// D_k = (uint32)(int64) llround((f_if + (lo + k*step)) * 2^32 / fs), without
// contraction so that it rounds exactly as written.
__device__ __forceinline__ uint32_t nco_step(const WipeArgs &a, int k)
{
    double fk = __dadd_rn(a.lo, __dmul_rn((double)k, a.step));
    double f = __dadd_rn(a.f_if, fk);
    double x = __ddiv_rn(__dmul_rn(f, 4294967296.0), a.fs);
    return (uint32_t)(long long)llround(x);
}

__device__ __forceinline__ void load_sample(const void *samples, int fmt, long long n, int &xr, int &xi)
{
    if (fmt == GNSS_CPLX_I8) {
        char2 v = ((const char2 *)samples)[n];
        xr = v.x;
        xi = v.y;
    } else if (fmt == GNSS_REAL_I8) {
        xr = ((const int8_t *)samples)[n];
        xi = 0;
    } else {
        uint32_t byte = ((const uint8_t *)samples)[n >> 2];
        uint32_t code = (byte >> (2 * (uint32_t)(n & 3))) & 3u;
        // 00:+1 01:+3 10:-1 11:-3
        int mag = (code & 1u) ? 3 : 1;
        xr = (code & 2u) ? -mag : mag;
        xi = 0;
    }
}

// y[n] = x[n] * (cosL - j sinL)[phase(n) >> 22], summed over the Tc
// milliseconds of coherent block b at in-block offset m.
__device__ __forceinline__ int2 wipe_fold_one(const void *samples, const WipeArgs &a,
                                              const uint32_t *lut, uint32_t D, int b, int m)
{
    int yr = 0, yi = 0;
    for (int c = 0; c < a.Tc; ++c) {
        long long ng = (long long)(b * a.Tc + c) * a.N + m;
        int xr, xi;
        load_sample(samples, a.fmt, ng, xr, xi);
        uint32_t ph = (uint32_t)(unsigned long long)ng * D;
        uint32_t e = lut[ph >> 22];
        int cs = (int)(int16_t)(e & 0xFFFFu), sn = (int)(int16_t)(e >> 16);
        yr += xr * cs + xi * sn;
        yi += xi * cs - xr * sn;
    }
    return make_int2(yr, yi);
}

// Standalone wipe + fold (stage entry): out[((k*Nnc + b)*N + m)*2 + {0,1}].
__global__ __launch_bounds__(256) void k_wipe_fold(const void *samples, const uint32_t *lut,
                                                   WipeArgs a, int2 *out)
{
    __shared__ uint32_t s_lut[1024];
    for (int i = threadIdx.x; i < 1024; i += 256) s_lut[i] = lut[i];
    const int k = blockIdx.x / a.Nnc, b = blockIdx.x % a.Nnc;
    const uint32_t D = nco_step(a, k);
    __syncthreads();
    int2 *dst = out + (long long)blockIdx.x * a.N;
    for (int m = threadIdx.x; m < a.N; m += 256) dst[m] = wipe_fold_one(samples, a, s_lut, D, b, m);
}

hipError_t launch_wipe_fold(const void *d_samples, const Plan &p, const uint32_t *d_lut,
                            int32_t *d_out, hipStream_t s)
{
    WipeArgs a{p.fmt, p.N, p.spc, p.Tc, p.Nnc, (double)p.fs_hz, p.f_if, p.lo, p.step};
    hipLaunchKernelGGL(k_wipe_fold, dim3(p.n_dopp * p.Nnc), dim3(256), 0, s, d_samples, d_lut, a,
                       (int2 *)d_out);
    return hipGetLastError();
}

// Hot-path stage A1: wipe + fold, then the one-chip boxcar
// F[n] = sum_{t<spc} f[(n+t) mod N], written split by phase:
// Fout[k][b][s][m] = F[spc m + s] (m < 1023), Fout[..][1023] = 0.  Each
// workgroup covers a chunk of kBoxChunk outputs of one (Doppler, block) and
// wipes the spc - 1 samples past it as a halo.  All integer, exact.
constexpr int kBoxChunk = 2048;
constexpr int kBoxRun = 8;
__device__ __forceinline__ int bpad(int i) { return i + (i >> 3); }  // bank-conflict padding

__global__ __launch_bounds__(256) void k_wipe_fold_box(const void *samples, const uint32_t *lut,
                                                       WipeArgs a, int2 *Fout, int n_chunks)
{
    __shared__ int2 s_f[(kBoxChunk + kMaxSpc) + (kBoxChunk + kMaxSpc) / 8 + 8];
    __shared__ uint32_t s_lut[1024];
    for (int i = threadIdx.x; i < 1024; i += 256) s_lut[i] = lut[i];
    const int chunk = blockIdx.x % n_chunks, kb = blockIdx.x / n_chunks;
    const int k = kb / a.Nnc, b = kb % a.Nnc;
    const uint32_t D = nco_step(a, k);
    const int N = a.N, spc = a.spc;
    const int n0 = chunk * kBoxChunk;
    const int cnt = min(kBoxChunk, N - n0);
    const int len = cnt + spc - 1;
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += 256) {
        int n = n0 + i;
        if (n >= N) n -= N;
        s_f[bpad(i)] = wipe_fold_one(samples, a, s_lut, D, b, n);
    }
    __syncthreads();
    int2 *dst = Fout + (long long)kb * spc * kPolyLen;
    const int n_runs = (cnt + kBoxRun - 1) / kBoxRun;
    for (int r = threadIdx.x; r < n_runs; r += 256) {
        const int i0 = r * kBoxRun;
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
    if (chunk == 0 && threadIdx.x < spc) dst[threadIdx.x * kPolyLen + (kPolyLen - 1)] = make_int2(0, 0);
}

hipError_t launch_wipe_fold_box(const void *d_samples, const Plan &p, const uint32_t *d_lut,
                                int2 *d_F, hipStream_t s)
{
    WipeArgs a{p.fmt, p.N, p.spc, p.Tc, p.Nnc, (double)p.fs_hz, p.f_if, p.lo, p.step};
    const int n_chunks = (p.N + kBoxChunk - 1) / kBoxChunk;
    const long long nwg = (long long)p.n_dopp * p.Nnc * n_chunks;
    hipLaunchKernelGGL(k_wipe_fold_box, dim3((unsigned)nwg), dim3(256), 0, s, d_samples, d_lut, a,
                       d_F, n_chunks);
    return hipGetLastError();
}

// ===========================================================================
// stage A2: forward 2048-point FFT of every polyphase component
// ===========================================================================
__global__ __launch_bounds__(256) void k_fft_poly(const int2 *F, const float2 *tw, float4 *G,
                                                  long long n_vec)
{
    __shared__ float2 s_tw[kTwElems];
    __shared__ float2 s_xb[4][kXbufElems];
    stage_twiddles(s_tw, tw, threadIdx.x, 256);
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const long long vec = (long long)blockIdx.x * 4 + w;
    if (vec >= n_vec) return;
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
    fft2048<true>(v, s_xb[w], s_tw, s_tw + kT1Elems, l);
    float4 *dst = G + vec * kVec;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj)
        dst[jj * 64 + l] = make_float4(v[2 * jj].x, v[2 * jj].y, v[2 * jj + 1].x, v[2 * jj + 1].y);
}

hipError_t launch_fft_poly(const int2 *d_F, const float2 *d_tw, float4 *d_G, int64_t n_vec,
                           hipStream_t s)
{
    long long blocks = (n_vec + 3) / 4;
    hipLaunchKernelGGL(k_fft_poly, dim3((unsigned)blocks), dim3(256), 0, s, d_F, d_tw, d_G,
                       (long long)n_vec);
    return hipGetLastError();
}

// ===========================================================================
// stage B: fused conj-multiply -> IFFT -> |.|^2 -> non-coherent sum
// ===========================================================================
struct CorrArgs {
    PrnList prns;
    int n_prn, n_dopp, N, spc, Nnc;
    int n_items;   // n_dopp * spc work items (Doppler bin, phase)
    int n_ptiles;
};

// Workgroups are dealt round-robin to the 8 XCDs; remap so that consecutive
// logical ids (the PRN tiles of one item chunk, which read the same G) run on
// the same XCD and share its L2.
__device__ __forceinline__ int xcd_remap(int bid, int nwg)
{
    const int X = 8, q = nwg / X, r = nwg % X;
    const int xcd = bid % X, local = bid / X;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

constexpr int kCorrWaves = 8;

// Staging of the finished sums for the grid write: [PT][1024 q][9] floats
// (8 waves + 1 pad, so both the per-wave writes and the per-row reads are
// free of bank conflicts).
constexpr int kStagePad = kCorrWaves + 1;

template <int PT>
__global__ __launch_bounds__(64 * kCorrWaves) void k_corr(const float4 *G,
                                                          const float4 *__restrict__ CS,
                                                          const float2 *__restrict__ tw,
                                                          float *__restrict__ grid, CorrArgs a)
{
    constexpr int kCcBytes = PT * kVec * (int)sizeof(float4);
    constexpr int kTwBytes = kTwElems * (int)sizeof(float2);
    constexpr int kXbBytes = kCorrWaves * kXbufElems * (int)sizeof(float2);
    constexpr int kStageBytes = PT * 1024 * kStagePad * (int)sizeof(float);
    constexpr int kSmem = (kCcBytes + kTwBytes + kXbBytes) > kStageBytes ? (kCcBytes + kTwBytes + kXbBytes)
                                                                          : kStageBytes;
    __shared__ __align__(16) unsigned char smem[kSmem];
    float4 *s_cc = (float4 *)smem;
    float2 *s_tw = (float2 *)(smem + kCcBytes);
    float2 *s_xb = (float2 *)(smem + kCcBytes + kTwBytes);
    float *s_stage = (float *)smem;  // reused after the transforms

    const int tid = threadIdx.x;
    const int logical = xcd_remap(blockIdx.x, gridDim.x);
    const int ptile = logical % a.n_ptiles, chunk = logical / a.n_ptiles;
    for (int i = tid; i < PT * kVec; i += 64 * kCorrWaves) {
        int p = i / kVec, e = i - p * kVec;
        int pi = ptile * PT + p;
        int prn = pi < a.n_prn ? a.prns.v[pi] : 0;
        s_cc[i] = CS[(long long)prn * kVec + e];
    }
    stage_twiddles(s_tw, tw, tid, 64 * kCorrWaves);
    __syncthreads();

    const int w = tid >> 6, l = tid & 63;
    const int item = chunk * kCorrWaves + w;
    const bool active = item < a.n_items;
    const int k = item / a.spc, s = item - k * a.spc;

    float acc[PT][16];
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[p][i] = 0.f;

    if (active) {
        const float4 *gk = G + ((long long)k * a.Nnc * a.spc + s) * kVec;
        float2 *xb = s_xb + w * kXbufElems;
        for (int b = 0; b < a.Nnc; ++b) {
            const float4 *gp = gk + (long long)b * a.spc * kVec;
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
                ifft2048<true>(z, xb, s_tw, s_tw + kT1Elems, l);
                phase_barrier();
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int k2b = 0; k2b < 4; ++k2b) {
                        float2 r = z[8 * u + k2b];
                        acc[p][4 * u + k2b] = fmaf(r.x, r.x, fmaf(r.y, r.y, acc[p][4 * u + k2b]));
                    }
            }
        }
    }

    // Grid write.  P = |IFFT|^2 * 2^-46 (2^-22 for the unnormalised 2048-point
    // IFFT, 2^-24 for the LUT scale).  Lag tau = spc*q + s interleaves the
    // waves' phases, so the sums are staged in LDS and written as contiguous
    // runs of consecutive tau.
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k2b = 0; k2b < 4; ++k2b) {
                int q = l + 64 * u + 256 * k2b;
                s_stage[(p * 1024 + q) * kStagePad + w] = acc[p][4 * u + k2b] * 0x1p-46f;
            }
    __syncthreads();
    const int first = chunk * kCorrWaves;
    const int n_items_here = min(kCorrWaves, a.n_items - first);
    int wa = 0;
    while (wa < n_items_here) {
        const int ka = (first + wa) / a.spc, sa = (first + wa) - ka * a.spc;
        int ns = min(a.spc - sa, n_items_here - wa);  // consecutive phases of Doppler bin ka
        const int total = kCodeLen * ns;
        for (int p = 0; p < PT; ++p) {
            const int pi = ptile * PT + p;
            if (pi >= a.n_prn) break;
            float *row = grid + ((long long)pi * a.n_dopp + ka) * a.N + sa;
            const float *st = s_stage + p * 1024 * kStagePad + wa;
            for (int idx = tid; idx < total; idx += 64 * kCorrWaves) {
                const int q = idx / ns, j = idx - q * ns;
                row[(long long)a.spc * q + j] = st[q * kStagePad + j];
            }
        }
        wa += ns;
    }
}

constexpr int kCorrPT = 4;

hipError_t launch_corr(const float4 *d_G, const float4 *d_cs, const float2 *d_tw, float *d_grid,
                       const Plan &p, hipStream_t s)
{
    CorrArgs a;
    a.prns = p.prns;
    a.n_prn = p.n_prn;
    a.n_dopp = p.n_dopp;
    a.N = p.N;
    a.spc = p.spc;
    a.Nnc = p.Nnc;
    a.n_items = p.n_dopp * p.spc;
    a.n_ptiles = (p.n_prn + kCorrPT - 1) / kCorrPT;
    const int n_chunks = (a.n_items + kCorrWaves - 1) / kCorrWaves;
    const long long nwg = (long long)n_chunks * a.n_ptiles;
    hipLaunchKernelGGL(k_corr<kCorrPT>, dim3((unsigned)nwg), dim3(64 * kCorrWaves), 0, s, d_G,
                       d_cs, d_tw, d_grid, a);
    return hipGetLastError();
}

// ===========================================================================
// detection: column max over Doppler, argmax, second peak, mean; refinement
// ===========================================================================
constexpr int kPeakThreads = 256;

size_t peak_scratch_part_elems(const Plan &p)
{
    return (size_t)p.n_prn * ((p.N + kPeakThreads - 1) / kPeakThreads);
}

// Q[p][tau] = max_k P (lowest k on ties), K = that k; part = per-block sum of P (FP64).
__global__ __launch_bounds__(kPeakThreads) void k_colmax(const float *grid, int n_dopp, int N,
                                                         float *Q, int32_t *K, double *part)
{
    __shared__ double red[kPeakThreads];
    const int p = blockIdx.y, tau = blockIdx.x * kPeakThreads + threadIdx.x;
    double colsum = 0.0;
    if (tau < N) {
        const float *col = grid + (long long)p * n_dopp * N + tau;
        float best = col[0];
        int kb = 0;
        colsum = (double)best;
        for (int k = 1; k < n_dopp; ++k) {
            float v = col[(long long)k * N];
            colsum += (double)v;
            if (v > best) {
                best = v;
                kb = k;
            }
        }
        Q[(long long)p * N + tau] = best;
        K[(long long)p * N + tau] = kb;
    }
    red[threadIdx.x] = colsum;
    __syncthreads();
    for (int st = kPeakThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)p * gridDim.x + blockIdx.x] = red[0];
}

struct PeakArgs {
    PrnList prns;
    int n_dopp, N, spc, n_parts;
    float threshold;
};

__global__ __launch_bounds__(kPeakThreads) void k_peak(const float *Q, const int32_t *K,
                                                       const double *part, PeakArgs a,
                                                       gnss_peak *out)
{
    __shared__ float sv[kPeakThreads];
    __shared__ int st[kPeakThreads];
    const int p = blockIdx.x, tid = threadIdx.x;
    const float *q = Q + (long long)p * a.N;
    // argmax, lowest tau on ties
    float bv = -INFINITY;
    int bt = 0x7fffffff;
    for (int tau = tid; tau < a.N; tau += kPeakThreads) {
        float v = q[tau];
        if (v > bv) {
            bv = v;
            bt = tau;
        }
    }
    sv[tid] = bv;
    st[tid] = bt;
    __syncthreads();
    for (int s = kPeakThreads / 2; s > 0; s >>= 1) {
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
    const int tstar = (st[0] >= 0 && st[0] < a.N) ? st[0] : 0;
    __syncthreads();
    // second peak outside +-spc (circular)
    float m2 = -INFINITY;
    for (int tau = tid; tau < a.N; tau += kPeakThreads) {
        int d = abs(tau - tstar);
        d = min(d, a.N - d);
        if (d > a.spc) m2 = fmaxf(m2, q[tau]);
    }
    sv[tid] = m2;
    __syncthreads();
    for (int s = kPeakThreads / 2; s > 0; s >>= 1) {
        if (tid < s) sv[tid] = fmaxf(sv[tid], sv[tid + s]);
        __syncthreads();
    }
    if (tid == 0) {
        float second = sv[0] == -INFINITY ? 0.f : sv[0];
        double sum = 0.0;
        for (int i = 0; i < a.n_parts; ++i) sum += part[(long long)p * a.n_parts + i];
        gnss_peak r;
        r.prn = a.prns.v[p];
        r.doppler_bin = K[(long long)p * a.N + tstar];
        r.code_phase = tstar;
        r.peak = peak;
        r.second = second;
        r.mean = (float)(sum / ((double)a.n_dopp * (double)a.N));
        r.ratio = second > 0.f ? peak / second : INFINITY;
        r.detected = r.ratio >= a.threshold ? 1 : 0;
        r.doppler_hz = 0.0;
        r.code_phase_frac = (double)tstar;
        out[p] = r;
    }
}

__device__ __forceinline__ double parabola(double ym, double y0, double yp)
{
    double den = ym - 2.0 * y0 + yp;
    if (den == 0.0) return 0.0;
    return 0.5 * (ym - yp) / den;
}

// FP64 sub-bin refinement (the only FP64 arithmetic on the hot path).
__global__ void k_interp(const float *grid, int n_prn, int n_dopp, int N, double lo, double step,
                         gnss_peak *out)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_prn) return;
    gnss_peak r = out[p];
    const float *G = grid + (long long)p * n_dopp * N;
    const int k = r.doppler_bin, t = r.code_phase;
    double y0 = G[(long long)k * N + t];
    double dc = parabola(G[(long long)k * N + (t - 1 + N) % N], y0, G[(long long)k * N + (t + 1) % N]);
    double dd = 0.0;
    if (k > 0 && k < n_dopp - 1) dd = parabola(G[(long long)(k - 1) * N + t], y0, G[(long long)(k + 1) * N + t]);
    double fk = __dadd_rn(lo, __dmul_rn((double)k, step));
    out[p].doppler_hz = __dadd_rn(fk, __dmul_rn(dd, step));
    out[p].code_phase_frac = __dadd_rn((double)t, dc);
}

hipError_t launch_peaks(const float *d_grid, const Plan &p, float threshold, float *d_Q,
                        int32_t *d_K, double *d_part, gnss_peak *d_peaks, hipStream_t s)
{
    const int nblk = (p.N + kPeakThreads - 1) / kPeakThreads;
    hipLaunchKernelGGL(k_colmax, dim3(nblk, p.n_prn), dim3(kPeakThreads), 0, s, d_grid, p.n_dopp,
                       p.N, d_Q, d_K, d_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    PeakArgs a{p.prns, p.n_dopp, p.N, p.spc, nblk, threshold};
    hipLaunchKernelGGL(k_peak, dim3(p.n_prn), dim3(kPeakThreads), 0, s, d_Q, d_K, d_part, a, d_peaks);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_interp, dim3((p.n_prn + 63) / 64), dim3(64), 0, s, d_grid, p.n_prn,
                       p.n_dopp, p.N, p.lo, p.step, d_peaks);
    return hipGetLastError();
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

}  // namespace gnss

// fft2048.hpp -- one 2048-point complex FFT per wavefront, for gfx950 (wave64).
//
// The acquisition channel's frequency-domain correlation (paper Sec. 3, Fig. 2:
// FFT of the mixed signal, FFT of the code replica, multiply, IFFT) is done
// here on 2048-point transforms: the length-1023 chip-rate circular
// correlations of the polyphase form (see gnss_kernels.hip) zero-padded to
// 2048 = 16 x 16 x 8.
//
// Data layout: each lane holds 32 complex values in registers (float2 v[32]).
// The inverse transform M (unnormalised, exp(+2 pi i nk/2048)) runs
//   I1 radix-16 in registers -> I2 twiddle W2048^(n2 k1) -> I3 LDS transpose ->
//   I4 radix-16 -> I5 twiddle W128^(m2 k2a) -> I6 LDS transpose -> I7 radix-8,
// taking its input in "storage order" and producing natural order.  The
// forward transform F is the conjugate transpose of M (same passes in reverse
// order, conjugated twiddles, inverse permutations), so it takes natural order
// and produces storage order.  Spectra are only ever multiplied element-wise,
// so they never need to be reordered.
//
// Storage order: lane l, register j = 16 h + n1 holds spectral index
//   128 n1 + l + 64 h.
// In memory a storage-order spectrum is 1024 float4: float4 index 64 jj + l
// holds registers (2 jj, 2 jj + 1) of lane l.
// Natural order (inverse output / forward input): lane l, register 8 u + k2b
// holds index l + 64 u + 256 k2b.
//
// Every pass is written once for two element types: float2 (one FP32
// transform) and hc2 (two FP16 transforms side by side: the low halves of
// re/im belong to one transform and the high halves to the other, so each
// packed FP16 instruction advances both).  Both are 8 bytes, so the LDS
// exchanges are the same for both.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gnss {

// ---------------------------------------------------------------------------
// compile-time trig for constant twiddles (Taylor series, |x| <= pi)
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double ct_sin(double x)
{
    double term = x, sum = x;
    for (int i = 1; i < 40; ++i) {
        term *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        sum += term;
    }
    return sum;
}

constexpr double ct_cos(double x)
{
    double term = 1.0, sum = 1.0;
    for (int i = 1; i < 40; ++i) {
        term *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        sum += term;
    }
    return sum;
}

// angle 2 pi k / n reduced to (-pi, pi]
constexpr double ct_angle(int k, int n)
{
    int kk = ((k % n) + n) % n;
    if (2 * kk > n) kk -= n;
    return 2.0 * kPi * (double)kk / (double)n;
}

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 c_mulc(float2 a, float2 b)  // a * conj(b)
{
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}

// Two complex FP16 values of two transforms: (re.x + i im.x) and (re.y + i im.y).
// A twiddle in this type carries the same value in both halves.
struct hc2 {
    __half2 re, im;
};
static_assert(sizeof(hc2) == sizeof(float2), "hc2 shares the float2 LDS layout");

__device__ __forceinline__ hc2 make_hc2(__half2 re, __half2 im)
{
    hc2 r;
    r.re = re;
    r.im = im;
    return r;
}
__device__ __forceinline__ hc2 c_add(hc2 a, hc2 b) { return make_hc2(__hadd2(a.re, b.re), __hadd2(a.im, b.im)); }
__device__ __forceinline__ hc2 c_sub(hc2 a, hc2 b) { return make_hc2(__hsub2(a.re, b.re), __hsub2(a.im, b.im)); }
__device__ __forceinline__ hc2 c_mul(hc2 a, hc2 w)
{
    return make_hc2(__hfma2(a.re, w.re, __hneg2(__hmul2(a.im, w.im))), __hfma2(a.re, w.im, __hmul2(a.im, w.re)));
}
__device__ __forceinline__ hc2 c_mulc(hc2 a, hc2 w)  // a * conj(w)
{
    return make_hc2(__hfma2(a.re, w.re, __hmul2(a.im, w.im)), __hfma2(a.im, w.re, __hneg2(__hmul2(a.re, w.im))));
}

// a * W_N^K with W_N = exp(+2 pi i / N) (inverse) or exp(-2 pi i / N) (forward)
template <int N, int K, bool INV>
__device__ __forceinline__ float2 tw(float2 a)
{
    constexpr int k = ((K % N) + N) % N;
    if constexpr (k == 0) {
        return a;
    } else if constexpr (2 * k == N) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (4 * k == N) {  // +i (inv) / -i (fwd)
        return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
    } else if constexpr (4 * k == 3 * N) {
        return INV ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
    } else if constexpr ((8 * k) % N == 0) {  // odd multiple of pi/4
        constexpr float r = 0.70710678118654752440f;
        constexpr int oct = 8 * k / N;                  // 1, 3, 5, 7
        constexpr float cs = (oct == 1 || oct == 7) ? 1.f : -1.f;
        constexpr float sn0 = (oct == 1 || oct == 3) ? 1.f : -1.f;
        constexpr float sn = INV ? sn0 : -sn0;
        // (x + i y)(cs + i sn) r
        return make_float2(r * (cs * a.x - sn * a.y), r * (sn * a.x + cs * a.y));
    } else {
        constexpr double th = ct_angle(K, N);
        constexpr float c = (float)ct_cos(th);
        constexpr float s = (float)(INV ? ct_sin(th) : -ct_sin(th));
        return c_mul(a, make_float2(c, s));
    }
}

template <int N, int K, bool INV>
__device__ __forceinline__ hc2 tw(hc2 a)
{
    constexpr int k = ((K % N) + N) % N;
    if constexpr (k == 0) {
        return a;
    } else if constexpr (2 * k == N) {
        return make_hc2(__hneg2(a.re), __hneg2(a.im));
    } else if constexpr (4 * k == N) {
        return INV ? make_hc2(__hneg2(a.im), a.re) : make_hc2(a.im, __hneg2(a.re));
    } else if constexpr (4 * k == 3 * N) {
        return INV ? make_hc2(a.im, __hneg2(a.re)) : make_hc2(__hneg2(a.im), a.re);
    } else if constexpr ((8 * k) % N == 0) {
        constexpr int oct = 8 * k / N;
        constexpr bool cpos = (oct == 1 || oct == 7);
        constexpr bool spos = ((oct == 1 || oct == 3) == INV);
        const __half2 r = __float2half2_rn(0.70710678118654752440f);
        // (x + i y)(cs + i sn) r with cs, sn = +-1
        const __half2 re = cpos ? (spos ? __hsub2(a.re, a.im) : __hadd2(a.re, a.im))
                                : (spos ? __hneg2(__hadd2(a.re, a.im)) : __hsub2(a.im, a.re));
        const __half2 im = cpos ? (spos ? __hadd2(a.re, a.im) : __hsub2(a.im, a.re))
                                : (spos ? __hsub2(a.re, a.im) : __hneg2(__hadd2(a.re, a.im)));
        return make_hc2(__hmul2(re, r), __hmul2(im, r));
    } else {
        constexpr double th = ct_angle(K, N);
        constexpr float c = (float)ct_cos(th);
        constexpr float s = (float)(INV ? ct_sin(th) : -ct_sin(th));
        return c_mul(a, make_hc2(__float2half2_rn(c), __float2half2_rn(s)));
    }
}

// ---------------------------------------------------------------------------
// small DFTs in registers (natural order in and out)
// ---------------------------------------------------------------------------
template <bool INV, typename T>
__device__ __forceinline__ void dft4(T &a0, T &a1, T &a2, T &a3)
{
    T t0 = c_add(a0, a2), t1 = c_sub(a0, a2);
    T t2 = c_add(a1, a3), t3 = tw<4, 1, INV>(c_sub(a1, a3));
    a0 = c_add(t0, t2);
    a2 = c_sub(t0, t2);
    a1 = c_add(t1, t3);
    a3 = c_sub(t1, t3);
}

// 4-point DFT of (a0, a1, 0, 0)
template <bool INV, typename T>
__device__ __forceinline__ void dft4_half(T &a0, T &a1, T &a2, T &a3)
{
    T x0 = a0, x1 = a1, t3 = tw<4, 1, INV>(x1);
    a0 = c_add(x0, x1);
    a2 = c_sub(x0, x1);
    a1 = c_add(x0, t3);
    a3 = c_sub(x0, t3);
}

// 8-point DFT on registers a[OFF .. OFF+8).  PRUNE_IN: inputs 4..7 are zero.
// PRUNE_OUT: only outputs 0..3 are needed (4..7 are left unspecified).
template <bool INV, bool PRUNE_IN, bool PRUNE_OUT, int OFF, typename T, int LEN>
__device__ __forceinline__ void dft8(T (&a)[LEN])
{
    T e0 = a[OFF + 0], e1 = a[OFF + 2], e2 = a[OFF + 4], e3 = a[OFF + 6];
    T o0 = a[OFF + 1], o1 = a[OFF + 3], o2 = a[OFF + 5], o3 = a[OFF + 7];
    if constexpr (PRUNE_IN) {
        dft4_half<INV>(e0, e1, e2, e3);
        dft4_half<INV>(o0, o1, o2, o3);
    } else {
        dft4<INV>(e0, e1, e2, e3);
        dft4<INV>(o0, o1, o2, o3);
    }
    o1 = tw<8, 1, INV>(o1);
    o2 = tw<8, 2, INV>(o2);
    o3 = tw<8, 3, INV>(o3);
    a[OFF + 0] = c_add(e0, o0);
    a[OFF + 1] = c_add(e1, o1);
    a[OFF + 2] = c_add(e2, o2);
    a[OFF + 3] = c_add(e3, o3);
    if constexpr (!PRUNE_OUT) {
        a[OFF + 4] = c_sub(e0, o0);
        a[OFF + 5] = c_sub(e1, o1);
        a[OFF + 6] = c_sub(e2, o2);
        a[OFF + 7] = c_sub(e3, o3);
    }
}

// 16-point DFT on registers a[OFF .. OFF+16): 4 x 4 four-step.
template <bool INV, int OFF, typename T, int LEN>
__device__ __forceinline__ void dft16(T (&a)[LEN])
{
    T y[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) y[i] = a[OFF + i];
    // DFT over n1 of y[4 n1 + n2] -> y[4 k1 + n2]
    dft4<INV>(y[0], y[4], y[8], y[12]);
    dft4<INV>(y[1], y[5], y[9], y[13]);
    dft4<INV>(y[2], y[6], y[10], y[14]);
    dft4<INV>(y[3], y[7], y[11], y[15]);
    // twiddle W16^(n2 k1)
    y[5] = tw<16, 1, INV>(y[5]);
    y[6] = tw<16, 2, INV>(y[6]);
    y[7] = tw<16, 3, INV>(y[7]);
    y[9] = tw<16, 2, INV>(y[9]);
    y[10] = tw<16, 4, INV>(y[10]);
    y[11] = tw<16, 6, INV>(y[11]);
    y[13] = tw<16, 3, INV>(y[13]);
    y[14] = tw<16, 6, INV>(y[14]);
    y[15] = tw<16, 9, INV>(y[15]);
    // DFT over n2 of y[4 k1 + n2] -> X[k1 + 4 k2] at y[4 k1 + k2]
    dft4<INV>(y[0], y[1], y[2], y[3]);
    dft4<INV>(y[4], y[5], y[6], y[7]);
    dft4<INV>(y[8], y[9], y[10], y[11]);
    dft4<INV>(y[12], y[13], y[14], y[15]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) a[OFF + k1 + 4 * k2] = y[4 * k1 + k2];
}

// ---------------------------------------------------------------------------
// wave-private LDS transposes
// ---------------------------------------------------------------------------
// Row strides (in float2) of the two transpose buffers.  A wave needs
// kXbufElems float2 of LDS scratch.  Exchange A writes rows of 128 and reads
// 8 rows x 8 columns per 32 lanes: a stride of 136 (= 8 mod 32 float2) puts the
// 8 rows in distinct 64-byte bank groups.  Exchange B is indexed
// kl*kStrideB + 8*k1 + (m2 ^ (k1 >> 2)); with kStrideB = 4 mod 8 both its
// write (8 k1 x 8 m2 per 32 lanes) and its read (16 k1 x 2 rows per 32 lanes)
// touch 32 distinct 8-byte bank slots.
constexpr int kStrideA = 136;
constexpr int kStrideB = 132;
constexpr int kXbufElems = 8 * kStrideA;
static_assert(8 * kStrideB <= kXbufElems, "transpose buffer");

__device__ __forceinline__ int xb_b(int kl, int k1, int m2)
{
    return kl * kStrideB + 8 * k1 + (m2 ^ ((k1 >> 2) & 7));
}

__device__ __forceinline__ void lds_fence()
{
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Keeps the machine scheduler from hoisting loads of a later phase above the
// current one (which would raise register pressure past the occupancy target).
__device__ __forceinline__ void phase_barrier()
{
    __builtin_amdgcn_sched_barrier(0);
}

// I3: (lane l, reg 16h + k1) holds Y[n2 = l + 64h][k1]
//  -> (lane l, reg 16h' + m1) holds Y[8 m1 + (l & 7)][(l >> 3) + 8h']
template <typename T>
__device__ __forceinline__ void transpose_a_inv(T (&v)[32], T *xb, int l)
{
    T nv[32];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) xb[kk * kStrideA + l + 64 * h] = v[16 * h + 8 * half + kk];
        lds_fence();
        const T *src = xb + (l >> 3) * kStrideA + (l & 7);
#pragma unroll
        for (int m1 = 0; m1 < 16; ++m1) nv[16 * half + m1] = src[8 * m1];
        lds_fence();
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = nv[i];
}

// adjoint of transpose_a_inv
template <typename T>
__device__ __forceinline__ void transpose_a_fwd(T (&v)[32], T *xb, int l)
{
    T nv[32];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        T *dst = xb + (l >> 3) * kStrideA + (l & 7);
#pragma unroll
        for (int m1 = 0; m1 < 16; ++m1) dst[8 * m1] = v[16 * half + m1];
        lds_fence();
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) nv[16 * h + 8 * half + kk] = xb[kk * kStrideA + l + 64 * h];
        lds_fence();
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = nv[i];
}

// I6: (lane l, reg 16h' + k2a) holds Y'[k1 = (l >> 3) + 8h'][m2 = l & 7][k2a]
//  -> (lane l, reg 8u + m2) holds Y'[k1 = l & 15][m2][k2a = (l >> 4) + 4u]
template <typename T>
__device__ __forceinline__ void transpose_b_inv(T (&v)[32], T *xb, int l)
{
    T nv[32];
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
#pragma unroll
        for (int hp = 0; hp < 2; ++hp)
#pragma unroll
            for (int kl = 0; kl < 8; ++kl)
                xb[xb_b(kl, (l >> 3) + 8 * hp, l & 7)] = v[16 * hp + 8 * hb + kl];
        lds_fence();
#pragma unroll
        for (int uu = 0; uu < 2; ++uu)
#pragma unroll
            for (int m2 = 0; m2 < 8; ++m2)
                nv[8 * (2 * hb + uu) + m2] = xb[xb_b((l >> 4) + 4 * uu, l & 15, m2)];
        lds_fence();
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = nv[i];
}

// adjoint of transpose_b_inv
template <typename T>
__device__ __forceinline__ void transpose_b_fwd(T (&v)[32], T *xb, int l)
{
    T nv[32];
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
#pragma unroll
        for (int uu = 0; uu < 2; ++uu)
#pragma unroll
            for (int m2 = 0; m2 < 8; ++m2)
                xb[xb_b((l >> 4) + 4 * uu, l & 15, m2)] = v[8 * (2 * hb + uu) + m2];
        lds_fence();
#pragma unroll
        for (int hp = 0; hp < 2; ++hp)
#pragma unroll
            for (int kl = 0; kl < 8; ++kl)
                nv[16 * hp + 8 * hb + kl] = xb[xb_b(kl, (l >> 3) + 8 * hp, l & 7)];
        lds_fence();
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = nv[i];
}

// Quarter-buffer variants of the four exchanges: the same permutations done
// in four rounds through a buffer half the size (kXbufElemsQ elements per
// wave).  Besides needing less LDS, they are faster on gfx950 than the full
// buffer, whose exchanges the compiler turns into two-address LDS accesses
// that conflict in the banks (measured: about one conflict cycle per LDS
// instruction there, almost none here).
// Exchange A splits by h (columns 64h .. 64h + 63 of the half) with row stride
// kStrideAQ = 72 (= 8 mod 32 elements: a half-wave's 4 rows x 8 columns hit 32
// distinct 8-byte banks); exchange B splits by the rows kl of one uu with the
// stride and swizzle of the full buffer.
constexpr int kStrideAQ = 72;
constexpr int kXbufElemsQ = 8 * kStrideAQ;
static_assert(4 * kStrideB <= kXbufElemsQ, "quarter transpose buffer");

template <typename T>
__device__ __forceinline__ void transpose_a_inv_q(T (&v)[32], T *xb, int l)
{
    T nv[32];
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) xb[kk * kStrideAQ + l] = v[16 * h + 8 * half + kk];
            lds_fence();
            const T *src = xb + (l >> 3) * kStrideAQ + (l & 7);
#pragma unroll
            for (int m = 0; m < 8; ++m) nv[16 * half + 8 * h + m] = src[8 * m];
            lds_fence();
        }
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = nv[i];
}

template <typename T>
__device__ __forceinline__ void transpose_a_fwd_q(T (&v)[32], T *xb, int l)
{
    T nv[32];
#pragma unroll
    for (int half = 0; half < 2; ++half)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            T *dst = xb + (l >> 3) * kStrideAQ + (l & 7);
#pragma unroll
            for (int m = 0; m < 8; ++m) dst[8 * m] = v[16 * half + 8 * h + m];
            lds_fence();
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) nv[16 * h + 8 * half + kk] = xb[kk * kStrideAQ + l];
            lds_fence();
        }
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = nv[i];
}

template <typename T>
__device__ __forceinline__ void transpose_b_inv_q(T (&v)[32], T *xb, int l)
{
    T nv[32];
#pragma unroll
    for (int hb = 0; hb < 2; ++hb)
#pragma unroll
        for (int uu = 0; uu < 2; ++uu) {
#pragma unroll
            for (int hp = 0; hp < 2; ++hp)
#pragma unroll
                for (int kq = 0; kq < 4; ++kq)
                    xb[xb_b(kq, (l >> 3) + 8 * hp, l & 7)] = v[16 * hp + 8 * hb + 4 * uu + kq];
            lds_fence();
#pragma unroll
            for (int m2 = 0; m2 < 8; ++m2) nv[8 * (2 * hb + uu) + m2] = xb[xb_b(l >> 4, l & 15, m2)];
            lds_fence();
        }
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = nv[i];
}

template <typename T>
__device__ __forceinline__ void transpose_b_fwd_q(T (&v)[32], T *xb, int l)
{
    T nv[32];
#pragma unroll
    for (int hb = 0; hb < 2; ++hb)
#pragma unroll
        for (int uu = 0; uu < 2; ++uu) {
#pragma unroll
            for (int m2 = 0; m2 < 8; ++m2) xb[xb_b(l >> 4, l & 15, m2)] = v[8 * (2 * hb + uu) + m2];
            lds_fence();
#pragma unroll
            for (int hp = 0; hp < 2; ++hp)
#pragma unroll
                for (int kq = 0; kq < 4; ++kq)
                    nv[16 * hp + 8 * hb + 4 * uu + kq] = xb[xb_b(kq, (l >> 3) + 8 * hp, l & 7)];
            lds_fence();
        }
#pragma unroll
    for (int i = 0; i < 32; ++i) v[i] = nv[i];
}

// ---------------------------------------------------------------------------
// twiddle tables (built once per context, staged in LDS by each workgroup)
//   T1[(16 h + k1) * 64 + l] = exp(+2 pi i (l + 64 h) k1 / 2048)
//   T2[k2a * 8 + m2]          = exp(+2 pi i m2 k2a / 128)
// ---------------------------------------------------------------------------
constexpr int kT1Elems = 2048;
constexpr int kT2Elems = 128;
constexpr int kTwElems = kT1Elems + kT2Elems;

// ---------------------------------------------------------------------------
// the transforms
// ---------------------------------------------------------------------------
// Inverse: storage order in, natural order out (unnormalised).
// PRUNE_OUT: only natural indices with k2b < 4 (i.e. < 1024) are produced.
// No scheduling barriers between its passes: the correlation kernels stay
// within their register targets without them and run 2.5-3.6% faster (the
// barriers around the callers' spectrum loads stay: without those the FP32
// kernel took 1.7x as long).
template <bool PRUNE_OUT, bool QUARTER = false, typename T>
__device__ __forceinline__ void ifft2048(T (&v)[32], T *xb, const T *t1, const T *t2, int l)
{
    dft16<true, 0>(v);
    dft16<true, 16>(v);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) v[16 * h + k1] = c_mul(v[16 * h + k1], t1[(16 * h + k1) * 64 + l]);
    }
    if constexpr (QUARTER)
        transpose_a_inv_q(v, xb, l);
    else
        transpose_a_inv(v, xb, l);
    dft16<true, 0>(v);
    dft16<true, 16>(v);
#pragma unroll
    for (int k2a = 1; k2a < 16; ++k2a) {
        const T w = t2[k2a * 8 + (l & 7)];
        v[k2a] = c_mul(v[k2a], w);
        v[16 + k2a] = c_mul(v[16 + k2a], w);
    }
    if constexpr (QUARTER)
        transpose_b_inv_q(v, xb, l);
    else
        transpose_b_inv(v, xb, l);
    dft8<true, false, PRUNE_OUT, 0>(v);
    dft8<true, false, PRUNE_OUT, 8>(v);
    dft8<true, false, PRUNE_OUT, 16>(v);
    dft8<true, false, PRUNE_OUT, 24>(v);
}

// Forward: natural order in, storage order out.
// PRUNE_IN: natural indices >= 1024 (k2b >= 4) are zero on input.
template <bool PRUNE_IN, bool QUARTER = false, typename T>
__device__ __forceinline__ void fft2048(T (&v)[32], T *xb, const T *t1, const T *t2, int l)
{
    dft8<false, PRUNE_IN, false, 0>(v);
    dft8<false, PRUNE_IN, false, 8>(v);
    dft8<false, PRUNE_IN, false, 16>(v);
    dft8<false, PRUNE_IN, false, 24>(v);
    phase_barrier();
    if constexpr (QUARTER)
        transpose_b_fwd_q(v, xb, l);
    else
        transpose_b_fwd(v, xb, l);
    phase_barrier();
#pragma unroll
    for (int k2a = 1; k2a < 16; ++k2a) {
        const T w = t2[k2a * 8 + (l & 7)];
        v[k2a] = c_mulc(v[k2a], w);
        v[16 + k2a] = c_mulc(v[16 + k2a], w);
    }
    phase_barrier();
    dft16<false, 0>(v);
    dft16<false, 16>(v);
    phase_barrier();
    if constexpr (QUARTER)
        transpose_a_fwd_q(v, xb, l);
    else
        transpose_a_fwd(v, xb, l);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        phase_barrier();
#pragma unroll
        for (int k1 = 1; k1 < 16; ++k1) v[16 * h + k1] = c_mulc(v[16 * h + k1], t1[(16 * h + k1) * 64 + l]);
    }
    phase_barrier();
    dft16<false, 0>(v);
    dft16<false, 16>(v);
}

}  // namespace gnss

// pfa1023.hpp -- exact-length 1023-point DFTs on the gfx950 matrix cores.
//
// The length-1023 circular correlations of the polyphase form need no zero
// padding when the transforms have length 1023 = 31 * 33.  Since 31 and 33
// are coprime, the Good-Thomas (prime factor) index maps turn the 1023-point
// DFT into a 31 x 33 two-dimensional DFT with no twiddle factors between the
// two passes:
//   time       m = (33 n1 + 31 n2) mod 1023,   n1 < 31, n2 < 33
//   frequency  k = (528 a + 496 b) mod 1023,   a < 31,  b < 33
//   X[k(a, b)] = sum_{n1, n2} x[m(n1, n2)] W31^(n1 a) W33^(n2 b),  W_L = e^(-2 pi i / L)
// (528 = 33 (33^-1 mod 31) and 496 = 31 (31^-1 mod 33), so k = a mod 31 and
// k = b mod 33; the cross terms of m k are multiples of 1023).  The inverse
// uses the same maps with conjugate weights.
//
// Each pass is a dense complex matrix product, done in real form on
// v_mfma_f32_16x16x32_f16 (FP16 operands, FP32 accumulation).  Lane layout
// (wave64, lane l = 16 g + c): A[c][8 g + j], B[8 g + j][c] (j < 8),
// D[4 g + r][c] (r < 4).  Every accumulation chain uses this one opcode: a
// chain through the accumulator operand across different MFMA opcodes needs
// more wait states than a same-opcode chain, which the hardware forwards.
// Data are the A operands; the DFT weights are fixed B operands held in
// registers.  A pass contracts the K slots (the input index of its length,
// real and imaginary parts) and its D rows are the other dimension, so a
// pass's D tiles, rounded to FP16, are directly the next pass's A operands
// (the D rows 4 g + r become the K slots 8 g + r and 8 g + 4 + r): no data
// moves between lanes.
//
// Layouts (t < 3 tiles of the 33-dimension, s < 2 K steps of the 31-one):
//   spectrum fragment (t, s): lane (g, c) holds the complex values at
//     a = 16 s + 4 g + j, b = 16 t + c, j < 4, as [re j=0..3, im j=0..3] (8 FP16)
//   31-pass output D31[t][n]: lane (g, c), r: Z_part[n1' = 16 (n & 1) + c][b = 16 t + 4 g + r],
//     part = n >> 1 (0 re, 1 im)
//   33-pass K slots: step t < 3 holds b = 16 t + 4 g + (j & 3), part j >> 2 (the
//     last step has b = 32 only, in lanes g = 0)
//   33-pass output D33[u][v]: lane (g, c), r: row 16 u + 4 g + r of the 31-dimension,
//     column n2' = 16 (v >> 1) + c, part v & 1 for v < 4; tile v = 4 holds column
//     32 (re in lane c = 0, im in lane c = 1) in the inverse, and tiles v = 4, 5
//     column 32 + c (re, im; valid for c = 0) in the forward transform.
// Padded slots (a = 31, b >= 33) carry zero weights, so they stay zero.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gnss {
namespace pfa {

constexpr int kN1 = 31, kN2 = 33, kLen = 1023;
constexpr int kKa = 528, kKb = 496;  // frequency map weights
// Stored spectra (block spectra, code spectra): fragments (t, s) for t < 2 as
// 64 lanes x 16 B each (unit (2 t + s) * 64 + lane), then the t = 2 fragments
// of the c = 0 lanes (unit 256 + 4 s + g); every other lane of t = 2 is zero.
constexpr int kUnits = 264;
constexpr int kTailUnit = 256;

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mma32(u4 a, u4 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
}
// two floats to FP16 (round to nearest even), first one in the low half
__device__ __forceinline__ uint32_t pack2(float x, float y)
{
    h2v v = {(_Float16)x, (_Float16)y};
    return __builtin_bit_cast(uint32_t, v);
}

// Weight tables (B fragments, per lane): u4 units frag * 64 + lane.
constexpr int kFragInv31 = 0;   // [s][n], s < 2, n < 4
constexpr int kFragInv33 = 8;   // [t][v], t < 3, v < 5
constexpr int kFragFwd31 = 23;  // [s][n]
constexpr int kFragFwd33 = 31;  // [t][v], t < 3, v < 6
constexpr int kFrags = 49;
constexpr size_t kFragBytes = (size_t)kFrags * 64 * 16;

struct InvB {
    u4 b31[2][4];
    u4 b33[3][5];
};
struct FwdB {
    u4 b31[2][4];
    u4 b33[3][6];
};

__device__ __forceinline__ void load_inv(InvB &B, const u4 *fr, int l)
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int n = 0; n < 4; ++n) B.b31[s][n] = fr[(kFragInv31 + 4 * s + n) * 64 + l];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int v = 0; v < 5; ++v) B.b33[t][v] = fr[(kFragInv33 + 5 * t + v) * 64 + l];
}

__device__ __forceinline__ void load_fwd(FwdB &B, const u4 *fr, int l)
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int n = 0; n < 4; ++n) B.b31[s][n] = fr[(kFragFwd31 + 4 * s + n) * 64 + l];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int v = 0; v < 6; ++v) B.b33[t][v] = fr[(kFragFwd33 + 6 * t + v) * 64 + l];
}

// 31-pass: D31[t][n] = sum_s A[t][s] B31[s][n]
__device__ __forceinline__ void pass31(const u4 (&a)[3][2], const u4 (&b31)[2][4], f4 (&d)[3][4])
{
    const f4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int n = 0; n < 4; ++n) d[t][n] = mma32(a[t][1], b31[1][n], mma32(a[t][0], b31[0][n], z));
}

// The 31-pass output as 33-pass operands (FP16): rows n1' = 16 u + c.
__device__ __forceinline__ void to_pass33(const f4 (&d)[3][4], u4 (&a)[2][3])
{
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const f4 re = d[t][u], im = d[t][u + 2];
            a[u][t] = u4{pack2(re.x, re.y), pack2(re.z, re.w), pack2(im.x, im.y), pack2(im.z, im.w)};
        }
}

template <int NV>
__device__ __forceinline__ void pass33(const u4 (&a)[2][3], const u4 (&b33)[3][NV], f4 (&d)[2][NV])
{
    const f4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < NV; ++v)
            d[u][v] = mma32(a[u][2], b33[2][v], mma32(a[u][1], b33[1][v], mma32(a[u][0], b33[0][v], z)));
}

// Unnormalised inverse DFT of a spectrum held as fragments: out[u][v] as
// described above (5 column tiles).
__device__ __forceinline__ void inverse(const u4 (&a1)[3][2], const InvB &B, f4 (&out)[2][5])
{
    f4 d1[3][4];
    pass31(a1, B.b31, d1);
    u4 a2[2][3];
    to_pass33(d1, a2);
    pass33<5>(a2, B.b33, out);
}

// Forward DFT: out[u][v], 6 column tiles; rows a = 16 u + 4 g + r, columns
// b = 16 (v >> 1) + c, part v & 1.
__device__ __forceinline__ void forward(const u4 (&a1)[3][2], const FwdB &B, f4 (&out)[2][6])
{
    f4 d1[3][4];
    pass31(a1, B.b31, d1);
    u4 a2[2][3];
    to_pass33(d1, a2);
    pass33<6>(a2, B.b33, out);
}

// Time index of (n1, n2) and frequency index of (a, b).
__host__ __device__ __forceinline__ int time_index(int n1, int n2) { return (33 * n1 + 31 * n2) % kLen; }
__host__ __device__ __forceinline__ int freq_index(int a, int b) { return (kKa * a + kKb * b) % kLen; }

}  // namespace pfa
}  // namespace gnss

// Split-bf16 ("bf16 x 3") and plain-bf16 helpers shared by the MFMA kernels.
//
// A float x is carried as hi = bf16(x) and lo = bf16(x - hi) (round to nearest
// even); a product is formed as hi*hi + hi*lo + lo*hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation, dropping the lo*lo term
// (about 2^-16 relative). The plain form keeps hi only and forms hi*hi (operand
// rounding at most 2^-8 relative). Complex numbers are packed as (re, im) bf16 pairs in
// one 32-bit word, element 0 in the low half.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace xo {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));

// (a, b) -> packed hi pair and lo pair
__device__ __forceinline__ void split2(float a, float b, uint32_t& hi, uint32_t& lo) {
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, bf2v));
  const float ah = __builtin_bit_cast(float, hi << 16), bh = __builtin_bit_cast(float, hi & 0xffff0000u);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a - ah, b - bh}, bf2v));
}
// (a, b) -> packed hi and lo pairs as split2, and the pairs of the rotation (b, -a) of
// both, converted from the same values (rounding is odd-symmetric, so they equal
// rot_pos(hi) and rot_pos(lo))
__device__ __forceinline__ void split2_rot(float a, float b, uint32_t& hi, uint32_t& lo, uint32_t& rhi,
                                           uint32_t& rlo) {
  hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{a, b}, bf2v));
  const float la = a - __builtin_bit_cast(float, hi << 16), lb = b - __builtin_bit_cast(float, hi & 0xffff0000u);
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{la, lb}, bf2v));
  rhi = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{b, -a}, bf2v));
  rlo = __builtin_bit_cast(uint32_t, __builtin_convertvector(f2v{lb, -la}, bf2v));
}
// (re, im) -> (-im, re)
__device__ __forceinline__ uint32_t rot_neg(uint32_t x) { return __builtin_amdgcn_alignbit(x, x, 16) ^ 0x8000u; }
// (re, im) -> (im, -re)
__device__ __forceinline__ uint32_t rot_pos(uint32_t x) { return __builtin_amdgcn_alignbit(x, x, 16) ^ 0x80000000u; }

__device__ __forceinline__ f4 mma(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                 0);
}
__device__ __forceinline__ f4 mma3(u4 ah, u4 al, u4 bh, u4 bl, f4 c) {
  c = mma(ah, bh, c);
  c = mma(ah, bl, c);
  c = mma(al, bh, c);
  return c;
}

// NP products per operand pair: 3 (split) or 1 (plain, the lo words unused)
template <int NP>
__device__ __forceinline__ f4 mma_np(u4 ah, u4 al, u4 bh, u4 bl, f4 c) {
  static_assert(NP == 1 || NP == 3, "one or three products");
  if constexpr (NP == 3)
    return mma3(ah, al, bh, bl, c);
  else
    return mma(ah, bh, c);
}

}  // namespace xo

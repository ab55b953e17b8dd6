// Rounding of an FP64 value to bfloat16 in one step (round to nearest, ties
// to even), without the detour through FP32 whose two roundings can differ
// from one: 1 + 2^-8 + 2^-30 goes to 1 + 2^-8 in FP32, a tie that then
// rounds to 1, while the nearest bfloat16 is 1 + 2^-7.
//
// Plain integer arithmetic on the IEEE-754 binary64 pattern, so the same
// function serves the kernels and a host test.  The bfloat16 grid below
// |x| = 2^e (e >= -126) has spacing 2^(e-7); under 2^-126 it is the
// subnormal spacing 2^-133.  Writing the input as sig * 2^ex with an integer
// significand, the result is k * 2^q with k = sig * 2^(ex-q) rounded to an
// integer, and its bit pattern is ((q + 133) << 7) + k for every k the
// rounding can give (k < 128 subnormal, 128 <= k <= 256 normal; k = 256 is
// the carry into the next binade), clamped to infinity at 0x7F80.
#pragma once
#include <stdint.h>

#ifdef __HIP__
#define TR_BF16_FN __host__ __device__ inline
#else
#define TR_BF16_FN inline
#endif

TR_BF16_FN uint16_t bf16_bits_rne(double x) {
  // values that binary32 holds exactly (data that was FP32 or bfloat16)
  // take the one rounding from binary32: add just under half the spacing,
  // plus the parity bit for ties, and drop the low 16 bits
  const float f = (float)x;
  if ((double)f == x) {
    uint32_t v;
    __builtin_memcpy(&v, &f, 4);
    v += 0x7FFFu + ((v >> 16) & 1u);
    return (uint16_t)(v >> 16);
  }
  uint64_t u;
  __builtin_memcpy(&u, &x, 8);
  const uint16_t sign = (uint16_t)((u >> 48) & 0x8000u);
  const int e = (int)((u >> 52) & 0x7FF);
  uint64_t sig = u & ((1ull << 52) - 1);
  if (e == 0x7FF) return (uint16_t)(sign | (sig ? 0x7FC0u : 0x7F80u));  // NaN stays NaN
  if (e == 0 && sig == 0) return sign;
  int ex = -1074;                        // |x| = sig * 2^ex
  if (e) {
    sig |= 1ull << 52;
    ex = e - 1075;
  }
  const int top = 63 - __builtin_clzll(sig);  // floor(log2 |x|) = top + ex
  int q = top + ex - 7;
  if (q < -133) q = -133;
  const int sh = q - ex;                 // low bits of sig below the grid
  uint64_t k;
  if (sh <= 0) {
    k = sig << -sh;                      // on the grid already (sh >= -7 here)
  } else if (sh > 54) {
    k = 0;                               // below a quarter of the spacing
  } else {
    k = sig >> sh;
    const uint64_t rem = sig & ((1ull << sh) - 1), half = 1ull << (sh - 1);
    if (rem > half || (rem == half && (k & 1))) ++k;
  }
  if (k == 0) return sign;
  uint64_t bits = ((uint64_t)(q + 133) << 7) + k;
  if (bits > 0x7F80u) bits = 0x7F80u;
  return (uint16_t)(sign | bits);
}

#undef TR_BF16_FN

// Exact float32 sums as fixed-point digits, and their rounding to double.
//
// Every finite float32 is m * 2^(k-149) with m < 2^24 and 0 <= k <= 253, so a
// sum of floats is an integer multiple of 2^-149: it is kept as signed
// base-2^32 digits d[0..kDigits) with value sum d[j] * 2^(32j) * 2^-149.  A
// float adds to two digits (k/32 and k/32 + 1); digits are 64-bit, so up to
// 2^31 floats add without overflow.  Host and device share this code.
#pragma once
#include <cstdint>

namespace agg {
namespace gb {

constexpr int kDigits = 9;            // digits a float lands in: k/32 <= 7, plus one
constexpr int kNormDigits = 11;       // after carries (|sum| < 2^31 * 2^128 * 2^149)

// The fixed-point digits of an exact sum, rounded once to double (ties to
// even); `flags` records non-finite items seen (1 NaN, 2 +Inf, 4 -Inf), which
// decide the result as in IEEE addition.  Only static indexing, so on the GPU
// the digits stay in registers.
__host__ __device__ inline double digits_to_double(const int64_t* src, int32_t flags) {
  if ((flags & 1) || ((flags & 2) && (flags & 4))) return __builtin_nan("");
  if (flags & 2) return __builtin_inf();
  if (flags & 4) return -__builtin_inf();
  int64_t d[kNormDigits];
#pragma unroll
  for (int k = 0; k < kNormDigits; ++k) d[k] = k < kDigits ? src[k] : 0;
#pragma unroll
  for (int k = 0; k < kNormDigits - 1; ++k) {  // carries: digits 0..9 into [0, 2^32)
    const int64_t c = d[k] >> 32;
    d[k] -= c * 4294967296ll;
    d[k + 1] += c;
  }
  const bool neg = d[kNormDigits - 1] < 0;
  if (neg) {
#pragma unroll
    for (int k = 0; k < kNormDigits; ++k) d[k] = -d[k];
#pragma unroll
    for (int k = 0; k < kNormDigits - 1; ++k) {
      const int64_t c = d[k] >> 32;
      d[k] -= c * 4294967296ll;
      d[k + 1] += c;
    }
  }
  // |sum| < 2^308 * 2^-149, so the top digit is zero and all are in [0, 2^32)
  int t = -1;  // highest nonzero digit
#pragma unroll
  for (int k = 0; k < kNormDigits; ++k)
    if (d[k] != 0) t = k;
  if (t < 0) return 0.0;
  // V = w2:w1:w0, digits t, t-1, t-2 (zero below digit 0); lower digits only
  // decide the sticky bit
  uint64_t w2 = 0, w1 = 0, w0 = 0;
  bool sticky = false;
#pragma unroll
  for (int k = 0; k < kNormDigits; ++k) {
    const uint64_t v = (uint64_t)d[k];
    if (k == t) w2 = v;
    if (k == t - 1) w1 = v;
    if (k == t - 2) w0 = v;
    if (k < t - 2) sticky |= v != 0;
  }
  const int p = 95 - __builtin_clz((uint32_t)w2);  // highest set bit of V, 64..95
  const int sh = p - 52;                            // low bits rounded away, 12..43
  const uint64_t hi = (w2 << 32) | w1;              // V = hi * 2^32 + w0
  uint64_t mant, rnd;
  if (sh <= 32) {
    mant = (hi << (32 - sh)) | (w0 >> sh);
    rnd = (w0 >> (sh - 1)) & 1u;
    sticky |= (w0 & ((1ull << (sh - 1)) - 1)) != 0;
  } else {
    const int r = sh - 33;  // the rounding bit's index in hi
    mant = hi >> (sh - 32);
    rnd = (hi >> r) & 1u;
    sticky |= (hi & ((1ull << r) - 1)) != 0 || w0 != 0;
  }
  int e = sh + 32 * (t - 2) - 149;
  if (rnd && (sticky || (mant & 1))) {
    ++mant;
    if (mant == (1ull << 53)) {
      mant >>= 1;
      ++e;
    }
  }
  const double r = __builtin_ldexp((double)mant, e);
  return neg ? -r : r;
}

}  // namespace gb
}  // namespace agg

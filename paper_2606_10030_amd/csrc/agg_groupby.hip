// Group-by aggregation on gfx950: SUM / MIN / MAX / COUNT / AVG per distinct
// key, keys int32 / int64, values int32 / int64 / float32.
//
// Table: open addressing over a power-of-two number of slots, keys claimed
// with a 64-bit compare-and-swap (INT64_MIN marks an empty slot; the key
// INT64_MIN itself lives in one extra slot), linear probing bounded by the
// table size -- no thread ever waits on another.  Each workgroup first
// aggregates into its own table in LDS (a few probes per item; items whose
// key finds no LDS slot go straight to the global table) and flushes the
// LDS table once at the end, so low-cardinality inputs cost LDS atomics
// rather than contended global ones.
//
// Determinism: integer SUM (mod 2^64), MIN, MAX and COUNT are exact in any
// order.  A float32 SUM is accumulated exactly: every float is m * 2^(k-149)
// with m < 2^24, added as two integer digits of a base-2^32 fixed-point
// number (12 digits per group), so the group sum is exact whatever the order
// and is rounded once to double at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "agg.h"
#include "agg_internal.hpp"

namespace agg {
namespace gb {

constexpr int64_t kEmpty = INT64_MIN;
constexpr int kDigits = 12;
constexpr int kThreads = 256;
constexpr int kLdsProbes = 16;

enum GOp { G_COUNT = 0, G_SUM_INT, G_MIN_INT, G_MAX_INT, G_SUM_F32, G_MIN_F32, G_MAX_F32 };

struct Table {
  int64_t* key;        // cap + 1 slots; slot cap holds the key INT64_MIN
  uint64_t* cnt;
  int64_t* val;        // integer SUM / MIN / MAX; float MIN / MAX as order-preserving ints
  int64_t* dig;        // float SUM: kDigits per slot
  int32_t* flags;      // float SUM: 1 NaN, 2 +Inf, 4 -Inf seen
  int32_t* state;      // [0] slot cap used, [1] overflow, [2..3] emitted count (uint64)
  int64_t cap;
};

struct Args {
  Table t;
  const void* keys;
  const void* vals;
  int64_t n;
  agg_group* out;
  int64_t max_groups;
  int64_t* ngroups;
  int32_t is_avg;
  int32_t op;
};

template <int G>
constexpr int64_t val_identity() {
  return (G == G_MIN_INT || G == G_MIN_F32) ? INT64_MAX : (G == G_MAX_INT || G == G_MAX_F32) ? INT64_MIN : 0;
}
template <int G>
constexpr int lds_slots() { return G == G_SUM_F32 ? 256 : 2048; }

__device__ __forceinline__ uint64_t mix64(uint64_t k) {  // MurmurHash3's 64-bit finaliser
  k ^= k >> 33;
  k *= 0xFF51AFD7ED558CCDull;
  k ^= k >> 33;
  k *= 0xC4CEB9FE1A85EC53ull;
  k ^= k >> 33;
  return k;
}

// Order-preserving map of non-NaN floats to int32 (and back).
__device__ __forceinline__ int32_t f32_order(float f) {
  const int32_t b = __float_as_int(f);
  return b >= 0 ? b : (b ^ 0x7FFFFFFF);
}
__device__ __forceinline__ float f32_unorder(int32_t o) { return __int_as_float(o >= 0 ? o : (o ^ 0x7FFFFFFF)); }

// The two fixed-point digits of a finite float (value = sum d[k] 2^(32k) 2^-149).
__device__ __forceinline__ void f32_digits(float x, int* k0, int64_t* lo, int64_t* hi) {
  const uint32_t bits = __float_as_uint(x);
  const uint32_t biased = (bits >> 23) & 0xFFu, frac = bits & 0x7FFFFFu;
  const uint64_t m = biased ? (frac | 0x800000u) : frac;
  const int k = biased ? (int)biased - 1 : 0;
  const uint64_t v = m << (k & 31);
  int64_t l = (int64_t)(v & 0xFFFFFFFFu), h = (int64_t)(v >> 32);
  if (bits >> 31) {
    l = -l;
    h = -h;
  }
  *k0 = k >> 5;
  *lo = l;
  *hi = h;
}

template <int KD>
__device__ __forceinline__ int64_t load_key(const void* p, int64_t i) {
  if constexpr (KD == AGG_I32) return (int64_t) static_cast<const int32_t*>(p)[i];
  else return static_cast<const int64_t*>(p)[i];
}
template <int VD>
__device__ __forceinline__ int64_t load_ival(const void* p, int64_t i) {
  if constexpr (VD == AGG_I32) return (int64_t) static_cast<const int32_t*>(p)[i];
  else return static_cast<const int64_t*>(p)[i];
}

// Fold one item into a slot (LDS or global: the pointers decide).
template <int G>
__device__ __forceinline__ void apply(uint64_t* cnt, int64_t* val, int64_t* dig, int32_t* flags, int64_t iv,
                                      float fv) {
  atomicAdd(reinterpret_cast<unsigned long long*>(cnt), 1ull);
  if constexpr (G == G_SUM_INT) atomicAdd(reinterpret_cast<unsigned long long*>(val), (unsigned long long)iv);
  if constexpr (G == G_MIN_INT) atomicMin(reinterpret_cast<long long*>(val), (long long)iv);
  if constexpr (G == G_MAX_INT) atomicMax(reinterpret_cast<long long*>(val), (long long)iv);
  if constexpr (G == G_MIN_F32 || G == G_MAX_F32) {
    if (!__builtin_isnan(fv)) {
      if constexpr (G == G_MIN_F32) atomicMin(reinterpret_cast<long long*>(val), (long long)f32_order(fv));
      else atomicMax(reinterpret_cast<long long*>(val), (long long)f32_order(fv));
    }
  }
  if constexpr (G == G_SUM_F32) {
    if (!__builtin_isfinite(fv)) {
      atomicOr(flags, __builtin_isnan(fv) ? 1 : (fv > 0 ? 2 : 4));
    } else {
      int k;
      int64_t lo, hi;
      f32_digits(fv, &k, &lo, &hi);
      if (lo) atomicAdd(reinterpret_cast<unsigned long long*>(dig + k), (unsigned long long)lo);
      if (hi) atomicAdd(reinterpret_cast<unsigned long long*>(dig + k + 1), (unsigned long long)hi);
    }
  }
}

// The global slot of key k, claiming an empty one; -1 when the table is full.
__device__ __forceinline__ int64_t global_slot(const Table& t, int64_t k) {
  if (k == kEmpty) {
    t.state[0] = 1;
    return t.cap;
  }
  const uint64_t mask = (uint64_t)t.cap - 1;
  uint64_t s = mix64((uint64_t)k) & mask;
  for (int64_t p = 0; p < t.cap; ++p, s = (s + 1) & mask) {
    const int64_t cur = t.key[s];
    if (cur == k) return (int64_t)s;
    if (cur == kEmpty) {
      const int64_t prev = (int64_t)atomicCAS(reinterpret_cast<unsigned long long*>(t.key + s),
                                              (unsigned long long)kEmpty, (unsigned long long)k);
      if (prev == kEmpty || prev == k) return (int64_t)s;
    }
  }
  t.state[1] = 1;  // overflow: more distinct keys than the table holds
  return -1;
}

template <int G>
__device__ __forceinline__ void apply_global(const Table& t, int64_t s, int64_t iv, float fv) {
  apply<G>(t.cnt + s, t.val + s, t.dig + (G == G_SUM_F32 ? s * kDigits : 0), t.flags + s, iv, fv);
}

template <int KD, int VD, int G>
__global__ void __launch_bounds__(kThreads) gb_aggregate_kernel(Args a) {
  constexpr int L = lds_slots<G>();
  constexpr bool kDig = G == G_SUM_F32;
  __shared__ int64_t lkey[L];
  __shared__ uint64_t lcnt[L];
  __shared__ int64_t lval[kDig ? 1 : L];
  __shared__ int64_t ldig[kDig ? L * kDigits : 1];
  __shared__ int32_t lflags[kDig ? L : 1];
  const Table& t = a.t;
  for (int e = threadIdx.x; e < L; e += kThreads) {
    lkey[e] = kEmpty;
    lcnt[e] = 0;
    if constexpr (!kDig) lval[e] = val_identity<G>();
    if constexpr (kDig) {
      lflags[e] = 0;
      for (int d = 0; d < kDigits; ++d) ldig[e * kDigits + d] = 0;
    }
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < a.n; i += stride) {
    const int64_t k = load_key<KD>(a.keys, i);
    int64_t iv = 0;
    float fv = 0.0f;
    if constexpr (G != G_COUNT) {
      if constexpr (VD == AGG_F32) fv = static_cast<const float*>(a.vals)[i];
      else iv = load_ival<VD>(a.vals, i);
    }
    int s = -1;
    if (k != kEmpty) {
      int h = (int)(mix64((uint64_t)k) & (L - 1));
      for (int p = 0; p < kLdsProbes; ++p, h = (h + 1) & (L - 1)) {
        const int64_t cur = lkey[h];
        if (cur == k) { s = h; break; }
        if (cur == kEmpty) {
          const int64_t prev = (int64_t)atomicCAS(reinterpret_cast<unsigned long long*>(&lkey[h]),
                                                  (unsigned long long)kEmpty, (unsigned long long)k);
          if (prev == kEmpty || prev == k) { s = h; break; }
        }
      }
    }
    if (s >= 0) {
      apply<G>(&lcnt[s], kDig ? nullptr : &lval[s], kDig ? &ldig[s * kDigits] : nullptr,
               kDig ? &lflags[s] : nullptr, iv, fv);
    } else {
      const int64_t g = global_slot(t, k);
      if (g >= 0) apply_global<G>(t, g, iv, fv);
    }
  }
  __syncthreads();
  // flush this workgroup's LDS table into the global table
  for (int e = threadIdx.x; e < L; e += kThreads) {
    const int64_t k = lkey[e];
    if (k == kEmpty) continue;
    const int64_t g = global_slot(t, k);
    if (g < 0) continue;
    atomicAdd(reinterpret_cast<unsigned long long*>(t.cnt + g), (unsigned long long)lcnt[e]);
    if constexpr (G == G_SUM_INT) atomicAdd(reinterpret_cast<unsigned long long*>(t.val + g), (unsigned long long)lval[e]);
    if constexpr (G == G_MIN_INT || G == G_MIN_F32) atomicMin(reinterpret_cast<long long*>(t.val + g), (long long)lval[e]);
    if constexpr (G == G_MAX_INT || G == G_MAX_F32) atomicMax(reinterpret_cast<long long*>(t.val + g), (long long)lval[e]);
    if constexpr (kDig) {
      if (lflags[e]) atomicOr(t.flags + g, lflags[e]);
      for (int d = 0; d < kDigits; ++d) {
        const int64_t v = ldig[e * kDigits + d];
        if (v) atomicAdd(reinterpret_cast<unsigned long long*>(t.dig + g * kDigits + d), (unsigned long long)v);
      }
    }
  }
}

template <int G>
__global__ void __launch_bounds__(kThreads) gb_init_kernel(Table t) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x; s <= t.cap; s += stride) {
    t.key[s] = s == t.cap ? INT64_MIN : kEmpty;
    t.cnt[s] = 0;
    t.val[s] = val_identity<G>();
    t.flags[s] = 0;
    if constexpr (G == G_SUM_F32)
      for (int d = 0; d < kDigits; ++d) t.dig[s * kDigits + d] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x < 4) t.state[threadIdx.x] = 0;
}

// The fixed-point digits of an exact sum, rounded once to double (ties to even).
__device__ double digits_to_double(const int64_t* src, int32_t flags) {
  if ((flags & 1) || ((flags & 2) && (flags & 4))) return __builtin_nan("");
  if (flags & 2) return __builtin_inf();
  if (flags & 4) return -__builtin_inf();
  int64_t d[kDigits];
  for (int k = 0; k < kDigits; ++k) d[k] = src[k];
  for (int k = 0; k < kDigits - 1; ++k) {  // carries: digits 0..10 into [0, 2^32)
    const int64_t c = d[k] >> 32;
    d[k] -= c * 4294967296ll;
    d[k + 1] += c;
  }
  const bool neg = d[kDigits - 1] < 0;
  if (neg) {
    for (int k = 0; k < kDigits; ++k) d[k] = -d[k];
    for (int k = 0; k < kDigits - 1; ++k) {
      const int64_t c = d[k] >> 32;
      d[k] -= c * 4294967296ll;
      d[k + 1] += c;
    }
  }
  auto bit = [&](int b) -> uint64_t { return (uint64_t)(d[b >> 5] >> (b & 31)) & 1u; };
  int top = -1;
  for (int b = 32 * kDigits - 1; b >= 0; --b)
    if (bit(b)) { top = b; break; }
  if (top < 0) return 0.0;
  uint64_t mant = 0;
  int e = 0;
  if (top <= 52) {
    for (int b = top; b >= 0; --b) mant = (mant << 1) | bit(b);
  } else {
    for (int b = top; b >= top - 52; --b) mant = (mant << 1) | bit(b);
    e = top - 52;
    const uint64_t rnd = bit(top - 53);
    bool sticky = false;
    for (int b = top - 54; b >= 0 && !sticky; --b) sticky = bit(b);
    if (rnd && (sticky || (mant & 1))) {
      ++mant;
      if (mant == (1ull << 53)) {
        mant >>= 1;
        ++e;
      }
    }
  }
  const double r = __builtin_ldexp((double)mant, e - 149);
  return neg ? -r : r;
}

template <int G>
__global__ void __launch_bounds__(kThreads) gb_emit_kernel(Args a) {
  const Table& t = a.t;
  unsigned long long* emitted = reinterpret_cast<unsigned long long*>(t.state + 2);
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x; s <= t.cap; s += stride) {
    const bool used = s < t.cap ? t.key[s] != kEmpty : t.state[0] != 0;
    if (!used) continue;
    const unsigned long long idx = atomicAdd(emitted, 1ull);
    if ((int64_t)idx >= a.max_groups) continue;
    agg_group g;
    g.key = t.key[s];
    g.count = (int64_t)t.cnt[s];
    g.i64 = 0;
    g.f64 = 0.0;
    if constexpr (G == G_COUNT) {
      g.i64 = g.count;
      g.f64 = (double)g.count;
    } else if constexpr (G == G_SUM_INT) {
      g.i64 = t.val[s];
      g.f64 = a.is_avg ? (double)g.i64 / (double)g.count : (double)g.i64;
    } else if constexpr (G == G_MIN_INT || G == G_MAX_INT) {
      g.i64 = t.val[s];
      g.f64 = (double)g.i64;
    } else if constexpr (G == G_SUM_F32) {
      const double sum = digits_to_double(t.dig + s * kDigits, t.flags[s]);
      g.f64 = a.is_avg ? sum / (double)g.count : sum;
    } else {  // float MIN / MAX: NaN when every item of the group is NaN
      const int64_t v = t.val[s];
      g.f64 = v == val_identity<G>() ? (double)__builtin_nanf("") : (double)f32_unorder((int32_t)v);
    }
    a.out[idx] = g;
  }
}

__global__ void gb_finish_kernel(Args a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const unsigned long long e = *reinterpret_cast<const unsigned long long*>(a.t.state + 2);
    *a.ngroups = (a.t.state[1] || (int64_t)e > a.max_groups) ? -1 : (int64_t)e;
  }
}

int gop_of(int32_t val_dtype, int32_t op) {
  if (op == AGG_COUNT) return G_COUNT;
  const bool f = val_dtype == AGG_F32;
  if (op == AGG_SUM || op == AGG_AVG) return f ? G_SUM_F32 : G_SUM_INT;
  if (op == AGG_MIN) return f ? G_MIN_F32 : G_MIN_INT;
  if (op == AGG_MAX) return f ? G_MAX_F32 : G_MAX_INT;
  return -1;
}

template <int KD, int VD>
const void* agg_row(int g) {
  if constexpr (VD == AGG_F32) {
    switch (g) {
      case G_COUNT: return reinterpret_cast<const void*>(&gb_aggregate_kernel<KD, VD, G_COUNT>);
      case G_SUM_F32: return reinterpret_cast<const void*>(&gb_aggregate_kernel<KD, VD, G_SUM_F32>);
      case G_MIN_F32: return reinterpret_cast<const void*>(&gb_aggregate_kernel<KD, VD, G_MIN_F32>);
      case G_MAX_F32: return reinterpret_cast<const void*>(&gb_aggregate_kernel<KD, VD, G_MAX_F32>);
      default: return nullptr;
    }
  } else {
    switch (g) {
      case G_COUNT: return reinterpret_cast<const void*>(&gb_aggregate_kernel<KD, VD, G_COUNT>);
      case G_SUM_INT: return reinterpret_cast<const void*>(&gb_aggregate_kernel<KD, VD, G_SUM_INT>);
      case G_MIN_INT: return reinterpret_cast<const void*>(&gb_aggregate_kernel<KD, VD, G_MIN_INT>);
      case G_MAX_INT: return reinterpret_cast<const void*>(&gb_aggregate_kernel<KD, VD, G_MAX_INT>);
      default: return nullptr;
    }
  }
}

template <int KD>
const void* agg_kernel(int32_t vd, int g) {
  switch (vd) {
    case AGG_I32: return agg_row<KD, AGG_I32>(g);
    case AGG_I64: return agg_row<KD, AGG_I64>(g);
    case AGG_F32: return agg_row<KD, AGG_F32>(g);
    default: return nullptr;
  }
}

const void* init_kernel(int g) {
  switch (g) {
    case G_COUNT: return reinterpret_cast<const void*>(&gb_init_kernel<G_COUNT>);
    case G_SUM_INT: return reinterpret_cast<const void*>(&gb_init_kernel<G_SUM_INT>);
    case G_MIN_INT: return reinterpret_cast<const void*>(&gb_init_kernel<G_MIN_INT>);
    case G_MAX_INT: return reinterpret_cast<const void*>(&gb_init_kernel<G_MAX_INT>);
    case G_SUM_F32: return reinterpret_cast<const void*>(&gb_init_kernel<G_SUM_F32>);
    case G_MIN_F32: return reinterpret_cast<const void*>(&gb_init_kernel<G_MIN_F32>);
    case G_MAX_F32: return reinterpret_cast<const void*>(&gb_init_kernel<G_MAX_F32>);
    default: return nullptr;
  }
}

const void* emit_kernel(int g) {
  switch (g) {
    case G_COUNT: return reinterpret_cast<const void*>(&gb_emit_kernel<G_COUNT>);
    case G_SUM_INT: return reinterpret_cast<const void*>(&gb_emit_kernel<G_SUM_INT>);
    case G_MIN_INT: return reinterpret_cast<const void*>(&gb_emit_kernel<G_MIN_INT>);
    case G_MAX_INT: return reinterpret_cast<const void*>(&gb_emit_kernel<G_MAX_INT>);
    case G_SUM_F32: return reinterpret_cast<const void*>(&gb_emit_kernel<G_SUM_F32>);
    case G_MIN_F32: return reinterpret_cast<const void*>(&gb_emit_kernel<G_MIN_F32>);
    case G_MAX_F32: return reinterpret_cast<const void*>(&gb_emit_kernel<G_MAX_F32>);
    default: return nullptr;
  }
}

}  // namespace gb
}  // namespace agg

using namespace agg;
using namespace agg::gb;

struct agg_groupby_s {
  int device = 0;
  int32_t key_dtype = 0, val_dtype = 0, op = 0;
  int gop = 0;
  int64_t max_n = 0, max_groups = 0;
  void* ws = nullptr;
  Table t{};
};

extern "C" {

int agg_groupby_plan(agg_groupby_t* out, int32_t key_dtype, int32_t val_dtype, int32_t op, int64_t max_n,
                     int64_t max_groups) {
  if (!out) return AGG_E_INVALID;
  *out = nullptr;
  const int g = gop_of(val_dtype, op);
  if ((key_dtype != AGG_I32 && key_dtype != AGG_I64) || width_of(val_dtype) == 0 || g < 0) return AGG_E_INVALID;
  if (max_n < 0 || max_groups < 1 || max_groups > ((int64_t)1 << 32)) return AGG_E_INVALID;
  if (g == G_SUM_F32 && max_n > ((int64_t)1 << 31)) return AGG_E_INVALID;  // digit headroom
  if (max_n > ((int64_t)1 << 40)) return AGG_E_INVALID;
  int dev = 0;
  const int dr = current_device(&dev);
  if (dr != AGG_OK) return dr;
  int64_t cap = 64;
  while (cap < 2 * max_groups) cap <<= 1;
  const int64_t slots = cap + 1;
  const bool dig = g == G_SUM_F32;
  auto up = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
  const int64_t b_key = up(slots * 8), b_cnt = up(slots * 8), b_val = up(slots * 8);
  const int64_t b_dig = dig ? up(slots * 8 * kDigits) : 256, b_flags = up(slots * 4), b_state = 256;
  agg_groupby_s* p = new (std::nothrow) agg_groupby_s();
  if (!p) return AGG_E_NOMEM;
  if (hipMalloc(&p->ws, (size_t)(b_key + b_cnt + b_val + b_dig + b_flags + b_state)) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return AGG_E_NOMEM;
  }
  char* base = static_cast<char*>(p->ws);
  p->t.key = reinterpret_cast<int64_t*>(base);
  p->t.cnt = reinterpret_cast<uint64_t*>(base + b_key);
  p->t.val = reinterpret_cast<int64_t*>(base + b_key + b_cnt);
  p->t.dig = reinterpret_cast<int64_t*>(base + b_key + b_cnt + b_val);
  p->t.flags = reinterpret_cast<int32_t*>(base + b_key + b_cnt + b_val + b_dig);
  p->t.state = reinterpret_cast<int32_t*>(base + b_key + b_cnt + b_val + b_dig + b_flags);
  p->t.cap = cap;
  p->device = dev;
  p->key_dtype = key_dtype;
  p->val_dtype = val_dtype;
  p->op = op;
  p->gop = g;
  p->max_n = max_n;
  p->max_groups = max_groups;
  *out = p;
  return AGG_OK;
}

int agg_groupby_run(agg_groupby_t p, const void* keys, const void* vals, int64_t n, agg_group* groups,
                    int64_t* ngroups, void* stream_v) {
  if (!p || !groups || !ngroups || n < 0 || n > p->max_n || (n > 0 && (!keys || !vals))) return AGG_E_INVALID;
  const int kw = width_of(p->key_dtype), vw = width_of(p->val_dtype);
  if (n > 0 && (reinterpret_cast<uintptr_t>(keys) % (uintptr_t)kw || reinterpret_cast<uintptr_t>(vals) % (uintptr_t)vw))
    return AGG_E_INVALID;
  if (n > 0) {
    int rc = check_pointer(keys, n * kw, AGG_SRC_DEVICE, p->device);
    if (rc == AGG_OK) rc = check_pointer(vals, n * vw, AGG_SRC_DEVICE, p->device);
    if (rc != AGG_OK) return rc;
  }
  int rc = check_out_pointer(groups, p->max_groups * (int64_t)sizeof(agg_group), p->device);
  if (rc == AGG_OK) rc = check_out_pointer(ngroups, sizeof(int64_t), p->device);
  if (rc != AGG_OK) return rc;
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  const int cu = device_cu(p->device);
  Args a;
  a.t = p->t;
  a.keys = keys;
  a.vals = vals;
  a.n = n;
  a.out = groups;
  a.max_groups = p->max_groups;
  a.ngroups = ngroups;
  a.is_avg = p->op == AGG_AVG;
  a.op = p->op;
  const int64_t table_grid = std::min<int64_t>(ceil_div(p->t.cap + 1, kThreads), (int64_t)cu * 8);
  rc = launch(init_kernel(p->gop), (int)std::max<int64_t>(table_grid, 1), kThreads, &a.t, stream);
  if (rc != AGG_OK) return rc;
  if (n > 0) {
    const void* fn = p->key_dtype == AGG_I32 ? agg_kernel<AGG_I32>(p->val_dtype, p->gop)
                                             : agg_kernel<AGG_I64>(p->val_dtype, p->gop);
    if (!fn) return AGG_E_INVALID;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kThreads * 16), (int64_t)cu * 4));
    rc = launch(fn, (int)grid, kThreads, &a, stream);
    if (rc != AGG_OK) return rc;
  }
  rc = launch(emit_kernel(p->gop), (int)std::max<int64_t>(table_grid, 1), kThreads, &a, stream);
  if (rc != AGG_OK) return rc;
  return launch(reinterpret_cast<const void*>(&gb_finish_kernel), 1, 64, &a, stream);
}

int agg_groupby_destroy(agg_groupby_t p) {
  if (!p) return AGG_E_INVALID;
  (void)hipDeviceSynchronize();
  if (p->ws) (void)hipFree(p->ws);
  delete p;
  return AGG_OK;
}

}  // extern "C"

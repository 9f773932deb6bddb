// Group-by aggregation on gfx950: SUM / MIN / MAX / COUNT / AVG per distinct
// key, keys int32 / int64, values int32 / int64 / float32.
//
// Table: open addressing over a power-of-two number of slots, keys claimed
// with a 64-bit compare-and-swap (INT64_MIN marks an empty slot; the key
// INT64_MIN itself lives in one extra slot), linear probing bounded by the
// table size -- no thread ever waits on another.  Rows are first aggregated
// into a workgroup's own table in LDS (a few probes per row; a row whose key
// finds no LDS slot goes straight to the global table) and each LDS table is
// flushed into the global table once, so the global table sees one update
// per (workgroup, key) instead of one per row.
//
// Two paths, chosen from the plan's max_groups:
//  * direct: workgroups stride over the rows; every workgroup's LDS table
//    holds all the groups in at most half of its slots (or, with up to twice
//    that many, in two passes over the rows, each taking the keys of one half
//    of the hash space).
//  * partitioned (more groups): rows are processed in chunks; each chunk is
//    radix-partitioned on the top bits of the key's hash (histogram, prefix
//    sums, scatter into a staging copy), so that one partition has few enough
//    distinct keys for an LDS table, and then one workgroup (or several, for
//    a partition with many rows) aggregates each partition in LDS (in several
//    passes, one per sub-partition, where the scatter's partitions are too
//    few for that).
//
// Determinism: integer SUM (mod 2^64), MIN, MAX and COUNT are exact in any
// order.  A float32 SUM is accumulated exactly: every finite float is
// m * 2^(k-149) with m < 2^24, added as two integer digits of a base-2^32
// fixed-point number, so the group sum is exact whatever the order and is
// rounded once to double at the end.  The row order inside a partition (set
// by LDS atomics) therefore never shows in a result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <new>
#include <type_traits>

#include "agg.h"
#include "agg_digits.hpp"
#include "agg_internal.hpp"

namespace agg {
namespace gb {

constexpr int64_t kEmpty = INT64_MIN;
constexpr int kThreads = 256;
constexpr int kLdsProbes = 16;
constexpr int kAggRows = 8;           // rows whose loads a thread keeps in flight
constexpr int kMaxPartBits = 14;      // at most 16384 (sub-)partitions
constexpr int kMinPartBits = 5;       // at least 32
// Rows are partitioned in chunks of up to 2^28: every chunk ends with each
// aggregation workgroup flushing the groups it holds, so fewer, larger
// chunks flush less (the staging area holds one chunk: up to 4 GiB).
constexpr int64_t kChunkRows = (int64_t)1 << 28;
constexpr int kMaxHistWg = 1024;                   // histogram / scatter workgroups per chunk
constexpr int64_t kMinHistRows = 8192;             // rows per such workgroup, at least
constexpr int kScanThreads = 1024;
constexpr int kTileThreads = 1024;    // scatter: rows staged in LDS per tile
constexpr int kTileMaxBits = 11;      // scatter into at most 2048 partitions
// Rows per scatter tile: as many as LDS holds next to the per-partition
// counters (at most 152 KiB in all), 16 per thread at most (registers).
// Longer tiles give longer runs per partition, so fewer partial cache lines.
// With values, LDS holds keys and values only and the store phase hashes the
// key again; a tile of keys only (COUNT) keeps each row's partition in LDS,
// and below 128 partitions, where runs are long anyway, takes 8192 rows
// (measured: 4% faster there, 3-9% slower above).
template <int KD, int VD, bool HASV, bool BIG>
constexpr int tile_rows() {
  return !HASV ? (!BIG ? 8192 : KD == AGG_I32 ? 16384 : 12288)
               : (KD == AGG_I32 ? 4 : 8) + (VD == AGG_I64 ? 8 : 4) == 8 ? 16384
               : (KD == AGG_I32 ? 4 : 8) + (VD == AGG_I64 ? 8 : 4) == 12 ? 10240 : 8192;
}
constexpr int kBigTileBits = 7;  // key-only tiles grow from 128 partitions on
// A staged row with a value is stored as one record, the key's 32-bit words
// then the value's (8, 12 or 16 bytes, over the keys' and the values'
// staging regions together), so a partition's run in a scatter tile is one
// contiguous run instead of two.
template <int KD, int VD>
struct StagedRow {
  static constexpr int KW = KD == AGG_I32 ? 1 : 2, VW = VD == AGG_I64 ? 2 : 1;
  uint32_t w[KW + VW];
};

enum GOp { G_COUNT = 0, G_SUM_INT, G_MIN_INT, G_MAX_INT, G_SUM_F32, G_MIN_F32, G_MAX_F32 };

// LDS tables: one 1024-thread workgroup per CU with one table of up to
// 148 KiB, on both paths: 8192 slots for 4-byte keys, 4096 for 8-byte keys
// (twice that for COUNT, which keeps no value; 2048 for float sums, whose
// slots carry 7 fixed-point digits).  Measured against three 256-thread
// workgroups per CU with half the slots: fewer, larger tables hold 2x the
// groups at the same load and fold faster.
constexpr int kDirectThreads = 1024;
constexpr int lds_slots_of(int g, int kd) {
  return g == G_SUM_F32 ? 2048 : (g == G_COUNT ? 2 : 1) * (kd == AGG_I32 ? 8192 : 4096);
}
// A float sum's LDS slot keeps digits 1..7 of the 9: a finite float
// m * 2^(k-149) touches digits k/32 and k/32 + 1, both within 1..7 for
// 32 <= k <= 223 (2^-94 <= |x| < 2^98: normal floats of biased exponent
// 33..224).  Zeros add nothing and non-finite floats only set flags; every
// other float is folded straight into the global table.  Seven digits
// instead of nine fit twice the slots in LDS.
constexpr int kLdsDigits = 7;
template <int G, int KD>
constexpr int lds_slots() { return lds_slots_of(G, KD); }
constexpr int kPartThreads = 1024;

struct Table {
  int64_t* key;        // cap + 1 slots; slot cap holds the key INT64_MIN
  uint64_t* cnt;
  int64_t* val;        // integer SUM / MIN / MAX; float MIN / MAX as order-preserving ints
  int64_t* dig;        // float SUM: kDigits per slot
  int32_t* flags;      // float SUM: 1 NaN, 2 +Inf, 4 -Inf seen
  int32_t* state;      // [0] slot cap used, [1] overflow, [2..3] emitted count (uint64)
  int64_t cap;
};

// Radix partitioning of one chunk of rows.
struct Part {
  uint32_t* hist;      // [P][g1]: rows of partition p in scatter workgroup g, then their prefix
  uint32_t* tot;       // [P] rows per partition
  uint32_t* start;     // [P + 1] first staged row of each partition
  void* pk;            // staged keys (one chunk)
  void* pv;            // staged values (none for COUNT)
  int32_t bits;        // log2 of the number of partitions the rows are scattered into
  int32_t sub_bits;    // log2 of the aggregation passes over each of them (one per sub-partition)
  int32_t g1;          // histogram / scatter workgroups of this chunk
  int64_t rows_per_wg; // rows each of them covers
};

struct Args {
  Table t;
  Part pt;
  const void* keys;    // this launch's rows (a chunk in the partitioned path)
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

__device__ __forceinline__ uint64_t mix64(uint64_t k) {  // MurmurHash3's 64-bit finaliser
  k ^= k >> 33;
  k *= 0xFF51AFD7ED558CCDull;
  k ^= k >> 33;
  k *= 0xC4CEB9FE1A85EC53ull;
  k ^= k >> 33;
  return k;
}

__device__ __forceinline__ int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

// The hash of a key that places it in LDS tables and partitions.  int64
// keys: the 64-bit finaliser above.  int32 keys: one 32 x 64-bit multiply by
// an odd constant (2^64 / golden ratio) and a fold of the high half into the
// low one -- two quarter-rate multiplies instead of the finaliser's eight,
// and a bijection on the 32-bit keys; the top bits (partitions, passes) come
// from the product's high half, the low bits (slots) mix both halves, and
// bits 32.. give the probe step.
template <int KD>
__device__ __forceinline__ uint64_t key_hash(int64_t k) {
  if constexpr (KD == AGG_I32) {
    const uint64_t p = (uint64_t)(uint32_t)k * 0x9E3779B97F4A7C15ull;
    return p ^ (p >> 32);
  } else {
    return mix64((uint64_t)k);
  }
}

// Partition of a key: the top bits of its hash (table slots use the low bits).
template <int KD>
__device__ __forceinline__ uint32_t part_of(int64_t k, int bits) {
  return (uint32_t)(key_hash<KD>(k) >> (64 - bits));
}

// The hash placing a key in a few-groups table (at most 256 slots, a single pass):
// one 32-bit multiply by 2^32 / golden ratio instead of key_hash's wider
// product.  Bits 24..31 pick the slot, bits 16..23 the probe step (the
// table reads the slot from the low half and the step from the high half).
// Where a key lands never shows in a result: only the probe count changes.
template <int KD>
__device__ __forceinline__ uint64_t few_hash(int64_t k) {
  uint32_t x = (uint32_t)k;
  if constexpr (KD != AGG_I32) x ^= (uint32_t)((uint64_t)k >> 32);
  const uint32_t h = x * 0x9E3779B1u;
  return ((uint64_t)(h >> 16) << 32) | (h >> 24);
}

// 7 * x for x < 2^24 as one full-rate 24-bit multiply (left to itself the
// compiler issues a quarter-rate 32-bit one for the float-sum slot's digit
// index).
static_assert(kLdsDigits == 7, "mul7_u24 scales by the LDS slot's digit count");
__device__ __forceinline__ uint32_t mul7_u24(uint32_t x) {
  uint32_t r;
  __asm__("v_mul_u32_u24 %0, 7, %1" : "=v"(r) : "v"(x));
  return r;
}

// Order-preserving map of non-NaN floats to int32 (and back).
__device__ __forceinline__ int32_t f32_order(float f) {
  const int32_t b = __float_as_int(f);
  return b >= 0 ? b : (b ^ 0x7FFFFFFF);
}
__device__ __forceinline__ float f32_unorder(int32_t o) { return __int_as_float(o >= 0 ? o : (o ^ 0x7FFFFFFF)); }

// The two fixed-point digits of a finite float (value = sum d[j] 2^(32j) 2^-149).
__device__ __forceinline__ void f32_digits(float x, int* k0, int64_t* lo, int64_t* hi) {
  const uint32_t bits = __float_as_uint(x);
  const uint32_t biased = (bits >> 23) & 0xFFu, frac = bits & 0x7FFFFFu;
  const uint64_t m = biased ? (frac | 0x800000u) : frac;
  const int k = biased ? (int)biased - 1 : 0;
  const uint64_t v = m << (k & 31);  // below 2^55
  // the signed product split as lo + hi * 2^32 with 0 <= lo < 2^32: one
  // 64-bit negation instead of one per digit (digits may take either sign)
  const int64_t sv = (bits >> 31) ? -(int64_t)v : (int64_t)v;
  *k0 = k >> 5;
  *lo = (int64_t)((uint64_t)sv & 0xFFFFFFFFu);
  *hi = sv >> 32;
}

// Whether an LDS float-sum slot (digits 1..7) can take x.
__device__ __forceinline__ bool lds_digits_hold(float x) {
  const uint32_t b = __float_as_uint(x);
  const uint32_t e = (b >> 23) & 0xFFu;
  return (e - 33u) <= 191u || (b << 1) == 0u || e == 0xFFu;
}

// Atomics on a slot of an LDS table (workgroup scope) or of the global
// table (device scope).  The LDS forms name the LDS address space: left to
// infer it, the compiler may merge a row's LDS update with the global one of
// the fallback path into a single generic (flat) atomic, which is far slower
// on LDS than a DS atomic.
typedef __attribute__((address_space(3))) unsigned int lds_u32;
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
typedef __attribute__((address_space(3))) long long lds_i64;
typedef __attribute__((address_space(3))) int lds_i32;

template <bool LDS>
__device__ __forceinline__ void at_add(unsigned int* p, unsigned int v) {
  if constexpr (LDS) __hip_atomic_fetch_add((lds_u32*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else atomicAdd(p, v);
}
template <bool LDS>
__device__ __forceinline__ void at_add(unsigned long long* p, unsigned long long v) {
  if constexpr (LDS) __hip_atomic_fetch_add((lds_u64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else atomicAdd(p, v);
}
template <bool LDS>
__device__ __forceinline__ void at_min(long long* p, long long v) {
  if constexpr (LDS) __hip_atomic_fetch_min((lds_i64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else atomicMin(p, v);
}
template <bool LDS>
__device__ __forceinline__ void at_max(long long* p, long long v) {
  if constexpr (LDS) __hip_atomic_fetch_max((lds_i64*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else atomicMax(p, v);
}
template <bool LDS>
__device__ __forceinline__ void at_or(int* p, int v) {
  if constexpr (LDS) __hip_atomic_fetch_or((lds_i32*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  else atomicOr(p, v);
}

// Fold one row into a slot of an LDS table (LDS) or of the global table.
template <int G, bool LDS, typename CT>
__device__ __forceinline__ void apply(CT* cnt, int64_t* val, int64_t* dig, int32_t* flags, int64_t iv, float fv) {
  if constexpr (sizeof(CT) == 8) at_add<LDS>(reinterpret_cast<unsigned long long*>(cnt), 1ull);
  else at_add<LDS>(reinterpret_cast<unsigned int*>(cnt), 1u);
  if constexpr (G == G_SUM_INT) at_add<LDS>(reinterpret_cast<unsigned long long*>(val), (unsigned long long)iv);
  if constexpr (G == G_MIN_INT) at_min<LDS>(reinterpret_cast<long long*>(val), (long long)iv);
  if constexpr (G == G_MAX_INT) at_max<LDS>(reinterpret_cast<long long*>(val), (long long)iv);
  if constexpr (G == G_MIN_F32 || G == G_MAX_F32) {
    if (!__builtin_isnan(fv)) {
      if constexpr (G == G_MIN_F32) at_min<LDS>(reinterpret_cast<long long*>(val), (long long)f32_order(fv));
      else at_max<LDS>(reinterpret_cast<long long*>(val), (long long)f32_order(fv));
    }
  }
  if constexpr (G == G_SUM_F32) {
    if (!__builtin_isfinite(fv)) {
      at_or<LDS>(flags, __builtin_isnan(fv) ? 1 : (fv > 0 ? 2 : 4));
    } else {
      int k;
      int64_t lo, hi;
      f32_digits(fv, &k, &lo, &hi);
      if (lo) at_add<LDS>(reinterpret_cast<unsigned long long*>(dig + k), (unsigned long long)lo);
      if (hi) at_add<LDS>(reinterpret_cast<unsigned long long*>(dig + k + 1), (unsigned long long)hi);
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
  apply<G, false>(t.cnt + s, t.val + s, t.dig + (G == G_SUM_F32 ? s * kDigits : 0), t.flags + s, iv, fv);
}

// ---- histogram / prefix sums / scatter of the partitioned path ----

template <int KD>
__global__ void __launch_bounds__(kThreads) gb_hist_kernel(Args a) {
  extern __shared__ uint32_t h[];
  const int P = 1 << a.pt.bits;
  for (int e = threadIdx.x; e < P; e += kThreads) h[e] = 0;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * a.pt.rows_per_wg;
  const int64_t hi = std::min<int64_t>(lo + a.pt.rows_per_wg, a.n);
  using KT = typename std::conditional<KD == AGG_I32, int32_t, int64_t>::type;
  // rows base + r * kThreads: one 64-bit clamp per batch, 32-bit offsets per row
  auto load = [&](KT* kk, int64_t base) {
    const int64_t b0 = std::min<int64_t>(base, hi - 1);
    const uint32_t room = (uint32_t)std::min<int64_t>(hi - 1 - b0, (int64_t)kAggRows * kThreads);
#pragma unroll
    for (int r = 0; r < kAggRows; ++r)
      kk[r] = (static_cast<const KT*>(a.keys) + b0)[std::min<uint32_t>((uint32_t)(r * kThreads), room)];
  };
  auto count = [&](KT* kk, int64_t base) {
    const uint32_t left = (uint32_t)std::max<int64_t>(0, std::min<int64_t>(hi - base, (int64_t)kAggRows * kThreads));
#pragma unroll
    for (int r = 0; r < kAggRows; ++r) __asm__ volatile("" : "+v"(kk[r]));
#pragma unroll
    for (int r = 0; r < kAggRows; ++r)
      if ((uint32_t)(r * kThreads) < left) atomicAdd(&h[part_of<KD>((int64_t)kk[r], a.pt.bits)], 1u);
  };
  // two batches alternate, so the next batch's loads are in flight while this
  // one is counted (2^28 rows: 1-3% off the partitioned paths)
  const int64_t first = lo + threadIdx.x, adv = (int64_t)kThreads * kAggRows;
  if (first < hi) {
    KT A[kAggRows], B[kAggRows];
    load(A, first);
    for (int64_t base = first;;) {
      load(B, base + adv);
      count(A, base);
      base += adv;
      if (base >= hi) break;
      load(A, base + adv);
      count(B, base);
      base += adv;
      if (base >= hi) break;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < P; e += kThreads) a.pt.hist[(int64_t)e * a.pt.g1 + blockIdx.x] = h[e];
}

// One wave per partition: exclusive prefix of its per-workgroup counts, in place.
__global__ void __launch_bounds__(kThreads) gb_scan_rows_kernel(Args a) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * (kThreads / 64) + threadIdx.x / 64;
  if (p >= ((int64_t)1 << a.pt.bits)) return;  // whole waves leave together
  uint32_t* row = a.pt.hist + p * a.pt.g1;
  const int q = (a.pt.g1 + 63) / 64;
  uint32_t s = 0;
  for (int j = 0; j < q; ++j) {
    const int idx = lane * q + j;
    if (idx < a.pt.g1) s += row[idx];
  }
  uint32_t incl = s;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  uint32_t run = incl - s;
  for (int j = 0; j < q; ++j) {
    const int idx = lane * q + j;
    if (idx < a.pt.g1) {
      const uint32_t v = row[idx];
      row[idx] = run;
      run += v;
    }
  }
  if (lane == 63) a.pt.tot[p] = incl;
}

// One workgroup: partition starts, the exclusive prefix of the totals.
__global__ void __launch_bounds__(kScanThreads) gb_scan_tot_kernel(Args a) {
  __shared__ uint32_t wsum[kScanThreads / 64];
  const int P = 1 << a.pt.bits;
  const int q = (P + kScanThreads - 1) / kScanThreads;
  const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
  uint32_t sum = 0;
  for (int j = 0; j < q; ++j) {
    const int idx = threadIdx.x * q + j;
    if (idx < P) sum += a.pt.tot[idx];
  }
  uint32_t incl = sum;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t run = incl - sum;
  for (int v = 0; v < w; ++v) run += wsum[v];
  for (int j = 0; j < q; ++j) {
    const int idx = threadIdx.x * q + j;
    if (idx < P) {
      a.pt.start[idx] = run;
      run += a.pt.tot[idx];
    }
  }
  if (threadIdx.x == kScanThreads - 1) a.pt.start[P] = run;  // the last thread ends on the total
}

// Each row lands at its partition's start + this workgroup's prefix (the
// histogram workgroup of the same rows) + its rank among the partition's
// rows of this workgroup.  Each tile of rows is counting-sorted by partition
// in LDS first, so the rows of one partition leave as one contiguous run
// (coalesced stores) instead of one scattered store per row.
template <int KD, int VD, bool HASV, bool BIG>
__global__ void __launch_bounds__(kTileThreads) gb_scatter_tiled_kernel(Args a) {
  using KT = typename std::conditional<KD == AGG_I32, int32_t, int64_t>::type;
  using VT = typename std::conditional<VD == AGG_I64, int64_t, uint32_t>::type;
  constexpr int TR = tile_rows<KD, VD, HASV, BIG>();
  constexpr int R = TR / kTileThreads;
  constexpr int PM = 1 << kTileMaxBits;
  __shared__ KT skey[TR];
  __shared__ VT sval[HASV ? TR : 1];
  __shared__ uint16_t spart[HASV ? 1 : TR];
  __shared__ uint32_t tcnt[PM], toff[PM], cur[PM];
  const int P = 1 << a.pt.bits;
  const int tid = threadIdx.x;
  for (int e = tid; e < P; e += kTileThreads) {
    cur[e] = a.pt.start[e] + a.pt.hist[(int64_t)e * a.pt.g1 + blockIdx.x];
    tcnt[e] = 0;
  }
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * a.pt.rows_per_wg;
  const int64_t hi = std::min<int64_t>(lo + a.pt.rows_per_wg, a.n);
  for (int64_t t0 = lo; t0 < hi; t0 += TR) {
    const int rows = (int)std::min<int64_t>(TR, hi - t0);
    KT k[R];
    VT v[R];
    uint32_t pp[R], rank[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {  // all loads first (rows past the tile re-load its last row)
      const int j = std::min(r * kTileThreads + tid, rows - 1);
      k[r] = static_cast<const KT*>(a.keys)[t0 + j];
      if constexpr (HASV) v[r] = static_cast<const VT*>(a.vals)[t0 + j];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r * kTileThreads + tid < rows) {
        pp[r] = part_of<KD>((int64_t)k[r], a.pt.bits);
        rank[r] = atomicAdd(&tcnt[pp[r]], 1u);
      }
    }
    __syncthreads();
    if (tid < 64) {  // one wave: exclusive prefix of the tile's counts
      const int q = (P + 63) / 64;
      uint32_t sum = 0;
      for (int j = 0; j < q; ++j) sum += (tid * q + j < P) ? tcnt[tid * q + j] : 0u;
      uint32_t incl = sum;
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (tid >= off) incl += y;
      }
      uint32_t run = incl - sum;
      for (int j = 0; j < q; ++j) {
        const int e = tid * q + j;
        if (e < P) {
          toff[e] = run;
          run += tcnt[e];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = r * kTileThreads + tid;
      if (j < rows) {
        const uint32_t d = toff[pp[r]] + rank[r];
        skey[d] = k[r];
        if constexpr (HASV) sval[d] = v[r];
        else spart[d] = (uint16_t)pp[r];
      }
    }
    __syncthreads();
    for (int j = tid; j < rows; j += kTileThreads) {
      uint32_t q;
      if constexpr (HASV) q = part_of<KD>((int64_t)skey[j], a.pt.bits);
      else q = spart[j];
      const uint32_t pos = cur[q] + (uint32_t)j - toff[q];
      if ((int64_t)pos >= a.n) continue;  // cannot happen: counts match the histogram
      if constexpr (HASV) {
        using SR = StagedRow<KD, VD>;
        SR row;
        const uint64_t kb = (uint64_t)(int64_t)skey[j], vb = (uint64_t)sval[j];
        row.w[0] = (uint32_t)kb;
        if constexpr (SR::KW == 2) row.w[1] = (uint32_t)(kb >> 32);
        row.w[SR::KW] = (uint32_t)vb;
        if constexpr (SR::VW == 2) row.w[SR::KW + 1] = (uint32_t)(vb >> 32);
        static_cast<SR*>(a.pt.pk)[pos] = row;
      } else {
        static_cast<KT*>(a.pt.pk)[pos] = skey[j];
      }
    }
    __syncthreads();
    for (int e = tid; e < P; e += kTileThreads) {
      cur[e] += tcnt[e];
      tcnt[e] = 0;
    }
    __syncthreads();
  }
}

// ---- aggregation into LDS tables, flushed into the global table ----

// One workgroup's table: L hashed slots keyed in the key column's own width
// (4-byte keys fit twice the slots of 8-byte ones), plus slot L for the one
// key whose bit pattern marks an empty slot.  Each slot has REP copies of its
// accumulators; lane l of a wave updates copy l % REP, so the lanes of one
// wave instruction whose rows share a key spread over REP addresses (LDS
// atomics on one address serialise), and the flush merges the copies (exact
// integer merges: the results do not depend on REP).
template <int G, int KD, int L_, int NT, int REP = 1>
struct LdsTable {
  using KT = typename std::conditional<KD == AGG_I32, int32_t, int64_t>::type;
  using UKT = typename std::conditional<KD == AGG_I32, unsigned int, unsigned long long>::type;
  static constexpr KT kMark = std::numeric_limits<KT>::min();  // empty hashed slot
  static constexpr int L = L_;
  static constexpr int E = (L + 1) * REP;  // accumulator entries: slot s, copy c at s * REP + c
  static constexpr bool kDig = G == G_SUM_F32;
  static constexpr bool kVal = !kDig && G != G_COUNT;
  static_assert((REP & (REP - 1)) == 0 && REP <= 64, "copies: a power of two, at most a wave");
  static_assert(REP == 1 || L <= 256, "tables with copies take few_hash's 8 slot bits");
  KT key[L];
  uint32_t cnt[E];  // rows per table stay below 2^32 (a workgroup's share is at most 2^28 rows)
  int64_t val[kVal ? E : 1];
  int64_t dig[kDig ? E * kLdsDigits : 1];  // digits 1..7 of a float sum
  int32_t flags[kDig ? E : 1];

  __device__ __forceinline__ void clear() {
    for (int e = threadIdx.x; e < L; e += NT) key[e] = kMark;
    for (int e = threadIdx.x; e < E; e += NT) {
      cnt[e] = 0;
      if constexpr (kVal) val[e] = val_identity<G>();
      if constexpr (kDig) {
        flags[e] = 0;
        for (int d = 0; d < kLdsDigits; ++d) dig[e * kLdsDigits + d] = 0;
      }
    }
  }

  // The slot holding key k (hash hk), claiming an empty one; -1 if none
  // within kLdsProbes probes.  Double hashing: an odd step from the hash's
  // high half, so probe chains do not cluster (a wave waits for its longest
  // chain).
  __device__ __forceinline__ int slot_of(KT k, uint64_t hk) {
    if (k == kMark) return L;
    int h = (int)(hk & (L - 1));
    const int step = (int)(((hk >> 32) | 1) & (L - 1));
    for (int p = 0; p < kLdsProbes; ++p, h = (h + step) & (L - 1)) {
      const KT cur = key[h];
      if (cur == k) return h;
      if (cur == kMark) {
        const KT prev = (KT)atomicCAS(reinterpret_cast<UKT*>(&key[h]), (UKT)kMark, (UKT)k);
        if (prev == kMark || prev == k) return h;
      }
    }
    return -1;
  }

  // Rows first, first + step, ... below last whose key hash has the bits
  // (hash >> sub_shift) & sub_mask equal to sub; a row whose key finds no
  // slot within kLdsProbes goes to the global table.
  // ROWS: keys holds staged (key, value) records.  SUB: the plan has
  // sub-partition passes (else every row belongs to the single pass and the
  // per-row test of its hash bits is left out)
  template <int VD, bool ROWS = false, bool SUB = true>
  __device__ __forceinline__ void fold_rows(const Table& t, const void* keys, const void* vals, int64_t first, int64_t last,
                            int64_t step, uint32_t sub_shift, uint32_t sub_mask, uint32_t sub) {
    constexpr int R = kAggRows;
    using IVT = typename std::conditional<VD == AGG_I64, int64_t, int32_t>::type;
    struct Batch {  // R rows' key and value registers
      KT k[R];
      IVT iv[R];
      float fv[R];
    };
    // rows past the end re-load the last row (in bounds, never folded): no
    // branch around the loads, so all of them issue before the first wait.
    // The batch's rows are base + r * step: one 64-bit clamp per batch, then
    // 32-bit offsets (R * step < 2^31), so a row's address costs a min and one
    // 64-bit add instead of a 64-bit compare, two selects and three adds
    const uint32_t step32 = (uint32_t)step;
    auto load = [&](Batch& b, int64_t base) {
      const int64_t b0 = std::min<int64_t>(base, last - 1);
      const uint32_t room = (uint32_t)std::min<int64_t>(last - 1 - b0, (int64_t)R * step);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const uint32_t rel = std::min<uint32_t>((uint32_t)r * step32, room);
        b.iv[r] = 0;
        b.fv[r] = 0.0f;
        if constexpr (ROWS && G != G_COUNT) {
          using SR = StagedRow<KD, VD == AGG_I64 ? AGG_I64 : AGG_I32>;
          const SR row = (static_cast<const SR*>(keys) + b0)[rel];
          if constexpr (SR::KW == 2) b.k[r] = (KT)(((uint64_t)row.w[1] << 32) | row.w[0]);
          else b.k[r] = (KT)(int32_t)row.w[0];
          if constexpr (VD == AGG_F32) b.fv[r] = __uint_as_float(row.w[SR::KW]);
          else if constexpr (VD == AGG_I64) b.iv[r] = (int64_t)(((uint64_t)row.w[SR::KW + 1] << 32) | row.w[SR::KW]);
          else b.iv[r] = (int32_t)row.w[SR::KW];
        } else {
          b.k[r] = (static_cast<const KT*>(keys) + b0)[rel];
          if constexpr (G != G_COUNT) {
            if constexpr (VD == AGG_F32) b.fv[r] = (static_cast<const float*>(vals) + b0)[rel];
            else b.iv[r] = (static_cast<const IVT*>(vals) + b0)[rel];
          }
        }
      }
    };
    auto fold = [&](Batch& b, int64_t base) {
      // rows of this batch that exist: r * step < last - base
      const uint32_t left = (uint32_t)std::max<int64_t>(0, std::min<int64_t>(last - base, (int64_t)R * step));
      // the batch's loads are complete before its first row is folded: left
      // alone, the compiler sinks a value load into the branch that uses it,
      // and that load's whole latency then stalls the wave
#pragma unroll
      for (int r = 0; r < R; ++r) {
        __asm__ volatile("" : "+v"(b.k[r]));
        if constexpr (G != G_COUNT) {
          if constexpr (VD == AGG_F32) __asm__ volatile("" : "+v"(b.fv[r]));
          else __asm__ volatile("" : "+v"(b.iv[r]));
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if ((uint32_t)r * step32 >= left) break;
        const KT k = b.k[r];
        const uint64_t hk = REP > 1 ? few_hash<KD>(k) : key_hash<KD>((int64_t)k);
        if (SUB && ((uint32_t)(hk >> sub_shift) & sub_mask) != sub) continue;  // another pass's row
        const float fv = b.fv[r];
        bool in_lds = true;
        if constexpr (kDig) in_lds = lds_digits_hold(fv);
        const int slot = in_lds ? slot_of(k, hk) : -1;  // outside the LDS slot's digits: the global table
        if (slot >= 0) {
          const int s = slot * REP + (int)(threadIdx.x & (REP - 1));  // this lane's copy
          if constexpr (kDig) {
            at_add<true>(&cnt[s], 1u);
            if (!__builtin_isfinite(fv)) {
              at_or<true>(&flags[s], __builtin_isnan(fv) ? 1 : (fv > 0 ? 2 : 4));
            } else {  // digit j of the sum sits at dig[s * kLdsDigits + j - 1]
              int dk;
              int64_t dlo, dhi;
              f32_digits(fv, &dk, &dlo, &dhi);
              // both adds unconditionally (no branch per digit): a float the slot
              // holds has 1 <= dk <= 6, and a zero (dk = 0, both digits 0) adds 0
              // to digit slots 0 and 1
              const int j = dk > 0 ? dk - 1 : 0;
              const int e0 = (int)mul7_u24((uint32_t)s) + j;
              at_add<true>(reinterpret_cast<unsigned long long*>(&dig[e0]), (unsigned long long)dlo);
              at_add<true>(reinterpret_cast<unsigned long long*>(&dig[e0 + 1]), (unsigned long long)dhi);
            }
          } else {
            apply<G, true>(&cnt[s], &val[kVal ? s : 0], &dig[0], &flags[0], (int64_t)b.iv[r], fv);
          }
        } else {
          const int64_t g = global_slot(t, (int64_t)k);
          if (g >= 0) apply_global<G>(t, g, (int64_t)b.iv[r], fv);
        }
      }
    };
    if (first >= last) return;
    const int64_t adv = step * R;
    // Rows of at most two 32-bit words (key and value registers): two batches
    // alternate, so the next batch's loads are in flight while this one is
    // folded (2^28 rows, int32 keys: COUNT at 16 groups 0.33 -> 0.25 ms, float
    // SUM at 1024 groups 1.07 -> 0.99 ms).  Wider rows fold one batch at a
    // time: two batches of int64 values took the fold to 128 registers and
    // ran 5-15% slower.  The few-groups table (REP > 1) runs two workgroups
    // per CU, which leaves two batches' registers only to COUNT's key-only rows.
    constexpr int kWords = (KD == AGG_I64 ? 2 : 1) + (G == G_COUNT ? 0 : VD == AGG_I64 ? 2 : 1);
    if constexpr (kWords <= 2 && (REP == 1 || kWords == 1)) {
      Batch A, B;
      load(A, first);
      for (int64_t base = first;;) {
        load(B, base + adv);
        fold(A, base);
        base += adv;
        if (base >= last) break;
        load(A, base + adv);
        fold(B, base);
        base += adv;
        if (base >= last) break;
      }
    } else {
      Batch A;
      for (int64_t base = first; base < last; base += adv) {
        load(A, base);
        fold(A, base);
      }
    }
  }

  __device__ __forceinline__ void flush(const Table& t) {
    // Every workgroup's table holds its keys in about the same slots (same
    // hash), so flushing all tables in slot order would have every workgroup
    // update the same global slots at the same moment, and device-scope
    // atomics on one address serialise.  Each workgroup starts its pass at
    // its own offset instead (2^28 rows, 1024 groups: COUNT 0.43 -> 0.39 ms;
    // the other cases within noise).
    const int off = (int)(((uint32_t)blockIdx.x * 2654435761u) % (uint32_t)(L + 1));
    for (int i = threadIdx.x; i <= L; i += NT) {
      const int e = i + off <= L ? i + off : i + off - (L + 1);
      const KT k = e < L ? key[e] : kMark;
      uint64_t c = 0;
      for (int r = 0; r < REP; ++r) c += cnt[e * REP + r];
      if (e < L ? k == kMark : c == 0) continue;
      const int64_t g = global_slot(t, (int64_t)k);
      if (g < 0) continue;
      atomicAdd(reinterpret_cast<unsigned long long*>(t.cnt + g), (unsigned long long)c);
      if constexpr (kVal) {
        int64_t v = val[e * REP];
        for (int r = 1; r < REP; ++r) {
          const int64_t w = val[e * REP + r];
          if constexpr (G == G_SUM_INT) v = (int64_t)((uint64_t)v + (uint64_t)w);
          else if constexpr (G == G_MIN_INT || G == G_MIN_F32) v = w < v ? w : v;
          else v = w > v ? w : v;
        }
        if constexpr (G == G_SUM_INT) atomicAdd(reinterpret_cast<unsigned long long*>(t.val + g), (unsigned long long)v);
        if constexpr (G == G_MIN_INT || G == G_MIN_F32) atomicMin(reinterpret_cast<long long*>(t.val + g), (long long)v);
        if constexpr (G == G_MAX_INT || G == G_MAX_F32) atomicMax(reinterpret_cast<long long*>(t.val + g), (long long)v);
      }
      if constexpr (kDig) {
        int32_t f = 0;
        for (int r = 0; r < REP; ++r) f |= flags[e * REP + r];
        if (f) atomicOr(t.flags + g, f);
        for (int d = 0; d < kLdsDigits; ++d) {
          uint64_t v = 0;  // digits add mod 2^64, as in the global table
          for (int r = 0; r < REP; ++r) v += (uint64_t)dig[(e * REP + r) * kLdsDigits + d];
          if (v) atomicAdd(reinterpret_cast<unsigned long long*>(t.dig + g * kDigits + d + 1), (unsigned long long)v);
        }
      }
    }
  }
};

// Float sums of few groups (at most kFewGroups): with a full-size table a
// wave's 64 rows fall on about as many slots as there are groups, and the
// LDS atomics of lanes that meet on a slot serialise (measured on MI355X: a
// 64-bit add from a wave whose rows spread over 16 slots takes about 24
// clocks, over 64 addresses 6); a float row makes three (two digits and the
// count).  A small table whose slots carry kFewCopies copies of the
// accumulators (lane l updates copy l % kFewCopies) cuts the meetings by that
// factor.  16 groups, 2^28 rows: 4 copies of 256 slots 0.626 -> 0.594 ms at
// one workgroup per CU; at two (the table is 65 KiB) 0.45-0.48 ms with 4
// copies, 0.44-0.45 with 8 copies of 128 slots and 0.44 with 16 of 64 (the
// 128-slot table keeps 32 groups a quarter full).  COUNT takes the same
// table (4.6 KiB of LDS) with its key loads pipelined and two workgroups per
// CU: 0.253 -> 0.241 ms at 16 groups, 0.255 -> 0.239 at 32 (at one
// workgroup per CU and 4 copies it had been slower: 0.338 -> 0.348 ms).
// Integer sums keep the full table: with copies and two workgroups per CU
// they ran 0.54 -> 0.64 ms at 16 groups.
constexpr int kFewGroups = 32;
constexpr int kFewCopies = 8;
constexpr int kFewSlots = 128;

// Direct path: every workgroup sweeps the rows grid-stride into one LDS
// table, in 2^sub_bits passes (each taking the keys of one sub-partition:
// the top bits of the key's hash) when the groups need more than one table.
// The few-groups table (65 KiB of LDS) leaves room for two workgroups per CU
// when the fold fits 64 registers: 16 groups, 2^28 rows, float SUM 0.60 ->
// 0.49 ms (8 waves per SIMD instead of 4 hide the LDS and memory latency).
template <int KD, int VD, int G, bool FEW, bool SUB>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, kDirectThreads), amdgpu_waves_per_eu(FEW ? 8 : 1)))
gb_aggregate_kernel(Args a) {
  static_assert(!FEW || G == G_SUM_F32 || G == G_COUNT, "the few-groups table is for float sums and counts");
  __shared__ LdsTable<G, KD, FEW ? kFewSlots : lds_slots<G, KD>(), kDirectThreads, FEW ? kFewCopies : 1> tab;
  const uint32_t sub_mask = (1u << a.pt.sub_bits) - 1u;
  const uint32_t sub_shift = a.pt.sub_bits ? (uint32_t)(64 - a.pt.sub_bits) : 0u;
  for (uint32_t sub = 0; sub <= sub_mask; ++sub) {
    tab.clear();
    __syncthreads();
    tab.template fold_rows<VD, false, SUB>(a.t, a.keys, a.vals, (int64_t)blockIdx.x * kDirectThreads + threadIdx.x,
                                           a.n, (int64_t)gridDim.x * kDirectThreads, sub_shift, sub_mask, sub);
    __syncthreads();
    tab.flush(a.t);
    __syncthreads();
  }
}

// Partitioned path: workgroup w takes the w-th equal share of the staged rows
// and folds it partition by partition, flushing its LDS table at each
// partition boundary (a partition's keys fit one table; the next partition's
// keys are all different).  Equal shares keep every workgroup equally busy
// whatever the partition sizes.  Where a partition holds more keys than one
// table (more partitions than the scatter takes), its rows are folded in
// several passes, each taking the rows of one sub-partition (the next bits of
// the key's hash) and flushing the table after it.
template <int KD, int VD, int G, bool SUB>
__global__ void __launch_bounds__(kPartThreads) gb_aggregate_part_kernel(Args a) {
  __shared__ LdsTable<G, KD, lds_slots<G, KD>(), kPartThreads> tab;
  const int P = 1 << a.pt.bits;
  int64_t r = a.n * (int64_t)blockIdx.x / gridDim.x;
  const int64_t r1 = a.n * ((int64_t)blockIdx.x + 1) / gridDim.x;
  if (r >= r1) return;  // the whole workgroup leaves together
  int lo = 0, hi = P - 1;  // the partition holding row r: the last p with start[p] <= r
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if ((int64_t)a.pt.start[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  int p = lo;
  const uint32_t sub_mask = (1u << a.pt.sub_bits) - 1u;
  const uint32_t sub_shift = a.pt.sub_bits ? (uint32_t)(64 - a.pt.bits - a.pt.sub_bits) : 0u;
  while (r < r1) {
    while ((int64_t)a.pt.start[p + 1] <= r) ++p;  // skip partitions that end before r
    const int64_t seg_end = std::min<int64_t>(r1, (int64_t)a.pt.start[p + 1]);
    for (uint32_t sub = 0; sub <= sub_mask; ++sub) {
      tab.clear();
      __syncthreads();
      tab.template fold_rows<VD, true, SUB>(a.t, a.pt.pk, a.pt.pv, r + threadIdx.x, seg_end, kPartThreads,
                                            sub_shift, sub_mask, sub);
      __syncthreads();
      tab.flush(a.t);
      __syncthreads();
    }
    r = seg_end;
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

// Workgroup w writes the used slots of its contiguous slot range: it counts
// them, takes one output range with a single atomic, and each thread writes
// its slots at its prefix within that range (one counter update per
// workgroup: updates of one address serialise).
template <int G>
__global__ void __launch_bounds__(kThreads) gb_emit_kernel(Args a) {
  __shared__ uint32_t wsum[kThreads / 64];
  __shared__ unsigned long long base_sh;
  const Table& t = a.t;
  const int64_t slots = t.cap + 1;
  const int64_t per = ceil_div_dev(slots, gridDim.x);
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = std::min<int64_t>(lo + per, slots);
  auto used = [&](int64_t s) { return s < t.cap ? t.key[s] != kEmpty : t.state[0] != 0; };
  uint32_t mine = 0;
  for (int64_t s = lo + threadIdx.x; s < hi; s += kThreads) mine += used(s) ? 1u : 0u;
  // exclusive prefix of the per-thread counts over the workgroup
  const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
  uint32_t incl = mine;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t before = incl - mine, total = 0;
  for (int v = 0; v < kThreads / 64; ++v) {
    if (v < w) before += wsum[v];
    total += wsum[v];
  }
  if (threadIdx.x == 0)
    base_sh = total ? atomicAdd(reinterpret_cast<unsigned long long*>(t.state + 2), (unsigned long long)total) : 0;
  __syncthreads();
  unsigned long long idx = base_sh + before;
  for (int64_t s = lo + threadIdx.x; s < hi; s += kThreads) {
    if (!used(s)) continue;
    const unsigned long long my = idx++;
    if ((int64_t)my >= a.max_groups) continue;
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
    } else {  // float MIN / MAX: NaN when every row of the group is NaN
      const int64_t v = t.val[s];
      g.f64 = v == val_identity<G>() ? (double)__builtin_nanf("") : (double)f32_unorder((int32_t)v);
    }
    a.out[my] = g;
  }
}

__global__ void gb_finish_kernel(Args a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const unsigned long long e = *reinterpret_cast<const unsigned long long*>(a.t.state + 2);
    *a.ngroups = (a.t.state[1] || (int64_t)e > a.max_groups) ? -1 : (int64_t)e;
  }
}

// ---- kernel tables ----

int gop_of(int32_t val_dtype, int32_t op) {
  if (op == AGG_COUNT) return G_COUNT;
  const bool f = val_dtype == AGG_F32;
  if (op == AGG_SUM || op == AGG_AVG) return f ? G_SUM_F32 : G_SUM_INT;
  if (op == AGG_MIN) return f ? G_MIN_F32 : G_MIN_INT;
  if (op == AGG_MAX) return f ? G_MAX_F32 : G_MAX_INT;
  return -1;
}

// PATH: 0 direct, 1 partitioned, 2 direct for float sums and counts of few
// groups (accumulator copies), 3 direct in sub-partition passes, 4 partitioned in
// sub-partition passes.  Plans without passes take kernels whose fold has no
// per-row pass test.
template <int KD, int VD, int PATH>
const void* agg_row(int g) {
#define GB_AGG(GG)                                                                                        \
  (PATH == 1 || PATH == 4                                                                                 \
       ? reinterpret_cast<const void*>(&gb_aggregate_part_kernel<KD, VD, GG, PATH == 4>)                  \
       : reinterpret_cast<const void*>(&gb_aggregate_kernel<KD, VD, GG, PATH == 2 && (GG == G_SUM_F32 || GG == G_COUNT), PATH == 3>))
  if constexpr (VD == AGG_F32) {
    switch (g) {
      case G_COUNT: return GB_AGG(G_COUNT);
      case G_SUM_F32: return GB_AGG(G_SUM_F32);
      case G_MIN_F32: return GB_AGG(G_MIN_F32);
      case G_MAX_F32: return GB_AGG(G_MAX_F32);
      default: return nullptr;
    }
  } else {
    switch (g) {
      case G_COUNT: return GB_AGG(G_COUNT);
      case G_SUM_INT: return GB_AGG(G_SUM_INT);
      case G_MIN_INT: return GB_AGG(G_MIN_INT);
      case G_MAX_INT: return GB_AGG(G_MAX_INT);
      default: return nullptr;
    }
  }
#undef GB_AGG
}

template <int KD, int PATH>
const void* agg_kernel_kd(int32_t vd, int g) {
  switch (vd) {
    case AGG_I32: return agg_row<KD, AGG_I32, PATH>(g);
    case AGG_I64: return agg_row<KD, AGG_I64, PATH>(g);
    case AGG_F32: return agg_row<KD, AGG_F32, PATH>(g);
    default: return nullptr;
  }
}

template <int KD>
const void* agg_kernel_path(int32_t vd, int g, int path) {
  switch (path) {
    case 1: return agg_kernel_kd<KD, 1>(vd, g);
    case 2: return agg_kernel_kd<KD, 2>(vd, g);
    case 3: return agg_kernel_kd<KD, 3>(vd, g);
    case 4: return agg_kernel_kd<KD, 4>(vd, g);
    default: return agg_kernel_kd<KD, 0>(vd, g);
  }
}

const void* agg_kernel(int32_t kd, int32_t vd, int g, int path) {
  return kd == AGG_I32 ? agg_kernel_path<AGG_I32>(vd, g, path) : agg_kernel_path<AGG_I64>(vd, g, path);
}

template <int KD>
const void* scatter_kd(int32_t vd, bool hasv, int bits) {
  if (!hasv)
    return bits >= kBigTileBits ? reinterpret_cast<const void*>(&gb_scatter_tiled_kernel<KD, AGG_I32, false, true>)
                                : reinterpret_cast<const void*>(&gb_scatter_tiled_kernel<KD, AGG_I32, false, false>);
  if (vd == AGG_I64) return reinterpret_cast<const void*>(&gb_scatter_tiled_kernel<KD, AGG_I64, true, true>);
  return reinterpret_cast<const void*>(&gb_scatter_tiled_kernel<KD, AGG_I32, true, true>);  // 4-byte values move as bits
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

int launch_lds(const void* fn, int64_t grid, int block, size_t lds, Args* args, hipStream_t stream) {
  void* kargs[] = {args};
  const hipError_t e = hipLaunchKernel(fn, dim3((unsigned)grid), dim3(block), kargs, lds, stream);
  if (e != hipSuccess) {
    record_hip_error((int32_t)e);
    (void)hipGetLastError();
    return AGG_E_HIP;
  }
  return AGG_OK;
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
  Part pt{};           // bits == 0: the direct path
  int path = 0;        // 0 direct, 1 partitioned, 2 few-groups float sums, 3 / 4: 0 / 1 in sub-partition passes
  int agg_blocks = 1;  // aggregation workgroups resident per CU
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
  if (max_n > ((int64_t)1 << 36)) return AGG_E_INVALID;
  int dev = 0;
  const int dr = current_device(&dev);
  if (dr != AGG_OK) return dr;
  int64_t cap = 64;
  while (cap < 2 * max_groups) cap <<= 1;
  const int64_t slots = cap + 1;
  const bool dig = g == G_SUM_F32;
  // LDS tables are filled at most half (with double hashing a half-full
  // table still probes fast; measured, linear probing slowed sharply past a
  // quarter): the direct path up to half of its table, or in two passes over
  // the rows up to a whole table's worth, partitions sized for half of
  // theirs.  (Measured on 2^28 rows: two direct passes take 0.65x the
  // partitioned path's time for int64 SUM, about the same for float sums,
  // but 1.09x for COUNT, which moves the fewest bytes when partitioned; each
  // pass costs about one direct run, so four would lose.)
  int bits = 0, direct_sub_bits = 0;
  const int64_t half_table = lds_slots_of(g, key_dtype) / 2;
  if (max_groups > half_table && max_groups <= 2 * half_table && g != G_COUNT) {
    direct_sub_bits = 1;
  } else if (max_groups > half_table) {
    auto bits_for = [max_groups](int64_t per_part) {
      int b = 0;
      while (b < kMaxPartBits && (per_part << b) < max_groups) ++b;
      return b;
    };
    bits = bits_for(half_table);
    bits = std::max(bits, kMinPartBits);  // few partitions would serialise the counting atomics
  }
  // The scatter takes at most 2^kTileMaxBits partitions (its per-partition
  // counters live in LDS, and more would shorten the coalesced runs); past
  // that each partition is folded in 2^sub_bits passes.
  const int sub_bits = bits ? std::max(0, bits - kTileMaxBits) : direct_sub_bits;
  bits -= bits ? sub_bits : 0;
  const int64_t P = bits ? (int64_t)1 << bits : 0;
  const int64_t crow = bits ? std::max<int64_t>(1, std::min<int64_t>(max_n, kChunkRows)) : 0;
  const int kw = width_of(key_dtype), vw = op == AGG_COUNT ? 0 : width_of(val_dtype);
  auto up = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
  const int64_t b_key = up(slots * 8), b_cnt = up(slots * 8), b_val = up(slots * 8);
  const int64_t b_dig = dig ? up(slots * 8 * kDigits) : 256, b_flags = up(slots * 4), b_state = 256;
  const int64_t b_hist = up(P * kMaxHistWg * 4), b_tot = up(P * 4 + 4), b_start = up(P * 4 + 4),
                b_pk = up(crow * kw), b_pv = up(crow * vw);
  const int64_t total = b_key + b_cnt + b_val + b_dig + b_flags + b_state + b_hist + b_tot + b_start +
                        b_pk + b_pv;
  agg_groupby_s* p = new (std::nothrow) agg_groupby_s();
  if (!p) return AGG_E_NOMEM;
  const int arc = device_alloc(&p->ws, (size_t)total);
  if (arc != AGG_OK) {
    delete p;
    return arc;
  }
  char* c = static_cast<char*>(p->ws);
  auto take = [&c](int64_t bytes) {
    char* r = c;
    c += bytes;
    return r;
  };
  p->t.key = reinterpret_cast<int64_t*>(take(b_key));
  p->t.cnt = reinterpret_cast<uint64_t*>(take(b_cnt));
  p->t.val = reinterpret_cast<int64_t*>(take(b_val));
  p->t.dig = reinterpret_cast<int64_t*>(take(b_dig));
  p->t.flags = reinterpret_cast<int32_t*>(take(b_flags));
  p->t.state = reinterpret_cast<int32_t*>(take(b_state));
  p->t.cap = cap;
  p->pt.hist = reinterpret_cast<uint32_t*>(take(b_hist));
  p->pt.tot = reinterpret_cast<uint32_t*>(take(b_tot));
  p->pt.start = reinterpret_cast<uint32_t*>(take(b_start));
  p->pt.pk = take(b_pk);
  p->pt.pv = vw ? take(b_pv) : nullptr;  // right after pk: staged (key, value) records span both
  p->pt.bits = bits;
  p->pt.sub_bits = sub_bits;
  p->device = dev;
  p->key_dtype = key_dtype;
  p->val_dtype = val_dtype;
  p->op = op;
  p->gop = g;
  p->max_n = max_n;
  p->max_groups = max_groups;
  // aggregation grids are sized to what the chip holds at once (no second, mostly idle wave of workgroups)
  int nb = 0;
  // Integer sums of few groups keep the kernel with the per-row pass test
  // (its masks are zero here, so every row passes): their LDS atomics collide
  // on a few addresses, and the leaner fold, which issues them faster, ran
  // slower (16 groups, 2^28 rows: 0.555 against 0.526 ms).
  p->path = bits ? (sub_bits ? 4 : 1)
                 : sub_bits ? 3
                 : max_groups <= kFewGroups ? (g == G_SUM_F32 || g == G_COUNT ? 2 : g == G_SUM_INT ? 3 : 0)
                                            : 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, agg_kernel(key_dtype, val_dtype, g, p->path),
                                                   bits ? kPartThreads : kDirectThreads, 0) !=
          hipSuccess ||
      nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  p->agg_blocks = nb;
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
    if (rc == AGG_OK && p->op != AGG_COUNT) rc = check_pointer(vals, n * vw, AGG_SRC_DEVICE, p->device);
    if (rc != AGG_OK) return rc;
  }
  int rc = check_out_pointer(groups, p->max_groups * (int64_t)sizeof(agg_group), p->device);
  if (rc == AGG_OK) rc = check_out_pointer(ngroups, sizeof(int64_t), p->device);
  if (rc != AGG_OK) return rc;
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  const int cu = device_cu(p->device);
  Args a{};
  a.t = p->t;
  a.pt = p->pt;
  a.keys = keys;
  a.vals = vals;
  a.n = n;
  a.out = groups;
  a.max_groups = p->max_groups;
  a.ngroups = ngroups;
  a.is_avg = p->op == AGG_AVG;
  a.op = p->op;
  const int64_t table_grid = std::max<int64_t>(1, std::min<int64_t>(ceil_div(p->t.cap + 1, kThreads), (int64_t)cu * 8));
  rc = launch(init_kernel(p->gop), (int)table_grid, kThreads, &a.t, stream);
  if (rc != AGG_OK) return rc;
  if (n > 0 && p->pt.bits == 0) {
    const int64_t grid =
        std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, kDirectThreads * 16), (int64_t)cu * p->agg_blocks));
    rc = launch(agg_kernel(p->key_dtype, p->val_dtype, p->gop, p->path), (int)grid, kDirectThreads, &a, stream);
    if (rc != AGG_OK) return rc;
  } else if (n > 0) {
    const int64_t P = (int64_t)1 << p->pt.bits;
    const size_t lds = (size_t)P * 4;
    const bool hasv = p->op != AGG_COUNT;
    const void* hist = p->key_dtype == AGG_I32 ? reinterpret_cast<const void*>(&gb_hist_kernel<AGG_I32>)
                                               : reinterpret_cast<const void*>(&gb_hist_kernel<AGG_I64>);
    const void* scat = p->key_dtype == AGG_I32 ? scatter_kd<AGG_I32>(p->val_dtype, hasv, p->pt.bits)
                                               : scatter_kd<AGG_I64>(p->val_dtype, hasv, p->pt.bits);
    const void* aggk = agg_kernel(p->key_dtype, p->val_dtype, p->gop, p->path);
    for (int64_t c0 = 0; c0 < n; c0 += kChunkRows) {
      const int64_t m = std::min<int64_t>(kChunkRows, n - c0);
      a.keys = static_cast<const char*>(keys) + c0 * kw;
      a.vals = static_cast<const char*>(vals) + c0 * vw;
      a.n = m;
      a.pt.g1 = (int)std::min<int64_t>(kMaxHistWg, ceil_div(m, kMinHistRows));
      a.pt.rows_per_wg = ceil_div(m, a.pt.g1);
      if ((rc = launch_lds(hist, a.pt.g1, kThreads, lds, &a, stream)) != AGG_OK) return rc;
      if ((rc = launch_lds(reinterpret_cast<const void*>(&gb_scan_rows_kernel), ceil_div(P, kThreads / 64), kThreads,
                           0, &a, stream)) != AGG_OK)
        return rc;
      if ((rc = launch_lds(reinterpret_cast<const void*>(&gb_scan_tot_kernel), 1, kScanThreads, 0, &a, stream)) !=
          AGG_OK)
        return rc;
      if ((rc = launch_lds(scat, a.pt.g1, kTileThreads, 0, &a, stream)) != AGG_OK)
        return rc;
      const int64_t agrid =
          std::max<int64_t>(1, std::min<int64_t>(ceil_div(m, kPartThreads * 8), (int64_t)cu * p->agg_blocks));
      if ((rc = launch_lds(aggk, agrid, kPartThreads, 0, &a, stream)) != AGG_OK) return rc;
    }
    a.keys = keys;
    a.vals = vals;
    a.n = n;
  }
  rc = launch(emit_kernel(p->gop), (int)table_grid, kThreads, &a, stream);
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

// Device building blocks of the aggregation scan (gfx950, wave64).
//
// The scan reads every item of a column once and folds it into one summary
// (paper Section 2.1, Figure 4).  Its GPU form follows the specialised design
// of Section 3.2 -- coalesced streaming reads, accumulation in registers, a
// local reduction per group of threads, then one merge of the group partials
// -- rebuilt for CDNA4: 16-byte loads per lane, one segment per wave, a DPP /
// permlane butterfly inside the wave, and a fixed-order merge of segment
// partials by the last workgroup to finish.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "agg.h"
#include "agg_internal.hpp"

namespace agg {

constexpr int kWave = 64;
constexpr int kVecBytes = 16;
constexpr int kRoundBytes = kWave * kVecBytes;  // one wave-wide load: 1 KiB
constexpr int kCombineLanes = 256;              // lanes of the canonical final combine

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ loads
// Columns live in global memory (device memory, or pinned host memory mapped
// into the device's address space), and the loads say so: a column address
// the compiler cannot trace to a kernel argument (one read from a batch work
// record) would otherwise get flat loads.
typedef __attribute__((address_space(1))) const u32x4 global_u32x4;
typedef __attribute__((address_space(1))) const uint32_t global_u32;
typedef __attribute__((address_space(1))) const uint64_t global_u64;

template <bool NT>
__device__ __forceinline__ u32x4 load_vec_aligned(const char* p) {
  global_u32x4* q = (global_u32x4*)p;
  if constexpr (NT) return __builtin_nontemporal_load(q);
  else return *q;
}

// 16 bytes at an address aligned only to the item width W (4 or 8).
template <bool NT, int W>
__device__ __forceinline__ u32x4 load_vec_unaligned(const char* p) {
  u32x4 v;
  if constexpr (W == 4) {
    global_u32* q = (global_u32*)p;
    v[0] = q[0]; v[1] = q[1]; v[2] = q[2]; v[3] = q[3];
  } else {
    global_u64* q = (global_u64*)p;
    uint64_t a = q[0], b = q[1];
    v[0] = (uint32_t)a; v[1] = (uint32_t)(a >> 32); v[2] = (uint32_t)b; v[3] = (uint32_t)(b >> 32);
  }
  return v;
}

// One item of type T (ragged tails).
template <typename T>
__device__ __forceinline__ T load_item(const char* p) {
  return *(__attribute__((address_space(1))) const T*)p;
}

template <bool NT, bool AL, int W>
__device__ __forceinline__ u32x4 load_vec(const char* p) {
  if constexpr (AL) return load_vec_aligned<NT>(p);
  else return load_vec_unaligned<NT, W>(p);
}

// ------------------------------------------------------------ fold traits
// Each trait gives: item width W and items per vector V; the lane
// accumulator `acc` with identity / add_vec / add_item / merge; the segment
// partial `part` (what is stored per segment) with to_part / pidentity /
// pmerge.  merge and pmerge are commutative bit for bit, so both lanes of a
// butterfly pair hold the same value after each step.

__device__ __forceinline__ int32_t as_i32(uint32_t v) { return (int32_t)v; }
__device__ __forceinline__ float as_f32(uint32_t v) { return __uint_as_float(v); }
__device__ __forceinline__ uint64_t as_u64(uint32_t lo, uint32_t hi) {
  return ((uint64_t)hi << 32) | lo;
}

template <int K> struct Fold;

// SUM of int32 into int64 (two's complement, mod 2^64)
template <> struct Fold<K_SUM_I32> {
  static constexpr int W = 4, V = 4;
  using acc = uint64_t; using part = uint64_t;
  static __device__ acc identity() { return 0; }
  static __device__ void add_item(acc& a, const char* p) { a += (uint64_t)(int64_t)load_item<int32_t>(p); }
  static __device__ void add_vec(acc* a, u32x4 x) {
    for (int k = 0; k < 4; ++k) a[k] += (uint64_t)(int64_t)as_i32(x[k]);
  }
  static __device__ acc merge(acc a, acc b) { return a + b; }
  static __device__ part to_part(acc a) { return a; }
  static __device__ part pidentity() { return 0; }
  static __device__ part pmerge(part a, part b) { return a + b; }
};

template <> struct Fold<K_SUM_I64> {
  static constexpr int W = 8, V = 2;
  using acc = uint64_t; using part = uint64_t;
  static __device__ acc identity() { return 0; }
  static __device__ void add_item(acc& a, const char* p) { a += load_item<uint64_t>(p); }
  static __device__ void add_vec(acc* a, u32x4 x) { a[0] += as_u64(x[0], x[1]); a[1] += as_u64(x[2], x[3]); }
  static __device__ acc merge(acc a, acc b) { return a + b; }
  static __device__ part to_part(acc a) { return a; }
  static __device__ part pidentity() { return 0; }
  static __device__ part pmerge(part a, part b) { return a + b; }
};

template <bool IS_MIN> struct FoldMinMaxI32 {
  static constexpr int W = 4, V = 4;
  using acc = int32_t; using part = int64_t;
  static __device__ acc identity() { return IS_MIN ? INT32_MAX : INT32_MIN; }
  static __device__ acc merge(acc a, acc b) { return IS_MIN ? min(a, b) : max(a, b); }
  static __device__ void add_item(acc& a, const char* p) { a = merge(a, load_item<int32_t>(p)); }
  static __device__ void add_vec(acc* a, u32x4 x) { for (int k = 0; k < 4; ++k) a[k] = merge(a[k], as_i32(x[k])); }
  static __device__ part to_part(acc a) { return (int64_t)a; }
  static __device__ part pidentity() { return IS_MIN ? INT64_MAX : INT64_MIN; }
  static __device__ part pmerge(part a, part b) { return IS_MIN ? min(a, b) : max(a, b); }
};
template <> struct Fold<K_MIN_I32> : FoldMinMaxI32<true> {};
template <> struct Fold<K_MAX_I32> : FoldMinMaxI32<false> {};

template <bool IS_MIN> struct FoldMinMaxI64 {
  static constexpr int W = 8, V = 2;
  using acc = int64_t; using part = int64_t;
  static __device__ acc identity() { return IS_MIN ? INT64_MAX : INT64_MIN; }
  static __device__ acc merge(acc a, acc b) { return IS_MIN ? min(a, b) : max(a, b); }
  static __device__ void add_item(acc& a, const char* p) { a = merge(a, load_item<int64_t>(p)); }
  static __device__ void add_vec(acc* a, u32x4 x) {
    a[0] = merge(a[0], (int64_t)as_u64(x[0], x[1]));
    a[1] = merge(a[1], (int64_t)as_u64(x[2], x[3]));
  }
  static __device__ part to_part(acc a) { return a; }
  static __device__ part pidentity() { return identity(); }
  static __device__ part pmerge(part a, part b) { return merge(a, b); }
};
template <> struct Fold<K_MIN_I64> : FoldMinMaxI64<true> {};
template <> struct Fold<K_MAX_I64> : FoldMinMaxI64<false> {};

// Plain float32 lanes.  PLAIN keeps float partials (float combine);
// F64C widens each segment's float total to double (double combine).
template <bool WIDE> struct FoldSumF32 {
  static constexpr int W = 4, V = 4;
  using acc = float;
  using part = typename std::conditional<WIDE, double, float>::type;
  static __device__ acc identity() { return 0.0f; }
  static __device__ void add_item(acc& a, const char* p) { a += load_item<float>(p); }
  static __device__ void add_vec(acc* a, u32x4 x) { for (int k = 0; k < 4; ++k) a[k] += as_f32(x[k]); }
  static __device__ acc merge(acc a, acc b) { return a + b; }
  static __device__ part to_part(acc a) { return (part)a; }
  static __device__ part pidentity() { return (part)0; }
  static __device__ part pmerge(part a, part b) { return a + b; }
};
template <> struct Fold<K_SUM_F32_PLAIN> : FoldSumF32<false> {};
template <> struct Fold<K_SUM_F32_F64C> : FoldSumF32<true> {};

// Neumaier-compensated float32: (s, c) with s + c tracking the running sum.
//
// The correction c gathers the exact rounding errors of the s additions, but
// c's own float32 additions round too; left alone, after m items those
// roundings can reach about m^2 u^2 sum|x| (the quadratic term of the bound for
// cascaded summation, Ogita, Rump and Oishi, SIAM J. Sci. Comput. 26(6),
// 2005, Prop. 4.5).  So every kNeuRenormRounds rounds the pair is
// renormalised by an exact two-sum, (s, c) <- (fl(s + c), error): the value
// s + c is unchanged and |c| drops back to at most u |s|.  The correction then
// only ever sums a few errors, and the rounding it adds is linear in m:
// at most ceil(m / R) * R (R + 3) / 2 * u^2 * sum|x| for R rounds per block
// (R = 8: 44 ceil(m / 8) u^2 sum|x|).
struct NeuPair { float s, c; };
constexpr int kNeuRenormRounds = 8;
template <> struct Fold<K_SUM_F32_NEU> {
  static constexpr int W = 4, V = 4;
  using acc = NeuPair; using part = double;
  static __device__ acc identity() { return {0.0f, 0.0f}; }
  // Knuth's two-sum: t = fl(a + b) and the exact error e = a + b - t, for
  // operands of any magnitude (Knuth, TAOCP vol. 2, 4.2.2).  e is unique, so
  // the pair does not depend on the operand order.
  static __device__ __forceinline__ acc two_sum(float a, float b) {
    const float t = a + b;
    const float bb = t - a;
    return {t, (a - (t - bb)) + (b - bb)};
  }
  // Neumaier's update: the rounding error of s + x is recovered exactly by
  // subtracting in the order that puts the larger magnitude first.
  static __device__ __forceinline__ void add(acc& a, float x) {
    float t = a.s + x;
    bool s_big = fabsf(a.s) >= fabsf(x);
    float big = s_big ? a.s : x;
    float small = s_big ? x : a.s;
    a.c += (big - t) + small;
    a.s = t;
  }
  static __device__ __forceinline__ acc renorm(acc a) { return two_sum(a.s, a.c); }
  static __device__ void add_item(acc& a, const char* p) { add(a, load_item<float>(p)); }
  static __device__ void add_vec(acc* a, u32x4 x) { for (int k = 0; k < 4; ++k) add(a[k], as_f32(x[k])); }
  // Two renormalised pairs: the exact two-sum of the leading parts, its error
  // joins the corrections, and the result is renormalised again.  Every step
  // is symmetric in the operands, so merge(a, b) and merge(b, a) agree bit
  // for bit.
  static __device__ acc merge(acc a, acc b) {
    const acc t = two_sum(a.s, b.s);
    return two_sum(t.s, (a.c + b.c) + t.c);
  }
  static __device__ part to_part(acc a) { return (double)a.s + (double)a.c; }
  static __device__ part pidentity() { return 0.0; }
  static __device__ part pmerge(part a, part b) { return a + b; }
};

// Rounds a lane folds between two renormalisations of its accumulators
// (0: the fold keeps no compensation to renormalise).
template <int K>
constexpr int renorm_rounds() { return K == K_SUM_F32_NEU ? kNeuRenormRounds : 0; }

template <int K>
__device__ __forceinline__ void renorm_all(typename Fold<K>::acc* a) {
  if constexpr (K == K_SUM_F32_NEU) {
#pragma unroll
    for (int v = 0; v < Fold<K>::V; ++v) a[v] = Fold<K>::renorm(a[v]);
  }
}

// After a lane has folded round r of its segment: renormalise when r closes a
// block of renorm_rounds rounds.  The blocks are fixed by the round index, so
// they fall at the same items whatever the number of loads in flight.
template <int K>
__device__ __forceinline__ void round_done(typename Fold<K>::acc* a, int64_t r) {
  constexpr int R = renorm_rounds<K>();
  if constexpr (R > 0) {
    if ((r + 1) % R == 0) renorm_all<K>(a);
  }
}

// The same inside an unrolled group of U rounds starting at round r0, a
// multiple of U: when U is a multiple of the block length, position u alone
// decides it (at compile time); otherwise the round index does.
template <int K, int U, int u>
__device__ __forceinline__ void round_done_unrolled(typename Fold<K>::acc* a, int64_t r0) {
  constexpr int R = renorm_rounds<K>();
  if constexpr (R > 0) {
    if constexpr (U % R == 0) {
      if constexpr ((u + 1) % R == 0) renorm_all<K>(a);
    } else {
      round_done<K>(a, r0 + u);
    }
  }
}

template <bool IS_MIN> struct FoldMinMaxF32 {
  static constexpr int W = 4, V = 4;
  using acc = float; using part = float;
  // fminf / fmaxf: IEEE minNum / maxNum, a NaN operand yields the other one.
  static __device__ acc identity() { return __builtin_nanf(""); }
  static __device__ acc merge(acc a, acc b) { return IS_MIN ? fminf(a, b) : fmaxf(a, b); }
  static __device__ void add_item(acc& a, const char* p) { a = merge(a, load_item<float>(p)); }
  static __device__ void add_vec(acc* a, u32x4 x) { for (int k = 0; k < 4; ++k) a[k] = merge(a[k], as_f32(x[k])); }
  static __device__ part to_part(acc a) { return a; }
  static __device__ part pidentity() { return identity(); }
  static __device__ part pmerge(part a, part b) { return merge(a, b); }
};
template <> struct Fold<K_MIN_F32> : FoldMinMaxF32<true> {};
template <> struct Fold<K_MAX_F32> : FoldMinMaxF32<false> {};

// COUNT: +1 per item covered; the loads are never used, so none are issued.
template <int WB> struct FoldCount {
  static constexpr int W = WB, V = 16 / WB;
  using acc = uint64_t; using part = uint64_t;
  static __device__ acc identity() { return 0; }
  static __device__ void add_item(acc& a, const char*) { a += 1; }
  static __device__ void add_vec(acc* a, u32x4) { for (int k = 0; k < V; ++k) a[k] += 1; }
  static __device__ acc merge(acc a, acc b) { return a + b; }
  static __device__ part to_part(acc a) { return a; }
  static __device__ part pidentity() { return 0; }
  static __device__ part pmerge(part a, part b) { return a + b; }
};
template <> struct Fold<K_COUNT_4> : FoldCount<4> {};
template <> struct Fold<K_COUNT_8> : FoldCount<8> {};

// ------------------------------------------------------------ lane moves
// DPP / permlane moves of any 4-byte-multiple value, one 32-bit word at a time.
template <int CTRL, class T>
__device__ __forceinline__ T dpp_move(T v) {
  static_assert(sizeof(T) % 4 == 0, "dpp_move needs 32-bit words");
  constexpr int NW = sizeof(T) / 4;
  int w[NW];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < NW; ++i) w[i] = __builtin_amdgcn_update_dpp(0, w[i], CTRL, 0xF, 0xF, false);
  T r;
  __builtin_memcpy(&r, w, sizeof(T));
  return r;
}

// v_permlane16_swap with both operands = v: `lo` gets the even 16-lane row of
// each row pair at every position, `hi` the odd row.  v_permlane32_swap does
// the same for the two 32-lane halves.
template <bool SWAP32, class T>
__device__ __forceinline__ void permlane_split(T v, T& lo, T& hi) {
  constexpr int NW = sizeof(T) / 4;
  unsigned w[NW], a[NW], b[NW];
  __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    if constexpr (SWAP32) {
      auto r = __builtin_amdgcn_permlane32_swap(w[i], w[i], false, false);
      a[i] = r[0]; b[i] = r[1];
    } else {
      auto r = __builtin_amdgcn_permlane16_swap(w[i], w[i], false, false);
      a[i] = r[0]; b[i] = r[1];
    }
  }
  __builtin_memcpy(&lo, a, sizeof(T));
  __builtin_memcpy(&hi, b, sizeof(T));
}

constexpr int kDppQuadXor1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppRowHalfMirror = 0x141; // lane i <- 7 - i within 8 lanes
constexpr int kDppRowMirror = 0x140;     // lane i <- 15 - i within 16 lanes

// The fixed wave64 butterfly.  Needs all 64 lanes active; every lane ends
// with the same total.
template <class T, class M>
__device__ __forceinline__ T wave_reduce(T x, M merge) {
  x = merge(x, dpp_move<kDppQuadXor1>(x));
  x = merge(x, dpp_move<kDppQuadXor2>(x));
  x = merge(x, dpp_move<kDppRowHalfMirror>(x));
  x = merge(x, dpp_move<kDppRowMirror>(x));
  T lo, hi;
  permlane_split<false>(x, lo, hi);
  x = merge(lo, hi);
  permlane_split<true>(x, lo, hi);
  return merge(lo, hi);
}

// ------------------------------------------------------------ segment fold
// Fold U loaded rounds in order (fold_round(u) folds round u of the group),
// renormalising where a block closes.
template <int K, int U, class FR, int... us>
__device__ __forceinline__ void fold_unrolled(typename Fold<K>::acc* a, int64_t r0, FR&& fold_round,
                                              std::integer_sequence<int, us...>) {
  ((fold_round(us), round_done_unrolled<K, U, us>(a, r0)), ...);
}


// One wave folds one segment: lane l reads the 16-byte vectors at
// seg + r * 1024 + 16 * l, r = 0, 1, ..., each component into its own
// accumulator in order of r.  `valid` is the segment's byte count (a
// multiple of the item width); U loads are kept in flight per lane.
template <int K, int U, bool NT, bool AL>
__device__ __forceinline__ typename Fold<K>::acc fold_segment(const char* __restrict__ seg,
                                                               int64_t valid, int lane) {
  using F = Fold<K>;
  const int64_t full = valid / kRoundBytes;
  if constexpr (K == K_COUNT_4 || K == K_COUNT_8) {
    // +1 per item this lane covers: V per full round, then its share of the
    // partial round -- the same coverage as the loads below, in closed form.
    const int rem = (int)(valid - full * kRoundBytes);
    const int lo = lane * kVecBytes;
    uint64_t c = (uint64_t)full * F::V;
    if (lo + kVecBytes <= rem) c += F::V;
    else if (lo < rem) c += (uint64_t)((rem - lo) / F::W);
    return c;
  }
  typename F::acc a[F::V];
#pragma unroll
  for (int v = 0; v < F::V; ++v) a[v] = F::identity();
  const char* p = seg + lane * kVecBytes;
  int64_t r = 0;
  if constexpr (K == K_SUM_F32_NEU && U <= 8) {
    // The compensated fold costs several operations an item: the next U
    // rounds' loads are issued before the current U are folded, so a wave's
    // arithmetic overlaps its own memory wait (same rounds, same order).
    // Two groups of loads in flight take 8 registers a round: up to U = 8.
    if (U <= full) {
      u32x4 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = load_vec<NT, AL, F::W>(p + u * kRoundBytes);
      for (; r + 2 * U <= full; r += U) {
        u32x4 y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) y[u] = load_vec<NT, AL, F::W>(p + (r + U + u) * kRoundBytes);
        fold_unrolled<K, U>(a, r, [&](int u) { F::add_vec(a, x[u]); }, std::make_integer_sequence<int, U>());
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = y[u];
      }
      fold_unrolled<K, U>(a, r, [&](int u) { F::add_vec(a, x[u]); }, std::make_integer_sequence<int, U>());
      r += U;
    }
  } else {
    for (; r + U <= full; r += U) {
      u32x4 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = load_vec<NT, AL, F::W>(p + (r + u) * kRoundBytes);
      fold_unrolled<K, U>(a, r, [&](int u) { F::add_vec(a, x[u]); }, std::make_integer_sequence<int, U>());
    }
  }
  for (; r < full; ++r) {
    F::add_vec(a, load_vec<NT, AL, F::W>(p + r * kRoundBytes));
    round_done<K>(a, r);
  }
  const int rem = (int)(valid - full * kRoundBytes);
  if (rem > 0) {
    const int lo = lane * kVecBytes;
    const char* q = p + full * kRoundBytes;
    if (lo + kVecBytes <= rem) {
      F::add_vec(a, load_vec<NT, AL, F::W>(q));
    } else if (lo < rem) {
      for (int k = 0; k * F::W < rem - lo; ++k) F::add_item(a[k], q + k * F::W);
    }
  }
  renorm_all<K>(a);  // close the last block (the partial round joins it)
  if constexpr (F::V == 4) return F::merge(F::merge(a[0], a[1]), F::merge(a[2], a[3]));
  else return F::merge(a[0], a[1]);
}

template <int K>
struct AccMerge {
  __device__ typename Fold<K>::acc operator()(typename Fold<K>::acc a, typename Fold<K>::acc b) const {
    return Fold<K>::merge(a, b);
  }
};
template <int K>
struct PartMerge {
  __device__ typename Fold<K>::part operator()(typename Fold<K>::part a, typename Fold<K>::part b) const {
    return Fold<K>::pmerge(a, b);
  }
};

// ------------------------------------------------------------ final combine
// The canonical merge of nseg segment partials by 256 virtual lanes in four
// virtual waves: lane L folds partials L, L + 256, ... in order, the wave
// butterfly merges each virtual wave, and the four totals merge as
// (w0 + w1) + (w2 + w3).  A workgroup of any size runs it (each physical wave
// takes virtual waves w, w + W, ...), so the bits do not depend on the block
// size.  Every thread of the workgroup must call it; thread 0 gets the total.
// COHERENT: the partials were stored in the same launch by other workgroups,
// so each is read with a device-scope load (served from the level every XCD
// sees rather than from this XCD's L2; about a microsecond per round trip).
template <bool COHERENT, typename P>
__device__ __forceinline__ P load_partial(const P* p) {
  if constexpr (COHERENT)
    return __hip_atomic_load(const_cast<P*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}

// M virtual waves (vw0, vw0 + stride, ...; those >= 4 are skipped) folded by
// one physical wave at once.  Each round issues all of its loads before it
// merges any (16 per lane: B per virtual wave), predicated on the index, so
// a short tail costs one round trip like a full round; the merges then run
// in each virtual lane's canonical order.  Indices are 32-bit (a column has
// at most kSegTarget partials).
template <int K, bool COHERENT, int M>
__device__ __forceinline__ void fold_virtual_waves(const typename Fold<K>::part* __restrict__ part, int nseg,
                                                   int vw0, int stride, int lane, typename Fold<K>::part* lds) {
  using F = Fold<K>;
  using P = typename F::part;
  constexpr int kVirtualWaves = kCombineLanes / kWave;
  constexpr int B = 16 / M;
  P acc[M];
#pragma unroll
  for (int m = 0; m < M; ++m) acc[m] = F::pidentity();
  for (int k0 = 0; k0 < nseg; k0 += B * kCombineLanes) {
    P v[M][B];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int vw = vw0 + m * stride;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = k0 + b * kCombineLanes + vw * kWave + lane;
        if (vw < kVirtualWaves && i < nseg) v[m][b] = load_partial<COHERENT>(part + i);
      }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int vw = vw0 + m * stride;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = k0 + b * kCombineLanes + vw * kWave + lane;
        if (vw < kVirtualWaves && i < nseg) acc[m] = F::pmerge(acc[m], v[m][b]);
      }
    }
  }
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int vw = vw0 + m * stride;
    if (vw < kVirtualWaves) {
      const P t = wave_reduce(acc[m], PartMerge<K>());
      if (lane == 0) lds[vw] = t;
    }
  }
}

template <int K, bool COHERENT = false>
__device__ typename Fold<K>::part combine_partials(const typename Fold<K>::part* __restrict__ part,
                                                   int64_t nseg64) {
  using F = Fold<K>;
  using P = typename F::part;
  constexpr int kVirtualWaves = kCombineLanes / kWave;
  __shared__ P lds[kVirtualWaves];
  const int nseg = (int)nseg64;
  const int lane = threadIdx.x & (kWave - 1);
  const int W = blockDim.x / kWave;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if constexpr (!COHERENT) {
    // the merge launches: four-wave workgroups, one virtual wave each
    for (int vw = w; vw < kVirtualWaves; vw += W) fold_virtual_waves<K, false, 1>(part, nseg, vw, W, lane, lds);
  } else if (w < kVirtualWaves) {
    // the in-launch merge runs on the scan's workgroup: a wave takes virtual
    // waves w, w + W, ... at once (four with one wave per workgroup, at most
    // two with two or three, one with four or more)
    if (W == 1)
      fold_virtual_waves<K, true, 4>(part, nseg, w, W, lane, lds);
    else if (W < kVirtualWaves)
      fold_virtual_waves<K, true, 2>(part, nseg, w, W, lane, lds);
    else
      fold_virtual_waves<K, true, 1>(part, nseg, w, W, lane, lds);
  }
  __syncthreads();
  P total = F::pidentity();
  if (threadIdx.x == 0) total = F::pmerge(F::pmerge(lds[0], lds[1]), F::pmerge(lds[2], lds[3]));
  // lds is free again only when thread 0 has read it: a second call in the
  // same workgroup (the filtered merge takes two) must not overwrite it first
  __syncthreads();
  return total;
}

// ------------------------------------------------------------ finalise
template <int K>
__device__ agg_result finalize(typename Fold<K>::part t, int64_t n, bool is_avg, int32_t prec_used) {
  agg_result r;
  r.i64 = 0; r.f64 = 0.0; r.count = n; r.is_null = 0; r.prec_used = prec_used;
  if constexpr (K == K_COUNT_4 || K == K_COUNT_8) {
    r.i64 = (int64_t)t; r.f64 = (double)(int64_t)t;
  } else if constexpr (K == K_SUM_I32 || K == K_SUM_I64) {
    int64_t s = (int64_t)t;
    r.i64 = s;
    if (is_avg) {
      if (n == 0) r.is_null = 1; else r.f64 = (double)s / (double)n;
    } else {
      r.f64 = (double)s;
    }
  } else if constexpr (K == K_MIN_I32 || K == K_MAX_I32 || K == K_MIN_I64 || K == K_MAX_I64) {
    if (n == 0) r.is_null = 1; else { r.i64 = (int64_t)t; r.f64 = (double)(int64_t)t; }
  } else if constexpr (K == K_MIN_F32 || K == K_MAX_F32) {
    if (n == 0) r.is_null = 1; else r.f64 = (double)t;
  } else {  // float sums
    double s = (double)t;
    if (is_avg) {
      if (n == 0) r.is_null = 1; else r.f64 = s / (double)n;
    } else {
      r.f64 = s;
    }
  }
  return r;
}

}  // namespace agg

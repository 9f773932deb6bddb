// Fused filter + aggregate: SUM / MIN / MAX / COUNT / AVG of the items of a
// value column whose companion item in a filter column lies in a range.
//
// The value column keeps its canonical shape (segments, lane mapping, merge
// order); an unselected item is replaced by the fold's identity, so the
// same code path folds it and an always-true predicate reproduces agg_run.
// Each lane also counts its selected items; segment counts merge exactly and
// finalise AVG and the null flags.
#include "agg_device.hpp"
#include "agg_internal.hpp"

namespace agg {
namespace {

// The 32-bit words of the fold identity for one item (the low word for
// 4-byte items; both words for 8-byte items).
template <int K>
constexpr uint64_t item_identity() {
  if constexpr (K == K_MIN_I32) return 0x7FFFFFFFull;
  else if constexpr (K == K_MAX_I32) return 0x80000000ull;
  else if constexpr (K == K_MIN_I64) return 0x7FFFFFFFFFFFFFFFull;
  else if constexpr (K == K_MAX_I64) return 0x8000000000000000ull;
  else if constexpr (K == K_MIN_F32 || K == K_MAX_F32) return 0x7FC00000ull;  // quiet NaN: minNum ignores it
  else return 0ull;                                                           // sums and counts
}

template <int FT>
__device__ __forceinline__ bool pred_test(uint32_t lo_word, uint32_t hi_word, const RangePred& q) {
  if constexpr (FT == AGG_F32) {
    const float x = __uint_as_float(lo_word);  // NaN fails both comparisons
    return x >= q.flo && x <= q.fhi;
  } else if constexpr (FT == AGG_I32) {
    const int32_t x = (int32_t)lo_word;
    return x >= (int32_t)q.ilo && x <= (int32_t)q.ihi;
  } else {
    const int64_t x = (int64_t)as_u64(lo_word, hi_word);
    return x >= q.ilo && x <= q.ihi;
  }
}

// FB bytes of filter items for one lane and round.
template <int FB, int FW, bool NT, bool AL>
__device__ __forceinline__ void load_filter(const char* p, uint32_t (&w)[FB / 4]) {
  if constexpr (AL && FB == 8) {
    const uint64_t v = *reinterpret_cast<const uint64_t*>(p);
    w[0] = (uint32_t)v;
    w[1] = (uint32_t)(v >> 32);
  } else if constexpr (AL) {
#pragma unroll
    for (int c = 0; c < FB / 16; ++c) {
      const u32x4 v = load_vec_aligned<NT>(p + 16 * c);
      w[4 * c] = v[0]; w[4 * c + 1] = v[1]; w[4 * c + 2] = v[2]; w[4 * c + 3] = v[3];
    }
  } else if constexpr (FW == 4) {
#pragma unroll
    for (int k = 0; k < FB / 4; ++k) w[k] = reinterpret_cast<const uint32_t*>(p)[k];
  } else {
#pragma unroll
    for (int k = 0; k < FB / 8; ++k) {
      const uint64_t v = reinterpret_cast<const uint64_t*>(p)[k];
      w[2 * k] = (uint32_t)v;
      w[2 * k + 1] = (uint32_t)(v >> 32);
    }
  }
}

// One wave folds the selected items of one segment; `cnt` gets this lane's
// selected count.  Same lane mapping and accumulation order as fold_segment.
template <int K, int FT, int U, bool NT, bool AL>
__device__ __forceinline__ typename Fold<K>::acc fold_segment_filtered(const char* __restrict__ vseg,
                                                                        const char* __restrict__ fseg,
                                                                        int64_t valid, int lane,
                                                                        const RangePred& q, uint64_t& cnt) {
  using F = Fold<K>;
  constexpr bool kCount = K == K_COUNT_4 || K == K_COUNT_8;
  constexpr int W = F::W, V = F::V;
  constexpr int FW = FT == AGG_I64 ? 8 : 4;
  constexpr int FB = V * FW;                       // filter bytes per lane and round
  constexpr int64_t RFB = (int64_t)kRoundBytes / W * FW;  // filter bytes per round
  constexpr uint64_t ID = item_identity<K>();
  typename F::acc a[V];
#pragma unroll
  for (int v = 0; v < V; ++v) a[v] = F::identity();
  uint32_t c = 0;
  const char* p = vseg + lane * kVecBytes;
  const char* f = fseg + lane * FB;
  const int64_t full = valid / kRoundBytes;

  auto fold_round = [&](u32x4 x, const uint32_t (&fw)[FB / 4]) {
#pragma unroll
    for (int k = 0; k < V; ++k) {
      const bool sel = pred_test<FT>(fw[k * (FW / 4)], FW == 8 ? fw[k * (FW / 4) + (FW / 4 - 1)] : 0u, q);
      c += sel ? 1u : 0u;
      if constexpr (!kCount) {
        if constexpr (W == 4) {
          x[k] = sel ? x[k] : (uint32_t)ID;
        } else {
          x[2 * k] = sel ? x[2 * k] : (uint32_t)ID;
          x[2 * k + 1] = sel ? x[2 * k + 1] : (uint32_t)(ID >> 32);
        }
      }
    }
    if constexpr (!kCount) F::add_vec(a, x);
  };

  int64_t r = 0;
  for (; r + U <= full; r += U) {
    u32x4 x[U];
    uint32_t fw[U][FB / 4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (!kCount) x[u] = load_vec<NT, AL, W>(p + (r + u) * kRoundBytes);
      load_filter<FB, FW, NT, AL>(f + (r + u) * RFB, fw[u]);
    }
    fold_unrolled<K, U>(
        a, r, [&](int u) { fold_round(kCount ? u32x4{0, 0, 0, 0} : x[u], fw[u]); },
        std::make_integer_sequence<int, U>());
  }
  for (; r < full; ++r) {
    uint32_t fw[FB / 4];
    load_filter<FB, FW, NT, AL>(f + r * RFB, fw);
    fold_round(kCount ? u32x4{0, 0, 0, 0} : load_vec<NT, AL, W>(p + r * kRoundBytes), fw);
    round_done<K>(a, r);
  }
  const int rem = (int)(valid - full * kRoundBytes);
  if (rem > 0) {
    const int lo = lane * kVecBytes;
    const char* pv = p + full * kRoundBytes;
    const char* pf = f + full * RFB;
    const int items = lo + kVecBytes <= rem ? V : (lo < rem ? (rem - lo) / W : 0);
    for (int k = 0; k < items; ++k) {
      uint32_t w0, w1 = 0;
      if constexpr (FW == 4) {
        w0 = reinterpret_cast<const uint32_t*>(pf)[k];
      } else {
        const uint64_t v = reinterpret_cast<const uint64_t*>(pf)[k];
        w0 = (uint32_t)v;
        w1 = (uint32_t)(v >> 32);
      }
      if (pred_test<FT>(w0, w1, q)) {
        ++c;
        if constexpr (!kCount) F::add_item(a[k], pv + k * W);
      }
    }
  }
  cnt = c;
  renorm_all<K>(a);  // close the last block, as fold_segment does
  if constexpr (kCount) {
    return (typename F::acc)c;
  } else {
    if constexpr (V == 4) return F::merge(F::merge(a[0], a[1]), F::merge(a[2], a[3]));
    else return F::merge(a[0], a[1]);
  }
}

struct U64Add {
  __device__ uint64_t operator()(uint64_t x, uint64_t y) const { return x + y; }
};

// Rounds whose loads a lane keeps in flight: 8 when value and filter items
// are both 4 bytes, else 4 (measured on 2^29-item columns: with an 8-byte
// value or filter column, 8 rounds in flight were 4-33% slower than 4; with
// two 4-byte columns 3-24% faster).  The fold order does not depend on it.
template <int K, int FT>
constexpr int filter_unroll() { return (Fold<K>::W == 4 && FT != AGG_I64) ? 8 : 4; }

template <int K, int FT, bool AL>
__global__ void __launch_bounds__(1024) filter_scan_kernel(FilterArgs a) {
  using F = Fold<K>;
  using P = typename F::part;
  constexpr int W = F::W;
  constexpr int FW = FT == AGG_I64 ? 8 : 4;
  const int lane = threadIdx.x & (kWave - 1);
  const int nw = blockDim.x / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * nw;
  const int64_t wave = (int64_t)blockIdx.x * nw + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  P* part = reinterpret_cast<P*>(a.part);
  for (int64_t j = wave; j < a.nseg; j += nwaves) {
    const int64_t begin = j * a.seg_bytes;
    const int64_t valid = a.col_bytes - begin < a.seg_bytes ? a.col_bytes - begin : a.seg_bytes;
    uint64_t cnt = 0;
    typename F::acc acc = fold_segment_filtered<K, FT, filter_unroll<K, FT>(), true, AL>(
        a.base + begin, a.fbase + begin / W * FW, valid, lane, a.pred, cnt);
    acc = wave_reduce(acc, AccMerge<K>());
    cnt = wave_reduce(cnt, U64Add());
    if (lane == 0) {
      part[j] = F::to_part(acc);
      a.cpart[j] = cnt;
    }
  }
}

template <int K>
__global__ void __launch_bounds__(256) filter_combine_kernel(FilterCombineArgs c) {
  using P = typename Fold<K>::part;
  const P total = combine_partials<K>(reinterpret_cast<const P*>(c.part), c.nseg);
  const uint64_t selected = combine_partials<K_COUNT_4>(c.cpart, c.nseg);
  if (threadIdx.x == 0) {
    P t = total;
    if constexpr (K == K_COUNT_4 || K == K_COUNT_8) t = selected;
    *c.out = finalize<K>(t, (int64_t)selected, c.is_avg != 0, c.prec_used);
  }
}

template <int K>
const void* filter_row(int32_t ft, bool al) {
  switch (ft) {
    case AGG_I32: return al ? reinterpret_cast<const void*>(&filter_scan_kernel<K, AGG_I32, true>)
                            : reinterpret_cast<const void*>(&filter_scan_kernel<K, AGG_I32, false>);
    case AGG_I64: return al ? reinterpret_cast<const void*>(&filter_scan_kernel<K, AGG_I64, true>)
                            : reinterpret_cast<const void*>(&filter_scan_kernel<K, AGG_I64, false>);
    case AGG_F32: return al ? reinterpret_cast<const void*>(&filter_scan_kernel<K, AGG_F32, true>)
                            : reinterpret_cast<const void*>(&filter_scan_kernel<K, AGG_F32, false>);
    default: return nullptr;
  }
}

template <int... Ks>
const void* filter_lookup(int kind, int32_t ft, bool al, std::integer_sequence<int, Ks...>) {
  const void* r = nullptr;
  ((kind == Ks ? (r = filter_row<Ks>(ft, al), 0) : 0), ...);
  return r;
}

template <int... Ks>
const void* filter_combine_lookup(int kind, std::integer_sequence<int, Ks...>) {
  const void* r = nullptr;
  ((kind == Ks ? (r = reinterpret_cast<const void*>(&filter_combine_kernel<Ks>), 0) : 0), ...);
  return r;
}

}  // namespace

const void* filter_scan_kernel_ptr(int kind, int32_t filter_dtype, bool aligned) {
  if (kind < 0 || kind >= K_NUM) return nullptr;
  return filter_lookup(kind, filter_dtype, aligned, std::make_integer_sequence<int, K_NUM>());
}

const void* filter_combine_kernel_ptr(int kind) {
  if (kind < 0 || kind >= K_NUM) return nullptr;
  return filter_combine_lookup(kind, std::make_integer_sequence<int, K_NUM>());
}

}  // namespace agg

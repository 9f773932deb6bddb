// Kernels of the aggregation scan for gfx950.
//
// scan_kernel + combine_kernel: the single-column scan (paper Section 3.2,
// GPU specialisation, rebuilt for CDNA4) as a deterministic two-pass
// reduction.  Pass 1: each wave folds whole segments of the column (see
// fold_segment) and stores one partial per segment.  Pass 2: one workgroup
// merges the segment partials in the canonical order and writes the result.
// The merge order is fixed, so the result is deterministic (the property the
// paper's FPGA design gets from its static reduction tree).  Pass 2 runs
// as its own launch (the launch boundary is the global synchronisation) or,
// for a small column scanned in one launch, inside it: the workgroup that
// finishes last merges, which saves the host a kernel launch (the paper's
// fused kernel takes a cooperative-groups grid barrier for this; a counter
// of finished workgroups needs no co-resident grid).  Both forms run the same
// merge, so their results are equal bit for bit.
//
// batch_scan_kernel / batch_combine_kernel: many columns of mixed type and
// function in one persistent launch; the same segment fold and the same
// canonical merge per column, so each column's result equals its agg_run
// result bit for bit.
#include <type_traits>

#include "agg_device.hpp"
#include "agg_internal.hpp"

namespace agg {

// Pass 2: merge the segment partials in the canonical order and write the
// result (every thread of the workgroup calls it).
template <int K, bool COHERENT = false>
__device__ __forceinline__ void combine_and_write(const CombineArgs& a) {
  using P = typename Fold<K>::part;
  const P total = combine_partials<K, COHERENT>(reinterpret_cast<const P*>(a.part), a.nseg);
  if (threadIdx.x == 0) {
    agg_result r = finalize<K>(total, a.n, a.is_avg != 0, a.prec_used);
    if (a.err) {  // a packed column with a corrupt block header: the result is marked invalid
      if (__hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) r.is_null = -1;
      __hip_atomic_store(a.err, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // ready for the next call
    }
    *a.out = r;
  }
}

// Pass 2 inside the scan launch.  The partials are stored with device-scope
// stores (written through to the level every XCD sees), and each wave waits
// for its stores to complete before the workgroup counts itself finished;
// the workgroup whose count completes the grid reads the partials with
// device-scope loads, merges, and zeroes the counter for the next launch.
// Fences would cost more than the combine launch they replace: a device-scope
// release fence in every wave writes back its XCD's whole L2 (2.5% slower at
// 2^30 items, measured), and an acquire in every wave also invalidates the
// L2 under the loads other waves still have in flight (4% slower).  Every
// workgroup reaches this point, so the count always completes.
template <int K>
__device__ __forceinline__ void finish_if_last(const CombineArgs& c, uint32_t* done) {
  __shared__ uint32_t last;
  __builtin_amdgcn_s_waitcnt(0);  // every memory operation of this wave has completed
  __syncthreads();
  if (threadIdx.x == 0)
    last = __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  combine_and_write<K, true>(c);
  if (threadIdx.x == 0) __hip_atomic_store(done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// FUSED: the single-launch form (a.done set); a separate instance, so the
// two-launch kernels' fold loop compiles exactly as without the merge.
template <int K, int U, bool NT, bool AL, bool FUSED>
__global__ void __launch_bounds__(1024) scan_kernel(ScanArgs a) {
  using F = Fold<K>;
  using P = typename F::part;
  const int lane = threadIdx.x & (kWave - 1);
  const int W = blockDim.x / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * W;
  // The wave index is the same in every lane; readfirstlane puts it (and so
  // the whole segment loop and its addresses) in scalar registers.
  const int64_t wave = (int64_t)blockIdx.x * W + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  P* part = reinterpret_cast<P*>(a.part);
  for (int64_t j = a.seg_lo + wave; j < a.seg_hi; j += nwaves) {
    const int64_t begin = j * a.seg_bytes;
    const int64_t valid = a.col_bytes - begin < a.seg_bytes ? a.col_bytes - begin : a.seg_bytes;
    const char* seg = a.base + (j - a.base_seg) * a.seg_bytes;
    typename F::acc acc = fold_segment<K, U, NT, AL>(seg, valid, lane);
    acc = wave_reduce(acc, AccMerge<K>());
    if (lane == 0) {
      if constexpr (FUSED)  // a device-scope store: the in-launch merge reads it from another XCD
        __hip_atomic_store(part + j, F::to_part(acc), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      else
        part[j] = F::to_part(acc);
    }
  }
  if constexpr (FUSED) finish_if_last<K>(a.fin, a.done);
}

// Pass 2 as its own launch: one workgroup.
template <int K>
__global__ void __launch_bounds__(256) combine_kernel(CombineArgs a) {
  combine_and_write<K>(a);
}

// ------------------------------------------------------------ packed columns
// Decoding scan of a frame-of-reference + bit-packed int32 column (layout in
// agg.h).  The bit width is uniform per block, so it selects one of 33
// decoders in which every shift is a compile-time constant.  A lane folds
// its 32 items as d = item - base: SUM adds valid * base + sum(d), MIN / MAX
// take base + min(d) / max(d).
template <int BITS, bool FULL>
__device__ __forceinline__ void decode_lane(const uint32_t* __restrict__ p, int lane, int valid, uint64_t& sum,
                                            uint32_t& dmin, uint32_t& dmax) {
  uint32_t w[BITS > 0 ? BITS : 1];
#pragma unroll
  for (int j = 0; j < BITS; ++j) w[j] = p[j * kWave + lane];
  uint64_t s = 0;
  uint32_t mn = 0xFFFFFFFFu, mx = 0u;
#pragma unroll
  for (int i = 0; i < kWave / 2; ++i) {
    uint32_t v = 0;
    if constexpr (BITS > 0) {
      const int pos = i * BITS, wi = pos >> 5, sh = pos & 31;
      v = w[wi] >> sh;
      if (sh + BITS > 32) v |= w[wi + 1] << (32 - sh);
      if (BITS < 32) v &= (1u << BITS) - 1u;
    }
    if (FULL || i < valid) {
      s += v;
      mn = v < mn ? v : mn;
      mx = v > mx ? v : mx;
    }
  }
  sum += s;
  dmin = mn;
  dmax = mx;
}

template <int BITS = 0>
__device__ __forceinline__ void decode_dispatch(uint32_t bits, bool full, const uint32_t* p, int lane, int valid,
                                                uint64_t& sum, uint32_t& dmin, uint32_t& dmax) {
  if constexpr (BITS <= 32) {
    if (bits == BITS) {
      if (full) decode_lane<BITS, true>(p, lane, valid, sum, dmin, dmax);
      else decode_lane<BITS, false>(p, lane, valid, sum, dmin, dmax);
      return;
    }
    decode_dispatch<BITS + 1>(bits, full, p, lane, valid, sum, dmin, dmax);
  }
}

template <int K>
__global__ void __launch_bounds__(1024) packed_scan_kernel(PackedArgs a) {
  using F = Fold<K>;
  using P = typename F::part;
  const int lane = threadIdx.x & (kWave - 1);
  const int W = blockDim.x / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * W;
  const int64_t wave = (int64_t)blockIdx.x * W + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  constexpr int kPerLane = AGG_PACK_BLOCK / kWave;
  uint64_t sum = 0;              // sum of items mod 2^64 (SUM)
  int32_t ext = K == K_MIN_I32 ? INT32_MAX : INT32_MIN;  // running MIN / MAX
  for (int64_t b = wave; b < a.nblocks; b += nwaves) {
    const agg_packed_block h = a.blocks[b];
    // a block whose payload would lie outside the buffer is never read; the
    // result is marked invalid (the combine reads the flag)
    if (h.bits > 32 || h.word_off < 0 || h.word_off + (int64_t)kWave * h.bits > a.payload_words) {
      if (lane == 0) __hip_atomic_fetch_or(a.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }
    const int64_t left = a.n - b * AGG_PACK_BLOCK;
    const bool full = left >= AGG_PACK_BLOCK;
    int valid = (int)(left - (int64_t)lane * kPerLane);
    valid = valid < 0 ? 0 : (valid > kPerLane ? kPerLane : valid);
    uint64_t dsum = 0;
    uint32_t dmin = 0xFFFFFFFFu, dmax = 0u;
    decode_dispatch(h.bits, full, a.payload + h.word_off, lane, valid, dsum, dmin, dmax);
    if constexpr (K == K_SUM_I32) {
      sum += dsum + (uint64_t)((int64_t)valid * (int64_t)h.base);
    } else if (valid > 0) {
      const int32_t lo = (int32_t)((uint32_t)h.base + dmin), hi = (int32_t)((uint32_t)h.base + dmax);
      ext = K == K_MIN_I32 ? min(ext, lo) : max(ext, hi);
    }
  }
  P partial;
  if constexpr (K == K_SUM_I32) partial = sum;
  else partial = (int64_t)ext;
  partial = wave_reduce(partial, PartMerge<K>());
  if (lane == 0) reinterpret_cast<P*>(a.part)[wave] = partial;
}

// ------------------------------------------------------------ batch
template <int K, int U, bool NT>
__device__ __forceinline__ void batch_item(const WorkItem& it, uint64_t* slots, int lane) {
  using F = Fold<K>;
  using P = typename F::part;
  P* part = reinterpret_cast<P*>(slots + it.part_off);
  const int64_t seg_bytes = (int64_t)1 << it.seg_log2;
  for (int64_t j = it.seg_lo; j < it.seg_hi; ++j) {
    const int64_t begin = j * seg_bytes;
    const int64_t valid = it.col_bytes - begin < seg_bytes ? it.col_bytes - begin : seg_bytes;
    typename F::acc acc = it.aligned ? fold_segment<K, U, NT, true>(it.ptr + begin, valid, lane)
                                     : fold_segment<K, 4, false, false>(it.ptr + begin, valid, lane);
    acc = wave_reduce(acc, AccMerge<K>());
    if (lane == 0) part[j] = F::to_part(acc);
  }
}

// A wave's items are i = wave, wave + P, wave + 2P, ... (P waves).  It reads
// their records 64 at a time, one per lane, and takes each out of its lane
// with readlane: one memory round trip per 64 items instead of one per item.
template <int U, bool NT>
__global__ void __launch_bounds__(1024) batch_scan_kernel(BatchArgs a) {
  static_assert(sizeof(WorkItem) == 32, "a work record is two 16-byte words");
  const int lane = threadIdx.x & (kWave - 1);
  const int W = blockDim.x / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * W;
  const int64_t wave = (int64_t)blockIdx.x * W + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (int64_t base = wave; base < a.nitems; base += kWave * nwaves) {
    const int64_t mine = base + lane * nwaves;
    u32x4 w0 = {0, 0, 0, 0}, w1 = w0;
    if (mine < a.nitems) {
      const u32x4* rec = reinterpret_cast<const u32x4*>(a.items + mine);
      w0 = rec[0];
      w1 = rec[1];
    }
    // The records are read once per 64 items; passing them through an empty
    // asm makes the wait for their loads happen here, once.  Otherwise the
    // registers still count as loaded at the top of the item loop below, and
    // every item began with a wait for all of the wave's memory operations
    // (the previous item's partial store included): a round trip per item.
    __asm__ volatile("" : "+v"(w0), "+v"(w1));
    const int64_t left = (a.nitems - base + nwaves - 1) / nwaves;
    const int cnt = left < kWave ? (int)left : kWave;
    for (int l = 0; l < cnt; ++l) {
      auto rd = [l](uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); };
      auto rd64 = [&](uint32_t lo, uint32_t hi) { return (int64_t)(((uint64_t)rd(hi) << 32) | rd(lo)); };
      WorkItem it;
      it.ptr = reinterpret_cast<const char*>(rd64(w0[0], w0[1]));
      it.col_bytes = rd64(w0[2], w0[3]);
      it.part_off = rd(w1[0]);
      const uint32_t range = rd(w1[1]), meta = rd(w1[2]);
      it.seg_lo = (uint16_t)(range & 0xFFFFu);
      it.seg_hi = (uint16_t)(range >> 16);
      it.seg_log2 = (uint8_t)(meta & 0xFFu);
      it.kind = (uint8_t)((meta >> 8) & 0xFFu);
      it.aligned = (uint8_t)((meta >> 16) & 0xFFu);
      switch (it.kind) {
        case K_SUM_I32: batch_item<K_SUM_I32, U, NT>(it, a.part, lane); break;
        case K_MIN_I32: batch_item<K_MIN_I32, U, NT>(it, a.part, lane); break;
        case K_MAX_I32: batch_item<K_MAX_I32, U, NT>(it, a.part, lane); break;
        case K_SUM_I64: batch_item<K_SUM_I64, U, NT>(it, a.part, lane); break;
        case K_MIN_I64: batch_item<K_MIN_I64, U, NT>(it, a.part, lane); break;
        case K_MAX_I64: batch_item<K_MAX_I64, U, NT>(it, a.part, lane); break;
        case K_SUM_F32_PLAIN: batch_item<K_SUM_F32_PLAIN, U, NT>(it, a.part, lane); break;
        case K_SUM_F32_F64C: batch_item<K_SUM_F32_F64C, U, NT>(it, a.part, lane); break;
        case K_SUM_F32_NEU: batch_item<K_SUM_F32_NEU, U, NT>(it, a.part, lane); break;
        case K_MIN_F32: batch_item<K_MIN_F32, U, NT>(it, a.part, lane); break;
        case K_MAX_F32: batch_item<K_MAX_F32, U, NT>(it, a.part, lane); break;
        case K_COUNT_4: batch_item<K_COUNT_4, U, NT>(it, a.part, lane); break;
        case K_COUNT_8: batch_item<K_COUNT_8, U, NT>(it, a.part, lane); break;
        default: break;
      }
    }
  }
}

template <int K>
__device__ __forceinline__ void batch_combine_col(const BatchColDev& c, uint64_t* slots, agg_result* out) {
  using P = typename Fold<K>::part;
  const P total = combine_partials<K>(reinterpret_cast<const P*>(slots + c.part_off), c.nseg);
  if (threadIdx.x == 0) *out = finalize<K>(total, c.n, c.is_avg != 0, c.prec_used);
}

// One workgroup of 256 threads per column.
__global__ void __launch_bounds__(256) batch_combine_kernel(BatchArgs a, int64_t ncols) {
  const int64_t col = blockIdx.x;
  if (col >= ncols) return;
  const BatchColDev c = a.cols[col];
  agg_result* out = a.results + col;
  switch (c.kind) {
    case K_SUM_I32: batch_combine_col<K_SUM_I32>(c, a.part, out); break;
    case K_MIN_I32: batch_combine_col<K_MIN_I32>(c, a.part, out); break;
    case K_MAX_I32: batch_combine_col<K_MAX_I32>(c, a.part, out); break;
    case K_SUM_I64: batch_combine_col<K_SUM_I64>(c, a.part, out); break;
    case K_MIN_I64: batch_combine_col<K_MIN_I64>(c, a.part, out); break;
    case K_MAX_I64: batch_combine_col<K_MAX_I64>(c, a.part, out); break;
    case K_SUM_F32_PLAIN: batch_combine_col<K_SUM_F32_PLAIN>(c, a.part, out); break;
    case K_SUM_F32_F64C: batch_combine_col<K_SUM_F32_F64C>(c, a.part, out); break;
    case K_SUM_F32_NEU: batch_combine_col<K_SUM_F32_NEU>(c, a.part, out); break;
    case K_MIN_F32: batch_combine_col<K_MIN_F32>(c, a.part, out); break;
    case K_MAX_F32: batch_combine_col<K_MAX_F32>(c, a.part, out); break;
    case K_COUNT_4: batch_combine_col<K_COUNT_4>(c, a.part, out); break;
    case K_COUNT_8: batch_combine_col<K_COUNT_8>(c, a.part, out); break;
    default: break;
  }
}

// ------------------------------------------------------------ dispatch tables
namespace {

template <int K>
struct ScanRow {
  // [fused][unroll index][nontemporal][aligned]; the unaligned variant is
  // one (U = 4, temporal) kernel per form, shared by every entry.
  template <bool FU>
  static const void* get_form(int ui, bool nt, bool al) {
    if (!al) return reinterpret_cast<const void*>(&scan_kernel<K, 4, false, false, FU>);
    static const void* t[4][2] = {
        {reinterpret_cast<const void*>(&scan_kernel<K, 4, false, true, FU>),
         reinterpret_cast<const void*>(&scan_kernel<K, 4, true, true, FU>)},
        {reinterpret_cast<const void*>(&scan_kernel<K, 8, false, true, FU>),
         reinterpret_cast<const void*>(&scan_kernel<K, 8, true, true, FU>)},
        {reinterpret_cast<const void*>(&scan_kernel<K, 16, false, true, FU>),
         reinterpret_cast<const void*>(&scan_kernel<K, 16, true, true, FU>)},
        {reinterpret_cast<const void*>(&scan_kernel<K, 32, false, true, FU>),
         reinterpret_cast<const void*>(&scan_kernel<K, 32, true, true, FU>)}};
    return t[ui][nt ? 1 : 0];
  }
  static const void* get(int ui, bool nt, bool al, bool fused) {
    return fused ? get_form<true>(ui, nt, al) : get_form<false>(ui, nt, al);
  }
};

template <int... Ks>
const void* scan_lookup(int kind, int ui, bool nt, bool al, bool fused, std::integer_sequence<int, Ks...>) {
  const void* r = nullptr;
  ((kind == Ks ? (r = ScanRow<Ks>::get(ui, nt, al, fused), 0) : 0), ...);
  return r;
}

}  // namespace

const void* scan_kernel_ptr(int kind, int unroll, bool nontemporal, bool aligned, bool fused) {
  const int ui = unroll_index(unroll);
  if (kind < 0 || kind >= K_NUM || ui < 0) return nullptr;
  return scan_lookup(kind, ui, nontemporal, aligned, fused, std::make_integer_sequence<int, K_NUM>());
}

namespace {
template <int... Ks>
const void* combine_lookup(int kind, std::integer_sequence<int, Ks...>) {
  const void* r = nullptr;
  ((kind == Ks ? (r = reinterpret_cast<const void*>(&combine_kernel<Ks>), 0) : 0), ...);
  return r;
}
}  // namespace

const void* combine_kernel_ptr(int kind) {
  if (kind < 0 || kind >= K_NUM) return nullptr;
  return combine_lookup(kind, std::make_integer_sequence<int, K_NUM>());
}

const void* packed_scan_kernel_ptr(int kind) {
  switch (kind) {
    case K_SUM_I32: return reinterpret_cast<const void*>(&packed_scan_kernel<K_SUM_I32>);
    case K_MIN_I32: return reinterpret_cast<const void*>(&packed_scan_kernel<K_MIN_I32>);
    case K_MAX_I32: return reinterpret_cast<const void*>(&packed_scan_kernel<K_MAX_I32>);
    default: return nullptr;
  }
}

const void* batch_scan_kernel_ptr(int unroll, bool nontemporal) {
  static const void* t[4][2] = {
      {reinterpret_cast<const void*>(&batch_scan_kernel<4, false>),
       reinterpret_cast<const void*>(&batch_scan_kernel<4, true>)},
      {reinterpret_cast<const void*>(&batch_scan_kernel<8, false>),
       reinterpret_cast<const void*>(&batch_scan_kernel<8, true>)},
      {reinterpret_cast<const void*>(&batch_scan_kernel<16, false>),
       reinterpret_cast<const void*>(&batch_scan_kernel<16, true>)},
      {reinterpret_cast<const void*>(&batch_scan_kernel<32, false>),
       reinterpret_cast<const void*>(&batch_scan_kernel<32, true>)}};
  const int ui = unroll_index(unroll);
  return ui < 0 ? nullptr : t[ui][nontemporal ? 1 : 0];
}

const void* batch_combine_kernel_ptr() { return reinterpret_cast<const void*>(&batch_combine_kernel); }

}  // namespace agg

// Kernels of the aggregation scan for gfx950.
//
// scan_kernel + combine_kernel: the single-column scan (paper Section 3.2,
// GPU specialisation, rebuilt for CDNA4) as a deterministic two-pass
// reduction.  Pass 1: each wave folds whole segments of the column (see
// fold_segment) and stores one partial per segment.  Pass 2: one workgroup
// merges the segment partials in the canonical order and writes the result.
// No atomics and no fences: the merge order is fixed, so the result is
// deterministic (the property the paper's FPGA design gets from its static
// reduction tree), and the launch boundary is the global synchronisation the
// paper's fused kernel takes from cooperative groups.
//
// batch_scan_kernel / batch_combine_kernel: many columns of mixed type and
// function in one persistent launch; the same segment fold and the same
// canonical merge per column, so each column's result equals its agg_run
// result bit for bit.
#include <type_traits>

#include "agg_device.hpp"
#include "agg_internal.hpp"

namespace agg {

template <int K, int U, bool NT, bool AL>
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
    if (lane == 0) part[j] = F::to_part(acc);
  }
}

// Second pass: one workgroup merges the nseg segment partials in the
// canonical order and writes the result.  The kernel boundary after the
// scan launches is the global synchronisation: no fences, no atomics.
template <int K>
__global__ void __launch_bounds__(256) combine_kernel(CombineArgs a) {
  using P = typename Fold<K>::part;
  const P total = combine_partials<K>(reinterpret_cast<const P*>(a.part), a.nseg);
  if (threadIdx.x == 0) *a.out = finalize<K>(total, a.n, a.is_avg != 0, a.prec_used);
}

// ------------------------------------------------------------ batch
template <int K, int U, bool NT>
__device__ __forceinline__ void batch_item(const BatchColDev& c, const WorkItem& it, uint64_t* slots,
                                           int lane) {
  using F = Fold<K>;
  using P = typename F::part;
  P* part = reinterpret_cast<P*>(slots + c.part_off);
  for (int64_t j = it.seg_lo; j < it.seg_hi; ++j) {
    const int64_t begin = j * c.seg_bytes;
    const int64_t valid = c.col_bytes - begin < c.seg_bytes ? c.col_bytes - begin : c.seg_bytes;
    typename F::acc acc = c.aligned ? fold_segment<K, U, NT, true>(c.ptr + begin, valid, lane)
                                    : fold_segment<K, 4, false, false>(c.ptr + begin, valid, lane);
    acc = wave_reduce(acc, AccMerge<K>());
    if (lane == 0) part[j] = F::to_part(acc);
  }
}

template <int U, bool NT>
__global__ void __launch_bounds__(1024) batch_scan_kernel(BatchArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int W = blockDim.x / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * W;
  const int64_t wave = (int64_t)blockIdx.x * W + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (int64_t i = wave; i < a.nitems; i += nwaves) {
    const WorkItem it = a.items[i];
    const BatchColDev c = a.cols[it.col];
    switch (c.kind) {
      case K_SUM_I32: batch_item<K_SUM_I32, U, NT>(c, it, a.part, lane); break;
      case K_MIN_I32: batch_item<K_MIN_I32, U, NT>(c, it, a.part, lane); break;
      case K_MAX_I32: batch_item<K_MAX_I32, U, NT>(c, it, a.part, lane); break;
      case K_SUM_I64: batch_item<K_SUM_I64, U, NT>(c, it, a.part, lane); break;
      case K_MIN_I64: batch_item<K_MIN_I64, U, NT>(c, it, a.part, lane); break;
      case K_MAX_I64: batch_item<K_MAX_I64, U, NT>(c, it, a.part, lane); break;
      case K_SUM_F32_PLAIN: batch_item<K_SUM_F32_PLAIN, U, NT>(c, it, a.part, lane); break;
      case K_SUM_F32_F64C: batch_item<K_SUM_F32_F64C, U, NT>(c, it, a.part, lane); break;
      case K_SUM_F32_NEU: batch_item<K_SUM_F32_NEU, U, NT>(c, it, a.part, lane); break;
      case K_MIN_F32: batch_item<K_MIN_F32, U, NT>(c, it, a.part, lane); break;
      case K_MAX_F32: batch_item<K_MAX_F32, U, NT>(c, it, a.part, lane); break;
      case K_COUNT_4: batch_item<K_COUNT_4, U, NT>(c, it, a.part, lane); break;
      case K_COUNT_8: batch_item<K_COUNT_8, U, NT>(c, it, a.part, lane); break;
      default: break;
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
  // [unroll index][nontemporal][aligned]; the unaligned variant is one
  // (U = 4, temporal) kernel, shared by every entry.
  static const void* get(int ui, bool nt, bool al) {
    if (!al) return reinterpret_cast<const void*>(&scan_kernel<K, 4, false, false>);
    static const void* t[4][2] = {
        {reinterpret_cast<const void*>(&scan_kernel<K, 4, false, true>),
         reinterpret_cast<const void*>(&scan_kernel<K, 4, true, true>)},
        {reinterpret_cast<const void*>(&scan_kernel<K, 8, false, true>),
         reinterpret_cast<const void*>(&scan_kernel<K, 8, true, true>)},
        {reinterpret_cast<const void*>(&scan_kernel<K, 16, false, true>),
         reinterpret_cast<const void*>(&scan_kernel<K, 16, true, true>)},
        {reinterpret_cast<const void*>(&scan_kernel<K, 32, false, true>),
         reinterpret_cast<const void*>(&scan_kernel<K, 32, true, true>)}};
    return t[ui][nt ? 1 : 0];
  }
};

template <int... Ks>
const void* scan_lookup(int kind, int ui, bool nt, bool al, std::integer_sequence<int, Ks...>) {
  const void* r = nullptr;
  ((kind == Ks ? (r = ScanRow<Ks>::get(ui, nt, al), 0) : 0), ...);
  return r;
}

}  // namespace

const void* scan_kernel_ptr(int kind, int unroll, bool nontemporal, bool aligned) {
  const int ui = unroll_index(unroll);
  if (kind < 0 || kind >= K_NUM || ui < 0) return nullptr;
  return scan_lookup(kind, ui, nontemporal, aligned, std::make_integer_sequence<int, K_NUM>());
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

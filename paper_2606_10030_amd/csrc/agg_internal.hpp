// Internal interface between the kernels (agg_kernels.hip) and the host
// runtime (agg_api.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "agg.h"

namespace agg {

// Fold kinds: one per (item type, function, precision).  AVG folds as SUM.
enum Kind : int {
  K_SUM_I32 = 0, K_MIN_I32, K_MAX_I32,
  K_SUM_I64, K_MIN_I64, K_MAX_I64,
  K_SUM_F32_PLAIN, K_SUM_F32_F64C, K_SUM_F32_NEU,
  K_MIN_F32, K_MAX_F32,
  K_COUNT_4, K_COUNT_8,
  K_NUM
};

// The single-column merge of all segment partials.
struct CombineArgs {
  const void* part;
  int64_t nseg;
  agg_result* out;
  int64_t n;
  int32_t is_avg;
  int32_t prec_used;
  uint32_t* err = nullptr;  // packed scans: nonzero if a corrupt block header was seen (read, then cleared)
};

// One launch of the single-column scan over segments [seg_lo, seg_hi).
struct ScanArgs {
  const char* base;      // address of segment base_seg of the column
  int64_t col_bytes;     // n * width
  int64_t seg_bytes;     // canonical segment size
  int64_t seg_lo, seg_hi;
  int64_t base_seg;      // segment index that `base` points at
  void* part;            // segment partials (8-byte slots), indexed by segment
  // Single-launch form (the launch covers every segment): a zeroed counter
  // of finished workgroups; the last one merges the partials as `fin` says
  // and zeroes the counter again.  nullptr: a separate combine launch follows.
  uint32_t* done = nullptr;
  CombineArgs fin{};
};

// One launch of the packed-column scan: each wave folds blocks wave,
// wave + nwaves, ... and writes one partial (integer results are exact in
// any order, so the partials need no canonical shape).
struct PackedArgs {
  const agg_packed_block* blocks;
  const uint32_t* payload;
  int64_t n;
  int64_t nblocks;
  int64_t payload_words;
  void* part;            // one partial per wave of the launch
  uint32_t* err;         // set to 1 when a block header is corrupt (the block is not read)
};

// The range predicate of a filtered scan, as the device sees it: the host
// turns every agg_filter into an inclusive range lo <= y <= hi in the filter
// column's own type (int32 / int64 / float32), selecting exactly the same
// items; an empty range has lo > hi.
struct RangePred {
  int64_t ilo, ihi;
  float flo, fhi;
};

// One launch of the filtered scan: value partials and selected counts per segment.
struct FilterArgs {
  const char* base;      // value column
  const char* fbase;     // filter column
  int64_t col_bytes;
  int64_t seg_bytes;
  int64_t nseg;
  void* part;            // nseg value partials
  uint64_t* cpart;       // nseg selected counts
  RangePred pred;
};

struct FilterCombineArgs {
  const void* part;
  const uint64_t* cpart;
  int64_t nseg;
  agg_result* out;
  int32_t is_avg;
  int32_t prec_used;
};

// One column of a batch, as the device sees it.
struct BatchColDev {
  const char* ptr;
  int64_t col_bytes;
  int64_t seg_bytes;
  int64_t nseg;
  int64_t part_off;      // first 8-byte partial slot of this column
  int64_t n;
  int32_t kind;
  int32_t is_avg;
  int32_t prec_used;
  int32_t aligned;       // ptr is 16-byte aligned
};

// A run of whole segments [seg_lo, seg_hi) of one column: the unit of work
// of the persistent batch kernel.
// A run of whole segments of one column, with the column fields the scan
// needs copied in (32 bytes), so a wave reads one record instead of an item
// and then its column.
struct WorkItem {
  const char* ptr;       // column base
  int64_t col_bytes;
  uint32_t part_off;     // first 8-byte partial slot of the column
  uint16_t seg_lo;       // segments [seg_lo, seg_hi) (a column has at most 8192)
  uint16_t seg_hi;
  uint8_t seg_log2;      // seg_bytes = 2^seg_log2
  uint8_t kind;
  uint8_t aligned;       // ptr is 16-byte aligned
  uint8_t pad[5];
};

struct BatchArgs {
  const BatchColDev* cols;
  const WorkItem* items;
  int64_t nitems;
  uint64_t* part;
  agg_result* results;
};

int kind_of(int32_t dtype, int32_t op, int32_t prec);  // -1 if invalid
int width_of(int32_t dtype);                          // 4 or 8, 0 if invalid
int unroll_index(int32_t unroll);                      // 0..3 for 4,8,16,32; -1 otherwise

// Host helpers shared by the runtime files.
void record_hip_error(int32_t e);                 // remembered for agg_last_hip_error
bool fault_hit(int site);                         // an injected failure is due at this site (agg_fault_inject)
int device_alloc(void** p, size_t bytes);         // hipMalloc: AGG_OK / AGG_E_NOMEM (also when injected) / AGG_E_HIP
int pinned_alloc(void** p, size_t bytes);         // hipHostMalloc: AGG_OK / AGG_E_NOMEM
int current_device(int* dev);                     // current HIP device, checked to be gfx950
int device_cu(int dev);                           // its compute-unit count
void shape_of(int32_t dtype, int64_t n, agg_shape* s);
void tune_for(int kind, int32_t src, int64_t bytes, agg_tune* t);
int check_pointer(const void* p, int64_t bytes, int32_t src, int dev);
int check_out_pointer(const void* p, int64_t bytes, int dev);
int grid_for(const agg_tune& t, int cu, int64_t nseg);
int launch(const void* fn, int grid, int block, void* args, hipStream_t stream);
int64_t ceil_div(int64_t a, int64_t b);

bool tune_is_valid(const agg_tune& t);
bool tune_cache_lookup(int kind, int32_t src, int64_t bytes, agg_tune* out);
void builtin_tune_for(int kind, agg_tune* out);

// fused: the single-launch form (ScanArgs::done set)
const void* scan_kernel_ptr(int kind, int unroll, bool nontemporal, bool aligned, bool fused = false);
const void* combine_kernel_ptr(int kind);
const void* packed_scan_kernel_ptr(int kind);   // K_SUM_I32, K_MIN_I32, K_MAX_I32
const void* filter_scan_kernel_ptr(int kind, int32_t filter_dtype, bool aligned);
const void* filter_combine_kernel_ptr(int kind);
const void* batch_scan_kernel_ptr(int unroll, bool nontemporal);
const void* batch_combine_kernel_ptr();

constexpr int64_t kSegMin = 16 * 1024;
constexpr int kCombineThreads = 256;   // workgroup of the combine kernels
constexpr int64_t kSegTarget = 8192;   // at most this many segments per column

}  // namespace agg

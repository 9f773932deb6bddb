// Host runtime of libagg.so: the C ABI declared in include/agg.h.
//
// Plans own their workspaces (segment partials, completion counter, and for
// pinned-host sources a device staging ring, a copy stream and events), so
// agg_run only validates, picks a kernel and enqueues.  Batches own a work
// table, partials, results and a captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <limits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "agg.h"
#include "agg_internal.hpp"

namespace agg {

int kind_of(int32_t dtype, int32_t op, int32_t prec) {
  if (op == AGG_COUNT) {
    if (dtype == AGG_I32 || dtype == AGG_F32) return K_COUNT_4;
    if (dtype == AGG_I64) return K_COUNT_8;
    return -1;
  }
  const bool sum = op == AGG_SUM || op == AGG_AVG;
  if (!sum && op != AGG_MIN && op != AGG_MAX) return -1;
  switch (dtype) {
    case AGG_I32: return sum ? K_SUM_I32 : (op == AGG_MIN ? K_MIN_I32 : K_MAX_I32);
    case AGG_I64: return sum ? K_SUM_I64 : (op == AGG_MIN ? K_MIN_I64 : K_MAX_I64);
    case AGG_F32:
      if (!sum) return op == AGG_MIN ? K_MIN_F32 : K_MAX_F32;
      if (prec == AGG_PREC_NEUMAIER) return K_SUM_F32_NEU;
      if (prec == AGG_PREC_F32) return K_SUM_F32_PLAIN;
      if (prec == AGG_PREC_F64_COMBINE) return K_SUM_F32_F64C;
      return -1;
    default: return -1;
  }
}

int width_of(int32_t dtype) {
  return dtype == AGG_I64 ? 8 : (dtype == AGG_I32 || dtype == AGG_F32) ? 4 : 0;
}

int unroll_index(int32_t unroll) {
  return unroll == 4 ? 0 : unroll == 8 ? 1 : unroll == 16 ? 2 : unroll == 32 ? 3 : -1;
}

}  // namespace agg

using namespace agg;

namespace agg {

thread_local int32_t g_last_hip = 0;
void record_hip_error(int32_t e) { g_last_hip = e; }

// ------------------------------------------------------------ fault injection
// Error paths that the hardware rarely takes are forced from the host: a
// countdown per site makes the n-th next event there fail as the runtime
// would report it (an allocation: out of memory; a shipped copy: a HIP
// error).  Armed by agg_fault_inject or, at the first library call, by the
// environment variable AGG_FAULT_INJECT="site:n[,site:n...]" (sites "alloc",
// "ship").  Nothing reaches the device: the failing call is never issued.
std::atomic<int32_t> g_fault[AGG_FAULT_SITES];
std::once_flag g_fault_env_once;

void fault_env() {
  std::call_once(g_fault_env_once, [] {
    const char* e = std::getenv("AGG_FAULT_INJECT");
    if (!e) return;
    const char* q = e;
    while (*q) {
      const char* colon = std::strchr(q, ':');
      if (!colon) return;
      const std::string site(q, (size_t)(colon - q));
      const long n = std::strtol(colon + 1, nullptr, 10);
      const int idx = site == "alloc" ? AGG_FAULT_ALLOC : site == "ship" ? AGG_FAULT_SHIP : -1;
      if (idx > 0 && n > 0 && n < INT32_MAX) g_fault[idx].store((int32_t)n);
      const char* comma = std::strchr(colon, ',');
      if (!comma) return;
      q = comma + 1;
    }
  });
}

bool fault_hit(int site) {
  fault_env();
  int32_t c = g_fault[site].load();
  while (c > 0 && !g_fault[site].compare_exchange_weak(c, c - 1)) {
  }
  return c == 1;
}

int device_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (fault_hit(AGG_FAULT_ALLOC)) return AGG_E_NOMEM;
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    *p = nullptr;
    return AGG_E_NOMEM;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    g_last_hip = (int32_t)e;
    return AGG_E_HIP;
  }
  return AGG_OK;
}

int pinned_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (fault_hit(AGG_FAULT_ALLOC)) return AGG_E_NOMEM;
  if (hipHostMalloc(p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return AGG_E_NOMEM;
  }
  return AGG_OK;
}

#define HIPCHK(expr)                                  \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) {                           \
      g_last_hip = (int32_t)e_;                       \
      return AGG_E_HIP;                               \
    }                                                 \
  } while (0)

constexpr int kMaxDevices = 64;
constexpr int64_t kMaxItems = (int64_t)1 << 40;  // keeps n * width far from overflow
constexpr int64_t kItemMaxBytes = 256 * 1024;     // batch work items: about this many bytes at most
constexpr int64_t kItemMinBytes = 64 * 1024;      // ... and at least

struct DeviceInfo {
  bool checked = false;
  int status = AGG_E_NODEVICE;
  int cu = 0;
  char arch[64] = {0};
};
std::mutex g_mu;
DeviceInfo g_dev[kMaxDevices];

int device_check(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return AGG_E_INVALID;
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceInfo& d = g_dev[dev];
  if (d.checked) return d.status;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || dev >= count) {
    (void)hipGetLastError();
    d.checked = true;
    d.status = AGG_E_NODEVICE;
    return d.status;
  }
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) {
    g_last_hip = (int32_t)e;
    return AGG_E_HIP;
  }
  std::snprintf(d.arch, sizeof d.arch, "%s", prop.gcnArchName);
  d.cu = prop.multiProcessorCount;
  d.checked = true;
  d.status = std::strncmp(d.arch, "gfx950", 6) == 0 ? AGG_OK : AGG_E_NODEVICE;
  return d.status;
}

int device_cu(int dev) { return (dev >= 0 && dev < kMaxDevices) ? g_dev[dev].cu : 0; }

int current_device(int* dev) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    (void)hipGetLastError();
    return AGG_E_NODEVICE;
  }
  HIPCHK(hipGetDevice(dev));
  return device_check(*dev);
}

bool tune_is_valid(const agg_tune& t) {
  const int w = t.waves_per_block;
  return (w == 1 || w == 2 || w == 4 || w == 8 || w == 16) &&
         t.blocks_per_cu >= 1 && t.blocks_per_cu <= 32 && unroll_index(t.unroll) >= 0 &&
         (t.nontemporal == 0 || t.nontemporal == 1) && t.chunk_bytes >= (1 << 20) &&
         t.chunk_bytes <= ((int64_t)1 << 32) && t.staging_depth >= 2 && t.staging_depth <= 4;
}

bool valid_tune(const agg_tune& t) { return tune_is_valid(t); }

// Launch parameters for a kind: the tuning cache, else the built-in table.
void tune_for(int kind, int32_t src, int64_t bytes, agg_tune* t) {
  if (!tune_cache_lookup(kind, src, bytes, t)) builtin_tune_for(kind, t);
}

// Batches mix kinds; two waves per CU with 16 loads in flight suits all of
// the plain kinds (agg_batch_autotune refines it).
void batch_builtin_tune(agg_tune* t) { builtin_tune_for(K_SUM_I32, t); }

namespace {
// The checks of check_pointer on attributes already queried.
int check_pointer_with(const hipPointerAttribute_t& at, const void* p, int64_t bytes, int32_t src, int dev) {
  if (src == AGG_SRC_DEVICE) {
    if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) return AGG_E_INVALID;
    if (at.type == hipMemoryTypeDevice && at.device != dev) return AGG_E_INVALID;
  } else {
    if (at.type != hipMemoryTypeHost) return AGG_E_INVALID;
  }
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess && base) {
    const char* b = static_cast<const char*>(base);
    const char* q = static_cast<const char*>(p);
    if (q < b || q + bytes > b + size) return AGG_E_INVALID;
  } else {
    // Without a known extent the scan could read past the allocation.
    (void)hipGetLastError();
    return AGG_E_INVALID;
  }
  return AGG_OK;
}
}  // namespace

// The memory behind [p, p + bytes) must be of the kind `src` names.
int check_pointer(const void* p, int64_t bytes, int32_t src, int dev) {
  hipPointerAttribute_t at;
  std::memset(&at, 0, sizeof at);
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return AGG_E_INVALID;
  }
  return check_pointer_with(at, p, bytes, src, dev);
}

// A result buffer: device memory of `dev` or page-locked host memory, with
// room for `bytes` bytes.  (Each call is two runtime queries, about 0.05 us
// each on MI355X; they are not cached across calls, since a range freed and
// reused would then pass unchecked.)
int check_out_pointer(const void* p, int64_t bytes, int dev) {
  hipPointerAttribute_t at;
  std::memset(&at, 0, sizeof at);
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return AGG_E_INVALID;
  }
  if (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged)
    return check_pointer_with(at, p, bytes, AGG_SRC_DEVICE, dev);
  if (at.type == hipMemoryTypeHost) return check_pointer_with(at, p, bytes, AGG_SRC_PINNED_HOST, dev);
  return AGG_E_INVALID;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

void shape_of(int32_t dtype, int64_t n, agg_shape* s) {
  const int w = width_of(dtype);
  const int64_t bytes = n * w;
  int64_t seg = kSegMin;
  const int64_t target = ceil_div(bytes, kSegTarget);
  while (seg < target) seg <<= 1;
  s->seg_bytes = seg;
  s->nseg = ceil_div(bytes, seg);
  s->elems_per_seg = seg / w;
  s->width = w;
  s->reserved = 0;
}

int grid_for(const agg_tune& t, int cu, int64_t nseg) {
  const int64_t need = ceil_div(std::max<int64_t>(nseg, 1), t.waves_per_block);
  return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)t.blocks_per_cu * cu, need));
}

int launch(const void* fn, int grid, int block, void* args, hipStream_t stream) {
  void* kargs[] = {args};
  HIPCHK(hipLaunchKernel(fn, dim3(grid), dim3(block), kargs, 0, stream));
  return AGG_OK;
}

}  // namespace agg

// The no-allocation entry point's scratch (agg_run_noalloc): 64 KiB for the
// partials of any canonical shape (at most kSegTarget segments), then 256
// bytes whose first word counts the scan's finished workgroups (zero between
// calls; a device array starts zeroed).
constexpr int64_t kScratchSlots = kSegTarget;
static __device__ __align__(256) uint64_t scratch[kScratchSlots + 32];

struct agg_plan_s {
  int device = 0;
  int32_t dtype = 0, op = 0, prec = 0, src = 0;
  int64_t max_n = 0;
  bool tune_given = false;
  agg_tune tune{};
  int kind = -1;
  int width = 0;
  void* ws = nullptr;             // segment partial slots
  uint64_t* part = nullptr;
  uint32_t* err = nullptr;        // packed scans: corrupt-header flag (zero between calls)
  uint32_t* done = nullptr;       // single-launch scans: finished-workgroup count (zero between calls)
  // pinned-host staging
  int depth = 0;
  int64_t stage_bytes = 0;
  char* stage[4] = {nullptr, nullptr, nullptr, nullptr};
  hipStream_t copy_stream = nullptr;
  hipEvent_t copied[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t consumed[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t start = nullptr;     // orders the copies after earlier work on the caller's stream
  bool slot_used[4] = {false, false, false, false};
};

struct agg_batch_s {
  int device = 0;
  int32_t ncols = 0;
  agg_tune tune{};
  int64_t nitems = 0;
  int64_t nslots = 0;
  void* ws = nullptr;
  BatchColDev* dcols = nullptr;
  WorkItem* ditems = nullptr;
  uint64_t* dpart = nullptr;
  agg_result* dres = nullptr;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void plan_release(agg_plan_s* p) {
  if (!p) return;
  for (int i = 0; i < 4; ++i) {
    if (p->copied[i]) (void)hipEventDestroy(p->copied[i]);
    if (p->consumed[i]) (void)hipEventDestroy(p->consumed[i]);
    if (p->stage[i]) (void)hipFree(p->stage[i]);
  }
  if (p->start) (void)hipEventDestroy(p->start);
  if (p->copy_stream) (void)hipStreamDestroy(p->copy_stream);
  if (p->ws) (void)hipFree(p->ws);
  delete p;
}

void batch_release(agg_batch_s* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  if (b->ws) (void)hipFree(b->ws);
  delete b;
}

int alloc_device(void** p, size_t bytes) { return device_alloc(p, bytes); }

#define RET_IF(x)            \
  do {                       \
    int rc_ = (x);           \
    if (rc_ != AGG_OK) {     \
      return rc_;            \
    }                        \
  } while (0)

int plan_create(agg_plan_s* p) {
  // segment partials, selected counts (filtered runs), the packed scan's error
  // word and the single-launch scan's workgroup counter (128 bytes apart)
  const size_t ws_bytes = (size_t)kSegTarget * 8 * 2 + 256;
  RET_IF(alloc_device(&p->ws, ws_bytes));
  p->part = static_cast<uint64_t*>(p->ws);
  p->err = reinterpret_cast<uint32_t*>(static_cast<char*>(p->ws) + (size_t)kSegTarget * 8 * 2);
  p->done = reinterpret_cast<uint32_t*>(static_cast<char*>(p->ws) + (size_t)kSegTarget * 8 * 2 + 128);
  HIPCHK(hipMemset(p->ws, 0, ws_bytes));
  if (p->src == AGG_SRC_PINNED_HOST) {
    agg_shape s;
    shape_of(p->dtype, p->max_n, &s);
    p->depth = p->tune.staging_depth;
    p->stage_bytes = std::max<int64_t>(p->tune.chunk_bytes, s.seg_bytes);
    p->stage_bytes = std::min<int64_t>(p->stage_bytes, std::max<int64_t>(s.nseg, 1) * s.seg_bytes);
    for (int i = 0; i < p->depth; ++i) {
      RET_IF(alloc_device(reinterpret_cast<void**>(&p->stage[i]), (size_t)p->stage_bytes));
      HIPCHK(hipEventCreateWithFlags(&p->copied[i], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&p->consumed[i], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&p->start, hipEventDisableTiming));
    HIPCHK(hipStreamCreateWithFlags(&p->copy_stream, hipStreamNonBlocking));
  }
  HIPCHK(hipDeviceSynchronize());
  return AGG_OK;
}

}  // namespace

namespace {

// Capture the batch graph for launch parameters t: the persistent scan over
// the work table, then one combine workgroup per column.  Replaces any
// previous graph.
int batch_capture(agg_batch_s* b, const agg_tune& t) {
  BatchArgs ba;
  ba.cols = b->dcols;
  ba.items = b->ditems;
  ba.nitems = b->nitems;
  ba.part = b->dpart;
  ba.results = b->dres;
  const void* scan_fn = batch_scan_kernel_ptr(t.unroll, t.nontemporal != 0);
  if (!scan_fn) return AGG_E_INVALID;
  const int grid = grid_for(t, g_dev[b->device].cu, b->nitems);
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  HIPCHK(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  if (b->nitems > 0) {
    void* kargs[] = {&ba};
    e = hipLaunchKernel(scan_fn, dim3(grid), dim3(64 * t.waves_per_block), kargs, 0, b->capture_stream);
  }
  if (e == hipSuccess && b->ncols > 0) {
    int64_t nc = b->ncols;
    void* kargs2[] = {&ba, &nc};
    e = hipLaunchKernel(batch_combine_kernel_ptr(), dim3(b->ncols), dim3(256), kargs2, 0, b->capture_stream);
  }
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->capture_stream, &g);
  b->graph = g;
  HIPCHK(e);
  HIPCHK(e2);
  HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  b->tune = t;
  return AGG_OK;
}

// Small columns take one launch: the scan's last workgroup merges, which
// saves the host one kernel launch (about 3 us of the call).  Only where the
// merge is one round trip of device-scope loads (at most 1024 partials: 16
// loads in flight per lane on a one-wave workgroup) and the finished-
// workgroup counter sees at most one increment per CU; beyond that the
// coherent merge rounds and the contended counter cost the GPU more than the
// separate merge launch (measured up to 2^26 items).
constexpr int64_t kFuseMaxPartials = 1024;

// The scan of a column the kernels can read directly (device memory, or
// page-locked host memory read over PCIe) and the combine (in the same
// launch for small columns), with `part` as the segment-partial scratch
// (kSegTarget 8-byte slots) and `done` as its zeroed workgroup counter.
// Shared by agg_run and agg_run_noalloc; the caller has validated everything.
int enqueue_resident(int kind, int32_t dtype, int32_t op, int32_t prec, const agg_tune& t, int cu, const void* col,
                     int64_t n, agg_result* out, uint64_t* part, uint32_t* done, hipStream_t stream) {
  agg_shape s;
  shape_of(dtype, n, &s);
  const bool is_float_sum = dtype == AGG_F32 && (op == AGG_SUM || op == AGG_AVG);
  CombineArgs c;
  c.part = part;
  c.nseg = s.nseg;
  c.out = out;
  c.n = n;
  c.is_avg = op == AGG_AVG;
  c.prec_used = is_float_sum ? prec : -1;
  const void* combine_fn = combine_kernel_ptr(kind);
  if (!combine_fn) return AGG_E_INVALID;
  if (s.nseg > 0) {
    const bool aligned = (reinterpret_cast<uintptr_t>(col) & 15) == 0;
    const int grid = grid_for(t, cu, s.nseg);
    const bool fused = s.nseg <= kFuseMaxPartials && grid <= cu;
    const void* fn = scan_kernel_ptr(kind, t.unroll, t.nontemporal != 0, aligned, fused);
    if (!fn) return AGG_E_INVALID;
    ScanArgs a;
    a.base = static_cast<const char*>(col);
    a.col_bytes = n * width_of(dtype);
    a.seg_bytes = s.seg_bytes;
    a.seg_lo = 0;
    a.seg_hi = s.nseg;
    a.base_seg = 0;
    a.part = part;
    if (fused) {
      a.done = done;
      a.fin = c;
      return launch(fn, grid, 64 * t.waves_per_block, &a, stream);
    }
    RET_IF(launch(fn, grid, 64 * t.waves_per_block, &a, stream));
  }
  return launch(combine_fn, 1, kCombineThreads, &c, stream);
}

// ------------------------------------------------------------ no-allocation scratch
// agg_run_noalloc's segment partials: one array per device, in the library's
// own device code (each device holds its copy until the process ends).  Its
// name is only a host-side stand-in; host code uses the address that
// hipGetSymbolAddress returns on each device, looked up once per device with
// that device current.
uint64_t* g_scratch[kMaxDevices] = {};

// The device's scratch address (dev must be current).
int scratch_of(int dev, uint64_t** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      g_last_hip = (int32_t)(e != hipSuccess ? e : hipErrorInvalidSymbol);
      return AGG_E_HIP;
    }
    g_scratch[dev] = static_cast<uint64_t*>(ptr);
  }
  *out = g_scratch[dev];
  return AGG_OK;
}

}  // namespace

extern "C" {

int agg_init(int32_t device) {
  RET_IF(device_check(device));
  // set up the no-allocation scratch of this device, with the device current
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != device) HIPCHK(hipSetDevice(device));
  uint64_t* sp = nullptr;
  const int rc = scratch_of(device, &sp);
  if (cur != device) HIPCHK(hipSetDevice(cur));
  return rc;
}

int agg_device_info(int32_t device, int32_t* cu_count, char* arch, int32_t arch_len) {
  const int rc = device_check(device);
  if (rc != AGG_OK && rc != AGG_E_NODEVICE) return rc;
  if (!g_dev[device].checked || g_dev[device].cu == 0) return AGG_E_NODEVICE;
  if (cu_count) *cu_count = g_dev[device].cu;
  if (arch && arch_len > 0) std::snprintf(arch, (size_t)arch_len, "%s", g_dev[device].arch);
  return rc;
}

int agg_canonical_shape(int32_t dtype, int64_t n, agg_shape* out) {
  if (!out || width_of(dtype) == 0 || n < 0 || n > kMaxItems) return AGG_E_INVALID;
  shape_of(dtype, n, out);
  return AGG_OK;
}

int agg_default_tune(int32_t dtype, int32_t op, int32_t prec, int64_t n, int32_t src, agg_tune* out) {
  const int kind = kind_of(dtype, op, prec);
  if (!out || kind < 0 || n < 0 || n > kMaxItems || src < AGG_SRC_DEVICE || src > AGG_SRC_ZEROCOPY)
    return AGG_E_INVALID;
  tune_for(kind, src, n * width_of(dtype), out);
  return AGG_OK;
}

int agg_plan(agg_plan_t* out, int32_t dtype, int32_t op, int32_t prec, int64_t max_n, int32_t src,
             const agg_tune* tune) {
  if (!out) return AGG_E_INVALID;
  *out = nullptr;
  const int kind = kind_of(dtype, op, prec);
  if (kind < 0 || max_n < 0 || max_n > kMaxItems || src < AGG_SRC_DEVICE || src > AGG_SRC_ZEROCOPY)
    return AGG_E_INVALID;
  agg_tune t;
  if (tune) {
    t = *tune;
    if (!valid_tune(t)) return AGG_E_INVALID;
  } else {
    agg_default_tune(dtype, op, prec, max_n, src, &t);
  }
  int dev = 0;
  RET_IF(current_device(&dev));
  agg_plan_s* p = new (std::nothrow) agg_plan_s();
  if (!p) return AGG_E_NOMEM;
  p->device = dev;
  p->dtype = dtype; p->op = op; p->prec = prec; p->src = src;
  p->max_n = max_n;
  p->tune = t;
  p->tune_given = tune != nullptr;
  p->kind = kind;
  p->width = width_of(dtype);
  const int rc = plan_create(p);
  if (rc != AGG_OK) {
    plan_release(p);
    return rc;
  }
  *out = p;
  return AGG_OK;
}

int agg_plan_info(agg_plan_t plan, int64_t n, agg_shape* shape, agg_tune* tune) {
  if (!plan || n < 0 || n > plan->max_n) return AGG_E_INVALID;
  if (shape) shape_of(plan->dtype, n, shape);
  if (tune) *tune = plan->tune;
  return AGG_OK;
}

int agg_run(agg_plan_t p, const void* col, int64_t n, agg_result* out, void* stream_v) {
  if (!p || !out || n < 0 || n > p->max_n || (n > 0 && !col)) return AGG_E_INVALID;
  if (n > 0 && reinterpret_cast<uintptr_t>(col) % (uintptr_t)p->width != 0) return AGG_E_INVALID;
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  agg_shape s;
  shape_of(p->dtype, n, &s);
  const int64_t bytes = n * p->width;
  if (n > 0) RET_IF(check_pointer(col, bytes, p->src == AGG_SRC_ZEROCOPY ? AGG_SRC_PINNED_HOST : p->src,
                                  p->device));
  RET_IF(check_out_pointer(out, sizeof(agg_result), p->device));
  const agg_tune& t = p->tune;
  const int cu = g_dev[p->device].cu;
  const bool is_float_sum = p->dtype == AGG_F32 && (p->op == AGG_SUM || p->op == AGG_AVG);

  ScanArgs a;
  a.col_bytes = bytes;
  a.seg_bytes = s.seg_bytes;
  a.part = p->part;
  CombineArgs c;
  c.part = p->part;
  c.nseg = s.nseg;
  c.out = out;
  c.n = n;
  c.is_avg = p->op == AGG_AVG;
  c.prec_used = is_float_sum ? p->prec : -1;
  const void* combine_fn = combine_kernel_ptr(p->kind);
  if (!combine_fn) return AGG_E_INVALID;

  if (p->src != AGG_SRC_PINNED_HOST || n == 0)
    return enqueue_resident(p->kind, p->dtype, p->op, p->prec, t, cu, col, n, out, p->part, p->done, stream);

  // Pinned host: copy chunks of whole segments into the staging ring on the
  // copy stream while the scan of earlier chunks runs on `stream`.
  const void* fn = scan_kernel_ptr(p->kind, t.unroll, t.nontemporal != 0, true);
  if (!fn) return AGG_E_INVALID;
  const int64_t cs = std::max<int64_t>(1, p->stage_bytes / s.seg_bytes);
  const int64_t nchunks = ceil_div(s.nseg, cs);
  const char* host = static_cast<const char*>(col);
  HIPCHK(hipEventRecord(p->start, stream));
  HIPCHK(hipStreamWaitEvent(p->copy_stream, p->start, 0));
  for (int64_t k = 0; k < nchunks; ++k) {
    const int slot = (int)(k % p->depth);
    const int64_t lo = k * cs, hi = std::min(s.nseg, lo + cs);
    const int64_t b0 = lo * s.seg_bytes;
    const int64_t nb = std::min(bytes, hi * s.seg_bytes) - b0;
    if (p->slot_used[slot]) HIPCHK(hipStreamWaitEvent(p->copy_stream, p->consumed[slot], 0));
    HIPCHK(hipMemcpyAsync(p->stage[slot], host + b0, (size_t)nb, hipMemcpyHostToDevice, p->copy_stream));
    HIPCHK(hipEventRecord(p->copied[slot], p->copy_stream));
    HIPCHK(hipStreamWaitEvent(stream, p->copied[slot], 0));
    a.base = p->stage[slot];
    a.seg_lo = lo;
    a.seg_hi = hi;
    a.base_seg = lo;
    RET_IF(launch(fn, grid_for(t, cu, hi - lo), 64 * t.waves_per_block, &a, stream));
    HIPCHK(hipEventRecord(p->consumed[slot], stream));
    p->slot_used[slot] = true;
  }
  return launch(combine_fn, 1, kCombineThreads, &c, stream);
}

int agg_run_noalloc(int32_t dtype, int32_t op, int32_t prec, int32_t src, const void* col, int64_t n,
                    agg_result* out, void* stream_v) {
  const int kind = kind_of(dtype, op, prec);
  if (kind < 0 || !out || n < 0 || n > kMaxItems || (n > 0 && !col)) return AGG_E_INVALID;
  if (src != AGG_SRC_DEVICE && src != AGG_SRC_ZEROCOPY) return AGG_E_INVALID;  // no staging ring
  const int w = width_of(dtype);
  if (n > 0 && reinterpret_cast<uintptr_t>(col) % (uintptr_t)w != 0) return AGG_E_INVALID;
  int dev = 0;
  RET_IF(current_device(&dev));
  agg_shape s;
  shape_of(dtype, n, &s);
  if (s.nseg > kScratchSlots) return AGG_E_INVALID;  // cannot happen: a canonical shape has <= 8192 segments
  if (n > 0) RET_IF(check_pointer(col, n * w, src == AGG_SRC_ZEROCOPY ? AGG_SRC_PINNED_HOST : AGG_SRC_DEVICE, dev));
  RET_IF(check_out_pointer(out, sizeof(agg_result), dev));
  uint64_t* part = nullptr;
  RET_IF(scratch_of(dev, &part));
  agg_tune t;
  tune_for(kind, src, n * w, &t);
  return enqueue_resident(kind, dtype, op, prec, t, g_dev[dev].cu, col, n, out, part,
                          reinterpret_cast<uint32_t*>(part + kScratchSlots), static_cast<hipStream_t>(stream_v));
}

namespace {

// An agg_filter as an inclusive range in the filter column's type that
// selects exactly the same items.  Integer bounds: x > a is x >= a + 1 and
// x < b is x <= b - 1, then clamped to the int32 range for int32 columns.
// Float bounds: the smallest float32 v with v >= lo (v > lo) and the largest
// with v <= hi (v < hi); a float32 x satisfies x >= lo exactly when x >= v.
// Returns false for NaN bounds.
bool normalize_filter(const agg_filter& f, RangePred* q) {
  q->ilo = 1;
  q->ihi = 0;
  q->flo = 1.0f;
  q->fhi = 0.0f;
  if (f.dtype == AGG_F32) {
    if (std::isnan(f.flo) || std::isnan(f.fhi)) return false;
    const float inf = std::numeric_limits<float>::infinity();
    if ((!f.lo_inclusive && f.flo == (double)inf) || (!f.hi_inclusive && f.fhi == -(double)inf)) return true;
    float lo = (float)f.flo;  // nearest float32; move up until it is the first one that qualifies
    if ((double)lo < f.flo || (!f.lo_inclusive && (double)lo == f.flo)) lo = std::nextafter(lo, inf);
    float hi = (float)f.fhi;
    if ((double)hi > f.fhi || (!f.hi_inclusive && (double)hi == f.fhi)) hi = std::nextafter(hi, -inf);
    q->flo = lo;
    q->fhi = hi;
    return true;
  }
  int64_t lo = f.ilo, hi = f.ihi;
  if (!f.lo_inclusive) {
    if (lo == INT64_MAX) return true;  // x > INT64_MAX: nothing
    ++lo;
  }
  if (!f.hi_inclusive) {
    if (hi == INT64_MIN) return true;
    --hi;
  }
  if (f.dtype == AGG_I32) {
    if (lo > INT32_MAX || hi < INT32_MIN) return true;
    lo = std::max<int64_t>(lo, INT32_MIN);
    hi = std::min<int64_t>(hi, INT32_MAX);
  }
  q->ilo = lo;
  q->ihi = hi;
  return true;
}

}  // namespace

int agg_run_filtered(agg_plan_t p, const void* col, int64_t n, const agg_filter* filter, agg_result* out,
                     void* stream_v) {
  if (!p || !filter || !out || n < 0 || n > p->max_n || (n > 0 && (!col || !filter->col))) return AGG_E_INVALID;
  if (p->src != AGG_SRC_DEVICE) return AGG_E_INVALID;
  const int fw = width_of(filter->dtype);
  if (fw == 0 || (filter->lo_inclusive != 0 && filter->lo_inclusive != 1) ||
      (filter->hi_inclusive != 0 && filter->hi_inclusive != 1))
    return AGG_E_INVALID;
  if (n > 0 && (reinterpret_cast<uintptr_t>(col) % (uintptr_t)p->width != 0 ||
                reinterpret_cast<uintptr_t>(filter->col) % (uintptr_t)fw != 0))
    return AGG_E_INVALID;
  if (n > 0) {
    RET_IF(check_pointer(col, n * p->width, AGG_SRC_DEVICE, p->device));
    RET_IF(check_pointer(filter->col, n * fw, AGG_SRC_DEVICE, p->device));
  }
  RET_IF(check_out_pointer(out, sizeof(agg_result), p->device));
  RangePred pred;
  if (!normalize_filter(*filter, &pred)) return AGG_E_INVALID;
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  agg_shape s;
  shape_of(p->dtype, n, &s);
  const bool aligned = ((reinterpret_cast<uintptr_t>(col) | reinterpret_cast<uintptr_t>(filter->col)) & 15) == 0;
  const void* fn = filter_scan_kernel_ptr(p->kind, filter->dtype, aligned);
  const void* comb = filter_combine_kernel_ptr(p->kind);
  if (!fn || !comb) return AGG_E_INVALID;
  uint64_t* cpart = p->part + kSegTarget;
  if (s.nseg > 0) {
    FilterArgs a;
    a.base = static_cast<const char*>(col);
    a.fbase = static_cast<const char*>(filter->col);
    a.col_bytes = n * p->width;
    a.seg_bytes = s.seg_bytes;
    a.nseg = s.nseg;
    a.part = p->part;
    a.cpart = cpart;
    // the predicate and the masking add VALU work: more waves than the plain
    // scan (4 per CU measured best for 4- and 8-byte value / filter pairs)
    agg_tune t = p->tune;
    if (!p->tune_given) {
      t.waves_per_block = 4;
      t.blocks_per_cu = 1;
    }
    a.pred = pred;
    RET_IF(launch(fn, grid_for(t, g_dev[p->device].cu, s.nseg), 64 * t.waves_per_block, &a, stream));
  }
  FilterCombineArgs c;
  c.part = p->part;
  c.cpart = cpart;
  c.nseg = s.nseg;
  c.out = out;
  c.is_avg = p->op == AGG_AVG;
  c.prec_used = (p->dtype == AGG_F32 && (p->op == AGG_SUM || p->op == AGG_AVG)) ? p->prec : -1;
  return launch(comb, 1, kCombineThreads, &c, stream);
}

int agg_run_packed(agg_plan_t p, const agg_packed* col, agg_result* out, void* stream_v) {
  if (!p || !col || !out || p->dtype != AGG_I32 || col->dtype != AGG_I32) return AGG_E_INVALID;
  if (p->src != AGG_SRC_DEVICE && p->src != AGG_SRC_ZEROCOPY) return AGG_E_INVALID;
  const int64_t n = col->n;
  if (n < 0 || n > p->max_n || col->payload_words < 0) return AGG_E_INVALID;
  const int64_t nblocks = ceil_div(n, AGG_PACK_BLOCK);
  if (nblocks > 0 && !col->blocks) return AGG_E_INVALID;
  if (col->payload_words > 0 && !col->payload) return AGG_E_INVALID;
  if (col->payload_words > nblocks * 64 * 32) return AGG_E_INVALID;
  const int32_t kind_src = p->src == AGG_SRC_ZEROCOPY ? AGG_SRC_PINNED_HOST : AGG_SRC_DEVICE;
  if (nblocks > 0)
    RET_IF(check_pointer(col->blocks, nblocks * (int64_t)sizeof(agg_packed_block), kind_src, p->device));
  if (col->payload_words > 0) RET_IF(check_pointer(col->payload, col->payload_words * 4, kind_src, p->device));
  RET_IF(check_out_pointer(out, sizeof(agg_result), p->device));
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  CombineArgs c;
  c.part = p->part;
  c.out = out;
  c.n = n;
  c.is_avg = p->op == AGG_AVG;
  c.prec_used = -1;
  c.nseg = 0;
  if (p->op == AGG_COUNT) {  // n, no decoding needed
    const void* comb = combine_kernel_ptr(p->kind);
    agg_shape s;
    shape_of(p->dtype, n, &s);
    if (s.nseg > 0) {  // count through the plain coverage kernel (issues no loads)
      ScanArgs a;
      a.base = nullptr;
      a.col_bytes = n * 4;
      a.seg_bytes = s.seg_bytes;
      a.seg_lo = 0;
      a.seg_hi = s.nseg;
      a.base_seg = 0;
      a.part = p->part;
      const void* fn = scan_kernel_ptr(p->kind, p->tune.unroll, p->tune.nontemporal != 0, true);
      RET_IF(launch(fn, grid_for(p->tune, g_dev[p->device].cu, s.nseg), 64 * p->tune.waves_per_block, &a, stream));
    }
    c.nseg = s.nseg;
    return launch(comb, 1, kCombineThreads, &c, stream);
  }
  const void* fn = packed_scan_kernel_ptr(p->kind);
  const void* comb = combine_kernel_ptr(p->kind);
  if (!fn || !comb) return AGG_E_INVALID;
  // The decode costs about 6 VALU operations per item, so it wants more
  // waves than the plain scan: 8 per CU unless the plan was given parameters.
  agg_tune t = p->tune;
  if (!p->tune_given) {
    t.waves_per_block = 8;
    t.blocks_per_cu = 1;
  }
  // one partial per wave: at most kSegTarget waves, at most one per block
  int64_t waves = std::min<int64_t>((int64_t)t.blocks_per_cu * g_dev[p->device].cu * t.waves_per_block,
                                    std::max<int64_t>(nblocks, 1));
  waves = std::min<int64_t>(waves, kSegTarget);
  const int grid = (int)std::max<int64_t>(1, waves / t.waves_per_block);
  PackedArgs a;
  a.blocks = col->blocks;
  a.payload = col->payload;
  a.n = n;
  a.nblocks = nblocks;
  a.payload_words = col->payload_words;
  a.part = p->part;
  a.err = p->err;
  c.nseg = (int64_t)grid * t.waves_per_block;
  c.err = p->err;
  RET_IF(launch(fn, grid, 64 * t.waves_per_block, &a, stream));
  return launch(comb, 1, kCombineThreads, &c, stream);
}

int agg_plan_destroy(agg_plan_t plan) {
  if (!plan) return AGG_E_INVALID;
  if (plan->copy_stream) (void)hipStreamSynchronize(plan->copy_stream);
  (void)hipDeviceSynchronize();
  plan_release(plan);
  return AGG_OK;
}

// ------------------------------------------------------------ batch
int agg_batch_plan(agg_batch_t* out, const agg_col* cols, int32_t ncols, const agg_tune* tune) {
  if (!out || ncols < 0 || (ncols > 0 && !cols)) return AGG_E_INVALID;
  *out = nullptr;
  agg_tune t;
  if (tune) {
    t = *tune;
    if (!valid_tune(t)) return AGG_E_INVALID;
  } else {
    batch_builtin_tune(&t);
  }
  for (int32_t i = 0; i < ncols; ++i) {  // host-side checks first
    const agg_col& c = cols[i];
    const int w = width_of(c.dtype);
    if (kind_of(c.dtype, c.op, c.prec) < 0 || c.n < 0 || c.n > kMaxItems || (c.n > 0 && !c.ptr))
      return AGG_E_INVALID;
    if (c.n > 0 && reinterpret_cast<uintptr_t>(c.ptr) % (uintptr_t)w != 0) return AGG_E_INVALID;
  }
  int dev = 0;
  RET_IF(current_device(&dev));

  // Work items of run_bytes: the batch's bytes over 64 items for each of
  // 4 waves per CU, as a power of two within [64 KiB, 256 KiB].  Smaller
  // items even out the waves' shares of a small batch; larger ones cost less
  // per byte (measured on the two 4096-column benchmark sets, 5.7 and 23.7 GB:
  // 64 KiB items 0.805 / 0.850 of HBM, 256 KiB 0.795 / 0.853, 1 MiB 0.74 / 0.83).
  int64_t total_bytes = 0;
  for (int32_t i = 0; i < ncols; ++i) total_bytes += cols[i].n * width_of(cols[i].dtype);
  const int64_t item_target = total_bytes / ((int64_t)std::max(1, g_dev[dev].cu) * 4 * 64);
  int64_t run_bytes = kItemMaxBytes;
  while (run_bytes > kItemMinBytes && run_bytes > item_target) run_bytes >>= 1;

  std::vector<BatchColDev> hc((size_t)ncols);
  std::vector<WorkItem> items;
  int64_t slots = 0;
  for (int32_t i = 0; i < ncols; ++i) {
    const agg_col& c = cols[i];
    const int kind = kind_of(c.dtype, c.op, c.prec);
    const int w = width_of(c.dtype);
    if (c.n > 0) RET_IF(check_pointer(c.ptr, c.n * w, AGG_SRC_DEVICE, dev));
    agg_shape s;
    shape_of(c.dtype, c.n, &s);
    BatchColDev& d = hc[(size_t)i];
    d.ptr = static_cast<const char*>(c.ptr);
    d.col_bytes = c.n * w;
    d.seg_bytes = s.seg_bytes;
    d.nseg = s.nseg;
    d.part_off = slots;
    d.n = c.n;
    d.kind = kind;
    d.is_avg = c.op == AGG_AVG;
    d.prec_used = (c.dtype == AGG_F32 && (c.op == AGG_SUM || c.op == AGG_AVG)) ? c.prec : -1;
    d.aligned = (reinterpret_cast<uintptr_t>(c.ptr) & 15) == 0;
    slots += s.nseg;
    if (slots > (int64_t)UINT32_MAX) return AGG_E_INVALID;  // partial slots are indexed by 32 bits
    const int64_t per = std::max<int64_t>(1, run_bytes / s.seg_bytes);
    for (int64_t lo = 0; lo < s.nseg; lo += per) {
      WorkItem it{};
      it.ptr = d.ptr;
      it.col_bytes = d.col_bytes;
      it.part_off = (uint32_t)d.part_off;
      it.seg_lo = (uint16_t)lo;
      it.seg_hi = (uint16_t)std::min<int64_t>(s.nseg, lo + per);
      it.seg_log2 = (uint8_t)__builtin_ctzll((uint64_t)d.seg_bytes);
      it.kind = (uint8_t)d.kind;
      it.aligned = (uint8_t)d.aligned;
      items.push_back(it);
    }
  }
  // Largest items first: waves take items w, w + P, w + 2P, ..., so this
  // evens out their totals (the order decides nothing about the results: each
  // segment's partial has its own slot and columns merge in canonical order).
  auto item_bytes = [](const WorkItem& it) {
    const int64_t sb = (int64_t)1 << it.seg_log2;
    return std::min(it.col_bytes, it.seg_hi * sb) - it.seg_lo * sb;
  };
  std::stable_sort(items.begin(), items.end(),
                   [&](const WorkItem& x, const WorkItem& y) { return item_bytes(x) > item_bytes(y); });

  agg_batch_s* b = new (std::nothrow) agg_batch_s();
  if (!b) return AGG_E_NOMEM;
  b->device = dev;
  b->ncols = ncols;
  b->tune = t;
  b->nitems = (int64_t)items.size();
  b->nslots = slots;
  auto fail = [&](int rc) {
    batch_release(b);
    return rc;
  };
  const size_t cols_b = sizeof(BatchColDev) * (size_t)std::max(ncols, 1);
  const size_t items_b = sizeof(WorkItem) * (size_t)std::max<int64_t>(b->nitems, 1);
  const size_t part_b = 8 * (size_t)std::max<int64_t>(slots, 1);
  const size_t res_b = sizeof(agg_result) * (size_t)std::max(ncols, 1);
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t total = up(cols_b) + up(items_b) + up(part_b) + up(res_b);
  int rc = alloc_device(&b->ws, total);
  if (rc != AGG_OK) return fail(rc);
  char* base = static_cast<char*>(b->ws);
  b->dcols = reinterpret_cast<BatchColDev*>(base);
  b->ditems = reinterpret_cast<WorkItem*>(base + up(cols_b));
  b->dpart = reinterpret_cast<uint64_t*>(base + up(cols_b) + up(items_b));
  b->dres = reinterpret_cast<agg_result*>(base + up(cols_b) + up(items_b) + up(part_b));
  auto hip_fail = [&](hipError_t e) {
    g_last_hip = (int32_t)e;
    return fail(AGG_E_HIP);
  };
  hipError_t e;
  if (ncols > 0 && (e = hipMemcpy(b->dcols, hc.data(), sizeof(BatchColDev) * (size_t)ncols,
                                  hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e);
  if (b->nitems > 0 && (e = hipMemcpy(b->ditems, items.data(), sizeof(WorkItem) * (size_t)b->nitems,
                                      hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e);
  if ((e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e);

  const int rc2 = batch_capture(b, t);
  if (rc2 != AGG_OK) return fail(rc2);
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e);
  *out = b;
  return AGG_OK;
}

int agg_batch_run(agg_batch_t b, agg_result* out, void* stream_v) {
  if (!b || (b->ncols > 0 && !out)) return AGG_E_INVALID;
  if (b->ncols == 0) return AGG_OK;
  RET_IF(check_out_pointer(out, (int64_t)sizeof(agg_result) * b->ncols, b->device));
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  HIPCHK(hipGraphLaunch(b->exec, stream));
  HIPCHK(hipMemcpyAsync(out, b->dres, sizeof(agg_result) * (size_t)b->ncols, hipMemcpyDefault, stream));
  return AGG_OK;
}

int agg_batch_destroy(agg_batch_t b) {
  if (!b) return AGG_E_INVALID;
  (void)hipDeviceSynchronize();
  batch_release(b);
  return AGG_OK;
}

int agg_batch_retune(agg_batch_t b, const agg_tune* tune) {
  if (!b || !tune || !valid_tune(*tune)) return AGG_E_INVALID;
  HIPCHK(hipStreamSynchronize(b->capture_stream));
  return batch_capture(b, *tune);
}

int agg_batch_info(agg_batch_t b, int64_t* nitems, int64_t* nseg_total, agg_tune* tune) {
  if (!b) return AGG_E_INVALID;
  if (nitems) *nitems = b->nitems;
  if (nseg_total) *nseg_total = b->nslots;
  if (tune) *tune = b->tune;
  return AGG_OK;
}

int agg_batch_autotune(agg_batch_t b, void* stream_v, agg_tune* best, double* best_ms_out) {
  if (!b) return AGG_E_INVALID;
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  if (b->ncols == 0) {
    if (best) *best = b->tune;
    if (best_ms_out) *best_ms_out = 0.0;
    return AGG_OK;
  }
  const int wb[][2] = {{1, 2}, {2, 1}, {4, 1}, {1, 3}, {2, 2}, {4, 2}, {8, 1}, {1, 4}};
  agg_tune best_t = b->tune;
  double best_ms = -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    HIPCHK(e);
  }
  int rc = AGG_OK;
  for (int u : {4, 8, 16}) {  // 32 spills registers in the batch kernel
    for (auto& p : wb) {
      agg_tune t = b->tune;
      t.unroll = u;
      t.waves_per_block = p[0];
      t.blocks_per_cu = p[1];
      rc = batch_capture(b, t);
      if (rc != AGG_OK) break;
      if ((e = hipGraphLaunch(b->exec, stream)) != hipSuccess) { g_last_hip = (int32_t)e; rc = AGG_E_HIP; break; }
      if ((e = hipEventRecord(e0, stream)) != hipSuccess) { g_last_hip = (int32_t)e; rc = AGG_E_HIP; break; }
      for (int r = 0; r < 3 && e == hipSuccess; ++r) e = hipGraphLaunch(b->exec, stream);
      if (e == hipSuccess) e = hipEventRecord(e1, stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) { g_last_hip = (int32_t)e; rc = AGG_E_HIP; break; }
      if (best_ms < 0 || ms / 3 < best_ms) {
        best_ms = ms / 3;
        best_t = t;
      }
    }
    if (rc != AGG_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != AGG_OK) return rc;
  RET_IF(batch_capture(b, best_t));
  if (best) *best = best_t;
  if (best_ms_out) *best_ms_out = best_ms;
  return AGG_OK;
}

int agg_fault_inject(int32_t site, int32_t countdown) {
  if (site <= AGG_FAULT_NONE || site >= AGG_FAULT_SITES || countdown < 0) return AGG_E_INVALID;
  fault_env();  // the environment is read first, so this call wins over it
  g_fault[site].store(countdown);
  return AGG_OK;
}

const char* agg_strerror(int32_t code) {
  switch (code) {
    case AGG_OK: return "ok";
    case AGG_E_INVALID: return "invalid argument";
    case AGG_E_NOMEM: return "out of device memory";
    case AGG_E_NODEVICE: return "no gfx950 HIP device";
    case AGG_E_HIP: return "HIP runtime error";
    default: return "unknown error";
  }
}

int32_t agg_last_hip_error(void) { return g_last_hip; }

}  // extern "C"

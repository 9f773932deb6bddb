// Serving: continuous admission of aggregation requests on one GPU.
//
// Requests arrive over time (Poisson in the benchmark workload).  The
// scheduler admits them in arrival order into a fixed number of slots as
// slots and HBM free up; a slot owns a compute stream and a copy stream, so
// the work of admitted requests overlaps on the device.  A resident request
// scans a column already in HBM.  A shipped request reserves room for its
// column in a device arena of `hbm_budget_bytes`, copies it over PCIe in
// chunks while the scan of earlier chunks runs (the paper's end-to-end
// setting, Section 5.3), and may stay resident afterwards in an LRU cache
// keyed by column id, so later requests for the same column skip the copy.
//
// Every request runs the same kernels and canonical reduction shape as
// agg_run, so its result is bit-identical alone and in any mix.
//
// The scheduler is plain host logic behind an executor interface: the HIP
// executor runs requests on the GPU; a simulated executor (modelled PCIe and
// HBM rates, simulated clock) drives the same scheduler on the CPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "agg.h"
#include "agg_internal.hpp"

namespace agg {
namespace serve {

constexpr int kMaxSlots = 64;
constexpr int64_t kGranule = 256;

int64_t round_up(int64_t b) { return (b + kGranule - 1) / kGranule * kGranule; }

// First-fit allocator over the device arena [0, capacity).
class Arena {
 public:
  explicit Arena(int64_t cap) : cap_(cap) {
    if (cap > 0) free_[0] = cap;
  }
  bool alloc(int64_t bytes, int64_t* off) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const int64_t rest = it->second - bytes, noff = it->first + bytes;
      free_.erase(it);
      if (rest) free_[noff] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = round_up(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t capacity() const { return cap_; }
  int64_t peak() const { return peak_; }

 private:
  int64_t cap_ = 0, used_ = 0, peak_ = 0;
  std::map<int64_t, int64_t> free_;
};

// Shipped columns kept in HBM after their request, least recently used first out.
struct CacheEntry {
  int64_t off, bytes;
  int users;
  uint64_t stamp;
};
class Cache {
 public:
  CacheEntry* lookup(int64_t id, int64_t bytes) {
    auto it = map_.find(id);
    if (it == map_.end() || it->second.bytes != bytes) return nullptr;
    it->second.stamp = ++clock_;
    return &it->second;
  }
  // Keep (off, bytes) for id; false if id is already cached (caller frees its copy).
  bool insert(int64_t id, int64_t off, int64_t bytes) {
    if (map_.count(id)) return false;
    map_[id] = CacheEntry{off, bytes, 0, ++clock_};
    return true;
  }
  // Allocate `bytes`, evicting idle entries in LRU order while needed.
  bool make_room(Arena& a, int64_t bytes, int64_t* off) {
    while (!a.alloc(bytes, off)) {
      auto victim = map_.end();
      for (auto it = map_.begin(); it != map_.end(); ++it)
        if (it->second.users == 0 && (victim == map_.end() || it->second.stamp < victim->second.stamp))
          victim = it;
      if (victim == map_.end()) return false;
      a.release(victim->second.off, victim->second.bytes);
      map_.erase(victim);
    }
    return true;
  }

 private:
  std::unordered_map<int64_t, CacheEntry> map_;
  uint64_t clock_ = 0;
};

struct Job {
  int req = -1;
  int kind = -1;
  bool ship = false;        // copy the column over PCIe into the arena
  bool from_arena = false;  // the column is read from the arena (shipped or cached)
  bool cached = false;      // a cache hit
  int64_t off = 0;
  int64_t bytes = 0;
};

class Executor {
 public:
  virtual ~Executor() {}
  virtual int start(int slot, const agg_request& r, const Job& j) = 0;
  virtual int poll(int slot) = 0;  // 1 done, 0 running, < 0 error
  virtual void finish(int slot, agg_result* out) = 0;
  virtual double now() = 0;
  virtual void wait(double until) = 0;
};

class Scheduler {
 public:
  Scheduler(const agg_serve_config& cfg, Executor& ex) : cfg_(cfg), ex_(ex), arena_(cfg.hbm_budget_bytes) {}

  int run(const agg_request* reqs, int32_t n, agg_result* results, agg_request_stats* stats,
          agg_serve_summary* sum) {
    std::vector<Job> slot(cfg_.max_slots);
    std::vector<bool> busy(cfg_.max_slots, false);
    std::deque<int> pending;
    int next = 0, finished = 0, nbusy = 0, peak_busy = 0, hits = 0, failed = 0, nship = 0;
    int64_t scanned = 0, shipped = 0;
    double first = n ? reqs[0].arrival_s : 0.0, last = 0.0;
    for (int i = 0; i < n; ++i) {
      std::memset(&stats[i], 0, sizeof stats[i]);
      std::memset(&results[i], 0, sizeof results[i]);
      stats[i].arrival_s = reqs[i].arrival_s;
      stats[i].slot = -1;
    }
    while (finished < n) {
      bool progress = false;
      const double now = ex_.now();
      while (next < n && reqs[next].arrival_s <= now) pending.push_back(next++);
      // completions
      for (int s = 0; s < cfg_.max_slots; ++s) {
        if (!busy[s]) continue;
        const int st = ex_.poll(s);
        if (st == 0) continue;
        Job& j = slot[s];
        agg_request_stats& rs = stats[j.req];
        if (st > 0) {
          ex_.finish(s, &results[j.req]);
          rs.status = AGG_OK;
        } else {
          rs.status = st;
          ++failed;
        }
        rs.done_s = ex_.now();
        last = std::max(last, rs.done_s);
        release(j, st > 0);
        busy[s] = false;
        --nbusy;
        nship -= j.ship ? 1 : 0;
        ++finished;
        progress = true;
        if (cfg_.progress_every > 0 && finished % cfg_.progress_every == 0) {
          std::fprintf(stderr, "agg_serve: %d of %d requests done at %.3f s\n", finished, n, rs.done_s - first);
          std::fflush(stderr);
        }
      }
      // admissions, in arrival order; a shipped request that does not fit
      // blocks later shipped requests (FIFO for HBM) but not resident or
      // cached ones, which need no memory.
      bool memory_blocked = false;
      for (auto it = pending.begin(); it != pending.end() && nbusy < cfg_.max_slots;) {
        const int i = *it;
        const agg_request& r = reqs[i];
        Job j;
        j.req = i;
        j.kind = kind_of(r.dtype, r.op, r.prec);
        j.bytes = r.n * width_of(r.dtype);
        bool admit = false;
        if (r.resident) {
          admit = true;
        } else if (CacheEntry* c = cfg_.cache_shipped ? cache_.lookup(r.column_id, j.bytes) : nullptr) {
          j.from_arena = j.cached = true;
          j.off = c->off;
          c->users++;
          admit = true;
        } else if (round_up(j.bytes) > arena_.capacity()) {
          stats[i].status = AGG_E_NOMEM;  // can never fit the budget
          stats[i].admit_s = stats[i].done_s = ex_.now();
          ++failed;
          ++finished;
          it = pending.erase(it);
          progress = true;
          continue;
        } else if (!memory_blocked && (j.bytes == 0 || (nship < cfg_.max_shipping &&
                                                         cache_.make_room(arena_, j.bytes, &j.off)))) {
          j.ship = j.bytes > 0;
          j.from_arena = j.bytes > 0;
          admit = true;
        } else {
          memory_blocked = true;
        }
        if (!admit) {
          ++it;
          continue;
        }
        int s = 0;
        while (busy[s]) ++s;
        agg_request_stats& rs = stats[i];
        rs.admit_s = ex_.now();
        rs.slot = s;
        rs.cache_hit = j.cached ? 1 : 0;
        rs.bytes_shipped = j.ship ? j.bytes : 0;
        const int rc = ex_.start(s, r, j);
        if (rc != AGG_OK) {
          rs.status = rc;
          rs.done_s = ex_.now();
          release(j, false);
          ++failed;
          ++finished;
        } else {
          slot[s] = j;
          busy[s] = true;
          ++nbusy;
          nship += j.ship ? 1 : 0;
          peak_busy = std::max(peak_busy, nbusy);
          scanned += j.bytes;
          shipped += rs.bytes_shipped;
          hits += j.cached ? 1 : 0;
        }
        it = pending.erase(it);
        progress = true;
      }
      if (!progress && finished < n) ex_.wait(next < n ? reqs[next].arrival_s : std::numeric_limits<double>::infinity());
    }
    sum->makespan_s = n ? last - first : 0.0;
    sum->bytes_scanned = scanned;
    sum->bytes_shipped = shipped;
    sum->peak_reserved_bytes = arena_.peak();
    sum->peak_busy_slots = peak_busy;
    sum->completed = n - failed;
    sum->failed = failed;
    sum->cache_hits = hits;
    return AGG_OK;
  }

 private:
  // The job's memory after it ended.  Only a shipped column whose request
  // succeeded may enter the cache: after a failed copy (or a failed start)
  // the region holds partial data, so it goes back to the arena.
  void release(const Job& j, bool ok) {
    if (j.cached) {
      if (CacheEntry* c = cache_.lookup(reqs_id(j), j.bytes)) c->users--;
      return;
    }
    if (!j.ship) return;
    if (ok && cfg_.cache_shipped && cache_.insert(cur_ids_[j.req], j.off, j.bytes)) return;
    arena_.release(j.off, j.bytes);
  }
  int64_t reqs_id(const Job& j) { return cur_ids_[j.req]; }

 public:
  std::vector<int64_t> cur_ids_;  // column id per request

 private:
  agg_serve_config cfg_;
  Executor& ex_;
  Arena arena_;
  Cache cache_;
};

// ------------------------------------------------------------ GPU executor
// Chunks of a shipped column in flight per slot.  The host drives the
// pipeline: it starts the scan of a chunk only after seeing its copy finish,
// and then starts the next copy, so no compute queue ever holds a wait on a
// PCIe copy.  Each in-flight chunk has a copy stream of its own, and the host
// sees its completion by querying that stream: an event recorded after a
// copy puts exactly such a wait into a hardware queue that other streams
// share (with more streams than hardware queues), and measured, it held a
// tiny kernel on an unrelated stream for the whole copy backlog (100+ ms)
// where the stream query left it at 15 us.
constexpr int kPipe = 4;

struct SlotRun {
  bool ship = false;
  bool combined = false;
  ScanArgs a{};
  CombineArgs c{};
  const void* scan_fn = nullptr;
  const void* comb_fn = nullptr;
  agg_tune t{};
  int64_t nseg = 0, seg_bytes = 0, cs = 1, nchunks = 0, bytes = 0;
  int64_t next_copy = 0, next_scan = 0;
  const char* host = nullptr;
  char* dst = nullptr;
};

class HipExecutor : public Executor {
 public:
  explicit HipExecutor(agg_server_s* s);
  int start(int slot, const agg_request& r, const Job& j) override;
  int poll(int slot) override;
  void finish(int slot, agg_result* out) override { *out = res_host_[slot]; }
  double now() override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }
  void wait(double until) override {
    const double dt = until - now();
    if (dt > 50e-6) std::this_thread::sleep_for(std::chrono::microseconds(20));
    else std::this_thread::yield();
  }

 private:
  int copy_chunk(int slot, int64_t k);
  int scan_chunk(int slot, int64_t k);
  int finish_launches(int slot);
  int fail(int slot, int rc);
  agg_server_s* s_;
  agg_result* res_host_;
  std::vector<SlotRun> run_;
  std::chrono::steady_clock::time_point t0_;
};

// ------------------------------------------------------------ simulated executor
class SimExecutor : public Executor {
 public:
  SimExecutor(int slots, double pcie_gbs, double hbm_gbs, double launch_s)
      : done_at_(slots, -1.0), failing_(slots, false), pcie_(pcie_gbs * 1e9), hbm_(hbm_gbs * 1e9),
        launch_(launch_s) {}
  int start(int slot, const agg_request& r, const Job& j) override {
    const double scan = (double)j.bytes / hbm_;
    double end = t_ + launch_ + scan;
    failing_[slot] = false;
    if (j.ship) {  // one shared link; the scan of the last chunk follows the copy
      const double begin = std::max(t_, link_free_);
      link_free_ = begin + (double)j.bytes / pcie_;
      end = std::max(end, link_free_ + launch_);
      failing_[slot] = fault_hit(AGG_FAULT_SHIP);  // the copy fails: the job ends with an error
    }
    done_at_[slot] = end;
    n_[slot] = r.n;
    return AGG_OK;
  }
  int poll(int slot) override {
    if (done_at_[slot] < 0 || t_ < done_at_[slot]) return 0;
    if (!failing_[slot]) return 1;
    done_at_[slot] = -1.0;
    return AGG_E_HIP;
  }
  void finish(int slot, agg_result* out) override {
    std::memset(out, 0, sizeof *out);
    out->count = n_[slot];
    out->prec_used = -1;
    done_at_[slot] = -1.0;
  }
  double now() override { return t_; }
  void wait(double until) override {
    double next = until;
    for (double d : done_at_)
      if (d >= 0 && d < next) next = d;
    if (!std::isfinite(next)) next = t_ + 1e-3;  // nothing scheduled: cannot happen with work pending
    t_ = std::max(t_, next);
  }

 private:
  std::vector<double> done_at_;
  std::vector<bool> failing_;
  std::map<int, int64_t> n_;
  double pcie_, hbm_, launch_;
  double t_ = 0.0, link_free_ = 0.0;
};

int validate(const agg_serve_config* cfg, const agg_request* reqs, int32_t n, bool need_device, int dev) {
  if (!cfg || n < 0 || (n > 0 && !reqs)) return AGG_E_INVALID;
  if (cfg->max_slots < 1 || cfg->max_slots > kMaxSlots || cfg->hbm_budget_bytes < 0) return AGG_E_INVALID;
  if (cfg->max_shipping < 1 || cfg->max_shipping > cfg->max_slots) return AGG_E_INVALID;
  if (cfg->chunk_bytes < (1 << 20) || cfg->chunk_bytes > ((int64_t)1 << 32)) return AGG_E_INVALID;
  for (int32_t i = 0; i < n; ++i) {
    const agg_request& r = reqs[i];
    if (kind_of(r.dtype, r.op, r.prec) < 0 || r.n < 0 || r.n > ((int64_t)1 << 40)) return AGG_E_INVALID;
    if (!(r.arrival_s >= 0.0) || (i > 0 && r.arrival_s < reqs[i - 1].arrival_s)) return AGG_E_INVALID;
    if (r.n > 0 && !r.ptr) return AGG_E_INVALID;
    const int w = width_of(r.dtype);
    if (r.n > 0 && reinterpret_cast<uintptr_t>(r.ptr) % (uintptr_t)w != 0) return AGG_E_INVALID;
    if (need_device && r.n > 0) {
      const int rc = check_pointer(r.ptr, r.n * w, r.resident ? AGG_SRC_DEVICE : AGG_SRC_PINNED_HOST, dev);
      if (rc != AGG_OK) return rc;
    }
  }
  return AGG_OK;
}

}  // namespace serve
}  // namespace agg

using namespace agg;
using namespace agg::serve;

struct agg_server_s {
  int device = 0;
  agg_serve_config cfg{};
  char* arena = nullptr;  // hbm_budget_bytes of device memory
  int slots = 0;
  hipStream_t comp[kMaxSlots] = {};
  hipStream_t copy[kMaxSlots][kPipe] = {};  // one chunk in flight on each
  hipEvent_t done[kMaxSlots] = {};
  uint64_t* part = nullptr;       // slots x kSegTarget partial slots
  agg_result* res_host = nullptr;  // slots results, page-locked host memory
};

namespace {

void server_release(agg_server_s* s) {
  if (!s) return;
  for (int i = 0; i < s->slots; ++i) {
    if (s->comp[i]) (void)hipStreamDestroy(s->comp[i]);
    for (int k = 0; k < kPipe; ++k)
      if (s->copy[i][k]) (void)hipStreamDestroy(s->copy[i][k]);
    if (s->done[i]) (void)hipEventDestroy(s->done[i]);
  }
  if (s->part) (void)hipFree(s->part);
  if (s->arena) (void)hipFree(s->arena);
  if (s->res_host) (void)hipHostFree(s->res_host);
  delete s;
}

}  // namespace

agg::serve::HipExecutor::HipExecutor(agg_server_s* s)
    : s_(s), res_host_(s->res_host), run_((size_t)s->slots), t0_(std::chrono::steady_clock::now()) {}

int agg::serve::HipExecutor::fail(int slot, int rc) {
  // let anything already queued for this slot drain before its memory is reused
  for (int k = 0; k < kPipe; ++k) (void)hipStreamSynchronize(s_->copy[slot][k]);
  (void)hipStreamSynchronize(s_->comp[slot]);
  (void)hipGetLastError();
  return rc;
}

int agg::serve::HipExecutor::copy_chunk(int slot, int64_t k) {
  SlotRun& r = run_[slot];
  const int64_t lo = k * r.cs, hi = std::min(r.nseg, lo + r.cs);
  const int64_t b0 = lo * r.seg_bytes;
  const int64_t nb = std::min(r.bytes, hi * r.seg_bytes) - b0;
  if (fault_hit(AGG_FAULT_SHIP)) {  // an injected copy failure: the copy is never issued
    record_hip_error((int32_t)hipErrorUnknown);
    return AGG_E_HIP;
  }
  // chunk k + kPipe is issued on this stream only after chunk k was seen complete
  const hipError_t e =
      hipMemcpyAsync(r.dst + b0, r.host + b0, (size_t)nb, hipMemcpyHostToDevice, s_->copy[slot][k % kPipe]);
  if (e != hipSuccess) {
    record_hip_error((int32_t)e);
    return AGG_E_HIP;
  }
  return AGG_OK;
}

int agg::serve::HipExecutor::scan_chunk(int slot, int64_t k) {
  SlotRun& r = run_[slot];
  r.a.seg_lo = k * r.cs;
  r.a.seg_hi = std::min(r.nseg, r.a.seg_lo + r.cs);
  return launch(r.scan_fn, grid_for(r.t, device_cu(s_->device), r.a.seg_hi - r.a.seg_lo),
                64 * r.t.waves_per_block, &r.a, s_->comp[slot]);
}

int agg::serve::HipExecutor::finish_launches(int slot) {
  SlotRun& r = run_[slot];
  const int rc = launch(r.comb_fn, 1, kCombineThreads, &r.c, s_->comp[slot]);
  if (rc != AGG_OK) return rc;
  const hipError_t e = hipEventRecord(s_->done[slot], s_->comp[slot]);
  if (e != hipSuccess) {
    record_hip_error((int32_t)e);
    return AGG_E_HIP;
  }
  r.combined = true;
  return AGG_OK;
}

int agg::serve::HipExecutor::start(int slot, const agg_request& req, const Job& j) {
  SlotRun& r = run_[slot];
  r = SlotRun();
  agg_shape sh;
  shape_of(req.dtype, req.n, &sh);
  tune_for(j.kind, AGG_SRC_DEVICE, j.bytes, &r.t);
  const char* col = j.from_arena ? s_->arena + j.off : static_cast<const char*>(req.ptr);
  const bool aligned = (reinterpret_cast<uintptr_t>(col) & 15) == 0;
  uint64_t* part = s_->part + (size_t)slot * kSegTarget;
  r.a.col_bytes = j.bytes;
  r.a.seg_bytes = sh.seg_bytes;
  r.a.part = part;
  r.a.base = col;
  r.a.base_seg = 0;
  r.c.part = part;
  r.c.nseg = sh.nseg;
  r.c.out = res_host_ + slot;
  r.c.n = req.n;
  r.c.is_avg = req.op == AGG_AVG;
  r.c.prec_used = (req.dtype == AGG_F32 && (req.op == AGG_SUM || req.op == AGG_AVG)) ? req.prec : -1;
  r.scan_fn = scan_kernel_ptr(j.kind, r.t.unroll, r.t.nontemporal != 0, aligned);
  r.comb_fn = combine_kernel_ptr(j.kind);
  if (!r.scan_fn || !r.comb_fn) return AGG_E_INVALID;
  r.nseg = sh.nseg;
  r.seg_bytes = sh.seg_bytes;
  r.bytes = j.bytes;
  if (sh.nseg > 0 && j.ship) {
    r.ship = true;
    r.cs = std::max<int64_t>(1, s_->cfg.chunk_bytes / sh.seg_bytes);
    r.nchunks = ceil_div(sh.nseg, r.cs);
    r.host = static_cast<const char*>(req.ptr);
    r.dst = s_->arena + j.off;
    for (; r.next_copy < std::min<int64_t>(kPipe, r.nchunks); ++r.next_copy) {
      const int rc = copy_chunk(slot, r.next_copy);
      if (rc != AGG_OK) return fail(slot, rc);
    }
    return AGG_OK;
  }
  if (sh.nseg > 0) {
    r.cs = sh.nseg;
    const int rc = scan_chunk(slot, 0);
    if (rc != AGG_OK) return fail(slot, rc);
  }
  const int rc = finish_launches(slot);
  return rc == AGG_OK ? rc : fail(slot, rc);
}

int agg::serve::HipExecutor::poll(int slot) {
  SlotRun& r = run_[slot];
  if (r.ship && !r.combined) {
    while (r.next_scan < r.next_copy) {
      const hipError_t e = hipStreamQuery(s_->copy[slot][r.next_scan % kPipe]);
      if (e == hipErrorNotReady) break;
      if (e != hipSuccess) {
        record_hip_error((int32_t)e);
        return fail(slot, AGG_E_HIP);
      }
      int rc = scan_chunk(slot, r.next_scan++);
      if (rc == AGG_OK && r.next_copy < r.nchunks) rc = copy_chunk(slot, r.next_copy++);
      if (rc != AGG_OK) return fail(slot, rc);
    }
    if (r.next_scan < r.nchunks) return 0;
    const int rc = finish_launches(slot);
    if (rc != AGG_OK) return fail(slot, rc);
  }
  const hipError_t e = hipEventQuery(s_->done[slot]);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  record_hip_error((int32_t)e);
  return fail(slot, AGG_E_HIP);
}

extern "C" {

int agg_serve_create(agg_server_t* out, const agg_serve_config* cfg) {
  if (!out) return AGG_E_INVALID;
  *out = nullptr;
  const int vr = validate(cfg, nullptr, 0, false, 0);
  if (vr != AGG_OK) return vr;
  int dev = 0;
  const int dr = current_device(&dev);
  if (dr != AGG_OK) return dr;
  agg_server_s* s = new (std::nothrow) agg_server_s();
  if (!s) return AGG_E_NOMEM;
  s->device = dev;
  s->cfg = *cfg;
  auto fail = [&](int rc) {
    server_release(s);
    return rc;
  };
  hipError_t e;
  int arc = AGG_OK;
  if (cfg->hbm_budget_bytes > 0) arc = device_alloc(reinterpret_cast<void**>(&s->arena), (size_t)cfg->hbm_budget_bytes);
  if (arc == AGG_OK) arc = device_alloc(reinterpret_cast<void**>(&s->part), (size_t)cfg->max_slots * kSegTarget * 8);
  if (arc == AGG_OK) arc = pinned_alloc(reinterpret_cast<void**>(&s->res_host), sizeof(agg_result) * cfg->max_slots);
  if (arc != AGG_OK) return fail(arc);
  for (int i = 0; i < cfg->max_slots; ++i) {
    s->slots = i + 1;
    e = hipStreamCreateWithFlags(&s->comp[i], hipStreamNonBlocking);
    for (int k = 0; k < kPipe && e == hipSuccess; ++k) e = hipStreamCreateWithFlags(&s->copy[i][k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->done[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      record_hip_error((int32_t)e);
      return fail(AGG_E_HIP);
    }
  }
  if ((e = hipDeviceSynchronize()) != hipSuccess) {
    record_hip_error((int32_t)e);
    return fail(AGG_E_HIP);
  }
  *out = s;
  return AGG_OK;
}

int agg_serve_run(agg_server_t s, const agg_request* reqs, int32_t n, agg_result* results,
                  agg_request_stats* stats, agg_serve_summary* summary) {
  if (!s || (n > 0 && (!results || !stats)) || !summary) return AGG_E_INVALID;
  const int vr = validate(&s->cfg, reqs, n, true, s->device);
  if (vr != AGG_OK) return vr;
  HipExecutor ex(s);
  Scheduler sched(s->cfg, ex);
  sched.cur_ids_.resize((size_t)n);
  for (int32_t i = 0; i < n; ++i) sched.cur_ids_[(size_t)i] = reqs[i].column_id;
  const int rc = sched.run(reqs, n, results, stats, summary);
  for (int i = 0; i < s->slots; ++i) (void)hipStreamSynchronize(s->comp[i]);
  return rc;
}

int agg_serve_destroy(agg_server_t s) {
  if (!s) return AGG_E_INVALID;
  (void)hipDeviceSynchronize();
  server_release(s);
  return AGG_OK;
}

int agg_serve_simulate(const agg_serve_config* cfg, const agg_request* reqs, int32_t n, double pcie_gbs,
                       double hbm_gbs, double launch_s, agg_request_stats* stats, agg_serve_summary* summary) {
  if (!summary || (n > 0 && !stats) || !(pcie_gbs > 0) || !(hbm_gbs > 0) || !(launch_s >= 0))
    return AGG_E_INVALID;
  const int vr = validate(cfg, reqs, n, false, 0);
  if (vr != AGG_OK) return vr;
  std::vector<agg_result> results((size_t)std::max(n, 1));
  SimExecutor ex(cfg->max_slots, pcie_gbs, hbm_gbs, launch_s);
  Scheduler sched(*cfg, ex);
  sched.cur_ids_.resize((size_t)n);
  for (int32_t i = 0; i < n; ++i) sched.cur_ids_[(size_t)i] = reqs[i].column_id;
  return sched.run(reqs, n, results.data(), stats, summary);
}

}  // extern "C"

// Autotuner and tuning cache.
//
// Launch parameters (waves per block, blocks per CU, loads in flight per
// lane, non-temporal loads, staging chunk and depth) never change a result
// bit, so they are free for the tuner.  agg_autotune times a fixed set of
// candidates on the caller's column with HIP events and keeps the fastest in
// an in-memory cache keyed by (fold kind, source, size bucket); plans created
// without explicit parameters look the cache up (agg_default_tune).  The
// cache persists as a small JSON file keyed by gfx arch and CU count; a file
// for another device, or one that does not parse, is ignored.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "agg.h"
#include "agg_internal.hpp"

namespace agg {
namespace {

struct Key {
  int kind, src, bucket;
  bool operator<(const Key& o) const {
    return std::tie(kind, src, bucket) < std::tie(o.kind, o.src, o.bucket);
  }
};
struct Entry {
  agg_tune tune;
  double gbs;
};

std::mutex g_tmu;
std::map<Key, Entry> g_cache;

int bucket_of(int64_t bytes) {  // ceil(log2(bytes)), at least 10
  int b = 10;
  while (b < 62 && ((int64_t)1 << b) < bytes) ++b;
  return b;
}

// Measured bests on MI355X for 2^30-item columns (device source): two waves
// per CU with 16 outstanding 16-byte loads per lane for most kinds; the
// compensated float sum has about 4x the VALU work per item and wants more
// waves to hide it.
void builtin_for(int kind, agg_tune* t) {
  t->nontemporal = 1;
  t->chunk_bytes = 64ll << 20;
  t->staging_depth = 3;
  t->reserved = 0;
  switch (kind) {
    case K_SUM_I64: case K_MIN_I64: case K_MAX_I64:
      t->waves_per_block = 1; t->blocks_per_cu = 2; t->unroll = 16; break;
    case K_SUM_F32_NEU:
      t->waves_per_block = 4; t->blocks_per_cu = 1; t->unroll = 8; break;
    case K_MIN_I32: case K_MAX_I32: case K_MIN_F32: case K_MAX_F32:
      t->waves_per_block = 2; t->blocks_per_cu = 1; t->unroll = 32; break;
    case K_COUNT_4: case K_COUNT_8:
      t->waves_per_block = 4; t->blocks_per_cu = 1; t->unroll = 8; break;
    default:  // K_SUM_I32, K_SUM_F32_PLAIN, K_SUM_F32_F64C
      t->waves_per_block = 2; t->blocks_per_cu = 1; t->unroll = 16; break;
  }
}

std::string device_key() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return "";
  }
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "";
  }
  char buf[128];
  std::snprintf(buf, sizeof buf, "%s/%d", p.gcnArchName, p.multiProcessorCount);
  return buf;
}

// Time `runs` launches of fn() on `stream` with events; returns ms per run or -1.
template <class F>
double time_runs(F fn, hipStream_t stream, int warm, int runs) {
  for (int i = 0; i < warm; ++i)
    if (fn() != AGG_OK) return -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    return -1.0;
  }
  double ms = -1.0;
  bool ok = hipEventRecord(e0, stream) == hipSuccess;
  for (int i = 0; ok && i < runs; ++i) ok = fn() == AGG_OK;
  ok = ok && hipEventRecord(e1, stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
  float f = 0.0f;
  if (ok && hipEventElapsedTime(&f, e0, e1) == hipSuccess) ms = f / runs;
  (void)hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

std::vector<agg_tune> kernel_candidates(int kind) {
  std::vector<agg_tune> v;
  agg_tune base;
  builtin_for(kind, &base);
  const int wb[][2] = {{1, 2}, {2, 1}, {4, 1}, {1, 3}, {2, 2}, {4, 2}, {8, 1}, {1, 4}};
  for (int u : {8, 16, 32})
    for (auto& p : wb) {
      agg_tune t = base;
      t.unroll = u;
      t.waves_per_block = p[0];
      t.blocks_per_cu = p[1];
      v.push_back(t);
    }
  return v;
}

}  // namespace

bool tune_cache_lookup(int kind, int32_t src, int64_t bytes, agg_tune* out) {
  std::lock_guard<std::mutex> lk(g_tmu);
  const int b = bucket_of(bytes);
  const Entry* best = nullptr;
  int best_d = 1 << 30;
  for (auto& kv : g_cache) {
    if (kv.first.kind != kind || kv.first.src != src) continue;
    const int d = std::abs(kv.first.bucket - b);
    if (d < best_d) {
      best_d = d;
      best = &kv.second;
    }
  }
  if (!best) return false;
  *out = best->tune;
  return true;
}

void builtin_tune_for(int kind, agg_tune* out) { builtin_for(kind, out); }

}  // namespace agg

using namespace agg;

extern "C" {

int agg_autotune(int32_t dtype, int32_t op, int32_t prec, const void* col, int64_t n, int32_t src,
                 void* stream_v, agg_tune* best, double* best_gbs) {
  const int kind = kind_of(dtype, op, prec);
  if (kind < 0 || n <= 0 || !col || src < AGG_SRC_DEVICE || src > AGG_SRC_ZEROCOPY) return AGG_E_INVALID;
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  std::vector<agg_tune> cands;
  if (src == AGG_SRC_PINNED_HOST) {
    agg_tune base;
    builtin_for(kind, &base);
    for (int64_t mb : {16, 32, 64, 128})
      for (int depth : {2, 3, 4}) {
        agg_tune t = base;
        t.chunk_bytes = mb << 20;
        t.staging_depth = depth;
        cands.push_back(t);
      }
  } else {
    cands = kernel_candidates(kind);
  }
  void* out = nullptr;
  const int arc = device_alloc(&out, sizeof(agg_result));
  if (arc != AGG_OK) return arc;
  const int64_t bytes = n * width_of(dtype);
  double best_ms = -1.0;
  agg_tune best_t{};
  int rc = AGG_OK;
  for (const agg_tune& t : cands) {
    agg_plan_t p = nullptr;
    rc = agg_plan(&p, dtype, op, prec, n, src, &t);
    if (rc != AGG_OK) break;
    const int runs = src == AGG_SRC_DEVICE ? 3 : 1;
    const double ms = time_runs([&] { return agg_run(p, col, n, static_cast<agg_result*>(out), stream); },
                                stream, 1, runs);
    agg_plan_destroy(p);
    if (ms < 0) {
      rc = AGG_E_HIP;
      break;
    }
    if (best_ms < 0 || ms < best_ms) {
      best_ms = ms;
      best_t = t;
    }
  }
  // the best candidate again with temporal loads
  if (rc == AGG_OK && best_ms > 0 && src == AGG_SRC_DEVICE) {
    agg_tune t = best_t;
    t.nontemporal = 0;
    agg_plan_t p = nullptr;
    if (agg_plan(&p, dtype, op, prec, n, src, &t) == AGG_OK) {
      const double ms = time_runs([&] { return agg_run(p, col, n, static_cast<agg_result*>(out), stream); },
                                  stream, 1, 3);
      agg_plan_destroy(p);
      if (ms > 0 && ms < best_ms) {
        best_ms = ms;
        best_t = t;
      }
    }
  }
  (void)hipFree(out);
  if (rc != AGG_OK) return rc;
  const double gbs = (double)bytes / (best_ms * 1e-3) / 1e9;
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_cache[Key{kind, src, bucket_of(bytes)}] = Entry{best_t, gbs};
  }
  if (best) *best = best_t;
  if (best_gbs) *best_gbs = gbs;
  return AGG_OK;
}

int agg_tune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_cache.clear();
  return AGG_OK;
}

int agg_tune_save(const char* path) {
  if (!path) return AGG_E_INVALID;
  const std::string dev = device_key();
  if (dev.empty()) return AGG_E_NODEVICE;
  FILE* f = std::fopen(path, "w");
  if (!f) return AGG_E_INVALID;
  std::lock_guard<std::mutex> lk(g_tmu);
  std::fprintf(f, "{\"version\": 1, \"device\": \"%s\", \"entries\": [\n", dev.c_str());
  size_t i = 0;
  for (auto& kv : g_cache) {
    const agg_tune& t = kv.second.tune;
    std::fprintf(f,
                 "  {\"kind\": %d, \"src\": %d, \"bucket\": %d, \"waves_per_block\": %d, \"blocks_per_cu\": %d, "
                 "\"unroll\": %d, \"nontemporal\": %d, \"chunk_bytes\": %lld, \"staging_depth\": %d, "
                 "\"gbs\": %.1f}%s\n",
                 kv.first.kind, kv.first.src, kv.first.bucket, t.waves_per_block, t.blocks_per_cu, t.unroll,
                 t.nontemporal, (long long)t.chunk_bytes, t.staging_depth, kv.second.gbs,
                 ++i < g_cache.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  const bool ok = std::fclose(f) == 0;
  return ok ? AGG_OK : AGG_E_INVALID;
}

namespace {
// Reads `"name": <integer or number>` inside [s, e); false if absent.
bool json_num(const char* s, const char* e, const char* name, double* v) {
  const std::string pat = std::string("\"") + name + "\":";
  const char* p = std::search(s, e, pat.begin(), pat.end());
  if (p == e) return false;
  p += pat.size();
  while (p < e && (*p == ' ' || *p == '\t')) ++p;
  char* end = nullptr;
  *v = std::strtod(p, &end);
  return end && end != p && end <= e;
}
}  // namespace

int agg_tune_load(const char* path) {
  if (!path) return AGG_E_INVALID;
  FILE* f = std::fopen(path, "rb");
  if (!f) return AGG_E_INVALID;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
  std::fclose(f);
  // the format first (no device needed), then whether it was written for this device
  if (text.find("\"version\": 1") == std::string::npos) return AGG_E_INVALID;
  std::map<Key, Entry> loaded;
  size_t pos = text.find("\"entries\"");
  if (pos == std::string::npos) return AGG_E_INVALID;
  while ((pos = text.find('{', pos + 1)) != std::string::npos) {
    const size_t end = text.find('}', pos);
    if (end == std::string::npos) return AGG_E_INVALID;
    const char* s = text.data() + pos;
    const char* e = text.data() + end;
    double kind, src, bucket, w, b, u, nt, chunk, depth, gbs;
    if (!json_num(s, e, "kind", &kind) || !json_num(s, e, "src", &src) || !json_num(s, e, "bucket", &bucket) ||
        !json_num(s, e, "waves_per_block", &w) || !json_num(s, e, "blocks_per_cu", &b) ||
        !json_num(s, e, "unroll", &u) || !json_num(s, e, "nontemporal", &nt) ||
        !json_num(s, e, "chunk_bytes", &chunk) || !json_num(s, e, "staging_depth", &depth) ||
        !json_num(s, e, "gbs", &gbs))
      return AGG_E_INVALID;
    // every field an integer in its range before it is converted (NaN fails every comparison)
    auto whole = [](double v, double lo, double hi) { return v >= lo && v <= hi && v == std::floor(v); };
    if (!whole(kind, 0, K_NUM - 1) || !whole(src, AGG_SRC_DEVICE, AGG_SRC_ZEROCOPY) || !whole(bucket, 0, 64) ||
        !whole(w, 1, 16) || !whole(b, 1, 32) || !whole(u, 4, 32) || !whole(nt, 0, 1) ||
        !whole(chunk, 1 << 20, (double)((int64_t)1 << 32)) || !whole(depth, 2, 4) || !(gbs >= 0.0 && gbs < 1e9))
      return AGG_E_INVALID;
    agg_tune t;
    t.waves_per_block = (int32_t)w;
    t.blocks_per_cu = (int32_t)b;
    t.unroll = (int32_t)u;
    t.nontemporal = (int32_t)nt;
    t.chunk_bytes = (int64_t)chunk;
    t.staging_depth = (int32_t)depth;
    t.reserved = 0;
    if (!tune_is_valid(t)) return AGG_E_INVALID;
    loaded[Key{(int)kind, (int)src, (int)bucket}] = Entry{t, gbs};
    pos = end;
  }
  const std::string dev = device_key();
  if (dev.empty()) return AGG_E_NODEVICE;
  const std::string want = "\"device\": \"" + dev + "\"";
  if (text.find(want) == std::string::npos) return AGG_E_INVALID;  // another device: ignore
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto& kv : loaded) g_cache[kv.first] = kv.second;
  return AGG_OK;
}

}  // extern "C"

// Host-only code under AddressSanitizer and UndefinedBehaviorSanitizer: the
// oracle, the input generator, the int32 packer, the serving scheduler on
// its simulated clock, the tuning-cache parser and the argument checks of
// the C ABI.  No device is touched (with no GPU, calls that need one return
// AGG_E_NODEVICE).  Buffers are allocated to their exact size so that any
// overrun lands outside them.  Exit status 0 = every check held and no
// sanitizer report (the sanitizers abort the process on their first report).
#include <cinttypes>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "agg.h"

extern "C" {
struct oracle_result {
  int64_t i64;
  double f64;
  int64_t count;
  int32_t is_null;
  int32_t reserved;
};
struct oracle_group {
  int64_t key, i64;
  double f64;
  int64_t count;
};
int oracle_aggregate(const void* col, int64_t n, int dtype, int op, int nthreads, oracle_result* out);
int64_t oracle_groupby(const void* keys, int key_dtype, const void* vals, int val_dtype, int64_t n, int op,
                       oracle_group* out, int64_t max_groups);
int oracle_block_aggregate(const void* col, int64_t n, int dtype, int op, int64_t block, int64_t* out,
                           int nthreads);
int oracle_read_ceiling(const void* buf, int64_t bytes, int nthreads, uint64_t* xor_out);
int dg_fill(void* out, int64_t n, int dtype, int dist, uint64_t seed, int64_t lo, int64_t hi, int nthreads);
}

static int failures = 0;
#define CHECK(c)                                                              \
  do {                                                                        \
    if (!(c)) {                                                               \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);    \
      ++failures;                                                             \
    }                                                                         \
  } while (0)

static const int kWidth[3] = {4, 8, 4};

static void check_generator_and_oracle() {
  const int64_t sizes[] = {0, 1, 7, 1000, 65537, 300001};
  for (int dt = 0; dt < 3; ++dt)
    for (int dist = 0; dist < 4; ++dist) {
      if (dist == 3 && dt != 2) continue;  // N(0,1) + outliers: float32 only
      for (int64_t n : sizes)
        for (int th : {1, 3, 8}) {
          void* x = std::malloc((size_t)(n ? n * kWidth[dt] : 1));
          CHECK(dg_fill(x, n, dt, dist, 7 + (uint64_t)n, 0, 0, th) == 0);
          for (int op = 0; op <= (dt == 2 ? 5 : 4); ++op) {
            oracle_result r;
            CHECK(oracle_aggregate(x, n, dt, op, th, &r) == 0);
            CHECK(r.count == n);
          }
          if (dt != 2) {
            for (int64_t block : {1, 7, 4096, 1 << 20}) {
              const int64_t nb = (n + block - 1) / block;
              std::vector<int64_t> t((size_t)(nb ? nb : 1));
              for (int op : {0, 1, 2}) CHECK(oracle_block_aggregate(x, n, dt, op, block, t.data(), th) == 0);
            }
          }
          uint64_t xr = 0;
          CHECK(oracle_read_ceiling(x, n * kWidth[dt], th, &xr) == 0);
          std::free(x);
        }
    }
  // custom integer ranges and invalid arguments
  std::vector<int32_t> k(100003);
  CHECK(dg_fill(k.data(), (int64_t)k.size(), 0, 0, 5, 1, 1001, 4) == 0);
  CHECK(dg_fill(k.data(), (int64_t)k.size(), 0, 2, 5, -50, 50, 4) == 0);
  CHECK(dg_fill(k.data(), -1, 0, 0, 5, 0, 0, 4) != 0);
  CHECK(dg_fill(k.data(), 10, 2, 0, 5, 1, 5, 4) != 0);   // a range for float32
  oracle_result r;
  CHECK(oracle_aggregate(k.data(), -1, 0, 0, 1, &r) != 0);
  CHECK(oracle_aggregate(k.data(), 10, 0, 5, 1, &r) != 0);  // ABS_SUM of ints
  // group-by over small key sets, every value dtype and op
  for (int kd : {0, 1})
    for (int vd = 0; vd < 3; ++vd)
      for (int op = 0; op <= 4; ++op)
        for (int64_t n : {0, 1, 5000}) {
          std::vector<int64_t> keys64((size_t)(n ? n : 1));
          std::vector<int32_t> keys32((size_t)(n ? n : 1));
          for (int64_t i = 0; i < n; ++i) keys64[(size_t)i] = keys32[(size_t)i] = (int32_t)((i * 2654435761u) % 97) - 40;
          void* vals = std::malloc((size_t)(n ? n * kWidth[vd] : 1));
          CHECK(dg_fill(vals, n, vd, 0, 11, 0, 0, 2) == 0);
          const void* keys = kd ? (const void*)keys64.data() : (const void*)keys32.data();
          const int64_t ng = oracle_groupby(keys, kd, vals, vd, n, op, nullptr, 0);
          CHECK(ng >= 0 && ng <= 97);
          std::vector<oracle_group> g((size_t)(ng > 0 ? ng : 1));
          CHECK(oracle_groupby(keys, kd, vals, vd, n, op, g.data(), ng) == ng);
          if (ng > 2) CHECK(oracle_groupby(keys, kd, vals, vd, n, op, g.data(), 2) == ng);  // capped output
          std::free(vals);
        }
}

static void check_packer() {
  for (int64_t n : {(int64_t)0, (int64_t)1, (int64_t)31, (int64_t)2047, (int64_t)2048, (int64_t)2049,
                    (int64_t)100003}) {
    std::vector<int32_t> x((size_t)(n ? n : 1));
    if (n) CHECK(dg_fill(x.data(), n, 0, 0, 3 + (uint64_t)n, -1000000, 1000000, 2) == 0);
    if (n > 5) x[5] = INT32_MIN, x[(size_t)n - 1] = INT32_MAX;  // a 32-bit-wide block
    int64_t bound = -1;
    CHECK(agg_pack_bound(n, &bound) == AGG_OK && bound >= 0);
    const int64_t nb = (n + AGG_PACK_BLOCK - 1) / AGG_PACK_BLOCK;
    for (int th : {1, 4}) {
      agg_packed_block* blocks = (agg_packed_block*)std::malloc((size_t)(nb ? nb : 1) * sizeof(agg_packed_block));
      uint32_t* payload = (uint32_t*)std::malloc((size_t)(bound ? bound : 1) * 4);
      int64_t used = -1;
      CHECK(agg_pack_i32(x.data(), n, blocks, payload, bound, &used, th) == AGG_OK);
      CHECK(used >= 0 && used <= bound);
      // decode on the host from the documented layout and compare
      for (int64_t b = 0; b < nb; ++b) {
        const agg_packed_block& h = blocks[b];
        CHECK(h.bits <= 32 && h.word_off >= 0 && h.word_off + 64 * (int64_t)h.bits <= used);
        for (int lane = 0; lane < 64; ++lane)
          for (int i = 0; i < 32; ++i) {
            const int64_t idx = b * AGG_PACK_BLOCK + lane * 32 + i;
            if (idx >= n) continue;
            uint64_t d = 0;
            for (uint32_t bit = 0; bit < h.bits; ++bit) {
              const uint64_t pos = (uint64_t)i * h.bits + bit;
              const uint32_t w = payload[h.word_off + (int64_t)(pos / 32) * 64 + lane];
              d |= (uint64_t)((w >> (pos % 32)) & 1u) << bit;
            }
            CHECK((int32_t)((uint32_t)h.base + (uint32_t)d) == x[(size_t)idx]);
          }
      }
      if (used > 0) CHECK(agg_pack_i32(x.data(), n, blocks, payload, 0, &used, th) != AGG_OK);  // no room
      std::free(blocks);
      std::free(payload);
    }
  }
}

static uint64_t lcg(uint64_t& s) {
  s = s * 6364136223846793005ull + 1442695040888963407ull;
  return s >> 11;
}

static void check_scheduler() {
  uint64_t seed = 12345;
  for (int trial = 0; trial < 40; ++trial) {
    const int n = 1 + (int)(lcg(seed) % 400);
    std::vector<agg_request> reqs((size_t)n);
    double t = 0.0;
    for (int i = 0; i < n; ++i) {
      agg_request& q = reqs[(size_t)i];
      t += (double)(lcg(seed) % 1000) * 1e-5;
      q.ptr = reinterpret_cast<const void*>((uintptr_t)(1 << 20) + 4 * (lcg(seed) % 1000));
      q.n = (int64_t)(lcg(seed) % (1ull << (10 + trial % 20)));
      q.column_id = (int64_t)(lcg(seed) % 8);
      q.arrival_s = t;
      q.dtype = (int32_t)(lcg(seed) % 3);
      q.op = (int32_t)(lcg(seed) % 5);
      q.prec = (int32_t)(lcg(seed) % 3);
      q.resident = (int32_t)(lcg(seed) % 3 == 0);
      if (q.dtype == AGG_I64) q.ptr = reinterpret_cast<const void*>((uintptr_t)(1 << 20) + 8 * (lcg(seed) % 1000));
    }
    agg_serve_config cfg{};
    cfg.hbm_budget_bytes = (int64_t)(lcg(seed) % (1ull << (12 + trial % 24)));
    cfg.max_slots = 1 + (int32_t)(lcg(seed) % 8);
    cfg.cache_shipped = (int32_t)(trial % 2);
    cfg.chunk_bytes = (int64_t)1 << (20 + trial % 6);
    cfg.max_shipping = 1 + (int32_t)(lcg(seed) % (uint64_t)cfg.max_slots);
    cfg.progress_every = 0;
    if (trial % 5 == 0) agg_fault_inject(AGG_FAULT_SHIP, 1 + trial % 3);
    std::vector<agg_request_stats> st((size_t)n);
    agg_serve_summary sm;
    CHECK(agg_serve_simulate(&cfg, reqs.data(), n, 50.0, 5000.0, 1e-5, st.data(), &sm) == AGG_OK);
    CHECK(sm.completed + sm.failed == n);
    CHECK(sm.peak_reserved_bytes <= cfg.hbm_budget_bytes);
    agg_fault_inject(AGG_FAULT_SHIP, 0);
  }
  agg_serve_config bad{};
  bad.max_slots = 0;
  agg_request_stats st[1];
  agg_serve_summary sm;
  CHECK(agg_serve_simulate(&bad, nullptr, 0, 50.0, 5000.0, 1e-5, st, &sm) == AGG_E_INVALID);
  CHECK(agg_serve_simulate(nullptr, nullptr, 0, 50.0, 5000.0, 1e-5, st, &sm) == AGG_E_INVALID);
}

static void check_tune_files(const char* dir) {
  const char* bodies[] = {
      "",
      "garbage",
      "{\"version\": 1",
      "{\"version\": 1, \"device\": \"gfx950:256\", \"entries\": [{",
      "{\"version\": 1, \"device\": \"gfx950:256\", \"entries\": [{\"kind\": 1e300, \"src\": 0, \"bucket\": 30, "
      "\"waves_per_block\": 2, \"blocks_per_cu\": 1, \"unroll\": 16, \"nontemporal\": 1, \"chunk_bytes\": 67108864, "
      "\"staging_depth\": 3, \"gbs\": 7000.0}]}",
      "{\"version\": 1, \"device\": \"gfx950:256\", \"entries\": [{\"kind\": 0, \"src\": 0, \"bucket\": 30, "
      "\"waves_per_block\": nan, \"blocks_per_cu\": -1e308, \"unroll\": 16, \"nontemporal\": 1, "
      "\"chunk_bytes\": 1e30, \"staging_depth\": 3, \"gbs\": 7000.0}]}",
      "{\"version\": 1, \"device\": \"gfx950:256\", \"entries\": [{\"kind\": 0, \"src\": 0, \"bucket\": 30, "
      "\"waves_per_block\": 2, \"blocks_per_cu\": 1, \"unroll\": 16, \"nontemporal\": 1, \"chunk_bytes\": 67108864, "
      "\"staging_depth\": 3, \"gbs\": 7000.0}]}",
      "{\"version\": 1, \"entries\": [{\"kind\":",
      "{{{{{{{{}}}}}}}}\"version\": 1 \"entries\" {\"kind\": 2.5}",
  };
  int i = 0;
  for (const char* body : bodies) {
    const std::string path = std::string(dir) + "/tune_" + std::to_string(i++) + ".json";
    FILE* f = std::fopen(path.c_str(), "w");
    if (!f) { ++failures; continue; }
    std::fputs(body, f);
    std::fclose(f);
    const int rc = agg_tune_load(path.c_str());
    CHECK(rc == AGG_E_INVALID || rc == AGG_E_NODEVICE || rc == AGG_OK);
  }
  CHECK(agg_tune_load(nullptr) == AGG_E_INVALID);
  CHECK(agg_tune_load("/nonexistent/dir/x.json") == AGG_E_INVALID);
}

static void check_abi_arguments() {
  agg_shape s;
  CHECK(agg_canonical_shape(AGG_I32, 0, &s) == AGG_OK && s.nseg == 0);
  CHECK(agg_canonical_shape(AGG_I64, (int64_t)1 << 40, &s) == AGG_OK && s.nseg <= 8192);
  CHECK(agg_canonical_shape(AGG_I32, ((int64_t)1 << 40) + 1, &s) == AGG_E_INVALID);
  CHECK(agg_canonical_shape(AGG_I32, -1, &s) == AGG_E_INVALID);
  CHECK(agg_canonical_shape(7, 10, &s) == AGG_E_INVALID);
  agg_tune t;
  CHECK(agg_default_tune(AGG_F32, AGG_SUM, AGG_PREC_NEUMAIER, 1 << 30, AGG_SRC_DEVICE, &t) == AGG_OK);
  CHECK(agg_default_tune(AGG_F32, AGG_SUM, 9, 10, AGG_SRC_DEVICE, &t) == AGG_E_INVALID);
  for (int c = -6; c <= 1; ++c) CHECK(agg_strerror(c) != nullptr);
  CHECK(agg_fault_inject(0, 1) == AGG_E_INVALID && agg_fault_inject(AGG_FAULT_SITES, 1) == AGG_E_INVALID);
  int64_t bound;
  CHECK(agg_pack_bound(-1, &bound) == AGG_E_INVALID);
}

int main(int argc, char** argv) {
  const char* dir = argc > 1 ? argv[1] : "/tmp";
  check_generator_and_oracle();
  check_packer();
  check_scheduler();
  check_tune_files(dir);
  check_abi_arguments();
  if (failures) {
    std::fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  std::printf("host checks ok\n");
  return 0;
}

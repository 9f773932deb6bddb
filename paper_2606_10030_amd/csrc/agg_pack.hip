// Host encoder of packed int32 columns (frame of reference + bit packing);
// the layout is documented with agg_packed in agg.h.  Blocks are encoded
// independently, so threads take contiguous runs of blocks in two passes:
// widths first (a prefix sum gives every block's payload offset), then bits.
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "agg.h"

namespace {

constexpr int64_t kBlock = AGG_PACK_BLOCK;
constexpr int kLanes = 64;
constexpr int kPerLane = kBlock / kLanes;  // 32

uint32_t width_of(uint32_t range) {
  uint32_t b = 0;
  while (b < 32 && (range >> b) != 0) ++b;
  return b;
}

void block_header(const int32_t* x, int64_t n, int64_t b, agg_packed_block* h) {
  const int64_t lo = b * kBlock, hi = std::min(n, lo + kBlock);
  int32_t mn = x[lo], mx = x[lo];
  for (int64_t i = lo + 1; i < hi; ++i) {
    mn = std::min(mn, x[i]);
    mx = std::max(mx, x[i]);
  }
  h->base = mn;
  h->bits = width_of((uint32_t)mx - (uint32_t)mn);
}

void block_payload(const int32_t* x, int64_t n, int64_t b, const agg_packed_block& h, uint32_t* out) {
  const int64_t lo = b * kBlock;
  const uint32_t bits = h.bits;
  if (bits == 0) return;
  for (int lane = 0; lane < kLanes; ++lane) {
    uint64_t acc = 0;  // bit buffer
    int have = 0, word = 0;
    for (int i = 0; i < kPerLane; ++i) {
      const int64_t idx = lo + (int64_t)lane * kPerLane + i;
      const uint32_t d = idx < n ? (uint32_t)x[idx] - (uint32_t)h.base : 0u;
      acc |= (uint64_t)d << have;
      have += (int)bits;
      while (have >= 32) {
        out[(int64_t)word * kLanes + lane] = (uint32_t)acc;
        acc >>= 32;
        have -= 32;
        ++word;
      }
    }
  }
}

template <class F>
void parallel_blocks(int64_t nblocks, int threads, F f) {
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(threads, nblocks));
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t)
    th.emplace_back([&, t] { f(nblocks * t / nt, nblocks * (t + 1) / nt); });
  f(0, nblocks / nt);
  for (auto& x : th) x.join();
}

}  // namespace

extern "C" {

int agg_pack_bound(int64_t n, int64_t* max_payload_words) {
  if (n < 0 || !max_payload_words) return AGG_E_INVALID;
  *max_payload_words = (n + kBlock - 1) / kBlock * kLanes * 32;
  return AGG_OK;
}

int agg_pack_i32(const int32_t* x, int64_t n, agg_packed_block* blocks, uint32_t* payload, int64_t payload_cap,
                 int64_t* payload_words, int32_t threads) {
  if (n < 0 || !payload_words || (n > 0 && (!x || !blocks))) return AGG_E_INVALID;
  const int64_t nblocks = (n + kBlock - 1) / kBlock;
  int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
  nt = std::min(nt, 64);
  parallel_blocks(nblocks, nt, [&](int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; ++b) block_header(x, n, b, &blocks[b]);
  });
  int64_t off = 0;
  for (int64_t b = 0; b < nblocks; ++b) {
    blocks[b].word_off = off;
    off += (int64_t)kLanes * blocks[b].bits;
  }
  *payload_words = off;
  if (off > payload_cap || (off > 0 && !payload)) return AGG_E_INVALID;
  parallel_blocks(nblocks, nt, [&](int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; ++b) block_payload(x, n, b, blocks[b], payload + blocks[b].word_off);
  });
  return AGG_OK;
}

}  // extern "C"

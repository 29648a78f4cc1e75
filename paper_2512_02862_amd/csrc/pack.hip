// Bit-packed columns: the scan side of the streamed query.
//
// A column is stored in blocks of 1024 values, each as a frame of reference:
// the block's minimum (base) and every value's offset from it in the fewest
// bits that hold the block's range, packed back to back in 32-bit words
// (value j of a block starts at bit j * bits of the block's words).  The
// encoder runs on the host, where columns are written; the device decodes a
// block per workgroup.  Streaming packed chunks moves fewer bytes over the
// host link, which bounds the streamed query (the data-loading cost that
// Sec. 4 moves from the CPU to the GPU, with a self-made encoding standing in
// for a file format's).
#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "pyst_internal.h"
#include "query.h"
#include "table.h"

namespace pyst {

constexpr int kPackBlock = PYST_PACK_BLOCK;

inline int max_bits(int dtype) { return dtype == PYST_I64 ? 64 : 32; }

// Checks a block table (host memory): offsets start at 0, grow by whole
// 32-word steps of at most max_bits(dtype) bits per value.
bool pack_blocks_ok(const pyst_pack_block *blocks, int64_t nblocks, int dtype) {
  if (blocks[0].word_off != 0) return false;
  for (int64_t b = 0; b < nblocks; ++b) {
    const int64_t d = blocks[b + 1].word_off - blocks[b].word_off;
    if (d < 0 || d % 32 != 0 || d / 32 > max_bits(dtype)) return false;
  }
  return true;
}

// Decodes the blocks [0, nblk) of a packed column into out[0, n): one block per
// workgroup, 4 values per thread.  Word offsets are relative to word_base.  A
// block whose header is malformed or whose words lie outside [0, nwords)
// latches kErrIndex and is left undecoded.
__global__ __launch_bounds__(256) void k_unpack(const pyst_pack_block *blocks, const uint32_t *words, int64_t nwords,
                                                int64_t word_base, int64_t n, int is64, void *out, uint32_t *err) {
  const int64_t blk = blockIdx.x;
  const int64_t lo = blocks[blk].word_off - word_base, hi = blocks[blk + 1].word_off - word_base;
  const int64_t d = hi - lo;
  if (d < 0 || d % 32 != 0 || d / 32 > (is64 ? 64 : 32) || lo < 0 || hi > nwords) {
    if (threadIdx.x == 0) latch(err, kErrIndex);
    return;
  }
  const int bits = static_cast<int>(d / 32);
  const uint64_t base = static_cast<uint64_t>(blocks[blk].base);
  const uint64_t mask = bits == 64 ? ~uint64_t{0} : ((uint64_t{1} << bits) - 1);
  const uint32_t *w = words + lo;
#pragma unroll
  for (int k = 0; k < kPackBlock / 256; ++k) {
    const int j = k * 256 + threadIdx.x;
    const int64_t i = blk * kPackBlock + j;
    if (i >= n) break;
    uint64_t x = 0;
    if (bits > 0) {
      const int64_t pos = int64_t{j} * bits;
      const int64_t q = pos >> 5;
      const int sh = static_cast<int>(pos & 31);
      uint64_t win = w[q];
      if (q + 1 < d) win |= uint64_t{w[q + 1]} << 32;
      x = win >> sh;
      if (sh + bits > 64 && q + 2 < d) x |= uint64_t{w[q + 2]} << (64 - sh);
      x &= mask;
    }
    const uint64_t v = base + x;
    if (is64)
      static_cast<int64_t *>(out)[i] = static_cast<int64_t>(v);
    else
      static_cast<int32_t *>(out)[i] = static_cast<int32_t>(static_cast<uint32_t>(v));
  }
}

pyst_status launch_unpack(pyst_ctx *ctx, const pyst_pack_block *blocks, const uint32_t *words, int64_t nwords,
                          int64_t word_base, int64_t n, int dtype, void *out, hipStream_t stream) {
  if (n == 0) return PYST_OK;
  TimedRegion timed(ctx, "unpack", stream);
  const int64_t nblk = ceil_div(n, kPackBlock);
  k_unpack<<<static_cast<unsigned>(nblk), 256, 0, stream>>>(blocks, words, nwords, word_base, n, dtype == PYST_I64,
                                                              out, ctx_err_word(ctx));
  PYST_LAUNCH_CHECK("k_unpack");
  return PYST_OK;
}

}  // namespace pyst

using namespace pyst;

static bool pack_col_ok(const pyst_col *c) {
  return c && c->n >= 0 && (c->n == 0 || c->data) && (c->dtype == PYST_I32 || c->dtype == PYST_I64);
}

// Bits of block b's frame of reference: the width of its range (0 when constant).
static int block_bits(const pyst_col &c, int64_t b) {
  const int64_t a = b * kPackBlock, e = std::min<int64_t>(c.n, a + kPackBlock);
  int64_t mn = INT64_MAX, mx = INT64_MIN;
  for (int64_t i = a; i < e; ++i) {
    const int64_t v = c.dtype == PYST_I64 ? static_cast<const int64_t *>(c.data)[i] : static_cast<const int32_t *>(c.data)[i];
    mn = std::min(mn, v);
    mx = std::max(mx, v);
  }
  const uint64_t range = static_cast<uint64_t>(mx) - static_cast<uint64_t>(mn);
  return range == 0 ? 0 : 64 - __builtin_clzll(range);
}

// Host threads for nblk blocks: one per 4096 blocks (4M values), at most the
// machine's hardware threads and 64.
static int pack_threads(int64_t nblk) {
  const int64_t hw = std::max(1u, std::thread::hardware_concurrency());
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>({hw, 64, ceil_div(nblk, 4096)})));
}

// Run fn(thread, first block, end block) over contiguous ranges of [0, nblk).
template <typename F>
static void parallel_blocks(int64_t nblk, F fn) {
  const int nt = pack_threads(nblk);
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back([&, t] { fn(t, nblk * t / nt, nblk * (t + 1) / nt); });
  fn(0, 0, nblk / nt);
  for (auto &th : pool) th.join();
}

extern "C" {

int64_t pyst_pack_words(const pyst_col *host_col) {
  if (!pack_col_ok(host_col)) return -1;
  const int64_t nblk = ceil_div(host_col->n, kPackBlock);
  std::vector<int64_t> part(pack_threads(nblk), 0);
  parallel_blocks(nblk, [&](int t, int64_t b0, int64_t b1) {
    int64_t total = 0;
    for (int64_t b = b0; b < b1; ++b) total += 32 * block_bits(*host_col, b);
    part[t] = total;
  });
  int64_t total = 0;
  for (int64_t x : part) total += x;
  return total;
}

// Two passes over the blocks, each split across host threads: every block's
// width (kept in word_off for the moment), a prefix sum that turns widths into
// word offsets, then every block's words.
pyst_status pyst_pack_encode(const pyst_col *host_col, pyst_pack_block *blocks, uint32_t *words) {
  if (!pack_col_ok(host_col)) return set_error(PYST_ERR_ARG, "pyst_pack_encode: bad column");
  if (!blocks || (host_col->n > 0 && !words)) return set_error(PYST_ERR_ARG, "pyst_pack_encode: NULL output");
  const int64_t n = host_col->n, nblk = ceil_div(n, kPackBlock);
  const bool is64 = host_col->dtype == PYST_I64;
  auto at = [&](int64_t i) -> int64_t {
    return is64 ? static_cast<const int64_t *>(host_col->data)[i] : static_cast<const int32_t *>(host_col->data)[i];
  };
  parallel_blocks(nblk, [&](int, int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; ++b) {
      int64_t mn = INT64_MAX;
      for (int64_t i = b * kPackBlock, e = std::min<int64_t>(n, (b + 1) * kPackBlock); i < e; ++i) mn = std::min(mn, at(i));
      blocks[b].base = mn;
      blocks[b].word_off = 32 * block_bits(*host_col, b);
    }
  });
  int64_t off = 0;
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t w = blocks[b].word_off;
    blocks[b].word_off = off;
    off += w;
  }
  blocks[nblk].base = 0;
  blocks[nblk].word_off = off;
  parallel_blocks(nblk, [&](int, int64_t b0, int64_t b1) {
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t a = b * kPackBlock, e = std::min<int64_t>(n, a + kPackBlock);
      const int bits = static_cast<int>((blocks[b + 1].word_off - blocks[b].word_off) / 32);
      const int64_t mn = blocks[b].base;
      uint32_t *w = words + blocks[b].word_off;
      std::memset(w, 0, sizeof(uint32_t) * 32 * bits);
      if (bits == 0) continue;
      for (int64_t i = a; i < e; ++i) {
        const uint64_t x = static_cast<uint64_t>(at(i)) - static_cast<uint64_t>(mn);
        const int64_t pos = (i - a) * bits;
        const int64_t q = pos >> 5;
        const int sh = static_cast<int>(pos & 31);
        w[q] |= static_cast<uint32_t>(x << sh);
        if (sh + bits > 32) w[q + 1] |= static_cast<uint32_t>(x >> (32 - sh));
        if (sh + bits > 64) w[q + 2] |= static_cast<uint32_t>(x >> (64 - sh));
      }
    }
  });
  return PYST_OK;
}

pyst_status pyst_pack_decode(pyst_ctx *ctx, const pyst_pack_block *d_blocks, const uint32_t *d_words, int64_t nwords,
                             int64_t n, int dtype, void *d_out, hipStream_t stream) {
  if (!ctx || n < 0 || nwords < 0 || !(dtype == PYST_I32 || dtype == PYST_I64))
    return set_error(PYST_ERR_ARG, "pyst_pack_decode: bad argument");
  if (n > 0 && (!d_blocks || !d_out || (nwords > 0 && !d_words)))
    return set_error(PYST_ERR_ARG, "pyst_pack_decode: NULL argument");
  if (n >= (int64_t{1} << 31)) return set_error(PYST_ERR_ARG, "pyst_pack_decode: fewer than 2^31 values");
  return launch_unpack(ctx, d_blocks, d_words, nwords, 0, n, dtype, d_out, stream);
}

}  // extern "C"

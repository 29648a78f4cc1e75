// Group-by SUM over materialized (key, value) pairs by hash partitioning and
// LDS aggregation.
//
// A hash table in HBM takes two L2 atomics per pair (claim the key, add the
// value), and random atomics on MI355X retire at about 23e9/s chip-wide, so 12M
// pairs cost a millisecond however the table is laid out.  Here the pairs are
// moved twice, 64 ways each time, by 6 bits of a hash of the key: one counting
// pass gives every first-move block's count per final bucket, two exclusive
// scans turn them into both moves' positions, then the first move splits all
// pairs and the second splits each of the 64 parts, so that pairs end in 4096
// contiguous buckets.  One block per bucket then adds its pairs up in
// an LDS hash table (indexed by low bits of the same hash) and writes out the
// groups.  64 ways keep every block's writes to a bucket in a few active lines
// that the L2 combines; one 4096-way move would write 8-byte fragments.
#include "pyst_internal.h"
#include "table.h"

namespace pyst {

constexpr int kAggBlock = 1024;
constexpr int kRadixLg = 6;
constexpr int kRadix = 1 << kRadixLg;
constexpr int kAggBuckets = kRadix * kRadix;   // 4096 buckets after two moves
constexpr int kAggSlotsLg = 13;
constexpr int kAggSlots = 1 << kAggSlotsLg;    // LDS table: 8192 x 16 bytes = 128 KiB per bucket
constexpr int kAggBlocks1 = 512;               // blocks of the first move
constexpr int kAggBlocks2 = 8;                 // blocks per part in the second move
constexpr uint64_t kAggSeed = 0xd6e8feb86659fd93ull;

__device__ __forceinline__ uint64_t agg_hash(int64_t key) { return fmix64(static_cast<uint64_t>(key) ^ kAggSeed); }

// The rows a block of a move reads: with b = xcd_block(blockIdx.x), segment b / bps of the input
// (segment s is [seg_off[s * seg_stride], seg_off[(s + 1) * seg_stride]), or the
// whole input [0, min(*count, cap)) without seg_off), split evenly into bps parts.
struct MoveArgs {
  const int64_t *keys;
  const int64_t *vals;
  const int64_t *count;
  int64_t cap;
  const int32_t *seg_off;
  int seg_stride;
  int bps;
  int shift;  // bucket = (hash >> shift) & (kRadix - 1)
  // With `aligned`, block part of segment seg reads the rows that the first
  // move's blocks [part * G, (part + 1) * G) wrote to it, G = seg_stride / bps
  // (their counts are known from the first pass), instead of an even split.
  int aligned = 0;
  // With kcol set, the pairs are read from the caller's columns instead: pair i
  // is row row_of(sel, i) of (kcol, vcol), int64 or int32 (sign-extended), and
  // an EMPTY key is latched in err (and skipped like any EMPTY key).
  const void *kcol = nullptr;
  const void *vcol = nullptr;
  const int32_t *sel = nullptr;
  int k64 = 0, v64 = 0;
  uint32_t *err = nullptr;
};

__device__ __forceinline__ int64_t move_key(const MoveArgs &m, int64_t i) {
  return m.kcol ? load_as_i64(m.kcol, m.k64, row_of(m.sel, i)) : m.keys[i];
}

__device__ __forceinline__ int64_t move_val(const MoveArgs &m, int64_t i) {
  return m.kcol ? load_as_i64(m.vcol, m.v64, row_of(m.sel, i)) : m.vals[i];
}

__device__ __forceinline__ void move_range(const MoveArgs &m, int *seg, int *part, int64_t *lo, int64_t *hi) {
  const int blk = static_cast<int>(xcd_block(blockIdx.x, gridDim.x));  // neighbouring ranges on one XCD
  *seg = blk / m.bps;
  *part = blk % m.bps;
  int64_t a, b;
  if (m.seg_off && m.aligned) {
    const int g = m.seg_stride / m.bps;
    *lo = m.seg_off[int64_t{*seg} * m.seg_stride + int64_t{*part} * g];
    *hi = m.seg_off[int64_t{*seg} * m.seg_stride + int64_t{*part + 1} * g];
    return;
  }
  if (m.seg_off) {
    a = m.seg_off[int64_t{*seg} * m.seg_stride];
    b = m.seg_off[int64_t{*seg + 1} * m.seg_stride];
  } else {
    a = 0;
    b = *m.count < m.cap ? *m.count : m.cap;
  }
  const int64_t per = (b - a + m.bps - 1) / m.bps;
  *lo = a + per * *part;
  *hi = *lo + per < b ? *lo + per : b;
  if (*lo > b) *lo = b;
}

// Pairs a thread of the counting pass takes per round, all loads first.
constexpr int kMoveItems = 8;

// Per first-move block: counts of its pairs in each of the 4096 final buckets
// (top 12 bits of the hash: the first move's 6 and the second's 6), from
// which both moves' positions follow (k_narrow_counts), so the second move
// needs no counting pass of its own.
__global__ __launch_bounds__(kAggBlock) void k_move_hist_both(MoveArgs m, int32_t *counts) {
  __shared__ int32_t s_c[kAggBuckets];
  for (int i = threadIdx.x; i < kAggBuckets; i += kAggBlock) s_c[i] = 0;
  __syncthreads();
  int seg, part;
  int64_t lo, hi;
  move_range(m, &seg, &part, &lo, &hi);
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += int64_t{kAggBlock} * kMoveItems) {
    int64_t k[kMoveItems];
#pragma unroll
    for (int u = 0; u < kMoveItems; ++u) {
      const int64_t i = i0 + int64_t{u} * kAggBlock;
      k[u] = i < hi ? move_key(m, i) : kEmpty64;
      if (m.kcol && i < hi && k[u] == kEmpty64) latch(m.err, kErrKey);
    }
#pragma unroll
    for (int u = 0; u < kMoveItems; ++u)
      if (k[u] != kEmpty64) atomicAdd(&s_c[agg_hash(k[u]) >> (64 - 2 * kRadixLg)], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kAggBuckets; i += kAggBlock) counts[(int64_t{seg} * m.bps + part) * kAggBuckets + i] = s_c[i];
}

// Writes each block's pairs to its positions (pos: the exclusive scan of the
// per-(segment, bucket, block) counts, in that order).  A tile of kMoveTile pairs is ranked by bucket in LDS
// (per-bucket counts with LDS atomics, one scan over kRadix buckets), laid out
// bucket-major in LDS, and written so that consecutive threads write
// consecutive slots of each bucket's run: every bucket's pairs of a tile leave
// in one contiguous piece (about 512 bytes) instead of as 8-byte fragments.
constexpr int kMoveTileItems = 4;
static_assert(kRadix == kWave, "one wave scans the bucket counts");
constexpr int kMoveTile = kAggBlock * kMoveTileItems;
__global__ __launch_bounds__(kAggBlock) void k_move_scatter(MoveArgs m, const int32_t *pos, int64_t *okeys,
                                                           int64_t *ovals) {
  __shared__ int64_t s_k[kMoveTile];
  __shared__ int64_t s_v[kMoveTile];
  __shared__ uint8_t s_b[kMoveTile];
  __shared__ int32_t s_base[kRadix], s_cnt[kRadix], s_off[kRadix + 1];
  int seg, part;
  int64_t lo, hi;
  move_range(m, &seg, &part, &lo, &hi);
  const int tid = static_cast<int>(threadIdx.x);
  if (tid < kRadix) s_base[tid] = pos[(int64_t{seg} * kRadix + tid) * m.bps + part];
  for (int64_t t0 = lo; t0 < hi; t0 += kMoveTile) {  // block-uniform
    if (tid < kRadix) s_cnt[tid] = 0;
    __syncthreads();
    int64_t k[kMoveTileItems], v[kMoveTileItems];
    int bk[kMoveTileItems], rk[kMoveTileItems];
#pragma unroll
    for (int u = 0; u < kMoveTileItems; ++u) {
      const int64_t i = t0 + int64_t{u} * kAggBlock + tid;
      k[u] = i < hi ? move_key(m, i) : kEmpty64;
      v[u] = i < hi ? move_val(m, i) : 0;
    }
#pragma unroll
    for (int u = 0; u < kMoveTileItems; ++u) {
      bk[u] = k[u] != kEmpty64 ? static_cast<int>((agg_hash(k[u]) >> m.shift) & (kRadix - 1)) : -1;
      rk[u] = bk[u] >= 0 ? atomicAdd(&s_cnt[bk[u]], 1) : 0;
    }
    __syncthreads();
    if (tid < kWave) {  // one wave: exclusive scan of the kRadix (= 64) counts
      const int c = s_cnt[tid];
      const int incl = wave_inclusive_scan(c);
      s_off[tid] = incl - c;
      if (tid == kWave - 1) s_off[kRadix] = incl;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMoveTileItems; ++u)
      if (bk[u] >= 0) {
        const int p = s_off[bk[u]] + rk[u];
        s_k[p] = k[u];
        s_v[p] = v[u];
        s_b[p] = static_cast<uint8_t>(bk[u]);
      }
    __syncthreads();
    const int n = s_off[kRadix];
    for (int t = tid; t < n; t += kAggBlock) {
      const int b = s_b[t];
      const int64_t o = int64_t{s_base[b]} + (t - s_off[b]);
      okeys[o] = s_k[t];
      ovals[o] = s_v[t];
    }
    __syncthreads();
    if (tid < kRadix) s_base[tid] += s_cnt[tid];
  }
}

// Adds up the pairs of each final bucket in an LDS hash table (indexed by low
// bits of the key hash) and writes out its groups.  One block per CU walks its
// buckets (blockIdx.x, + gridDim.x, ...): the table is cleared as it is written
// out, and the next bucket's first pairs are loaded before the block waits for
// the output position of the current one (one counter atomic per bucket), so a
// bucket costs about one memory round trip.  *d_ngroups must be zero on entry.
__global__ __launch_bounds__(kAggBlock) void k_bucket_groups(const int64_t *keys, const int64_t *vals,
                                                            const int32_t *pos, int bps, int64_t *out_keys,
                                                            int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                                                            uint32_t *err) {
  __shared__ uint64_t s_key[kAggSlots];
  __shared__ uint64_t s_sum[kAggSlots];
  __shared__ int32_t s_w[kAggBlock / kWave];
  __shared__ int64_t s_base;
  constexpr int U = 4;  // pairs per thread per round, loaded before any insert
  constexpr int PER = kAggSlots / kAggBlock;  // each thread counts, writes out and clears PER consecutive slots
  const int tid = static_cast<int>(threadIdx.x);
  for (int s = tid; s < kAggSlots; s += kAggBlock) {
    s_key[s] = static_cast<uint64_t>(kEmpty64);
    s_sum[s] = 0;
  }
  bool full = false;
  int64_t kk[U], vv[U];  // the first round of the bucket about to be added up
  auto load_round = [&](int64_t i0, int64_t hi) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + int64_t{u} * kAggBlock;
      kk[u] = i < hi ? keys[i] : kEmpty64;
      vv[u] = i < hi ? vals[i] : 0;
    }
  };
  auto insert_round = [&]() {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (kk[u] == kEmpty64) continue;
      uint32_t s = static_cast<uint32_t>(agg_hash(kk[u])) & (kAggSlots - 1);
      for (int probes = 0;; ++probes) {
        if (probes == kAggSlots) {
          full = true;
          break;
        }
        const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long *>(&s_key[s]),
                                       static_cast<unsigned long long>(kEmpty64), static_cast<unsigned long long>(kk[u]));
        if (old == static_cast<uint64_t>(kEmpty64) || old == static_cast<uint64_t>(kk[u])) {
          atomicAdd(reinterpret_cast<unsigned long long *>(&s_sum[s]), static_cast<unsigned long long>(vv[u]));
          break;
        }
        s = (s + 1) & (kAggSlots - 1);
      }
    }
  };
  int b = static_cast<int>(blockIdx.x);
  if (b < kAggBuckets) load_round(pos[int64_t{b} * bps] + tid, pos[int64_t{b + 1} * bps]);
  __syncthreads();  // the cleared table
  for (; b < kAggBuckets; b += static_cast<int>(gridDim.x)) {  // block-uniform
    const int64_t lo = pos[int64_t{b} * bps], hi = pos[int64_t{b + 1} * bps];
    insert_round();
    for (int64_t i0 = lo + tid + int64_t{kAggBlock} * U; i0 < hi; i0 += int64_t{kAggBlock} * U) {  // large buckets
      load_round(i0, hi);
      insert_round();
    }
    __syncthreads();
    const int s0 = tid * PER;
    int c = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) c += s_key[s0 + j] != static_cast<uint64_t>(kEmpty64);
    const int incl = wave_inclusive_scan(c);
    const int w = tid / kWave;
    if (lane_id() == kWave - 1) s_w[w] = incl;
    __syncthreads();
    // the next bucket's first round goes out before the wait for this one's position
    const int nb = b + static_cast<int>(gridDim.x);
    if (nb < kAggBuckets) load_round(pos[int64_t{nb} * bps] + tid, pos[int64_t{nb + 1} * bps]);
    if (tid == 0) {
      int64_t tot = 0;
      for (int k = 0; k < kAggBlock / kWave; ++k) tot += s_w[k];
      s_base = tot ? static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long *>(d_ngroups),
                                                    static_cast<unsigned long long>(tot)))
                   : 0;
    }
    __syncthreads();
    int64_t p = s_base + incl - c;
    for (int k = 0; k < w; ++k) p += s_w[k];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const uint64_t k = s_key[s0 + j];
      if (k == static_cast<uint64_t>(kEmpty64)) continue;
      if (p < out_cap) {
        out_keys[p] = static_cast<int64_t>(k);
        out_sums[p] = static_cast<int64_t>(s_sum[s0 + j]);
      } else {
        latch(err, kErrCapacity);
      }
      ++p;
      s_key[s0 + j] = static_cast<uint64_t>(kEmpty64);
      s_sum[s0 + j] = 0;
    }
    __syncthreads();  // the table is clear (and s_base read) before the next bucket
  }
  if (full) latch(err, kErrTableFull);
}

// Groups of the pairs [0, min(*count, cap)) of keys/vals (kEmpty64 keys are
// skipped) into out_keys/out_sums, their number into *d_ngroups (which must be
// zero on entry).  keys/vals are overwritten (they hold the second move).
// Fewer than 2^31 pairs; a bucket may hold at most kAggSlots distinct keys
// (about 8192 x 4096 keys in all for keys that hash evenly), else the table-full
// error is latched.
// The moves and the bucket pass; the first move reads `first` (pairs or columns),
// the second writes keys/vals (cap entries each).
__global__ void k_narrow_counts(const int32_t *counts, int32_t *c1, int32_t *c2);

pyst_status pair_groupby_from(pyst_ctx *ctx, MoveArgs first, int64_t *keys, int64_t *vals, const int64_t *count,
                              int64_t cap, int64_t *out_keys, int64_t *out_sums, int64_t out_cap,
                              int64_t *d_ngroups, hipStream_t stream) {
  if (cap >= (int64_t{1} << 31)) return set_error(PYST_ERR_ARG, "group-by: too many pairs");
  const int64_t n1 = int64_t{kRadix} * kAggBlocks1, n2 = int64_t{kAggBuckets} * kAggBlocks2;
  const size_t counts = (static_cast<size_t>(kAggBlocks1) * kAggBuckets + static_cast<size_t>(n1 + 1 + n2 + 1) * 2) *
                        sizeof(int32_t);
  Scratch sc(ctx, (counts + 255) / 256 * 256 + static_cast<size_t>(cap) * 16, stream);
  if (!sc.p) return set_error(PYST_ERR_NOMEM, "group-by: arena exhausted");
  int32_t *cnt = sc.as<int32_t>();
  int32_t *h1 = cnt + static_cast<int64_t>(kAggBlocks1) * kAggBuckets, *p1 = h1 + n1 + 1, *h2 = p1 + n1 + 1,
          *p2 = h2 + n2 + 1;
  int64_t *tk = reinterpret_cast<int64_t *>(static_cast<char *>(sc.p) + (counts + 255) / 256 * 256);
  int64_t *tv = tk + cap;
  // One counting pass over all pairs gives every first-move block's counts
  // per final bucket; the first move's positions are per part (hash bits
  // 58..63), the second's per bucket (bits 52..57) and second-move block.
  // The scans run over one more entry than the counts (zero), so that the
  // last offset is the total.
  MoveArgs m1 = first;
  m1.count = count;
  m1.cap = cap;
  m1.seg_off = nullptr;
  m1.seg_stride = 0;
  m1.bps = kAggBlocks1;
  m1.shift = 64 - kRadixLg;
  k_move_hist_both<<<kAggBlocks1, kAggBlock, 0, stream>>>(m1, cnt);
  PYST_LAUNCH_CHECK("k_move_hist_both");
  k_narrow_counts<<<static_cast<unsigned>(ceil_div(n1 + n2 + 1, 256)), 256, 0, stream>>>(cnt, h1, h2);
  PYST_LAUNCH_CHECK("k_narrow_counts");
  pyst_status st = scan_excl_i32(ctx, h1, p1, n1 + 1, nullptr, stream);
  if (st == PYST_OK) st = scan_excl_i32(ctx, h2, p2, n2 + 1, nullptr, stream);
  if (st != PYST_OK) return st;
  k_move_scatter<<<kAggBlocks1, kAggBlock, 0, stream>>>(m1, p1, tk, tv);
  PYST_LAUNCH_CHECK("k_move_scatter");
  // Second move: block j of part p reads what the first move's blocks
  // [64 j, 64 (j + 1)) wrote to part p, and writes it by bucket into keys/vals.
  MoveArgs m2{tk, tv, count, cap, p1, kAggBlocks1, kAggBlocks2, 64 - 2 * kRadixLg};
  m2.aligned = 1;
  k_move_scatter<<<kRadix * kAggBlocks2, kAggBlock, 0, stream>>>(m2, p2, keys, vals);
  PYST_LAUNCH_CHECK("k_move_scatter");
  const int gblocks = static_cast<int>(std::min<int64_t>(kAggBuckets, std::max(1, ctx_num_cus(ctx))));
  k_bucket_groups<<<gblocks, kAggBlock, 0, stream>>>(keys, vals, p2, kAggBlocks2, out_keys, out_sums, out_cap,
                                                     d_ngroups, ctx_err_word(ctx));
  PYST_LAUNCH_CHECK("k_bucket_groups");
  return PYST_OK;
}

// ---------------------------------------------------------------- narrow pairs
// Group-by of int32 keys with int32 values: a pair travels as ONE 8-byte word
// (key << 32 | value), half the bytes of the (int64, int64) pairs above, and
// both moves take their counts from one pass over the keys.  The bucket of a
// key is the top 12 bits of a 32-bit hash: bits 26..31 pick its part in the
// first move, bits 20..25 its bucket within the part in the second, bits 0..12
// its LDS slot.  The second move's block j of part p reads exactly the pairs
// that the first move's blocks [j G, (j + 1) G) wrote to part p (G = kNB1 /
// kNB2), so its counts are sums of the first pass's per-block counts and no
// second pass over the pairs is needed to count them.
constexpr int kNB1 = 512;                // blocks of the first move (and of the counting pass)
constexpr int kNB2 = 8;                  // blocks per part in the second move
constexpr int kNG = kNB1 / kNB2;         // first-move blocks behind one second-move block
constexpr int kNItems = 8;               // rows per thread and round of the counting pass
constexpr uint32_t kNarrowSeed = 0x6b43a9b5u;
static_assert(kNB1 % kNB2 == 0, "second-move blocks cover whole groups of first-move blocks");
static_assert(kNB1 == kAggBlocks1 && kNB2 == kAggBlocks2, "the wide pair moves share the count layout");

__device__ __forceinline__ uint32_t narrow_hash(int32_t key) { return fmix32(static_cast<uint32_t>(key) ^ kNarrowSeed); }

struct NarrowArgs {
  const int32_t *kcol;
  const int32_t *vcol;
  const int32_t *sel;    // nullptr: rows 0..count-1
  const int64_t *count;  // rows (or selected rows) to group
  int64_t cap;           // upper bound of *count
};

__device__ __forceinline__ void narrow_range(const NarrowArgs &a, int blk, int nblk, int64_t *lo, int64_t *hi) {
  const int64_t n = *a.count < a.cap ? *a.count : a.cap;
  const int64_t per = (n + nblk - 1) / nblk;
  *lo = per * blk < n ? per * blk : n;
  *hi = *lo + per < n ? *lo + per : n;
}

// Per first-move block: counts of its rows in each of the 4096 buckets.
__global__ __launch_bounds__(kAggBlock) void k_narrow_hist(NarrowArgs a, int32_t *counts) {
  __shared__ int32_t s_c[kAggBuckets];
  for (int i = threadIdx.x; i < kAggBuckets; i += kAggBlock) s_c[i] = 0;
  __syncthreads();
  int64_t lo, hi;
  const int blk = static_cast<int>(xcd_block(blockIdx.x, gridDim.x));  // as k_narrow_move<true>
  narrow_range(a, blk, kNB1, &lo, &hi);
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += int64_t{kAggBlock} * kNItems) {
    int32_t k[kNItems];
#pragma unroll
    for (int u = 0; u < kNItems; ++u) {
      const int64_t i = i0 + int64_t{u} * kAggBlock;
      k[u] = i < hi ? a.kcol[row_of(a.sel, i)] : 0;
    }
#pragma unroll
    for (int u = 0; u < kNItems; ++u)
      if (i0 + int64_t{u} * kAggBlock < hi) atomicAdd(&s_c[narrow_hash(k[u]) >> 20], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kAggBuckets; i += kAggBlock) counts[int64_t{blk} * kAggBuckets + i] = s_c[i];
}

// c1[p * kNB1 + b]: rows of first-move block b in part p; c2[(p * 64 + q) * kNB2
// + j]: rows of bucket (p, q) that second-move block j of part p moves.  The
// entry after each array is zero so that its exclusive scan ends in the total.
__global__ void k_narrow_counts(const int32_t *counts, int32_t *c1, int32_t *c2) {
  const int64_t t = blockIdx.x * int64_t{blockDim.x} + threadIdx.x;
  constexpr int64_t n1 = int64_t{kRadix} * kNB1, n2 = int64_t{kAggBuckets} * kNB2;
  if (t < n1) {
    const int p = static_cast<int>(t / kNB1), b = static_cast<int>(t % kNB1);
    int32_t c = 0;
    for (int q = 0; q < kRadix; ++q) c += counts[int64_t{b} * kAggBuckets + p * kRadix + q];
    c1[t] = c;
  } else if (t < n1 + n2) {
    const int64_t u = t - n1;
    const int bucket = static_cast<int>(u / kNB2), j = static_cast<int>(u % kNB2);
    int32_t c = 0;
    for (int b = j * kNG; b < (j + 1) * kNG; ++b) c += counts[int64_t{b} * kAggBuckets + bucket];
    c2[u] = c;
  } else if (t == n1 + n2) {
    c1[n1] = 0;
    c2[n2] = 0;
  }
}

// One move of narrow pairs.  FIRST: block b reads its rows of the columns and
// writes them by part (bits 26..31) at pos1; else block p * kNB2 + j reads the
// pairs of its range of part p and writes them by bucket (bits 20..25) at pos2.
// Each 4096-pair tile is ranked by destination in LDS and every destination's
// pairs of the tile leave as one contiguous run (as k_move_scatter does).
template <bool FIRST>
__global__ __launch_bounds__(kAggBlock) void k_narrow_move(NarrowArgs a, const uint64_t *in, const int32_t *pos1,
                                                          const int32_t *pos2, uint64_t *out) {
  __shared__ uint64_t s_p[kMoveTile];
  __shared__ uint8_t s_b[kMoveTile];
  __shared__ int32_t s_base[kRadix], s_cnt[kRadix], s_off[kRadix + 1];
  const int tid = static_cast<int>(threadIdx.x);
  int64_t lo, hi;
  int part = 0;
  const int blk = static_cast<int>(xcd_block(blockIdx.x, gridDim.x));  // neighbouring ranges on one XCD
  if (FIRST) {
    narrow_range(a, blk, kNB1, &lo, &hi);
    if (tid < kRadix) s_base[tid] = pos1[int64_t{tid} * kNB1 + blk];
  } else {
    part = blk / kNB2;
    const int j = blk % kNB2;
    lo = pos1[int64_t{part} * kNB1 + j * kNG];
    hi = pos1[int64_t{part} * kNB1 + (j + 1) * kNG];
    if (tid < kRadix) s_base[tid] = pos2[(int64_t{part} * kRadix + tid) * kNB2 + j];
  }
  const int shift = FIRST ? 26 : 20;
  for (int64_t t0 = lo; t0 < hi; t0 += kMoveTile) {  // block-uniform
    if (tid < kRadix) s_cnt[tid] = 0;
    __syncthreads();
    uint64_t pr[kMoveTileItems];
    int bk[kMoveTileItems], rk[kMoveTileItems];
#pragma unroll
    for (int u = 0; u < kMoveTileItems; ++u) {
      const int64_t i = t0 + int64_t{u} * kAggBlock + tid;
      if (FIRST) {
        const int64_t r = i < hi ? row_of(a.sel, i) : 0;
        const int32_t k = i < hi ? a.kcol[r] : 0, v = i < hi ? a.vcol[r] : 0;
        pr[u] = (static_cast<uint64_t>(static_cast<uint32_t>(k)) << 32) | static_cast<uint32_t>(v);
      } else {
        pr[u] = i < hi ? in[i] : 0;
      }
    }
#pragma unroll
    for (int u = 0; u < kMoveTileItems; ++u) {
      const int64_t i = t0 + int64_t{u} * kAggBlock + tid;
      bk[u] = i < hi ? static_cast<int>((narrow_hash(static_cast<int32_t>(pr[u] >> 32)) >> shift) & (kRadix - 1)) : -1;
      rk[u] = bk[u] >= 0 ? atomicAdd(&s_cnt[bk[u]], 1) : 0;
    }
    __syncthreads();
    if (tid < kWave) {
      const int c = s_cnt[tid];
      const int incl = wave_inclusive_scan(c);
      s_off[tid] = incl - c;
      if (tid == kWave - 1) s_off[kRadix] = incl;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMoveTileItems; ++u)
      if (bk[u] >= 0) {
        const int p = s_off[bk[u]] + rk[u];
        s_p[p] = pr[u];
        s_b[p] = static_cast<uint8_t>(bk[u]);
      }
    __syncthreads();
    const int n = s_off[kRadix];
    for (int t = tid; t < n; t += kAggBlock) {
      const int b = s_b[t];
      out[int64_t{s_base[b]} + (t - s_off[b])] = s_p[t];
    }
    __syncthreads();
    if (tid < kRadix) s_base[tid] += s_cnt[tid];
  }
}

// Inverse of the narrow hash: fmix32 is a bijection (xor-shifts and odd
// multipliers), undone step by step with the multipliers' inverses mod 2^32.
__host__ __device__ constexpr uint32_t inv_odd32(uint32_t c) {
  uint32_t x = c;  // Newton's iteration for the inverse mod 2^32 (c odd): 3, 6, 12, 24, 48 bits
  for (int i = 0; i < 5; ++i) x *= 2u - c * x;
  return x;
}
static_assert(0x85ebca6bu * inv_odd32(0x85ebca6bu) == 1u && 0xc2b2ae35u * inv_odd32(0xc2b2ae35u) == 1u, "inverse");
__device__ __forceinline__ int32_t narrow_unhash(uint32_t h) {
  h ^= h >> 16;
  h *= inv_odd32(0xc2b2ae35u);
  h ^= (h >> 13) ^ (h >> 26);
  h *= inv_odd32(0x85ebca6bu);
  h ^= h >> 16;
  return static_cast<int32_t>(h ^ kNarrowSeed);
}

// Sums every bucket's narrow pairs in an LDS table and writes its groups, one
// block per CU walking the buckets as k_bucket_groups does.  The table holds
// each key's 32-bit hash (slot: its low 13 bits), which identifies the key
// because the hash is a bijection; every hash of bucket b has b as its top 12
// bits, so a hash with other top bits marks an empty slot of that bucket.  A
// slot is read before it is claimed: a key seen before in the bucket costs one
// LDS read and one add instead of a compare-and-swap and an add.  *d_ngroups
// must be zero on entry.
__device__ __forceinline__ uint32_t narrow_empty(int b) { return static_cast<uint32_t>(~b & (kAggBuckets - 1)) << 20; }

__global__ __launch_bounds__(kAggBlock) void k_narrow_groups(const uint64_t *pairs, const int32_t *pos2,
                                                            int64_t *out_keys, int64_t *out_sums, int64_t out_cap,
                                                            int64_t *d_ngroups, uint32_t *err) {
  __shared__ uint32_t s_h[kAggSlots];
  __shared__ uint64_t s_sum[kAggSlots];
  __shared__ int32_t s_w[kAggBlock / kWave];
  __shared__ int64_t s_base;
  constexpr int U = 16;  // a whole bucket (14.6k pairs on average at 60M rows) in one round
  constexpr int PER = kAggSlots / kAggBlock;
  const int tid = static_cast<int>(threadIdx.x);
  int b = static_cast<int>(blockIdx.x);
  for (int s = tid; s < kAggSlots; s += kAggBlock) {
    s_h[s] = narrow_empty(b);
    s_sum[s] = 0;
  }
  bool full = false;
  uint64_t pp[U];
  bool have[U];
  auto load_round = [&](int64_t i0, int64_t hi) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + int64_t{u} * kAggBlock;
      have[u] = i < hi;
      pp[u] = have[u] ? pairs[i] : 0;
    }
  };
  // The home slots of all U pairs are read together first; a pair whose key
  // already sits in its home slot (most of them: keys repeat) is added at once,
  // the others walk their runs one by one, claiming an empty slot with a CAS.
  auto insert_round = [&](uint32_t empty) {
    uint32_t h[U], cur[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      h[u] = narrow_hash(static_cast<int32_t>(pp[u] >> 32));
      cur[u] = have[u] ? s_h[h[u] & (kAggSlots - 1)] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!have[u]) continue;
      const uint64_t val = static_cast<uint64_t>(static_cast<int64_t>(static_cast<int32_t>(pp[u] & 0xffffffffu)));
      uint32_t s = h[u] & (kAggSlots - 1);
      uint32_t c = cur[u];
      for (int probes = 0;; ++probes) {
        if (c == empty) c = atomicCAS(&s_h[s], empty, h[u]);
        if (c == empty || c == h[u]) {
          atomicAdd(reinterpret_cast<unsigned long long *>(&s_sum[s]), static_cast<unsigned long long>(val));
          break;
        }
        if (probes + 1 == kAggSlots) {
          full = true;
          break;
        }
        s = (s + 1) & (kAggSlots - 1);
        c = s_h[s];
      }
    }
  };
  if (b < kAggBuckets) load_round(pos2[int64_t{b} * kNB2] + tid, pos2[int64_t{b + 1} * kNB2]);
  __syncthreads();
  for (; b < kAggBuckets; b += static_cast<int>(gridDim.x)) {  // block-uniform
    const uint32_t empty = narrow_empty(b);
    const int64_t lo = pos2[int64_t{b} * kNB2], hi = pos2[int64_t{b + 1} * kNB2];
    insert_round(empty);
    for (int64_t i0 = lo + tid + int64_t{kAggBlock} * U; i0 < hi; i0 += int64_t{kAggBlock} * U) {
      load_round(i0, hi);
      insert_round(empty);
    }
    __syncthreads();
    // Compact the bucket's groups to the front of the table (each thread holds
    // its PER slots in registers across the barrier), then write them out with
    // consecutive threads on consecutive positions.
    const int s0 = tid * PER;
    uint32_t hh[PER];
    uint64_t ss[PER];
    int c = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      hh[j] = s_h[s0 + j];
      ss[j] = s_sum[s0 + j];
      c += hh[j] != empty;
    }
    const int incl = wave_inclusive_scan(c);
    const int w = tid / kWave;
    if (lane_id() == kWave - 1) s_w[w] = incl;
    __syncthreads();
    const int nb = b + static_cast<int>(gridDim.x);
    if (nb < kAggBuckets) load_round(pos2[int64_t{nb} * kNB2] + tid, pos2[int64_t{nb + 1} * kNB2]);
    int tot = 0, q = incl - c;
    for (int k = 0; k < kAggBlock / kWave; ++k) {
      tot += s_w[k];
      if (k < w) q += s_w[k];
    }
    if (tid == 0)
      s_base = tot ? static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long *>(d_ngroups),
                                                    static_cast<unsigned long long>(tot)))
                   : 0;
#pragma unroll
    for (int j = 0; j < PER; ++j)
      if (hh[j] != empty) {
        s_h[q] = hh[j];
        s_sum[q] = ss[j];
        ++q;
      }
    __syncthreads();
    const int64_t base = s_base;
    for (int i = tid; i < tot; i += kAggBlock) {
      if (base + i < out_cap) {
        out_keys[base + i] = narrow_unhash(s_h[i]);
        out_sums[base + i] = static_cast<int64_t>(s_sum[i]);
      } else {
        latch(err, kErrCapacity);
      }
    }
    __syncthreads();
    const uint32_t next_empty = narrow_empty(nb);
    for (int i = tid; i < kAggSlots; i += kAggBlock) {
      s_h[i] = next_empty;
      s_sum[i] = 0;
    }
    __syncthreads();
  }
  if (full) latch(err, kErrTableFull);
}

// Bytes of scratch narrow_groupby needs for up to `cap` rows.
size_t narrow_groupby_bytes(int64_t cap) {
  const int64_t n1 = int64_t{kRadix} * kNB1, n2 = int64_t{kAggBuckets} * kNB2;
  const size_t counts = static_cast<size_t>(kNB1) * kAggBuckets + 2 * static_cast<size_t>(n1 + 1 + n2 + 1);
  return (counts * sizeof(int32_t) + 255) / 256 * 256 + static_cast<size_t>(cap) * 16 + 256;
}

// GROUP BY key SUM(val) of the rows [0, *count) (of the selection sel) of int32
// columns through narrow pairs, in scratch `ws` of narrow_groupby_bytes(cap).
// *d_ngroups must be zero on entry.  Fewer than 2^31 rows.
pyst_status narrow_groupby(pyst_ctx *ctx, const int32_t *kcol, const int32_t *vcol, const int32_t *sel,
                           const int64_t *count, int64_t cap, void *ws, int64_t *out_keys, int64_t *out_sums,
                           int64_t out_cap, int64_t *d_ngroups, hipStream_t stream) {
  if (cap >= (int64_t{1} << 31)) return set_error(PYST_ERR_ARG, "group-by: too many rows");
  const int64_t n1 = int64_t{kRadix} * kNB1, n2 = int64_t{kAggBuckets} * kNB2;
  int32_t *counts = static_cast<int32_t *>(ws);
  int32_t *c1 = counts + static_cast<int64_t>(kNB1) * kAggBuckets, *p1 = c1 + n1 + 1, *c2 = p1 + n1 + 1,
          *p2 = c2 + n2 + 1;
  const size_t cbytes = (static_cast<size_t>(kNB1) * kAggBuckets + 2 * static_cast<size_t>(n1 + 1 + n2 + 1)) *
                        sizeof(int32_t);
  uint64_t *tmp = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + (cbytes + 255) / 256 * 256);
  uint64_t *pairs = tmp + cap;
  NarrowArgs a{kcol, vcol, sel, count, cap};
  k_narrow_hist<<<kNB1, kAggBlock, 0, stream>>>(a, counts);
  PYST_LAUNCH_CHECK("k_narrow_hist");
  k_narrow_counts<<<static_cast<unsigned>(ceil_div(n1 + n2 + 1, 256)), 256, 0, stream>>>(counts, c1, c2);
  PYST_LAUNCH_CHECK("k_narrow_counts");
  pyst_status st = scan_excl_i32(ctx, c1, p1, n1 + 1, nullptr, stream);
  if (st == PYST_OK) st = scan_excl_i32(ctx, c2, p2, n2 + 1, nullptr, stream);
  if (st != PYST_OK) return st;
  k_narrow_move<true><<<kNB1, kAggBlock, 0, stream>>>(a, nullptr, p1, p2, tmp);
  PYST_LAUNCH_CHECK("k_narrow_move<1>");
  k_narrow_move<false><<<kRadix * kNB2, kAggBlock, 0, stream>>>(a, tmp, p1, p2, pairs);
  PYST_LAUNCH_CHECK("k_narrow_move<2>");
  const int gblocks = static_cast<int>(std::min<int64_t>(kAggBuckets, std::max(1, ctx_num_cus(ctx))));
  k_narrow_groups<<<gblocks, kAggBlock, 0, stream>>>(pairs, p2, out_keys, out_sums, out_cap, d_ngroups,
                                                     ctx_err_word(ctx));
  PYST_LAUNCH_CHECK("k_narrow_groups");
  return PYST_OK;
}

pyst_status pair_groupby(pyst_ctx *ctx, int64_t *keys, int64_t *vals, const int64_t *count, int64_t cap,
                         int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                         hipStream_t stream) {
  MoveArgs first{};
  first.keys = keys;
  first.vals = vals;
  return pair_groupby_from(ctx, first, keys, vals, count, cap, out_keys, out_sums, out_cap, d_ngroups, stream);
}

// Group-by of the rows [0, *count) of a selection over (key, val) columns: the
// first move reads the columns, so no widened copy of the pairs is written.
// pk/pv: scratch for cap pairs.
pyst_status column_groupby(pyst_ctx *ctx, const pyst_col *key, const pyst_col *val, const int32_t *sel,
                           const int64_t *count, int64_t *pk, int64_t *pv, int64_t *out_keys, int64_t *out_sums,
                           int64_t out_cap, int64_t *d_ngroups, hipStream_t stream) {
  MoveArgs first{};
  first.kcol = key->data;
  first.vcol = val->data;
  first.sel = sel;
  first.k64 = key->dtype == PYST_I64;
  first.v64 = val->dtype == PYST_I64;
  first.err = ctx_err_word(ctx);
  return pair_groupby_from(ctx, first, pk, pv, count, key->n, out_keys, out_sums, out_cap, d_ngroups, stream);
}

}  // namespace pyst

// Fast path of pyst_query for the plan shapes the path is measured on:
// 1 or 2 joins on int32 keys, fact predicates on int32 columns, group key made
// of join keys / join payloads, value = v0 or v0 * (c - v1).
//
// Design for CDNA4 (measured on MI355X):
//  * The fact pass is bound by L2 request throughput, not HBM: every probe of
//    a 4 MB table is a random L2 request.  So (1) rows rejected by the fact
//    predicates or by an LDS-resident blocked Bloom filter of the first join
//    issue no table access at all, and (2) the first probe of each row is a
//    raw buffer load whose offset is forced out of range for dead rows: the
//    hardware returns zeros without a memory access, so the probes of a
//    thread's rows issue back to back with no branches and no serializing
//    waits between them.
//  * Group existence for sums kept in join-table slots is recorded only by
//    the first add to a slot (the atomic returns the old sum 0), instead of a
//    store per matching row.
//  * The dimension filter compacts per block (no global counter to clear);
//    the table initializer sums the per-block counts to size the table, so
//    the whole query needs no host synchronization and no memset.
#include <algorithm>
#include <cstring>

#include "pyst_internal.h"
#include "query.h"
#include "table.h"

namespace pyst {

#define PYST_GLOBAL __attribute__((address_space(1)))

constexpr int kBloomLgw = 15;                       // 2^15 words = 128 KiB of LDS
constexpr int64_t kPairRun = 2048;                  // pair slots a wave reserves at a time
constexpr int kBloomWords = 1 << kBloomLgw;
constexpr int64_t kBloomMaxKeys = (int64_t{32} << kBloomLgw) * 2 / 3;  // above this the filter passes almost all
constexpr int kDimTile = 4096;                      // rows per block of the dimension filter
constexpr int kFastBlock = 1024;                    // one block of 16 waves per CU next to the 128 KiB filter
constexpr int kBufOob = 0x7ffffff0;                 // buffer offset beyond any table: load returns 0, no access
constexpr int kNonTemporal = 2;                     // cache policy of streamed columns: keep the table in the L2
constexpr int kBufferDword3 = 0x00020000;           // raw buffer resource word 3 on CDNA

// Bucketed slot sums (single-join queries grouped by the join key).  Random
// 64-bit atomic adds on MI355X retire at about 23e9/s chip-wide whatever the
// table size (one L2 atomic per cache line touched), so a fact pass that adds
// every matching row into the join table is bound by them.  Instead the pass
// stages (slot, value) pairs in LDS and moves them, bucket by bucket of
// kBucketSlots slots, into chunks in HBM; a second kernel adds each bucket up
// in LDS.  That costs 8 bytes written and read per matching row (a value that
// does not fit in 43 bits is added directly).
constexpr int kBucketLg = 13;
constexpr int64_t kBucketSlots = int64_t{1} << kBucketLg;  // 64 KiB of LDS sums in the second kernel
constexpr int kMaxBuckets = 256;                            // staged join tables: up to 2^21 slots
constexpr int kMaxSumBuckets = 512;                         // second-kernel blocks: tables up to 2^22 slots
constexpr uint32_t kStageCap = 3448;                        // staged pairs per block (27 KiB: the LDS the filter leaves)
constexpr uint32_t kFlushAt = 1024;                         // staged pairs that trigger a move to HBM
constexpr uint32_t kCheckMax = 8;                           // most steps between the block's staging checks
constexpr int kStageSlotBits = 21;                          // slot bits of a staged pair: kMaxBuckets buckets
constexpr int kStarRows = 4;                                // rows per lane and step of the staged fact pass
constexpr uint32_t kChunkLg = 9;                            // pairs per chunk of the single query: 512
constexpr uint32_t kChunk = 1u << kChunkLg;
constexpr uint32_t kNoChunk = 0xffffffffu;

// Direct addressing (the first join table of a query summed in its slots):
// when the selected dimension keys span a range [kmin, kmin + range) with
// range <= the memory reserved for the hash table and <= 2^kStageSlotBits,
// key k owns slot k - kmin.  The table is then a bitmap of the selected keys
// over the range (in the key array's memory), so a probe is one bit and never
// walks; the LDS filter holds the bitmap itself (range <= 2^20 bits: exact) or
// each pair of its bits ORed into one (range <= 2^21: the exact bit is read
// from the bitmap in the L2).  The table initializer decides on the device,
// from the selected keys' minimum and maximum, and records the mode in the
// table header (TableDev::hdr[kHdrDirect], [kHdrKmin], [kHdrRange]).  The
// build marks each key in a byte map (one plain byte store per key: no atomic,
// and stores need no reply); the filter pass then packs the byte map into the
// bitmap and the LDS filter and counts the distinct keys into
// hdr[kHdrDistinct].  Fewer distinct keys than selected rows means a duplicate
// key, which the fact pass reports.
constexpr int kHdrDirect = 2, kHdrKmin = 3, kHdrRange = 4, kHdrDistinct = 5;
// Header byte kHdrAddedByte + b is set (by plain stores: no read, no atomic,
// so nothing in the fact pass waits on it) when a pass adds a sum straight
// into a slot of bucket b instead of staging it; the bucket sums then read
// that bucket's slot flags.  Cleared by the table initializers.
constexpr int kHdrAddedByte = 512;
static_assert(kHdrAddedByte + kMaxSumBuckets <= static_cast<int>(kHdrBytes), "header bytes");

// Only for tables of at most kMaxSumBuckets buckets (those with bucketed sums).
__device__ __forceinline__ void mark_added(const TableDev &t, int64_t s) {
  reinterpret_cast<uint8_t *>(t.hdr)[kHdrAddedByte + (s >> kBucketLg)] = 1;
}
__device__ __forceinline__ bool bucket_added(const TableDev &t, uint32_t b) {
  return reinterpret_cast<const uint8_t *>(t.hdr)[kHdrAddedByte + b] != 0;
}
constexpr int64_t kFilterBits = int64_t{32} << kBloomLgw;  // 2^20

static_assert((int64_t{kMaxBuckets} << kBucketLg) == (int64_t{1} << kStageSlotBits), "staged slot bits");

// A staged pair is one 8-byte word, value << kStageSlotBits | slot, so the
// value must fit in 64 - kStageSlotBits bits (two's complement); others are
// added directly.  (Its chunk record, value << kBucketLg | slot within the
// bucket, then fits too.)
__device__ __forceinline__ bool fits_stage(int64_t v) {
  const int64_t t = v >> (63 - kStageSlotBits);
  return t == 0 || t == -1;
}

// The chunks past the blocks' first ones are split evenly between the nb
// buckets of the table (nb is known on the device only), so that bucket b's
// later chunks are the first next[b] of its own region: the second kernel
// reads them without searching the pool.  A bucket whose region is used up
// adds its further pairs directly.
struct BucketPool {
  uint64_t *rec;     // pair e of chunk c at [c * chunk + e]: value << kBucketLg | slot within the bucket
  uint32_t *fill;    // pairs in each chunk
  uint32_t *next;    // [kMaxSumBuckets] chunks each bucket has taken from its region (zeroed with the table)
  uint32_t nchunks;  // chunks in the pool
  uint32_t blocks;   // fact-pass blocks; block k starts with chunks [k * stride, k * stride + nb)
  uint32_t stride;   // buckets a block's first chunks are reserved for; a table with more
                     // buckets than this (its size is only known on the device) is not staged
  uint32_t chunk_lg; // log2 of the pairs per chunk
};
constexpr size_t kPoolHeadBytes = kMaxSumBuckets * sizeof(uint32_t);  // the next[] counters ahead of the records

__host__ __device__ inline uint32_t bucket_count(int64_t cap) {
  return cap > kBucketSlots ? static_cast<uint32_t>(cap >> kBucketLg) : 1u;
}

// Bucket b's region: chunks [region_first(bp, nb, b), + region_chunks(bp, nb)).
__device__ __forceinline__ uint32_t region_chunks(const BucketPool &bp, uint32_t nb) {
  return (bp.nchunks - bp.blocks * bp.stride) / nb;
}
__device__ __forceinline__ uint32_t region_first(const BucketPool &bp, uint32_t nb, uint32_t b) {
  return bp.blocks * bp.stride + b * region_chunks(bp, nb);
}

// The Bloom filter reuses the join table's key hash h.  The word is the top
// kBloomLgw bits of the key's home slot (h & mask), so that the keys of word w
// sit, up to probe displacement, in one run of table slots and the filter can
// be built from the table without a global atomic per key; the two bits come
// from a multiplicative remix of h.
__device__ __forceinline__ int bloom_shift(int64_t cap) {
  int lg = 0;
  while ((int64_t{1} << lg) < cap) ++lg;
  return lg > kBloomLgw ? lg - kBloomLgw : 0;
}
__device__ __forceinline__ uint32_t bloom_word(uint32_t h, int64_t mask, int shift) {
  return static_cast<uint32_t>((h & mask) >> shift);
}
__device__ __forceinline__ uint32_t bloom_bits(uint32_t h) {
  const uint32_t p = h * 0x9e3779b1u;
  return (1u << (p >> 27)) | (1u << ((p >> 22) & 31));
}

template <typename T>
__device__ __forceinline__ const PYST_GLOBAL T *gmem(const T *p) { return (const PYST_GLOBAL T *)p; }

// ------------------------------------------------------------------ dimension filter (block-local)
// Block b writes its selected row ids, in order, to sel[b*kDimTile ...] and their
// number to cnt[b]; no global counter.  With `key`, also the least and the
// greatest selected key of the block to kmin_b[b] / kmax_b[b] (INT32_MAX /
// INT32_MIN when it selects none), from which the table initializer decides
// on direct addressing.
__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// The keys of a filter tile's rows (rows past n read as 0), loaded before the
// predicate columns so that both are in flight together.
template <int ITEMS>
__device__ __forceinline__ void load_keys(const int32_t *key, const int64_t (&rows)[ITEMS], int64_t n,
                                          int32_t (&kv)[ITEMS]) {
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) kv[j] = rows[j] < n ? key[rows[j]] : 0;
}

// The least and greatest key of a wave's kept rows into s_min[w] / s_max[w].
template <int ITEMS>
__device__ __forceinline__ void wave_key_bounds(const int32_t (&kv)[ITEMS], const bool (&keep)[ITEMS], int w,
                                                int32_t *s_min, int32_t *s_max) {
  int32_t mn = INT32_MAX, mx = INT32_MIN;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j)
    if (keep[j]) {
      mn = min(mn, kv[j]);
      mx = max(mx, kv[j]);
    }
  mn = wave_min_i32(mn);
  mx = wave_max_i32(mx);
  if (lane_id() == 0) {
    s_min[w] = mn;
    s_max[w] = mx;
  }
}

// A direct table's byte map sits in its key memory after the bitmap, 16-byte
// aligned; the initializer clears whole 64-key groups of it (the most that one
// filter word packs).
__host__ __device__ __forceinline__ int64_t direct_bytemap_off(int64_t range) {
  return ((range + 31) / 32 * 4 + 15) / 16 * 16;
}
__host__ __device__ __forceinline__ int64_t direct_bytemap_len(int64_t range) { return (range + 63) / 64 * 64; }

// Whether a table whose selected keys (total of them) lie in [kmin, kmax] is
// direct-addressed: a keys-only table (4-byte slots) becomes a bitmap, a
// key + payload table (8-byte slots) keeps its slot format with key k in slot
// k - kmin.  max_range: the largest range its consumer takes.
__device__ __forceinline__ bool direct_fits(const TableDev &t, int64_t total, int64_t kmin, int64_t kmax,
                                            int64_t max_range) {
  const int64_t range = kmax - kmin + 1;
  if (total <= 0 || range > t.cap_alloc || range > max_range) return false;
  if (t.slot_bytes == 8) return true;
  return t.slot_bytes == 4 && direct_bytemap_off(range) + direct_bytemap_len(range) <= 4 * t.cap_alloc;
}

// Clears the slot sums and flags of slots [0, cap) (and at most one sum and 15
// flags past them, still inside the cap_alloc slots: cap_alloc is a power of
// two >= 64) with 16-byte stores, threads tid, tid + nthr, ... of a grid.
__device__ __forceinline__ void clear_sums(const TableDev &t, int64_t cap, int64_t tid, int64_t nthr) {
  uint4 *sums = reinterpret_cast<uint4 *>(t.sums), *flags = reinterpret_cast<uint4 *>(t.flags);
  for (int64_t i = tid; i < (cap + 1) / 2; i += nthr) sums[i] = uint4{0u, 0u, 0u, 0u};
  for (int64_t i = tid; i < (cap + 15) / 16; i += nthr) flags[i] = uint4{0u, 0u, 0u, 0u};
}

// Clears a direct table's byte map (threads tid, tid + nthr, ... of a grid).
__device__ __forceinline__ void direct_clear(const TableDev &t, int64_t range, int64_t tid, int64_t nthr) {
  uint4 *bytes = reinterpret_cast<uint4 *>(static_cast<char *>(t.slots) + direct_bytemap_off(range));
  for (int64_t i = tid; i < direct_bytemap_len(range) / 16; i += nthr) bytes[i] = uint4{0u, 0u, 0u, 0u};
}

// Slots of a direct-addressed table: the range, rounded up to whole buckets of
// sums (the table's reserved slots are a power of two >= the range, so they
// hold that many).
__host__ __device__ __forceinline__ int64_t direct_cap(int64_t range) {
  return range <= kBucketSlots ? range : (range + kBucketSlots - 1) / kBucketSlots * kBucketSlots;
}

// Words of a direct-addressed table's LDS filter: one bit per key up to 2^20
// keys, else one bit per key pair.
__host__ __device__ __forceinline__ int64_t direct_filter_words(int64_t range) {
  return ((range > kFilterBits ? (range + 1) / 2 : range) + 31) / 32;
}

__global__ __launch_bounds__(256) void k_dim_filter(PredSet ps, int64_t n, int32_t *sel, int32_t *cnt,
                                                    const int32_t *key, int32_t *kmin_b, int32_t *kmax_b) {
  constexpr int NW = 256 / kWave, ITEMS = kDimTile / 256;
  __shared__ int32_t s_cnt[NW], s_min[NW], s_max[NW];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t wbase = int64_t{blockIdx.x} * kDimTile + int64_t{w} * kWave * ITEMS;
  int64_t rows[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) rows[j] = wbase + int64_t{j} * kWave + lane;
  int32_t kv[ITEMS];
  if (key) load_keys<ITEMS>(key, rows, n, kv);  // uniform
  bool keep[ITEMS];
  eval_preds_items<ITEMS>(ps, rows, n, keep);
  if (key) wave_key_bounds<ITEMS>(kv, keep, w, s_min, s_max);  // uniform
  uint64_t m[ITEMS];
  int c = 0;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    m[j] = __ballot(keep[j]);
    c += __popcll(m[j]);
  }
  if (lane == 0) s_cnt[w] = c;
  __syncthreads();
  int pos = 0;
  for (int k = 0; k < w; ++k) pos += s_cnt[k];
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int k = 0; k < NW; ++k) tot += s_cnt[k];
    cnt[blockIdx.x] = tot;
    if (key) {
      int32_t mn = INT32_MAX, mx = INT32_MIN;
      for (int k = 0; k < NW; ++k) {
        mn = min(mn, s_min[k]);
        mx = max(mx, s_max[k]);
      }
      kmin_b[blockIdx.x] = mn;
      kmax_b[blockIdx.x] = mx;
    }
  }
  int32_t *out = sel + int64_t{blockIdx.x} * kDimTile;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if ((m[j] >> lane) & 1ull) out[pos + mbcnt(m[j])] = static_cast<int32_t>(wbase + int64_t{j} * kWave + lane);
    pos += __popcll(m[j]);
  }
}

// Table initialization sized from the per-block counts (or n without a filter);
// also clears the Bloom words and the caller's group/pair counters.  With the
// per-block key bounds (kmin_b / kmax_b) it chooses direct addressing when the
// selected keys' range allows it: the header then holds the mode, kmin and
// the range, hdr[0] the range rounded up to whole buckets (the slot count the
// sums and their buckets use), and the bitmap words are cleared instead of keys.
__global__ void k_fast_table_init(TableDev t, const int32_t *cnt, int64_t nblocks, int64_t n, double max_load,
                                  int64_t *zero0, int64_t *zero1, const int32_t *kmin_b, const int32_t *kmax_b,
                                  int64_t max_range, uint32_t *pool_next) {
  __shared__ int64_t s_total, s_kmin, s_kmax;
  if (threadIdx.x < kWave) {
    int64_t part = 0;
    int32_t mn = INT32_MAX, mx = INT32_MIN;
    if (cnt)
      for (int64_t b = threadIdx.x; b < nblocks; b += kWave) {
        part += cnt[b];
        if (kmin_b) {
          mn = min(mn, kmin_b[b]);
          mx = max(mx, kmax_b[b]);
        }
      }
    part = wave_sum(part);
    mn = wave_min_i32(mn);
    mx = wave_max_i32(mx);
    if (threadIdx.x == 0) {
      s_total = cnt ? part : n;
      s_kmin = mn;
      s_kmax = mx;
    }
  }
  __syncthreads();
  const int64_t total = s_total;
  const int64_t range = s_kmax - s_kmin + 1;
  const bool direct = kmin_b && direct_fits(t, total, s_kmin, s_kmax, max_range);
  const bool bitmap = direct && t.slot_bytes == 4;
  // a direct key + payload table: the range rounded up to whole 16-byte groups
  const int64_t cap = bitmap ? direct_cap(range) : direct ? (range + 1) / 2 * 2 : table_capacity(total, max_load, t.cap_alloc);
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < kMaxSumBuckets; i += nthr) {
    reinterpret_cast<uint8_t *>(t.hdr)[kHdrAddedByte + i] = 0;
    if (pool_next) pool_next[i] = 0;
  }
  if (tid == 0) {
    t.hdr[0] = cap;
    t.hdr[1] = total;
    t.hdr[kHdrDirect] = direct;
    t.hdr[kHdrKmin] = direct ? s_kmin : 0;
    t.hdr[kHdrRange] = direct ? range : 0;
    t.hdr[kHdrDistinct] = 0;
    if (zero0) *zero0 = 0;
    if (zero1) *zero1 = 0;
  }
  if (bitmap) {  // uniform: the byte map, the slot sums, the filter (the bitmap is packed whole later)
    direct_clear(t, range, tid, nthr);
    if (t.sums) clear_sums(t, cap, tid, nthr);
    if (t.bloom)
      for (int64_t i = tid; i < kBloomWords; i += nthr) t.bloom[i] = 0;
    return;
  }
  const int64_t words = t.slot_bytes == 4 ? cap / 2 : cap;
  const uint64_t fillv = t.slot_bytes == 4 ? (uint64_t{static_cast<uint32_t>(kEmpty32)} * 0x100000001ull)
                                           : uint64_t{static_cast<uint32_t>(kEmpty32)};
  uint64_t *p = static_cast<uint64_t *>(t.slots);
  for (int64_t i = tid; i < words; i += nthr) p[i] = fillv;
  if (t.sums) clear_sums(t, cap, tid, nthr);
  if (t.bloom)
    for (int64_t i = tid; i < kBloomWords; i += nthr) t.bloom[i] = 0;
}

// Build of a keys-only table from a block-local selection (or all rows): block
// b inserts the rows of dimension tile b (kDimTile rows, the dimension
// filter's tile), 16 per thread.  Each thread loads all of its row ids, then
// all of its keys, then issues the compare-and-swap of every row's home slot
// (a fresh table is mostly empty, so no read first) before it looks at any
// result: 16 inserts in flight per thread instead of one chain of dependent
// accesses; only rows whose home slot was taken walk on.
__device__ __forceinline__ void build_tile(const int32_t *key, const int32_t *sel, const int32_t *cnt, int64_t n,
                                           int64_t tile, const TableDev &t, uint32_t *err) {
  constexpr int ITEMS = kDimTile / 256;
  const int64_t mask = t.hdr[0] - 1;
  const int64_t base = tile * kDimTile;
  const int64_t rest = n - base;
  const int64_t have = sel ? cnt[tile] : (rest < kDimTile ? rest : kDimTile);
  int64_t row[ITEMS];
  bool v[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t i = int64_t{j} * 256 + threadIdx.x;
    v[j] = i < have;
    row[j] = v[j] ? (sel ? static_cast<int64_t>(sel[base + i]) : base + i) : 0;
  }
  int32_t k[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) k[j] = v[j] ? key[row[j]] : kEmpty32;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j)
    if (v[j] && k[j] == kEmpty32) {
      latch(err, kErrKey);
      v[j] = false;
    }
  int32_t *keys = static_cast<int32_t *>(t.slots);
  int64_t s[ITEMS];
  int32_t cur[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    s[j] = (table_hash32(k[j]) & mask) & ~int64_t{3};
    cur[j] = v[j] ? atomicCAS(&keys[s[j]], kEmpty32, k[j]) : kEmpty32;
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (!v[j]) continue;
    bool done = false;
    for (int64_t step = 0; step <= mask; ++step) {
      if (cur[j] == kEmpty32) {
        done = true;
        break;
      }
      if (cur[j] == k[j]) {
        latch(err, kErrDup);
        done = true;
        break;
      }
      s[j] = (s[j] + 1) & mask;
      cur[j] = atomicCAS(&keys[s[j]], kEmpty32, k[j]);
    }
    if (!done) latch(err, kErrTableFull);
  }
}

// The same tile into a direct-addressed table: one byte store per key marks
// it in the byte map (duplicates are found when the byte map is packed).
__device__ __forceinline__ void build_tile_direct(const int32_t *key, const int32_t *sel, const int32_t *cnt,
                                                  int64_t n, int64_t tile, const TableDev &t, uint32_t *err) {
  constexpr int ITEMS = kDimTile / 256;
  const uint32_t kmin = static_cast<uint32_t>(t.hdr[kHdrKmin]);
  uint8_t *bytes = static_cast<uint8_t *>(t.slots) + direct_bytemap_off(t.hdr[kHdrRange]);
  const int64_t base = tile * kDimTile;
  const int64_t rest = n - base;
  const int64_t have = sel ? cnt[tile] : (rest < kDimTile ? rest : kDimTile);
  int64_t row[ITEMS];
  bool v[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t i = int64_t{j} * 256 + threadIdx.x;
    v[j] = i < have;
    row[j] = v[j] ? (sel ? static_cast<int64_t>(sel[base + i]) : base + i) : 0;
  }
  int32_t k[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) k[j] = v[j] ? key[row[j]] : kEmpty32;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (v[j] && k[j] == kEmpty32) {
      latch(err, kErrKey);
      v[j] = false;
    }
    if (v[j]) bytes[static_cast<uint32_t>(k[j]) - kmin] = 1;  // < range: the range spans the selected keys
  }
}

// Tables built here always went through k_fast_table_init, which set the mode.
__global__ __launch_bounds__(256) void k_fast_build(const int32_t *key, const int32_t *sel, const int32_t *cnt, int64_t n,
                                                    TableDev t, uint32_t *err) {
  if (t.hdr[kHdrDirect]) build_tile_direct(key, sel, cnt, n, blockIdx.x, t, err);
  else build_tile(key, sel, cnt, n, blockIdx.x, t, err);
}

// Build of a key + payload table (8-byte slots), one row per thread: the
// slot is read first and claimed with a compare-and-swap where empty (a CAS
// straight to a cold line measured slower; so did 16 rows per thread, whose
// reads wait for each other before any claim).  A direct-addressed table
// takes one plain store per row into the key's own slot (the scattered
// 8-byte stores bound it: four rows per thread measured the same).
__global__ __launch_bounds__(256) void k_fast_build_payload(const int32_t *key, const int32_t *payload,
                                                            const int32_t *sel, const int32_t *cnt, int64_t n,
                                                            TableDev t, uint32_t *err) {
  const int64_t mask = t.hdr[0] - 1;
  uint64_t *slots = static_cast<uint64_t *>(t.slots);
  const uint64_t empty = static_cast<uint32_t>(kEmpty32);
  const bool direct = t.hdr[kHdrDirect] != 0;  // uniform
  const uint32_t kmin = static_cast<uint32_t>(t.hdr[kHdrKmin]);
  const int64_t nthr = int64_t{gridDim.x} * blockDim.x, tid = blockIdx.x * int64_t{blockDim.x} + threadIdx.x;
  for (int64_t i = tid; i < n; i += nthr) {
    int64_t row = i;
    if (sel) {
      if ((i % kDimTile) >= cnt[i / kDimTile]) continue;
      row = sel[i];
    }
    const int32_t k = key[row];
    if (k == kEmpty32) {
      latch(err, kErrKey);
      continue;
    }
    const uint64_t packed = uint64_t{static_cast<uint32_t>(k)} |
                            (uint64_t{static_cast<uint32_t>(payload ? payload[row] : static_cast<int32_t>(row))} << 32);
    if (direct) {  // a plain store into the key's own slot (k - kmin < range: the range spans the selected keys)
      slots[static_cast<uint32_t>(k) - kmin] = packed;
      continue;
    }
    int64_t s = (table_hash32(k) & mask) & ~int64_t{1};
    bool done = false;
    for (int64_t step = 0; step <= mask; ++step) {
      uint64_t cur = slots[s];
      if (static_cast<int32_t>(cur) == kEmpty32) {
        const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long *>(&slots[s]), empty, packed);
        if (old == empty) {
          done = true;
          break;
        }
        cur = old;
      }
      if (static_cast<int32_t>(cur) == k) {
        latch(err, kErrDup);
        done = true;
        break;
      }
      s = (s + 1) & mask;
    }
    if (!done) latch(err, kErrTableFull);
  }
}

// Bloom filter of a built keys-only table: thread w reads the slots whose home
// word is w and ORs their keys' bits into word w with one atomic; a key that
// probing moved into another word's slots ORs into its own word.
// Sets the filter bits of the keys whose home slots map to word w (words are
// 1 << shift consecutive slots; a key displaced past its word's slots is
// added to its own word with an atomic).  The filter must be clear first.
__device__ __forceinline__ void bloom_build_word(const TableDev &t, int64_t w) {
  const int64_t cap = t.hdr[0], mask = cap - 1;
  const int shift = bloom_shift(cap);
  const int64_t lo = w << shift, hi = (w + 1) << shift;
  if (lo >= cap) return;
  const int32_t *keys = static_cast<const int32_t *>(t.slots);
  uint32_t acc = 0;
  for (int64_t s0 = lo; s0 < hi; s0 += 32) {  // up to 32 slots (8 16-byte loads) per round, loads first
    int32_t k[32];
    if (hi - s0 >= 32) {  // runs of 32 and more are 16-byte aligned (powers of two)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const v4i32 v = reinterpret_cast<const v4i32 *>(keys + s0)[q];
        k[4 * q] = v.x;
        k[4 * q + 1] = v.y;
        k[4 * q + 2] = v.z;
        k[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 32; ++q) k[q] = s0 + q < hi ? keys[s0 + q] : kEmpty32;
    }
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      if (k[q] == kEmpty32) continue;
      const uint32_t h = table_hash32(k[q]);
      const uint32_t ww = bloom_word(h, mask, shift);
      if (ww == static_cast<uint32_t>(w)) acc |= bloom_bits(h);
      else atomicOr(&t.bloom[ww], bloom_bits(h));
    }
  }
  if (acc) atomicOr(&t.bloom[w], acc);
}

// Words of the filter a table of capacity cap uses: a word covers 1 << shift
// slots, so a table of fewer than kBloomWords slots uses one word per slot.
__host__ __device__ __forceinline__ int64_t bloom_words(int64_t cap) {
  return cap < kBloomWords ? cap : kBloomWords;
}

// The 16 bits of x's bit pairs, each pair ORed into one bit (pair i -> bit i).
__device__ __forceinline__ uint32_t pair_or16(uint32_t x) {
  x = (x | (x >> 1)) & 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0f0f0f0fu;
  x = (x | (x >> 4)) & 0x00ff00ffu;
  x = (x | (x >> 8)) & 0x0000ffffu;
  return x;
}

// The 16 bytes of a byte map (each 0 or 1) as 16 bits, byte i -> bit i.
__device__ __forceinline__ uint32_t pack_bytes16(uint4 q) {
  auto p4 = [](uint32_t x) { return ((x & 0x01010101u) * 0x01020408u) >> 24; };
  return p4(q.x) | (p4(q.y) << 4) | (p4(q.z) << 8) | (p4(q.w) << 12);
}

// One thread per filter word: packs the keys that filter word w covers from
// the byte map into the bitmap and returns the word; *keys receives how many
// keys it holds.  A direct-addressed table's filter is its bitmap (range <=
// 2^20 bits) or the bitmap with each bit pair ORed into one (range <= 2^21):
// filter bit j stands for the keys kmin + 2j and kmin + 2j + 1.
__device__ __forceinline__ uint32_t direct_pack_word(const TableDev &t, int64_t w, int *keys) {
  const int64_t range = t.hdr[kHdrRange], nwords = (range + 31) / 32;
  uint32_t *bm = static_cast<uint32_t *>(t.slots);
  const uint4 *bytes = reinterpret_cast<const uint4 *>(static_cast<const char *>(t.slots) + direct_bytemap_off(range));
  const bool paired = range > kFilterBits;
  uint32_t bits[2] = {0u, 0u};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t bw = paired ? 2 * w + h : w;
    if ((h == 0 || paired) && bw < nwords) {  // its 32 bytes lie within the cleared 64-key groups
      bits[h] = pack_bytes16(bytes[2 * bw]) | (pack_bytes16(bytes[2 * bw + 1]) << 16);
      bm[bw] = bits[h];
    }
  }
  *keys = __popc(bits[0]) + __popc(bits[1]);
  return paired ? pair_or16(bits[0]) | (pair_or16(bits[1]) << 16) : bits[0];
}

// Adds a block's count of distinct keys to the table header (one atomic per block).
__device__ __forceinline__ void add_distinct(const TableDev &t, int keys) {
  __shared__ int s_k[256 / kWave];
  const int v = wave_sum(keys);
  if (lane_id() == 0) s_k[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int sum = 0;
    for (int i = 0; i < static_cast<int>(blockDim.x) / kWave; ++i) sum += s_k[i];
    if (sum) atomicAdd(reinterpret_cast<unsigned long long *>(&t.hdr[kHdrDistinct]), static_cast<unsigned long long>(sum));
  }
}

__global__ __launch_bounds__(256) void k_fast_bloom(TableDev t) {
  if (t.hdr[kHdrDirect]) {  // uniform
    const int64_t w = blockIdx.x * int64_t{blockDim.x} + threadIdx.x;
    int keys;
    t.bloom[w] = direct_pack_word(t, w, &keys);
    add_distinct(t, keys);
    return;
  }
  if (t.hdr[1] > kBloomMaxKeys) return;  // the fact pass will not use the filter
  bloom_build_word(t, blockIdx.x * int64_t{blockDim.x} + threadIdx.x);
}

// Distinct keys of a direct-addressed key + payload table (slots not EMPTY)
// into hdr[kHdrDistinct]: a duplicate key's rows share one slot, so the count
// falls short of the selected rows.
// Each thread reads four 16-byte groups (eight slots) at once; few blocks
// (each adds its count with one atomic on the same header word, and those
// atomics serialize).
__global__ __launch_bounds__(256) void k_direct_count(TableDev t) {
  if (!t.hdr[kHdrDirect]) return;  // uniform
  constexpr int U = 4;
  const int64_t ng = t.hdr[0] / 2;  // the slot count is even
  const ulonglong2 *grp = static_cast<const ulonglong2 *>(t.slots);
  const ulonglong2 none{static_cast<uint32_t>(kEmpty32), static_cast<uint32_t>(kEmpty32)};
  int keys = 0;
  for (int64_t i0 = blockIdx.x * int64_t{256 * U} + threadIdx.x; i0 < ng; i0 += int64_t{gridDim.x} * 256 * U) {
    ulonglong2 q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = i0 + u * 256 < ng ? grp[i0 + u * 256] : none;
#pragma unroll
    for (int u = 0; u < U; ++u)
      keys += (static_cast<int32_t>(q[u].x) != kEmpty32) + (static_cast<int32_t>(q[u].y) != kEmpty32);
  }
  add_distinct(t, keys);
}

// ------------------------------------------------------------------ the fact pass
// Every memory access of the pass is a raw buffer access.  An offset at or past
// a resource's byte count reads zeros and writes nothing, without touching
// memory, so a dead row is an offset rather than a branch and all lanes of a
// wave issue the same instructions.  That keeps the compiler's count of
// outstanding memory operations exact around the loop: a store or atomic that
// some path skips would make every later wait for an older load (the next
// rows, loaded one iteration ahead) wait for the stores as well.
extern "C" __device__ long long pyst_buffer_atomic_add_i64(long long v, __amdgpu_buffer_rsrc_t r, int off, int soff,
                                                           int aux) __asm("llvm.amdgcn.raw.ptr.buffer.atomic.add.i64");

typedef uint32_t v2u32 __attribute__((ext_vector_type(2)));


__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, static_cast<int>(bytes), kBufferDword3);
}

// Rows [wbase, min(wbase + wr, end)) of a column as a buffer; empty for a null column.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t window(const void *col, int esz, int64_t wbase, int64_t end,
                                                         int64_t wr) {
  int64_t rows = end - wbase;
  rows = rows < 0 ? 0 : rows > wr ? wr : rows;
  const char *p = col ? static_cast<const char *>(col) + wbase * esz : nullptr;
  return rsrc(p, col ? rows * esz : 0);
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(x));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(static_cast<uint64_t>(x) >> 32));
  return static_cast<int64_t>((uint64_t{hi} << 32) | lo);
}

__device__ __forceinline__ v2u32 split64(int64_t x) {
  return v2u32{static_cast<uint32_t>(x), static_cast<uint32_t>(static_cast<uint64_t>(x) >> 32)};
}

// x in [lo, lo + span] as 32-bit integers, negated when neg (the host turns every comparison into this form).
__device__ __forceinline__ bool in_range(int32_t x, int32_t lo, uint32_t span, int32_t neg) {
  return (static_cast<uint32_t>(x) - static_cast<uint32_t>(lo) <= span) != (neg != 0);
}

// The columns read before the probes, for a lane's R consecutive rows (R / 4
// 16-byte loads per column).
template <int R>
struct FactRows {
  v4i32 f0[R / 4], f1[R / 4], c0[R / 4], c1[R / 4];
};

template <int N>
__device__ __forceinline__ int32_t row_of(const v4i32 (&x)[N], int r) {
  return x[r >> 2][r & 3];
}

// The lane whose R rows run past the end of the range reads its live rows one
// by one: a 16-byte load that is only partly in range is not used.
template <int R>
__device__ __forceinline__ void fix_tail(v4i32 (&x)[R / 4], __amdgpu_buffer_rsrc_t r, int lane, int left) {
  const bool mine = lane == left / R;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int row = lane * R + k;
    const int32_t v =
        static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(r, mine && row < left ? row * 4 : kBufOob, 0, 0));
    if (mine) x[k >> 2][k & 3] = v;
  }
}

template <int NJ, int R>
__device__ __forceinline__ FactRows<R> load_rows(const FastArgs &a, int64_t wbase, int64_t end, int lane) {
  constexpr int64_t WR = int64_t{kWave} * R;
  const __amdgpu_buffer_rsrc_t rf0 = window(a.fk[0], 4, wbase, end, WR);
  const __amdgpu_buffer_rsrc_t rf1 = window(NJ > 1 ? a.fk[1] : nullptr, 4, wbase, end, WR);
  const __amdgpu_buffer_rsrc_t rc0 = window(a.pcol[0], 4, wbase, end, WR);
  const __amdgpu_buffer_rsrc_t rc1 = window(a.pcol[1], 4, wbase, end, WR);
  const int off = lane * 4 * R;
  FactRows<R> x;
#pragma unroll
  for (int q = 0; q < R / 4; ++q) {
    x.f0[q] = __builtin_amdgcn_raw_buffer_load_b128(rf0, off + 16 * q, 0, kNonTemporal);
    x.f1[q] = NJ > 1 ? v4i32(__builtin_amdgcn_raw_buffer_load_b128(rf1, off + 16 * q, 0, kNonTemporal))
                     : v4i32{0, 0, 0, 0};
    x.c0[q] = __builtin_amdgcn_raw_buffer_load_b128(rc0, off + 16 * q, 0, kNonTemporal);
  }
  // (a uniform branch: a plan without a second predicate issues no load for it)
#pragma unroll
  for (int q = 0; q < R / 4; ++q)
    x.c1[q] = a.pcol[1] ? v4i32(__builtin_amdgcn_raw_buffer_load_b128(rc1, off + 16 * q, 0, kNonTemporal))
                        : v4i32{0, 0, 0, 0};
  const int64_t left = end - wbase;
  if (left > 0 && left < WR && (left & 3)) {  // wave-uniform; once per range
    const int l = static_cast<int>(left);
    fix_tail<R>(x.f0, rf0, lane, l);
    if (NJ > 1) fix_tail<R>(x.f1, rf1, lane, l);
    fix_tail<R>(x.c0, rc0, lane, l);
    if (a.pcol[1]) fix_tail<R>(x.c1, rc1, lane, l);
  }
  return x;
}

// First match of k in a 16-byte group of 4 keys: index, or -1 (none), and whether it holds EMPTY.
__device__ __forceinline__ int match4(v4i32 q, int32_t k, bool *empty) {
  *empty = q.x == kEmpty32 || q.y == kEmpty32 || q.z == kEmpty32 || q.w == kEmpty32;
  return q.x == k ? 0 : q.y == k ? 1 : q.z == k ? 2 : q.w == k ? 3 : -1;
}

#define PYST_LDS __attribute__((address_space(3)))

__device__ __forceinline__ uint32_t lds_add(PYST_LDS uint32_t *p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A block's LDS staging area of (slot, value) pairs and its current chunk per bucket.
struct StageLds {
  PYST_LDS uint64_t *ent;      // staged pairs: value << kStageSlotBits | slot
  PYST_LDS uint32_t *cnt;      // staged pairs (may exceed kStageCap: the excess was added directly)
  PYST_LDS uint32_t *chunk;    // [kMaxBuckets] current chunk
  PYST_LDS uint32_t *fill;     // [kMaxBuckets] pairs in it
  PYST_LDS uint32_t *hist;     // [kMaxBuckets] staged pairs per bucket
  PYST_LDS uint32_t *rank;     // [kMaxBuckets] pairs placed so far in this move
  PYST_LDS uint32_t *newbase;  // [kMaxBuckets] first chunk added in this move
};

// Moves the staged pairs into the block's chunks, bucket by bucket.  Every
// thread of the block calls it; it leaves the staging area empty.  Pairs that
// find the pool used up are added straight into the table's slot sums (the
// second kernel merges those in), so a pool smaller than the worst case only
// costs atomics.
__device__ __forceinline__ void stage_flush(const StageLds &sl, const BucketPool &bp, const TableDev &t, uint32_t nb) {
  const uint32_t tid = threadIdx.x;
  const uint32_t CH = 1u << bp.chunk_lg;
  const uint32_t n = *sl.cnt < kStageCap ? *sl.cnt : kStageCap;
  constexpr uint64_t slot_mask = (uint64_t{1} << kStageSlotBits) - 1;
  for (uint32_t i = tid; i < n; i += kFastBlock)
    lds_add(&sl.hist[static_cast<uint32_t>(sl.ent[i] & slot_mask) >> kBucketLg], 1u);
  __syncthreads();
  if (tid < nb) {
    const uint32_t t = sl.fill[tid] + sl.hist[tid];
    const uint32_t k = t > CH ? (t - 1) >> bp.chunk_lg : 0;  // chunks to add once the current one is full
    uint32_t first = 0;
    if (k) {
      const uint32_t reg = region_chunks(bp, nb), used = atomicAdd(&bp.next[tid], k);
      first = region_first(bp, nb, tid) + used;
      if (used + k > reg) {  // the region is used up: its chunks of this range stay empty
        for (uint32_t j = used; j < reg; ++j) bp.fill[region_first(bp, nb, tid) + j] = 0;
        first = kNoChunk;
      } else {
        bp.fill[sl.chunk[tid]] = CH;
        for (uint32_t j = 0; j + 1 < k; ++j) bp.fill[first + j] = CH;
      }
    }
    sl.newbase[tid] = first;
    sl.rank[tid] = 0;
  }
  __syncthreads();
  for (uint32_t i = tid; i < n; i += kFastBlock) {
    const uint64_t en = sl.ent[i];
    const uint32_t s = static_cast<uint32_t>(en & slot_mask), b = s >> kBucketLg;
    const uint32_t pos = sl.fill[b] + lds_add(&sl.rank[b], 1u);
    if (pos >= CH && sl.newbase[b] == kNoChunk) {  // pool used up: add directly
      atomicAdd(reinterpret_cast<unsigned long long *>(&t.sums[s]),
                static_cast<unsigned long long>(static_cast<int64_t>(en) >> kStageSlotBits));
      t.flags[s] = 1;
      mark_added(t, s);
      continue;
    }
    const uint32_t c = pos < CH ? sl.chunk[b] : sl.newbase[b] + (pos >> bp.chunk_lg) - 1;
    const size_t e = (size_t{c} << bp.chunk_lg) + (pos & (CH - 1));
    bp.rec[e] = static_cast<uint64_t>((static_cast<int64_t>(en) >> kStageSlotBits) << kBucketLg) |
                (s & (kBucketSlots - 1));
  }
  __syncthreads();
  if (tid < nb) {
    const uint32_t t = sl.fill[tid] + sl.hist[tid];
    if (t > CH && sl.newbase[tid] != kNoChunk) {
      const uint32_t k = (t - 1) >> bp.chunk_lg;
      sl.chunk[tid] = sl.newbase[tid] + k - 1;
      sl.fill[tid] = t - (k << bp.chunk_lg);
    } else {
      sl.fill[tid] = t < CH ? t : CH;
    }
    sl.hist[tid] = 0;
  }
  if (tid == 0) *sl.cnt = 0;
  __syncthreads();
}

// The general fact pass over rows [begin, end), adding into a group table
// (AGG 1) or writing (group key, value) pairs (AGG 2), one or two joins, rows
// probed where they are (the one-join slot sums and the two-join pairs have
// the faster star_range and chain_range).  Wave w of the block takes the 256
// rows at begin + 256*w, then steps by `step` rows.  The next step's columns
// are loaded while the current step's probes are in flight.  s_bloom is the
// block's LDS copy of join 0's filter (used when use_bloom).
// VX: the value may be v0 * (c - v1) (the plan says which at run time); without
// it the value is the column v0 and the v1 column is never read.
template <int NJ, int SB1, int AGG, bool V64, bool VX, int R = 4>
__device__ __forceinline__ void fact_range(const FastArgs &a, const TableDev &t0, const TableDev &t1, const GroupDev &g,
                                           const PairsOut &po, uint32_t *err, const PYST_LDS uint32_t *s_bloom,
                                           bool use_bloom, int64_t begin, int64_t step, int64_t end) {
  static_assert(AGG == 1 || AGG == 2, "sums into the join table go through star_range");
  constexpr int64_t WR = int64_t{kWave} * R;  // rows of one wave step: R consecutive rows per lane
  const int64_t cap0 = t0.hdr[0], mask0 = cap0 - 1;
  const int bshift = bloom_shift(cap0);
  const int64_t cap1 = NJ > 1 ? t1.hdr[0] : 4, mask1 = cap1 - 1;
  const int64_t gmask = AGG == 1 ? g.hdr[0] - 1 : 0;
  const __amdgpu_buffer_rsrc_t r0 = rsrc(t0.slots, cap0 * 4);
  const __amdgpu_buffer_rsrc_t r1 = rsrc(NJ > 1 ? t1.slots : t0.slots, cap1 * SB1);
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  int64_t wpos = 0, wend = 0;  // the wave's pair run (AGG 2), wave-uniform
  int64_t wbase = begin + int64_t{wv} * WR;
  FactRows<R> cur = load_rows<NJ, R>(a, wbase, end, lane);
  // Stand-ins for the stores that end every step, into an empty buffer (no
  // memory access), so that the loop is entered with as many operations younger
  // than `cur` as it repeats with.  Distinct per-lane offsets keep the compiler
  // from merging them.
  if (AGG == 2) {
    const __amdgpu_buffer_rsrc_t none = rsrc(nullptr, 0);
#pragma unroll
    for (int r = 0; r < 2 * R; ++r) __builtin_amdgcn_raw_buffer_store_b64(v2u32{0, 0}, none, lane * 128 + r * 8, 0, 0);
  }
  for (; wbase < end; wbase += step) {
    const int64_t left64 = end - wbase;
    const int left = static_cast<int>(left64 < WR ? left64 : WR);
    bool live[R];
    int32_t s0[R];
    v4i32 q0[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bool l = lane * R + r < left && in_range(row_of(cur.c0, r), a.plo[0], a.pspan[0], a.pneg[0]) &&
               in_range(row_of(cur.c1, r), a.plo[1], a.pspan[1], a.pneg[1]);
      const uint32_t h = table_hash32(row_of(cur.f0, r));
      if (use_bloom) {
        const uint32_t m = bloom_bits(h);
        l = l && (s_bloom[bloom_word(h, mask0, bshift)] & m) == m;
      }
      live[r] = l;
      s0[r] = static_cast<int32_t>((h & mask0) & ~int64_t{3});
      q0[r] = __builtin_amdgcn_raw_buffer_load_b128(r0, l ? s0[r] * 4 : kBufOob, 0, 0);
    }
    // the value columns of live rows only
    const __amdgpu_buffer_rsrc_t rv = window(a.v0, V64 ? 8 : 4, wbase, end, WR);
    const __amdgpu_buffer_rsrc_t rw = window(a.v1, 4, wbase, end, WR);
    int64_t x0[R];
    int32_t w1[R] = {};
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int row = lane * R + r;
      if (V64) {
        const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(rv, live[r] ? row * 8 : kBufOob, 0, 0);
        x0[r] = static_cast<int64_t>((uint64_t{v.y} << 32) | v.x);
      } else {
        x0[r] = static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rv, live[r] ? row * 4 : kBufOob, 0, 0));
      }
    }
    if (VX)  // an empty resource when the plan's value is a plain column
#pragma unroll
      for (int r = 0; r < R; ++r)
        w1[r] = static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rw, live[r] ? (lane * R + r) * 4 : kBufOob, 0, 0));
    const FactRows<R> nxt = load_rows<NJ, R>(a, wbase + step, end, lane);
    int32_t slot0[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bool empty;
      const int32_t k = row_of(cur.f0, r);
      const int hit = match4(q0[r], k, &empty);
      slot0[r] = live[r] && hit >= 0 ? s0[r] + hit : -1;
      if (live[r] && hit < 0 && !empty) {  // the run continues past the first group (rare)
        int32_t s = s0[r];
        for (int64_t st = 4; st <= mask0; st += 4) {
          s = static_cast<int32_t>((s + 4) & mask0);
          const int h2 = match4(__builtin_amdgcn_raw_buffer_load_b128(r0, s * 4, 0, 0), k, &empty);
          if (h2 >= 0) {
            slot0[r] = s + h2;
            break;
          }
          if (empty) break;
        }
      }
    }
    int32_t pay1[R] = {};
    if (NJ > 1) {
      int32_t s1[R];
      v4i32 q1[R];
      constexpr int GS = 16 / SB1;  // slots per 16-byte load
#pragma unroll
      for (int r = 0; r < R; ++r) {
        s1[r] = static_cast<int32_t>((table_hash32(row_of(cur.f1, r)) & mask1) & ~int64_t{GS - 1});
        q1[r] = __builtin_amdgcn_raw_buffer_load_b128(r1, slot0[r] >= 0 ? s1[r] * SB1 : kBufOob, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int32_t k = row_of(cur.f1, r);
        // state of the probe after one 16-byte group: 1 found, 0 absent, -1 continue
        int state;
        int32_t pl = 0;
        if (SB1 == 4) {
          bool empty;
          const int h = match4(q1[r], k, &empty);
          state = h >= 0 ? 1 : (empty ? 0 : -1);
        } else {
          const v4i32 q = q1[r];
          state = q.x == k ? 1 : q.x == kEmpty32 ? 0 : q.z == k ? 2 : q.z == kEmpty32 ? 0 : -1;
          pl = state == 1 ? q.y : q.w;
          state = state == 2 ? 1 : state;
        }
        if (slot0[r] >= 0 && state < 0) {  // the run continues past the first group (rare)
          int32_t s = s1[r];
          state = 0;
          for (int64_t st = GS; st <= mask1; st += GS) {
            s = static_cast<int32_t>((s + GS) & mask1);
            const v4i32 q = __builtin_amdgcn_raw_buffer_load_b128(r1, s * SB1, 0, 0);
            int sx;
            if (SB1 == 4) {
              bool empty;
              const int h = match4(q, k, &empty);
              sx = h >= 0 ? 1 : (empty ? 0 : -1);
            } else {
              sx = q.x == k ? 1 : q.x == kEmpty32 ? 0 : q.z == k ? 2 : q.z == kEmpty32 ? 0 : -1;
              pl = sx == 1 ? q.y : q.w;
              sx = sx == 2 ? 1 : sx;
            }
            if (sx >= 0) {
              state = sx;
              break;
            }
          }
        }
        if (state != 1) slot0[r] = -1;
        pay1[r] = pl;
      }
    }
    int64_t val[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
      val[r] = !VX || a.vexpr == PYST_V_COL ? x0[r]
                                     : static_cast<int64_t>(static_cast<uint64_t>(x0[r]) *
                                                            static_cast<uint64_t>(a.vconst - static_cast<int64_t>(w1[r])));
    {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool hit = slot0[r] >= 0;
        const int64_t lo = a.lo_src == PYST_G_JOIN_KEY ? (a.lo_idx == 0 ? row_of(cur.f0, r) : row_of(cur.f1, r)) : pay1[r];
        const int64_t hi = a.hi_src == PYST_G_JOIN_KEY ? (a.hi_idx == 0 ? row_of(cur.f0, r) : row_of(cur.f1, r)) : pay1[r];
        const int64_t gkey = a.hi_src == PYST_G_NONE
                                 ? lo
                                 : static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | static_cast<uint32_t>(lo));
        if (hit && gkey == kEmpty64) latch(err, kErrKey);
        if (AGG == 1) {
          if (hit && gkey != kEmpty64 && !group_add(g.slots, gmask, gkey, static_cast<uint64_t>(val[r])))
            latch(err, kErrTableFull);
        } else {
          // Pairs go to the wave's current run of kPairRun slots; a new run is
          // reserved with one atomic when it fills (a counter bumped by every
          // wave for every group of rows serializes the whole pass).
          const uint64_t m = __ballot(hit);
          const int c = __popcll(m);
          if (c > 0 && wpos + c > wend) {  // wave-uniform, once per kPairRun pairs
            for (int64_t p = wpos + lane; p < wend; p += kWave)
              if (p < po.cap) po.keys[p] = kEmpty64;
            unsigned long long rb = 0;
            if (lane == 0)
              rb = atomicAdd(reinterpret_cast<unsigned long long *>(po.count), static_cast<unsigned long long>(kPairRun));
            wpos = uniform64(static_cast<int64_t>(__shfl(rb, 0)));
            wend = wpos + kPairRun;
          }
          // the 64 pair slots from wpos, clipped to the buffer
          int64_t room = po.cap - wpos;
          room = room < 0 ? 0 : room > kWave ? kWave : room;
          const __amdgpu_buffer_rsrc_t rk = rsrc(po.keys + wpos, room * 8);
          const __amdgpu_buffer_rsrc_t rvv = rsrc(po.vals + wpos, room * 8);
          const int off = hit ? static_cast<int>(mbcnt(m)) * 8 : kBufOob;
          __builtin_amdgcn_raw_buffer_store_b64(split64(gkey), rk, off, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b64(split64(val[r]), rvv, off, 0, 0);
          wpos += c;
        }
      }
    }
    cur = nxt;
  }
  if (AGG == 2)
    for (int64_t p = wpos + lane; p < wend; p += kWave)
      if (p < po.cap) po.keys[p] = kEmpty64;
}

// Pushes the live rows of a wave step to consecutive lanes: the row with
// compact index j (rows taken r-major: every lane's row 0, then row 1, ...)
// lands in lane j - w0.  m[r]: the lanes whose row r is live; b[r]: the compact
// index of the first of them.  The other lanes are pushed to the remaining
// lanes, so each push is a permutation.  Gives this lane's compact row: its NV
// values v[.][r] and its row within the step (lane * R + r).
template <int R, int NV>
__device__ __forceinline__ void compact_rows(const uint64_t (&m)[R], const uint32_t (&b)[R],
                                             const int32_t (&v)[NV][R], int lane, uint32_t w0, int32_t (&out)[NV],
                                             int32_t *crow) {
  int32_t pv[NV][R], lv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t below = mbcnt(m[r]);
    const uint32_t c = static_cast<uint32_t>(__popcll(m[r]));
    const uint32_t pos = (m[r] >> lane) & 1 ? below : c + (static_cast<uint32_t>(lane) - below);
    const int dst = static_cast<int>((pos + b[r] - w0) & (kWave - 1));
#pragma unroll
    for (int i = 0; i < NV; ++i) pv[i][r] = __builtin_amdgcn_ds_permute(dst << 2, v[i][r]);
    lv[r] = __builtin_amdgcn_ds_permute(dst << 2, lane);
  }
  const uint32_t j = w0 + static_cast<uint32_t>(lane);
  int32_t src = lv[0], rr = 0;
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = pv[i][0];
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const bool mine = j >= b[r];
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = mine ? pv[i][r] : out[i];
    src = mine ? lv[r] : src;
    rr = mine ? r : rr;
  }
  *crow = src * R + rr;
}

// Walks the run of full groups after group `s` for key k, reading at most
// `groups` more groups; the slot of k, or -1.
__device__ __forceinline__ int32_t walk_run(__amdgpu_buffer_rsrc_t r0, int32_t mask, int32_t s, int32_t groups,
                                            int32_t k) {
  for (; groups > 0; --groups) {
    s = (s + 4) & mask;
    bool empty;
    const int h = match4(__builtin_amdgcn_raw_buffer_load_b128(r0, s * 4, 0, 0), k, &empty);
    if (h >= 0) return s + h;
    if (empty) return -1;
  }
  return -1;
}

// Steps until the next staging check: c pairs are staged, cprev were at the
// last check `since` steps ago; after a flush the whole area is free.
__device__ __forceinline__ uint32_t next_check(uint32_t c, uint32_t cprev, uint32_t since, bool flush) {
  const uint32_t rate = (c - cprev) / since;
  const uint32_t per = rate + rate / 8 + 1;
  const uint32_t room = flush ? kStageCap : c < kStageCap ? kStageCap - c : 0;
  const uint32_t fit = room / per;
  return fit < 1 ? 1 : fit > kCheckMax ? kCheckMax : fit;
}

// The one-join fact pass (star query) over rows [begin, end), summing into the
// join table's slots: AGG 0 adds with buffer atomics plus a group-exists flag,
// AGG 3 stages (slot, value) pairs in LDS and moves them to the bucket pool.
//
// Each wave takes R rows per lane per step.  After the predicates and the
// Bloom filter only a fifth of the rows are live, so they are first pushed
// together (compact_rows): one 16-byte probe, one value load, one match and
// one staging step per lane then serve 64 live rows, where per-row probing
// repeats each of them R times, mostly for dead lanes.  A key not settled by
// its first 16-byte group is
// carried to the next step, whose probes load its next group (no round trip of
// its own); one carried key per lane, another one walks its run at once.
template <int AGG, bool V64, bool VX, int R>
__device__ __forceinline__ void star_range(const FastArgs &a, const TableDev &t0, uint32_t *err,
                                           const PYST_LDS uint32_t *s_bloom, bool use_bloom, int64_t begin,
                                           int64_t step, int64_t end, const BucketPool *bp, const StageLds *sl) {
  static_assert(AGG == 0 || AGG == 3, "star_range sums into the join table");
  constexpr int64_t WR = int64_t{kWave} * R;
  const int64_t cap0 = t0.hdr[0];
  const int32_t mask0 = static_cast<int32_t>(cap0 - 1);
  const int32_t groups0 = static_cast<int32_t>(cap0 >> 2);  // 16-byte groups in the table
  const int bshift = bloom_shift(cap0);
  const __amdgpu_buffer_rsrc_t r0 = rsrc(t0.slots, cap0 * 4);
  const __amdgpu_buffer_rsrc_t rsum = rsrc(AGG == 0 ? t0.sums : nullptr, AGG == 0 ? cap0 * 8 : 0);
  const __amdgpu_buffer_rsrc_t rflag = rsrc(AGG == 0 ? t0.flags : nullptr, AGG == 0 ? cap0 : 0);
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  int64_t wbase = begin + int64_t{wv} * WR;
  bool pend = false;  // the carried key of this lane
  int32_t pkey = 0, ppos = 0, pleft = 0;  // key, its next group, groups it may still read
  int64_t pval = 0;
  FactRows<R> cur = load_rows<1, R>(a, wbase, end, lane);
  if (AGG == 0) {
    // Stand-ins for the adds that end every step, into an empty buffer (no
    // memory access), so that the loop is entered with as many operations
    // younger than `cur` as it repeats with.  Distinct per-lane offsets keep
    // the compiler from merging them.
    const __amdgpu_buffer_rsrc_t none = rsrc(nullptr, 0);
#pragma unroll
    for (int e = 0; e < 2; ++e) pyst_buffer_atomic_add_i64(0, none, lane * 128 + e * 8, 0, 0);
#pragma unroll
    for (int e = 0; e < 2; ++e)
      __builtin_amdgcn_raw_buffer_store_b8(static_cast<uint8_t>(1), none, lane * 128 + 64 + e, 0, 0);
  }
  const uint32_t nb = AGG == 3 ? bucket_count(cap0) : 0;
  const uint32_t stage_cap = AGG == 3 && nb <= bp->stride ? kStageCap : 0;  // 0: every pair is added directly
  // Adds this lane's entries (slot -1: none): AGG 0 adds in place, AGG 3 stages.
  auto add = [&](const int32_t (&es)[2], const int64_t (&ev)[2]) {
    if (AGG == 0) {
#pragma unroll
      for (int e = 0; e < 2; ++e) pyst_buffer_atomic_add_i64(ev[e], rsum, es[e] >= 0 ? es[e] * 8 : kBufOob, 0, 0);
#pragma unroll
      for (int e = 0; e < 2; ++e)
        __builtin_amdgcn_raw_buffer_store_b8(static_cast<uint8_t>(1), rflag, es[e] >= 0 ? es[e] : kBufOob, 0, 0);
    } else {
      uint64_t m[2];
      bool st[2];  // staged, else added directly
      uint32_t cw = 0;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        st[e] = es[e] >= 0 && fits_stage(ev[e]);
        m[e] = __ballot(st[e]);
        cw += static_cast<uint32_t>(__popcll(m[e]));
      }
      uint32_t off = 0;
      if (cw) {  // wave-uniform
        if (lane == 0) off = lds_add(sl->cnt, cw);
        off = __builtin_amdgcn_readfirstlane(off);
      }
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        if (es[e] >= 0) {
          const uint32_t p = st[e] ? off + mbcnt(m[e]) : stage_cap;
          if (p < stage_cap) {
            sl->ent[p] = (static_cast<uint64_t>(ev[e]) << kStageSlotBits) | static_cast<uint32_t>(es[e]);
          } else {  // staging full: add directly (the second kernel adds these in)
            atomicAdd(reinterpret_cast<unsigned long long *>(&t0.sums[es[e]]), static_cast<unsigned long long>(ev[e]));
            t0.flags[es[e]] = 1;
            mark_added(t0, es[e]);
          }
        }
        off += static_cast<uint32_t>(__popcll(m[e]));
      }
    }
  };
  auto value = [&](int64_t x, int32_t w) -> int64_t {
    return !VX || a.vexpr == PYST_V_COL
               ? x
               : static_cast<int64_t>(static_cast<uint64_t>(x) * static_cast<uint64_t>(a.vconst - static_cast<int64_t>(w)));
  };
  uint32_t since = 0, every = 2;  // steps since the last staging check; steps between checks
  uint32_t cprev = 0;              // staged pairs at the last check (0 after a flush)
  // AGG 3 steps the whole block together (it meets at a barrier every
  // `every` steps); otherwise each wave runs on its own.
  for (; (AGG == 3 ? wbase - int64_t{wv} * WR : wbase) < end; wbase += step) {
    const int64_t left64 = end - wbase;
    const int left = static_cast<int>(left64 < WR ? left64 : WR);
    uint64_t m[R];
    uint32_t b[R], n = 0;
    int32_t key[1][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bool l = lane * R + r < left && in_range(row_of(cur.c0, r), a.plo[0], a.pspan[0], a.pneg[0]) &&
               in_range(row_of(cur.c1, r), a.plo[1], a.pspan[1], a.pneg[1]);
      key[0][r] = row_of(cur.f0, r);
      if (use_bloom) {
        const uint32_t h = table_hash32(key[0][r]);
        const uint32_t bits = bloom_bits(h);
        l = l && (s_bloom[bloom_word(h, cap0 - 1, bshift)] & bits) == bits;
      }
      m[r] = __ballot(l);
      b[r] = n;
      n += static_cast<uint32_t>(__popcll(m[r]));
    }
    n = __builtin_amdgcn_readfirstlane(n);
    const __amdgpu_buffer_rsrc_t rv = window(a.v0, V64 ? 8 : 4, wbase, end, WR);
    const __amdgpu_buffer_rsrc_t rw = window(VX ? a.v1 : nullptr, 4, wbase, end, WR);
    // the first 64 live rows, the carried keys, then the next step's columns
    int32_t ck, crow;
    {
      int32_t o[1];
      compact_rows<R, 1>(m, b, key, lane, 0, o, &crow);
      ck = o[0];
    }
    bool ok = static_cast<uint32_t>(lane) < n;
    int32_t cs = static_cast<int32_t>(table_hash32(ck)) & mask0 & ~3;
    const v4i32 q = __builtin_amdgcn_raw_buffer_load_b128(r0, ok ? cs * 4 : kBufOob, 0, 0);
    const v4i32 qp = __builtin_amdgcn_raw_buffer_load_b128(r0, pend ? ppos * 4 : kBufOob, 0, 0);
    int64_t x;
    if (V64) {
      const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(rv, ok ? crow * 8 : kBufOob, 0, kNonTemporal);
      x = static_cast<int64_t>((uint64_t{v.y} << 32) | v.x);
    } else {
      x = static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rv, ok ? crow * 4 : kBufOob, 0, 0));
    }
    const int32_t w = VX ? static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rw, ok ? crow * 4 : kBufOob, 0, 0)) : 0;
    const FactRows<R> nxt = load_rows<1, R>(a, wbase + step, end, lane);
    bool npend = false, nold = false;  // a key carried to the next step; it is the carried key again
    int32_t nkey = 0, npos = 0, nleft = 0;
    int32_t es[2] = {-1, -1};
    {
      bool empty;
      const int h = match4(q, ck, &empty);
      es[0] = ok && h >= 0 ? cs + h : -1;
      if (ok && h < 0 && !empty && groups0 > 1) {
        npend = true;
        nkey = ck;
        npos = (cs + 4) & mask0;
        nleft = groups0 - 1;
      }
    }
    if (pend) {
      bool empty;
      const int h = match4(qp, pkey, &empty);
      if (h >= 0) {
        es[1] = ppos + h;
      } else if (!empty && pleft > 1) {
        if (!npend) {
          npend = nold = true;
          nkey = pkey;
          npos = (ppos + 4) & mask0;
          nleft = pleft - 1;
        } else {
          es[1] = walk_run(r0, mask0, ppos, pleft - 1, pkey);
        }
      }
    }
    const int64_t v0 = value(x, w);
    add(es, {v0, pval});
    pval = nold ? pval : v0;
    pend = npend;
    pkey = nkey;
    ppos = npos;
    pleft = nleft;
    // more than 64 live rows (rare at R = 4)
    for (uint32_t w0 = kWave; w0 < n; w0 += kWave) {  // wave-uniform
      {
        int32_t o[1];
        compact_rows<R, 1>(m, b, key, lane, w0, o, &crow);
        ck = o[0];
      }
      ok = w0 + static_cast<uint32_t>(lane) < n;
      cs = static_cast<int32_t>(table_hash32(ck)) & mask0 & ~3;
      const v4i32 q2 = __builtin_amdgcn_raw_buffer_load_b128(r0, ok ? cs * 4 : kBufOob, 0, 0);
      int64_t x2;
      if (V64) {
        const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(rv, ok ? crow * 8 : kBufOob, 0, 0);
        x2 = static_cast<int64_t>((uint64_t{v.y} << 32) | v.x);
      } else {
        x2 = static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rv, ok ? crow * 4 : kBufOob, 0, 0));
      }
      const int32_t w2 =
          VX ? static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rw, ok ? crow * 4 : kBufOob, 0, 0)) : 0;
      bool empty;
      const int h = match4(q2, ck, &empty);
      int32_t s2[2] = {ok && h >= 0 ? cs + h : -1, -1};
      const int64_t v2 = value(x2, w2);
      if (ok && h < 0 && !empty && groups0 > 1) {
        if (!pend) {
          pend = true;
          pkey = ck;
          ppos = (cs + 4) & mask0;
          pleft = groups0 - 1;
          pval = v2;
        } else {
          s2[0] = walk_run(r0, mask0, cs, groups0 - 1, ck);
        }
      }
      add(s2, {v2, 0});
    }
    // Every `every` steps the block meets and moves its staged pairs to HBM
    // once there are kFlushAt of them (pairs past kStageCap in between were
    // added directly).  The next interval is the number of steps whose pairs,
    // at the rate of the last interval plus an eighth, fit in the room the
    // staging area has left (all threads read the same count after the
    // barrier, so it stays block-uniform).
    if (AGG == 3 && stage_cap > 0 && ++since == every) {  // block-uniform
      __syncthreads();
      const uint32_t c = *sl->cnt;
      const bool flush = c >= kFlushAt;
      every = next_check(c, cprev, since, flush);
      since = 0;
      cprev = flush ? 0 : c;
      if (flush) stage_flush(*sl, *bp, t0, nb);
    }
    cur = nxt;
  }
  if (pend) {  // the key still carried walks the rest of its run and is added directly
    const int32_t s = walk_run(r0, mask0, (ppos - 4) & mask0, pleft, pkey);
    if (s >= 0) {
      atomicAdd(reinterpret_cast<unsigned long long *>(&t0.sums[s]), static_cast<unsigned long long>(pval));
      t0.flags[s] = 1;
      if (AGG == 3) mark_added(t0, s);  // (AGG 0's table may have more buckets than the header has bytes)
    }
  }
  if (AGG == 3 && stage_cap > 0) {
    __syncthreads();
    if (*sl->cnt > 0) stage_flush(*sl, *bp, t0, nb);  // block-uniform
    if (threadIdx.x < nb) bp->fill[sl->chunk[threadIdx.x]] = sl->fill[threadIdx.x];
  }
}

// star_range over a direct-addressed table (staged sums only).  Row r of a
// lane is live when it passes the predicates and key - kmin falls in the range
// with its filter bit set; the live rows are pushed together as in star_range,
// and when the filter is not exact each reads its one bitmap word (an L2 hit:
// the bitmap of 2^21 keys is 256 KiB).  A live row's slot is key - kmin, so
// nothing walks.  The loads of a step's live rows (value, bitmap word) are
// consumed one step later: the step issues them, then the next step's column
// loads, then stages the previous step's rows, whose loads have long
// completed, so no step waits a memory round trip of its own.
template <bool V64, bool VX, int R>
__device__ __forceinline__ void star_direct(const FastArgs &a, const TableDev &t0, const PYST_LDS uint32_t *s_filt,
                                            int64_t begin, int64_t step, int64_t end, const BucketPool *bp,
                                            const StageLds *sl) {
  constexpr int64_t WR = int64_t{kWave} * R;
  const uint32_t kmin = static_cast<uint32_t>(t0.hdr[kHdrKmin]);
  const uint32_t range = static_cast<uint32_t>(t0.hdr[kHdrRange]);
  const int fshift = range > kFilterBits ? 1 : 0;
  const __amdgpu_buffer_rsrc_t rbm = rsrc(t0.slots, fshift ? (int64_t{range} + 31) / 32 * 4 : 0);
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  int64_t wbase = begin + int64_t{wv} * WR;
  FactRows<R> cur = load_rows<1, R>(a, wbase, end, lane);
  const uint32_t nb = bucket_count(t0.hdr[0]);
  const uint32_t stage_cap = nb <= bp->stride ? kStageCap : 0;  // 0: every pair is added directly
  // Stages this lane's pair (slot < 0: none), or adds it directly when it does not fit a staged word.
  auto add = [&](int32_t es, int64_t ev) {
    const bool st = es >= 0 && fits_stage(ev);
    const uint64_t m = __ballot(st);
    const uint32_t cw = static_cast<uint32_t>(__popcll(m));
    uint32_t off = 0;
    if (cw) {  // wave-uniform
      if (lane == 0) off = lds_add(sl->cnt, cw);
      off = __builtin_amdgcn_readfirstlane(off);
    }
    if (es >= 0) {
      const uint32_t p = st ? off + mbcnt(m) : stage_cap;
      if (p < stage_cap) {
        sl->ent[p] = (static_cast<uint64_t>(ev) << kStageSlotBits) | static_cast<uint32_t>(es);
      } else {  // staging full: add directly (the second kernel adds these in)
        atomicAdd(reinterpret_cast<unsigned long long *>(&t0.sums[es]), static_cast<unsigned long long>(ev));
        t0.flags[es] = 1;
        mark_added(t0, es);
      }
    }
  };
  auto value = [&](int64_t x, int32_t w) -> int64_t {
    return !VX || a.vexpr == PYST_V_COL
               ? x
               : static_cast<int64_t>(static_cast<uint64_t>(x) * static_cast<uint64_t>(a.vconst - static_cast<int64_t>(w)));
  };
  // the compacted row of lane `lane` in pass w0: its slot if it is a member, else -1
  auto probe = [&](int32_t d, bool ok, __amdgpu_buffer_rsrc_t rv, __amdgpu_buffer_rsrc_t rw, int32_t crow,
                   int64_t *x, int32_t *w) -> int32_t {
    const uint32_t bw = fshift ? __builtin_amdgcn_raw_buffer_load_b32(rbm, ok ? (d >> 5) * 4 : kBufOob, 0, 0) : 1u;
    if (V64) {
      const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(rv, ok ? crow * 8 : kBufOob, 0, kNonTemporal);
      *x = static_cast<int64_t>((uint64_t{v.y} << 32) | v.x);
    } else {
      *x = static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rv, ok ? crow * 4 : kBufOob, 0, 0));
    }
    *w = VX ? static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rw, ok ? crow * 4 : kBufOob, 0, 0)) : 0;
    const bool hit = ok && (fshift == 0 || ((bw >> (d & 31)) & 1u));
    return hit ? d : -1;
  };
  uint32_t since = 0, every = 2;  // steps since the last staging check; steps between checks
  uint32_t cprev = 0;              // staged pairs at the last check (0 after a flush)
  uint32_t lag = 1;                // the first interval's first step staged nothing (pairs go in a step late)
  // the previous step's first 64 live rows: slot, bitmap word, value, whether the lane holds one
  int32_t pd = 0;
  uint32_t pbw = 0;
  int64_t px = 0;
  int32_t pw = 0;
  bool pok = false;
  for (; wbase - int64_t{wv} * WR < end; wbase += step) {  // the whole block steps together
    const int64_t left64 = end - wbase;
    const int left = static_cast<int>(left64 < WR ? left64 : WR);
    uint64_t m[R];
    uint32_t b[R], n = 0;
    int32_t dk[1][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t d = static_cast<uint32_t>(row_of(cur.f0, r)) - kmin;
      const uint32_t fb = d >> fshift;
      const bool l = lane * R + r < left && in_range(row_of(cur.c0, r), a.plo[0], a.pspan[0], a.pneg[0]) &&
                     in_range(row_of(cur.c1, r), a.plo[1], a.pspan[1], a.pneg[1]) && d < range &&
                     ((s_filt[(fb >> 5) & (kBloomWords - 1)] >> (fb & 31)) & 1u);
      dk[0][r] = static_cast<int32_t>(d);
      m[r] = __ballot(l);
      b[r] = n;
      n += static_cast<uint32_t>(__popcll(m[r]));
    }
    n = __builtin_amdgcn_readfirstlane(n);
    const __amdgpu_buffer_rsrc_t rv = window(a.v0, V64 ? 8 : 4, wbase, end, WR);
    const __amdgpu_buffer_rsrc_t rw = window(VX ? a.v1 : nullptr, 4, wbase, end, WR);
    // the first 64 live rows, then the next step's columns
    int32_t cd, crow;
    {
      int32_t o[1];
      compact_rows<R, 1>(m, b, dk, lane, 0, o, &crow);
      cd = o[0];
    }
    const bool ok = static_cast<uint32_t>(lane) < n;
    const uint32_t bw = fshift ? __builtin_amdgcn_raw_buffer_load_b32(rbm, ok ? (cd >> 5) * 4 : kBufOob, 0, 0) : 1u;
    int64_t x;
    if (V64) {
      const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(rv, ok ? crow * 8 : kBufOob, 0, kNonTemporal);
      x = static_cast<int64_t>((uint64_t{v.y} << 32) | v.x);
    } else {
      x = static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rv, ok ? crow * 4 : kBufOob, 0, 0));
    }
    const int32_t w = VX ? static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rw, ok ? crow * 4 : kBufOob, 0, 0)) : 0;
    const FactRows<R> nxt = load_rows<1, R>(a, wbase + step, end, lane);
    add(pok && (fshift == 0 || ((pbw >> (pd & 31)) & 1u)) ? pd : -1, value(px, pw));
    pd = cd;
    pbw = bw;
    px = x;
    pw = w;
    pok = ok;
    for (uint32_t w0 = kWave; w0 < n; w0 += kWave) {  // more than 64 live rows (wave-uniform, rare)
      {
        int32_t o[1];
        compact_rows<R, 1>(m, b, dk, lane, w0, o, &crow);
        cd = o[0];
      }
      int64_t x2;
      int32_t w2;
      const int32_t es2 = probe(cd, w0 + static_cast<uint32_t>(lane) < n, rv, rw, crow, &x2, &w2);
      add(es2, value(x2, w2));
    }
    if (stage_cap > 0 && ++since == every) {  // block-uniform: as in star_range
      __syncthreads();
      const uint32_t c = *sl->cnt;
      const bool flush = c >= kFlushAt;
      every = next_check(c, cprev, since - lag, flush);
      lag = 0;
      since = 0;
      cprev = flush ? 0 : c;
      if (flush) stage_flush(*sl, *bp, t0, nb);
    }
    cur = nxt;
  }
  add(pok && (fshift == 0 || ((pbw >> (pd & 31)) & 1u)) ? pd : -1, value(px, pw));  // the last step's rows
  if (stage_cap > 0) {
    __syncthreads();
    if (*sl->cnt > 0) stage_flush(*sl, *bp, t0, nb);  // block-uniform
    if (threadIdx.x < nb) bp->fill[sl->chunk[threadIdx.x]] = sl->fill[threadIdx.x];
  }
}

// The two-join fact pass writing (group key, value) pairs (the chain query).
// Rows that pass the predicates and join 0's Bloom filter are pushed to
// consecutive lanes (compact_rows), probe join 0 and, when found there, join 1.
// A probe not settled by its first 16-byte group reads the next group of every
// such lane of the wave at once: one round trip per group for the whole wave,
// where per-row probes would wait once per row.  Pairs go to the wave's current
// run of kPairRun slots; a new run is reserved with one atomic when it fills
// (a counter bumped by every wave for every group of rows serializes the pass).
template <int SB1, bool V64, bool VX, int R>
__device__ __forceinline__ void chain_range(const FastArgs &a, const TableDev &t0, const TableDev &t1,
                                            const PairsOut &po, uint32_t *err, const PYST_LDS uint32_t *s_bloom,
                                            bool use_bloom, int64_t begin, int64_t step, int64_t end) {
  constexpr int64_t WR = int64_t{kWave} * R;
  constexpr int GS = 16 / SB1;  // join 1 slots per 16-byte load
  constexpr int NW = R / 4;     // windows of 64 live rows a step provides for (about a fifth of its rows live)
  const int64_t cap0 = t0.hdr[0], cap1 = t1.hdr[0];
  const int32_t mask0 = static_cast<int32_t>(cap0 - 1), mask1 = static_cast<int32_t>(cap1 - 1);
  const int32_t groups0 = static_cast<int32_t>(cap0 / 4), groups1 = static_cast<int32_t>(cap1 / GS);
  const int bshift = bloom_shift(cap0);
  const __amdgpu_buffer_rsrc_t r0 = rsrc(t0.slots, cap0 * 4);
  const __amdgpu_buffer_rsrc_t r1 = rsrc(t1.slots, cap1 * SB1);
  // Direct-addressed joins (uniform): join 0's LDS filter is then its exact
  // bitmap (range <= kFilterBits), so a live row is found and join 0's table
  // is never read; join 1 (8-byte slots) keeps key k in slot k - kmin1, one
  // 16-byte load and no walk.
  const bool dir0 = t0.hdr[kHdrDirect] != 0, dir1 = SB1 == 8 && t1.hdr[kHdrDirect] != 0;
  const uint32_t kmin0 = static_cast<uint32_t>(t0.hdr[kHdrKmin]), range0 = static_cast<uint32_t>(t0.hdr[kHdrRange]);
  const uint32_t kmin1 = static_cast<uint32_t>(t1.hdr[kHdrKmin]), range1 = static_cast<uint32_t>(t1.hdr[kHdrRange]);
  const int lane = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  int64_t wpos = 0, wend = 0;  // the wave's pair run, wave-uniform
  int64_t wbase = begin + int64_t{wv} * WR;
  FactRows<R> cur = load_rows<2, R>(a, wbase, end, lane);
  v4i32 stand_in[NW];
  {
    // Stand-ins for join 1's probe and the two pair stores that end every
    // step, on an empty buffer (no memory access), so that the loop is entered
    // with as many operations younger than `cur` as it repeats with.
    const __amdgpu_buffer_rsrc_t none = rsrc(nullptr, 0);
#pragma unroll
    for (int k = 0; k < NW; ++k) stand_in[k] = __builtin_amdgcn_raw_buffer_load_b128(none, lane * 128 + 64 + 16 * k, 0, 0);
#pragma unroll
    for (int e = 0; e < 2 * NW; ++e)
      __builtin_amdgcn_raw_buffer_store_b64(v2u32{0, 0}, none, lane * 128 + e * 8, 0, 0);
  }
  // join 1 after one 16-byte group: 1 found (payload in *pl), 0 absent, -1 the run goes on
  auto probe1 = [&](v4i32 q, int32_t k, int32_t *pl) -> int {
    if (SB1 == 4) {
      bool empty;
      const int h = match4(q, k, &empty);
      *pl = 0;
      return h >= 0 ? 1 : empty ? 0 : -1;
    }
    const int st = q.x == k ? 1 : q.x == kEmpty32 ? 0 : q.z == k ? 2 : q.z == kEmpty32 ? 0 : -1;
    *pl = st == 1 ? q.y : q.w;
    return st == 2 ? 1 : st;
  };
  struct Win {
    int32_t k0, k1, crow, s0;
    bool ok;
    v4i32 q0;
    int64_t x;
    int32_t w;
  };
  // compact window w0 of the live rows and load its first group of join 0 and its values
  auto issue = [&](const uint64_t (&m)[R], const uint32_t (&b)[R], const int32_t (&kv)[2][R], uint32_t w0,
                   uint32_t n, __amdgpu_buffer_rsrc_t rv, __amdgpu_buffer_rsrc_t rw) -> Win {
    Win W;
    int32_t o[2];
    compact_rows<R, 2>(m, b, kv, lane, w0, o, &W.crow);
    W.k0 = o[0];
    W.k1 = o[1];
    W.ok = w0 + static_cast<uint32_t>(lane) < n;
    W.s0 = static_cast<int32_t>(table_hash32(W.k0)) & mask0 & ~3;
    W.q0 = __builtin_amdgcn_raw_buffer_load_b128(r0, W.ok && !dir0 ? W.s0 * 4 : kBufOob, 0, 0);
    if (V64) {
      const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(rv, W.ok ? W.crow * 8 : kBufOob, 0, kNonTemporal);
      W.x = static_cast<int64_t>((uint64_t{v.y} << 32) | v.x);
    } else {
      W.x = static_cast<int32_t>(__builtin_amdgcn_raw_buffer_load_b32(rv, W.ok ? W.crow * 4 : kBufOob, 0, kNonTemporal));
    }
    W.w = VX ? static_cast<int32_t>(
                   __builtin_amdgcn_raw_buffer_load_b32(rw, W.ok ? W.crow * 4 : kBufOob, 0, kNonTemporal))
             : 0;
    return W;
  };
  // The pairs of one window: hit, the payload of join 1 in pl.
  auto emit = [&](const Win &W, bool hit, int32_t pl) {
    const int64_t lo = a.lo_src == PYST_G_JOIN_KEY ? (a.lo_idx == 0 ? W.k0 : W.k1) : pl;
    const int64_t hi = a.hi_src == PYST_G_JOIN_KEY ? (a.hi_idx == 0 ? W.k0 : W.k1) : pl;
    const int64_t gkey = a.hi_src == PYST_G_NONE
                             ? lo
                             : static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | static_cast<uint32_t>(lo));
    if (hit && gkey == kEmpty64) latch(err, kErrKey);
    const int64_t val = !VX || a.vexpr == PYST_V_COL
                            ? W.x
                            : static_cast<int64_t>(static_cast<uint64_t>(W.x) *
                                                   static_cast<uint64_t>(a.vconst - static_cast<int64_t>(W.w)));
    const uint64_t mm = __ballot(hit);
    const int c = __popcll(mm);
    if (c > 0 && wpos + c > wend) {  // wave-uniform, once per kPairRun pairs
      for (int64_t p = wpos + lane; p < wend; p += kWave)
        if (p < po.cap) po.keys[p] = kEmpty64;
      unsigned long long rb = 0;
      if (lane == 0)
        rb = atomicAdd(reinterpret_cast<unsigned long long *>(po.count), static_cast<unsigned long long>(kPairRun));
      wpos = uniform64(static_cast<int64_t>(__shfl(rb, 0)));
      wend = wpos + kPairRun;
    }
    // the 64 pair slots from wpos, clipped to the buffer
    int64_t room = po.cap - wpos;
    room = room < 0 ? 0 : room > kWave ? kWave : room;
    const __amdgpu_buffer_rsrc_t rk = rsrc(po.keys + wpos, room * 8);
    const __amdgpu_buffer_rsrc_t rvv = rsrc(po.vals + wpos, room * 8);
    const int off = hit ? static_cast<int>(mbcnt(mm)) * 8 : kBufOob;
    __builtin_amdgcn_raw_buffer_store_b64(split64(gkey), rk, off, 0, 0);
    __builtin_amdgcn_raw_buffer_store_b64(split64(val), rvv, off, 0, 0);
    wpos += c;
  };
  // Both probes of the windows W[0..K).  Each table is read for all K windows
  // before any wait, and runs that go on past their first 16-byte group read
  // their next group in one round trip for all lanes and windows that need it.
  auto both_probes = [&](const auto &W) {
    constexpr int K = sizeof(W) / sizeof(W[0]);
    int32_t slot0[K], s[K];
    bool need[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      bool empty;
      const int h = match4(W[k].q0, W[k].k0, &empty);
      slot0[k] = W[k].ok && (dir0 || h >= 0) ? (dir0 ? 0 : W[k].s0 + h) : -1;
      need[k] = W[k].ok && !dir0 && h < 0 && !empty && groups0 > 1;
      s[k] = W[k].s0;
    }
    for (int32_t g = groups0 - 1;; --g) {
      bool any = false;
#pragma unroll
      for (int k = 0; k < K; ++k) any = any || need[k];
      if (__ballot(any) == 0) break;  // wave-uniform
      v4i32 q[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        s[k] = (s[k] + 4) & mask0;
        q[k] = __builtin_amdgcn_raw_buffer_load_b128(r0, need[k] ? s[k] * 4 : kBufOob, 0, 0);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        bool empty;
        const int h = match4(q[k], W[k].k0, &empty);
        if (need[k] && h >= 0) slot0[k] = s[k] + h;
        need[k] = need[k] && h < 0 && !empty && g > 1;
      }
    }
    v4i32 q1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t d1 = static_cast<uint32_t>(W[k].k1) - kmin1;
      const bool go = slot0[k] >= 0 && (!dir1 || d1 < range1);
      s[k] = dir1 ? static_cast<int32_t>(d1 & ~1u) : static_cast<int32_t>(table_hash32(W[k].k1)) & mask1 & ~(GS - 1);
      q1[k] = __builtin_amdgcn_raw_buffer_load_b128(r1, go ? s[k] * SB1 : kBufOob, 0, 0);
    }
    int state[K];
    int32_t pl[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (dir1) {  // the key's own slot: the first or the second of the group
        const bool odd = (static_cast<uint32_t>(W[k].k1) - kmin1) & 1u;
        const int32_t key = odd ? q1[k].z : q1[k].x;
        pl[k] = odd ? q1[k].w : q1[k].y;
        state[k] = key == W[k].k1 ? 1 : 0;  // a slot outside the range read as zeros: key 0 only if k1 is 0
        if (static_cast<uint32_t>(W[k].k1) - kmin1 >= range1) state[k] = 0;
      } else {
        state[k] = probe1(q1[k], W[k].k1, &pl[k]);
      }
      need[k] = slot0[k] >= 0 && state[k] < 0 && groups1 > 1;
    }
    for (int32_t g = groups1 - 1;; --g) {
      bool any = false;
#pragma unroll
      for (int k = 0; k < K; ++k) any = any || need[k];
      if (__ballot(any) == 0) break;  // wave-uniform
#pragma unroll
      for (int k = 0; k < K; ++k) {
        s[k] = (s[k] + GS) & mask1;
        q1[k] = __builtin_amdgcn_raw_buffer_load_b128(r1, need[k] ? s[k] * SB1 : kBufOob, 0, 0);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        int32_t pl2;
        const int st2 = probe1(q1[k], W[k].k1, &pl2);
        if (need[k] && st2 >= 0) {
          state[k] = st2;
          pl[k] = pl2;
        }
        need[k] = need[k] && st2 < 0 && g > 1;
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) emit(W[k], slot0[k] >= 0 && state[k] == 1, pl[k]);
  };
  for (; wbase < end; wbase += step) {
    const int64_t left64 = end - wbase;
    const int left = static_cast<int>(left64 < WR ? left64 : WR);
    uint64_t m[R];
    uint32_t b[R], n = 0;
    int32_t kv[2][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      bool l = lane * R + r < left && in_range(row_of(cur.c0, r), a.plo[0], a.pspan[0], a.pneg[0]) &&
               in_range(row_of(cur.c1, r), a.plo[1], a.pspan[1], a.pneg[1]);
      kv[0][r] = row_of(cur.f0, r);
      kv[1][r] = row_of(cur.f1, r);
      if (dir0) {
        const uint32_t d0 = static_cast<uint32_t>(kv[0][r]) - kmin0;
        l = l && d0 < range0 && ((s_bloom[d0 >> 5] >> (d0 & 31)) & 1u);
      } else if (use_bloom) {
        const uint32_t h = table_hash32(kv[0][r]);
        const uint32_t bits = bloom_bits(h);
        l = l && (s_bloom[bloom_word(h, cap0 - 1, bshift)] & bits) == bits;
      }
      m[r] = __ballot(l);
      b[r] = n;
      n += static_cast<uint32_t>(__popcll(m[r]));
    }
    n = __builtin_amdgcn_readfirstlane(n);
    const __amdgpu_buffer_rsrc_t rv = window(a.v0, V64 ? 8 : 4, wbase, end, WR);
    const __amdgpu_buffer_rsrc_t rw = window(VX ? a.v1 : nullptr, 4, wbase, end, WR);
    // NW windows go through each probe together, so that a step waits for
    // each table once; windows past them (rare) go one at a time.
    Win W[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) W[k] = issue(m, b, kv, k * kWave, n, rv, rw);
    const FactRows<R> nxt = load_rows<2, R>(a, wbase + step, end, lane);
    both_probes(W);
    for (uint32_t w0 = NW * kWave; w0 < n; w0 += kWave) {  // wave-uniform; rare
      Win W2[1] = {issue(m, b, kv, w0, n, rv, rw)};
      both_probes(W2);
    }
    cur = nxt;
  }
  for (int64_t p = wpos + lane; p < wend; p += kWave)
    if (p < po.cap) po.keys[p] = kEmpty64;
#pragma unroll
  for (int k = 0; k < NW; ++k)
    if (stand_in[k].x != 0) latch(err, kErrKey);  // never: an empty buffer reads 0
}

template <int NJ, int SB1, int AGG, bool V64, bool VX, int R = 4>
__global__ __launch_bounds__(kFastBlock) void k_fast_fact(FastArgs a, TableDev t0, TableDev t1, GroupDev g, PairsOut po,
                                                         BucketPool bp, uint32_t *err) {
  __shared__ uint32_t s_bloom[kBloomWords];
  __shared__ uint64_t s_ent[AGG == 3 ? kStageCap : 1];
  __shared__ uint32_t s_bk[AGG == 3 ? 5 * kMaxBuckets + 1 : 1];
  StageLds sl;
  sl.ent = (PYST_LDS uint64_t *)s_ent;
  sl.chunk = (PYST_LDS uint32_t *)s_bk;
  sl.fill = sl.chunk + kMaxBuckets;
  sl.hist = sl.fill + kMaxBuckets;
  sl.rank = sl.hist + kMaxBuckets;
  sl.newbase = sl.rank + kMaxBuckets;
  sl.cnt = sl.newbase + kMaxBuckets;
  if (AGG == 3) {
    const uint32_t nb = bucket_count(t0.hdr[0]);
    if (nb <= bp.stride && threadIdx.x < bp.stride) {  // the block's first chunks, one per bucket
      const uint32_t c = blockIdx.x * bp.stride + threadIdx.x;
      bp.fill[c] = 0;
      if (threadIdx.x < nb) {
        sl.chunk[threadIdx.x] = c;
        sl.fill[threadIdx.x] = 0;
        sl.hist[threadIdx.x] = 0;
      }
    }
    if (threadIdx.x == 0) *sl.cnt = 0;
  }
  // Direct-addressed tables come from k_fast_table_init, for the staged one-join
  // pass (join 0) and the two-join pair pass (both joins) only.
  constexpr bool kMayDirect = (NJ == 1 && AGG == 3) || (NJ == 2 && AGG == 2);
  const bool direct = kMayDirect && t0.hdr[kHdrDirect] != 0;
  if (kMayDirect && blockIdx.x == 0 && threadIdx.x == 0) {  // duplicate keys seen while the tables were built
    if (direct && t0.hdr[kHdrDistinct] != t0.hdr[1]) latch(err, kErrDup);
    if (NJ == 2 && t1.hdr[kHdrDirect] != 0 && t1.hdr[kHdrDistinct] != t1.hdr[1]) latch(err, kErrDup);
  }
  const bool use_bloom = direct || (t0.bloom != nullptr && t0.hdr[1] <= kBloomMaxKeys);
  if (use_bloom)
    for (int i = threadIdx.x; i < kBloomWords; i += kFastBlock) s_bloom[i] = gmem(t0.bloom)[i];
  if (use_bloom || AGG == 3) __syncthreads();
  const int64_t begin = int64_t{blockIdx.x} * kFastBlock * R, step = int64_t{gridDim.x} * kFastBlock * R;
  if constexpr (NJ == 1 && AGG == 3) {
    if (direct) star_direct<V64, VX, R>(a, t0, (const PYST_LDS uint32_t *)s_bloom, begin, step, a.n, &bp, &sl);
    else star_range<AGG, V64, VX, R>(a, t0, err, (const PYST_LDS uint32_t *)s_bloom, use_bloom, begin, step, a.n, &bp, &sl);
  } else if constexpr (NJ == 1 && AGG == 0)
    star_range<AGG, V64, VX, R>(a, t0, err, (const PYST_LDS uint32_t *)s_bloom, use_bloom, begin, step, a.n, &bp, &sl);
  else if constexpr (NJ == 2 && AGG == 2)
    chain_range<SB1, V64, VX, R>(a, t0, t1, po, err, (const PYST_LDS uint32_t *)s_bloom, use_bloom, begin, step, a.n);
  else
    fact_range<NJ, SB1, AGG, V64, VX, R>(a, t0, t1, g, po, err, (const PYST_LDS uint32_t *)s_bloom, use_bloom, begin,
                                         step, a.n);
}

// Adds the pairs of up to 4 chunks (kNoChunk: none) into the LDS sums of their
// bucket and marks their slots present (s_pres: one byte per slot).  One wave; every lane loads its pairs of all 4 chunks before any add,
// so 4 chunks cost one memory round trip per 256 pairs each.
__device__ __forceinline__ void add_chunks(const BucketPool &bp, const uint32_t (&c)[4], int64_t lo, uint64_t *s_sum,
                                           uint32_t *s_pres) {
  constexpr int U = 4;
  uint32_t f[4], fmax = 0;
  size_t base[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    f[i] = c[i] != kNoChunk ? bp.fill[c[i]] : 0;
    base[i] = size_t{c[i] != kNoChunk ? c[i] : 0} << bp.chunk_lg;
    fmax = f[i] > fmax ? f[i] : fmax;
  }
  for (uint32_t e0 = 0; e0 < fmax; e0 += U * kWave) {  // wave-uniform
    uint64_t q[4 * U];
    bool ok[4 * U];
#pragma unroll
    for (int u = 0; u < 4 * U; ++u) {
      const uint32_t e = e0 + (u % U) * kWave + lane_id();
      ok[u] = e < f[u / U];
      q[u] = ok[u] ? bp.rec[base[u / U] + e] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4 * U; ++u) {
      if (!ok[u]) continue;
      const uint32_t s = static_cast<uint32_t>(q[u]) & (kBucketSlots - 1);
      atomicAdd(reinterpret_cast<unsigned long long *>(&s_sum[s]),
                static_cast<unsigned long long>(static_cast<int64_t>(q[u]) >> kBucketLg));
      reinterpret_cast<uint8_t *>(s_pres)[s] = 1;  // idempotent: a plain byte store, no atomic
    }
  }
}

// Second kernel of the bucketed slot sums: block b adds up the pairs of bucket
// b in LDS, adds the sums the fact pass made directly, and writes the groups
// present with one counter atomic.  *d_ngroups must be zero on entry.  The LDS
// arrays come from the calling kernel (s_sum: kBucketSlots, s_pres:
// kBucketSlots / 4 words of presence bytes, s_wsum: kFastBlock / kWave, s_base: 1); blockDim.x is
// kFastBlock.  may_direct: the table's header records its mode (tables from
// k_fast_table_init); a direct-addressed slot s holds the key kmin + s.
__device__ __forceinline__ void bucket_sums_block(const TableDev &t, const BucketPool &bp, uint32_t b,
                                                  int64_t *out_keys, int64_t *out_sums, int64_t out_cap,
                                                  int64_t *d_ngroups, uint32_t *err, uint64_t *s_sum,
                                                  uint32_t *s_pres, uint32_t *s_wsum, int64_t *s_base,
                                                  bool may_direct) {
  const int64_t cap = t.hdr[0];
  const uint32_t nb = bucket_count(cap);
  if (b >= nb) return;  // block-uniform
  const uint32_t tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
  const int64_t lo = int64_t{b} << kBucketLg;
  const uint32_t span = static_cast<uint32_t>(cap - lo < kBucketSlots ? cap - lo : kBucketSlots);
  for (uint32_t i = tid; i < kBucketSlots; i += kFastBlock) s_sum[i] = 0;
  for (uint32_t i = tid; i < kBucketSlots / 4; i += kFastBlock) s_pres[i] = 0;
  __syncthreads();
  if (nb <= bp.stride) {  // pairs were staged
    // the blocks' first chunks of bucket b, then the chunks it took from its region
    constexpr uint32_t NW = kFastBlock / kWave;
    for (uint32_t k = wv; k < bp.blocks; k += 4 * NW) {
      uint32_t cs[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) cs[i] = k + i * NW < bp.blocks ? (k + i * NW) * bp.stride + b : kNoChunk;
      add_chunks(bp, cs, lo, s_sum, s_pres);
    }
    const uint32_t reg = region_chunks(bp, nb), first = region_first(bp, nb, b);
    const uint32_t used = bp.next[b] < reg ? bp.next[b] : reg;
    for (uint32_t k = wv; k < used; k += 4 * NW) {
      uint32_t cs[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) cs[i] = k + i * NW < used ? first + k + i * NW : kNoChunk;
      add_chunks(bp, cs, lo, s_sum, s_pres);
    }
  }
  __syncthreads();
  if (bucket_added(t, b))  // block-uniform: a slot of the bucket holds a sum of its own
    for (uint32_t s = tid; s < span; s += kFastBlock)
      if (t.flags[lo + s]) {
        s_sum[s] += t.sums[lo + s];
        reinterpret_cast<uint8_t *>(s_pres)[s] = 1;
      }
  __syncthreads();
  constexpr uint32_t kPer = kBucketSlots / kFastBlock;  // each thread writes out kPer consecutive slots
  const uint32_t s0 = tid * kPer;
  static_assert(kPer == 8, "a thread's slots are two words of presence bytes");
  const uint32_t p0 = s_pres[s0 / 4], p1 = s_pres[s0 / 4 + 1];  // byte i -> bit i
  uint32_t m = (((p0 & 0x01010101u) * 0x01020408u) >> 24) | ((((p1 & 0x01010101u) * 0x01020408u) >> 24) << 4);
  const uint32_t c = static_cast<uint32_t>(__popc(m));
  const uint32_t incl = wave_inclusive_scan(c);
  if (lane == kWave - 1) s_wsum[wv] = incl;
  __syncthreads();
  if (tid == 0) {
    uint32_t tot = 0;
    for (int k = 0; k < kFastBlock / kWave; ++k) tot += s_wsum[k];
    *s_base = tot ? static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long *>(d_ngroups),
                                                   static_cast<unsigned long long>(tot)))
                  : 0;
  }
  __syncthreads();
  int64_t pos = *s_base + incl - c;
  for (uint32_t k = 0; k < wv; ++k) pos += s_wsum[k];
  const int32_t *keys = static_cast<const int32_t *>(t.slots);
  const bool direct = may_direct && t.hdr[kHdrDirect] != 0;
  const int32_t kmin = direct ? static_cast<int32_t>(t.hdr[kHdrKmin]) : 0;
  while (m) {
    const uint32_t j = static_cast<uint32_t>(__ffs(m) - 1);
    m &= m - 1;
    if (pos < out_cap) {
      out_keys[pos] = direct ? static_cast<int32_t>(static_cast<uint32_t>(kmin) + static_cast<uint32_t>(lo + s0 + j))
                             : keys[lo + s0 + j];
      out_sums[pos] = static_cast<int64_t>(s_sum[s0 + j]);
    } else {
      latch(err, kErrCapacity);
    }
    ++pos;
  }
}

__global__ __launch_bounds__(kFastBlock) void k_bucket_sums(TableDev t, BucketPool bp, int64_t *out_keys,
                                                           int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                                                           uint32_t *err) {
  __shared__ uint64_t s_sum[kBucketSlots];
  __shared__ uint32_t s_pres[kBucketSlots / 4];
  __shared__ uint32_t s_wsum[kFastBlock / kWave];
  __shared__ int64_t s_base;
  bucket_sums_block(t, bp, blockIdx.x, out_keys, out_sums, out_cap, d_ngroups, err, s_sum, s_pres, s_wsum, &s_base,
                    true);
}

// Unordered compaction of groups (slot sums or a group table): one counter
// atomic per wave; *d_ngroups must be zero on entry.
template <bool SLOTS>
__global__ __launch_bounds__(256) void k_compact_unordered(TableDev t, GroupDev g, int64_t *out_keys, int64_t *out_sums,
                                                          int64_t out_cap, int64_t *d_ngroups, uint32_t *err) {
  // Each block compacts whole tiles and takes ONE counter atomic per tile (a
  // counter bumped by every wave serializes the kernel on a single address).
  constexpr int ITEMS = 8, NW = 256 / kWave;
  constexpr int64_t TILE = 256 * ITEMS;
  __shared__ int32_t s_cnt[NW];
  __shared__ int64_t s_base;
  const int64_t cap = SLOTS ? t.hdr[0] : g.hdr[0];
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int64_t tile = blockIdx.x; tile * TILE < cap; tile += gridDim.x) {  // block-uniform
    const int64_t wbase = tile * TILE + int64_t{w} * kWave * ITEMS;
    int64_t key[ITEMS], sum[ITEMS];
    bool keep[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {  // every load issued before any use
      const int64_t s = wbase + int64_t{j} * kWave + lane;
      const int64_t sc = s < cap ? s : cap - 1;
      if (SLOTS) {
        keep[j] = t.flags[sc] != 0 && s < cap;
        key[j] = static_cast<const int32_t *>(t.slots)[sc];
        sum[j] = static_cast<int64_t>(t.sums[sc]);
      } else {
        key[j] = static_cast<int64_t>(g.slots[2 * sc]);
        sum[j] = static_cast<int64_t>(g.slots[2 * sc + 1]);
        keep[j] = key[j] != kEmpty64 && s < cap;
      }
    }
    uint64_t m[ITEMS];
    int c = 0;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      m[j] = __ballot(keep[j]);
      c += __popcll(m[j]);
    }
    if (lane == 0) s_cnt[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t tot = 0;
      for (int k = 0; k < NW; ++k) tot += s_cnt[k];
      s_base = tot ? static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long *>(d_ngroups),
                                                    static_cast<unsigned long long>(tot)))
                   : 0;
    }
    __syncthreads();
    int64_t pos = s_base;
    for (int k = 0; k < w; ++k) pos += s_cnt[k];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (keep[j]) {
        const int64_t p = pos + mbcnt(m[j]);
        if (p < out_cap) {
          out_keys[p] = key[j];
          out_sums[p] = sum[j];
        } else {
          latch(err, kErrCapacity);
        }
      }
      pos += __popcll(m[j]);
    }
    __syncthreads();  // s_cnt / s_base are reused by the next tile
  }
}

__global__ void k_zero_i64(int64_t *p) { *p = 0; }

// ------------------------------------------------------------------ host side
// A comparison "x OP c" of an int32 column with an int64 constant as the
// range form the fact pass evaluates: x in [lo, lo + span] XOR neg.
static void pred_range(int op, int64_t c, int32_t *lo, uint32_t *span, int32_t *neg) {
  // past the int32 range by one, the constant compares with every x as c does
  c = std::min<int64_t>(std::max<int64_t>(c, int64_t{INT32_MIN} - 1), int64_t{INT32_MAX} + 1);
  int64_t l = INT32_MIN, h = INT32_MAX;
  bool n = false;
  switch (op) {
    case PYST_EQ: l = h = c; break;
    case PYST_NE: l = h = c; n = true; break;
    case PYST_LT: h = c - 1; break;
    case PYST_LE: h = c; break;
    case PYST_GT: l = c + 1; break;
    default: l = c; break;  // PYST_GE
  }
  l = std::max<int64_t>(l, INT32_MIN);
  h = std::min<int64_t>(h, INT32_MAX);
  if (l > h) {  // no int32 value is in the range: the result is the constant n
    *lo = INT32_MIN;
    *span = 0xffffffffu;
    *neg = n ? 0 : 1;
    return;
  }
  *lo = static_cast<int32_t>(l);
  *span = static_cast<uint32_t>(h - l);
  *neg = n ? 1 : 0;
}

// Can this plan take the fast path?  Fills the kernel arguments if so.
bool fast_shape(const pyst_plan *plan, const pyst_col *fact, const QueryShape &q, FastArgs *fa) {
  std::memset(fa, 0, sizeof(*fa));
  if (plan->npreds > 2) return false;
  if (plan->njoins == 2 && q.need_payload[0]) return false;  // join 0 is a keys-only table
  if (plan->njoins == 1 && !q.slot_agg && q.need_payload[0]) return false;
  for (int j = 0; j < plan->njoins; ++j) fa->fk[j] = static_cast<const int32_t *>(fact[plan->joins[j].probe_col].data);
  auto is_src = [&](int src) { return src == PYST_G_NONE || src == PYST_G_JOIN_KEY || src == PYST_G_JOIN_PAYLOAD; };
  if (!is_src(plan->hi_src) || !is_src(plan->lo_src)) return false;
  if ((plan->hi_src == PYST_G_JOIN_PAYLOAD && plan->hi_index != 1) ||
      (plan->lo_src == PYST_G_JOIN_PAYLOAD && plan->lo_index != 1))
    return false;  // only join 1 carries a payload on the fast path
  fa->hi_src = plan->hi_src;
  fa->hi_idx = plan->hi_index;
  fa->lo_src = plan->lo_src;
  fa->lo_idx = plan->lo_index;
  fa->v0 = fact[plan->v0].data;
  fa->v0_64 = fact[plan->v0].dtype == PYST_I64;
  fa->vexpr = plan->vexpr;
  fa->vconst = plan->vconst;
  if (plan->vexpr == PYST_V_COL_TIMES_C_MINUS) {
    if (fact[plan->v1].dtype != PYST_I32) return false;
    fa->v1 = static_cast<const int32_t *>(fact[plan->v1].data);
  }
  for (int k = 0; k < 2; ++k) {
    fa->plo[k] = INT32_MIN;
    fa->pspan[k] = 0xffffffffu;
  }
  for (int k = 0; k < plan->npreds; ++k) {
    const int c = plan->preds[k].col;
    if (fact[c].dtype != PYST_I32) return false;
    fa->pcol[k] = static_cast<const int32_t *>(fact[c].data);
    pred_range(plan->preds[k].cmp, plan->preds[k].value, &fa->plo[k], &fa->pspan[k], &fa->pneg[k]);
  }
  fa->n = fact[0].n;
  // buffer resources address less than kBufOob bytes of a table
  for (int j = 0; j < plan->njoins; ++j) {
    const int sb = (j == 0 && q.slot_agg) ? 8 : (j == 1 && q.need_payload[1]) ? 8 : 4;
    if (table_capacity_host(plan->joins[j].key.n, plan->joins[j].max_load) * sb >= kBufOob) return false;
  }
  return true;
}

// Fact pass with staged (slot, value) pairs, then the per-bucket sums and the
// output (single join, sums grouped by the join key).
static pyst_status bucketed_sums(pyst_ctx *ctx, const FastArgs &a, const DimTables &d, const BucketPool &bp,
                                 int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                                 hipStream_t stream) {
  uint32_t *err = ctx_err_word(ctx);
  {
    TimedRegion timed(ctx, "fact_pass", stream);
    const dim3 grid(bp.blocks), block(kFastBlock);
    const bool vx = a.vexpr != PYST_V_COL;
    constexpr int R = kStarRows;
    if (a.v0_64 && vx) k_fast_fact<1, 4, 3, true, true, R><<<grid, block, 0, stream>>>(a, d.t[0], d.t[1], GroupDev{}, PairsOut{}, bp, err);
    else if (a.v0_64) k_fast_fact<1, 4, 3, true, false, R><<<grid, block, 0, stream>>>(a, d.t[0], d.t[1], GroupDev{}, PairsOut{}, bp, err);
    else if (vx) k_fast_fact<1, 4, 3, false, true, R><<<grid, block, 0, stream>>>(a, d.t[0], d.t[1], GroupDev{}, PairsOut{}, bp, err);
    else k_fast_fact<1, 4, 3, false, false, R><<<grid, block, 0, stream>>>(a, d.t[0], d.t[1], GroupDev{}, PairsOut{}, bp, err);
    PYST_LAUNCH_CHECK("k_fast_fact");
  }
  k_bucket_sums<<<bucket_count(d.t[0].cap_alloc), kFastBlock, 0, stream>>>(d.t[0], bp, out_keys, out_sums, out_cap,
                                                                           d_ngroups, err);
  PYST_LAUNCH_CHECK("k_bucket_sums");
  return PYST_OK;
}

pyst_status fast_query(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, const FastArgs &fa,
                       int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                       hipStream_t stream) {
  DimTables d;
  std::memset(&d, 0, sizeof(d));
  AggState s;
  std::memset(&s, 0, sizeof(s));
  pyst_status st = PYST_OK;
  if (q.agg_mode == 1) {
    const int64_t bound = std::min<int64_t>(plan->max_groups, std::max<int64_t>(fa.n, 1));
    const int64_t cap = table_capacity_host(bound, plan->group_max_load);
    s.mem = ctx_alloc(ctx, group_bytes(cap), stream);
    if (!s.mem) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (group table)");
    s.g = group_view(s.mem, cap);
    st = group_init(s.g, nullptr, bound, 0, plan->group_max_load, stream);
  } else if (q.agg_mode == 2) {
    // every wave may leave up to one partly used run of kPairRun slots
    const int64_t cap = std::max<int64_t>(fa.n, 1) + int64_t{fast_grid(ctx, fa.n)} * (kFastBlock / kWave) * kPairRun;
    s.mem = ctx_alloc(ctx, 256 + static_cast<size_t>(cap) * 16, stream);
    if (!s.mem) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (pair buffer)");
    s.po.count = static_cast<int64_t *>(s.mem);
    s.po.keys = reinterpret_cast<int64_t *>(static_cast<char *>(s.mem) + 256);
    s.po.vals = s.po.keys + cap;
    s.po.cap = cap;
  }
  // Sums kept in join-table slots go through bucketed pairs when the arena
  // holds the pair pool and the table has at most kMaxSumBuckets buckets; the
  // fact pass stages pairs when the table it sized on the device has at most
  // kMaxBuckets buckets, and otherwise adds into the slots directly.
  BucketPool bp;
  std::memset(&bp, 0, sizeof(bp));
  void *pool = nullptr;
  if (st == PYST_OK && q.agg_mode == 0 && plan->njoins == 1 && fa.n > 0) {
    const int64_t cap_alloc = table_capacity_host(plan->joins[0].key.n, plan->joins[0].max_load);
    const int64_t grid = fast_grid(ctx, fa.n);
    const int64_t stride = std::min<int64_t>(kMaxBuckets, bucket_count(cap_alloc));
    const int64_t nchunks = grid * stride + ceil_div(fa.n, int64_t{kChunk}) + 1;
    if (cap_alloc <= kBucketSlots * kMaxSumBuckets && nchunks < (int64_t{1} << 31))
      pool = ctx_alloc(ctx, kPoolHeadBytes + static_cast<size_t>(nchunks) * (size_t{kChunk} * 8 + 4), stream);
    if (pool) {
      char *p = static_cast<char *>(pool);
      bp.next = reinterpret_cast<uint32_t *>(p);  // zeroed by the table initializer
      bp.rec = reinterpret_cast<uint64_t *>(p + kPoolHeadBytes);
      bp.fill = reinterpret_cast<uint32_t *>(bp.rec + static_cast<size_t>(nchunks) * kChunk);
      bp.nchunks = static_cast<uint32_t>(nchunks);
      bp.chunk_lg = kChunkLg;
      bp.blocks = static_cast<uint32_t>(grid);
      bp.stride = static_cast<uint32_t>(stride);
    }
  }
  if (st == PYST_OK)
    st = fast_build_dimensions(ctx, plan, q, &d, d_ngroups, pool ? nullptr : s.po.count, stream,
                               (pool != nullptr || (plan->njoins == 2 && q.agg_mode == 2 && fa.n > 0)) &&
                                   !ctx_hash_join_only(ctx),
                               pool ? bp.next : nullptr);
  if (pool) {
    if (st == PYST_OK) st = bucketed_sums(ctx, fa, d, bp, out_keys, out_sums, out_cap, d_ngroups, stream);
    ctx_free(ctx, pool, stream);
  } else {
    if (st == PYST_OK) st = fast_fact_pass(ctx, plan->njoins, q.agg_mode, fa, d, s.g, s.po, stream);
    if (st == PYST_OK) st = fast_finish(ctx, plan, q, d, &s, out_keys, out_sums, out_cap, d_ngroups, stream);
  }
  ctx_free(ctx, s.mem, stream);
  free_dimensions(ctx, &d, stream);
  return st;
}

// Dimension tables of the fast path: join 0 keys-only with a Bloom filter, or,
// with allow_direct (its consumers handle the direct-addressed mode) and keys
// that allow it, direct-addressed: join 0 of the staged one-join pass (range
// up to 2^kStageSlotBits), both joins of the two-join pair pass (join 0 up to
// kFilterBits keys, so that its LDS filter is exact; join 1 with payloads).
pyst_status fast_build_dimensions(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, DimTables *d,
                                  int64_t *zero0, int64_t *zero1, hipStream_t stream, bool allow_direct,
                                  uint32_t *pool_next) {
  for (int j = 0; j < plan->njoins; ++j) {
    const pyst_join_spec &js = plan->joins[j];
    const int64_t nb = js.key.n;
    const int sb = (j == 1 && q.need_payload[1]) ? 8 : 4;
    const bool sums = j == 0 && q.slot_agg;
    const int64_t cap_alloc = table_capacity_host(nb, js.max_load);
    const size_t tbytes = table_bytes(cap_alloc, sb, sums);
    const size_t bloom_off = (tbytes + 255) / 256 * 256;
    const size_t bloom_bytes = j == 0 ? size_t{kBloomWords} * 4 : 0;
    d->mem[j] = ctx_alloc(ctx, bloom_off + bloom_bytes, stream);
    if (!d->mem[j]) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (dimension table)");
    d->t[j] = table_view(d->mem[j], cap_alloc, sb, sums);
    if (j == 0) d->t[j].bloom = reinterpret_cast<uint32_t *>(static_cast<char *>(d->mem[j]) + bloom_off);
    const int32_t *sel = nullptr;
    int32_t *cnt = nullptr, *kmin_b = nullptr, *kmax_b = nullptr;
    const int64_t nblk = std::max<int64_t>(1, ceil_div(nb, kDimTile));
    const bool chain = plan->njoins == 2 && q.agg_mode == 2;
    const bool direct_ok = allow_direct && nb > 0 && js.key.dtype == PYST_I32 &&
                           ((j == 0 && sb == 4 && (sums || chain)) || (j == 1 && sb == 8 && chain));
    const int64_t max_range = j == 1 ? INT64_MAX : sums ? (int64_t{1} << kStageSlotBits) : int64_t{kFilterBits};
    if (js.npreds > 0 || direct_ok) {  // (direct addressing needs the selected keys' bounds from the filter)
      const int64_t nblk64 = (nblk + 63) / 64 * 64;
      d->sel_mem[j] = ctx_alloc(ctx, static_cast<size_t>(nblk) * kDimTile * sizeof(int32_t) +
                                         static_cast<size_t>(3 * nblk64) * sizeof(int32_t) + 256, stream);
      if (!d->sel_mem[j]) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (dimension selection)");
      cnt = static_cast<int32_t *>(d->sel_mem[j]);
      if (direct_ok) {
        kmin_b = cnt + nblk64;
        kmax_b = kmin_b + nblk64;
      }
      int32_t *s = cnt + 3 * nblk64;
      PredSet ps;
      std::memset(&ps, 0, sizeof(ps));
      ps.n = js.npreds;
      for (int k = 0; k < js.npreds; ++k) {
        const int c = js.preds[k].col;
        if (c < 0 || c >= js.ncols) return set_error(PYST_ERR_ARG, "pyst_query: dimension predicate names a missing column");
        ps.col[k] = js.cols[c].data;
        ps.is64[k] = js.cols[c].dtype == PYST_I64;
        ps.op[k] = js.preds[k].cmp;
        ps.val[k] = js.preds[k].value;
      }
      k_dim_filter<<<static_cast<unsigned>(nblk), 256, 0, stream>>>(
          ps, nb, s, cnt, direct_ok ? static_cast<const int32_t *>(js.key.data) : nullptr, kmin_b, kmax_b);
      PYST_LAUNCH_CHECK("k_dim_filter");
      sel = s;
    }
    const int iblocks = static_cast<int>(std::min<int64_t>(std::max<int64_t>(ceil_div(cap_alloc, 256), 64), 2048));
    k_fast_table_init<<<iblocks, 256, 0, stream>>>(d->t[j], cnt, nblk, nb, js.max_load, j == 0 ? zero0 : nullptr,
                                                   j == 0 ? zero1 : nullptr, kmin_b, kmax_b, max_range,
                                                   j == 0 ? pool_next : nullptr);
    PYST_LAUNCH_CHECK("k_fast_table_init");
    if (nb > 0) {
      const int32_t *key = static_cast<const int32_t *>(js.key.data);
      const int32_t *pay = static_cast<const int32_t *>(js.payload.data);
      if (js.npreds == 0) sel = nullptr;  // the filter ran for the key bounds only: every row is selected
      if (sb == 4) {  // one block per dimension tile (the filter's tiles)
        k_fast_build<<<static_cast<unsigned>(nblk), 256, 0, stream>>>(key, sel, cnt, nb, d->t[j], ctx_err_word(ctx));
      } else {
        const int blocks = static_cast<int>(std::min<int64_t>(ceil_div(nb, 256), int64_t{1} << 20));
        k_fast_build_payload<<<blocks, 256, 0, stream>>>(key, pay, sel, cnt, nb, d->t[j], ctx_err_word(ctx));
        if (direct_ok) {  // (a no-op unless the initializer chose direct addressing)
          PYST_LAUNCH_CHECK("k_fast_build_payload");
          k_direct_count<<<static_cast<unsigned>(std::min<int64_t>(ceil_div(cap_alloc / 2, 256 * 4), 256)), 256, 0,
                           stream>>>(d->t[j]);
        }
      }
      PYST_LAUNCH_CHECK("k_fast_build");
      if (d->t[j].bloom) {  // keys-only (join 0)
        k_fast_bloom<<<kBloomWords / 256, 256, 0, stream>>>(d->t[j]);
        PYST_LAUNCH_CHECK("k_fast_bloom");
      }
    }
  }
  return PYST_OK;
}

// One 1024-thread block per CU (the 128 KiB Bloom filter takes most of the LDS).
int fast_grid(pyst_ctx *ctx, int64_t n) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 4 * kFastBlock), ctx_num_cus(ctx))));
}

template <int NJ, int SB1, int AGG, bool V64, bool VX>
static void launch_fast(int grid, const FastArgs &a, const DimTables &d, const GroupDev &g, const PairsOut &po,
                        uint32_t *err, hipStream_t stream) {
  k_fast_fact<NJ, SB1, AGG, V64, VX><<<grid, kFastBlock, 0, stream>>>(a, d.t[0], d.t[1], g, po, BucketPool{}, err);
}

pyst_status fast_fact_pass(pyst_ctx *ctx, int njoins, int agg_mode, const FastArgs &a, const DimTables &d,
                           const GroupDev &g, const PairsOut &po, hipStream_t stream) {
  if (a.n <= 0) return PYST_OK;
  if (ctx_fail_this_pass(ctx)) return set_error(PYST_ERR_HIP, "fact pass: failure injected by PYST_OPT_FAIL_FACT_PASS");
  const int grid = fast_grid(ctx, a.n);
  uint32_t *err = ctx_err_word(ctx);
  const int sb1 = njoins > 1 ? d.t[1].slot_bytes : 4;
  const bool v64 = a.v0_64 != 0;
  TimedRegion timed(ctx, "fact_pass", stream);
#define PYST_FAST_CASE(NJ_, S1_, AG_)                                                    \
  if (njoins == NJ_ && sb1 == S1_ && agg_mode == AG_) {                                 \
    if (v64) launch_fast<NJ_, S1_, AG_, true, true>(grid, a, d, g, po, err, stream);     \
    else launch_fast<NJ_, S1_, AG_, false, true>(grid, a, d, g, po, err, stream);        \
    PYST_LAUNCH_CHECK("k_fast_fact");                                                   \
    return PYST_OK;                                                                     \
  }
  if (njoins == 1 && agg_mode == 0 && a.vexpr == PYST_V_COL) {  // sums of a plain column in the join slots
    if (v64) launch_fast<1, 4, 0, true, false>(grid, a, d, g, po, err, stream);
    else launch_fast<1, 4, 0, false, false>(grid, a, d, g, po, err, stream);
    PYST_LAUNCH_CHECK("k_fast_fact");
    return PYST_OK;
  }
  PYST_FAST_CASE(1, 4, 0)
  PYST_FAST_CASE(1, 4, 1)
  PYST_FAST_CASE(1, 4, 2)
  PYST_FAST_CASE(2, 4, 1)
  PYST_FAST_CASE(2, 4, 2)
  PYST_FAST_CASE(2, 8, 1)
  PYST_FAST_CASE(2, 8, 2)
#undef PYST_FAST_CASE
  return set_error(PYST_ERR_UNSUPPORTED, "pyst_query: no fast kernel for this shape");
}

// The groups of the fact pass: slot sums or a group table are compacted
// (unordered); materialized pairs are grouped by pair_groupby.  *d_ngroups must
// be zero on entry (the table initializer clears it).
pyst_status fast_finish(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, const DimTables &d, AggState *s,
                        int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                        hipStream_t stream) {
  const int cgrid = 2048;
  if (q.agg_mode == 0) {
    k_compact_unordered<true><<<cgrid, 256, 0, stream>>>(d.t[0], GroupDev{}, out_keys, out_sums, out_cap, d_ngroups,
                                                        ctx_err_word(ctx));
    PYST_LAUNCH_CHECK("k_compact_unordered");
    return PYST_OK;
  }
  if (q.agg_mode == 2)  // pairs: hash-partitioned LDS aggregation
    return pair_groupby(ctx, s->po.keys, s->po.vals, s->po.count, s->po.cap, out_keys, out_sums, out_cap, d_ngroups,
                        stream);
  k_compact_unordered<false><<<cgrid, 256, 0, stream>>>(TableDev{}, s->g, out_keys, out_sums, out_cap, d_ngroups,
                                                       ctx_err_word(ctx));
  PYST_LAUNCH_CHECK("k_compact_unordered");
  return PYST_OK;
}

}  // namespace pyst

// Batched execution of many independent query fragments.
//
// Small inputs lose efficiency when each is processed by its own sequence of
// launches and host round trips; the paper accumulates small chunks before
// size-sensitive operators for the same reason (Sec. 5.3, "Dynamic
// Buffering").  Here all fragments of a batch run through six launches in
// total -- dimension filter, table init, build, Bloom filter, fact pass,
// compaction -- each launch covering every fragment.  A block finds its fragment by binary search
// over per-kernel block prefixes held in device memory.
//
// The batch path serves star-shaped fragments (one join, group by the join
// key, slot sums); every fragment has its own dimension, fact and outputs.
#include <algorithm>
#include <new>
#include <chrono>
#include <cstring>
#include <vector>

#include "pyst_internal.h"
#include "query.h"
#include "table.h"

namespace pyst {

struct BatFrag {
  PredSet bpred;           // dimension predicates
  const int32_t *bkey;     // dimension keys
  int64_t nb;
  int32_t *sel;            // block-local selection (nblk * kDimTile)
  int32_t *cnt;            // per-block selected counts
  int32_t *kmin_b, *kmax_b;  // per-block selected key bounds (direct addressing allowed), else null
  int64_t nblk;
  TableDev t;              // keys-only table with slot sums
  double max_load;
  FastArgs fa;             // fact side (single join)
  int64_t rows_per_unit;   // rows of one fact work unit (multiple of 4)
  int64_t *out_keys, *out_sums;
  int64_t out_cap;
  int64_t *d_ngroups;
  BucketPool bp;           // staged batches: the fragment's pool of pair chunks (next == nullptr: none)
};

// Per-kernel block prefixes: blocks of fragment f are [pre[f], pre[f+1]).
enum { kPreFilter = 0, kPreInit = 1, kPreBuild = 2, kPreBloom = 3, kPreFact = 4, kPreCompact = 5, kPreKinds = 6 };

__device__ __forceinline__ int frag_of(const int64_t *pre, int nfrag, int64_t b) {
  int lo = 0, hi = nfrag - 1;  // largest f with pre[f] <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (pre[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

#define PYST_BLOCK_FRAG_AT(kind, blk)                                      \
  __shared__ int s_frag;                                                   \
  const int64_t blk_ = (blk);                                              \
  if (threadIdx.x == 0) s_frag = frag_of(pre + (kind) * (nfrag + 1), nfrag, blk_); \
  __syncthreads();                                                         \
  const int f = s_frag;                                                    \
  const BatFrag &fr = frags[f];                                            \
  const int64_t local = blk_ - pre[(kind) * (nfrag + 1) + f];              \
  const int64_t nloc = pre[(kind) * (nfrag + 1) + f + 1] - pre[(kind) * (nfrag + 1) + f];
#define PYST_BLOCK_FRAG(kind) PYST_BLOCK_FRAG_AT(kind, blockIdx.x)

// The fact pass lays its blocks out by fragment in the order kept after the
// prefixes (pre[kPreKinds * (nfrag + 1) + i]: the fragment at position i),
// largest work units first, so that the long units start early and the end
// of the launch is made of short ones.
#define PYST_BLOCK_FRAG_ORDERED(kind)                                                        \
  __shared__ int s_frag, s_pos;                                                              \
  if (threadIdx.x == 0) {                                                                    \
    s_pos = frag_of(pre + (kind) * (nfrag + 1), nfrag, blockIdx.x);                          \
    s_frag = static_cast<int>(pre[kPreKinds * (nfrag + 1) + s_pos]);                         \
  }                                                                                          \
  __syncthreads();                                                                           \
  const int f = s_frag;                                                                      \
  const BatFrag &fr = frags[f];                                                              \
  const int64_t local = blockIdx.x - pre[(kind) * (nfrag + 1) + s_pos];                      \
  const int64_t nloc = pre[(kind) * (nfrag + 1) + s_pos + 1] - pre[(kind) * (nfrag + 1) + s_pos];

__global__ __launch_bounds__(256) void k_bat_filter(const BatFrag *frags, const int64_t *pre, int nfrag) {
  PYST_BLOCK_FRAG(kPreFilter)
  (void)nloc;
  constexpr int NW = 256 / kWave, ITEMS = kDimTile / 256;
  __shared__ int32_t s_cnt[NW];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t wbase = local * kDimTile + int64_t{w} * kWave * ITEMS;
  int64_t rows[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) rows[j] = wbase + int64_t{j} * kWave + lane;
  int32_t kv[ITEMS];
  if (fr.kmin_b) load_keys<ITEMS>(fr.bkey, rows, fr.nb, kv);  // uniform
  bool keep[ITEMS];
  eval_preds_items<ITEMS>(fr.bpred, rows, fr.nb, keep);
  __shared__ int32_t s_min[NW], s_max[NW];
  if (fr.kmin_b) wave_key_bounds<ITEMS>(kv, keep, w, s_min, s_max);  // uniform
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
    fr.cnt[local] = tot;
    if (fr.kmin_b) {
      int32_t mn = INT32_MAX, mx = INT32_MIN;
      for (int k = 0; k < NW; ++k) {
        mn = min(mn, s_min[k]);
        mx = max(mx, s_max[k]);
      }
      fr.kmin_b[local] = mn;
      fr.kmax_b[local] = mx;
    }
  }
  int32_t *out = fr.sel + local * kDimTile;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if ((m[j] >> lane) & 1ull) out[pos + mbcnt(m[j])] = static_cast<int32_t>(wbase + int64_t{j} * kWave + lane);
    pos += __popcll(m[j]);
  }
}

// As k_fast_table_init, per fragment: the table's size and mode (direct
// addressing when the fragment allows it and its selected keys fit), cleared.
__global__ __launch_bounds__(256) void k_bat_init(const BatFrag *frags, const int64_t *pre, int nfrag) {
  PYST_BLOCK_FRAG(kPreInit)
  __shared__ int64_t s_total, s_kmin, s_kmax;
  if (threadIdx.x < kWave) {
    int64_t part = 0;
    int32_t mn = INT32_MAX, mx = INT32_MIN;
    for (int64_t b = threadIdx.x; b < fr.nblk; b += kWave) {
      part += fr.cnt[b];
      if (fr.kmin_b) {
        mn = min(mn, fr.kmin_b[b]);
        mx = max(mx, fr.kmax_b[b]);
      }
    }
    part = wave_sum(part);
    mn = wave_min_i32(mn);
    mx = wave_max_i32(mx);
    if (threadIdx.x == 0) {
      s_total = part;
      s_kmin = mn;
      s_kmax = mx;
    }
  }
  __syncthreads();
  const TableDev &t = fr.t;
  const bool direct = fr.kmin_b && direct_fits(t, s_total, s_kmin, s_kmax, int64_t{1} << kStageSlotBits);
  const int64_t range = s_kmax - s_kmin + 1;
  const int64_t cap = direct ? direct_cap(range) : table_capacity(s_total, fr.max_load, t.cap_alloc);
  const int64_t tid = local * 256 + threadIdx.x, nthr = nloc * 256;
  for (int64_t i = tid; i < kMaxSumBuckets; i += nthr) {
    reinterpret_cast<uint8_t *>(t.hdr)[kHdrAddedByte + i] = 0;
    if (fr.bp.next) fr.bp.next[i] = 0;
  }
  if (tid == 0) {
    t.hdr[0] = cap;
    t.hdr[1] = s_total;
    t.hdr[kHdrDirect] = direct;
    t.hdr[kHdrKmin] = direct ? s_kmin : 0;
    t.hdr[kHdrRange] = direct ? range : 0;
    t.hdr[kHdrDistinct] = 0;

    *fr.d_ngroups = 0;
  }
  if (direct) {  // block-uniform: the byte map and the slot sums (the bitmap is packed whole later)
    direct_clear(t, range, tid, nthr);
    clear_sums(t, cap, tid, nthr);
    return;
  }
  // 16-byte stores (a hashed table's capacity is a power of two >= 64)
  uint4 *keys = static_cast<uint4 *>(t.slots);
  const uint32_t e = static_cast<uint32_t>(kEmpty32);
  for (int64_t i = tid; i < cap / 4; i += nthr) keys[i] = uint4{e, e, e, e};
  clear_sums(t, cap, tid, nthr);
  const int64_t words = bloom_words(cap);
  for (int64_t i = tid; i < words; i += nthr) t.bloom[i] = 0;
}

// One dimension tile of one fragment per block (as k_fast_build).
__global__ __launch_bounds__(256) void k_bat_build(const BatFrag *frags, const int64_t *pre, int nfrag, uint32_t *err) {
  PYST_BLOCK_FRAG_AT(kPreBuild, xcd_block(blockIdx.x, gridDim.x))
  (void)nloc;
  if (fr.t.hdr[kHdrDirect]) build_tile_direct(fr.bkey, fr.sel, fr.cnt, fr.nb, local, fr.t, err);
  else build_tile(fr.bkey, fr.sel, fr.cnt, fr.nb, local, fr.t, err);
}

// Each fragment's Bloom filter, from its finished table (words past the ones
// its capacity uses stay clear and are never read).
__global__ __launch_bounds__(256) void k_bat_bloom(const BatFrag *frags, const int64_t *pre, int nfrag) {
  PYST_BLOCK_FRAG(kPreBloom)
  if (fr.t.hdr[kHdrDirect]) {  // the bitmap as the filter (fits the words reserved for the Bloom filter)
    const int64_t words = direct_filter_words(fr.t.hdr[kHdrRange]);
    int keys = 0;
    for (int64_t w = local * 256 + threadIdx.x; w < words; w += nloc * 256) {
      int k;
      fr.t.bloom[w] = direct_pack_word(fr.t, w, &k);
      keys += k;
    }
    add_distinct(fr.t, keys);
    return;
  }
  if (fr.t.hdr[1] > kBloomMaxKeys) return;  // the fact pass will not use it
  const int64_t words = bloom_words(fr.t.hdr[0]);
  for (int64_t w = local * 256 + threadIdx.x; w < words; w += nloc * 256) bloom_build_word(fr.t, w);
}

// A work unit of a fragment's fact rows.  The block first copies the words of
// the fragment's filter its table uses into LDS (a small table uses one word
// per slot, so a small fragment copies little).
template <int BS, bool V64>
__global__ __launch_bounds__(BS) void k_bat_fact(const BatFrag *frags, const int64_t *pre, int nfrag, uint32_t *err) {
  PYST_BLOCK_FRAG_ORDERED(kPreFact)
  (void)nloc;
  __shared__ uint32_t s_bloom[kBloomWords];
  const bool use_bloom = fr.t.hdr[1] <= kBloomMaxKeys;
  if (use_bloom) {
    const int64_t words = bloom_words(fr.t.hdr[0]);
    for (int64_t i = threadIdx.x; i < words; i += BS) s_bloom[i] = gmem(fr.t.bloom)[i];
  }
  __syncthreads();
  const int64_t begin = local * fr.rows_per_unit;
  const int64_t end = begin + fr.rows_per_unit < fr.fa.n ? begin + fr.rows_per_unit : fr.fa.n;
  star_range<0, V64, true, 4>(fr.fa, fr.t, err, (const PYST_LDS uint32_t *)s_bloom, use_bloom, begin,
                              int64_t{BS} * 4, end, nullptr, nullptr);
}

// The staged fact pass of a batch (blocks of kFastBlock threads): as the
// single star query's pass, every work unit stages its matching (slot, value)
// pairs in LDS and moves them bucket by bucket into its fragment's chunk pool,
// instead of one global atomic per matching row; k_bat_sums then adds each
// fragment's buckets up.
template <bool V64>
__global__ __launch_bounds__(kFastBlock) void k_bat_fact_staged(const BatFrag *frags, const int64_t *pre, int nfrag,
                                                                uint32_t *err) {
  PYST_BLOCK_FRAG_ORDERED(kPreFact)
  (void)nloc;
  __shared__ uint32_t s_bloom[kBloomWords];
  __shared__ uint64_t s_ent[kStageCap];
  __shared__ uint32_t s_bk[5 * kMaxBuckets + 1];
  StageLds sl;
  sl.ent = (PYST_LDS uint64_t *)s_ent;
  sl.chunk = (PYST_LDS uint32_t *)s_bk;
  sl.fill = sl.chunk + kMaxBuckets;
  sl.hist = sl.fill + kMaxBuckets;
  sl.rank = sl.hist + kMaxBuckets;
  sl.newbase = sl.rank + kMaxBuckets;
  sl.cnt = sl.newbase + kMaxBuckets;
  const BucketPool &bp = fr.bp;
  const uint32_t nb = bucket_count(fr.t.hdr[0]);
  if (local == 0 && threadIdx.x == 0 && fr.t.hdr[kHdrDirect] && fr.t.hdr[kHdrDistinct] != fr.t.hdr[1])
    latch(err, kErrDup);  // every fragment has a first unit
  if (nb <= bp.stride && threadIdx.x < bp.stride) {  // the unit's first chunks, one per bucket
    const uint32_t c = static_cast<uint32_t>(local) * bp.stride + threadIdx.x;
    bp.fill[c] = 0;
    if (threadIdx.x < nb) {
      sl.chunk[threadIdx.x] = c;
      sl.fill[threadIdx.x] = 0;
      sl.hist[threadIdx.x] = 0;
    }
  }
  if (threadIdx.x == 0) *sl.cnt = 0;
  const bool direct = fr.t.hdr[kHdrDirect] != 0;
  const bool use_bloom = direct || fr.t.hdr[1] <= kBloomMaxKeys;
  if (use_bloom) {
    const int64_t words = direct ? direct_filter_words(fr.t.hdr[kHdrRange]) : bloom_words(fr.t.hdr[0]);
    for (int64_t i = threadIdx.x; i < words; i += kFastBlock) s_bloom[i] = gmem(fr.t.bloom)[i];
  }
  __syncthreads();
  const int64_t begin = local * fr.rows_per_unit;
  const int64_t end = begin + fr.rows_per_unit < fr.fa.n ? begin + fr.rows_per_unit : fr.fa.n;
  if (direct)
    star_direct<V64, true, 4>(fr.fa, fr.t, (const PYST_LDS uint32_t *)s_bloom, begin, int64_t{kFastBlock} * 4, end,
                              &bp, &sl);
  else
    star_range<3, V64, true, 4>(fr.fa, fr.t, err, (const PYST_LDS uint32_t *)s_bloom, use_bloom, begin,
                                int64_t{kFastBlock} * 4, end, &bp, &sl);
}

// Bucket b of a staged fragment per block: its pairs and direct sums added
// up in LDS and its groups written out.
__global__ __launch_bounds__(kFastBlock) void k_bat_sums(const BatFrag *frags, const int64_t *pre, int nfrag,
                                                         uint32_t *err) {
  PYST_BLOCK_FRAG(kPreCompact)
  (void)nloc;
  __shared__ uint64_t s_sum[kBucketSlots];
  __shared__ uint32_t s_pres[kBucketSlots / 4];
  __shared__ uint32_t s_wsum[kFastBlock / kWave];
  __shared__ int64_t s_base;
  bucket_sums_block(fr.t, fr.bp, static_cast<uint32_t>(local), fr.out_keys, fr.out_sums, fr.out_cap, fr.d_ngroups,
                    err, s_sum, s_pres, s_wsum, &s_base, true);
}

__global__ __launch_bounds__(256) void k_bat_compact(const BatFrag *frags, const int64_t *pre, int nfrag, uint32_t *err) {
  PYST_BLOCK_FRAG(kPreCompact)
  // whole tiles per block, one counter atomic per tile
  constexpr int ITEMS = 8, NW = 256 / kWave;
  constexpr int64_t TILE = 256 * ITEMS;
  __shared__ int32_t s_cnt[NW];
  __shared__ int64_t s_base;
  const TableDev &t = fr.t;
  const int64_t cap = t.hdr[0];
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int64_t tile = local; tile * TILE < cap; tile += nloc) {  // block-uniform
    const int64_t wbase = tile * TILE + int64_t{w} * kWave * ITEMS;
    bool keep[ITEMS];
    int64_t key[ITEMS], sum[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int64_t s = wbase + int64_t{j} * kWave + lane;
      const int64_t sc = s < cap ? s : cap - 1;
      keep[j] = t.flags[sc] != 0 && s < cap;
      key[j] = static_cast<const int32_t *>(t.slots)[sc];
      sum[j] = static_cast<int64_t>(t.sums[sc]);
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
      s_base = tot ? static_cast<int64_t>(atomicAdd(reinterpret_cast<unsigned long long *>(fr.d_ngroups),
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
        if (p < fr.out_cap) {
          fr.out_keys[p] = key[j];
          fr.out_sums[p] = sum[j];
        } else {
          latch(err, kErrCapacity);
        }
      }
      pos += __popcll(m[j]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ host side
struct BatchPlan {
  std::vector<BatFrag> frags;
  std::vector<int64_t> pre;  // kPreKinds * (nfrag + 1)
  size_t table_bytes_total = 0, sel_bytes_total = 0, pool_bytes_total = 0;
  std::vector<int64_t> pool_chunks;  // staged: chunks of each fragment's pool
  bool staged = false;
};

// A staged batch gives each fragment a pool of pair chunks: every work unit's
// first chunk per bucket, plus shared chunks for a quarter of its fact rows
// (a fragment whose matching rows outgrow that adds the rest directly).
constexpr int64_t kBatchPoolRowShare = 8;
constexpr uint32_t kBatchChunkLg = 7;  // 128-pair chunks: a partly filled chunk per unit and bucket wastes less

static bool batch_shape(const pyst_fragment &fg, QueryShape *q, FastArgs *fa) {
  if (prepare_query(fg.plan, fg.fact, fg.nfact, q) != PYST_OK) return false;
  if (fg.plan->njoins != 1 || !q->slot_agg) return false;
  return fast_shape(fg.plan, fg.fact, *q, fa);
}

static pyst_status batch_layout(pyst_ctx *ctx, const pyst_fragment *fr, int nfrag, const pyst_tuning &tu, bool allow_staged,
                                BatchPlan *bp) {
  bp->frags.resize(nfrag);
  bp->pre.assign(static_cast<size_t>(kPreKinds) * (nfrag + 1), 0);
  const int64_t cus = ctx_num_cus(ctx);
  // Staged pair sums need kFastBlock-thread fact blocks and tables of at most
  // kMaxSumBuckets buckets (decided for the whole batch).
  bp->staged = allow_staged && tu.block == kFastBlock;
  for (int f = 0; f < nfrag && bp->staged; ++f)
    if (fr[f].plan && fr[f].plan->njoins >= 1)
      bp->staged = table_capacity_host(fr[f].plan->joins[0].key.n,
                                       tu.max_load > 0 ? tu.max_load : fr[f].plan->joins[0].max_load) <=
                   kBucketSlots * kMaxSumBuckets;
  bp->pool_chunks.assign(nfrag, 0);
  for (int f = 0; f < nfrag; ++f) {
    QueryShape q;
    FastArgs fa;
    if (!batch_shape(fr[f], &q, &fa))
      return set_error(PYST_ERR_UNSUPPORTED, "pyst_query_batch: fragments must be single-join star queries on int32 columns");
    const pyst_join_spec &js = fr[f].plan->joins[0];
    BatFrag &b = bp->frags[f];
    std::memset(&b, 0, sizeof(b));
    b.bkey = static_cast<const int32_t *>(js.key.data);
    b.nb = js.key.n;
    b.nblk = std::max<int64_t>(1, ceil_div(b.nb, kDimTile));
    b.bpred.n = js.npreds;
    for (int k = 0; k < js.npreds; ++k) {
      const int c = js.preds[k].col;
      if (c < 0 || c >= js.ncols) return set_error(PYST_ERR_ARG, "pyst_query_batch: dimension predicate names a missing column");
      b.bpred.col[k] = js.cols[c].data;
      b.bpred.is64[k] = js.cols[c].dtype == PYST_I64;
      b.bpred.op[k] = js.preds[k].cmp;
      b.bpred.val[k] = js.preds[k].value;
    }
    b.max_load = tu.max_load > 0 ? tu.max_load : js.max_load;
    b.fa = fa;
    const int64_t units = std::max<int64_t>(1, std::min<int64_t>(tu.fanout, ceil_div(fa.n, int64_t{4} * tu.block)));
    b.rows_per_unit = std::max<int64_t>(4, ceil_div(ceil_div(fa.n, units), 4) * 4);
    b.out_keys = fr[f].out_keys;
    b.out_sums = fr[f].out_sums;
    b.out_cap = fr[f].out_cap;
    b.d_ngroups = fr[f].d_ngroups;
    const int64_t cap_alloc = table_capacity_host(b.nb, b.max_load);
    b.t.cap_alloc = cap_alloc;
    b.t.slot_bytes = 4;
    bp->table_bytes_total += (table_bytes(cap_alloc, 4, true) + 255) / 256 * 256 +
                             (static_cast<size_t>(bloom_words(cap_alloc)) * 4 + 255) / 256 * 256;
    bp->sel_bytes_total += (static_cast<size_t>(b.nblk) * (kDimTile + 1) * 4 + 255 + 256) / 256 * 256 +
                           static_cast<size_t>(2 * ((b.nblk + 63) / 64 * 64)) * 4;
    const int64_t fact_units = ceil_div(std::max<int64_t>(fa.n, 1), b.rows_per_unit);
    const int64_t blocks[kPreKinds] = {
        b.nblk,
        std::max<int64_t>(1, std::min<int64_t>(ceil_div(cap_alloc, 256 * 8), 4 * cus)),
        b.nb > 0 ? b.nblk : 0,  // build: one block per dimension tile
        std::max<int64_t>(1, std::min<int64_t>(ceil_div(bloom_words(cap_alloc), 256), 4 * cus)),
        fact_units,
        bp->staged ? static_cast<int64_t>(bucket_count(cap_alloc))
                   : std::max<int64_t>(1, std::min<int64_t>(ceil_div(cap_alloc, 256 * 8), 4 * cus))};
    if (bp->staged) {
      const int64_t stride = std::min<int64_t>(kMaxBuckets, bucket_count(cap_alloc));
      const int64_t nchunks =
          fact_units * stride + ceil_div(ceil_div(fa.n, kBatchPoolRowShare), int64_t{1} << kBatchChunkLg) + 1;
      if (nchunks >= (int64_t{1} << 31)) return set_error(PYST_ERR_UNSUPPORTED, "pyst_query_batch: fragment too large");
      bp->pool_chunks[f] = nchunks;
      b.bp.nchunks = static_cast<uint32_t>(nchunks);
      b.bp.chunk_lg = kBatchChunkLg;
      b.bp.blocks = static_cast<uint32_t>(fact_units);
      b.bp.stride = static_cast<uint32_t>(stride);
      bp->pool_bytes_total +=
          kPoolHeadBytes + (static_cast<size_t>(nchunks) * ((size_t{8} << kBatchChunkLg) + 4) + 255) / 256 * 256;
    }
    for (int k = 0; k < kPreKinds; ++k) bp->pre[k * (nfrag + 1) + f + 1] = bp->pre[k * (nfrag + 1) + f] + blocks[k];
  }
  // fact blocks: fragments by work-unit size, largest first (their order follows the prefixes)
  std::vector<int> order(nfrag);
  for (int f = 0; f < nfrag; ++f) order[f] = f;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return bp->frags[x].rows_per_unit > bp->frags[y].rows_per_unit; });
  int64_t *fp = bp->pre.data() + kPreFact * (nfrag + 1);
  for (int i = 0; i < nfrag; ++i) {
    const BatFrag &b = bp->frags[order[i]];
    fp[i + 1] = fp[i] + ceil_div(std::max<int64_t>(b.fa.n, 1), b.rows_per_unit);
  }
  for (int i = 0; i < nfrag; ++i) bp->pre.push_back(order[i]);
  return PYST_OK;
}

// A laid-out batch in device memory: descriptors, block prefixes, tables and
// selections in one arena allocation, and the grid of each of its launches.
struct BatchRun {
  char *mem = nullptr;
  const BatFrag *d_frags = nullptr;
  const int64_t *d_pre = nullptr;
  unsigned grid[kPreKinds] = {};
  int nfrag = 0, block = 0;
  bool v64 = false;
  bool staged = false;  // staged pair sums (k_bat_fact_staged + k_bat_sums) instead of atomics + compaction
};

// Lays the fragments out, allocates their device memory and uploads the
// descriptors on `stream`.
static pyst_status batch_prepare(pyst_ctx *ctx, const pyst_fragment *fr, int nfrag, const pyst_tuning &tu,
                                 hipStream_t stream, BatchRun *run) {
  BatchPlan bp;
  pyst_status st = batch_layout(ctx, fr, nfrag, tu, true, &bp);
  if (st != PYST_OK) return st;
  const bool v64 = bp.frags[0].fa.v0_64 != 0;
  for (int f = 1; f < nfrag; ++f)
    if ((bp.frags[f].fa.v0_64 != 0) != v64)
      return set_error(PYST_ERR_UNSUPPORTED, "pyst_query_batch: value columns must share one dtype");
  const size_t desc_bytes = sizeof(BatFrag) * nfrag;
  const size_t pre_bytes = sizeof(int64_t) * bp.pre.size();
  const size_t meta = (desc_bytes + 255) / 256 * 256 + (pre_bytes + 255) / 256 * 256;
  char *mem = static_cast<char *>(
      ctx_alloc(ctx, meta + bp.table_bytes_total + bp.sel_bytes_total + bp.pool_bytes_total, stream));
  if (!mem && bp.staged) {  // no room for the pair pools: per-row atomics instead
    bp = BatchPlan();
    if ((st = batch_layout(ctx, fr, nfrag, tu, false, &bp)) != PYST_OK) return st;
    mem = static_cast<char *>(ctx_alloc(ctx, meta + bp.table_bytes_total + bp.sel_bytes_total, stream));
  }
  if (!mem) return set_error(PYST_ERR_NOMEM, "pyst_query_batch: arena cannot hold the batch");
  char *p = mem + meta;
  for (int f = 0; f < nfrag; ++f) {
    BatFrag &b = bp.frags[f];
    b.t = table_view(p, b.t.cap_alloc, 4, true);
    p += (table_bytes(b.t.cap_alloc, 4, true) + 255) / 256 * 256;
    b.t.bloom = reinterpret_cast<uint32_t *>(p);
    p += (static_cast<size_t>(bloom_words(b.t.cap_alloc)) * 4 + 255) / 256 * 256;
  }
  // direct addressing needs staged sums (the per-row atomic pass probes hash tables only)
  const bool allow_direct = bp.staged && !ctx_hash_join_only(ctx);
  for (int f = 0; f < nfrag; ++f) {
    BatFrag &b = bp.frags[f];
    const int64_t nblk64 = (b.nblk + 63) / 64 * 64;
    b.cnt = reinterpret_cast<int32_t *>(p);
    b.sel = b.cnt + nblk64;
    p += (static_cast<size_t>(b.nblk) * (kDimTile + 1) * 4 + 255 + 256) / 256 * 256;
    b.kmin_b = allow_direct ? reinterpret_cast<int32_t *>(p) : nullptr;
    b.kmax_b = allow_direct ? b.kmin_b + nblk64 : nullptr;
    p += static_cast<size_t>(2 * nblk64) * 4;
  }
  for (int f = 0; f < nfrag && bp.staged; ++f) {  // pools: per-bucket counters, records, fills
    BatFrag &b = bp.frags[f];
    const size_t nchunks = static_cast<size_t>(bp.pool_chunks[f]);
    b.bp.next = reinterpret_cast<uint32_t *>(p);
    b.bp.rec = reinterpret_cast<uint64_t *>(p + kPoolHeadBytes);
    b.bp.fill = reinterpret_cast<uint32_t *>(b.bp.rec + (nchunks << kBatchChunkLg));
    p += kPoolHeadBytes + (nchunks * ((size_t{8} << kBatchChunkLg) + 4) + 255) / 256 * 256;
  }
  // Descriptors go up through pinned staging (a pageable copy would stall other streams).
  char *stage = ctx_pinned_staging(ctx, meta);
  if (!stage) {
    ctx_free(ctx, mem, stream);
    return set_error(PYST_ERR_NOMEM, "pyst_query_batch: pinned staging");
  }
  std::memcpy(stage, bp.frags.data(), desc_bytes);
  std::memcpy(stage + (desc_bytes + 255) / 256 * 256, bp.pre.data(), pre_bytes);
  hipError_t e = hipMemcpyAsync(mem, stage, meta, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = ctx_staging_record(ctx, stream);
  if (e != hipSuccess) {
    ctx_free(ctx, mem, stream);
    return hip_error(e, "pyst_query_batch: descriptor upload");
  }
  run->mem = mem;
  run->d_frags = reinterpret_cast<const BatFrag *>(mem);
  run->d_pre = reinterpret_cast<const int64_t *>(mem + (desc_bytes + 255) / 256 * 256);
  for (int k = 0; k < kPreKinds; ++k) run->grid[k] = static_cast<unsigned>(bp.pre[k * (nfrag + 1) + nfrag]);
  run->nfrag = nfrag;
  run->block = tu.block;
  run->v64 = v64;
  run->staged = bp.staged;
  return PYST_OK;
}

// The batch's six launches (also what a captured batch graph holds).
static hipError_t batch_enqueue(const BatchRun &r, uint32_t *err, hipStream_t stream) {
  const BatFrag *d_frags = r.d_frags;
  const int64_t *d_pre = r.d_pre;
  const int nfrag = r.nfrag;
  k_bat_filter<<<r.grid[kPreFilter], 256, 0, stream>>>(d_frags, d_pre, nfrag);
  k_bat_init<<<r.grid[kPreInit], 256, 0, stream>>>(d_frags, d_pre, nfrag);
  if (r.grid[kPreBuild] > 0) k_bat_build<<<r.grid[kPreBuild], 256, 0, stream>>>(d_frags, d_pre, nfrag, err);
  k_bat_bloom<<<r.grid[kPreBloom], 256, 0, stream>>>(d_frags, d_pre, nfrag);
#define PYST_BAT_FACT(BS_)                                                                                      \
  if (r.block == BS_) {                                                                                       \
    if (r.v64) k_bat_fact<BS_, true><<<r.grid[kPreFact], BS_, 0, stream>>>(d_frags, d_pre, nfrag, err);        \
    else k_bat_fact<BS_, false><<<r.grid[kPreFact], BS_, 0, stream>>>(d_frags, d_pre, nfrag, err);             \
  }
  if (r.staged) {
    if (r.v64) k_bat_fact_staged<true><<<r.grid[kPreFact], kFastBlock, 0, stream>>>(d_frags, d_pre, nfrag, err);
    else k_bat_fact_staged<false><<<r.grid[kPreFact], kFastBlock, 0, stream>>>(d_frags, d_pre, nfrag, err);
    k_bat_sums<<<r.grid[kPreCompact], kFastBlock, 0, stream>>>(d_frags, d_pre, nfrag, err);
    return hipGetLastError();
  }
  PYST_BAT_FACT(256)
  PYST_BAT_FACT(512)
  PYST_BAT_FACT(1024)
#undef PYST_BAT_FACT
  k_bat_compact<<<r.grid[kPreCompact], 256, 0, stream>>>(d_frags, d_pre, nfrag, err);
  return hipGetLastError();
}

static pyst_status batch_run(pyst_ctx *ctx, const pyst_fragment *fr, int nfrag, const pyst_tuning &tu,
                             hipStream_t stream) {
  BatchRun r;
  pyst_status st = batch_prepare(ctx, fr, nfrag, tu, stream, &r);
  if (st != PYST_OK) return st;
  hipError_t e;
  {
    TimedRegion timed(ctx, "batch", stream);
    e = batch_enqueue(r, ctx_err_word(ctx), stream);
  }
  ctx_free(ctx, r.mem, stream);
  if (e != hipSuccess) return hip_error(e, "pyst_query_batch: launch");
  return PYST_OK;
}

}  // namespace pyst

struct pyst_batch_graph {
  pyst_ctx *ctx = nullptr;
  char *mem = nullptr;  // the batch's arena memory, held while the graph exists
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace pyst {

static pyst_status check_fragments(const pyst_fragment *frags, int nfrag, const char *who) {
  for (int f = 0; f < nfrag; ++f)
    if (!frags[f].plan || !frags[f].fact || !frags[f].d_ngroups || frags[f].out_cap < 0 ||
        (frags[f].out_cap > 0 && (!frags[f].out_keys || !frags[f].out_sums)))
      return set_error(PYST_ERR_ARG, who);
  return PYST_OK;
}

static bool tuning_ok(const pyst_tuning &t) {
  return (t.block == 256 || t.block == 512 || t.block == 1024) && t.fanout >= 1 && t.fanout <= 65536 &&
         (t.max_load == 0.0 || (t.max_load > 0.0 && t.max_load <= 0.95));
}

}  // namespace pyst

using namespace pyst;

extern "C" {

pyst_status pyst_query_batch(pyst_ctx *ctx, const pyst_fragment *frags, int nfrag, const pyst_tuning *tuning,
                             hipStream_t stream) {
  if (!ctx || (!frags && nfrag > 0) || nfrag < 0) return set_error(PYST_ERR_ARG, "pyst_query_batch: NULL argument");
  if (nfrag == 0) return PYST_OK;
  pyst_tuning tu = tuning ? *tuning : pyst_tuning{64, 512, 0.0};
  if (!tuning_ok(tu)) return set_error(PYST_ERR_ARG, "pyst_query_batch: tuning fanout 1..65536, block 256/512/1024, max_load 0 or (0, 0.95]");
  const pyst_status st = check_fragments(frags, nfrag, "pyst_query_batch: bad fragment");
  if (st != PYST_OK) return st;
  return batch_run(ctx, frags, nfrag, tu, stream);
}

pyst_status pyst_batch_graph_create(pyst_ctx *ctx, const pyst_fragment *frags, int nfrag, const pyst_tuning *tuning,
                                    hipStream_t stream, pyst_batch_graph **out) {
  if (!ctx || !frags || nfrag <= 0 || !out) return set_error(PYST_ERR_ARG, "pyst_batch_graph_create: NULL argument");
  *out = nullptr;
  pyst_tuning tu = tuning ? *tuning : pyst_tuning{64, 512, 0.0};
  if (!tuning_ok(tu)) return set_error(PYST_ERR_ARG, "pyst_batch_graph_create: bad tuning");
  pyst_status st = check_fragments(frags, nfrag, "pyst_batch_graph_create: bad fragment");
  if (st != PYST_OK) return st;
  BatchRun r;
  st = batch_prepare(ctx, frags, nfrag, tu, stream, &r);
  if (st != PYST_OK) return st;
  auto fail = [&](hipError_t e, const char *what, hipStream_t cs, hipGraph_t g) {
    if (g) (void)hipGraphDestroy(g);
    if (cs) (void)hipStreamDestroy(cs);
    (void)hipStreamSynchronize(stream);
    ctx_free(ctx, r.mem, stream);
    return hip_error(e, what);
  };
  // the descriptors must be on the device before the graph may run
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(e, "pyst_batch_graph_create: descriptor upload", nullptr, nullptr);
  hipStream_t cs = nullptr;
  if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
    return fail(e, "pyst_batch_graph_create: stream", nullptr, nullptr);
  if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return fail(e, "pyst_batch_graph_create: begin capture", cs, nullptr);
  const hipError_t le = batch_enqueue(r, ctx_err_word(ctx), cs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(cs, &g);
  if (le != hipSuccess) return fail(le, "pyst_batch_graph_create: launch", cs, g);
  if (e != hipSuccess) return fail(e, "pyst_batch_graph_create: end capture", cs, g);
  hipGraphExec_t x = nullptr;
  if ((e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0)) != hipSuccess)
    return fail(e, "pyst_batch_graph_create: instantiate", cs, g);
  (void)hipStreamDestroy(cs);
  auto *bg = new (std::nothrow) pyst_batch_graph;
  if (!bg) {
    (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    ctx_free(ctx, r.mem, stream);
    return set_error(PYST_ERR_NOMEM, "pyst_batch_graph_create: host memory");
  }
  bg->ctx = ctx;
  bg->mem = r.mem;
  bg->graph = g;
  bg->exec = x;
  *out = bg;
  return PYST_OK;
}

pyst_status pyst_batch_graph_launch(pyst_batch_graph *g, hipStream_t stream) {
  if (!g) return set_error(PYST_ERR_ARG, "pyst_batch_graph_launch: NULL graph");
  const hipError_t e = hipGraphLaunch(g->exec, stream);
  return e == hipSuccess ? PYST_OK : hip_error(e, "pyst_batch_graph_launch");
}

pyst_status pyst_batch_graph_destroy(pyst_batch_graph *g) {
  if (!g) return PYST_OK;
  const hipError_t e = hipDeviceSynchronize();  // no launch of the graph may still run
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  ctx_free_eager(g->ctx, g->mem, nullptr);
  delete g;
  return e == hipSuccess ? PYST_OK : hip_error(e, "pyst_batch_graph_destroy");
}

pyst_status pyst_autotune(pyst_ctx *ctx, const pyst_fragment *frags, int nfrag, int reps, pyst_tuning *out,
                          double *best_ms) {
  if (!ctx || !frags || nfrag <= 0 || !out) return set_error(PYST_ERR_ARG, "pyst_autotune: NULL argument");
  if (reps < 1) reps = 1;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return set_error(PYST_ERR_HIP, "pyst_autotune: stream");
  hipEvent_t a = nullptr, b = nullptr;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  const int fanouts[] = {16, 32, 64, 128, 256};
  const int blocks[] = {256, 512, 1024};
  const double loads[] = {0.5, 0.7};
  double best = 1e30;
  pyst_tuning best_t{64, 512, 0.5};
  pyst_status st = PYST_OK;
  for (double ld : loads)
    for (int bs : blocks)
      for (int fo : fanouts) {
        const pyst_tuning t{fo, bs, ld};
        st = batch_run(ctx, frags, nfrag, t, s);  // warm-up
        if (st != PYST_OK) break;
        (void)hipEventRecord(a, s);
        for (int r = 0; r < reps && st == PYST_OK; ++r) st = batch_run(ctx, frags, nfrag, t, s);
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (st == PYST_OK && ms / reps < best) {
          best = ms / reps;
          best_t = t;
        }
      }
  (void)hipStreamSynchronize(s);
  ctx_stream_idle(ctx, s);  // before the private stream goes away
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipStreamDestroy(s);
  if (st != PYST_OK) return st;
  *out = best_t;
  if (best_ms) *best_ms = best;
  return PYST_OK;
}

}  // extern "C"

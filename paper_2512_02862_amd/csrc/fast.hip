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
constexpr int kBufferDword3 = 0x00020000;           // raw buffer resource word 3 on CDNA

__device__ __forceinline__ uint32_t bloom_hash(int32_t k) { return fmix32(static_cast<uint32_t>(k) ^ 0x9e3779b9u); }
__device__ __forceinline__ uint32_t bloom_word(uint32_t h) { return h & (kBloomWords - 1); }
__device__ __forceinline__ uint32_t bloom_bits(uint32_t h) { return (1u << ((h >> 17) & 31)) | (1u << ((h >> 22) & 31)); }

template <typename T>
__device__ __forceinline__ const PYST_GLOBAL T *gmem(const T *p) { return (const PYST_GLOBAL T *)p; }

// ------------------------------------------------------------------ dimension filter (block-local)
// Block b writes its selected row ids, in order, to sel[b*kDimTile ...] and their
// number to cnt[b]; no global counter.
__global__ __launch_bounds__(256) void k_dim_filter(PredSet ps, int64_t n, int32_t *sel, int32_t *cnt) {
  constexpr int NW = 256 / kWave, ITEMS = kDimTile / 256;
  __shared__ int32_t s_cnt[NW];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t wbase = int64_t{blockIdx.x} * kDimTile + int64_t{w} * kWave * ITEMS;
  int64_t rows[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) rows[j] = wbase + int64_t{j} * kWave + lane;
  bool keep[ITEMS];
  eval_preds_items<ITEMS>(ps, rows, n, keep);
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
  }
  int32_t *out = sel + int64_t{blockIdx.x} * kDimTile;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if ((m[j] >> lane) & 1ull) out[pos + mbcnt(m[j])] = static_cast<int32_t>(wbase + int64_t{j} * kWave + lane);
    pos += __popcll(m[j]);
  }
}

// Table initialization sized from the per-block counts (or n without a filter);
// also clears the Bloom words and the caller's group/pair counters.
__global__ void k_fast_table_init(TableDev t, const int32_t *cnt, int64_t nblocks, int64_t n, double max_load,
                                  int64_t *zero0, int64_t *zero1) {
  __shared__ int64_t s_total;
  if (threadIdx.x < kWave) {
    int64_t part = 0;
    if (cnt)
      for (int64_t b = threadIdx.x; b < nblocks; b += kWave) part += cnt[b];
    part = wave_sum(part);
    if (threadIdx.x == 0) s_total = cnt ? part : n;
  }
  __syncthreads();
  const int64_t total = s_total;
  const int64_t cap = table_capacity(total, max_load, t.cap_alloc);
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0) {
    t.hdr[0] = cap;
    t.hdr[1] = total;
    if (zero0) *zero0 = 0;
    if (zero1) *zero1 = 0;
  }
  const int64_t words = t.slot_bytes == 4 ? cap / 2 : cap;
  const uint64_t fillv = t.slot_bytes == 4 ? (uint64_t{static_cast<uint32_t>(kEmpty32)} * 0x100000001ull)
                                           : uint64_t{static_cast<uint32_t>(kEmpty32)};
  uint64_t *p = static_cast<uint64_t *>(t.slots);
  for (int64_t i = tid; i < words; i += nthr) p[i] = fillv;
  if (t.sums)
    for (int64_t i = tid; i < cap; i += nthr) {
      t.sums[i] = 0;
      t.flags[i] = 0;
    }
  if (t.bloom)
    for (int64_t i = tid; i < kBloomWords; i += nthr) t.bloom[i] = 0;
}

// Build from a block-local selection (or all rows); sets the Bloom bits too.
template <int SB>
__global__ __launch_bounds__(256) void k_fast_build(const int32_t *key, const int32_t *payload, const int32_t *sel,
                                                    const int32_t *cnt, int64_t n, TableDev t, uint32_t *err) {
  const int64_t mask = t.hdr[0] - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
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
    if (t.bloom) {
      const uint32_t h = bloom_hash(k);
      atomicOr(&t.bloom[bloom_word(h)], bloom_bits(h));
    }
    bool done = false;
    if (SB == 4) {
      // A fresh table is mostly empty: try the CAS first instead of reading the slot.
      int32_t *keys = static_cast<int32_t *>(t.slots);
      int64_t s = (table_hash32(k) & mask) & ~int64_t{3};
      for (int64_t step = 0; step <= mask; ++step) {
        const int32_t cur = atomicCAS(&keys[s], kEmpty32, k);
        if (cur == kEmpty32) {
          done = true;
          break;
        }
        if (cur == k) {
          latch(err, kErrDup);
          done = true;
          break;
        }
        s = (s + 1) & mask;
      }
    } else {
      uint64_t *slots = static_cast<uint64_t *>(t.slots);
      const uint64_t empty = static_cast<uint32_t>(kEmpty32);
      const uint64_t packed = uint64_t{static_cast<uint32_t>(k)} |
                              (uint64_t{static_cast<uint32_t>(payload ? payload[row] : static_cast<int32_t>(row))} << 32);
      int64_t s = (table_hash32(k) & mask) & ~int64_t{1};
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
    }
    if (!done) latch(err, kErrTableFull);
  }
}

// ------------------------------------------------------------------ the fact pass
__device__ __forceinline__ v4i32 ld4(const int32_t *p, int64_t base) {
  return __builtin_nontemporal_load(reinterpret_cast<const PYST_GLOBAL v4i32 *>(gmem(p) + base));
}

// First match of k in a 16-byte group of 4 keys: index, or -1 (none), and whether it holds EMPTY.
__device__ __forceinline__ int match4(v4i32 q, int32_t k, bool *empty) {
  *empty = q.x == kEmpty32 || q.y == kEmpty32 || q.z == kEmpty32 || q.w == kEmpty32;
  return q.x == k ? 0 : q.y == k ? 1 : q.z == k ? 2 : q.w == k ? 3 : -1;
}

#define PYST_LDS __attribute__((address_space(3)))

// The fact pass over rows [begin + 4*threadIdx.x, end) in steps of `step` rows;
// s_bloom is the block's LDS copy of join 0's filter (used when use_bloom).
template <int NJ, int SB1, int AGG, bool V64>
__device__ __forceinline__ void fact_range(const FastArgs &a, const TableDev &t0, const TableDev &t1, const GroupDev &g,
                                           const PairsOut &po, uint32_t *err, const PYST_LDS uint32_t *s_bloom,
                                           bool use_bloom, int64_t begin, int64_t step, int64_t end) {
  const int64_t cap0 = t0.hdr[0], mask0 = cap0 - 1;
  const int64_t cap1 = NJ > 1 ? t1.hdr[0] : 4, mask1 = cap1 - 1;
  const int64_t gmask = AGG == 1 ? g.hdr[0] - 1 : 0;
  const __amdgpu_buffer_rsrc_t r0 =
      __builtin_amdgcn_make_buffer_rsrc(t0.slots, 0, static_cast<int>(cap0 * 4), kBufferDword3);
  const __amdgpu_buffer_rsrc_t r1 =
      __builtin_amdgcn_make_buffer_rsrc(NJ > 1 ? t1.slots : t0.slots, 0, static_cast<int>(cap1 * SB1), kBufferDword3);
  const int64_t n = end;
  int64_t wpos = 0, wend = 0;  // the wave's pair run (AGG 2), wave-uniform
  // The loop is wave-uniform (lanes past the end have no live rows), so the
  // wave-level state above stays consistent across lanes.
  const int64_t wofs = int64_t{threadIdx.x & ~(kWave - 1)} * 4, lofs = int64_t{threadIdx.x & (kWave - 1)} * 4;
  for (int64_t wbase = begin + wofs; wbase < n; wbase += step) {
    const int64_t base = wbase + lofs;
    const bool full = base + 4 <= n;
    v4i32 f0 = 0, f1 = 0, c0 = 0, c1 = 0, w1 = 0;
    int64_t x0[4] = {0, 0, 0, 0};
    if (full) {
      f0 = ld4(a.fk[0], base);
      if (NJ > 1) f1 = ld4(a.fk[1], base);
      if (a.npred > 0 && a.psrc[0] == 0) c0 = ld4(a.pcol[0], base);
      if (a.npred > 1 && a.psrc[1] == 0) c1 = ld4(a.pcol[1], base);
      if (V64) {
        const v2i64 lo = __builtin_nontemporal_load(reinterpret_cast<const PYST_GLOBAL v2i64 *>(gmem(static_cast<const int64_t *>(a.v0)) + base));
        const v2i64 hi = __builtin_nontemporal_load(reinterpret_cast<const PYST_GLOBAL v2i64 *>(gmem(static_cast<const int64_t *>(a.v0)) + base + 2));
        x0[0] = lo.x; x0[1] = lo.y; x0[2] = hi.x; x0[3] = hi.y;
      } else {
        const v4i32 v = ld4(static_cast<const int32_t *>(a.v0), base);
        x0[0] = v.x; x0[1] = v.y; x0[2] = v.z; x0[3] = v.w;
      }
      if (a.vexpr == PYST_V_COL_TIMES_C_MINUS) w1 = ld4(a.v1, base);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (base + r >= n) continue;
        f0[r] = a.fk[0][base + r];
        if (NJ > 1) f1[r] = a.fk[1][base + r];
        if (a.npred > 0 && a.psrc[0] == 0) c0[r] = a.pcol[0][base + r];
        if (a.npred > 1 && a.psrc[1] == 0) c1[r] = a.pcol[1][base + r];
        x0[r] = V64 ? static_cast<const int64_t *>(a.v0)[base + r] : static_cast<const int32_t *>(a.v0)[base + r];
        if (a.vexpr == PYST_V_COL_TIMES_C_MINUS) w1[r] = a.v1[base + r];
      }
    }
    bool live[4];
    int32_t s0[4];
    v4i32 q0[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      bool l = base + r < n;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        if (k < a.npred) {
          const int32_t x = a.psrc[k] == 0 ? (k == 0 ? c0[r] : c1[r])
                            : a.psrc[k] == 1 ? f0[r] : a.psrc[k] == 2 ? f1[r] : w1[r];
          l = l && compare_op(x, a.pop[k], a.pval[k]);
        }
      }
      if (use_bloom) {
        const uint32_t h = bloom_hash(f0[r]);
        const uint32_t m = bloom_bits(h);
        l = l && (s_bloom[bloom_word(h)] & m) == m;
      }
      live[r] = l;
      s0[r] = static_cast<int32_t>((table_hash32(f0[r]) & mask0) & ~int64_t{3});
      q0[r] = __builtin_amdgcn_raw_buffer_load_b128(r0, l ? s0[r] * 4 : kBufOob, 0, 0);
    }
    int32_t slot0[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      bool empty;
      const int hit = match4(q0[r], f0[r], &empty);
      slot0[r] = live[r] && hit >= 0 ? s0[r] + hit : -1;
      if (live[r] && hit < 0 && !empty) {  // the run continues past the first group (rare)
        int32_t s = s0[r];
        for (int64_t step = 4; step <= mask0; step += 4) {
          s = static_cast<int32_t>((s + 4) & mask0);
          const int h2 = match4(__builtin_amdgcn_raw_buffer_load_b128(r0, s * 4, 0, 0), f0[r], &empty);
          if (h2 >= 0) {
            slot0[r] = s + h2;
            break;
          }
          if (empty) break;
        }
      }
    }
    int32_t pay1[4] = {0, 0, 0, 0};
    if (NJ > 1) {
      int32_t s1[4];
      v4i32 q1[4];
      constexpr int GS = 16 / SB1;  // slots per 16-byte load
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        s1[r] = static_cast<int32_t>((table_hash32(f1[r]) & mask1) & ~int64_t{GS - 1});
        q1[r] = __builtin_amdgcn_raw_buffer_load_b128(r1, slot0[r] >= 0 ? s1[r] * SB1 : kBufOob, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int32_t k = f1[r];
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
          for (int64_t step = GS; step <= mask1; step += GS) {
            s = static_cast<int32_t>((s + GS) & mask1);
            const v4i32 q = __builtin_amdgcn_raw_buffer_load_b128(r1, s * SB1, 0, 0);
            int st;
            if (SB1 == 4) {
              bool empty;
              const int h = match4(q, k, &empty);
              st = h >= 0 ? 1 : (empty ? 0 : -1);
            } else {
              st = q.x == k ? 1 : q.x == kEmpty32 ? 0 : q.z == k ? 2 : q.z == kEmpty32 ? 0 : -1;
              pl = st == 1 ? q.y : q.w;
              st = st == 2 ? 1 : st;
            }
            if (st >= 0) {
              state = st;
              break;
            }
          }
        }
        if (state != 1) slot0[r] = -1;
        pay1[r] = pl;
      }
    }
    int64_t val[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
      val[r] = a.vexpr == PYST_V_COL ? x0[r]
                                     : static_cast<int64_t>(static_cast<uint64_t>(x0[r]) *
                                                            static_cast<uint64_t>(a.vconst - static_cast<int64_t>(w1[r])));
    if (AGG == 0) {
      uint64_t old[4] = {1, 1, 1, 1};
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (slot0[r] >= 0) old[r] = atomicAdd(reinterpret_cast<unsigned long long *>(&t0.sums[slot0[r]]),
                                              static_cast<unsigned long long>(val[r]));
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (slot0[r] >= 0 && old[r] == 0) t0.flags[slot0[r]] = 1;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool hit = slot0[r] >= 0;
        int64_t gkey = 0;
        if (hit) {
          const int64_t lo = a.lo_src == PYST_G_JOIN_KEY ? (a.lo_idx == 0 ? f0[r] : f1[r]) : pay1[r];
          if (a.hi_src == PYST_G_NONE) {
            gkey = lo;
          } else {
            const int64_t hi = a.hi_src == PYST_G_JOIN_KEY ? (a.hi_idx == 0 ? f0[r] : f1[r]) : pay1[r];
            gkey = static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | static_cast<uint32_t>(lo));
          }
          if (gkey == kEmpty64) latch(err, kErrKey);
        }
        if (AGG == 1) {
          if (hit && gkey != kEmpty64 && !group_add(g.slots, gmask, gkey, static_cast<uint64_t>(val[r])))
            latch(err, kErrTableFull);
        } else {
          // Pairs go to the wave's current run of kPairRun slots; a new run is
          // reserved with one atomic when it fills (a counter bumped by every
          // wave for every group of rows serializes the whole pass).
          const uint64_t m = __ballot(hit);
          const int c = __popcll(m);
          if (c) {
            if (wpos + c > wend) {
              for (int64_t p = wpos + lane_id(); p < wend; p += kWave) po.keys[p] = kEmpty64;
              unsigned long long rb = 0;
              if (lane_id() == 0)
                rb = atomicAdd(reinterpret_cast<unsigned long long *>(po.count), static_cast<unsigned long long>(kPairRun));
              rb = __shfl(rb, 0);
              wpos = static_cast<int64_t>(rb);
              wend = wpos + kPairRun;
            }
            if (hit) {
              const int64_t p = wpos + mbcnt(m);
              if (p < po.cap) {
                po.keys[p] = gkey;
                po.vals[p] = val[r];
              }
            }
            wpos += c;
          }
        }
      }
    }
  }
  if (AGG == 2)
    for (int64_t p = wpos + lane_id(); p < wend; p += kWave)
      if (p < po.cap) po.keys[p] = kEmpty64;
}

template <int NJ, int SB1, int AGG, bool V64>
__global__ __launch_bounds__(kFastBlock) void k_fast_fact(FastArgs a, TableDev t0, TableDev t1, GroupDev g, PairsOut po,
                                                         uint32_t *err) {
  __shared__ uint32_t s_bloom[kBloomWords];
  const bool use_bloom = t0.bloom != nullptr && t0.hdr[1] <= kBloomMaxKeys;
  if (use_bloom) {
    for (int i = threadIdx.x; i < kBloomWords; i += kFastBlock) s_bloom[i] = gmem(t0.bloom)[i];
    __syncthreads();
  }
  fact_range<NJ, SB1, AGG, V64>(a, t0, t1, g, po, err, (const PYST_LDS uint32_t *)s_bloom, use_bloom,
                                int64_t{blockIdx.x} * kFastBlock * 4, int64_t{gridDim.x} * kFastBlock * 4, a.n);
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
  fa->npred = plan->npreds;
  for (int k = 0; k < plan->npreds; ++k) {
    const int c = plan->preds[k].col;
    if (fact[c].dtype != PYST_I32) return false;
    fa->pop[k] = plan->preds[k].cmp;
    fa->pval[k] = plan->preds[k].value;
    if (c == plan->joins[0].probe_col) fa->psrc[k] = 1;
    else if (plan->njoins > 1 && c == plan->joins[1].probe_col) fa->psrc[k] = 2;
    else if (plan->vexpr == PYST_V_COL_TIMES_C_MINUS && c == plan->v1) fa->psrc[k] = 3;
    else {
      fa->psrc[k] = 0;
      fa->pcol[k] = static_cast<const int32_t *>(fact[c].data);
    }
  }
  fa->n = fact[0].n;
  // buffer resources address at most 2^31 bytes of a table
  for (int j = 0; j < plan->njoins; ++j) {
    const int sb = (j == 1 && q.need_payload[1]) ? 8 : 4;
    if (table_capacity_host(plan->joins[j].key.n, plan->joins[j].max_load) * sb >= (int64_t{1} << 31)) return false;
  }
  return true;
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
  if (st == PYST_OK) st = fast_build_dimensions(ctx, plan, q, &d, d_ngroups, s.po.count, stream);
  if (st == PYST_OK) st = fast_fact_pass(ctx, plan->njoins, q.agg_mode, fa, d, s.g, s.po, stream);
  if (st == PYST_OK) st = fast_finish(ctx, plan, q, d, &s, out_keys, out_sums, out_cap, d_ngroups, stream);
  ctx_free(ctx, s.mem, stream);
  free_dimensions(ctx, &d, stream);
  return st;
}

// Dimension tables of the fast path: join 0 keys-only with a Bloom filter.
pyst_status fast_build_dimensions(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, DimTables *d,
                                  int64_t *zero0, int64_t *zero1, hipStream_t stream) {
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
    int32_t *cnt = nullptr;
    const int64_t nblk = std::max<int64_t>(1, ceil_div(nb, kDimTile));
    if (js.npreds > 0) {
      d->sel_mem[j] = ctx_alloc(ctx, static_cast<size_t>(nblk) * (kDimTile + 1) * sizeof(int32_t) + 256, stream);
      if (!d->sel_mem[j]) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (dimension selection)");
      cnt = static_cast<int32_t *>(d->sel_mem[j]);
      int32_t *s = cnt + (nblk + 63) / 64 * 64;
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
      k_dim_filter<<<static_cast<unsigned>(nblk), 256, 0, stream>>>(ps, nb, s, cnt);
      PYST_LAUNCH_CHECK("k_dim_filter");
      sel = s;
    }
    const int iblocks = static_cast<int>(std::min<int64_t>(std::max<int64_t>(ceil_div(cap_alloc, 256), 64), 2048));
    k_fast_table_init<<<iblocks, 256, 0, stream>>>(d->t[j], cnt, nblk, nb, js.max_load, j == 0 ? zero0 : nullptr,
                                                   j == 0 ? zero1 : nullptr);
    PYST_LAUNCH_CHECK("k_fast_table_init");
    if (nb > 0) {
      // one row per thread: each insert is a chain of dependent memory operations
      const int blocks = static_cast<int>(std::min<int64_t>(ceil_div(nb, 256), int64_t{1} << 20));
      const int32_t *key = static_cast<const int32_t *>(js.key.data);
      const int32_t *pay = static_cast<const int32_t *>(js.payload.data);
      if (sb == 4) k_fast_build<4><<<blocks, 256, 0, stream>>>(key, pay, sel, cnt, nb, d->t[j], ctx_err_word(ctx));
      else k_fast_build<8><<<blocks, 256, 0, stream>>>(key, pay, sel, cnt, nb, d->t[j], ctx_err_word(ctx));
      PYST_LAUNCH_CHECK("k_fast_build");
    }
  }
  return PYST_OK;
}

// One 1024-thread block per CU (the 128 KiB Bloom filter takes most of the LDS).
int fast_grid(pyst_ctx *ctx, int64_t n) {
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 4 * kFastBlock), ctx_num_cus(ctx))));
}

template <int NJ, int SB1, int AGG, bool V64>
static void launch_fast(int grid, const FastArgs &a, const DimTables &d, const GroupDev &g, const PairsOut &po,
                        uint32_t *err, hipStream_t stream) {
  k_fast_fact<NJ, SB1, AGG, V64><<<grid, kFastBlock, 0, stream>>>(a, d.t[0], d.t[1], g, po, err);
}

pyst_status fast_fact_pass(pyst_ctx *ctx, int njoins, int agg_mode, const FastArgs &a, const DimTables &d,
                           const GroupDev &g, const PairsOut &po, hipStream_t stream) {
  if (a.n <= 0) return PYST_OK;
  const int grid = fast_grid(ctx, a.n);
  uint32_t *err = ctx_err_word(ctx);
  const int sb1 = njoins > 1 ? d.t[1].slot_bytes : 4;
  const bool v64 = a.v0_64 != 0;
  TimedRegion timed(ctx, "fact_pass", stream);
#define PYST_FAST_CASE(NJ_, S1_, AG_)                                                    \
  if (njoins == NJ_ && sb1 == S1_ && agg_mode == AG_) {                                 \
    if (v64) launch_fast<NJ_, S1_, AG_, true>(grid, a, d, g, po, err, stream);           \
    else launch_fast<NJ_, S1_, AG_, false>(grid, a, d, g, po, err, stream);              \
    PYST_LAUNCH_CHECK("k_fast_fact");                                                   \
    return PYST_OK;                                                                     \
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

// Group-by over materialized pairs, then unordered compaction.  *d_ngroups is
// cleared here, on the stream, before the compaction adds to it.
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
  GroupDev g = s->g;
  void *gm = nullptr;
  if (q.agg_mode == 2) {
    const int64_t cap = table_capacity_host(s->po.cap, plan->group_max_load);
    gm = ctx_alloc(ctx, group_bytes(cap), stream);
    if (!gm) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (group table)");
    g = group_view(gm, cap);
    pyst_status st = group_init(g, s->po.count, s->po.cap, 0, plan->group_max_load, stream);
    if (st != PYST_OK) {
      ctx_free(ctx, gm, stream);
      return st;
    }
    const int blocks = grid_for(ctx, s->po.cap, 256, 8);
    k_gb_insert<<<blocks, 256, 0, stream>>>(s->po.keys, 1, s->po.vals, 1, nullptr, s->po.count, s->po.cap, g,
                                            ctx_err_word(ctx), 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      ctx_free(ctx, gm, stream);
      return hip_error(e, "k_gb_insert");
    }
  }
  k_compact_unordered<false><<<cgrid, 256, 0, stream>>>(TableDev{}, g, out_keys, out_sums, out_cap, d_ngroups,
                                                       ctx_err_word(ctx));
  hipError_t e = hipGetLastError();
  if (gm) ctx_free(ctx, gm, stream);
  if (e != hipSuccess) return hip_error(e, "k_compact_unordered");
  return PYST_OK;
}

}  // namespace pyst

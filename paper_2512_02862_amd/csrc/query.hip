// Fused filter + join + group-by SUM over a fact table (one build pass per
// dimension, then one pass over the fact columns).
//
// The paper runs filter, partition, build/probe and aggregation as separate
// tensor operators (Sec. 3.1, "A Naive Implementation in PyTorch"); here the
// probe-side operators are fused into one kernel so the fact columns cross HBM
// exactly once, which is what bounds the query on this chip.
#include <algorithm>
#include <cstring>

#include "pyst_internal.h"
#include "query.h"
#include "table.h"

namespace pyst {

// ------------------------------------------------------------------ device helpers
__device__ __forceinline__ int64_t pick(const int64_t (&v)[kMaxFactCols][4], int slot, int r) {
  int64_t x = v[0][r];
#pragma unroll
  for (int c = 1; c < kMaxFactCols; ++c) x = slot == c ? v[c][r] : x;
  return x;
}

// Load 4 consecutive rows [base, base+4) of a column as int64 (16-byte vector loads
// when the group is complete, guarded scalar loads at the tail).
__device__ __forceinline__ void load4(const void *p, int is64, int64_t base, int64_t n, int64_t (&o)[4]) {
  if (base + 4 <= n) {
    if (is64) {
      const v2i64 a = __builtin_nontemporal_load(reinterpret_cast<const v2i64 *>(static_cast<const int64_t *>(p) + base));
      const v2i64 b = __builtin_nontemporal_load(reinterpret_cast<const v2i64 *>(static_cast<const int64_t *>(p) + base + 2));
      o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    } else {
      const v4i32 a = __builtin_nontemporal_load(reinterpret_cast<const v4i32 *>(static_cast<const int32_t *>(p) + base));
      o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = base + r < n ? load_as_i64(p, is64, base + r) : 0;
  }
}

// Find key k in a join table.  Returns the slot index or -1; *pay gets the payload
// (8-byte layout only).  Probes 4 (or 2) slots per 16-byte load.
template <int SLOT_BYTES>
__device__ __forceinline__ int64_t find_slot(const TableDev &t, int64_t mask, int32_t k, int32_t *pay) {
  if (SLOT_BYTES == 4) {
    const int32_t *keys = static_cast<const int32_t *>(t.slots);
    int64_t s = (table_hash32(k) & mask) & ~int64_t{3};
    for (int64_t step = 0; step <= mask; step += 4) {
      const int4 q = *reinterpret_cast<const int4 *>(keys + s);
      if (q.x == k) return s;
      if (q.x == kEmpty32) return -1;
      if (q.y == k) return s + 1;
      if (q.y == kEmpty32) return -1;
      if (q.z == k) return s + 2;
      if (q.z == kEmpty32) return -1;
      if (q.w == k) return s + 3;
      if (q.w == kEmpty32) return -1;
      s = (s + 4) & mask;
    }
    return -1;
  } else {
    const uint64_t *slots = static_cast<const uint64_t *>(t.slots);
    int64_t s = (table_hash32(k) & mask) & ~int64_t{1};
    for (int64_t step = 0; step <= mask; step += 2) {
      const ulonglong2 q = *reinterpret_cast<const ulonglong2 *>(slots + s);
      if (static_cast<int32_t>(q.x) == k) {
        *pay = static_cast<int32_t>(q.x >> 32);
        return s;
      }
      if (static_cast<int32_t>(q.x) == kEmpty32) return -1;
      if (static_cast<int32_t>(q.y) == k) {
        *pay = static_cast<int32_t>(q.y >> 32);
        return s + 1;
      }
      if (static_cast<int32_t>(q.y) == kEmpty32) return -1;
      s = (s + 2) & mask;
    }
    return -1;
  }
}

__device__ __forceinline__ int64_t gsrc_value(int src, int idx, const int64_t (&v)[kMaxFactCols][4], int r,
                                              int32_t key0, int32_t key1, int32_t pay0, int32_t pay1) {
  switch (src) {
    case PYST_G_JOIN_KEY: return idx == 0 ? key0 : key1;
    case PYST_G_JOIN_PAYLOAD: return idx == 0 ? pay0 : pay1;
    case PYST_G_FACT_COL: return pick(v, idx, r);
    default: return 0;
  }
}

// ------------------------------------------------------------------ keys-only build
// Insert the selected dimension rows into a 4-byte-key table (unique keys).
__global__ __launch_bounds__(256) void k_build_keys(const int32_t *key, const int32_t *sel, const int64_t *d_nsel,
                                                    int64_t n, TableDev t, uint32_t *err) {
  const int64_t cnt = d_nsel ? *d_nsel : n;
  const int64_t mask = t.hdr[0] - 1;
  int32_t *keys = static_cast<int32_t *>(t.slots);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k = key[sel ? sel[i] : i];
    if (k == kEmpty32) {
      latch(err, kErrKey);
      continue;
    }
    int64_t s = (table_hash32(k) & mask) & ~int64_t{3};
    bool done = false;
    for (int64_t step = 0; step <= mask; ++step) {
      int32_t cur = keys[s];
      if (cur == kEmpty32) {
        const int32_t old = atomicCAS(&keys[s], kEmpty32, k);
        if (old == kEmpty32) {
          done = true;
          break;
        }
        cur = old;
      }
      if (cur == k) {
        latch(err, kErrDup);
        done = true;
        break;
      }
      s = (s + 1) & mask;
    }
    if (!done) latch(err, kErrTableFull);
  }
}

// ------------------------------------------------------------------ the fact pass
// AGG: 0 = sums in the slots of join 0 (group key = join-0 key), 1 = group table,
//      2 = materialize (group key, value) pairs for a following group-by.
template <int NJ, int SB0, int SB1, int AGG>
__global__ __launch_bounds__(256) void k_fact_pass(FactArgs a, TableDev t0, TableDev t1, GroupDev g, PairsOut po,
                                                   uint32_t *err) {
  const int64_t mask0 = t0.hdr[0] - 1;
  const int64_t mask1 = NJ > 1 ? t1.hdr[0] - 1 : 0;
  const int64_t gmask = AGG == 1 ? g.hdr[0] - 1 : 0;
  const int64_t stride = int64_t{gridDim.x} * blockDim.x * 4;
  for (int64_t base = (int64_t{blockIdx.x} * blockDim.x + threadIdx.x) * 4; base < a.n; base += stride) {
    int64_t v[kMaxFactCols][4];
#pragma unroll
    for (int c = 0; c < kMaxFactCols; ++c) {
      if (c < a.ncol) load4(a.col[c], a.is64[c], base, a.n, v[c]);
      else v[c][0] = v[c][1] = v[c][2] = v[c][3] = 0;
    }
    bool live[4];
    int32_t fk0[4];
    int64_t slot0[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      bool keep = base + r < a.n;
      for (int k = 0; k < a.npred; ++k) keep = keep && compare_op(pick(v, a.pslot[k], r), a.pop[k], a.pval[k]);
      live[r] = keep;
      fk0[r] = static_cast<int32_t>(pick(v, a.fk_slot[0], r));
    }
    int32_t pay0[4] = {0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) slot0[r] = live[r] ? find_slot<SB0>(t0, mask0, fk0[r], &pay0[r]) : -1;
    int32_t fk1[4] = {0, 0, 0, 0}, pay1[4] = {0, 0, 0, 0};
    if (NJ > 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        fk1[r] = static_cast<int32_t>(pick(v, a.fk_slot[1], r));
        if (slot0[r] >= 0 && find_slot<SB1>(t1, mask1, fk1[r], &pay1[r]) < 0) slot0[r] = -1;
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool hit = slot0[r] >= 0;
      int64_t val = 0, gkey = 0;
      if (hit) {
        const int64_t x = pick(v, a.v0_slot, r);
        val = a.vexpr == PYST_V_COL ? x
                                    : static_cast<int64_t>(static_cast<uint64_t>(x) *
                                                           static_cast<uint64_t>(a.vconst - pick(v, a.v1_slot, r)));
        if (AGG != 0) {
          const int64_t lo = gsrc_value(a.lo_src, a.lo_idx, v, r, fk0[r], fk1[r], pay0[r], pay1[r]);
          if (a.hi_src != PYST_G_NONE) {
            const int64_t hi = gsrc_value(a.hi_src, a.hi_idx, v, r, fk0[r], fk1[r], pay0[r], pay1[r]);
            gkey = static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | static_cast<uint32_t>(lo));
          } else {
            gkey = lo;
          }
        }
      }
      if (AGG == 0) {
        if (hit) {
          atomicAdd(reinterpret_cast<unsigned long long *>(&t0.sums[slot0[r]]), static_cast<unsigned long long>(val));
          t0.flags[slot0[r]] = 1;
        }
      } else if (AGG == 1) {
        if (hit) {
          if (gkey == kEmpty64) latch(err, kErrKey);
          else if (!group_add(g.slots, gmask, gkey, static_cast<uint64_t>(val))) latch(err, kErrTableFull);
        }
      } else {
        const uint64_t m = __ballot(hit);
        if (m) {
          const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
          unsigned long long wb = 0;
          if (lane_id() == leader) wb = atomicAdd(reinterpret_cast<unsigned long long *>(po.count), static_cast<unsigned long long>(__popcll(m)));
          wb = __shfl(wb, leader);
          if (hit) {
            const int64_t p = static_cast<int64_t>(wb) + mbcnt(m);
            if (gkey == kEmpty64) latch(err, kErrKey);
            if (p < po.cap) {
              po.keys[p] = gkey;
              po.vals[p] = val;
            }
          }
        }
      }
    }
  }
}

// Ordered compaction of the groups held in the slots of a join table.
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_slot_compact(TableDev t, int64_t *out_keys, int64_t *out_sums,
                                                       int64_t out_cap, int64_t *d_ngroups, uint64_t *status,
                                                       unsigned long long *ticket, int64_t ntiles, uint32_t *err) {
  constexpr int NW = BLOCK / kWave;
  constexpr int64_t TILE = int64_t{BLOCK} * ITEMS;
  __shared__ int64_t s_tile, s_prefix;
  __shared__ int32_t s_cnt[NW];
  if (threadIdx.x == 0) s_tile = static_cast<int64_t>(atomicAdd(ticket, 1ull));
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t cap = t.hdr[0];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t wbase = tile * TILE + int64_t{w} * kWave * ITEMS;
  uint64_t m[ITEMS];
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t s = wbase + int64_t{j} * kWave + lane;
    m[j] = __ballot(s < cap && t.flags[s] != 0);
    cnt += __popcll(m[j]);
  }
  if (lane == 0) s_cnt[w] = cnt;
  __syncthreads();
  if (w == 0) {
    const int64_t c = lane < NW ? s_cnt[lane] : 0;
    const int64_t agg = wave_sum(c);
    const int64_t ex = lookback_exclusive(status, tile, agg);
    if (lane == 0) {
      s_prefix = ex;
      if (tile == ntiles - 1) {
        *d_ngroups = ex + agg;
        if (ex + agg > out_cap) latch(err, kErrCapacity);
      }
    }
  }
  __syncthreads();
  int64_t pos = s_prefix;
  for (int k = 0; k < w; ++k) pos += s_cnt[k];
  const int32_t *keys = static_cast<const int32_t *>(t.slots);
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t s = wbase + int64_t{j} * kWave + lane;
    if ((m[j] >> lane) & 1ull) {
      const int64_t p = pos + mbcnt(m[j]);
      if (p < out_cap) {
        out_keys[p] = keys[s];
        out_sums[p] = static_cast<int64_t>(t.sums[s]);
      }
    }
    pos += __popcll(m[j]);
  }
}

// ------------------------------------------------------------------ host side
pyst_status prepare_query(const pyst_plan *plan, const pyst_col *fact, int nfact, QueryShape *q) {
  if (!plan || !fact) return set_error(PYST_ERR_ARG, "pyst_query: NULL plan or fact");
  std::memset(q, 0, sizeof(*q));
  if (plan->njoins < 1 || plan->njoins > 2) return set_error(PYST_ERR_ARG, "pyst_query: 1 or 2 joins");
  if (nfact < 1 || nfact > PYST_MAX_COLS) return set_error(PYST_ERR_ARG, "pyst_query: 1..8 fact columns");
  const int64_t n = fact[0].n;
  for (int c = 0; c < nfact; ++c)
    if (!(fact[c].dtype == PYST_I32 || fact[c].dtype == PYST_I64) || fact[c].n != n || (n > 0 && !fact[c].data))
      return set_error(PYST_ERR_ARG, "pyst_query: fact columns must be int32/int64 of equal length");
  for (int c = 0; c < nfact; ++c)
    if (reinterpret_cast<uintptr_t>(fact[c].data) % 16 != 0)
      return set_error(PYST_ERR_ARG, "pyst_query: fact columns must be 16-byte aligned (vector loads)");
  if (n >= (int64_t{1} << 31)) return set_error(PYST_ERR_ARG, "pyst_query: fewer than 2^31 fact rows per call");
  FactArgs &a = q->fact;
  a.n = n;
  int slot_of[PYST_MAX_COLS];
  for (int c = 0; c < PYST_MAX_COLS; ++c) slot_of[c] = -1;
  auto use = [&](int c) -> int {
    if (c < 0 || c >= nfact) return -1;
    if (slot_of[c] < 0) {
      if (a.ncol >= kMaxFactCols) return -2;
      slot_of[c] = a.ncol;
      a.col[a.ncol] = fact[c].data;
      a.is64[a.ncol] = fact[c].dtype == PYST_I64;
      ++a.ncol;
    }
    return slot_of[c];
  };
  if (plan->npreds < 0 || plan->npreds > PYST_MAX_PREDS || (plan->npreds > 0 && !plan->preds))
    return set_error(PYST_ERR_ARG, "pyst_query: bad fact predicates");
  a.npred = plan->npreds;
  for (int k = 0; k < plan->npreds; ++k) {
    const int s = use(plan->preds[k].col);
    if (s < 0) return set_error(PYST_ERR_ARG, "pyst_query: predicate names a missing fact column");
    if (plan->preds[k].cmp < PYST_EQ || plan->preds[k].cmp > PYST_GE) return set_error(PYST_ERR_ARG, "pyst_query: bad comparison");
    a.pslot[k] = s;
    a.pop[k] = plan->preds[k].cmp;
    a.pval[k] = plan->preds[k].value;
  }
  for (int j = 0; j < plan->njoins; ++j) {
    const pyst_join_spec &js = plan->joins[j];
    if (js.key.dtype != PYST_I32 || js.key.n < 0 || js.key.n >= (int64_t{1} << 31) || (js.key.n > 0 && !js.key.data))
      return set_error(PYST_ERR_ARG, "pyst_query: join keys are int32 columns");
    if (js.payload.data && (js.payload.dtype != PYST_I32 || js.payload.n != js.key.n))
      return set_error(PYST_ERR_ARG, "pyst_query: join payload must be int32 with the key's length");
    if (!(js.max_load > 0.0 && js.max_load <= 0.95)) return set_error(PYST_ERR_ARG, "pyst_query: join max_load in (0, 0.95]");
    if (js.npreds < 0 || js.npreds > PYST_MAX_PREDS || js.ncols < 0 || js.ncols > PYST_MAX_COLS ||
        (js.npreds > 0 && (!js.preds || !js.cols)))
      return set_error(PYST_ERR_ARG, "pyst_query: bad dimension predicates");
    for (int c = 0; c < js.ncols; ++c)
      if (js.cols[c].n != js.key.n || !(js.cols[c].dtype == PYST_I32 || js.cols[c].dtype == PYST_I64))
        return set_error(PYST_ERR_ARG, "pyst_query: dimension columns must match the key's length");
    const int s = use(js.probe_col);
    if (s < 0) return set_error(PYST_ERR_ARG, "pyst_query: probe column missing");
    if (fact[js.probe_col].dtype != PYST_I32) return set_error(PYST_ERR_UNSUPPORTED, "pyst_query: probe keys are int32");
    a.fk_slot[j] = s;
  }
  auto check_src = [&](int src, int idx, int32_t *out_idx) -> bool {
    switch (src) {
      case PYST_G_NONE: *out_idx = 0; return true;
      case PYST_G_JOIN_KEY: *out_idx = idx; return idx >= 0 && idx < plan->njoins;
      case PYST_G_JOIN_PAYLOAD:
        *out_idx = idx;
        if (idx < 0 || idx >= plan->njoins || !plan->joins[idx].payload.data) return false;
        q->need_payload[idx] = true;
        return true;
      case PYST_G_FACT_COL: {
        const int s = use(idx);
        *out_idx = s;
        return s >= 0;
      }
    }
    return false;
  };
  if (plan->lo_src == PYST_G_NONE || !check_src(plan->lo_src, plan->lo_index, &a.lo_idx) ||
      !check_src(plan->hi_src, plan->hi_index, &a.hi_idx))
    return set_error(PYST_ERR_ARG, "pyst_query: bad group key");
  a.lo_src = plan->lo_src;
  a.hi_src = plan->hi_src;
  if (plan->vexpr != PYST_V_COL && plan->vexpr != PYST_V_COL_TIMES_C_MINUS) return set_error(PYST_ERR_ARG, "pyst_query: bad value expression");
  a.vexpr = plan->vexpr;
  a.v0_slot = use(plan->v0);
  a.v1_slot = plan->vexpr == PYST_V_COL ? 0 : use(plan->v1);
  a.vconst = plan->vconst;
  if (a.v0_slot < 0 || a.v1_slot < 0) return set_error(PYST_ERR_ARG, "pyst_query: value column missing");
  if (!(plan->group_max_load > 0.0 && plan->group_max_load <= 0.95) && !(plan->njoins == 1 && plan->hi_src == PYST_G_NONE && plan->lo_src == PYST_G_JOIN_KEY))
    return set_error(PYST_ERR_ARG, "pyst_query: group_max_load in (0, 0.95]");
  q->slot_agg = plan->njoins == 1 && plan->hi_src == PYST_G_NONE && plan->lo_src == PYST_G_JOIN_KEY && plan->lo_index == 0;
  q->agg_mode = q->slot_agg ? 0 : (plan->max_groups > 0 ? 1 : 2);
  return PYST_OK;
}

// Filter + build every dimension of the plan into tables allocated by the caller.
pyst_status build_dimensions(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, DimTables *d,
                             hipStream_t stream) {
  for (int j = 0; j < plan->njoins; ++j) {
    const pyst_join_spec &js = plan->joins[j];
    const int64_t nb = js.key.n;
    const int sb = q.need_payload[j] ? 8 : 4;
    const bool sums = j == 0 && q.slot_agg;
    const int64_t cap_alloc = table_capacity_host(nb, js.max_load);
    d->mem[j] = ctx_alloc(ctx, table_bytes(cap_alloc, sb, sums), stream);
    if (!d->mem[j]) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (dimension table)");
    d->t[j] = table_view(d->mem[j], cap_alloc, sb, sums);
    const int32_t *sel = nullptr;
    const int64_t *d_nsel = nullptr;
    if (js.npreds > 0) {
      d->sel_mem[j] = ctx_alloc(ctx, static_cast<size_t>(std::max<int64_t>(nb, 1)) * sizeof(int32_t) + 256, stream);
      if (!d->sel_mem[j]) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (dimension selection)");
      int64_t *cnt = static_cast<int64_t *>(d->sel_mem[j]);
      int32_t *s = reinterpret_cast<int32_t *>(static_cast<char *>(d->sel_mem[j]) + 256);
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
      pyst_status st = filter_impl(ctx, ps, nb, s, cnt, stream);
      if (st != PYST_OK) return st;
      sel = s;
      d_nsel = cnt;
    }
    pyst_status st = table_init(d->t[j], d_nsel, nb, js.max_load, stream);
    if (st != PYST_OK) return st;
    if (nb > 0) {
      const int blocks = grid_for(ctx, nb, 256, 8);
      const int bblocks = grid_for(ctx, ceil_div(nb, int64_t{kBuildItems}), 256, 8);
      if (sb == 4) {
        k_build_keys<<<blocks, 256, 0, stream>>>(static_cast<const int32_t *>(js.key.data), sel, d_nsel, nb, d->t[j],
                                                 ctx_err_word(ctx));
        PYST_LAUNCH_CHECK("k_build_keys");
      } else {
        k_join_build<256, kBuildItems><<<bblocks, 256, 0, stream>>>(static_cast<const int32_t *>(js.key.data),
                                                 static_cast<const int32_t *>(js.payload.data), sel, d_nsel, nb,
                                                 d->t[j], 1, ctx_err_word(ctx));
        PYST_LAUNCH_CHECK("k_join_build");
      }
    }
  }
  return PYST_OK;
}

void free_dimensions(pyst_ctx *ctx, DimTables *d, hipStream_t stream) {
  for (int j = 0; j < 2; ++j) {
    ctx_free(ctx, d->mem[j], stream);
    ctx_free(ctx, d->sel_mem[j], stream);
    d->mem[j] = d->sel_mem[j] = nullptr;
  }
}

template <int NJ, int SB0, int SB1, int AGG>
static void launch_fact(int grid, const FactArgs &a, const DimTables &d, const GroupDev &g, const PairsOut &po,
                        uint32_t *err, hipStream_t stream) {
  k_fact_pass<NJ, SB0, SB1, AGG><<<grid, 256, 0, stream>>>(a, d.t[0], d.t[1], g, po, err);
}

pyst_status fact_pass(pyst_ctx *ctx, const QueryShape &q, int njoins, const FactArgs &a, const DimTables &d,
                      const GroupDev &g, const PairsOut &po, int grid, hipStream_t stream) {
  if (a.n <= 0) return PYST_OK;
  if (grid <= 0) grid = grid_for(ctx, ceil_div(a.n, 4), 256, 8);
  uint32_t *err = ctx_err_word(ctx);
  TimedRegion timed(ctx, "fact_pass", stream);
  const int sb0 = d.t[0].slot_bytes, sb1 = njoins > 1 ? d.t[1].slot_bytes : 4;
  const int mode = q.agg_mode;
#define PYST_FACT_CASE(NJ_, S0_, S1_, AG_)                                           \
  if (njoins == NJ_ && sb0 == S0_ && sb1 == S1_ && mode == AG_) {                  \
    launch_fact<NJ_, S0_, S1_, AG_>(grid, a, d, g, po, err, stream);                 \
    PYST_LAUNCH_CHECK("k_fact_pass");                                               \
    return PYST_OK;                                                                 \
  }
  PYST_FACT_CASE(1, 4, 4, 0)
  PYST_FACT_CASE(1, 4, 4, 1)
  PYST_FACT_CASE(1, 4, 4, 2)
  PYST_FACT_CASE(1, 8, 4, 1)
  PYST_FACT_CASE(1, 8, 4, 2)
  PYST_FACT_CASE(2, 4, 4, 1)
  PYST_FACT_CASE(2, 4, 4, 2)
  PYST_FACT_CASE(2, 4, 8, 1)
  PYST_FACT_CASE(2, 4, 8, 2)
  PYST_FACT_CASE(2, 8, 4, 1)
  PYST_FACT_CASE(2, 8, 4, 2)
  PYST_FACT_CASE(2, 8, 8, 1)
  PYST_FACT_CASE(2, 8, 8, 2)
#undef PYST_FACT_CASE
  return set_error(PYST_ERR_UNSUPPORTED, "pyst_query: unsupported plan shape");
}

pyst_status slot_compact(pyst_ctx *ctx, const TableDev &t, int64_t *out_keys, int64_t *out_sums, int64_t out_cap,
                         int64_t *d_ngroups, hipStream_t stream) {
  constexpr int BLOCK = 256, ITEMS = 8;
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(t.cap_alloc, int64_t{BLOCK} * ITEMS));
  Scratch sc(ctx, (ntiles + 1) * sizeof(uint64_t), stream);
  if (!sc.p) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (compaction)");
  pyst_status st = fill_u64(sc.p, ntiles + 1, 0, stream);
  if (st != PYST_OK) return st;
  uint64_t *status = sc.as<uint64_t>();
  k_slot_compact<BLOCK, ITEMS><<<static_cast<unsigned>(ntiles), BLOCK, 0, stream>>>(
      t, out_keys, out_sums, out_cap, d_ngroups, status, reinterpret_cast<unsigned long long *>(status + ntiles),
      ntiles, ctx_err_word(ctx));
  PYST_LAUNCH_CHECK("k_slot_compact");
  return PYST_OK;
}

// Aggregation state for one query: the group table (mode 1) or the pair
// buffer (mode 2) plus its device counter.
pyst_status agg_alloc(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, int64_t rows_bound, AggState *s,
                      hipStream_t stream) {
  std::memset(s, 0, sizeof(*s));
  if (q.agg_mode == 1) {
    const int64_t cap = table_capacity_host(std::min<int64_t>(plan->max_groups, std::max<int64_t>(rows_bound, 1)),
                                            plan->group_max_load);
    s->mem = ctx_alloc(ctx, group_bytes(cap), stream);
    if (!s->mem) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (group table)");
    s->g = group_view(s->mem, cap);
    return group_init(s->g, nullptr, std::min<int64_t>(plan->max_groups, std::max<int64_t>(rows_bound, 1)), 0,
                      plan->group_max_load, stream);
  }
  if (q.agg_mode == 2) {
    const int64_t cap = std::max<int64_t>(rows_bound, 1);
    s->mem = ctx_alloc(ctx, 256 + static_cast<size_t>(cap) * 16, stream);
    if (!s->mem) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (pair buffer)");
    s->po.count = static_cast<int64_t *>(s->mem);
    s->po.keys = reinterpret_cast<int64_t *>(static_cast<char *>(s->mem) + 256);
    s->po.vals = s->po.keys + cap;
    s->po.cap = cap;
    return fill_u64(s->po.count, 1, 0, stream);
  }
  return PYST_OK;
}

pyst_status agg_finish(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, const DimTables &d, AggState *s,
                       int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                       hipStream_t stream) {
  pyst_status st = PYST_OK;
  if (q.agg_mode == 0) {
    st = slot_compact(ctx, d.t[0], out_keys, out_sums, out_cap, d_ngroups, stream);
  } else if (q.agg_mode == 1) {
    st = group_compact(ctx, s->g, out_keys, out_sums, out_cap, d_ngroups, stream);
  } else {
    // group-by over the materialized pairs, table sized from their device count
    const int64_t cap = table_capacity_host(s->po.cap, plan->group_max_load);
    void *gm = ctx_alloc(ctx, group_bytes(cap), stream);
    if (!gm) return set_error(PYST_ERR_NOMEM, "pyst_query: arena exhausted (group table)");
    GroupDev g = group_view(gm, cap);
    st = group_init(g, s->po.count, s->po.cap, 0, plan->group_max_load, stream);
    if (st == PYST_OK) {
      const int blocks = grid_for(ctx, s->po.cap, 256, 8);
      k_gb_insert<<<blocks, 256, 0, stream>>>(s->po.keys, 1, s->po.vals, 1, nullptr, s->po.count, s->po.cap, g,
                                              ctx_err_word(ctx), 0);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) st = hip_error(e, "k_gb_insert");
    }
    if (st == PYST_OK) st = group_compact(ctx, g, out_keys, out_sums, out_cap, d_ngroups, stream);
    ctx_free(ctx, gm, stream);
  }
  ctx_free(ctx, s->mem, stream);
  s->mem = nullptr;
  return st;
}

}  // namespace pyst

using namespace pyst;

extern "C" pyst_status pyst_query(pyst_ctx *ctx, const pyst_plan *plan, const pyst_col *fact, int nfact,
                                  int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                                  hipStream_t stream) {
  if (!ctx || !d_ngroups) return set_error(PYST_ERR_ARG, "pyst_query: NULL ctx or d_ngroups");
  if (out_cap < 0 || (out_cap > 0 && (!out_keys || !out_sums))) return set_error(PYST_ERR_ARG, "pyst_query: bad outputs");
  QueryShape q;
  pyst_status st = prepare_query(plan, fact, nfact, &q);
  if (st != PYST_OK) return st;
  FastArgs fa;
  if (!ctx_generic_only(ctx) && fast_shape(plan, fact, q, &fa))
    return fast_query(ctx, plan, q, fa, out_keys, out_sums, out_cap, d_ngroups, stream);
  DimTables d;
  std::memset(&d, 0, sizeof(d));
  st = build_dimensions(ctx, plan, q, &d, stream);
  AggState s;
  std::memset(&s, 0, sizeof(s));
  if (st == PYST_OK) st = agg_alloc(ctx, plan, q, q.fact.n, &s, stream);
  if (st == PYST_OK) st = fact_pass(ctx, q, plan->njoins, q.fact, d, s.g, s.po, 0, stream);
  if (st == PYST_OK) st = agg_finish(ctx, plan, q, d, &s, out_keys, out_sums, out_cap, d_ngroups, stream);
  if (s.mem) ctx_free(ctx, s.mem, stream);
  free_dimensions(ctx, &d, stream);
  return st;
}

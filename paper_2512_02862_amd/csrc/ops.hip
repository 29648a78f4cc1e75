// Relational operators for gfx950: filter, hash partition, hash-join build and
// probe, hash group-by SUM.  Every data-dependent size stays in device memory.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>

#include "pyst_internal.h"
#include "table.h"

// Scratch of pyst_partition_noalloc: every GPU the library runs on holds its
// own copy until the process ends.
constexpr int kNoallocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[PYST_NOALLOC_SCRATCH_BYTES];

namespace pyst {

// ============================================================== fill kernels
__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

pyst_status fill_u64(void *p, int64_t n, uint64_t v, hipStream_t stream) {
  if (n <= 0) return PYST_OK;
  const int blocks = static_cast<int>(std::min<int64_t>(ceil_div(n, 256), 8192));
  k_fill_u64<<<blocks, 256, 0, stream>>>(static_cast<uint64_t *>(p), n, v);
  PYST_LAUNCH_CHECK("k_fill_u64");
  return PYST_OK;
}
pyst_status fill_u32(void *p, int64_t n, uint32_t v, hipStream_t stream) {
  if (n <= 0) return PYST_OK;
  const int blocks = static_cast<int>(std::min<int64_t>(ceil_div(n, 256), 8192));
  k_fill_u32<<<blocks, 256, 0, stream>>>(static_cast<uint32_t *>(p), n, v);
  PYST_LAUNCH_CHECK("k_fill_u32");
  return PYST_OK;
}

// ============================================================== argument helpers
namespace {

bool col_ok(const pyst_col *c) {
  return c && (c->dtype == PYST_I32 || c->dtype == PYST_I64) && c->n >= 0 && (c->data || c->n == 0) &&
         c->n < (int64_t{1} << 31);
}

pyst_status build_predset(const pyst_col *cols, int ncols, const pyst_pred *preds, int np, PredSet *ps,
                          const char *who) {
  if (np < 0 || np > PYST_MAX_PREDS) return set_error(PYST_ERR_ARG, std::string(who) + ": too many predicates");
  if (np > 0 && !preds) return set_error(PYST_ERR_ARG, std::string(who) + ": preds is NULL");
  std::memset(ps, 0, sizeof(*ps));
  ps->n = np;
  for (int k = 0; k < np; ++k) {
    const int c = preds[k].col;
    if (c < 0 || c >= ncols) return set_error(PYST_ERR_ARG, std::string(who) + ": predicate names a missing column");
    if (preds[k].cmp < PYST_EQ || preds[k].cmp > PYST_GE) return set_error(PYST_ERR_ARG, std::string(who) + ": bad comparison");
    ps->col[k] = cols[c].data;
    ps->is64[k] = cols[c].dtype == PYST_I64;
    ps->op[k] = preds[k].cmp;
    ps->val[k] = preds[k].value;
  }
  return PYST_OK;
}

// Rows [tile*TILE, (tile+1)*TILE) of a selection (or of all rows): row id of position i.
__device__ __forceinline__ int64_t row_of(const int32_t *sel, int64_t i) { return sel ? static_cast<int64_t>(sel[i]) : i; }
__device__ __forceinline__ int64_t count_of(const int64_t *d_nsel, int64_t n) { return d_nsel ? *d_nsel : n; }

// In-place exclusive scan of arr[0..len) by one block (len <= BLOCK * 8).
template <int BLOCK>
__device__ void block_exclusive_scan(int32_t *arr, int len, int32_t *s_wave) {
  constexpr int NW = BLOCK / kWave;
  const int per = (len + BLOCK - 1) / BLOCK;
  const int lo = threadIdx.x * per;
  int32_t local = 0;
  for (int k = 0; k < per; ++k)
    if (lo + k < len) local += arr[lo + k];
  const int32_t incl = wave_inclusive_scan(local);
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) s_wave[w] = incl;
  __syncthreads();
  int32_t wave_off = 0;
  for (int k = 0; k < w; ++k) wave_off += s_wave[k];
  int32_t run = wave_off + incl - local;
  __syncthreads();
  for (int k = 0; k < per; ++k) {
    if (lo + k < len) {
      const int32_t v = arr[lo + k];
      arr[lo + k] = run;
      run += v;
    }
  }
  (void)NW;
}

}  // namespace

// ============================================================== filter
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_filter(PredSet ps, int64_t n, int32_t *sel_out, int64_t *d_nsel,
                                                 uint64_t *status, unsigned long long *ticket, int64_t ntiles) {
  constexpr int NW = BLOCK / kWave;
  constexpr int64_t TILE = int64_t{BLOCK} * ITEMS;
  __shared__ int64_t s_tile, s_prefix;
  __shared__ int32_t s_cnt[NW];
  if (threadIdx.x == 0) s_tile = static_cast<int64_t>(atomicAdd(ticket, 1ull));
  __syncthreads();
  const int64_t t = s_tile;
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t wbase = t * TILE + int64_t{w} * kWave * ITEMS;
  int64_t rows[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) rows[j] = wbase + int64_t{j} * kWave + lane;
  bool keep[ITEMS];
  eval_preds_items<ITEMS>(ps, rows, n, keep);
  uint64_t m[ITEMS];
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    m[j] = __ballot(keep[j]);
    cnt += __popcll(m[j]);
  }
  if (lane == 0) s_cnt[w] = cnt;
  __syncthreads();
  if (w == 0) {
    const int64_t c = lane < NW ? s_cnt[lane] : 0;
    const int64_t agg = wave_sum(c);
    const int64_t ex = lookback_exclusive(status, t, agg);
    if (lane == 0) {
      s_prefix = ex;
      if (t == ntiles - 1) *d_nsel = ex + agg;
    }
  }
  __syncthreads();
  int64_t pos = s_prefix;
  for (int k = 0; k < w; ++k) pos += s_cnt[k];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if ((m[j] >> lane) & 1ull) sel_out[pos + mbcnt(m[j])] = static_cast<int32_t>(wbase + int64_t{j} * kWave + lane);
    pos += __popcll(m[j]);
  }
}

pyst_status filter_impl(pyst_ctx *ctx, const PredSet &ps, int64_t n, int32_t *sel_out, int64_t *d_nsel,
                        hipStream_t stream) {
  constexpr int BLOCK = 256, ITEMS = 16;
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(n, int64_t{BLOCK} * ITEMS));
  Scratch sc(ctx, (ntiles + 1) * sizeof(uint64_t), stream);
  if (!sc.p) return set_error(PYST_ERR_NOMEM, "pyst_filter: arena exhausted");
  pyst_status st = fill_u64(sc.p, ntiles + 1, 0, stream);
  if (st != PYST_OK) return st;
  uint64_t *status = sc.as<uint64_t>();
  k_filter<BLOCK, ITEMS><<<static_cast<unsigned>(ntiles), BLOCK, 0, stream>>>(
      ps, n, sel_out, d_nsel, status, reinterpret_cast<unsigned long long *>(status + ntiles), ntiles);
  PYST_LAUNCH_CHECK("k_filter");
  return PYST_OK;
}

// ============================================================== partition
struct PartArgs {
  const void *key;
  int32_t key64;
  int32_t npay;
  const void *pay[PYST_MAX_PART_PAYLOADS];
  int32_t pay64[PYST_MAX_PART_PAYLOADS];
  void *out[PYST_MAX_PART_PAYLOADS + 1];
  const int32_t *sel;
  const int64_t *d_nsel;
  int64_t n;
  uint32_t fanout;
  int32_t fbits;        // bits needed to hold fanout - 1
  int32_t radix_shift;  // >= 0: destination = byte of (key ^ sign bit) at this shift (sort pass); < 0: hash
};

__device__ __forceinline__ uint32_t part_dest(const PartArgs &a, int64_t row) {
  if (a.radix_shift >= 0) {
    const uint64_t k = static_cast<uint64_t>(load_as_i64(a.key, a.key64, row)) ^ (1ull << 63);
    return static_cast<uint32_t>((k >> a.radix_shift) & 0xffu);
  }
  uint32_t h;
  if (a.key64) h = static_cast<uint32_t>(fmix64(static_cast<uint64_t>(static_cast<const int64_t *>(a.key)[row])));
  else h = fmix32(static_cast<uint32_t>(static_cast<const int32_t *>(a.key)[row]));
  return (a.fanout & (a.fanout - 1)) == 0 ? (h & (a.fanout - 1)) : (h % a.fanout);
}

__device__ __forceinline__ uint32_t part_dest_key(const PartArgs &a, int64_t k) {
  if (a.radix_shift >= 0) return static_cast<uint32_t>(((static_cast<uint64_t>(k) ^ (1ull << 63)) >> a.radix_shift) & 0xffu);
  const uint32_t h = a.key64 ? static_cast<uint32_t>(fmix64(static_cast<uint64_t>(k)))
                             : fmix32(static_cast<uint32_t>(static_cast<int32_t>(k)));
  return (a.fanout & (a.fanout - 1)) == 0 ? (h & (a.fanout - 1)) : (h % a.fanout);
}

// Row ids and keys of a wave's ITEMS items (all loads issued before any use).
// Items at or past `cnt` get a valid clamped row; callers mask them.
template <int ITEMS>
__device__ __forceinline__ void part_load(const PartArgs &a, int64_t wbase, int64_t cnt, int64_t (&row)[ITEMS],
                                          int64_t (&key)[ITEMS]) {
  const int lane = lane_id();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) row[j] = wbase + int64_t{j} * kWave + lane;
  if (wbase >= cnt) {  // the whole wave is past the end (uniform)
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) key[j] = 0;
    return;
  }
  if (a.sel) {
    int64_t r[ITEMS];
    load_items<ITEMS>(a.sel, 0, row, cnt, r);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) row[j] = r[j];
    load_items<ITEMS>(a.key, a.key64, row, a.n, key);
  } else {
    load_items<ITEMS>(a.key, a.key64, row, cnt, key);
  }
}

// Lanes of `valid` holding the same destination as the calling lane (AMD has no
// match instruction: intersect one ballot per destination bit).
__device__ __forceinline__ uint64_t match_peers(uint32_t d, uint64_t valid, int fbits) {
  uint64_t peers = valid;
  for (int b = 0; b < fbits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t ones = __ballot(bit);
    peers &= bit ? ones : ~ones;
  }
  return peers;
}

constexpr int kPartBlock = 256;
constexpr int kPartItems = 16;
constexpr int64_t kPartTile = int64_t{kPartBlock} * kPartItems;

// Pass 1: per-tile destination histogram, stored destination-major so that one
// exclusive scan of the flat array yields every (destination, tile) offset.
template <int BLOCK, int ITEMS, int FMAX>
__global__ __launch_bounds__(BLOCK) void k_part_hist(PartArgs a, int32_t *hist, int64_t ntiles) {
  constexpr int64_t TILE = int64_t{BLOCK} * ITEMS;
  __shared__ int32_t s_h[FMAX];
  for (int p = threadIdx.x; p < static_cast<int>(a.fanout); p += BLOCK) s_h[p] = 0;
  __syncthreads();
  const int64_t cnt = count_of(a.d_nsel, a.n);
  const int64_t t = blockIdx.x;
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t wbase = t * TILE + int64_t{w} * kWave * ITEMS;
  int64_t row[ITEMS], key[ITEMS];
  part_load<ITEMS>(a, wbase, cnt, row, key);
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t i = wbase + int64_t{j} * kWave + lane;
    const bool valid = i < cnt;
    const uint32_t d = valid ? part_dest_key(a, key[j]) : 0u;
    const uint64_t vm = __ballot(valid);
    const uint64_t peers = match_peers(d, vm, a.fbits);
    if (valid && lane == __ffsll(static_cast<unsigned long long>(peers)) - 1) atomicAdd(&s_h[d], __popcll(peers));
  }
  __syncthreads();
  for (int p = threadIdx.x; p < static_cast<int>(a.fanout); p += BLOCK) hist[int64_t{p} * ntiles + t] = s_h[p];
}

// Exclusive scan of an int32 array (decoupled look-back); total -> *d_total.
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_scan_excl_i32(const int32_t *in, int32_t *out, int64_t len,
                                                        uint64_t *status, unsigned long long *ticket, int64_t ntiles,
                                                        int64_t *d_total) {
  constexpr int NW = BLOCK / kWave;
  constexpr int64_t TILE = int64_t{BLOCK} * ITEMS;
  __shared__ int64_t s_tile, s_prefix;
  __shared__ int32_t s_w[NW];
  if (threadIdx.x == 0) s_tile = static_cast<int64_t>(atomicAdd(ticket, 1ull));
  __syncthreads();
  const int64_t t = s_tile;
  const int64_t base = t * TILE + int64_t{threadIdx.x} * ITEMS;
  int32_t v[ITEMS];
  int32_t local = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    v[k] = base + k < len ? in[base + k] : 0;
    local += v[k];
  }
  const int32_t incl = wave_inclusive_scan(local);
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) s_w[w] = incl;
  __syncthreads();
  if (w == 0) {
    const int64_t c = lane_id() < NW ? s_w[lane_id()] : 0;
    const int64_t agg = wave_sum(c);
    const int64_t ex = lookback_exclusive(status, t, agg);
    if (lane_id() == 0) {
      s_prefix = ex;
      if (t == ntiles - 1 && d_total) *d_total = ex + agg;
    }
  }
  __syncthreads();
  int64_t run = s_prefix + incl - local;
  for (int k = 0; k < w; ++k) run += s_w[k];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    if (base + k < len) out[base + k] = static_cast<int32_t>(run);
    run += v[k];
  }
}

__global__ void k_part_offsets(const int32_t *scan, uint32_t fanout, int64_t ntiles, const int64_t *d_nsel, int64_t n,
                               int64_t *d_offsets) {
  const int64_t cnt = count_of(d_nsel, n);
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p <= fanout; p += gridDim.x * blockDim.x)
    d_offsets[p] = p < fanout ? static_cast<int64_t>(scan[int64_t{p} * ntiles]) : cnt;
}

// Pass 3: stable scatter.  Each wave ranks its rows per destination with
// ballots; the block lays the tile out destination-major in LDS, then writes
// every destination's run with consecutive threads on consecutive addresses
// (software write combining: whole lines per destination, not scattered words).
// Histogram of one 4096-row tile for the common case: int32 keys read in
// place (no selection), hash destinations, F <= 64.  Each thread reads its 16
// rows as four 16-byte loads.  Up to 8 destinations are counted in registers
// and summed across the wave; more go to per-wave LDS counters.
template <int FMAX>
__global__ __launch_bounds__(256) void k_part_hist_i32(PartArgs a, int32_t *hist, int64_t ntiles) {
  constexpr int BLOCK = 256, NW = BLOCK / kWave;
  constexpr int64_t TILE = 4096;
  __shared__ int32_t s_h[NW][FMAX];
  const int F = static_cast<int>(a.fanout);
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int p = lane; p < F; p += kWave) s_h[w][p] = 0;
  const int64_t t = blockIdx.x;
  const int64_t n = a.n;
  const int32_t *key = static_cast<const int32_t *>(a.key);
  int32_t k[16];
  bool ok[16];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t r0 = t * TILE + int64_t{q} * 1024 + int64_t{threadIdx.x} * 4;
    if (r0 + 4 <= n) {
      const v4i32 v = *reinterpret_cast<const v4i32 *>(key + r0);
      k[4 * q] = v.x;
      k[4 * q + 1] = v.y;
      k[4 * q + 2] = v.z;
      k[4 * q + 3] = v.w;
#pragma unroll
      for (int j = 0; j < 4; ++j) ok[4 * q + j] = true;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        ok[4 * q + j] = r0 + j < n;
        k[4 * q + j] = ok[4 * q + j] ? key[r0 + j] : 0;
      }
    }
  }
  __syncthreads();
  if (F <= 8) {  // uniform
    int32_t c[8] = {};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint32_t d = part_dest_key(a, k[j]);
#pragma unroll
      for (int f = 0; f < 8; ++f) c[f] += (ok[j] && d == static_cast<uint32_t>(f)) ? 1 : 0;
    }
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      const int32_t tot = wave_sum(c[f]);
      if (lane == 0 && f < F) s_h[w][f] = tot;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j)
      if (ok[j]) atomicAdd(&s_h[w][part_dest_key(a, k[j])], 1);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < F; p += BLOCK) {
    int32_t tot = 0;
#pragma unroll
    for (int v = 0; v < NW; ++v) tot += s_h[v][p];
    hist[int64_t{p} * ntiles + t] = tot;
  }
}

template <int BLOCK, int ITEMS, int FMAX>
__global__ __launch_bounds__(BLOCK) void k_part_scatter(PartArgs a, const int32_t *scan, int64_t ntiles) {
  constexpr int NW = BLOCK / kWave;
  constexpr int TILE = BLOCK * ITEMS;
  __shared__ int32_t s_cnt[NW][FMAX];
  __shared__ int32_t s_start[FMAX];
  __shared__ int32_t s_goff[FMAX];
  __shared__ int32_t s_wave[NW];
  __shared__ uint16_t s_dest[TILE];
  __shared__ int64_t s_stage[TILE];

  const int F = static_cast<int>(a.fanout);
  const int64_t t = xcd_block(blockIdx.x, gridDim.x);  // consecutive tiles on one XCD
  const int64_t cnt = count_of(a.d_nsel, a.n);
  for (int p = threadIdx.x; p < F; p += BLOCK) {
    for (int w = 0; w < NW; ++w) s_cnt[w][p] = 0;
    s_goff[p] = scan[int64_t{p} * ntiles + t];
  }
  __syncthreads();

  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t wbase = t * TILE + int64_t{w} * kWave * ITEMS;
  int32_t rowv[ITEMS];
  int32_t pos[ITEMS];
  uint16_t dst[ITEMS];
  int64_t keyv[ITEMS];
  // The first payload columns are loaded with the keys (one memory round
  // trip per tile instead of one per column); later ones in the column loop.
  // (Two with 512 threads; one with 1024, whose 4 rows per thread then fit in
  // 56 registers: two blocks of 16 waves per CU.)
  constexpr int PRE = BLOCK >= 1024 ? 1 : 2;
  int64_t pre[PRE][ITEMS];
  {
    int64_t r64[ITEMS];
    part_load<ITEMS>(a, wbase, cnt, r64, keyv);
#pragma unroll
    for (int c = 0; c < PRE; ++c)
      if (c < a.npay && wbase < cnt) load_items<ITEMS>(a.pay[c], a.pay64[c], r64, a.n, pre[c]);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) rowv[j] = static_cast<int32_t>(r64[j]);
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t i = wbase + int64_t{j} * kWave + lane;
    const bool valid = i < cnt;
    const uint32_t d = valid ? part_dest_key(a, keyv[j]) : 0u;
    dst[j] = static_cast<uint16_t>(d);
    const uint64_t vm = __ballot(valid);
    const uint64_t peers = match_peers(d, vm, a.fbits);
    const int32_t base = valid ? s_cnt[w][d] : 0;
    pos[j] = valid ? base + static_cast<int32_t>(mbcnt(peers)) : -1;
    if (valid && lane == __ffsll(static_cast<unsigned long long>(peers)) - 1) s_cnt[w][d] = base + __popcll(peers);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < F; p += BLOCK) {
    int32_t run = 0;
    for (int k = 0; k < NW; ++k) {
      const int32_t c = s_cnt[k][p];
      s_cnt[k][p] = run;
      run += c;
    }
    s_start[p] = run;
  }
  __syncthreads();
  block_exclusive_scan<BLOCK>(s_start, F, s_wave);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (pos[j] >= 0) {
      pos[j] += s_start[dst[j]] + s_cnt[w][dst[j]];
      s_dest[pos[j]] = dst[j];
    }
  }
  const int tile_rows = static_cast<int>(std::min<int64_t>(TILE, std::max<int64_t>(0, cnt - t * TILE)));
  for (int c = 0; c <= a.npay; ++c) {
    const int is64 = c == 0 ? a.key64 : a.pay64[c - 1];
    if (c == 0) {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j)
        if (pos[j] >= 0) s_stage[pos[j]] = keyv[j];
    } else if (c <= PRE && wbase < cnt) {
#pragma unroll
      for (int q = 0; q < PRE; ++q)
        if (q == c - 1)
#pragma unroll
          for (int j = 0; j < ITEMS; ++j)
            if (pos[j] >= 0) s_stage[pos[j]] = pre[q][j];
    } else if (wbase < cnt) {
      int64_t rr[ITEMS], x[ITEMS];
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) rr[j] = rowv[j];
      load_items<ITEMS>(a.pay[c - 1], is64, rr, a.n, x);
#pragma unroll
      for (int j = 0; j < ITEMS; ++j)
        if (pos[j] >= 0) s_stage[pos[j]] = x[j];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < tile_rows; i += BLOCK) {
      const int d = s_dest[i];
      const int64_t g = int64_t{s_goff[d]} + (i - s_start[d]);
      if (is64) static_cast<int64_t *>(a.out[c])[g] = s_stage[i];
      else static_cast<int32_t *>(a.out[c])[g] = static_cast<int32_t>(s_stage[i]);
    }
    __syncthreads();
  }
}

template <int FMAX>
static void launch_partition(const PartArgs &a, int32_t *hist, int32_t *scan, int64_t ntiles, hipStream_t stream,
                             bool hist_phase) {
  if (hist_phase && FMAX <= 64 && !a.sel && !a.key64 && a.radix_shift < 0 && !a.d_nsel && kPartTile == 4096 &&
      (reinterpret_cast<uintptr_t>(a.key) & 15) == 0)
    k_part_hist_i32<64><<<static_cast<unsigned>(ntiles), 256, 0, stream>>>(a, hist, ntiles);
  else if (hist_phase)
    k_part_hist<kPartBlock, kPartItems, FMAX><<<static_cast<unsigned>(ntiles), kPartBlock, 0, stream>>>(a, hist, ntiles);
  else if (FMAX <= 256)
    // the same 4096-row tiles as the histogram, as 1024 threads x 4 rows (few
    // registers per thread: 32 waves per CU; at fanout 64, 524 against 567 us
    // per 60M-row partition as 512 threads x 8 rows)
    k_part_scatter<4 * kPartBlock, kPartItems / 4, FMAX><<<static_cast<unsigned>(ntiles), 4 * kPartBlock, 0, stream>>>(
        a, scan, ntiles);
  else  // 1024 destinations: the per-wave counters of 16 waves would not leave LDS for two blocks
    k_part_scatter<2 * kPartBlock, kPartItems / 2, FMAX><<<static_cast<unsigned>(ntiles), 2 * kPartBlock, 0, stream>>>(
        a, scan, ntiles);
}

pyst_status scan_excl_i32(pyst_ctx *ctx, const int32_t *in, int32_t *out, int64_t len, int64_t *d_total,
                          hipStream_t stream);

constexpr int kScanBlock = 256, kScanItems = 8;

// Scratch of one partition: per-tile destination counts, their exclusive scan
// and the scan's look-back status words.
static size_t partition_scratch_bytes(int64_t n, uint32_t fanout) {
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(n, kPartTile));
  const int64_t hlen = ntiles * fanout;
  const int64_t stiles = std::max<int64_t>(1, ceil_div(hlen, int64_t{kScanBlock} * kScanItems));
  const size_t counts = (static_cast<size_t>(2 * hlen) * sizeof(int32_t) + 256 + 255) / 256 * 256;
  return counts + static_cast<size_t>(stiles + 1) * sizeof(uint64_t);
}

pyst_status scan_excl_i32_ws(const int32_t *in, int32_t *out, int64_t len, int64_t *d_total, uint64_t *status,
                             hipStream_t stream);

// histogram -> scan -> (offsets) -> stable scatter, in `ws` of
// partition_scratch_bytes(a.n, a.fanout) bytes; ctx (may be null) only for timing.
static pyst_status partition_run_ws(pyst_ctx *ctx, const PartArgs &a, int64_t *d_offsets, void *ws,
                                    hipStream_t stream) {
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(a.n, kPartTile));
  const int64_t hlen = ntiles * a.fanout;
  int32_t *hist = static_cast<int32_t *>(ws);
  int32_t *scan = hist + hlen + 64;
  uint64_t *status = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) +
                                                  (static_cast<size_t>(2 * hlen) * sizeof(int32_t) + 256 + 255) / 256 * 256);
  if (a.fanout <= 64) launch_partition<64>(a, hist, scan, ntiles, stream, true);
  else if (a.fanout <= 256) launch_partition<256>(a, hist, scan, ntiles, stream, true);
  else launch_partition<1024>(a, hist, scan, ntiles, stream, true);
  PYST_LAUNCH_CHECK("k_part_hist");
  pyst_status st = scan_excl_i32_ws(hist, scan, hlen, nullptr, status, stream);
  if (st != PYST_OK) return st;
  if (d_offsets) {
    k_part_offsets<<<static_cast<unsigned>(ceil_div(a.fanout + 1, 256)), 256, 0, stream>>>(scan, a.fanout, ntiles,
                                                                                          a.d_nsel, a.n, d_offsets);
    PYST_LAUNCH_CHECK("k_part_offsets");
  }
  TimedRegion timed(ctx, "part_scatter", stream);
  if (a.fanout <= 64) launch_partition<64>(a, hist, scan, ntiles, stream, false);
  else if (a.fanout <= 256) launch_partition<256>(a, hist, scan, ntiles, stream, false);
  else launch_partition<1024>(a, hist, scan, ntiles, stream, false);
  PYST_LAUNCH_CHECK("k_part_scatter");
  return PYST_OK;
}

static pyst_status partition_run(pyst_ctx *ctx, const PartArgs &a, int64_t *d_offsets, hipStream_t stream) {
  Scratch sc(ctx, partition_scratch_bytes(a.n, a.fanout), stream);
  if (!sc.p) return set_error(PYST_ERR_NOMEM, "partition: arena exhausted");
  return partition_run_ws(ctx, a, d_offsets, sc.p, stream);
}

// LSD radix sort of (key, value) int64 pairs, 8 stable byte passes; the first
// *d_count of `cap` entries are sorted in place (ping-pong through scratch).
pyst_status sort_pairs_by_key(pyst_ctx *ctx, int64_t *keys, int64_t *vals, const int64_t *d_count, int64_t cap,
                              hipStream_t stream) {
  if (cap <= 0) return PYST_OK;
  Scratch tmp(ctx, 2 * cap * sizeof(int64_t), stream);
  if (!tmp.p) return set_error(PYST_ERR_NOMEM, "sort: arena exhausted");
  int64_t *bk[2] = {keys, tmp.as<int64_t>()};
  int64_t *bv[2] = {vals, tmp.as<int64_t>() + cap};
  for (int pass = 0; pass < 8; ++pass) {
    const int src = pass & 1, dst = src ^ 1;
    PartArgs a;
    std::memset(&a, 0, sizeof(a));
    a.key = bk[src];
    a.key64 = 1;
    a.npay = 1;
    a.pay[0] = bv[src];
    a.pay64[0] = 1;
    a.out[0] = bk[dst];
    a.out[1] = bv[dst];
    a.d_nsel = d_count;
    a.n = cap;
    a.fanout = 256;
    a.fbits = 8;
    a.radix_shift = 8 * pass;
    pyst_status st = partition_run(ctx, a, nullptr, stream);
    if (st != PYST_OK) return st;
  }
  return PYST_OK;
}

// Exclusive scan with caller-provided look-back status: (tiles + 1) words,
// cleared here by a kernel.
pyst_status scan_excl_i32_ws(const int32_t *in, int32_t *out, int64_t len, int64_t *d_total, uint64_t *status,
                             hipStream_t stream) {
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(len, int64_t{kScanBlock} * kScanItems));
  pyst_status st = fill_u64(status, ntiles + 1, 0, stream);
  if (st != PYST_OK) return st;
  k_scan_excl_i32<kScanBlock, kScanItems><<<static_cast<unsigned>(ntiles), kScanBlock, 0, stream>>>(
      in, out, len, status, reinterpret_cast<unsigned long long *>(status + ntiles), ntiles, d_total);
  PYST_LAUNCH_CHECK("k_scan_excl_i32");
  return PYST_OK;
}

pyst_status scan_excl_i32(pyst_ctx *ctx, const int32_t *in, int32_t *out, int64_t len, int64_t *d_total,
                          hipStream_t stream) {
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(len, int64_t{kScanBlock} * kScanItems));
  Scratch sc(ctx, (ntiles + 1) * sizeof(uint64_t), stream);
  if (!sc.p) return set_error(PYST_ERR_NOMEM, "scan: arena exhausted");
  return scan_excl_i32_ws(in, out, len, d_total, sc.as<uint64_t>(), stream);
}

// ============================================================== join build / probe
// Key + payload table of int32 keys and int32 payloads (or row ids): 8-byte
// slots, (uint32 key) | (uint32 payload) << 32, EMPTY key INT32_MIN.
// A table keyed by int64, or carrying int64 payloads, takes 16-byte slots
// {int64 key, int64 payload} with EMPTY key INT64_MIN instead ("wide"): the
// key word is claimed by CAS and the payload stored after it, which a probe
// (a later launch) then sees.
constexpr uint64_t kEmptySlot = static_cast<uint32_t>(kEmpty32);

__global__ void k_table_init(TableDev t, const int64_t *d_nsel, int64_t n, double max_load) {
  const int64_t cnt = count_of(d_nsel, n);
  const int64_t cap = table_capacity(cnt, max_load, t.cap_alloc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    t.hdr[0] = cap;
    t.hdr[1] = cnt;
  }
  const int64_t words = t.slot_bytes == 4 ? cap / 2 : t.slot_bytes == 16 ? 2 * cap : cap;  // in 8-byte words
  const uint64_t fillv = t.slot_bytes == 4    ? (uint64_t{static_cast<uint32_t>(kEmpty32)} * 0x100000001ull)
                         : t.slot_bytes == 16 ? static_cast<uint64_t>(kEmpty64)
                                              : kEmptySlot;
  uint64_t *p = static_cast<uint64_t *>(t.slots);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = fillv;
  if (t.sums)
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cap; i += (int64_t)gridDim.x * blockDim.x) {
      t.sums[i] = 0;
      t.flags[i] = 0;
    }
}

// Each lane inserts ITEMS rows, one wave64 row apart: the ITEMS home slots are
// read together, then CAS'd together where empty (the read brings the line
// into the L2, where the atomic then runs; a CAS straight to a cold line
// measured slower), and only rows whose home slot was taken walk on.
constexpr int kBuildItems = 4;

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_join_build(const int32_t *key, const int32_t *payload, const int32_t *sel,
                                                      const int64_t *d_nsel, int64_t n, TableDev t, int unique,
                                                      uint32_t *err) {
  const int64_t cnt = count_of(d_nsel, n);
  const int64_t mask = t.hdr[0] - 1;
  auto *slots = reinterpret_cast<unsigned long long *>(t.slots);
  constexpr int64_t TILE = int64_t{BLOCK} * ITEMS;
  for (int64_t base = int64_t{blockIdx.x} * TILE + threadIdx.x; base < cnt; base += int64_t{gridDim.x} * TILE) {
    int32_t k[ITEMS];
    uint64_t packed[ITEMS], old[ITEMS];
    int64_t s[ITEMS];
    bool live[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int64_t i = base + int64_t{j} * BLOCK;
      live[j] = i < cnt;
      const int64_t row = live[j] ? row_of(sel, i) : 0;
      k[j] = live[j] ? key[row] : kEmpty32;
      const uint32_t pl = payload ? static_cast<uint32_t>(live[j] ? payload[row] : 0) : static_cast<uint32_t>(row);
      packed[j] = uint64_t{static_cast<uint32_t>(k[j])} | (uint64_t{pl} << 32);
      if (live[j] && k[j] == kEmpty32) {
        latch(err, kErrKey);
        live[j] = false;
      }
      s[j] = (table_hash32(k[j]) & mask) & ~int64_t{1};
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) old[j] = live[j] ? slots[s[j]] : kEmptySlot;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (live[j] && static_cast<int32_t>(old[j]) == kEmpty32) old[j] = atomicCAS(&slots[s[j]], kEmptySlot, packed[j]);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (!live[j] || old[j] == kEmptySlot) continue;
      bool done = false;
      uint64_t cur = old[j];
      int64_t p = s[j];
      for (int64_t step = 0; step <= mask; ++step) {
        if (unique && static_cast<int32_t>(cur) == k[j]) {
          latch(err, kErrDup);
          done = true;
          break;
        }
        p = (p + 1) & mask;
        cur = slots[p];
        if (static_cast<int32_t>(cur) == kEmpty32) {
          cur = atomicCAS(&slots[p], kEmptySlot, packed[j]);
          if (cur == kEmptySlot) {
            done = true;
            break;
          }
        }
      }
      if (!done) latch(err, kErrTableFull);
    }
  }
}

// Key of `row` in an int32 or int64 column, sign-extended; false for the
// column type's EMPTY sentinel, which is never stored and matches nothing.
__device__ __forceinline__ bool join_key(const void *key, int key64, int64_t row, int64_t &k) {
  if (key64) {
    k = static_cast<const int64_t *>(key)[row];
    return k != kEmpty64;
  }
  k = static_cast<const int32_t *>(key)[row];
  return k != kEmpty32;
}

// Insertion into a wide table, ITEMS rows per lane as in k_join_build.
template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_join_build_wide(const void *key, int key64, const void *payload, int pay64,
                                                           const int32_t *sel, const int64_t *d_nsel, int64_t n,
                                                           TableDev t, int unique, uint32_t *err) {
  const int64_t cnt = count_of(d_nsel, n);
  const int64_t mask = t.hdr[0] - 1;
  auto *slots = reinterpret_cast<unsigned long long *>(t.slots);  // slot s: words 2s (key), 2s + 1 (payload)
  constexpr unsigned long long kE = static_cast<unsigned long long>(kEmpty64);
  constexpr int64_t TILE = int64_t{BLOCK} * ITEMS;
  for (int64_t base = int64_t{blockIdx.x} * TILE + threadIdx.x; base < cnt; base += int64_t{gridDim.x} * TILE) {
    int64_t k[ITEMS], pl[ITEMS], s[ITEMS];
    unsigned long long old[ITEMS];
    bool live[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int64_t i = base + int64_t{j} * BLOCK;
      const int64_t row = i < cnt ? row_of(sel, i) : 0;
      k[j] = kEmpty64;
      live[j] = i < cnt && join_key(key, key64, row, k[j]);
      if (i < cnt && !live[j]) latch(err, kErrKey);
      pl[j] = payload ? (live[j] ? load_as_i64(payload, pay64, row) : 0) : row;
      s[j] = static_cast<int64_t>(table_hash64(k[j])) & mask;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) old[j] = live[j] ? slots[2 * s[j]] : kE;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (live[j] && old[j] == kE) old[j] = atomicCAS(&slots[2 * s[j]], kE, static_cast<unsigned long long>(k[j]));
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (!live[j]) continue;
      int64_t p = s[j];
      bool done = old[j] == kE, dup = false;  // done: took its home slot
      unsigned long long cur = old[j];
      for (int64_t step = 0; !done && step <= mask; ++step) {
        if (unique && static_cast<int64_t>(cur) == k[j]) {
          dup = true;
          break;
        }
        p = (p + 1) & mask;
        cur = slots[2 * p];
        if (cur == kE) {
          cur = atomicCAS(&slots[2 * p], kE, static_cast<unsigned long long>(k[j]));
          done = cur == kE;
        }
      }
      if (done) slots[2 * p + 1] = static_cast<unsigned long long>(pl[j]);
      else latch(err, dup ? kErrDup : kErrTableFull);
    }
  }
}

// Probe the key+payload table two slots (16 bytes) per load; calls on_match(payload)
// for each match in table order until on_match returns false or an EMPTY slot ends the run.
template <typename F>
__device__ __forceinline__ void probe_kp(const uint64_t *slots, int64_t mask, int32_t k, F &&on_match) {
  int64_t s = (table_hash32(k) & mask) & ~int64_t{1};
  for (int64_t step = 0; step <= mask; step += 2) {
    const ulonglong2 pair = *reinterpret_cast<const ulonglong2 *>(&slots[s]);
    const int32_t k0 = static_cast<int32_t>(pair.x), k1 = static_cast<int32_t>(pair.y);
    if (k0 == k) {
      if (!on_match(static_cast<int32_t>(pair.x >> 32))) return;
    } else if (k0 == kEmpty32) {
      return;
    }
    if (k1 == k) {
      if (!on_match(static_cast<int32_t>(pair.y >> 32))) return;
    } else if (k1 == kEmpty32) {
      return;
    }
    s = (s + 2) & mask;
  }
}

// Visits the two slots of one 16-byte group in table order: counts matches of
// k (remembering the first payload) and returns false once the run ends (an
// EMPTY slot, or the first match under unique keys).
__device__ __forceinline__ bool visit_pair(ulonglong2 pair, int32_t k, int unique, int32_t &c, int32_t &first) {
  const uint64_t sl[2] = {pair.x, pair.y};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int32_t key = static_cast<int32_t>(sl[h]);
    if (key == k) {
      if (c == 0) first = static_cast<int32_t>(sl[h] >> 32);
      ++c;
      if (unique) return false;
    } else if (key == kEmpty32) {
      return false;
    }
  }
  return true;
}

// The same for one slot {key, payload} of a wide table.
__device__ __forceinline__ bool visit_wide(ulonglong2 slot, int64_t k, int unique, int32_t &c, int64_t &first) {
  const int64_t key = static_cast<int64_t>(slot.x);
  if (key == k) {
    if (c == 0) first = static_cast<int64_t>(slot.y);
    ++c;
    return !unique;
  }
  return key != kEmpty64;
}

// Walks the run of k in a wide table, calling on_match(payload) per match
// until it returns false or an EMPTY slot ends the run.
template <typename F>
__device__ __forceinline__ void probe_wide(const uint64_t *slots, int64_t mask, int64_t k, F &&on_match) {
  int64_t s = static_cast<int64_t>(table_hash64(k)) & mask;
  for (int64_t step = 0; step <= mask; ++step) {
    const ulonglong2 sl = *reinterpret_cast<const ulonglong2 *>(&slots[2 * s]);
    if (static_cast<int64_t>(sl.x) == k) {
      if (!on_match(static_cast<int64_t>(sl.y))) return;
    } else if (static_cast<int64_t>(sl.x) == kEmpty64) {
      return;
    }
    s = (s + 1) & mask;
  }
}

// Each lane probes ITEMS rows, one wave64 row apart: the keys, then the ITEMS
// home groups (narrow table: two slots; wide: one) are loaded together, and
// only rows whose run goes on past their home group walk on.  Keys compare by
// value: an int64 probe key outside int32 range matches nothing in a narrow
// table, and a probe key equal to its column's EMPTY sentinel matches nothing.
// K64: the probe key column is int64.  PayT: int64 for stored payloads, int32
// for the build rows of a materializing join.
template <int BLOCK, int ITEMS, bool WIDE, bool K64, typename PayT>
__global__ __launch_bounds__(BLOCK) void k_join_probe(const void *key, const int32_t *sel,
                                                     const int64_t *d_nsel, int64_t n, TableDev t, int unique,
                                                     int32_t *out_row, PayT *out_pay, int64_t out_cap, int64_t *d_nout,
                                                     uint64_t *status, unsigned long long *ticket, int64_t ntiles,
                                                     uint32_t *err) {
  constexpr int NW = BLOCK / kWave;
  constexpr int64_t TILE = int64_t{BLOCK} * ITEMS;
  __shared__ int64_t s_tile, s_prefix;
  __shared__ int64_t s_w[NW];
  if (threadIdx.x == 0) s_tile = static_cast<int64_t>(atomicAdd(ticket, 1ull));
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t cnt = count_of(d_nsel, n);
  const int64_t mask = t.hdr[0] - 1;
  const uint64_t *slots = static_cast<const uint64_t *>(t.slots);
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t wbase = tile * TILE + int64_t{w} * kWave * ITEMS;
  constexpr int64_t GS = WIDE ? 1 : 2;  // slots per 16-byte group
  using KeyT = std::conditional_t<K64, int64_t, int32_t>;              // probe column
  using CmpT = std::conditional_t<WIDE || K64, int64_t, int32_t>;      // key as held
  using StoredT = std::conditional_t<WIDE, int64_t, int32_t>;          // table payload
  constexpr KeyT kColEmpty = K64 ? static_cast<KeyT>(kEmpty64) : static_cast<KeyT>(kEmpty32);
  CmpT kk[ITEMS];
  StoredT first_pay[ITEMS];
  int32_t c[ITEMS];
  int64_t s[ITEMS];
  ulonglong2 g[ITEMS];
  bool live[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t i = wbase + int64_t{j} * kWave + lane;
    const KeyT v = i < cnt ? static_cast<const KeyT *>(key)[row_of(sel, i)] : kColEmpty;
    kk[j] = v;
    live[j] = v != kColEmpty;
    if (!WIDE && K64) live[j] = live[j] && v > kEmpty32 && v <= INT32_MAX;  // fits the int32 table keys
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (WIDE) {
      s[j] = static_cast<int64_t>(table_hash64(static_cast<int64_t>(kk[j]))) & mask;
      g[j] = live[j] ? *reinterpret_cast<const ulonglong2 *>(&slots[2 * s[j]])
                     : ulonglong2{static_cast<uint64_t>(kEmpty64), 0};
    } else {
      s[j] = (table_hash32(static_cast<int32_t>(kk[j])) & mask) & ~int64_t{1};
      g[j] = live[j] ? *reinterpret_cast<const ulonglong2 *>(&slots[s[j]]) : ulonglong2{kEmptySlot, kEmptySlot};
    }
  }
  auto visit = [&](ulonglong2 x, int j) {
    if constexpr (WIDE) return visit_wide(x, kk[j], unique, c[j], first_pay[j]);
    else return visit_pair(x, static_cast<int32_t>(kk[j]), unique, c[j], first_pay[j]);
  };
  int64_t wave_total = 0;
  int64_t lane_off[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    c[j] = 0;
    first_pay[j] = 0;
    if (live[j] && visit(g[j], j)) {
      int64_t p = s[j];
      for (int64_t step = GS; step <= mask; step += GS) {
        p = (p + GS) & mask;
        if (!visit(*reinterpret_cast<const ulonglong2 *>(&slots[WIDE ? 2 * p : p]), j)) break;
      }
    }
    const int64_t incl = wave_inclusive_scan<int64_t>(c[j]);
    lane_off[j] = wave_total + incl - c[j];
    wave_total += __shfl(incl, kWave - 1);
  }
  if (lane == 0) s_w[w] = wave_total;
  __syncthreads();
  if (w == 0) {
    const int64_t v = lane < NW ? s_w[lane] : 0;
    const int64_t agg = wave_sum(v);
    const int64_t ex = lookback_exclusive(status, tile, agg);
    if (lane == 0) {
      s_prefix = ex;
      if (tile == ntiles - 1) {
        *d_nout = ex + agg;
        if (ex + agg > out_cap) latch(err, kErrCapacity);
      }
    }
  }
  __syncthreads();
  int64_t base = s_prefix;
  for (int k = 0; k < w; ++k) base += s_w[k];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (c[j] == 0) continue;
    const int64_t i = wbase + int64_t{j} * kWave + lane;
    const int32_t row = static_cast<int32_t>(row_of(sel, i));
    int64_t p = base + lane_off[j];
    if (c[j] == 1) {
      if (p < out_cap) {
        out_row[p] = row;
        out_pay[p] = static_cast<PayT>(first_pay[j]);
      }
    } else {
      auto emit = [&](int64_t pl) {
        if (p < out_cap) {
          out_row[p] = row;
          out_pay[p] = static_cast<PayT>(pl);
        }
        ++p;
        return true;
      };
      if constexpr (WIDE) probe_wide(slots, mask, kk[j], emit);
      else probe_kp(slots, mask, static_cast<int32_t>(kk[j]), emit);
    }
  }
}

// ============================================================== group-by SUM
// 16-byte slots {int64 key, uint64 sum}; EMPTY key = INT64_MIN.
__global__ void k_gb_init(GroupDev g, const int64_t *d_nsel, int64_t n, int64_t max_groups, double max_load) {
  int64_t cnt = count_of(d_nsel, n);
  if (max_groups > 0 && max_groups < cnt) cnt = max_groups;
  const int64_t cap = table_capacity(cnt, max_load, g.cap_alloc);
  if (blockIdx.x == 0 && threadIdx.x == 0) g.hdr[0] = cap;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cap; i += (int64_t)gridDim.x * blockDim.x) {
    g.slots[2 * i] = static_cast<uint64_t>(kEmpty64);
    g.slots[2 * i + 1] = 0;
  }
}

__global__ __launch_bounds__(256) void k_gb_insert(const void *key, int key64, const void *val, int val64,
                                                   const int32_t *sel, const int64_t *d_nsel, int64_t n, GroupDev g,
                                                   uint32_t *err, int skip_empty) {
  // skip_empty: the input is a pair buffer whose unused slots hold the EMPTY key
  int64_t cnt = count_of(d_nsel, n);
  if (cnt > n) cnt = n;
  const int64_t mask = g.hdr[0] - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = row_of(sel, i);
    const int64_t k = load_as_i64(key, key64, row);
    if (k == kEmpty64) {
      if (!skip_empty) latch(err, kErrKey);
      continue;
    }
    const int64_t v = load_as_i64(val, val64, row);
    if (!group_add(g.slots, mask, k, static_cast<uint64_t>(v))) latch(err, kErrTableFull);
  }
}

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_gb_compact(GroupDev g, int64_t *out_keys, int64_t *out_sums,
                                                     int64_t out_cap, int64_t *d_ngroups, uint64_t *status,
                                                     unsigned long long *ticket, int64_t ntiles, uint32_t *err) {
  constexpr int NW = BLOCK / kWave;
  constexpr int64_t TILE = int64_t{BLOCK} * ITEMS;
  __shared__ int64_t s_tile, s_prefix;
  __shared__ int32_t s_cnt[NW];
  if (threadIdx.x == 0) s_tile = static_cast<int64_t>(atomicAdd(ticket, 1ull));
  __syncthreads();
  const int64_t t = s_tile;
  const int64_t cap = g.hdr[0];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int64_t wbase = t * TILE + int64_t{w} * kWave * ITEMS;
  uint64_t m[ITEMS];
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t s = wbase + int64_t{j} * kWave + lane;
    const bool keep = s < cap && static_cast<int64_t>(g.slots[2 * s]) != kEmpty64;
    m[j] = __ballot(keep);
    cnt += __popcll(m[j]);
  }
  if (lane == 0) s_cnt[w] = cnt;
  __syncthreads();
  if (w == 0) {
    const int64_t c = lane < NW ? s_cnt[lane] : 0;
    const int64_t agg = wave_sum(c);
    const int64_t ex = lookback_exclusive(status, t, agg);
    if (lane == 0) {
      s_prefix = ex;
      if (t == ntiles - 1) {
        *d_ngroups = ex + agg;
        if (ex + agg > out_cap) latch(err, kErrCapacity);
      }
    }
  }
  __syncthreads();
  int64_t pos = s_prefix;
  for (int k = 0; k < w; ++k) pos += s_cnt[k];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t s = wbase + int64_t{j} * kWave + lane;
    if ((m[j] >> lane) & 1ull) {
      const int64_t p = pos + mbcnt(m[j]);
      if (p < out_cap) {
        out_keys[p] = static_cast<int64_t>(g.slots[2 * s]);
        out_sums[p] = static_cast<int64_t>(g.slots[2 * s + 1]);
      }
    }
    pos += __popcll(m[j]);
  }
}

pyst_status group_compact(pyst_ctx *ctx, const GroupDev &g, int64_t *out_keys, int64_t *out_sums, int64_t out_cap,
                          int64_t *d_ngroups, hipStream_t stream) {
  constexpr int BLOCK = 256, ITEMS = 8;
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(g.cap_alloc, int64_t{BLOCK} * ITEMS));
  Scratch sc(ctx, (ntiles + 1) * sizeof(uint64_t), stream);
  if (!sc.p) return set_error(PYST_ERR_NOMEM, "group compaction: arena exhausted");
  pyst_status st = fill_u64(sc.p, ntiles + 1, 0, stream);
  if (st != PYST_OK) return st;
  uint64_t *status = sc.as<uint64_t>();
  k_gb_compact<BLOCK, ITEMS><<<static_cast<unsigned>(ntiles), BLOCK, 0, stream>>>(
      g, out_keys, out_sums, out_cap, d_ngroups, status, reinterpret_cast<unsigned long long *>(status + ntiles),
      ntiles, ctx_err_word(ctx));
  PYST_LAUNCH_CHECK("k_gb_compact");
  return PYST_OK;
}

pyst_status group_init(const GroupDev &g, const int64_t *d_nsel, int64_t n, int64_t max_groups, double max_load,
                       hipStream_t stream) {
  const int blocks = static_cast<int>(std::min<int64_t>(ceil_div(g.cap_alloc, 256), 4096));
  k_gb_init<<<blocks, 256, 0, stream>>>(g, d_nsel, n, max_groups, max_load);
  PYST_LAUNCH_CHECK("k_gb_init");
  return PYST_OK;
}

// ============================================================== gather (materialize)
// Row-wise materialization of join results: dst[c][i] = src[c][idx[i]].  Each
// lane owns ITEMS output rows, one wave64 row apart, so the index loads and
// the stores of a wave are coalesced and the ITEMS value loads of a lane (one
// per row, random for a hash join's build side, ascending for its probe side)
// are in flight together.  An index outside [0, nsrc) is latched and its row
// left unwritten; no load is made for it.
struct GatherArgs {
  const void *src[PYST_MAX_COLS];
  void *dst[PYST_MAX_COLS];
  int32_t w64[PYST_MAX_COLS];
  int32_t ncols;
  int64_t nsrc;
};

template <int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_gather(GatherArgs a, const int32_t *idx, const int64_t *d_n, int64_t cap,
                                                  uint32_t *err) {
  int64_t n = d_n ? *d_n : cap;
  if (n > cap) n = cap;
  constexpr int64_t TILE = int64_t{BLOCK} * ITEMS;
  for (int64_t base = int64_t{blockIdx.x} * TILE + threadIdx.x; base < n; base += int64_t{gridDim.x} * TILE) {
    int64_t r[ITEMS];
    bool ok[ITEMS];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int64_t i = base + int64_t{j} * BLOCK;
      r[j] = i < n ? static_cast<int64_t>(__builtin_nontemporal_load(&idx[i])) : -1;
      ok[j] = r[j] >= 0 && r[j] < a.nsrc;
      bad |= i < n && !ok[j];
    }
    if (bad) latch(err, kErrIndex);
    for (int c = 0; c < a.ncols; ++c) {
      if (a.w64[c]) {
        const int64_t *s = static_cast<const int64_t *>(a.src[c]);
        int64_t *d = static_cast<int64_t *>(a.dst[c]);
        int64_t v[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) v[j] = ok[j] ? s[r[j]] : 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
          if (ok[j]) __builtin_nontemporal_store(v[j], &d[base + int64_t{j} * BLOCK]);
      } else {
        const int32_t *s = static_cast<const int32_t *>(a.src[c]);
        int32_t *d = static_cast<int32_t *>(a.dst[c]);
        int32_t v[ITEMS];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) v[j] = ok[j] ? s[r[j]] : 0;
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
          if (ok[j]) __builtin_nontemporal_store(v[j], &d[base + int64_t{j} * BLOCK]);
      }
    }
  }
}

// Row-major copy of a side's columns for random gathers: row r holds the
// ncols values (sign-extended to int64) at words [r*RS, r*RS + ncols), RS a
// power of two >= ncols, so one row is one aligned RS*8-byte block (at most a
// 64-byte line) and a gather reads it with RS/2 16-byte loads instead of
// ncols separate random 8-byte loads.
template <int RS>
__global__ __launch_bounds__(256) void k_pack_rows(GatherArgs a, int64_t *rows) {
  for (int64_t r = int64_t{blockIdx.x} * blockDim.x + threadIdx.x; r < a.nsrc; r += int64_t{gridDim.x} * blockDim.x) {
    int64_t v[RS];
#pragma unroll
    for (int c = 0; c < RS; ++c) {
      v[c] = 0;
      if (c < a.ncols)
        v[c] = a.w64[c] ? __builtin_nontemporal_load(&static_cast<const int64_t *>(a.src[c])[r])
                        : static_cast<int64_t>(__builtin_nontemporal_load(&static_cast<const int32_t *>(a.src[c])[r]));
    }
    if constexpr (RS == 1) {
      rows[r] = v[0];
    } else {
#pragma unroll
      for (int c = 0; c < RS; c += 2)
        *reinterpret_cast<longlong2 *>(&rows[r * RS + c]) = longlong2{v[c], v[c + 1]};
    }
  }
}

// dst[c][i] = column c of packed row idx[i], narrowed to the column's dtype;
// ITEMS rows per lane, one wave64 row apart, as k_gather.
template <int RS, int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_gather_rows(const int64_t *rows, GatherArgs a, const int32_t *idx,
                                                       const int64_t *d_n, int64_t cap, uint32_t *err) {
  int64_t n = d_n ? *d_n : cap;
  if (n > cap) n = cap;
  constexpr int64_t TILE = int64_t{BLOCK} * ITEMS;
  for (int64_t base = int64_t{blockIdx.x} * TILE + threadIdx.x; base < n; base += int64_t{gridDim.x} * TILE) {
    int64_t r[ITEMS];
    bool ok[ITEMS];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int64_t i = base + int64_t{j} * BLOCK;
      r[j] = i < n ? static_cast<int64_t>(__builtin_nontemporal_load(&idx[i])) : -1;
      ok[j] = r[j] >= 0 && r[j] < a.nsrc;
      bad |= i < n && !ok[j];
    }
    if (bad) latch(err, kErrIndex);
    int64_t v[ITEMS][RS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if constexpr (RS == 1) {
        v[j][0] = ok[j] ? rows[r[j]] : 0;
      } else {
#pragma unroll
        for (int c = 0; c < RS; c += 2) {
          const longlong2 x = ok[j] ? *reinterpret_cast<const longlong2 *>(&rows[r[j] * RS + c]) : longlong2{0, 0};
          v[j][c] = x.x;
          v[j][c + 1] = x.y;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < RS; ++c) {
      if (c >= a.ncols) break;
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        if (!ok[j]) continue;
        const int64_t i = base + int64_t{j} * BLOCK;
        if (a.w64[c])
          __builtin_nontemporal_store(v[j][c], &static_cast<int64_t *>(a.dst[c])[i]);
        else
          __builtin_nontemporal_store(static_cast<int32_t>(v[j][c]), &static_cast<int32_t *>(a.dst[c])[i]);
      }
    }
  }
}

// Defined with the pair aggregation and the context.
pyst_status column_groupby(pyst_ctx *ctx, const pyst_col *key, const pyst_col *val, const int32_t *sel,
                           const int64_t *count, int64_t *pk, int64_t *pv, int64_t *out_keys, int64_t *out_sums,
                           int64_t out_cap, int64_t *d_ngroups, hipStream_t stream);
bool ctx_groupby_hash_only(const pyst_ctx *ctx);

size_t narrow_groupby_bytes(int64_t cap);
pyst_status narrow_groupby(pyst_ctx *ctx, const int32_t *kcol, const int32_t *vcol, const int32_t *sel,
                           const int64_t *count, int64_t cap, void *ws, int64_t *out_keys, int64_t *out_sums,
                           int64_t out_cap, int64_t *d_ngroups, hipStream_t stream);

// The radix path groups 4096 hash buckets in an LDS table of 8192 slots each:
// up to 16M groups a bucket holds 4096 keys on average, 64 standard deviations
// below its capacity.  Below 1M rows the HBM hash table stays in the L2.
constexpr int64_t kRadixGroupsMax = int64_t{1} << 24;
constexpr int64_t kRadixRowsMin = int64_t{1} << 20;

int grid_for(pyst_ctx *ctx, int64_t work, int block, int per_cu) {
  const int64_t want = ceil_div(std::max<int64_t>(work, 1), block);
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, int64_t{ctx_num_cus(ctx)} * per_cu)));
}

pyst_status table_init(const TableDev &t, const int64_t *d_nsel, int64_t n, double max_load, hipStream_t stream) {
  const int blocks = static_cast<int>(std::min<int64_t>(ceil_div(t.cap_alloc, 256), 4096));
  k_table_init<<<blocks, 256, 0, stream>>>(t, d_nsel, n, max_load);
  PYST_LAUNCH_CHECK("k_table_init");
  return PYST_OK;
}

// Slot size of a join table: 8 bytes for int32 keys with int32 payloads (or
// row ids), 16 for int64 keys or int64 payloads.
static int join_slot_bytes(const pyst_col *key, const pyst_col *payload) {
  return key->dtype == PYST_I64 || (payload && payload->dtype == PYST_I64) ? 16 : 8;
}

// Table init + insertion of the selected rows (payload: a column of the key's
// length, or null for row ids); t.slot_bytes is join_slot_bytes of the columns.
pyst_status launch_join_build(pyst_ctx *ctx, const TableDev &t, const pyst_col *key, const pyst_col *payload,
                              const int32_t *sel, const int64_t *d_nsel, double max_load, int unique,
                              hipStream_t stream) {
  pyst_status st = table_init(t, d_nsel, key->n, max_load, stream);
  if (st != PYST_OK || key->n == 0) return st;
  const int blocks = grid_for(ctx, ceil_div(key->n, int64_t{kBuildItems}), 256, 8);
  if (t.slot_bytes == 16) {
    k_join_build_wide<256, kBuildItems><<<blocks, 256, 0, stream>>>(
        key->data, key->dtype == PYST_I64, payload ? payload->data : nullptr, payload && payload->dtype == PYST_I64,
        sel, d_nsel, key->n, t, unique, ctx_err_word(ctx));
  } else {
    k_join_build<256, kBuildItems><<<blocks, 256, 0, stream>>>(
        static_cast<const int32_t *>(key->data), payload ? static_cast<const int32_t *>(payload->data) : nullptr, sel,
        d_nsel, key->n, t, unique, ctx_err_word(ctx));
  }
  PYST_LAUNCH_CHECK("k_join_build");
  return PYST_OK;
}

template <typename PayT>
pyst_status launch_join_probe(pyst_ctx *ctx, const TableDev &t, int unique, const pyst_col *key, const int32_t *sel,
                              const int64_t *d_nsel, int32_t *out_row, PayT *out_pay, int64_t out_cap,
                              int64_t *d_nout, hipStream_t stream) {
  constexpr int BLOCK = 256, ITEMS = 8;
  const int64_t ntiles = std::max<int64_t>(1, ceil_div(key->n, int64_t{BLOCK} * ITEMS));
  Scratch sc(ctx, (ntiles + 1) * sizeof(uint64_t), stream);
  if (!sc.p) return set_error(PYST_ERR_NOMEM, "join probe: arena exhausted");
  pyst_status st = fill_u64(sc.p, ntiles + 1, 0, stream);
  if (st != PYST_OK) return st;
  uint64_t *status = sc.as<uint64_t>();
  auto *ticket = reinterpret_cast<unsigned long long *>(status + ntiles);
  const unsigned grid = static_cast<unsigned>(ntiles);
  uint32_t *err = ctx_err_word(ctx);
  const bool wide = t.slot_bytes == 16, k64 = key->dtype == PYST_I64;
  if (wide && k64)
    k_join_probe<BLOCK, ITEMS, true, true, PayT><<<grid, BLOCK, 0, stream>>>(
        key->data, sel, d_nsel, key->n, t, unique, out_row, out_pay, out_cap, d_nout, status, ticket, ntiles, err);
  else if (wide)
    k_join_probe<BLOCK, ITEMS, true, false, PayT><<<grid, BLOCK, 0, stream>>>(
        key->data, sel, d_nsel, key->n, t, unique, out_row, out_pay, out_cap, d_nout, status, ticket, ntiles, err);
  else if (k64)
    k_join_probe<BLOCK, ITEMS, false, true, PayT><<<grid, BLOCK, 0, stream>>>(
        key->data, sel, d_nsel, key->n, t, unique, out_row, out_pay, out_cap, d_nout, status, ticket, ntiles, err);
  else
    k_join_probe<BLOCK, ITEMS, false, false, PayT><<<grid, BLOCK, 0, stream>>>(
        key->data, sel, d_nsel, key->n, t, unique, out_row, out_pay, out_cap, d_nout, status, ticket, ntiles, err);
  PYST_LAUNCH_CHECK("k_join_probe");
  return PYST_OK;
}

// Validates the columns of one gather call into `a`.
pyst_status gather_args(const pyst_col *cols, int ncols, void *const *out_cols, int64_t cap, GatherArgs *a,
                        const char *who) {
  if (ncols < 1 || ncols > PYST_MAX_COLS) return set_error(PYST_ERR_ARG, std::string(who) + ": 1..8 columns");
  if (!cols || !out_cols) return set_error(PYST_ERR_ARG, std::string(who) + ": NULL columns");
  std::memset(a, 0, sizeof(*a));
  a->ncols = ncols;
  a->nsrc = cols[0].n;
  for (int c = 0; c < ncols; ++c) {
    if (!col_ok(&cols[c]) || cols[c].n != a->nsrc)
      return set_error(PYST_ERR_ARG, std::string(who) + ": bad column or length mismatch");
    if (cap > 0 && !out_cols[c]) return set_error(PYST_ERR_ARG, std::string(who) + ": NULL output column");
    a->src[c] = cols[c].data;
    a->dst[c] = out_cols[c];
    a->w64[c] = cols[c].dtype == PYST_I64;
  }
  return PYST_OK;
}

pyst_status launch_gather(pyst_ctx *ctx, const GatherArgs &a, const int32_t *idx, const int64_t *d_n, int64_t cap,
                          hipStream_t stream) {
  if (cap == 0) return PYST_OK;
  TimedRegion timed(ctx, "gather", stream);
  constexpr int BLOCK = 256, ITEMS = 8;
  const int blocks = grid_for(ctx, ceil_div(cap, int64_t{ITEMS}), BLOCK, 8);
  k_gather<BLOCK, ITEMS><<<blocks, BLOCK, 0, stream>>>(a, idx, d_n, cap, ctx_err_word(ctx));
  PYST_LAUNCH_CHECK("k_gather");
  return PYST_OK;
}

int row_words(int ncols) {
  int rs = 1;
  while (rs < ncols) rs *= 2;
  return rs;
}

template <int RS>
pyst_status launch_rows(pyst_ctx *ctx, const GatherArgs &a, int64_t *rows, const int32_t *idx, const int64_t *d_n,
                        int64_t cap, hipStream_t stream) {
  {
    TimedRegion timed(ctx, "pack_rows", stream);
    const int blocks = grid_for(ctx, a.nsrc, 256, 8);
    k_pack_rows<RS><<<blocks, 256, 0, stream>>>(a, rows);
    PYST_LAUNCH_CHECK("k_pack_rows");
  }
  if (cap == 0) return PYST_OK;
  TimedRegion timed(ctx, "gather_rows", stream);
  constexpr int BLOCK = 256, ITEMS = RS >= 8 ? 4 : 8;
  const int blocks = grid_for(ctx, ceil_div(cap, int64_t{ITEMS}), BLOCK, 8);
  k_gather_rows<RS, BLOCK, ITEMS><<<blocks, BLOCK, 0, stream>>>(rows, a, idx, d_n, cap, ctx_err_word(ctx));
  PYST_LAUNCH_CHECK("k_gather_rows");
  return PYST_OK;
}

// Gather through a row-major copy of the source columns (`rows`: nsrc * row_words(ncols) int64).
pyst_status launch_gather_rows(pyst_ctx *ctx, const GatherArgs &a, int64_t *rows, const int32_t *idx,
                               const int64_t *d_n, int64_t cap, hipStream_t stream) {
  if (a.nsrc == 0) return launch_gather(ctx, a, idx, d_n, cap, stream);
  switch (row_words(a.ncols)) {
    case 1: return launch_rows<1>(ctx, a, rows, idx, d_n, cap, stream);
    case 2: return launch_rows<2>(ctx, a, rows, idx, d_n, cap, stream);
    case 4: return launch_rows<4>(ctx, a, rows, idx, d_n, cap, stream);
    default: return launch_rows<8>(ctx, a, rows, idx, d_n, cap, stream);
  }
}

}  // namespace pyst

// ============================================================== C ABI
using namespace pyst;

struct pyst_table {
  pyst_ctx *ctx;
  void *mem;
  TableDev dev;
  int unique;
  hipStream_t stream;
};

extern "C" {

pyst_status pyst_filter(pyst_ctx *ctx, const pyst_col *cols, int ncols, const pyst_pred *preds, int npreds,
                        int32_t *sel_out, int64_t *d_nsel, hipStream_t stream) {
  if (!ctx || !d_nsel) return set_error(PYST_ERR_ARG, "pyst_filter: NULL ctx or d_nsel");
  if (ncols < 1 || ncols > PYST_MAX_COLS || !cols) return set_error(PYST_ERR_ARG, "pyst_filter: 1..8 columns required");
  const int64_t n = cols[0].n;
  for (int c = 0; c < ncols; ++c)
    if (!col_ok(&cols[c]) || cols[c].n != n) return set_error(PYST_ERR_ARG, "pyst_filter: bad column or length mismatch");
  if (n > 0 && !sel_out) return set_error(PYST_ERR_ARG, "pyst_filter: sel_out is NULL");
  PredSet ps;
  pyst_status st = build_predset(cols, ncols, preds, npreds, &ps, "pyst_filter");
  if (st != PYST_OK) return st;
  return filter_impl(ctx, ps, n, sel_out, d_nsel, stream);
}

// Argument checks and kernel arguments shared by the partition entry points.
static pyst_status partition_args(const pyst_col *key, const pyst_col *payloads, int npay, const int32_t *sel,
                                  const int64_t *d_nsel, uint32_t fanout, void *const *out_cols, int64_t *d_offsets,
                                  PartArgs *out) {
  if (!key || !out_cols || !d_offsets) return set_error(PYST_ERR_ARG, "pyst_partition: NULL argument");
  if (fanout < 1 || fanout > PYST_MAX_FANOUT) return set_error(PYST_ERR_ARG, "pyst_partition: fanout must be 1..1024");
  if (npay < 0 || npay > PYST_MAX_PART_PAYLOADS || (npay > 0 && !payloads))
    return set_error(PYST_ERR_ARG, "pyst_partition: 0..15 payload columns");
  if ((sel == nullptr) != (d_nsel == nullptr)) return set_error(PYST_ERR_ARG, "pyst_partition: sel and d_nsel go together");
  if (!col_ok(key)) return set_error(PYST_ERR_ARG, "pyst_partition: bad key column");
  for (int j = 0; j < npay; ++j)
    if (!col_ok(&payloads[j]) || payloads[j].n != key->n)
      return set_error(PYST_ERR_ARG, "pyst_partition: payload length mismatch");
  for (int j = 0; j <= npay; ++j)
    if (!out_cols[j] && key->n > 0) return set_error(PYST_ERR_ARG, "pyst_partition: NULL output column");
  PartArgs &a = *out;
  std::memset(&a, 0, sizeof(a));
  a.key = key->data;
  a.key64 = key->dtype == PYST_I64;
  a.npay = npay;
  for (int j = 0; j < npay; ++j) {
    a.pay[j] = payloads[j].data;
    a.pay64[j] = payloads[j].dtype == PYST_I64;
  }
  for (int j = 0; j <= npay; ++j) a.out[j] = out_cols[j];
  a.sel = sel;
  a.d_nsel = d_nsel;
  a.n = key->n;
  a.fanout = fanout;
  int bits = 0;
  while ((1u << bits) < fanout) ++bits;
  a.fbits = bits;
  a.radix_shift = -1;
  return PYST_OK;
}

pyst_status pyst_partition(pyst_ctx *ctx, const pyst_col *key, const pyst_col *payloads, int npay, const int32_t *sel,
                           const int64_t *d_nsel, uint32_t fanout, void *const *out_cols, int64_t *d_offsets,
                           hipStream_t stream) {
  if (!ctx) return set_error(PYST_ERR_ARG, "pyst_partition: NULL argument");
  PartArgs a;
  pyst_status st = partition_args(key, payloads, npay, sel, d_nsel, fanout, out_cols, d_offsets, &a);
  if (st != PYST_OK) return st;
  TimedRegion timed(ctx, "partition", stream);
  return partition_run(ctx, a, d_offsets, stream);
}

// The partition of callers that cannot allocate: its scratch is `scratch`, a
// fixed array in every GPU's copy of the code object.  Host code must not pass
// the array's name to a kernel (on the host it is only a stand-in): each
// device's address is taken once with hipGetSymbolAddress and kept here.
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[kNoallocMaxDevices];

static pyst_status noalloc_scratch(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_error(e, "pyst_partition_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kNoallocMaxDevices) return set_error(PYST_ERR_UNSUPPORTED, "pyst_partition_noalloc: device id over 63");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_error(e, "pyst_partition_noalloc: hipGetSymbolAddress(scratch)");
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return PYST_OK;
}

pyst_status pyst_partition_noalloc(const pyst_col *key, const pyst_col *payloads, int npay, const int32_t *sel,
                                   const int64_t *d_nsel, uint32_t fanout, void *const *out_cols,
                                   int64_t *d_offsets, hipStream_t stream) {
  PartArgs a;
  pyst_status st = partition_args(key, payloads, npay, sel, d_nsel, fanout, out_cols, d_offsets, &a);
  if (st != PYST_OK) return st;
  const size_t need = partition_scratch_bytes(a.n, a.fanout);
  if (need > sizeof(scratch))
    return set_error(PYST_ERR_CAPACITY, "pyst_partition_noalloc: " + std::to_string(a.n) + " rows at fanout " +
                                            std::to_string(a.fanout) + " need " + std::to_string(need) +
                                            " bytes of scratch, more than the fixed " +
                                            std::to_string(sizeof(scratch)));
  void *ws = nullptr;
  if ((st = noalloc_scratch(&ws)) != PYST_OK) return st;
  return partition_run_ws(nullptr, a, d_offsets, ws, stream);
}

pyst_status pyst_join_build(pyst_ctx *ctx, const pyst_col *key, const pyst_col *payload, const int32_t *sel,
                            const int64_t *d_nsel, double max_load, int unique_keys, pyst_table **out,
                            hipStream_t stream) {
  if (!ctx || !key || !out) return set_error(PYST_ERR_ARG, "pyst_join_build: NULL argument");
  *out = nullptr;
  if (!col_ok(key)) return set_error(PYST_ERR_ARG, "pyst_join_build: bad key column");
  if (payload && (!col_ok(payload) || payload->n != key->n))
    return set_error(PYST_ERR_ARG, "pyst_join_build: payload must be a column of the key's length");
  if (!(max_load > 0.0 && max_load <= 0.95)) return set_error(PYST_ERR_ARG, "pyst_join_build: max_load in (0, 0.95]");
  if ((sel == nullptr) != (d_nsel == nullptr)) return set_error(PYST_ERR_ARG, "pyst_join_build: sel and d_nsel go together");
  TimedRegion timed(ctx, "join_build", stream);
  const int64_t cap_alloc = table_capacity_host(key->n, max_load);
  const int slot_bytes = join_slot_bytes(key, payload);
  const size_t bytes = table_bytes(cap_alloc, slot_bytes, false);
  void *mem = ctx_alloc(ctx, bytes, stream);
  if (!mem) return set_error(PYST_ERR_NOMEM, "pyst_join_build: arena exhausted");
  auto *t = new pyst_table();
  t->ctx = ctx;
  t->mem = mem;
  t->dev = table_view(mem, cap_alloc, slot_bytes, false);
  t->unique = unique_keys != 0;
  t->stream = stream;
  pyst_status st = launch_join_build(ctx, t->dev, key, payload, sel, d_nsel, max_load, t->unique, stream);
  if (st != PYST_OK) {
    pyst_table_destroy(t, stream);
    return st;
  }
  *out = t;
  return PYST_OK;
}

pyst_status pyst_join_probe(pyst_ctx *ctx, const pyst_table *table, const pyst_col *key, const int32_t *sel,
                            const int64_t *d_nsel, int32_t *out_probe_row, int64_t *out_payload, int64_t out_cap,
                            int64_t *d_nout, hipStream_t stream) {
  if (!ctx || !table || !key || !d_nout) return set_error(PYST_ERR_ARG, "pyst_join_probe: NULL argument");
  if (!col_ok(key)) return set_error(PYST_ERR_ARG, "pyst_join_probe: bad key column");
  if (out_cap < 0 || (out_cap > 0 && (!out_probe_row || !out_payload)))
    return set_error(PYST_ERR_ARG, "pyst_join_probe: bad output");
  if ((sel == nullptr) != (d_nsel == nullptr)) return set_error(PYST_ERR_ARG, "pyst_join_probe: sel and d_nsel go together");
  TimedRegion timed(ctx, "join_probe", stream);
  pyst_status st = launch_join_probe(ctx, table->dev, table->unique, key, sel, d_nsel, out_probe_row, out_payload,
                                     out_cap, d_nout, stream);
  if (st != PYST_OK) return st;
  const_cast<pyst_table *>(table)->stream = stream;
  return PYST_OK;
}

pyst_status pyst_gather(pyst_ctx *ctx, const int32_t *idx, const int64_t *d_n, int64_t cap, const pyst_col *cols,
                        int ncols, void *const *out_cols, hipStream_t stream) {
  if (!ctx) return set_error(PYST_ERR_ARG, "pyst_gather: ctx is NULL");
  if (cap < 0 || cap > INT32_MAX) return set_error(PYST_ERR_ARG, "pyst_gather: cap in [0, 2^31)");
  if (cap > 0 && !idx) return set_error(PYST_ERR_ARG, "pyst_gather: idx is NULL");
  GatherArgs a;
  pyst_status st = gather_args(cols, ncols, out_cols, cap, &a, "pyst_gather");
  if (st != PYST_OK) return st;
  return launch_gather(ctx, a, idx, d_n, cap, stream);
}

pyst_status pyst_join_materialize(pyst_ctx *ctx, const pyst_col *build_key, const pyst_col *build_cols, int nbcols,
                                  const pyst_col *probe_key, const pyst_col *probe_cols, int npcols, double max_load,
                                  int unique_keys, void *const *out_cols, int32_t *out_probe_row,
                                  int32_t *out_build_row, int64_t out_cap, int64_t *d_nout, hipStream_t stream) {
  if (!ctx || !build_key || !probe_key || !d_nout) return set_error(PYST_ERR_ARG, "pyst_join_materialize: NULL argument");
  if (!col_ok(build_key) || !col_ok(probe_key)) return set_error(PYST_ERR_ARG, "pyst_join_materialize: bad key column");
  if (!(max_load > 0.0 && max_load <= 0.95)) return set_error(PYST_ERR_ARG, "pyst_join_materialize: max_load in (0, 0.95]");
  if (out_cap < 0 || out_cap > INT32_MAX || (out_cap > 0 && (!out_probe_row || !out_build_row)))
    return set_error(PYST_ERR_ARG, "pyst_join_materialize: bad output");
  if (npcols > 0 && !out_cols) return set_error(PYST_ERR_ARG, "pyst_join_materialize: NULL output columns");
  if (nbcols > 0 && !out_cols) return set_error(PYST_ERR_ARG, "pyst_join_materialize: NULL output columns");
  GatherArgs ga[2];
  const pyst_col *keys[2] = {probe_key, build_key};
  const pyst_col *cols[2] = {probe_cols, build_cols};
  const int nc[2] = {npcols, nbcols};
  for (int side = 0; side < 2; ++side) {
    if (nc[side] < 0 || nc[side] > PYST_MAX_COLS) return set_error(PYST_ERR_ARG, "pyst_join_materialize: 0..8 columns a side");
    if (nc[side] == 0) continue;
    pyst_status st = gather_args(cols[side], nc[side], out_cols + (side ? npcols : 0), out_cap, &ga[side],
                                 "pyst_join_materialize");
    if (st != PYST_OK) return st;
    if (ga[side].nsrc != keys[side]->n) return set_error(PYST_ERR_ARG, "pyst_join_materialize: column length differs from its key");
  }
  const int64_t cap_alloc = table_capacity_host(build_key->n, max_load);
  const int slot_bytes = join_slot_bytes(build_key, nullptr);
  Scratch mem(ctx, table_bytes(cap_alloc, slot_bytes, false), stream);
  if (!mem.p) return set_error(PYST_ERR_NOMEM, "pyst_join_materialize: arena exhausted");
  const TableDev t = table_view(mem.p, cap_alloc, slot_bytes, false);
  pyst_status st;
  {
    TimedRegion timed(ctx, "join_build", stream);
    st = launch_join_build(ctx, t, build_key, nullptr, nullptr, nullptr, max_load, unique_keys != 0, stream);
  }
  if (st != PYST_OK) return st;
  {
    TimedRegion timed(ctx, "join_probe", stream);
    st = launch_join_probe(ctx, t, unique_keys != 0, probe_key, nullptr, nullptr, out_probe_row, out_build_row, out_cap,
                           d_nout, stream);
  }
  if (st != PYST_OK) return st;
  if (npcols > 0 && (st = launch_gather(ctx, ga[0], out_probe_row, d_nout, out_cap, stream)) != PYST_OK) return st;
  if (nbcols == 1 && (st = launch_gather(ctx, ga[1], out_build_row, d_nout, out_cap, stream)) != PYST_OK) return st;
  if (nbcols > 1) {
    // several build columns: one random read of a packed row per match instead of one per column
    Scratch rows(ctx, static_cast<size_t>(build_key->n) * row_words(nbcols) * sizeof(int64_t), stream);
    if (!rows.p && build_key->n > 0) return set_error(PYST_ERR_NOMEM, "pyst_join_materialize: arena exhausted");
    if ((st = launch_gather_rows(ctx, ga[1], rows.as<int64_t>(), out_build_row, d_nout, out_cap, stream)) != PYST_OK)
      return st;
  }
  return PYST_OK;
}

pyst_status pyst_table_info(const pyst_table *table, int64_t *d_out, hipStream_t stream) {
  if (!table || !d_out) return set_error(PYST_ERR_ARG, "pyst_table_info: NULL argument");
  hipError_t e = hipMemcpyAsync(d_out, table->dev.hdr, 2 * sizeof(int64_t), hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(table header)");
  return PYST_OK;
}

void pyst_table_destroy(pyst_table *table, hipStream_t stream) {
  if (!table) return;
  (void)hipStreamSynchronize(stream);
  if (table->stream && table->stream != stream) (void)hipStreamSynchronize(table->stream);
  ctx_free_eager(table->ctx, table->mem, stream);  // the caller's stream may go away after this
  delete table;
}

pyst_status pyst_groupby_sum(pyst_ctx *ctx, const pyst_col *key, const pyst_col *val, const int32_t *sel,
                             const int64_t *d_nsel, int64_t max_groups, double max_load, int64_t *out_keys,
                             int64_t *out_sums, int64_t *d_ngroups, int sort_by_key, hipStream_t stream) {
  if (!ctx || !key || !val || !d_ngroups) return set_error(PYST_ERR_ARG, "pyst_groupby_sum: NULL argument");
  if (!col_ok(key) || !col_ok(val) || key->n != val->n)
    return set_error(PYST_ERR_ARG, "pyst_groupby_sum: bad columns or length mismatch");
  if (!(max_load > 0.0 && max_load <= 0.95)) return set_error(PYST_ERR_ARG, "pyst_groupby_sum: max_load in (0, 0.95]");
  if ((sel == nullptr) != (d_nsel == nullptr)) return set_error(PYST_ERR_ARG, "pyst_groupby_sum: sel and d_nsel go together");
  const int64_t bound = max_groups > 0 ? std::min<int64_t>(max_groups, key->n) : key->n;
  const int64_t out_cap = max_groups > 0 ? max_groups : key->n;
  if (out_cap > 0 && (!out_keys || !out_sums)) return set_error(PYST_ERR_ARG, "pyst_groupby_sum: NULL outputs");
  if (!ctx_groupby_hash_only(ctx) && key->n >= kRadixRowsMin && bound <= kRadixGroupsMax) {
    // Radix-partitioned: the rows are moved twice by hash bits into 4096 buckets
    // (the first move reading the columns) and each bucket is summed in LDS,
    // instead of two random L2 atomics per row.
    TimedRegion timed(ctx, "groupby_radix", stream);
    if (key->dtype == PYST_I32 && val->dtype == PYST_I32) {  // 8-byte pairs
      Scratch ws(ctx, narrow_groupby_bytes(key->n) + 256, stream);
      if (!ws.p) return set_error(PYST_ERR_NOMEM, "pyst_groupby_sum: arena exhausted");
      int64_t *d_cnt = reinterpret_cast<int64_t *>(static_cast<char *>(ws.p) + narrow_groupby_bytes(key->n));
      pyst_status st = fill_u64(d_ngroups, 1, 0, stream);
      if (st == PYST_OK && !d_nsel) st = fill_u64(d_cnt, 1, static_cast<uint64_t>(key->n), stream);
      if (st == PYST_OK)
        st = narrow_groupby(ctx, static_cast<const int32_t *>(key->data), static_cast<const int32_t *>(val->data), sel,
                            d_nsel ? d_nsel : d_cnt, key->n, ws.p, out_keys, out_sums, out_cap, d_ngroups, stream);
      if (st != PYST_OK) return st;
      if (sort_by_key) return sort_pairs_by_key(ctx, out_keys, out_sums, d_ngroups, out_cap, stream);
      return PYST_OK;
    }
    Scratch pairs(ctx, static_cast<size_t>(key->n) * 16 + 256, stream);
    if (!pairs.p) return set_error(PYST_ERR_NOMEM, "pyst_groupby_sum: arena exhausted");
    int64_t *pk = pairs.as<int64_t>(), *pv = pk + key->n, *d_cnt = pv + key->n;
    pyst_status st = fill_u64(d_ngroups, 1, 0, stream);
    if (st == PYST_OK && !d_nsel) st = fill_u64(d_cnt, 1, static_cast<uint64_t>(key->n), stream);
    if (st != PYST_OK) return st;
    st = column_groupby(ctx, key, val, sel, d_nsel ? d_nsel : d_cnt, pk, pv, out_keys, out_sums, out_cap, d_ngroups,
                        stream);
    if (st != PYST_OK) return st;
    if (sort_by_key) return sort_pairs_by_key(ctx, out_keys, out_sums, d_ngroups, out_cap, stream);
    return PYST_OK;
  }
  TimedRegion timed(ctx, "groupby_hash", stream);
  const int64_t cap_alloc = table_capacity_host(bound, max_load);
  Scratch mem(ctx, group_bytes(cap_alloc), stream);
  if (!mem.p) return set_error(PYST_ERR_NOMEM, "pyst_groupby_sum: arena exhausted");
  GroupDev g = group_view(mem.p, cap_alloc);
  pyst_status st = group_init(g, d_nsel, key->n, max_groups, max_load, stream);
  if (st != PYST_OK) return st;
  if (key->n > 0) {
    const int blocks = grid_for(ctx, key->n, 256, 8);
    k_gb_insert<<<blocks, 256, 0, stream>>>(key->data, key->dtype == PYST_I64, val->data, val->dtype == PYST_I64, sel,
                                            d_nsel, key->n, g, ctx_err_word(ctx), 0);
    PYST_LAUNCH_CHECK("k_gb_insert");
  }
  st = group_compact(ctx, g, out_keys, out_sums, out_cap, d_ngroups, stream);
  if (st != PYST_OK) return st;
  if (sort_by_key) return sort_pairs_by_key(ctx, out_keys, out_sums, d_ngroups, out_cap, stream);
  return PYST_OK;
}

}  // extern "C"

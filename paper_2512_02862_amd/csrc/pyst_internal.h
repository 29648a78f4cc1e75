// Internal definitions shared by the HIP translation units of libpyst.
// gfx950 (CDNA4) only: wave64, no dual code paths.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "pyst.h"

namespace pyst {

constexpr int kWave = 64;

// Clang vector types (usable with the nontemporal load/store builtins).
typedef int32_t v4i32 __attribute__((ext_vector_type(4)));
typedef int64_t v2i64 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------ error latch
// Bits set by kernels in the context's device error word (see pyst_ctx_check).
enum : uint32_t { kErrKey = 1u, kErrTableFull = 2u, kErrCapacity = 4u, kErrDup = 8u, kErrIndex = 16u };

__device__ inline void latch(uint32_t *err, uint32_t bit) { atomicOr(err, bit); }

// ------------------------------------------------------------------ hashing
// MurmurHash3 finalizers (public domain), used for partition destinations.
__host__ __device__ inline uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

__host__ __device__ inline uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// Hash-table slot hashes are seeded so their bits are independent of the
// partition destination bits (a partition holds keys with equal fmix32 low
// bits; an unseeded table would crowd them into 1/F of its slots).
constexpr uint32_t kTableSeed32 = 0x2545f491u;
constexpr uint64_t kTableSeed64 = 0x9e3779b97f4a7c15ull;
__device__ inline uint32_t table_hash32(int32_t key) { return fmix32(static_cast<uint32_t>(key) ^ kTableSeed32); }
__device__ inline uint64_t table_hash64(int64_t key) { return fmix64(static_cast<uint64_t>(key) ^ kTableSeed64); }

constexpr int32_t kEmpty32 = INT32_MIN;
constexpr int64_t kEmpty64 = INT64_MIN;

// ------------------------------------------------------------------ predicates
struct PredSet {
  const void *col[PYST_MAX_PREDS];
  int32_t is64[PYST_MAX_PREDS];
  int32_t op[PYST_MAX_PREDS];
  int64_t val[PYST_MAX_PREDS];
  int32_t n;
};

__device__ __forceinline__ bool compare_op(int64_t x, int op, int64_t c) {
  switch (op) {
    case PYST_EQ: return x == c;
    case PYST_NE: return x != c;
    case PYST_LT: return x < c;
    case PYST_LE: return x <= c;
    case PYST_GT: return x > c;
    default: return x >= c;
  }
}

__device__ __forceinline__ int64_t load_as_i64(const void *p, int is64, int64_t i) {
  return is64 ? static_cast<const int64_t *>(p)[i] : static_cast<int64_t>(static_cast<const int32_t *>(p)[i]);
}

// Load element rows[j] of a column for every item before any of them is used,
// so the ITEMS loads of a wave are in flight together.  Rows are clamped to
// [0, n) so every address is valid; callers mask the out-of-range items.
template <int ITEMS>
__device__ __forceinline__ void load_items(const void *col, int is64, const int64_t (&rows)[ITEMS], int64_t n,
                                           int64_t (&x)[ITEMS]) {
  const int64_t last = n > 0 ? n - 1 : 0;
  if (is64) {
    const int64_t *p = static_cast<const int64_t *>(col);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) x[j] = p[rows[j] < last ? rows[j] : last];
  } else {
    const int32_t *p = static_cast<const int32_t *>(col);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) x[j] = p[rows[j] < last ? rows[j] : last];
  }
}

// keep[j] = rows[j] < n and every predicate holds for row rows[j].
template <int ITEMS>
__device__ __forceinline__ void eval_preds_items(const PredSet &ps, const int64_t (&rows)[ITEMS], int64_t n,
                                                 bool (&keep)[ITEMS]) {
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) keep[j] = rows[j] < n;
  if (n <= 0) return;
  for (int k = 0; k < ps.n; ++k) {
    int64_t x[ITEMS];
    load_items<ITEMS>(ps.col[k], ps.is64[k], rows, n, x);
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) keep[j] = keep[j] && compare_op(x[j], ps.op[k], ps.val[k]);
  }
}

__device__ __forceinline__ bool eval_preds(const PredSet &ps, int64_t row) {
  bool keep = true;
  for (int k = 0; k < ps.n; ++k) keep = keep && compare_op(load_as_i64(ps.col[k], ps.is64[k], row), ps.op[k], ps.val[k]);
  return keep;
}

// ------------------------------------------------------------------ XCD-aware block order
// Workgroups are dispatched round-robin over the chip's 8 XCDs (block b runs
// on XCD b mod 8), and every XCD has its own L2.  xcd_block maps the launch
// order to a work order in which each XCD takes one contiguous range of the
// n work items, in order: kernels whose consecutive items write neighbouring
// addresses (the pieces that consecutive tiles write into each destination)
// then have those writes meet in one L2, which merges them into whole lines.
// A bijection on [0, n) for any n.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t n) {
  const int64_t q = n / kXcds, r = n % kXcds, x = b % kXcds, i = b / kXcds;
  return x * q + (x < r ? x : r) + i;
}

// ------------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x) & (kWave - 1); }

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Inclusive prefix sum over the lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T u = __shfl_up(v, o);
    if (lane >= o) v += u;
  }
  return v;
}

// ------------------------------------------------------------------ decoupled look-back
// Ordered compaction across tiles in one pass: tile t publishes its aggregate,
// then walks back over its predecessors until it meets an inclusive prefix.
// Tiles take ids from an atomic ticket in dispatch order, so a tile only ever
// waits on tiles that are already running; the wait always ends.
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kValMask = (1ull << 62) - 1;

__device__ __forceinline__ void status_store(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t status_load(uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by all 64 lanes of ONE wave; returns the exclusive prefix of tile t.
__device__ inline int64_t lookback_exclusive(uint64_t *status, int64_t t, int64_t agg) {
  const int lane = lane_id();
  if (t == 0) {
    if (lane == 0) status_store(&status[0], kFlagInc | static_cast<uint64_t>(agg));
    return 0;
  }
  if (lane == 0) status_store(&status[t], kFlagAgg | static_cast<uint64_t>(agg));
  int64_t excl = 0;
  int64_t hi = t - 1;
  while (true) {
    const int64_t idx = hi - lane;
    const uint64_t s = idx >= 0 ? status_load(&status[idx]) : kFlagInc;
    const uint64_t inc = __ballot((s >> 62) == 2);
    const uint64_t bad = __ballot((s >> 62) == 0);
    const int first = inc ? __ffsll(static_cast<unsigned long long>(inc)) - 1 : kWave - 1;
    const uint64_t need = first >= kWave - 1 ? ~0ull : ((2ull << first) - 1ull);
    if (bad & need) {
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    int64_t v = lane <= first ? static_cast<int64_t>(s & kValMask) : 0;
    excl += wave_sum(v);
    if (inc) break;
    hi -= kWave;
  }
  if (lane == 0) status_store(&status[t], kFlagInc | static_cast<uint64_t>(excl + agg));
  return excl;
}

// ------------------------------------------------------------------ host side
struct Arena;

struct CtxImpl;  // defined in ctx.cpp

// Stream-ordered sub-allocation from the context arena (see ctx.cpp).
void *ctx_alloc(pyst_ctx *ctx, size_t bytes, hipStream_t stream);
// ctx_free keeps the block for `stream` (reused by it at once; other streams
// get it after an event that is recorded only when they need the memory), so
// `stream` must stay valid until pyst_ctx_check on it or the context's end.
// ctx_free_eager records that event at once (for streams the context does not
// outlive, and where other streams reuse memory all the time).
void ctx_free(pyst_ctx *ctx, void *p, hipStream_t stream);
void ctx_free_eager(pyst_ctx *ctx, void *p, hipStream_t stream);
// All work on `stream` has completed: what was freed on it goes to the free list.
void ctx_stream_idle(pyst_ctx *ctx, hipStream_t stream);
uint32_t *ctx_err_word(pyst_ctx *ctx);
// Make kernels launched through `ctx` latch errors into `word` (device memory)
// until reset with nullptr; used by the server to give each request its own word.
void ctx_set_err_word(pyst_ctx *ctx, uint32_t *word);
// Test hook (PYST_OPT_FAIL_FACT_PASS): true for the one fact pass it names.
bool ctx_fail_this_pass(pyst_ctx *ctx);
// The status a set of latched error bits stands for (PYST_OK for none).
pyst_status status_of_error_bits(uint32_t bits);
int ctx_device(const pyst_ctx *ctx);
int ctx_num_cus(const pyst_ctx *ctx);

pyst_status set_error(pyst_status st, const std::string &msg);
pyst_status hip_error(hipError_t e, const char *what);

// Records HIP events around a region on `stream` when the context's timing is on.
struct TimedRegion {
  pyst_ctx *ctx;
  hipStream_t stream;
  const char *label;
  hipEvent_t start = nullptr, stop = nullptr;
  TimedRegion(pyst_ctx *c, const char *name, hipStream_t s);
  ~TimedRegion();
};

// RAII scratch block that returns to the arena in stream order.
struct Scratch {
  pyst_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  void *p = nullptr;
  Scratch() = default;
  Scratch(pyst_ctx *c, size_t bytes, hipStream_t s) : ctx(c), stream(s), p(ctx_alloc(c, bytes, s)) {}
  Scratch(const Scratch &) = delete;
  Scratch &operator=(const Scratch &) = delete;
  ~Scratch() {
    if (p) ctx_free(ctx, p, stream);
  }
  template <typename T>
  T *as() const { return static_cast<T *>(p); }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Fill `n` 64-bit words with `v` on `stream` (a kernel, never a memset node,
// so the call stays safe inside captured graphs).
pyst_status fill_u64(void *p, int64_t n, uint64_t v, hipStream_t stream);
pyst_status fill_u32(void *p, int64_t n, uint32_t v, hipStream_t stream);

#define PYST_LAUNCH_CHECK(what)                                  \
  do {                                                           \
    hipError_t e_ = hipGetLastError();                           \
    if (e_ != hipSuccess) return ::pyst::hip_error(e_, what);    \
  } while (0)

}  // namespace pyst

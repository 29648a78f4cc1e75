// Hash-table layouts shared by the join, group-by and fused-query kernels.
//
// Join table: power-of-two capacity, linear probing from a 16-byte aligned
// start, so one vector load covers the first 4 (4-byte key slots) or 2
// (8-byte key|payload slots) candidates.  Inserts take the first EMPTY slot of
// the sequence by compare-and-swap, so the occupied slots of any probe
// sequence form a prefix and an EMPTY slot ends a probe.
//
// Group table: 16-byte slots {int64 key, uint64 sum}, key inserted by CAS and
// the sum accumulated with a 64-bit atomic add (wraps modulo 2^64).
//
// Capacity: the smallest power of two >= max(64, cnt / max_load, cnt + 1),
// clamped to the memory reserved for the upper bound.  The device evaluates it
// from the selected-row count it reads from memory, so no host sync is needed.
#pragma once

#include <cmath>

#include "pyst_internal.h"

namespace pyst {

struct TableDev {
  void *slots;     // int32 keys (slot_bytes 4) or uint64 key|payload<<32 (slot_bytes 8)
  int64_t *hdr;    // [0] effective capacity, [1] rows offered for insertion
  uint64_t *sums;  // optional per-slot SUM (group by the join key), else null
  uint8_t *flags;  // optional per-slot "group exists" flags
  uint32_t *bloom; // optional blocked Bloom filter over the inserted keys (fast path)
  int64_t cap_alloc;
  int32_t slot_bytes;
  int32_t reserved;
};

struct GroupDev {
  uint64_t *slots;  // 2 words per slot
  int64_t *hdr;     // [0] effective capacity
  int64_t cap_alloc;
};

__host__ __device__ inline int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

__host__ __device__ inline int64_t table_capacity(int64_t cnt, double max_load, int64_t cap_alloc) {
  int64_t need = static_cast<int64_t>(static_cast<double>(cnt) / max_load) + 1;
  if (need < cnt + 1) need = cnt + 1;
  if (need < 64) need = 64;
  int64_t cap = next_pow2(need);
  return cap > cap_alloc ? cap_alloc : cap;
}

inline int64_t table_capacity_host(int64_t n, double max_load) { return table_capacity(n, max_load, INT64_MAX); }

// Header of every table: int64 words (capacity, count, mode, ...) in the
// first 256 bytes; bytes [512, 1024) are one byte per bucket of slot sums.
constexpr size_t kHdrBytes = 1024;

inline size_t table_bytes(int64_t cap, int slot_bytes, bool with_sums) {
  size_t b = kHdrBytes + static_cast<size_t>(cap) * slot_bytes;
  if (with_sums) b += static_cast<size_t>(cap) * (sizeof(uint64_t) + 1);
  return b;
}

inline TableDev table_view(void *mem, int64_t cap, int slot_bytes, bool with_sums) {
  TableDev t{};
  char *p = static_cast<char *>(mem);
  t.hdr = reinterpret_cast<int64_t *>(p);
  t.slots = p + kHdrBytes;
  t.cap_alloc = cap;
  t.slot_bytes = slot_bytes;
  if (with_sums) {
    t.sums = reinterpret_cast<uint64_t *>(p + kHdrBytes + static_cast<size_t>(cap) * slot_bytes);
    t.flags = reinterpret_cast<uint8_t *>(t.sums + cap);
  }
  return t;
}

inline size_t group_bytes(int64_t cap) { return kHdrBytes + static_cast<size_t>(cap) * 16; }

inline GroupDev group_view(void *mem, int64_t cap) {
  GroupDev g{};
  g.hdr = static_cast<int64_t *>(mem);
  g.slots = reinterpret_cast<uint64_t *>(static_cast<char *>(mem) + kHdrBytes);
  g.cap_alloc = cap;
  return g;
}

// Add v to the group of key k (inserting the key if absent).  False: table full.
__device__ __forceinline__ bool group_add(uint64_t *slots, int64_t mask, int64_t k, uint64_t v) {
  int64_t s = static_cast<int64_t>(table_hash64(k)) & mask;
  for (int64_t step = 0; step <= mask; ++step) {
    uint64_t cur = slots[2 * s];
    if (static_cast<int64_t>(cur) == kEmpty64) {
      const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long *>(&slots[2 * s]),
                                     static_cast<unsigned long long>(kEmpty64), static_cast<unsigned long long>(k));
      cur = old == static_cast<uint64_t>(kEmpty64) ? static_cast<uint64_t>(k) : old;
    }
    if (static_cast<int64_t>(cur) == k) {
      atomicAdd(reinterpret_cast<unsigned long long *>(&slots[2 * s + 1]), static_cast<unsigned long long>(v));
      return true;
    }
    s = (s + 1) & mask;
  }
  return false;
}

// Host helpers implemented in ops.hip / sort.hip.
pyst_status table_init(const TableDev &t, const int64_t *d_nsel, int64_t n, double max_load, hipStream_t stream);
pyst_status group_init(const GroupDev &g, const int64_t *d_nsel, int64_t n, int64_t max_groups, double max_load,
                       hipStream_t stream);
pyst_status group_compact(pyst_ctx *ctx, const GroupDev &g, int64_t *out_keys, int64_t *out_sums, int64_t out_cap,
                          int64_t *d_ngroups, hipStream_t stream);
pyst_status filter_impl(pyst_ctx *ctx, const PredSet &ps, int64_t n, int32_t *sel_out, int64_t *d_nsel,
                        hipStream_t stream);
pyst_status scan_excl_i32(pyst_ctx *ctx, const int32_t *in, int32_t *out, int64_t len, int64_t *d_total,
                          hipStream_t stream);
pyst_status sort_pairs_by_key(pyst_ctx *ctx, int64_t *keys, int64_t *vals, const int64_t *d_count, int64_t cap,
                              hipStream_t stream);
int grid_for(pyst_ctx *ctx, int64_t work, int block, int per_cu);

}  // namespace pyst

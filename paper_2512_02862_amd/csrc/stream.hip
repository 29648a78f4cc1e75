// Streamed fused query: fact columns in pinned host memory are copied to the
// device chunk by chunk and consumed as they arrive.
//
// This is the chunking of Sec. 3.2 ("Partial Overlap Using Chunking"): the
// query runs on chunks instead of whole columns, so copies overlap compute and
// device memory holds only the dimension tables, the aggregation state and a
// ring of `nbuf` chunk buffers (Sec. 3.4, "Reduced GPU Memory Requirements").
// Copies run on the context's copy stream, the fact pass on the caller's
// stream; buffer reuse is ordered with events on the device, so the host only
// enqueues work and never waits -- no synchronizing step sits between chunks
// (the aim of Sec. 3.3, "Deferred Synchronization").
#include <algorithm>
#include <cstring>
#include <vector>

#include "pyst_internal.h"
#include "query.h"
#include "table.h"

namespace pyst {

// Defined with the packed columns.
pyst_status launch_unpack(pyst_ctx *ctx, const pyst_pack_block *blocks, const uint32_t *words, int64_t nwords,
                          int64_t word_base, int64_t n, int dtype, void *out, hipStream_t stream);

// host_fact gives every column's shape; with `packed`, each chunk of column c is
// copied as its packed blocks (packed[c]) and decoded on the device, otherwise
// copied as is from host_fact[c].data.
pyst_status streamed_query(pyst_ctx *ctx, const pyst_plan *plan, const pyst_col *host_fact, int nfact,
                           const pyst_packed_col *packed, int64_t chunk_rows, int nbuf, int64_t *out_keys,
                           int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups, hipStream_t stream) {
  QueryShape q;
  pyst_status st = prepare_query(plan, host_fact, nfact, &q);
  if (st != PYST_OK) return st;
  if (q.agg_mode == 2) return set_error(PYST_ERR_UNSUPPORTED, "pyst_query_streamed: set plan->max_groups for non-slot aggregation");
  const int64_t n = host_fact[0].n;
  // Kernel arguments are rebuilt per chunk against the device ring; check the shape once.
  FastArgs fa;
  if (!fast_shape(plan, host_fact, q, &fa)) return set_error(PYST_ERR_UNSUPPORTED, "pyst_query_streamed: plan shape has no streamed kernel");
  hipStream_t cs = ctx_copy_stream(ctx);
  if (!cs) return set_error(PYST_ERR_HIP, "pyst_query_streamed: cannot create the copy stream");

  const int64_t nchunks = ceil_div(n, chunk_rows);
  // Per column and ring slot: the decoded chunk, and with packed input its block
  // headers and the most words any chunk of the column has.
  auto round = [](size_t x) { return (x + 255) / 256 * 256; };
  std::vector<size_t> col_bytes(nfact), hdr_bytes(nfact, 0), word_bytes(nfact, 0);
  for (int c = 0; c < nfact; ++c) {
    col_bytes[c] = round(static_cast<size_t>(chunk_rows) * (host_fact[c].dtype == PYST_I64 ? 8 : 4));
    if (!packed) continue;
    hdr_bytes[c] = round(static_cast<size_t>(chunk_rows / PYST_PACK_BLOCK + 1) * sizeof(pyst_pack_block));
    int64_t most = 0;
    for (int64_t ch = 0; ch < nchunks; ++ch) {
      const int64_t b0 = ch * chunk_rows / PYST_PACK_BLOCK;
      const int64_t b1 = ceil_div(std::min<int64_t>(n, (ch + 1) * chunk_rows), PYST_PACK_BLOCK);
      most = std::max(most, packed[c].blocks[b1].word_off - packed[c].blocks[b0].word_off);
    }
    word_bytes[c] = round(static_cast<size_t>(most) * sizeof(uint32_t));
  }
  size_t slot_bytes = 0;
  for (int c = 0; c < nfact; ++c) slot_bytes += col_bytes[c] + hdr_bytes[c] + word_bytes[c];
  void *ring = ctx_alloc(ctx, static_cast<size_t>(nbuf) * slot_bytes, stream);
  if (!ring) return set_error(PYST_ERR_NOMEM, "pyst_query_streamed: arena cannot hold the chunk ring");
  std::vector<std::vector<char *>> buf(nbuf, std::vector<char *>(nfact)), hdr = buf, wbuf = buf;
  char *p = static_cast<char *>(ring);
  for (int b = 0; b < nbuf; ++b)
    for (int c = 0; c < nfact; ++c) {
      buf[b][c] = p;
      hdr[b][c] = p + col_bytes[c];
      wbuf[b][c] = p + col_bytes[c] + hdr_bytes[c];
      p += col_bytes[c] + hdr_bytes[c] + word_bytes[c];
    }
  std::vector<hipEvent_t> copied(nbuf, nullptr), consumed(nbuf, nullptr);
  for (int b = 0; b < nbuf && st == PYST_OK; ++b) {
    if (hipEventCreateWithFlags(&copied[b], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&consumed[b], hipEventDisableTiming) != hipSuccess)
      st = set_error(PYST_ERR_HIP, "pyst_query_streamed: hipEventCreate");
  }

  DimTables d;
  std::memset(&d, 0, sizeof(d));
  AggState s;
  std::memset(&s, 0, sizeof(s));
  if (st == PYST_OK && q.agg_mode == 1) {
    const int64_t bound = std::min<int64_t>(plan->max_groups, std::max<int64_t>(n, 1));
    const int64_t cap = table_capacity_host(bound, plan->group_max_load);
    s.mem = ctx_alloc(ctx, group_bytes(cap), stream);
    if (!s.mem) st = set_error(PYST_ERR_NOMEM, "pyst_query_streamed: arena exhausted (group table)");
    else {
      s.g = group_view(s.mem, cap);
      st = group_init(s.g, nullptr, bound, 0, plan->group_max_load, stream);
    }
  }
  if (st == PYST_OK) st = fast_build_dimensions(ctx, plan, q, &d, d_ngroups, nullptr, stream, false, nullptr);
  // The copy stream must not overwrite ring memory before `stream` has reached this point.
  hipEvent_t start = nullptr;
  if (st == PYST_OK) {
    if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess || hipEventRecord(start, stream) != hipSuccess ||
        hipStreamWaitEvent(cs, start, 0) != hipSuccess)
      st = set_error(PYST_ERR_HIP, "pyst_query_streamed: ordering the copy stream");
  }
  std::vector<pyst_col> dev_fact(host_fact, host_fact + nfact);
  for (int64_t ch = 0; ch < nchunks && st == PYST_OK; ++ch) {
    const int b = static_cast<int>(ch % nbuf);
    const int64_t off = ch * chunk_rows;
    const int64_t rows = std::min<int64_t>(chunk_rows, n - off);
    if (ch >= nbuf && hipStreamWaitEvent(cs, consumed[b], 0) != hipSuccess) {
      st = set_error(PYST_ERR_HIP, "pyst_query_streamed: hipStreamWaitEvent");
      break;
    }
    {
      TimedRegion timed(ctx, "h2d_chunk", cs);
      for (int c = 0; c < nfact && st == PYST_OK; ++c) {
        dev_fact[c].data = buf[b][c];
        dev_fact[c].n = rows;
        hipError_t e = hipSuccess;
        if (!packed) {
          const size_t w = host_fact[c].dtype == PYST_I64 ? 8 : 4;
          e = hipMemcpyAsync(buf[b][c], static_cast<const char *>(host_fact[c].data) + off * w,
                             static_cast<size_t>(rows) * w, hipMemcpyHostToDevice, cs);
        } else {
          const int64_t b0 = off / PYST_PACK_BLOCK, b1 = ceil_div(off + rows, PYST_PACK_BLOCK);
          const int64_t w0 = packed[c].blocks[b0].word_off, w1 = packed[c].blocks[b1].word_off;
          e = hipMemcpyAsync(hdr[b][c], packed[c].blocks + b0, static_cast<size_t>(b1 - b0 + 1) * sizeof(pyst_pack_block),
                             hipMemcpyHostToDevice, cs);
          if (e == hipSuccess && w1 > w0)
            e = hipMemcpyAsync(wbuf[b][c], packed[c].words + w0, static_cast<size_t>(w1 - w0) * sizeof(uint32_t),
                               hipMemcpyHostToDevice, cs);
        }
        if (e != hipSuccess) st = hip_error(e, "pyst_query_streamed: hipMemcpyAsync");
      }
    }
    if (st != PYST_OK) break;
    if (hipEventRecord(copied[b], cs) != hipSuccess || hipStreamWaitEvent(stream, copied[b], 0) != hipSuccess) {
      st = set_error(PYST_ERR_HIP, "pyst_query_streamed: chunk event");
      break;
    }
    // Packed chunks are decoded on `stream`, into the slot the fact pass reads, so
    // the copy stream goes on with the next chunk meanwhile; the slot's packed
    // buffers are reused only after `consumed`, recorded after the fact pass.
    for (int c = 0; packed && c < nfact && st == PYST_OK; ++c) {
      const int64_t b0 = off / PYST_PACK_BLOCK, b1 = ceil_div(off + rows, PYST_PACK_BLOCK);
      const int64_t w0 = packed[c].blocks[b0].word_off, w1 = packed[c].blocks[b1].word_off;
      st = launch_unpack(ctx, reinterpret_cast<const pyst_pack_block *>(hdr[b][c]),
                         reinterpret_cast<const uint32_t *>(wbuf[b][c]), w1 - w0, w0, rows, host_fact[c].dtype,
                         buf[b][c], stream);
    }
    if (st != PYST_OK) break;
    FastArgs ca;
    fast_shape(plan, dev_fact.data(), q, &ca);
    st = fast_fact_pass(ctx, plan->njoins, q.agg_mode, ca, d, s.g, s.po, stream);
    if (st == PYST_OK && hipEventRecord(consumed[b], stream) != hipSuccess)
      st = set_error(PYST_ERR_HIP, "pyst_query_streamed: hipEventRecord");
  }
  if (st == PYST_OK) st = fast_finish(ctx, plan, q, d, &s, out_keys, out_sums, out_cap, d_ngroups, stream);
  // Frees are stream ordered on `stream`, which has waited for every copy.
  ctx_free(ctx, s.mem, stream);
  free_dimensions(ctx, &d, stream);
  ctx_free(ctx, ring, stream);
  // Events may be destroyed while pending: HIP releases them after completion.
  for (int b = 0; b < nbuf; ++b) {
    if (copied[b]) (void)hipEventDestroy(copied[b]);
    if (consumed[b]) (void)hipEventDestroy(consumed[b]);
  }
  if (start) (void)hipEventDestroy(start);
  return st;
}

}  // namespace pyst

using namespace pyst;

extern "C" pyst_status pyst_query_streamed(pyst_ctx *ctx, const pyst_plan *plan, const pyst_col *host_fact, int nfact,
                                           int64_t chunk_rows, int nbuf, int64_t *out_keys, int64_t *out_sums,
                                           int64_t out_cap, int64_t *d_ngroups, hipStream_t stream) {
  if (!ctx || !plan || !host_fact || !d_ngroups) return set_error(PYST_ERR_ARG, "pyst_query_streamed: NULL argument");
  if (chunk_rows < 4 || chunk_rows % 4 != 0 || chunk_rows >= (int64_t{1} << 31))
    return set_error(PYST_ERR_ARG, "pyst_query_streamed: chunk_rows must be a positive multiple of 4 below 2^31");
  if (nbuf < 2 || nbuf > 8) return set_error(PYST_ERR_ARG, "pyst_query_streamed: nbuf in 2..8");
  if (out_cap < 0 || (out_cap > 0 && (!out_keys || !out_sums))) return set_error(PYST_ERR_ARG, "pyst_query_streamed: bad outputs");
  return streamed_query(ctx, plan, host_fact, nfact, nullptr, chunk_rows, nbuf, out_keys, out_sums, out_cap, d_ngroups,
                        stream);
}

// Only the shape of these columns is checked (dtype, length, a non-null 16-byte
// aligned address); no byte of them is read.
alignas(16) static const char kShapeOnly[16] = {};

extern "C" pyst_status pyst_query_streamed_packed(pyst_ctx *ctx, const pyst_plan *plan,
                                                  const pyst_packed_col *host_fact, int nfact, int64_t chunk_rows,
                                                  int nbuf, int64_t *out_keys, int64_t *out_sums, int64_t out_cap,
                                                  int64_t *d_ngroups, hipStream_t stream) {
  if (!ctx || !plan || !host_fact || !d_ngroups) return set_error(PYST_ERR_ARG, "pyst_query_streamed_packed: NULL argument");
  if (chunk_rows < PYST_PACK_BLOCK || chunk_rows % PYST_PACK_BLOCK != 0 || chunk_rows >= (int64_t{1} << 31))
    return set_error(PYST_ERR_ARG, "pyst_query_streamed_packed: chunk_rows must be a positive multiple of 1024 below 2^31");
  if (nbuf < 2 || nbuf > 8) return set_error(PYST_ERR_ARG, "pyst_query_streamed_packed: nbuf in 2..8");
  if (nfact < 1 || nfact > PYST_MAX_COLS) return set_error(PYST_ERR_ARG, "pyst_query_streamed_packed: 1..8 fact columns");
  if (out_cap < 0 || (out_cap > 0 && (!out_keys || !out_sums)))
    return set_error(PYST_ERR_ARG, "pyst_query_streamed_packed: bad outputs");
  std::vector<pyst_col> shape(nfact);
  for (int c = 0; c < nfact; ++c) {
    const pyst_packed_col &pc = host_fact[c];
    if (!(pc.dtype == PYST_I32 || pc.dtype == PYST_I64) || pc.n < 0 || pc.n != host_fact[0].n || !pc.blocks ||
        (pc.n > 0 && !pc.words))
      return set_error(PYST_ERR_ARG, "pyst_query_streamed_packed: bad packed column");
    if (!pack_blocks_ok(pc.blocks, ceil_div(pc.n, PYST_PACK_BLOCK), pc.dtype))
      return set_error(PYST_ERR_ARG, "pyst_query_streamed_packed: malformed block table");
    shape[c] = pyst_col{kShapeOnly, pc.n, pc.dtype, 0};
  }
  return streamed_query(ctx, plan, shape.data(), nfact, host_fact, chunk_rows, nbuf, out_keys, out_sums, out_cap,
                        d_ngroups, stream);
}

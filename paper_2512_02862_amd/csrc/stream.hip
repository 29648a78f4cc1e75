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

pyst_status streamed_query(pyst_ctx *ctx, const pyst_plan *plan, const pyst_col *host_fact, int nfact,
                           int64_t chunk_rows, int nbuf, int64_t *out_keys, int64_t *out_sums, int64_t out_cap,
                           int64_t *d_ngroups, hipStream_t stream) {
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

  size_t row_bytes = 0;
  for (int c = 0; c < nfact; ++c) row_bytes += host_fact[c].dtype == PYST_I64 ? 8 : 4;
  const size_t ring_bytes = static_cast<size_t>(nbuf) * static_cast<size_t>(chunk_rows) * row_bytes + 256 * nfact * nbuf;
  void *ring = ctx_alloc(ctx, ring_bytes, stream);
  if (!ring) return set_error(PYST_ERR_NOMEM, "pyst_query_streamed: arena cannot hold the chunk ring");
  std::vector<std::vector<char *>> buf(nbuf, std::vector<char *>(nfact));
  char *p = static_cast<char *>(ring);
  for (int b = 0; b < nbuf; ++b)
    for (int c = 0; c < nfact; ++c) {
      buf[b][c] = p;
      p += (static_cast<size_t>(chunk_rows) * (host_fact[c].dtype == PYST_I64 ? 8 : 4) + 255) / 256 * 256;
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
  if (st == PYST_OK) st = fast_build_dimensions(ctx, plan, q, &d, d_ngroups, nullptr, stream);
  // The copy stream must not overwrite ring memory before `stream` has reached this point.
  hipEvent_t start = nullptr;
  if (st == PYST_OK) {
    if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess || hipEventRecord(start, stream) != hipSuccess ||
        hipStreamWaitEvent(cs, start, 0) != hipSuccess)
      st = set_error(PYST_ERR_HIP, "pyst_query_streamed: ordering the copy stream");
  }
  const int64_t nchunks = ceil_div(n, chunk_rows);
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
        const size_t w = host_fact[c].dtype == PYST_I64 ? 8 : 4;
        const hipError_t e = hipMemcpyAsync(buf[b][c], static_cast<const char *>(host_fact[c].data) + off * w,
                                            static_cast<size_t>(rows) * w, hipMemcpyHostToDevice, cs);
        if (e != hipSuccess) st = hip_error(e, "pyst_query_streamed: hipMemcpyAsync");
        dev_fact[c].data = buf[b][c];
        dev_fact[c].n = rows;
      }
    }
    if (st != PYST_OK) break;
    if (hipEventRecord(copied[b], cs) != hipSuccess || hipStreamWaitEvent(stream, copied[b], 0) != hipSuccess) {
      st = set_error(PYST_ERR_HIP, "pyst_query_streamed: chunk event");
      break;
    }
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
  return streamed_query(ctx, plan, host_fact, nfact, chunk_rows, nbuf, out_keys, out_sums, out_cap, d_ngroups, stream);
}

// Host/device descriptors of a fused query, shared by the plain, streamed,
// batched and served executors.
#pragma once

#include "pyst_internal.h"
#include "table.h"

namespace pyst {

constexpr int kMaxFactCols = 6;

// The distinct fact columns a plan reads ("slots") and what the fact pass
// does with them.
struct FactArgs {
  const void *col[kMaxFactCols];
  int32_t is64[kMaxFactCols];
  int32_t ncol;
  int32_t npred;
  int32_t pslot[PYST_MAX_PREDS];
  int32_t pop[PYST_MAX_PREDS];
  int64_t pval[PYST_MAX_PREDS];
  int32_t fk_slot[2];
  int32_t hi_src, hi_idx, lo_src, lo_idx;
  int32_t vexpr, v0_slot, v1_slot;
  int64_t vconst;
  int64_t n;
};

struct PairsOut {
  int64_t *count;
  int64_t *keys;
  int64_t *vals;
  int64_t cap;
};

struct QueryShape {
  FactArgs fact;
  bool need_payload[2];
  bool slot_agg;   // group key is the key of the single join: sums live in its slots
  int agg_mode;    // 0 slot sums, 1 group table sized by max_groups, 2 pairs + group-by
};

struct DimTables {
  TableDev t[2];
  void *mem[2];
  void *sel_mem[2];
};

struct AggState {
  void *mem;
  GroupDev g;
  PairsOut po;
};

// Kernel arguments of the specialized fact pass (int32 keys and predicate
// columns, group key from join keys / the payload of join 1).
struct FastArgs {
  const int32_t *fk[2];
  const void *v0;
  const int32_t *v1;
  int32_t v0_64;
  int32_t vexpr;
  int64_t vconst;
  // Up to two predicates on int32 fact columns, each as "x in [plo, plo + pspan]"
  // (32-bit wrap-around arithmetic) XOR pneg; an unused one has a null column
  // and the full range.
  const int32_t *pcol[2];
  int32_t plo[2];
  uint32_t pspan[2];
  int32_t pneg[2];
  int32_t hi_src, hi_idx, lo_src, lo_idx;
  int64_t n;
};

pyst_status prepare_query(const pyst_plan *plan, const pyst_col *fact, int nfact, QueryShape *q);
bool fast_shape(const pyst_plan *plan, const pyst_col *fact, const QueryShape &q, FastArgs *fa);
pyst_status fast_query(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, const FastArgs &fa,
                       int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                       hipStream_t stream);
pyst_status fast_build_dimensions(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, DimTables *d,
                                  int64_t *zero0, int64_t *zero1, hipStream_t stream, bool allow_direct,
                                  uint32_t *pool_next);
pyst_status fast_fact_pass(pyst_ctx *ctx, int njoins, int agg_mode, const FastArgs &a, const DimTables &d,
                           const GroupDev &g, const PairsOut &po, hipStream_t stream);
pyst_status fast_finish(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, const DimTables &d, AggState *s,
                        int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                        hipStream_t stream);
pyst_status pair_groupby(pyst_ctx *ctx, int64_t *keys, int64_t *vals, const int64_t *count, int64_t cap,
                         int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                         hipStream_t stream);
bool ctx_generic_only(const pyst_ctx *ctx);
bool ctx_hash_join_only(const pyst_ctx *ctx);
int fast_grid(pyst_ctx *ctx, int64_t n);
hipStream_t ctx_copy_stream(pyst_ctx *ctx);
char *ctx_pinned_staging(pyst_ctx *ctx, size_t bytes);
size_t ctx_budget_free(const pyst_ctx *ctx);
hipError_t ctx_staging_record(pyst_ctx *ctx, hipStream_t stream);
pyst_status build_dimensions(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, DimTables *d,
                             hipStream_t stream);
void free_dimensions(pyst_ctx *ctx, DimTables *d, hipStream_t stream);
pyst_status fact_pass(pyst_ctx *ctx, const QueryShape &q, int njoins, const FactArgs &a, const DimTables &d,
                      const GroupDev &g, const PairsOut &po, int grid, hipStream_t stream);
pyst_status agg_alloc(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, int64_t rows_bound, AggState *s,
                      hipStream_t stream);
pyst_status agg_finish(pyst_ctx *ctx, const pyst_plan *plan, const QueryShape &q, const DimTables &d, AggState *s,
                       int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                       hipStream_t stream);

}  // namespace pyst

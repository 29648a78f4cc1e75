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

pyst_status prepare_query(const pyst_plan *plan, const pyst_col *fact, int nfact, QueryShape *q);
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

/*
 * pyst -- per-GPU relational hot path of a tensor-runtime OLAP engine, for
 * AMD Instinct MI355X (gfx950).
 *
 * The operators are those of the distributed hash join and the queries built
 * on it in PystachIO (arXiv 2512.02862): a pushed-down filter (Sec. 4,
 * introduction), the hash partition that splits a table by join key into
 * per-destination buffers, i.e. the send side of the shuffle (Sec. 3.1,
 * "Anatomy of a Distributed Hash Join"), the hash-table build and probe
 * (same paragraph; Sec. 3.2 builds the table once over the fully
 * materialized build side), and the group-by SUM aggregation (Sec. 6.3,
 * observation (5)).  Chunked streaming follows Sec. 3.2 ("Partial Overlap
 * Using Chunking") and the queue-based, memory-regulated scheduling of
 * Sec. 5.4 ("Queue-Based Scheduling", "Adaptive Regulation").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Column data pointers are DEVICE pointers unless a parameter says "host".
 *   They are borrowed: the caller owns them and keeps them alive until the
 *   work enqueued on `stream` has completed.
 * - Every call only ENQUEUES work on `stream` and returns without waiting for
 *   the device, except those documented as blocking (pyst_ctx_check,
 *   pyst_ctx_destroy, pyst_table_destroy, the server calls).  Data-dependent
 *   sizes (selected rows, join matches, groups, partition offsets) are written
 *   to device memory and consumed from there by later calls: no host-side
 *   sizing, which is what forces stream synchronizations in a tensor runtime
 *   (Sec. 3.2, "Stream-Synchronizing Operations Limit Overlap").
 * - A selection is the pair (sel, d_nsel): an ascending int32 row-id vector and
 *   a device int64 count.  Passing NULL, NULL means "all rows".
 * - Row ids are int32, so a column passed to one call has fewer than 2^31 rows.
 * - Argument errors are returned synchronously.  Errors found by a kernel
 *   (an EMPTY-sentinel key, a full table, an output over capacity, a duplicate
 *   key under a unique-key promise) are latched in the context and returned by
 *   the next pyst_ctx_check.
 * - Integer sums wrap modulo 2^64 (two's complement), so results do not depend
 *   on the order in which the device adds them.
 * - A context is not thread-safe; use one per host thread.  Its arena
 *   allocations are stream ordered: memory freed by work on one stream is
 *   reused by another stream only after that work has completed.  The context
 *   marks that point with an event on the freeing stream only when another
 *   stream needs the memory, so a stream used with a context must stay valid
 *   until pyst_ctx_check(ctx, that stream) returns or the context is destroyed.
 */
#ifndef PYST_H
#define PYST_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pyst_status {
  PYST_OK = 0,
  PYST_ERR_ARG = 1,         /* invalid argument (returned synchronously)              */
  PYST_ERR_NOMEM = 2,       /* the context's device-memory budget cannot hold the call */
  PYST_ERR_HIP = 3,         /* a HIP runtime call failed                              */
  PYST_ERR_CAPACITY = 4,    /* output capacity exceeded; the count holds the need     */
  PYST_ERR_KEY = 5,         /* a key equal to the EMPTY sentinel was seen              */
  PYST_ERR_TABLE_FULL = 6,  /* a hash table had no free slot                          */
  PYST_ERR_UNSUPPORTED = 7, /* a valid but unsupported combination                    */
  PYST_ERR_DUP_KEY = 8,     /* duplicate build key although unique_keys was promised  */
  PYST_ERR_INDEX = 9        /* a gather index outside [0, rows of its columns)        */
} pyst_status;

typedef enum pyst_dtype { PYST_I32 = 0, PYST_I64 = 1 } pyst_dtype;

/* One column: `n` values of `dtype` at device address `data` (contiguous). */
typedef struct pyst_col {
  const void *data;
  int64_t n;
  int32_t dtype; /* pyst_dtype */
  int32_t reserved;
} pyst_col;

typedef enum pyst_cmp { PYST_EQ = 0, PYST_NE = 1, PYST_LT = 2, PYST_LE = 3, PYST_GT = 4, PYST_GE = 5 } pyst_cmp;

/* One predicate term `cols[col] <cmp> value`; the value is compared as int64
   after sign extension.  A predicate list is the AND of its terms. */
typedef struct pyst_pred {
  int32_t col;
  int32_t cmp; /* pyst_cmp */
  int64_t value;
} pyst_pred;

#define PYST_MAX_COLS 8
#define PYST_MAX_PART_PAYLOADS 15 /* payload columns one pyst_partition call carries */
#define PYST_MAX_PREDS 8
#define PYST_MAX_FANOUT 1024

typedef struct pyst_ctx pyst_ctx;
typedef struct pyst_table pyst_table;

/* ---------------------------------------------------------------- context */

/* Create a context on `device` with a device arena of `budget_bytes`
   (allocated once; every internal table and scratch buffer comes from it, the
   analog of the pooled allocator of Sec. 3.1 "(2) Runtime Memory Allocation").
   On success *out owns the arena.  Errors: PYST_ERR_ARG (bad device, NULL
   out), PYST_ERR_NOMEM (the arena cannot be allocated), PYST_ERR_HIP. */
pyst_status pyst_ctx_create(int device, size_t budget_bytes, pyst_ctx **out);

/* Wait for all device work, then free the arena and the context.  NULL is a no-op. */
void pyst_ctx_destroy(pyst_ctx *ctx);

/* Synchronize `stream`, then return and clear the errors latched by kernels
   (PYST_OK if none).  This is the only place device-detected errors surface. */
pyst_status pyst_ctx_check(pyst_ctx *ctx, hipStream_t stream);

/* Bytes of the arena currently allocated, and its total size. */
size_t pyst_ctx_used(const pyst_ctx *ctx);
size_t pyst_ctx_budget(const pyst_ctx *ctx);

/* Message describing the last error returned on the calling thread. */
const char *pyst_last_error(void);

/* The device's memory clock (kHz) and bus width (bits) as its properties
   report them, and the HBM peak they imply (GB/s) at HBM3 / HBM3E's 4
   transfers a pin per reported clock: the properties-derived peak recorded
   beside the published one as the roofline of the measurements on this
   hardware (Sec. 6 reports its numbers against the A100's own peaks).
   Errors: PYST_ERR_ARG (a NULL output), PYST_ERR_HIP (a bad device). */
pyst_status pyst_device_hbm(int device, int64_t *mem_clock_khz, int32_t *bus_bits, double *peak_gbs);

/* Kernel timing for measurement.  When enabled, the library records a pair of
   HIP events on the launch stream around its timed regions: "fact_pass" (the
   fused probe + aggregation kernel of pyst_query), "partition" (the whole of
   pyst_partition) and "part_scatter" (its scatter kernel).
   pyst_ctx_kernel_time waits for the recorded events of region `name`, returns
   their summed duration in milliseconds and the number of launches, and
   forgets them.  Errors: PYST_ERR_ARG, PYST_ERR_HIP. */
pyst_status pyst_ctx_timing(pyst_ctx *ctx, int enable);

/* Context options.  PYST_OPT_GENERIC_ONLY != 0 makes pyst_query use its
   generic fact pass even where a plan-shape-specialized kernel exists.
   PYST_OPT_GROUPBY_HASH_ONLY != 0 makes pyst_groupby_sum always use its HBM
   hash table instead of the radix-partitioned path.  Both paths compute the
   same result; tests compare them.  Errors: PYST_ERR_ARG. */
#define PYST_OPT_GENERIC_ONLY 1
#define PYST_OPT_GROUPBY_HASH_ONLY 2
/* Test hook for failure handling: value n > 0 makes the n-th fused fact pass
   issued through the context from now on fail on the host with PYST_ERR_HIP
   before it launches anything (0 clears it).  No device fault is involved. */
#define PYST_OPT_FAIL_FACT_PASS 3
/* PYST_OPT_HASH_JOIN_ONLY != 0 keeps pyst_query's join tables hash tables:
   without it, a one-join query grouped by the join key direct-addresses its
   dimension table (key k in slot k - min key) when the selected dimension
   keys span at most 2^21 values and no more than the table's reserved slots,
   and a two-join query whose pairs are grouped (the chain of Sec. 6.1)
   direct-addresses its first join when the selected keys span at most 2^20
   values and its second (key + payload) join when its keys span no more than
   that table's reserved slots.  The choice is made on the device from the
   selected keys' least and greatest value.  Both compute the same result;
   tests compare them.  Duplicate dimension keys are reported
   (PYST_ERR_DUP_KEY) in either mode. */
#define PYST_OPT_HASH_JOIN_ONLY 4
pyst_status pyst_ctx_option(pyst_ctx *ctx, int key, int64_t value);
pyst_status pyst_ctx_kernel_time(pyst_ctx *ctx, const char *name, double *total_ms, int64_t *launches);

/* ---------------------------------------------------------------- filter */

/* Filter pushdown (Sec. 4, introduction): select the rows i < n of
   cols[0..ncols) (all of n rows) for which every predicate holds.
   sel_out: device int32[n], receives the ascending row ids.
   d_nsel: device int64, receives the number selected.
   Errors: PYST_ERR_ARG (column counts or lengths disagree, ncols or np over
   the maxima, a predicate names a missing column). */
pyst_status pyst_filter(pyst_ctx *ctx, const pyst_col *cols, int ncols, const pyst_pred *preds,
                        int npreds, int32_t *sel_out, int64_t *d_nsel, hipStream_t stream);

/* ---------------------------------------------------------------- partition */

/* Hash partition, the send side of the shuffle (Sec. 3.1, "Anatomy of a
   Distributed Hash Join": the local table is partitioned by join key before
   it is shuffled).  Destination of a row: h(key) mod fanout, with
   h = MurmurHash3 fmix32(uint32 key) for int32 keys and the low 32 bits of
   fmix64(uint64 key) for int64 keys.
   Rows (all n, or the selection) are written STABLY into `fanout` contiguous
   segments: out_cols[0] receives the key column, out_cols[1 + j] payload j;
   each output has room for key->n values of its column's dtype.
   d_offsets: device int64[fanout + 1]; segment p is [d_offsets[p], d_offsets[p+1]).
   Errors: PYST_ERR_ARG (fanout outside 1..PYST_MAX_FANOUT, npay over
   PYST_MAX_PART_PAYLOADS, lengths disagree), PYST_ERR_NOMEM. */
pyst_status pyst_partition(pyst_ctx *ctx, const pyst_col *key, const pyst_col *payloads, int npay,
                           const int32_t *sel, const int64_t *d_nsel, uint32_t fanout,
                           void *const *out_cols, int64_t *d_offsets, hipStream_t stream);

/* For callers that cannot allocate device memory -- code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc: the same
   partition as pyst_partition (same arguments and results, no context), which
   allocates nothing.  Its scratch (per-tile destination counts, their scan and
   the scan's look-back words: 8 * ceil(n / 4096) * fanout bytes plus 1/2048
   of that) lives in a fixed device array of PYST_NOALLOC_SCRATCH_BYTES
   that every GPU the library runs on holds until the process ends; the
   current device's copy is used.  A call whose scratch would exceed it
   returns PYST_ERR_CAPACITY before any work is enqueued (e.g. fanout 64 up to
   about 260M rows, fanout 1024 up to about 16M rows).  Every call on one GPU
   shares that GPU's array and leaves its contents behind (the kernels clear
   what must start at zero), so calls that overlap on one GPU -- on different
   streams or from different threads -- race and must be ordered by the
   caller.  Errors: as pyst_partition, PYST_ERR_CAPACITY, PYST_ERR_HIP. */
#define PYST_NOALLOC_SCRATCH_BYTES (32u << 20)
pyst_status pyst_partition_noalloc(const pyst_col *key, const pyst_col *payloads, int npay, const int32_t *sel,
                                   const int64_t *d_nsel, uint32_t fanout, void *const *out_cols,
                                   int64_t *d_offsets, hipStream_t stream);

/* ---------------------------------------------------------------- join */

/* Hash-join build (Sec. 3.1 "Anatomy..."; the table is built over the fully
   materialized build side, Sec. 3.2 "Scheduling Overlap With GPU Streams").
   Inserts the selected rows of the int32 or int64 `key` column into a
   power-of-two open-addressing table with linear probing and atomic
   compare-and-swap.  payload: int32 or int64 column of the key's length
   stored with each key, or NULL to store the row id.  Layout: int32 keys with
   int32 (or no) payloads take 8-byte slots; int64 keys or int64 payloads take
   16-byte slots {int64 key, int64 payload}.
   max_load in (0, 0.95]: the capacity is the smallest power of two with
   load <= max_load for the number of rows actually selected (read on the
   device, so no host synchronization is needed; memory is reserved for the
   unfiltered n).  unique_keys != 0 promises distinct keys: probes stop at
   the first match, and a duplicate latches PYST_ERR_DUP_KEY.
   The key INT32_MIN (int32 key column) or INT64_MIN (int64 key column) is
   reserved as EMPTY and latches PYST_ERR_KEY.
   *out receives a table owned by the caller (pyst_table_destroy).
   Errors: PYST_ERR_ARG, PYST_ERR_NOMEM. */
pyst_status pyst_join_build(pyst_ctx *ctx, const pyst_col *key, const pyst_col *payload,
                            const int32_t *sel, const int64_t *d_nsel, double max_load,
                            int unique_keys, pyst_table **out, hipStream_t stream);

/* Hash-join probe: for every selected row of the int32 or int64 `key` column,
   in ascending row order, emit one (probe row, stored payload) pair per
   matching build row.  Keys compare by value whatever the two columns' types;
   a probe key equal to its own column's EMPTY sentinel matches nothing.
   out_probe_row: device int32[out_cap]; out_payload: device int64[out_cap]
   (int32 payloads sign-extended, row ids as they are).
   d_nout: device int64, receives the number of matches; when it exceeds
   out_cap only the first out_cap pairs are written and PYST_ERR_CAPACITY is
   latched.  With duplicate build keys the matches of one probe row come in
   table order.  Errors: PYST_ERR_ARG. */
pyst_status pyst_join_probe(pyst_ctx *ctx, const pyst_table *table, const pyst_col *key,
                            const int32_t *sel, const int64_t *d_nsel, int32_t *out_probe_row,
                            int64_t *out_payload, int64_t out_cap, int64_t *d_nout,
                            hipStream_t stream);

/* Materialize join results (Sec. 3.1 "Anatomy...": the probe emits matching
   tuples; the microbenchmarks of Sec. 3 carry 1..8 8-byte columns per tuple).
   For every i < min(*d_n, cap): out_cols[c][i] = cols[c].data[idx[i]], for
   c < ncols.  idx: device int32[cap], e.g. the probe rows or the stored row
   ids that pyst_join_probe emits.  d_n: device int64 count of valid entries
   of idx, or NULL for all cap entries.  cols: 1..8 int32 or int64 columns of
   one common length; out_cols[c]: device buffers of cols[c]'s dtype with room
   for cap values, owned by the caller.  An index outside [0, cols[0].n)
   latches PYST_ERR_INDEX and leaves its output row unwritten.
   Errors: PYST_ERR_ARG (NULL pointers, 0 or more than 8 columns, length
   mismatch, cap outside [0, 2^31)). */
pyst_status pyst_gather(pyst_ctx *ctx, const int32_t *idx, const int64_t *d_n, int64_t cap, const pyst_col *cols,
                        int ncols, void *const *out_cols, hipStream_t stream);

/* One-call materializing equi-join, the receive-side work of one GPU in the
   join microbenchmark of Sec. 3 (build + probe + materialize; the send side is
   pyst_partition): builds a table over build_key (int32 or int64; keys
   compare by value as in pyst_join_probe), probes it with
   every row of probe_key, and for each match, in ascending probe row, writes
   the probe row, the build row and the tuple npcols probe columns then nbcols
   build columns (each 0..8, int32 or int64, of their key's length):
   out_cols[c] for c < npcols holds probe_cols[c] at the probe row,
   out_cols[npcols + c] build_cols[c] at the build row.
   unique_keys != 0 promises distinct build keys (a duplicate latches
   PYST_ERR_DUP_KEY) and lets a probe stop at its first match; with
   unique_keys == 0 duplicate build keys are joined with SQL semantics (a
   many-to-many join): a probe row emits one tuple per matching build row, the
   tuples of one probe row consecutive in table order (so the canonical order
   of the result is by (probe row, build row) after a sort within each probe
   row's run).
   out_probe_row / out_build_row: device int32[out_cap]; out_cols: device
   buffers of their source's dtype with room for out_cap values, all owned by
   the caller.  d_nout: device int64, receives the number of matches; above
   out_cap only the first out_cap are written and PYST_ERR_CAPACITY is
   latched (read the count and call again with room for it).  The table lives
   in the context's arena for the call only.
   Errors: PYST_ERR_ARG, PYST_ERR_NOMEM. */
pyst_status pyst_join_materialize(pyst_ctx *ctx, const pyst_col *build_key, const pyst_col *build_cols, int nbcols,
                                  const pyst_col *probe_key, const pyst_col *probe_cols, int npcols, double max_load,
                                  int unique_keys, void *const *out_cols, int32_t *out_probe_row,
                                  int32_t *out_build_row, int64_t out_cap, int64_t *d_nout, hipStream_t stream);

/* Enqueue a copy of the table's header into d_out (device int64[2]):
   [0] the effective capacity chosen on the device, [1] the number of rows
   offered for insertion.  For tests and diagnostics.  Errors: PYST_ERR_ARG. */
pyst_status pyst_table_info(const pyst_table *table, int64_t *d_out, hipStream_t stream);

/* Free a table.  Blocks until the work enqueued on `stream` (the last stream
   that used it) has completed.  NULL is a no-op. */
void pyst_table_destroy(pyst_table *table, hipStream_t stream);

/* ---------------------------------------------------------------- group-by */

/* GROUP BY key SUM(val) (the aggregation of Sec. 6.3, observation (5)).
   key: int32 or int64; val: int32 or int64; both sign-extended to int64.
   A group exists for every key that occurs (no zero rows).
   max_groups: upper bound on distinct keys (<= 0 means the row count).
   Output: out_keys / out_sums: device int64[max_groups]; d_ngroups: device
   int64.  Groups come out in table order, or ascending by key when
   sort_by_key != 0.  The key INT64_MIN is reserved (PYST_ERR_KEY); more than
   max_groups groups latch PYST_ERR_CAPACITY.
   Errors: PYST_ERR_ARG, PYST_ERR_NOMEM. */
pyst_status pyst_groupby_sum(pyst_ctx *ctx, const pyst_col *key, const pyst_col *val,
                             const int32_t *sel, const int64_t *d_nsel, int64_t max_groups,
                             double max_load, int64_t *out_keys, int64_t *out_sums,
                             int64_t *d_ngroups, int sort_by_key, hipStream_t stream);

/* ---------------------------------------------------------------- fused query */

/* A join step of a query plan: the dimension side is built into a hash table
   over int32 `key`, restricted by `preds` over `cols`; `payload` (int32, or
   data == NULL for none) is stored with each key.  The fact rows probe it
   with fact column `probe_col`. */
typedef struct pyst_join_spec {
  pyst_col key;
  pyst_col payload;
  const pyst_col *cols;
  int32_t ncols;
  int32_t npreds;
  const pyst_pred *preds;
  int32_t probe_col;
  int32_t reserved;
  double max_load;
} pyst_join_spec;

/* Source of one half of the group key. */
typedef enum pyst_gsrc {
  PYST_G_NONE = 0,
  PYST_G_JOIN_KEY = 1,     /* the matched build key of join `index`      */
  PYST_G_JOIN_PAYLOAD = 2, /* the stored payload of join `index`         */
  PYST_G_FACT_COL = 3      /* fact column `index`                        */
} pyst_gsrc;

typedef enum pyst_vexpr {
  PYST_V_COL = 0,              /* fact[v0]                                */
  PYST_V_COL_TIMES_C_MINUS = 1 /* fact[v0] * (vconst - fact[v1])          */
} pyst_vexpr;

/* Query: filter the fact table by `preds`, inner-join it with 1 or 2
   dimensions (a row survives if every join matches), then
   GROUP BY key SUM(value).  The group key is (int64(hi) << 32) | uint32(lo)
   when hi is set, else lo sign-extended.  Dimensions must have unique keys. */
typedef struct pyst_plan {
  int32_t njoins; /* 1 or 2 */
  int32_t npreds;
  pyst_join_spec joins[2];
  const pyst_pred *preds;
  int32_t hi_src, hi_index; /* pyst_gsrc */
  int32_t lo_src, lo_index;
  int32_t vexpr; /* pyst_vexpr */
  int32_t v0, v1;
  int32_t reserved;
  int64_t vconst;
  int64_t max_groups; /* <= 0: bounded by the rows reaching the aggregation */
  double group_max_load;
} pyst_plan;

/* Fused filter + join + group-by over the fact columns fact[0..nfact).  One
   build pass per dimension, then ONE pass over the fact table.  When the
   group key is the key of the single join, sums accumulate in the join
   table's slots (no second table).  out_keys / out_sums: device
   int64[out_cap]; d_ngroups: device int64; more than out_cap groups latch
   PYST_ERR_CAPACITY.  Errors: PYST_ERR_ARG, PYST_ERR_UNSUPPORTED,
   PYST_ERR_NOMEM. */
pyst_status pyst_query(pyst_ctx *ctx, const pyst_plan *plan, const pyst_col *fact, int nfact,
                       int64_t *out_keys, int64_t *out_sums, int64_t out_cap, int64_t *d_ngroups,
                       hipStream_t stream);

/* ---------------------------------------------------------------- packed columns */

/* A bit-packed column (the scan side: columns arrive compressed and are
   decoded on the GPU, Sec. 4, with a self-made encoding in place of a file
   format's).  Values are cut into blocks of PYST_PACK_BLOCK; block b stores
   its minimum as `base` and each value's offset from it in `bits` bits, where
   bits = 0..32 (int32) or 0..64 (int64) is the width of the block's range.
   Value j of block b occupies bits [j * bits, (j + 1) * bits) of the 32-bit
   little-endian words starting at words[blocks[b].word_off]; the block owns
   32 * bits words, so blocks[b + 1].word_off - blocks[b].word_off = 32 * bits
   and the block table has ceil(n / PYST_PACK_BLOCK) + 1 entries, the last
   holding the total word count (and base 0). */
#define PYST_PACK_BLOCK 1024

typedef struct pyst_pack_block {
  int64_t base;
  int64_t word_off;
} pyst_pack_block;

typedef struct pyst_packed_col {
  const pyst_pack_block *blocks; /* ceil(n / PYST_PACK_BLOCK) + 1 entries */
  const uint32_t *words;         /* blocks[nblocks].word_off words */
  int64_t n;                     /* values */
  int32_t dtype;                 /* pyst_dtype of the decoded column */
  int32_t reserved;
} pyst_packed_col;

/* Host only (no device work): the number of 32-bit words pyst_pack_encode
   writes for the HOST column host_col, or -1 for a bad column. */
int64_t pyst_pack_words(const pyst_col *host_col);

/* Host only: encode the HOST column host_col into blocks
   (ceil(n / PYST_PACK_BLOCK) + 1 entries) and words (pyst_pack_words(host_col)
   entries), both host memory owned by the caller.  Errors: PYST_ERR_ARG. */
pyst_status pyst_pack_encode(const pyst_col *host_col, pyst_pack_block *blocks, uint32_t *words);

/* Decode a packed column held in DEVICE memory (d_blocks with
   ceil(n / PYST_PACK_BLOCK) + 1 entries, d_words with nwords words) into the
   device column d_out (n values of `dtype`).  A block whose header is
   malformed or whose words fall outside [0, nwords) latches PYST_ERR_INDEX
   and leaves its values unwritten.  Errors: PYST_ERR_ARG. */
pyst_status pyst_pack_decode(pyst_ctx *ctx, const pyst_pack_block *d_blocks, const uint32_t *d_words, int64_t nwords,
                             int64_t n, int dtype, void *d_out, hipStream_t stream);

/* ---------------------------------------------------------------- streamed query */

/* pyst_query over a fact table held in PINNED HOST memory (hipHostMalloc or
   pinned torch tensors), streamed to the device in chunks (Sec. 3.2,
   "Partial Overlap Using Chunking"; memory relief of Sec. 3.4).
   host_fact[c].data are host pointers (16-byte aligned, total rows < 2^31);
   the plan's dimension columns are device pointers as in pyst_query.
   chunk_rows (a positive multiple of 4) rows of every fact column are copied
   on the context's copy stream into a ring of nbuf (2..8) device buffers
   taken from the arena, and the fused fact pass runs per chunk on `stream`;
   buffer reuse is ordered by device events, so the call only enqueues work and
   returns (no host synchronization between chunks).  The host buffers must
   stay alive and unchanged until `stream` completes.
   Only plans served by the specialized fact pass can be streamed, and group
   keys other than the single join key need plan->max_groups > 0 (the group
   table must exist before the first chunk).
   Errors: PYST_ERR_ARG, PYST_ERR_UNSUPPORTED, PYST_ERR_NOMEM, PYST_ERR_HIP. */
pyst_status pyst_query_streamed(pyst_ctx *ctx, const pyst_plan *plan, const pyst_col *host_fact, int nfact,
                                int64_t chunk_rows, int nbuf, int64_t *out_keys, int64_t *out_sums,
                                int64_t out_cap, int64_t *d_ngroups, hipStream_t stream);

/* pyst_query_streamed over PACKED fact columns in PINNED HOST memory (block
   tables and words): each chunk of chunk_rows (a positive multiple of
   PYST_PACK_BLOCK below 2^31) rows moves as its packed blocks on the copy
   stream and is decoded on the device into the chunk ring before the fused
   pass, so the host link carries the packed bytes.  The block tables are
   checked on the host first (offsets from 0 in whole 32-word steps of at most
   32 or 64 bits a value).  Otherwise as pyst_query_streamed.
   Errors: PYST_ERR_ARG, PYST_ERR_UNSUPPORTED, PYST_ERR_NOMEM, PYST_ERR_HIP. */
pyst_status pyst_query_streamed_packed(pyst_ctx *ctx, const pyst_plan *plan, const pyst_packed_col *host_fact,
                                       int nfact, int64_t chunk_rows, int nbuf, int64_t *out_keys, int64_t *out_sums,
                                       int64_t out_cap, int64_t *d_ngroups, hipStream_t stream);

/* ---------------------------------------------------------------- batched fragments */

/* One independent query fragment: a plan (its own dimension columns), its own
   device fact columns, and its outputs (as for pyst_query). */
typedef struct pyst_fragment {
  const pyst_plan *plan;
  const pyst_col *fact;
  int32_t nfact;
  int32_t reserved;
  int64_t *out_keys;
  int64_t *out_sums;
  int64_t out_cap;
  int64_t *d_ngroups;
} pyst_fragment;

/* Batch execution parameters.
   fanout   : the number of work units each fragment's fact table is split into
              (at least 4 * block rows per unit), i.e. how finely large
              fragments spread over the chip next to small ones;
   block    : threads per block of the fact pass (256, 512 or 1024);
   max_load : hash-table load bound of every fragment (0: the plan's). */
typedef struct pyst_tuning {
  int32_t fanout;
  int32_t block;
  double max_load;
} pyst_tuning;

/* Run nfrag fragments as one batch: six launches in total (dimension filter,
   table init, build, Bloom filter, fact pass, compaction), each covering every fragment, in
   place of a launch sequence and a host round trip per fragment -- the
   small-work inefficiency the paper counters by buffering small chunks into
   larger units (Sec. 5.3, "Dynamic Buffering").  Every fragment must be a
   single-join star query grouped by the join key on int32 columns with the
   same value dtype; each gets exactly the result pyst_query gives it.
   tuning may be NULL (defaults {64, 512, 0}).  Errors: PYST_ERR_ARG,
   PYST_ERR_UNSUPPORTED, PYST_ERR_NOMEM, PYST_ERR_HIP. */
pyst_status pyst_query_batch(pyst_ctx *ctx, const pyst_fragment *frags, int nfrag, const pyst_tuning *tuning,
                             hipStream_t stream);

/* Search fanout {16,32,64,128,256} x block {256,512,1024} x max_load
   {0.5,0.7} for the fastest pyst_query_batch of these fragments (mean of
   `reps` timed runs after one warm-up, HIP events on a private stream).
   Blocks until done; writes the winner to *out and its time to *best_ms
   (may be NULL).  Errors: as pyst_query_batch. */
pyst_status pyst_autotune(pyst_ctx *ctx, const pyst_fragment *frags, int nfrag, int reps, pyst_tuning *out,
                          double *best_ms);

/* A batch captured once as a HIP graph of its six launches and replayed with
   one hipGraphLaunch: the whole batch of uneven fragments becomes one unit of
   work for the stream, with no host-side layout, upload or launch sequence per
   run (the buffering of small work into large units, Sec. 5.3, carried down to
   the launch itself).  pyst_batch_graph_create lays the batch out, allocates its
   device memory from the context arena (held until destroy), uploads the
   descriptors on `stream` and waits for them, then captures the launches on a
   private stream.  Every replay recomputes every fragment from the current
   contents of the inputs named at creation and overwrites the fragments'
   outputs; the graph holds no memset node (tables are cleared by kernels).
   Replays on one stream are ordered; replays that overlap on different streams
   race on the batch's tables.  Errors: as pyst_query_batch. */
typedef struct pyst_batch_graph pyst_batch_graph;
pyst_status pyst_batch_graph_create(pyst_ctx *ctx, const pyst_fragment *frags, int nfrag, const pyst_tuning *tuning,
                                    hipStream_t stream, pyst_batch_graph **out);
/* Enqueue one replay on `stream`.  Errors: PYST_ERR_ARG, PYST_ERR_HIP. */
pyst_status pyst_batch_graph_launch(pyst_batch_graph *g, hipStream_t stream);
/* Wait for the device to be idle, then free the graph and its arena memory
   (NULL: no-op).  Errors: PYST_ERR_HIP. */
pyst_status pyst_batch_graph_destroy(pyst_batch_graph *g);

/* ---------------------------------------------------------------- serving */

/* A query server over one fact table in pinned host memory, after the
   queue-based scheduling of Sec. 5.4: client threads submit requests into a
   multi-producer queue; one scheduler thread issues all GPU work.  It admits
   requests while stream slots and device memory allow (adaptive regulation:
   excess load waits in the queue), keeps built dimension tables resident
   across requests, and runs the active requests on shared chunks of the fact
   table -- the next chunk copied is, among the next chunks of the active
   requests (each reads its chunks in order), the one the most of them still
   need (ties to the oldest request); it is copied to the device once and
   consumed by every active request that needs it (the reader combining of
   Sec. 5.2).  The scheduler reuses a ring buffer only after that buffer's
   previous readers have finished, so it decides each chunk just in time.
   Requests arriving while others run are admitted at once and ride along on
   the shared chunks (continuous batching).  max_active = 1 gives
   one-at-a-time FIFO service over the same machinery. */
typedef struct pyst_server pyst_server;

typedef struct pyst_server_cfg {
  size_t budget_bytes; /* device memory for dimension tables and aggregation state */
  int32_t max_active;  /* concurrently served requests (1..64), one stream each      */
  int32_t nbuf;        /* chunk buffers in the device ring (2..8)                   */
  int64_t chunk_rows;  /* fact rows per chunk (a positive multiple of 4)            */
} pyst_server_cfg;

/* A request: plan over the server's fact columns (same column order as at
   creation; dimension columns are device pointers that must stay alive until
   the request completes), scanning fact rows [0, rows).  The plan is copied at
   submit.  Outputs are device buffers as in pyst_query. */
typedef struct pyst_request {
  const pyst_plan *plan;
  int64_t rows;
  int64_t *out_keys;
  int64_t *out_sums;
  int64_t out_cap;
  int64_t *d_ngroups;
} pyst_request;

typedef struct pyst_server_stats {
  int64_t submitted;
  int64_t completed;
  int64_t chunks_copied;
  int64_t admission_waits;  /* times the queue head waited for memory or a slot */
  int64_t max_active_seen;
  double bytes_copied;      /* host-to-device bytes of fact chunks       */
  double fact_rows_processed; /* sum over requests of fact rows consumed  */
} pyst_server_stats;

/* Create a server on `device` over host_fact[0..nfact) (pinned host columns,
   kept alive by the caller until pyst_server_destroy).  Allocates its own
   context (arena = cfg->budget_bytes plus the chunk ring) and starts the
   scheduler thread.  Errors: PYST_ERR_ARG, PYST_ERR_NOMEM, PYST_ERR_HIP. */
pyst_status pyst_server_create(int device, const pyst_server_cfg *cfg, const pyst_col *host_fact, int nfact,
                               pyst_server **out);

/* pyst_server_create over PACKED fact columns in pinned host memory (see
   pyst_pack_encode), kept alive by the caller until pyst_server_destroy: each
   chunk moves over the host link as its packed blocks and is decoded on the
   device before the requests that share it run.  cfg->chunk_rows must be a
   multiple of PYST_PACK_BLOCK; block tables are checked on the host.
   Errors: PYST_ERR_ARG, PYST_ERR_NOMEM, PYST_ERR_HIP. */
pyst_status pyst_server_create_packed(int device, const pyst_server_cfg *cfg, const pyst_packed_col *host_fact,
                                      int nfact, pyst_server **out);

/* Queue a request (thread-safe, never blocks on the GPU); *ticket identifies
   it.  Only plans served by the specialized fact pass are accepted, and group
   keys other than the single join key need plan->max_groups > 0.
   Errors: PYST_ERR_ARG, PYST_ERR_UNSUPPORTED. */
pyst_status pyst_server_submit(pyst_server *server, const pyst_request *req, uint64_t *ticket);

/* Block until request `ticket` has completed (its outputs are then final);
   *latency_ms = completion - submission.  Returns the request's own status:
   PYST_ERR_NOMEM if it can never fit the budget, a host-side error of one of
   its launches (the request then stops at that chunk and is finished), or an
   error its kernels latched (each request has its own device error word, and
   so has each resident dimension table: a capacity overflow of one request,
   or a duplicate key in its dimension, fails that request and no other).
   A ticket is waited once. */
pyst_status pyst_server_wait(pyst_server *server, uint64_t ticket, double *latency_ms);

/* Non-blocking form of pyst_server_wait (the scheduler's queues are polled,
   Sec. 5.4 "Queue-Based Scheduling"): never waits for the GPU, only for the
   server's own lock.  While request `ticket` runs, *done = 0 and PYST_OK is
   returned; once it has completed, *done = 1, *latency_ms (may be NULL) is
   set, and the request's own status is returned exactly as pyst_server_wait
   would, after which the ticket is forgotten.
   Errors: PYST_ERR_ARG (NULL server or done, unknown or already reported
   ticket), else the request's status. */
pyst_status pyst_server_poll(pyst_server *server, uint64_t ticket, int *done, double *latency_ms);

/* Counters since creation.  Errors: PYST_ERR_ARG. */
pyst_status pyst_server_get_stats(pyst_server *server, pyst_server_stats *out);

/* Resident dimension tables are identified by the device addresses and lengths
   of their dimension columns and by their predicates, not by the columns'
   contents.  Before a caller frees, reuses or overwrites the memory of a
   dimension column it has used in a request, it calls this with that column's
   data pointer (NULL: every column): the cached tables built over it are
   dropped (their memory is returned once the active requests using them have
   finished), so a later request rebuilds them from the current contents.
   Requests submitted after this call returns never see the dropped tables.
   Tables that no active request uses are also dropped when a new one does not
   fit the budget.  Errors: PYST_ERR_ARG. */
pyst_status pyst_server_forget_tables(pyst_server *server, const void *dim_col_data);

/* Set a context option (PYST_OPT_*) of the server's own context, e.g. the
   PYST_OPT_FAIL_FACT_PASS test hook.  Takes effect for work the scheduler
   issues after the call.  Errors: PYST_ERR_ARG. */
pyst_status pyst_server_option(pyst_server *server, int key, int64_t value);

/* Wait for the device and return the errors latched by the server's kernels. */
pyst_status pyst_server_check(pyst_server *server);

/* Finish every submitted request, stop the scheduler and free everything. */
void pyst_server_destroy(pyst_server *server);

#ifdef __cplusplus
}
#endif

#endif /* PYST_H */

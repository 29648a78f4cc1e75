/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded definitions of what the relational hot path
 * computes.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this library; the product path never does.  It shares no
 * code, header or constant table with the GPU library: it has its own hash
 * finalizer, predicate evaluator and key packing.
 *
 * Operators (PystachIO, arXiv 2512.02862):
 *   - filter      : predicates pushed into the scan (Sec. 4, introduction;
 *                   Sec. 6.1 "Hardware" notes scans run with filter pushdown).
 *   - partition   : split rows by join key into per-destination buffers, the
 *                   first step of the distributed hash join (Sec. 3.1 "Anatomy
 *                   of a Distributed Hash Join"; "A Naive Implementation in
 *                   PyTorch" partitions by modulo + masked selection).  The
 *                   destination function is the MurmurHash3 32-bit finalizer
 *                   of the key, mod F (the workload definition names it).
 *   - join        : build a hash table over the fully materialized left side,
 *                   probe it with the right side and emit the join tuples
 *                   (Sec. 3.1 "Anatomy..."; Sec. 3.2 "Scheduling Overlap").
 *   - group-by SUM: the aggregation operator (Sec. 6.3, observation (5)); the
 *                   paper gives no design, so it is defined by SQL semantics.
 *   - star / chain queries: compositions of the above in plan order, over
 *                   dictionary-encoded integer columns (Sec. 6.1 "Workload").
 *
 * All arithmetic is integer; sums wrap modulo 2^64 (two's complement), which
 * makes them independent of summation order.
 */
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

/* MurmurHash3 32-bit finalizer (Appleby, public domain): xor-shift / multiply rounds. */
uint32_t murmur_fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

/* MurmurHash3 64-bit finalizer. */
uint64_t murmur_fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

/* Read row i of a column holding int32 (is64 == 0) or int64 values, as int64. */
int64_t value_at(const void *col, int is64, int64_t i) {
  if (is64) return static_cast<const int64_t *>(col)[i];
  return static_cast<int64_t>(static_cast<const int32_t *>(col)[i]);
}

/* Comparison codes: 0 ==, 1 !=, 2 <, 3 <=, 4 >, 5 >=. */
bool compare(int64_t x, int op, int64_t c) {
  switch (op) {
    case 0: return x == c;
    case 1: return x != c;
    case 2: return x < c;
    case 3: return x <= c;
    case 4: return x > c;
    case 5: return x >= c;
  }
  return false;
}

/* Row ids in order: the selection if one is given, else 0..n-1. */
std::vector<int64_t> rows_of(int64_t n, const int32_t *sel, int64_t nsel) {
  std::vector<int64_t> r;
  if (sel) {
    r.reserve(static_cast<size_t>(nsel));
    for (int64_t i = 0; i < nsel; ++i) r.push_back(sel[i]);
  } else {
    r.reserve(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) r.push_back(i);
  }
  return r;
}

uint32_t partition_hash(const void *key, int key64, int64_t row) {
  if (key64) {
    uint64_t k = static_cast<uint64_t>(value_at(key, 1, row));
    return static_cast<uint32_t>(murmur_fmix64(k) & 0xffffffffull);
  }
  return murmur_fmix32(static_cast<uint32_t>(static_cast<int32_t>(value_at(key, 0, row))));
}

/* Join result: (probe position, build row) pairs. */
using Pairs = std::vector<std::pair<int64_t, int64_t>>;

/*
 * Inner equi-join of build rows `brows` of key column bkey with probe keys
 * pkeys[0..np-1].  Build side: unordered_map key -> build rows (ascending).
 * For every probe position in ascending order, every matching build row in
 * ascending order is emitted.
 */
Pairs equi_join(const void *bkey, int b64, const std::vector<int64_t> &brows,
                const std::vector<int64_t> &pkeys) {
  std::unordered_map<int64_t, std::vector<int64_t>> table;
  for (int64_t j : brows) table[value_at(bkey, b64, j)].push_back(j);
  Pairs out;
  for (size_t i = 0; i < pkeys.size(); ++i) {
    auto it = table.find(pkeys[i]);
    if (it == table.end()) continue;
    for (int64_t j : it->second) out.emplace_back(static_cast<int64_t>(i), j);
  }
  return out;
}

/* Group (key, value) pairs: sort by key, then run-length sum modulo 2^64. */
int64_t group_sum(std::vector<std::pair<int64_t, int64_t>> kv, int64_t *out_keys,
                  int64_t *out_sums) {
  std::sort(kv.begin(), kv.end(),
            [](const std::pair<int64_t, int64_t> &a, const std::pair<int64_t, int64_t> &b) {
              return a.first < b.first;
            });
  int64_t g = 0;
  size_t i = 0;
  while (i < kv.size()) {
    const int64_t k = kv[i].first;
    uint64_t s = 0;
    while (i < kv.size() && kv[i].first == k) {
      s += static_cast<uint64_t>(kv[i].second);
      ++i;
    }
    if (out_keys) out_keys[g] = k;
    if (out_sums) out_sums[g] = static_cast<int64_t>(s);
    ++g;
  }
  return g;
}

std::vector<int64_t> filter_rows(const void *const *cols, const int32_t *is64, int64_t n,
                                 const int32_t *pcol, const int32_t *pop, const int64_t *pval,
                                 int npred) {
  std::vector<int64_t> out;
  for (int64_t i = 0; i < n; ++i) {
    bool keep = true;
    for (int p = 0; p < npred && keep; ++p)
      keep = compare(value_at(cols[pcol[p]], is64[pcol[p]], i), pop[p], pval[p]);
    if (keep) out.push_back(i);
  }
  return out;
}

}  // namespace

extern "C" {

uint32_t oracle_fmix32(uint32_t h) { return murmur_fmix32(h); }
uint64_t oracle_fmix64(uint64_t k) { return murmur_fmix64(k); }

/*
 * Filter: row i is selected iff every predicate (column pcol[p], comparison
 * pop[p], constant pval[p]) holds; values are sign-extended to int64 first.
 * Writes the ascending selection vector and returns its length.
 */
int64_t oracle_filter(const void *const *cols, const int32_t *is64, int ncols, int64_t n,
                      const int32_t *pcol, const int32_t *pop, const int64_t *pval, int npred,
                      int32_t *sel_out) {
  for (int p = 0; p < npred; ++p)
    if (pcol[p] < 0 || pcol[p] >= ncols) return -1;
  std::vector<int64_t> rows = filter_rows(cols, is64, n, pcol, pop, pval, npred);
  for (size_t i = 0; i < rows.size(); ++i) sel_out[i] = static_cast<int32_t>(rows[i]);
  return static_cast<int64_t>(rows.size());
}

/*
 * Hash partition into F destinations: dest = h(key) mod F with
 * h = fmix32(uint32 key) for int32 keys and low32(fmix64(uint64 key)) for
 * int64 keys.  offsets = exclusive prefix sum of the per-destination counts
 * (F + 1 entries); rows are scattered stably (input order kept inside a
 * destination).  pay_width[j] is 4 or 8 bytes.  Returns the row count.
 */
int64_t oracle_partition(const void *key, int key64, int64_t n, const int32_t *sel, int64_t nsel,
                         const void *const *pay, const int32_t *pay_width, int npay,
                         uint32_t fanout, void *out_key, void *const *out_pay, int64_t *offsets) {
  if (fanout == 0) return -1;
  std::vector<int64_t> rows = rows_of(n, sel, nsel);
  std::vector<uint32_t> dest(rows.size());
  std::vector<int64_t> count(fanout, 0);
  for (size_t i = 0; i < rows.size(); ++i) {
    dest[i] = partition_hash(key, key64, rows[i]) % fanout;
    count[dest[i]]++;
  }
  offsets[0] = 0;
  for (uint32_t p = 0; p < fanout; ++p) offsets[p + 1] = offsets[p] + count[p];
  std::vector<int64_t> cursor(offsets, offsets + fanout);
  const int kw = key64 ? 8 : 4;
  for (size_t i = 0; i < rows.size(); ++i) {
    const int64_t o = cursor[dest[i]]++;
    std::memcpy(static_cast<char *>(out_key) + o * kw,
                static_cast<const char *>(key) + rows[i] * kw, kw);
    for (int j = 0; j < npay; ++j) {
      const int w = pay_width[j];
      std::memcpy(static_cast<char *>(out_pay[j]) + o * w,
                  static_cast<const char *>(pay[j]) + rows[i] * w, w);
    }
  }
  return static_cast<int64_t>(rows.size());
}

/*
 * Inner equi-join of the selected build rows (key column bkey) with the
 * selected probe rows (key column pkey).  Emits (probe row, build row) in
 * ascending probe row, then ascending build row.  Writes at most cap pairs
 * and returns the full result size.
 */
int64_t oracle_join(const void *bkey, int b64, int64_t nb, const int32_t *bsel, int64_t nbsel,
                    const void *pkey, int p64, int64_t np, const int32_t *psel, int64_t npsel,
                    int32_t *out_probe, int32_t *out_build, int64_t cap) {
  std::vector<int64_t> brows = rows_of(nb, bsel, nbsel);
  std::vector<int64_t> prows = rows_of(np, psel, npsel);
  std::vector<int64_t> pkeys(prows.size());
  for (size_t i = 0; i < prows.size(); ++i) pkeys[i] = value_at(pkey, p64, prows[i]);
  Pairs pairs = equi_join(bkey, b64, brows, pkeys);
  const int64_t m = static_cast<int64_t>(pairs.size());
  for (int64_t t = 0; t < m && t < cap; ++t) {
    out_probe[t] = static_cast<int32_t>(prows[static_cast<size_t>(pairs[t].first)]);
    out_build[t] = static_cast<int32_t>(pairs[t].second);
  }
  return m;
}

/*
 * GROUP BY key SUM(val) over the selected rows.  Keys and values are
 * sign-extended to int64; sums wrap modulo 2^64.  Groups come out in
 * ascending key order; only keys that occur form groups.  Returns the
 * number of groups (out arrays need room for the number of rows).
 */
int64_t oracle_groupby_sum(const void *key, int k64, const void *val, int v64, int64_t n,
                           const int32_t *sel, int64_t nsel, int64_t *out_keys,
                           int64_t *out_sums) {
  std::vector<int64_t> rows = rows_of(n, sel, nsel);
  std::vector<std::pair<int64_t, int64_t>> kv;
  kv.reserve(rows.size());
  for (int64_t r : rows) kv.emplace_back(value_at(key, k64, r), value_at(val, v64, r));
  return group_sum(std::move(kv), out_keys, out_sums);
}

/*
 * Star query: SELECT b.key, SUM(p.price) FROM build b JOIN probe p ON p.fk = b.key
 * WHERE <build predicates> AND <probe predicates> GROUP BY b.key.
 * Build columns are [key, segment] (int32); probe columns are
 * [fk int32, date int32, price int64].  Returns the number of groups.
 */
int64_t oracle_star_query(const int32_t *bkey, const int32_t *bseg, int64_t nb,
                          const int32_t *bpcol, const int32_t *bpop, const int64_t *bpval,
                          int nbpred, const int32_t *fk, const int32_t *date,
                          const int64_t *price, int64_t np, const int32_t *ppcol,
                          const int32_t *ppop, const int64_t *ppval, int nppred,
                          int64_t *out_keys, int64_t *out_sums) {
  const void *bcols[2] = {bkey, bseg};
  const int32_t b64[2] = {0, 0};
  const void *pcols[3] = {fk, date, price};
  const int32_t p64[3] = {0, 0, 1};
  std::vector<int64_t> brows = filter_rows(bcols, b64, nb, bpcol, bpop, bpval, nbpred);
  std::vector<int64_t> prows = filter_rows(pcols, p64, np, ppcol, ppop, ppval, nppred);
  std::vector<int64_t> pkeys(prows.size());
  for (size_t i = 0; i < prows.size(); ++i) pkeys[i] = fk[prows[i]];
  Pairs joined = equi_join(bkey, 0, brows, pkeys);
  std::vector<std::pair<int64_t, int64_t>> kv;
  kv.reserve(joined.size());
  for (const auto &pr : joined) {
    const int64_t prow = prows[static_cast<size_t>(pr.first)];
    kv.emplace_back(static_cast<int64_t>(bkey[pr.second]), price[prow]);
  }
  return group_sum(std::move(kv), out_keys, out_sums);
}

/*
 * Two-join chain: fact JOIN B ON fact.b_fk = B.key JOIN A ON fact.a_fk = A.key,
 * GROUP BY (B.key, A.date) SUM(price * (vconst - discount)).
 * The group key is packed as (int64(B.key) << 32) | uint32(A.date).
 * A columns [key, date], B columns [key, segment], fact columns
 * [a_fk, b_fk, date, price (int64), discount].  Returns the number of groups.
 */
int64_t oracle_chain_query(const int32_t *akey, const int32_t *adate, int64_t na,
                           const int32_t *apcol, const int32_t *apop, const int64_t *apval,
                           int napred, const int32_t *bkey, const int32_t *bseg, int64_t nb,
                           const int32_t *bpcol, const int32_t *bpop, const int64_t *bpval,
                           int nbpred, const int32_t *a_fk, const int32_t *b_fk,
                           const int32_t *fdate, const int64_t *price, const int32_t *discount,
                           int64_t nf, const int32_t *fpcol, const int32_t *fpop,
                           const int64_t *fpval, int nfpred, int64_t vconst, int64_t *out_keys,
                           int64_t *out_sums) {
  const void *acols[2] = {akey, adate};
  const int32_t a64[2] = {0, 0};
  const void *bcols[2] = {bkey, bseg};
  const int32_t b64[2] = {0, 0};
  const void *fcols[5] = {a_fk, b_fk, fdate, price, discount};
  const int32_t f64[5] = {0, 0, 0, 1, 0};
  std::vector<int64_t> arows = filter_rows(acols, a64, na, apcol, apop, apval, napred);
  std::vector<int64_t> brows = filter_rows(bcols, b64, nb, bpcol, bpop, bpval, nbpred);
  std::vector<int64_t> frows = filter_rows(fcols, f64, nf, fpcol, fpop, fpval, nfpred);

  /* fact JOIN B: tuples (fact row, B row). */
  std::vector<int64_t> keys1(frows.size());
  for (size_t i = 0; i < frows.size(); ++i) keys1[i] = b_fk[frows[i]];
  Pairs j1 = equi_join(bkey, 0, brows, keys1);

  /* (fact JOIN B) JOIN A: probe A with a_fk of every tuple of the first join. */
  std::vector<int64_t> keys2(j1.size());
  for (size_t t = 0; t < j1.size(); ++t) keys2[t] = a_fk[frows[static_cast<size_t>(j1[t].first)]];
  Pairs j2 = equi_join(akey, 0, arows, keys2);

  std::vector<std::pair<int64_t, int64_t>> kv;
  kv.reserve(j2.size());
  for (const auto &pr : j2) {
    const auto &t1 = j1[static_cast<size_t>(pr.first)];
    const int64_t frow = frows[static_cast<size_t>(t1.first)];
    const int64_t brow = t1.second;
    const int64_t arow = pr.second;
    const uint64_t hi = static_cast<uint64_t>(static_cast<int64_t>(bkey[brow])) << 32;
    const uint64_t lo = static_cast<uint64_t>(static_cast<uint32_t>(adate[arow]));
    const uint64_t v = static_cast<uint64_t>(price[frow]) *
                       static_cast<uint64_t>(vconst - static_cast<int64_t>(discount[frow]));
    kv.emplace_back(static_cast<int64_t>(hi | lo), static_cast<int64_t>(v));
  }
  return group_sum(std::move(kv), out_keys, out_sums);
}

}  // extern "C"

/*
 * THREADED CPU BASELINE -- TEST AND MEASUREMENT INFRASTRUCTURE ONLY.
 *
 * The star query of the oracle (filter, inner equi-join, GROUP BY join key
 * SUM(price); the operators of Sec. 3.1 "Anatomy of a Distributed Hash Join"
 * and the aggregation of Sec. 6.3) spread over host threads, so that the GPU
 * path can be set beside every host core and not only one.  Same algorithm as
 * the single-threaded oracle:
 *   - the filtered build rows go into one std::unordered_map (key -> build
 *     rows), built once and then shared read-only by every thread;
 *   - each thread takes a contiguous range of probe rows, filters them, probes
 *     the map and collects (key, price) pairs in its own vector;
 *   - each thread sorts its pairs by key and sums runs modulo 2^64;
 *   - the sorted per-thread group lists are merged pairwise (merge sort of
 *     runs), adding the sums of equal keys.
 * Sums wrap modulo 2^64, so the result equals the oracle's whatever the
 * thread count; a CPU test checks that.  Nothing here is shared with the GPU
 * library or with the oracle's source.
 */
#include <algorithm>
#include <cstdint>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

namespace {

using Group = std::pair<int64_t, uint64_t>;  // (key, sum mod 2^64)

bool holds(int64_t x, int op, int64_t c) {
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

/* Merge two key-sorted group lists, adding the sums of keys present in both. */
std::vector<Group> merge_groups(const std::vector<Group> &a, const std::vector<Group> &b) {
  std::vector<Group> out;
  out.reserve(a.size() + b.size());
  size_t i = 0, j = 0;
  while (i < a.size() || j < b.size()) {
    if (j == b.size() || (i < a.size() && a[i].first < b[j].first)) {
      out.push_back(a[i++]);
    } else if (i == a.size() || b[j].first < a[i].first) {
      out.push_back(b[j++]);
    } else {
      out.emplace_back(a[i].first, a[i].second + b[j].second);
      ++i;
      ++j;
    }
  }
  return out;
}

}  // namespace

extern "C" {

/*
 * Star query on `nthreads` host threads (<= 0: every hardware thread).
 * Build columns [key, segment] (int32); probe columns [fk int32, date int32,
 * price int64]; predicate codes 0 ==, 1 !=, 2 <, 3 <=, 4 >, 5 >= on the named
 * column index, all of a list must hold.  Writes (key ascending, sum) and
 * returns the number of groups; *threads_used receives the thread count.
 */
int64_t baseline_star_query_mt(const int32_t *bkey, const int32_t *bseg, int64_t nb, const int32_t *bpcol,
                               const int32_t *bpop, const int64_t *bpval, int nbpred, const int32_t *fk,
                               const int32_t *date, const int64_t *price, int64_t np, const int32_t *ppcol,
                               const int32_t *ppop, const int64_t *ppval, int nppred, int nthreads,
                               int64_t *out_keys, int64_t *out_sums, int32_t *threads_used) {
  if (nthreads <= 0) nthreads = static_cast<int>(std::max(1u, std::thread::hardware_concurrency()));
  if (threads_used) *threads_used = nthreads;

  std::unordered_map<int32_t, std::vector<int64_t>> table;
  for (int64_t j = 0; j < nb; ++j) {
    bool keep = true;
    for (int p = 0; p < nbpred && keep; ++p) {
      const int64_t x = bpcol[p] == 0 ? bkey[j] : bseg[j];
      keep = holds(x, bpop[p], bpval[p]);
    }
    if (keep) table[bkey[j]].push_back(j);
  }

  std::vector<std::vector<Group>> part(static_cast<size_t>(nthreads));
  auto work = [&](int t) {
    const int64_t lo = np * t / nthreads, hi = np * (t + 1) / nthreads;
    std::vector<std::pair<int64_t, int64_t>> kv;
    for (int64_t i = lo; i < hi; ++i) {
      bool keep = true;
      for (int p = 0; p < nppred && keep; ++p) {
        const int64_t x = ppcol[p] == 0 ? fk[i] : ppcol[p] == 1 ? date[i] : price[i];
        keep = holds(x, ppop[p], ppval[p]);
      }
      if (!keep) continue;
      auto it = table.find(fk[i]);
      if (it == table.end()) continue;
      for (int64_t j : it->second) kv.emplace_back(static_cast<int64_t>(bkey[j]), price[i]);
    }
    std::sort(kv.begin(), kv.end(),
              [](const std::pair<int64_t, int64_t> &a, const std::pair<int64_t, int64_t> &b) { return a.first < b.first; });
    std::vector<Group> &g = part[static_cast<size_t>(t)];
    for (size_t k = 0; k < kv.size();) {
      const int64_t key = kv[k].first;
      uint64_t s = 0;
      for (; k < kv.size() && kv[k].first == key; ++k) s += static_cast<uint64_t>(kv[k].second);
      g.emplace_back(key, s);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto &th : pool) th.join();

  // pairwise merge rounds (the merge step of a merge sort over the runs)
  while (part.size() > 1) {
    std::vector<std::vector<Group>> next((part.size() + 1) / 2);
    std::vector<std::thread> mpool;
    for (size_t k = 0; k + 1 < part.size(); k += 2)
      mpool.emplace_back([&, k] { next[k / 2] = merge_groups(part[k], part[k + 1]); });
    if (part.size() % 2) next.back() = std::move(part.back());
    for (auto &th : mpool) th.join();
    part.swap(next);
  }
  const std::vector<Group> &all = part[0];
  for (size_t k = 0; k < all.size(); ++k) {
    out_keys[k] = all[k].first;
    out_sums[k] = static_cast<int64_t>(all[k].second);
  }
  return static_cast<int64_t>(all.size());
}

}  // extern "C"

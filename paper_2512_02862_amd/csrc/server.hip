// Serving loop: continuous batching of queries over one fact table held in
// pinned host memory.
//
// Structure after the paper's queue-based scheduling (Sec. 5.4): client
// threads push requests into a multi-producer queue; one scheduler thread
// consumes it and is the only thread that issues GPU work.  Admission is
// regulated by device memory (Sec. 5.4, "Adaptive Regulation"): a request
// starts only when its aggregation state fits in the server's arena, so load
// beyond the budget waits in the queue instead of failing.  All active
// requests share one scan of the fact table, driven by the oldest request --
// each chunk is copied once and consumed by every request that still needs
// it, the analog of one I/O pool serving every scan of a plan (Sec. 5.2,
// "Reader Combining").
// Dimension tables are built once and stay resident for later requests.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pyst_internal.h"
#include "query.h"
#include "table.h"

namespace pyst {

// Clears a request's group counter and, for slot sums, the sums and flags of
// the table's slots -- never past the request's own arrays (t.cap_alloc
// slots): a header claiming more slots latches kErrIndex instead.
__global__ void k_req_init(TableDev t, int64_t *d_ngroups, uint32_t *err) {
  int64_t cap = t.hdr[0];
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (tid == 0) *d_ngroups = 0;
  if (t.sums && (cap < 0 || cap > t.cap_alloc)) {
    if (tid == 0) latch(err, kErrIndex);
    cap = cap < 0 ? 0 : t.cap_alloc;
  }
  if (t.sums)
    for (int64_t i = tid; i < cap; i += (int64_t)gridDim.x * blockDim.x) {
      t.sums[i] = 0;
      t.flags[i] = 0;
    }
}

// A deep copy of a plan (the caller's arrays may go away after submit).
struct PlanCopy {
  pyst_plan plan;
  std::vector<pyst_pred> preds;
  std::vector<pyst_pred> jpreds[2];
  std::vector<pyst_col> jcols[2];
  void take(const pyst_plan &p) {
    plan = p;
    preds.assign(p.preds, p.preds + std::max(0, p.npreds));
    plan.preds = preds.data();
    for (int j = 0; j < p.njoins && j < 2; ++j) {
      jpreds[j].assign(p.joins[j].preds, p.joins[j].preds + std::max(0, p.joins[j].npreds));
      jcols[j].assign(p.joins[j].cols, p.joins[j].cols + std::max(0, p.joins[j].ncols));
      plan.joins[j].preds = jpreds[j].data();
      plan.joins[j].cols = jcols[j].data();
    }
  }
  std::string dim_signature() const {
    std::string s;
    char buf[160];
    for (int j = 0; j < plan.njoins; ++j) {
      const pyst_join_spec &js = plan.joins[j];
      snprintf(buf, sizeof buf, "j%d:%p:%lld:%p:%g:", j, js.key.data, static_cast<long long>(js.key.n), js.payload.data,
               js.max_load);
      s += buf;
      for (const auto &pr : jpreds[j]) {
        const void *cp = pr.col >= 0 && pr.col < static_cast<int>(jcols[j].size()) ? jcols[j][pr.col].data : nullptr;
        snprintf(buf, sizeof buf, "%p,%d,%lld;", cp, pr.cmp, static_cast<long long>(pr.value));
        s += buf;
      }
    }
    // payload needs depend on the group key
    snprintf(buf, sizeof buf, "g%d,%d,%d,%d", plan.hi_src, plan.hi_index, plan.lo_src, plan.lo_index);
    return s + buf;
  }
};

struct DimEntry {
  DimTables d;
  hipEvent_t ready = nullptr;
  uint32_t *d_err = nullptr;        // error word of the build (arena), read by every request using the tables
  int users = 0;                    // active requests using the tables
  std::vector<const void *> cols;   // device columns the tables were built over
};

struct Request {
  uint64_t id = 0;
  PlanCopy pc;
  int64_t rows = 0;
  int64_t *out_keys = nullptr, *out_sums = nullptr, *d_ngroups = nullptr;
  int64_t out_cap = 0;
  QueryShape q;
  int slot = -1;
  DimEntry *dims = nullptr;
  DimTables d;      // the cached tables with this request's own sums
  AggState s;
  void *sums_mem = nullptr;
  int64_t nchunks = 0, remaining = 0, cursor = 0;
  std::vector<char> done;
  hipEvent_t finish = nullptr;
  std::chrono::steady_clock::time_point t_submit, t_done;
  pyst_status status = PYST_OK;
  bool completed = false;
};

}  // namespace pyst

struct pyst_server {
  pyst_ctx *ctx = nullptr;
  pyst_server_cfg cfg{};
  std::vector<pyst_col> fact;
  std::vector<pyst_packed_col> packed;  // with packed input: the columns' blocks (fact then gives shapes only)
  int64_t fact_rows = 0;
  size_t row_bytes = 0;
  std::vector<hipStream_t> slots;
  std::vector<int> slot_free;
  // ring of chunk buffers
  void *ring = nullptr;
  std::vector<std::vector<char *>> buf;
  std::vector<std::vector<char *>> hdr, wbuf;  // packed blocks of each slot and column
  std::vector<hipEvent_t> copied;
  std::vector<std::vector<hipEvent_t>> users;  // events of the streams that consumed each buffer
  int64_t next_ring = 0;
  // queue and bookkeeping
  std::mutex mu;
  std::condition_variable cv_submit, cv_done;
  std::deque<std::shared_ptr<pyst::Request>> pending;
  std::unordered_map<uint64_t, std::shared_ptr<pyst::Request>> all;
  std::vector<std::shared_ptr<pyst::Request>> active;
  std::map<std::string, std::unique_ptr<pyst::DimEntry>> dim_cache;
  std::vector<std::unique_ptr<pyst::DimEntry>> retired;  // dropped from the cache, freed once unused
  std::vector<const void *> forget_q;                    // pyst_server_forget_tables calls not yet applied
  std::vector<std::pair<int, int64_t>> option_q;         // pyst_server_option calls not yet applied
  uint32_t *d_req_err = nullptr;  // per slot: the running request's error word (arena, 256 B apart)
  uint32_t *h_req_err = nullptr;  // per slot, pinned: [2 s] its tables' word, [2 s + 1] its own word
  uint64_t next_id = 1;
  bool stop = false;
  std::thread thr;
  pyst_server_stats stats{};
};

namespace pyst {

static double ms_between(std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

static uint32_t *req_err_word(pyst_server *sv, int slot) { return sv->d_req_err + static_cast<size_t>(slot) * 64; }

// Kernels launched while one of these lives latch into the given word.
struct ErrScope {
  pyst_ctx *ctx;
  ErrScope(pyst_ctx *c, uint32_t *word) : ctx(c) { ctx_set_err_word(ctx, word); }
  ~ErrScope() { ctx_set_err_word(ctx, nullptr); }
};

static void free_entry(pyst_server *sv, DimEntry &e) {
  if (e.ready) {
    (void)hipEventSynchronize(e.ready);
    (void)hipEventDestroy(e.ready);
    e.ready = nullptr;
  }
  free_dimensions(sv->ctx, &e.d, nullptr);
  if (e.d_err) ctx_free(sv->ctx, e.d_err, nullptr);
  e.d_err = nullptr;
}

// Free the dropped tables that no active request uses any more.
static void free_retired(pyst_server *sv) {
  for (size_t i = 0; i < sv->retired.size();) {
    if (sv->retired[i]->users == 0) {
      free_entry(sv, *sv->retired[i]);
      sv->retired.erase(sv->retired.begin() + static_cast<long>(i));
    } else {
      ++i;
    }
  }
}

// Drop cached tables built over column `col` (nullptr: all) or, with
// idle_only, every table no active request uses.  Returns how many.
static int drop_tables(pyst_server *sv, const void *col, bool idle_only) {
  int n = 0;
  for (auto it = sv->dim_cache.begin(); it != sv->dim_cache.end();) {
    DimEntry &e = *it->second;
    const bool match = idle_only ? e.users == 0
                                 : (col == nullptr || std::find(e.cols.begin(), e.cols.end(), col) != e.cols.end());
    if (match) {
      sv->retired.push_back(std::move(it->second));
      it = sv->dim_cache.erase(it);
      ++n;
    } else {
      ++it;
    }
  }
  free_retired(sv);
  return n;
}

// Apply the forget and option calls made so far (scheduler thread, sv->mu held).
static void apply_client_calls(pyst_server *sv) {
  for (const void *col : sv->forget_q) drop_tables(sv, col, false);
  sv->forget_q.clear();
  for (auto &kv : sv->option_q) (void)pyst_ctx_option(sv->ctx, kv.first, kv.second);
  sv->option_q.clear();
}

// Aggregation-state bytes a request reserves while active (its admission cost).
static size_t request_bytes(const pyst_server *sv, const Request &r) {
  if (r.q.agg_mode == 0)
    return table_capacity_host(r.pc.plan.joins[0].key.n, r.pc.plan.joins[0].max_load) * (sizeof(uint64_t) + 1) + 512;
  const int64_t bound = std::min<int64_t>(r.pc.plan.max_groups, std::max<int64_t>(r.rows, 1));
  (void)sv;
  return group_bytes(table_capacity_host(bound, r.pc.plan.group_max_load)) + 256;
}

// Start a request: dimension tables (cached), own aggregation state, zeroed outputs.
// Build the dimension tables of a plan into a new cache entry, or nullptr
// with *ps set (PYST_ERR_NOMEM when the budget cannot hold them now).
static std::unique_ptr<DimEntry> build_entry(pyst_server *sv, const Request &r, hipStream_t st, pyst_status *ps) {
  auto e = std::make_unique<DimEntry>();
  std::memset(&e->d, 0, sizeof(e->d));
  e->d_err = static_cast<uint32_t *>(ctx_alloc(sv->ctx, 256, st));
  if (!e->d_err) {
    *ps = PYST_ERR_NOMEM;
    return nullptr;
  }
  *ps = fill_u32(e->d_err, 1, 0u, st);
  if (*ps == PYST_OK) {
    ErrScope scope(sv->ctx, e->d_err);
    *ps = fast_build_dimensions(sv->ctx, &r.pc.plan, r.q, &e->d, nullptr, nullptr, st, false, nullptr);
  }
  if (*ps != PYST_OK) {
    free_dimensions(sv->ctx, &e->d, st);
    ctx_free(sv->ctx, e->d_err, st);
    return nullptr;
  }
  for (int j = 0; j < r.pc.plan.njoins; ++j) {
    e->cols.push_back(r.pc.plan.joins[j].key.data);
    if (r.pc.plan.joins[j].payload.data) e->cols.push_back(r.pc.plan.joins[j].payload.data);
    for (const auto &c : r.pc.jcols[j]) e->cols.push_back(c.data);
  }
  (void)hipEventCreateWithFlags(&e->ready, hipEventDisableTiming);
  (void)hipEventRecord(e->ready, st);
  return e;
}

static void *alloc_or_evict(pyst_server *sv, size_t bytes, hipStream_t st) {
  void *p = ctx_alloc(sv->ctx, bytes, st);
  if (!p && drop_tables(sv, nullptr, true) > 0) p = ctx_alloc(sv->ctx, bytes, st);
  return p;
}

static bool admit(pyst_server *sv, const std::shared_ptr<Request> &r) {
  const std::string sig = r->pc.dim_signature();
  auto it = sv->dim_cache.find(sig);
  hipStream_t st = sv->slots[r->slot];
  uint32_t *word = req_err_word(sv, r->slot);
  if (fill_u32(word, 1, 0u, st) != PYST_OK) {
    r->status = PYST_ERR_HIP;
    return true;
  }
  if (it == sv->dim_cache.end()) {
    pyst_status ps = PYST_OK;
    auto e = build_entry(sv, *r, st, &ps);
    // tables that no active request uses give way to a new one that does not fit
    if (!e && ps == PYST_ERR_NOMEM && drop_tables(sv, nullptr, true) > 0) e = build_entry(sv, *r, st, &ps);
    if (!e) {
      if (ps == PYST_ERR_NOMEM) return false;  // retry once memory frees up
      r->status = ps;
      return true;
    }
    it = sv->dim_cache.emplace(sig, std::move(e)).first;
  }
  r->dims = it->second.get();
  r->dims->users++;
  (void)hipStreamWaitEvent(st, r->dims->ready, 0);
  r->d = r->dims->d;
  std::memset(&r->s, 0, sizeof(r->s));
  ErrScope scope(sv->ctx, word);
  if (r->q.agg_mode == 0) {
    const int64_t cap = r->d.t[0].cap_alloc;
    r->sums_mem = alloc_or_evict(sv, static_cast<size_t>(cap) * (sizeof(uint64_t) + 1) + 256, st);
    if (!r->sums_mem) {
      r->dims->users--;
      r->dims = nullptr;
      return false;
    }
    r->d.t[0].sums = static_cast<uint64_t *>(r->sums_mem);
    r->d.t[0].flags = reinterpret_cast<uint8_t *>(r->d.t[0].sums + cap);
    k_req_init<<<static_cast<unsigned>(std::min<int64_t>(ceil_div(cap, 256), 2048)), 256, 0, st>>>(r->d.t[0], r->d_ngroups,
                                                                                          ctx_err_word(sv->ctx));
  } else {
    const int64_t bound = std::min<int64_t>(r->pc.plan.max_groups, std::max<int64_t>(r->rows, 1));
    const int64_t cap = table_capacity_host(bound, r->pc.plan.group_max_load);
    r->s.mem = alloc_or_evict(sv, group_bytes(cap), st);
    if (!r->s.mem) {
      r->dims->users--;
      r->dims = nullptr;
      return false;
    }
    r->s.g = group_view(r->s.mem, cap);
    (void)group_init(r->s.g, nullptr, bound, 0, r->pc.plan.group_max_load, st);
    TableDev t{};
    t.hdr = r->d.t[0].hdr;
    k_req_init<<<1, 64, 0, st>>>(t, r->d_ngroups, ctx_err_word(sv->ctx));
  }
  r->nchunks = ceil_div(r->rows, sv->cfg.chunk_rows);
  r->remaining = r->nchunks;
  r->done.assign(static_cast<size_t>(r->nchunks), 0);
  return true;
}

static void release(pyst_server *sv, Request &r) {
  hipStream_t st = sv->slots[r.slot];
  // an event at once: other slots' requests reuse this memory all the time
  if (r.sums_mem) ctx_free_eager(sv->ctx, r.sums_mem, st);
  if (r.s.mem) ctx_free_eager(sv->ctx, r.s.mem, st);
  r.sums_mem = r.s.mem = nullptr;
  if (r.dims) {
    r.dims->users--;
    r.dims = nullptr;
    free_retired(sv);
  }
  sv->slot_free.push_back(r.slot);
}

// Copy chunk c once and run the fact pass of every active request needing it.
static void serve_chunk(pyst_server *sv, int64_t c) {
  const int b = static_cast<int>(sv->next_ring++ % sv->cfg.nbuf);
  hipStream_t cs = ctx_copy_stream(sv->ctx);
  // Backpressure: wait on the host until the buffer's previous consumers are
  // done, so the scheduler runs at most nbuf chunks ahead of the device and
  // chooses each chunk when it is needed -- requests that arrive meanwhile can
  // still share it.  (Enqueuing ahead would fix every choice at admission.)
  for (hipEvent_t e : sv->users[b]) (void)hipEventSynchronize(e);
  for (hipEvent_t e : sv->users[b]) (void)hipEventDestroy(e);
  sv->users[b].clear();
  const int64_t off = c * sv->cfg.chunk_rows;
  int64_t need = 0;  // rows of this chunk that any active request reads
  for (auto &r : sv->active)
    if (c < r->nchunks && !r->done[c]) need = std::max(need, std::min(sv->cfg.chunk_rows, r->rows - off));
  double bytes = 0;
  {
    TimedRegion timed(sv->ctx, "h2d_chunk", cs);
    for (size_t k = 0; k < sv->fact.size(); ++k) {
      if (sv->packed.empty()) {
        const size_t w = sv->fact[k].dtype == PYST_I64 ? 8 : 4;
        (void)hipMemcpyAsync(sv->buf[b][k], static_cast<const char *>(sv->fact[k].data) + off * w,
                             static_cast<size_t>(need) * w, hipMemcpyHostToDevice, cs);
        bytes += static_cast<double>(need) * w;
      } else if (need > 0) {
        const pyst_packed_col &pc = sv->packed[k];
        const int64_t b0 = off / PYST_PACK_BLOCK, b1 = ceil_div(off + need, PYST_PACK_BLOCK);
        const int64_t w0 = pc.blocks[b0].word_off, w1 = pc.blocks[b1].word_off;
        (void)hipMemcpyAsync(sv->hdr[b][k], pc.blocks + b0, static_cast<size_t>(b1 - b0 + 1) * sizeof(pyst_pack_block),
                             hipMemcpyHostToDevice, cs);
        if (w1 > w0)
          (void)hipMemcpyAsync(sv->wbuf[b][k], pc.words + w0, static_cast<size_t>(w1 - w0) * sizeof(uint32_t),
                               hipMemcpyHostToDevice, cs);
        bytes += static_cast<double>(b1 - b0 + 1) * sizeof(pyst_pack_block) + static_cast<double>(w1 - w0) * 4;
      }
    }
  }
  // packed chunks are decoded into the slot on the copy stream, before the slot is published
  for (size_t k = 0; !sv->packed.empty() && need > 0 && k < sv->fact.size(); ++k) {
    const pyst_packed_col &pc = sv->packed[k];
    const int64_t b0 = off / PYST_PACK_BLOCK, b1 = ceil_div(off + need, PYST_PACK_BLOCK);
    const int64_t w0 = pc.blocks[b0].word_off, w1 = pc.blocks[b1].word_off;
    (void)launch_unpack(sv->ctx, reinterpret_cast<const pyst_pack_block *>(sv->hdr[b][k]),
                        reinterpret_cast<const uint32_t *>(sv->wbuf[b][k]), w1 - w0, w0, need, pc.dtype, sv->buf[b][k],
                        cs);
  }
  (void)hipEventRecord(sv->copied[b], cs);
  sv->stats.chunks_copied++;
  sv->stats.bytes_copied += bytes;
  std::vector<pyst_col> dev(sv->fact);
  for (auto &r : sv->active) {
    if (c >= r->nchunks || r->done[c] || r->status != PYST_OK) continue;
    hipStream_t st = sv->slots[r->slot];
    (void)hipStreamWaitEvent(st, sv->copied[b], 0);
    const int64_t rows = std::min(sv->cfg.chunk_rows, r->rows - off);
    for (size_t k = 0; k < dev.size(); ++k) {
      dev[k].data = sv->buf[b][k];
      dev[k].n = rows;
    }
    FastArgs fa;
    fast_shape(&r->pc.plan, dev.data(), r->q, &fa);
    pyst_status ps;
    {
      ErrScope scope(sv->ctx, req_err_word(sv, r->slot));
      ps = fast_fact_pass(sv->ctx, r->pc.plan.njoins, r->q.agg_mode, fa, r->d, r->s.g, r->s.po, st);
    }
    if (ps != PYST_OK) r->status = ps;  // the request stops here and is finished without its later chunks
    hipEvent_t ev = nullptr;
    (void)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    (void)hipEventRecord(ev, st);
    sv->users[b].push_back(ev);
    r->done[c] = 1;
    r->remaining--;
    sv->stats.fact_rows_processed += static_cast<double>(rows);
  }
}

// A request is finished when every chunk it reads has been through its fact
// pass, or at once when one of its launches failed on the host (its later
// chunks are skipped), so a failed request never holds its slot and memory.
static void finish_ready(pyst_server *sv) {
  for (auto &r : sv->active) {
    if (r->finish || (r->remaining > 0 && r->status == PYST_OK)) continue;
    hipStream_t st = sv->slots[r->slot];
    uint32_t *word = req_err_word(sv, r->slot);
    if (r->status == PYST_OK) {
      ErrScope scope(sv->ctx, word);
      r->status = fast_finish(sv->ctx, &r->pc.plan, r->q, r->d, &r->s, r->out_keys, r->out_sums, r->out_cap,
                              r->d_ngroups, st);
    }
    // the request's error bits: its own word and that of the tables it used
    uint32_t *h = sv->h_req_err + 2 * r->slot;
    h[0] = h[1] = 0;
    if (r->dims) (void)hipMemcpyAsync(h, r->dims->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    (void)hipMemcpyAsync(h + 1, word, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    (void)hipEventCreateWithFlags(&r->finish, hipEventDisableTiming);
    (void)hipEventRecord(r->finish, st);
  }
}

static void reap_done(pyst_server *sv) {
  for (size_t i = 0; i < sv->active.size();) {
    auto r = sv->active[i];
    if (r->finish && hipEventQuery(r->finish) == hipSuccess) {
      (void)hipEventDestroy(r->finish);
      r->finish = nullptr;
      r->t_done = std::chrono::steady_clock::now();
      const uint32_t bits = sv->h_req_err[2 * r->slot] | sv->h_req_err[2 * r->slot + 1];
      if (r->status == PYST_OK && bits) r->status = status_of_error_bits(bits);
      release(sv, *r);
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        r->completed = true;
        sv->stats.completed++;
      }
      sv->cv_done.notify_all();
      sv->active.erase(sv->active.begin() + static_cast<long>(i));
    } else {
      ++i;
    }
  }
}

static void scheduler(pyst_server *sv) {
  (void)hipSetDevice(ctx_device(sv->ctx));
  while (true) {
    // admit while slots and memory allow (FIFO; the head blocks the rest)
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (sv->active.empty() && sv->pending.empty()) {
        apply_client_calls(sv);
        if (sv->stop) break;
        sv->cv_submit.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
      apply_client_calls(sv);
      while (!sv->pending.empty() && !sv->slot_free.empty()) {
        apply_client_calls(sv);  // a forget made before a submit applies before its admission
        auto r = sv->pending.front();
        if (ctx_budget_free(sv->ctx) < request_bytes(sv, *r) && !sv->active.empty() &&
            (drop_tables(sv, nullptr, true) == 0 || ctx_budget_free(sv->ctx) < request_bytes(sv, *r))) {
          sv->stats.admission_waits++;
          break;
        }
        r->slot = sv->slot_free.back();
        sv->slot_free.pop_back();
        lk.unlock();
        const bool ok = admit(sv, r);
        lk.lock();
        if (!ok) {  // out of memory: wait for an active request to finish
          sv->slot_free.push_back(r->slot);
          r->slot = -1;
          if (sv->active.empty()) {  // can never fit
            sv->pending.pop_front();
            r->status = PYST_ERR_NOMEM;
            r->completed = true;
            r->t_done = std::chrono::steady_clock::now();
            sv->cv_done.notify_all();
            continue;
          }
          sv->stats.admission_waits++;
          break;
        }
        sv->pending.pop_front();
        sv->active.push_back(r);
        sv->stats.max_active_seen = std::max<int64_t>(sv->stats.max_active_seen, static_cast<int64_t>(sv->active.size()));
      }
    }
    // Next chunk: among the next chunks of the active requests (each request
    // reads its chunks in order), the one the most active requests still need;
    // ties go to the oldest request.  Every request needing the chunk consumes
    // the same copy, so requests waiting together share their common prefix,
    // and a request alone proceeds as under one-at-a-time service.
    int64_t pick = -1, best = 0;
    for (auto &r : sv->active) {
      if (r->status != PYST_OK) continue;
      while (r->cursor < r->nchunks && r->done[r->cursor]) ++r->cursor;
      if (r->cursor >= r->nchunks) continue;
      const int64_t c = r->cursor;
      int64_t users = 0;
      for (auto &o : sv->active)
        if (o->status == PYST_OK && c < o->nchunks && !o->done[c]) ++users;
      if (users > best) {  // strict: earlier (older) requests win ties
        best = users;
        pick = c;
      }
    }
    if (pick >= 0) serve_chunk(sv, pick);
    finish_ready(sv);
    reap_done(sv);
    if (pick < 0 && !sv->active.empty()) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

}  // namespace pyst

using namespace pyst;

extern "C" {

// host_fact gives the columns (raw input) or their shapes (with `packed`).
static pyst_status server_create(int device, const pyst_server_cfg *cfg, const pyst_col *host_fact, int nfact,
                                 const pyst_packed_col *packed, pyst_server **out) {
  if (!cfg || !host_fact || !out || nfact < 1 || nfact > PYST_MAX_COLS)
    return set_error(PYST_ERR_ARG, "pyst_server_create: bad argument");
  *out = nullptr;
  if (cfg->max_active < 1 || cfg->max_active > 64 || cfg->nbuf < 2 || cfg->nbuf > 8 || cfg->chunk_rows < 4 ||
      cfg->chunk_rows % 4 != 0 || cfg->chunk_rows >= (int64_t{1} << 31))
    return set_error(PYST_ERR_ARG, "pyst_server_create: max_active 1..64, nbuf 2..8, chunk_rows a multiple of 4");
  const int64_t n = host_fact[0].n;
  for (int c = 0; c < nfact; ++c)
    if (host_fact[c].n != n || !(host_fact[c].dtype == PYST_I32 || host_fact[c].dtype == PYST_I64) || !host_fact[c].data)
      return set_error(PYST_ERR_ARG, "pyst_server_create: fact columns must be int32/int64 of equal length");
  // Per slot and column: the decoded chunk, and with packed input its block
  // headers and the most words any chunk of the column has.
  auto round = [](size_t x) { return (x + 255) / 256 * 256; };
  std::vector<size_t> col_bytes(nfact), hdr_bytes(nfact, 0), word_bytes(nfact, 0);
  const int64_t nchunks = ceil_div(n, cfg->chunk_rows);
  for (int c = 0; c < nfact; ++c) {
    col_bytes[c] = round(static_cast<size_t>(cfg->chunk_rows) * (host_fact[c].dtype == PYST_I64 ? 8 : 4));
    if (!packed) continue;
    hdr_bytes[c] = round(static_cast<size_t>(cfg->chunk_rows / PYST_PACK_BLOCK + 1) * sizeof(pyst_pack_block));
    int64_t most = 0;
    for (int64_t ch = 0; ch < nchunks; ++ch) {
      const int64_t b0 = ch * cfg->chunk_rows / PYST_PACK_BLOCK;
      const int64_t b1 = ceil_div(std::min<int64_t>(n, (ch + 1) * cfg->chunk_rows), PYST_PACK_BLOCK);
      most = std::max(most, packed[c].blocks[b1].word_off - packed[c].blocks[b0].word_off);
    }
    word_bytes[c] = round(static_cast<size_t>(most) * sizeof(uint32_t));
  }
  size_t slot_bytes = 0;
  for (int c = 0; c < nfact; ++c) slot_bytes += col_bytes[c] + hdr_bytes[c] + word_bytes[c];
  auto *sv = new pyst_server();
  sv->cfg = *cfg;
  sv->fact.assign(host_fact, host_fact + nfact);
  if (packed) sv->packed.assign(packed, packed + nfact);
  sv->fact_rows = n;
  for (int c = 0; c < nfact; ++c) sv->row_bytes += host_fact[c].dtype == PYST_I64 ? 8 : 4;
  const size_t ring_bytes = static_cast<size_t>(cfg->nbuf) * slot_bytes;
  const size_t word_bytes_all = static_cast<size_t>(cfg->max_active) * 256;
  pyst_status st = pyst_ctx_create(device, cfg->budget_bytes + ring_bytes + word_bytes_all, &sv->ctx);
  if (st != PYST_OK) {
    delete sv;
    return st;
  }
  sv->ring = ctx_alloc(sv->ctx, ring_bytes, nullptr);
  if (!sv->ring) {
    pyst_ctx_destroy(sv->ctx);
    delete sv;
    return set_error(PYST_ERR_NOMEM, "pyst_server_create: chunk ring");
  }
  char *p = static_cast<char *>(sv->ring);
  sv->buf.assign(cfg->nbuf, std::vector<char *>(nfact));
  sv->hdr = sv->buf;
  sv->wbuf = sv->buf;
  sv->copied.assign(cfg->nbuf, nullptr);
  sv->users.assign(cfg->nbuf, {});
  for (int b = 0; b < cfg->nbuf; ++b) {
    (void)hipEventCreateWithFlags(&sv->copied[b], hipEventDisableTiming);
    for (int c = 0; c < nfact; ++c) {
      sv->buf[b][c] = p;
      sv->hdr[b][c] = p + col_bytes[c];
      sv->wbuf[b][c] = p + col_bytes[c] + hdr_bytes[c];
      p += col_bytes[c] + hdr_bytes[c] + word_bytes[c];
    }
  }
  sv->d_req_err = static_cast<uint32_t *>(ctx_alloc(sv->ctx, static_cast<size_t>(cfg->max_active) * 256, nullptr));
  if (!sv->d_req_err ||
      hipHostMalloc(reinterpret_cast<void **>(&sv->h_req_err), static_cast<size_t>(cfg->max_active) * 2 * sizeof(uint32_t),
                    hipHostMallocDefault) != hipSuccess) {
    pyst_ctx_destroy(sv->ctx);
    delete sv;
    return set_error(PYST_ERR_NOMEM, "pyst_server_create: error words");
  }
  sv->slots.resize(cfg->max_active);
  for (int i = 0; i < cfg->max_active; ++i) {
    (void)hipStreamCreateWithFlags(&sv->slots[i], hipStreamNonBlocking);  // default priority
    sv->slot_free.push_back(cfg->max_active - 1 - i);
  }
  sv->thr = std::thread(scheduler, sv);
  *out = sv;
  return PYST_OK;
}

pyst_status pyst_server_create(int device, const pyst_server_cfg *cfg, const pyst_col *host_fact, int nfact,
                               pyst_server **out) {
  return server_create(device, cfg, host_fact, nfact, nullptr, out);
}

pyst_status pyst_server_create_packed(int device, const pyst_server_cfg *cfg, const pyst_packed_col *host_fact,
                                      int nfact, pyst_server **out) {
  if (!cfg || !host_fact || !out || nfact < 1 || nfact > PYST_MAX_COLS)
    return set_error(PYST_ERR_ARG, "pyst_server_create_packed: bad argument");
  if (cfg->chunk_rows < PYST_PACK_BLOCK || cfg->chunk_rows % PYST_PACK_BLOCK != 0)
    return set_error(PYST_ERR_ARG, "pyst_server_create_packed: chunk_rows must be a multiple of 1024");
  std::vector<pyst_col> shape(nfact);
  for (int c = 0; c < nfact; ++c) {
    const pyst_packed_col &pc = host_fact[c];
    if (!(pc.dtype == PYST_I32 || pc.dtype == PYST_I64) || pc.n < 0 || pc.n != host_fact[0].n || !pc.blocks ||
        (pc.n > 0 && !pc.words))
      return set_error(PYST_ERR_ARG, "pyst_server_create_packed: bad packed column");
    if (!pack_blocks_ok(pc.blocks, ceil_div(pc.n, PYST_PACK_BLOCK), pc.dtype))
      return set_error(PYST_ERR_ARG, "pyst_server_create_packed: malformed block table");
    shape[c] = pyst_col{kShapeOnly, pc.n, pc.dtype, 0};  // shape only: the raw copy path is not taken
  }
  return server_create(device, cfg, shape.data(), nfact, host_fact, out);
}

pyst_status pyst_server_submit(pyst_server *sv, const pyst_request *req, uint64_t *ticket) {
  if (!sv || !req || !req->plan || !ticket || !req->d_ngroups || req->rows < 0 || req->rows > sv->fact_rows ||
      req->out_cap < 0 || (req->out_cap > 0 && (!req->out_keys || !req->out_sums)))
    return set_error(PYST_ERR_ARG, "pyst_server_submit: bad request");
  auto r = std::make_shared<Request>();
  r->pc.take(*req->plan);
  r->rows = req->rows;
  r->out_keys = req->out_keys;
  r->out_sums = req->out_sums;
  r->out_cap = req->out_cap;
  r->d_ngroups = req->d_ngroups;
  std::vector<pyst_col> shape(sv->fact);
  for (auto &c : shape) {
    c.n = std::max<int64_t>(req->rows, 0);
    c.data = reinterpret_cast<const void *>(uintptr_t{256});  // any aligned non-null address: shape checks only
  }
  pyst_status st = prepare_query(&r->pc.plan, shape.data(), static_cast<int>(shape.size()), &r->q);
  if (st != PYST_OK) return st;
  FastArgs fa;
  if (!fast_shape(&r->pc.plan, shape.data(), r->q, &fa))
    return set_error(PYST_ERR_UNSUPPORTED, "pyst_server_submit: plan shape cannot be served");
  if (r->q.agg_mode == 2) return set_error(PYST_ERR_UNSUPPORTED, "pyst_server_submit: set plan->max_groups");
  r->t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return set_error(PYST_ERR_ARG, "pyst_server_submit: server is stopping");
    r->id = sv->next_id++;
    sv->all[r->id] = r;
    sv->pending.push_back(r);
    sv->stats.submitted++;
  }
  sv->cv_submit.notify_one();
  *ticket = r->id;
  return PYST_OK;
}

pyst_status pyst_server_wait(pyst_server *sv, uint64_t ticket, double *latency_ms) {
  if (!sv) return set_error(PYST_ERR_ARG, "pyst_server_wait: NULL server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return set_error(PYST_ERR_ARG, "pyst_server_wait: unknown ticket");
  auto r = it->second;
  sv->cv_done.wait(lk, [&] { return r->completed; });
  if (latency_ms) *latency_ms = ms_between(r->t_submit, r->t_done);
  sv->all.erase(it);
  if (r->status != PYST_OK) return set_error(r->status, "pyst_server_wait: request failed");
  return PYST_OK;
}

pyst_status pyst_server_poll(pyst_server *sv, uint64_t ticket, int *done, double *latency_ms) {
  if (!sv || !done) return set_error(PYST_ERR_ARG, "pyst_server_poll: NULL argument");
  *done = 0;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return set_error(PYST_ERR_ARG, "pyst_server_poll: unknown ticket");
  auto r = it->second;
  if (!r->completed) return PYST_OK;
  *done = 1;
  if (latency_ms) *latency_ms = ms_between(r->t_submit, r->t_done);
  sv->all.erase(it);
  if (r->status != PYST_OK) return set_error(r->status, "pyst_server_poll: request failed");
  return PYST_OK;
}

pyst_status pyst_server_get_stats(pyst_server *sv, pyst_server_stats *out) {
  if (!sv || !out) return set_error(PYST_ERR_ARG, "pyst_server_get_stats: NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->stats;
  return PYST_OK;
}

pyst_status pyst_server_forget_tables(pyst_server *sv, const void *dim_col_data) {
  if (!sv) return set_error(PYST_ERR_ARG, "pyst_server_forget_tables: NULL server");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->forget_q.push_back(dim_col_data);
  }
  sv->cv_submit.notify_one();
  return PYST_OK;
}

pyst_status pyst_server_option(pyst_server *sv, int key, int64_t value) {
  if (!sv) return set_error(PYST_ERR_ARG, "pyst_server_option: NULL server");
  if (key != PYST_OPT_GENERIC_ONLY && key != PYST_OPT_GROUPBY_HASH_ONLY && key != PYST_OPT_FAIL_FACT_PASS &&
      key != PYST_OPT_HASH_JOIN_ONLY)
    return set_error(PYST_ERR_ARG, "pyst_server_option: unknown option");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->option_q.emplace_back(key, value);
  }
  sv->cv_submit.notify_one();
  return PYST_OK;
}

pyst_status pyst_server_check(pyst_server *sv) {
  if (!sv) return set_error(PYST_ERR_ARG, "pyst_server_check: NULL server");
  (void)hipDeviceSynchronize();
  return pyst_ctx_check(sv->ctx, nullptr);
}

void pyst_server_destroy(pyst_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_submit.notify_all();
  if (sv->thr.joinable()) sv->thr.join();
  (void)hipDeviceSynchronize();
  for (auto &kv : sv->dim_cache) free_entry(sv, *kv.second);
  for (auto &e : sv->retired) free_entry(sv, *e);
  if (sv->h_req_err) (void)hipHostFree(sv->h_req_err);
  for (auto &u : sv->users)
    for (hipEvent_t e : u) (void)hipEventDestroy(e);
  for (hipEvent_t e : sv->copied) (void)hipEventDestroy(e);
  for (hipStream_t s : sv->slots) (void)hipStreamDestroy(s);
  pyst_ctx_destroy(sv->ctx);
  delete sv;
}

}  // extern "C"

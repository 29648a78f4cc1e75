// Context: device selection, the device-memory arena, and the error latch.
//
// The arena is one hipMalloc of the whole budget made at context creation;
// every table and scratch buffer is carved out of it (first fit, coalescing
// free list).  This is the pooled-allocation remedy for per-operator
// allocation cost (Sec. 3.1, "(2) Runtime Memory Allocation in PyTorch"),
// and the hard budget is what admission control and backpressure account
// against (Sec. 5.4, "Adaptive Regulation").
//
// Frees are stream ordered: a freed block stays pending on the freeing stream.
// That stream may reuse it at once (its later work is ordered after the
// earlier work), and an allocation on a stream first takes back the smallest
// block that stream freed; no event is recorded for this, since each event
// record is a packet of its own in the stream (a query that freed three blocks
// ran 20 us slower per call for them).  Only when another stream needs the
// memory is one event recorded per stream that holds pending blocks; those
// blocks return to the shared free list once it has completed.
#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "pyst_internal.h"

struct pyst_ctx {
  int device = 0;
  int cus = 0;
  char *base = nullptr;
  size_t budget = 0;
  size_t used = 0;
  uint32_t *d_err = nullptr;    // device error word (first 256 B of the arena)
  uint32_t *err_override = nullptr;  // when set, kernels latch here instead (per-request words of the server)
  int64_t fail_pass_countdown = 0;   // test hook: > 0 makes the n-th fact pass from now fail on the host
  uint32_t *h_err = nullptr;    // pinned host copy
  std::map<size_t, size_t> free_blocks;          // offset -> size
  std::unordered_map<size_t, size_t> live;       // offset -> size
  struct Pending {
    size_t off, size;
    hipStream_t stream;
    hipEvent_t ev;  // nullptr until another stream needs the memory
  };
  std::deque<Pending> pending;
  std::vector<hipEvent_t> events;
  // optional per-kernel timing: name -> (start, stop) event pairs of each launch
  bool timing = false;
  bool generic_only = false;  // PYST_OPT_GENERIC_ONLY
  bool groupby_hash_only = false;  // PYST_OPT_GROUPBY_HASH_ONLY
  bool hash_join_only = false;  // PYST_OPT_HASH_JOIN_ONLY
  hipStream_t copy_stream = nullptr;  // host-to-device chunk copies (created on first use)
  char *staging = nullptr;            // pinned host staging for descriptor uploads
  size_t staging_bytes = 0;
  hipEvent_t staging_done = nullptr;  // recorded after the last copy out of `staging`
  std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> timed;
};

namespace pyst {

namespace {
thread_local std::string g_last_error;
constexpr size_t kAlign = 256;

hipEvent_t take_event(pyst_ctx *c) {
  if (!c->events.empty()) {
    hipEvent_t e = c->events.back();
    c->events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

void insert_free(pyst_ctx *c, size_t off, size_t size) {
  auto it = c->free_blocks.emplace(off, size).first;
  auto next = std::next(it);
  if (next != c->free_blocks.end() && it->first + it->second == next->first) {
    it->second += next->second;
    c->free_blocks.erase(next);
  }
  if (it != c->free_blocks.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      c->free_blocks.erase(it);
    }
  }
}

// Pending blocks whose event has completed go back to the free list; an event
// shared by several blocks returns to the event pool with the last of them.
void reap(pyst_ctx *c) {
  std::vector<hipEvent_t> done;
  for (auto it = c->pending.begin(); it != c->pending.end();) {
    if (it->ev && (std::find(done.begin(), done.end(), it->ev) != done.end() || hipEventQuery(it->ev) == hipSuccess)) {
      if (std::find(done.begin(), done.end(), it->ev) == done.end()) done.push_back(it->ev);
      insert_free(c, it->off, it->size);
      it = c->pending.erase(it);
    } else {
      ++it;
    }
  }
  for (hipEvent_t e : done) {
    bool used = false;
    for (const auto &p : c->pending) used = used || p.ev == e;
    if (!used) c->events.push_back(e);
  }
}

// Every pending block back to the free list (the device is idle).
void release_all_pending(pyst_ctx *c) {
  std::vector<hipEvent_t> evs;
  for (const auto &p : c->pending) {
    insert_free(c, p.off, p.size);
    if (p.ev && std::find(evs.begin(), evs.end(), p.ev) == evs.end()) evs.push_back(p.ev);
  }
  c->pending.clear();
  for (hipEvent_t e : evs) c->events.push_back(e);
}

// Record one event on every stream that holds pending blocks without one.
// Returns false when an event could not be recorded (the caller then waits
// for the device instead).
bool mark_pending(pyst_ctx *c) {
  bool ok = true;
  for (auto &p : c->pending) {
    if (p.ev) continue;
    hipEvent_t e = take_event(c);
    if (!e || hipEventRecord(e, p.stream) != hipSuccess) {
      if (e) c->events.push_back(e);
      ok = false;
      continue;
    }
    for (auto &q : c->pending)
      if (!q.ev && q.stream == p.stream) q.ev = e;
  }
  return ok;
}

bool take_first_fit(pyst_ctx *c, size_t bytes, size_t *off) {
  for (auto it = c->free_blocks.begin(); it != c->free_blocks.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t rest_off = it->first + bytes;
      c->free_blocks.erase(it);
      if (rest) c->free_blocks.emplace(rest_off, rest);
      c->live[*off] = bytes;
      return true;
    }
  }
  return false;
}
}  // namespace

pyst_status set_error(pyst_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

pyst_status hip_error(hipError_t e, const char *what) {
  return set_error(PYST_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

void *ctx_alloc(pyst_ctx *c, size_t bytes, hipStream_t stream) {
  bytes = (bytes + kAlign - 1) / kAlign * kAlign;
  if (bytes == 0) bytes = kAlign;
  size_t off = 0;
  while (true) {
    reap(c);
    // The smallest block this stream freed that fits: no wait, no event.
    auto best = c->pending.end();
    for (auto it = c->pending.begin(); it != c->pending.end(); ++it)
      if (it->stream == stream && it->size >= bytes && (best == c->pending.end() || it->size < best->size)) best = it;
    if (best != c->pending.end()) {  // the front part; the rest stays pending on the stream
      off = best->off;
      c->live[off] = bytes;
      if (best->size > bytes) {
        best->off += bytes;
        best->size -= bytes;
      } else {
        const hipEvent_t e = best->ev;
        c->pending.erase(best);
        if (e) {
          bool used = false;
          for (const auto &p : c->pending) used = used || p.ev == e;
          if (!used) c->events.push_back(e);
        }
      }
      break;
    }
    if (take_first_fit(c, bytes, &off)) break;
    if (c->pending.empty()) return nullptr;
    // Backpressure: give every pending block an event, wait for the oldest, retry.
    if (!mark_pending(c)) {  // an event could not be recorded: wait for the whole device
      (void)hipDeviceSynchronize();
      release_all_pending(c);
      continue;
    }
    (void)hipEventSynchronize(c->pending.front().ev);
  }
  c->used += c->live[off];
  return c->base + off;
}

void ctx_free(pyst_ctx *c, void *p, hipStream_t stream) {
  if (!p) return;
  const size_t off = static_cast<size_t>(static_cast<char *>(p) - c->base);
  auto it = c->live.find(off);
  if (it == c->live.end()) return;
  const size_t size = it->second;
  c->live.erase(it);
  c->used -= size;
  c->pending.push_back({off, size, stream, nullptr});
}

void ctx_free_eager(pyst_ctx *c, void *p, hipStream_t stream) {
  if (!p) return;
  ctx_free(c, p, stream);
  hipEvent_t ev = take_event(c);
  if (ev && hipEventRecord(ev, stream) == hipSuccess) {
    c->pending.back().ev = ev;
  } else {
    if (ev) c->events.push_back(ev);
    (void)hipStreamSynchronize(stream);
    const auto blk = c->pending.back();
    c->pending.pop_back();
    insert_free(c, blk.off, blk.size);
  }
}

void ctx_stream_idle(pyst_ctx *c, hipStream_t stream) {
  for (auto it = c->pending.begin(); it != c->pending.end();) {
    if (it->stream == stream && !it->ev) {
      insert_free(c, it->off, it->size);
      it = c->pending.erase(it);
    } else {
      ++it;
    }
  }
}

uint32_t *ctx_err_word(pyst_ctx *c) { return c->err_override ? c->err_override : c->d_err; }
void ctx_set_err_word(pyst_ctx *c, uint32_t *word) { c->err_override = word; }

bool ctx_fail_this_pass(pyst_ctx *c) {
  if (c->fail_pass_countdown <= 0) return false;
  return --c->fail_pass_countdown == 0;
}

pyst_status status_of_error_bits(uint32_t bits) {
  if (bits == 0) return PYST_OK;
  if (bits & kErrKey) return set_error(PYST_ERR_KEY, "a key equal to the reserved EMPTY sentinel was seen");
  if (bits & kErrDup) return set_error(PYST_ERR_DUP_KEY, "duplicate build key under a unique-key promise");
  if (bits & kErrTableFull) return set_error(PYST_ERR_TABLE_FULL, "hash table full");
  if (bits & kErrIndex) return set_error(PYST_ERR_INDEX, "a gather index outside its columns");
  return set_error(PYST_ERR_CAPACITY, "output capacity exceeded");
}
bool ctx_generic_only(const pyst_ctx *c) { return c->generic_only; }
bool ctx_groupby_hash_only(const pyst_ctx *c) { return c->groupby_hash_only; }
bool ctx_hash_join_only(const pyst_ctx *c) { return c->hash_join_only; }

// Bytes not currently allocated (free or pending reuse); an allocation of this
// size may still fail when the space is fragmented.
size_t ctx_budget_free(const pyst_ctx *c) { return c->budget - c->used; }

// Pinned staging area for small host-to-device uploads; waits until the copy
// issued from its previous contents has finished before handing it out again.
char *ctx_pinned_staging(pyst_ctx *c, size_t bytes) {
  if (c->staging_done) (void)hipEventSynchronize(c->staging_done);
  if (bytes > c->staging_bytes) {
    if (c->staging) (void)hipHostFree(c->staging);
    c->staging = nullptr;
    c->staging_bytes = 0;
    const size_t want = std::max<size_t>(bytes, size_t{1} << 20);
    if (hipHostMalloc(reinterpret_cast<void **>(&c->staging), want, hipHostMallocDefault) != hipSuccess) return nullptr;
    c->staging_bytes = want;
  }
  return c->staging;
}

hipError_t ctx_staging_record(pyst_ctx *c, hipStream_t stream) {
  if (!c->staging_done) {
    hipError_t e = hipEventCreateWithFlags(&c->staging_done, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  return hipEventRecord(c->staging_done, stream);
}

hipStream_t ctx_copy_stream(pyst_ctx *c) {
  if (!c->copy_stream &&
      hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking) != hipSuccess)  // default priority
    c->copy_stream = nullptr;
  return c->copy_stream;
}

TimedRegion::TimedRegion(pyst_ctx *c, const char *name, hipStream_t s) : ctx(c), stream(s), label(name) {
  if (!c || !c->timing) return;
  if (hipEventCreate(&start) != hipSuccess || hipEventCreate(&stop) != hipSuccess) return;
  (void)hipEventRecord(start, stream);
}

TimedRegion::~TimedRegion() {
  if (!start || !stop) return;
  (void)hipEventRecord(stop, stream);
  ctx->timed[label].emplace_back(start, stop);
}
int ctx_device(const pyst_ctx *c) { return c->device; }
int ctx_num_cus(const pyst_ctx *c) { return c->cus; }

}  // namespace pyst

using namespace pyst;

extern "C" {

const char *pyst_last_error(void) { return g_last_error.c_str(); }

pyst_status pyst_ctx_create(int device, size_t budget_bytes, pyst_ctx **out) {
  if (!out) return set_error(PYST_ERR_ARG, "pyst_ctx_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_error(e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return set_error(PYST_ERR_ARG, "pyst_ctx_create: no such device");
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_error(e, "hipSetDevice");
  auto *c = new pyst_ctx();
  c->device = device;
  (void)hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device);
  if (c->cus <= 0) c->cus = 256;
  const size_t total = (budget_bytes + kAlign - 1) / kAlign * kAlign + kAlign;
  if ((e = hipMalloc(reinterpret_cast<void **>(&c->base), total)) != hipSuccess) {
    delete c;
    (void)hipGetLastError();
    return set_error(PYST_ERR_NOMEM, std::string("pyst_ctx_create: arena allocation failed: ") + hipGetErrorString(e));
  }
  if ((e = hipHostMalloc(reinterpret_cast<void **>(&c->h_err), sizeof(uint32_t), hipHostMallocDefault)) != hipSuccess) {
    (void)hipFree(c->base);
    delete c;
    return hip_error(e, "hipHostMalloc");
  }
  c->d_err = reinterpret_cast<uint32_t *>(c->base);
  c->base += kAlign;  // block offsets are relative to the first usable byte
  c->budget = total - kAlign;
  c->free_blocks.emplace(0, c->budget);
  pyst_status st = fill_u32(c->d_err, 1, 0u, nullptr);
  if (st == PYST_OK && (e = hipDeviceSynchronize()) != hipSuccess) st = hip_error(e, "hipDeviceSynchronize");
  if (st != PYST_OK) {
    pyst_ctx_destroy(c);
    return st;
  }
  *out = c;
  return PYST_OK;
}

void pyst_ctx_destroy(pyst_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  {
    std::vector<hipEvent_t> evs;
    for (auto &p : c->pending)
      if (p.ev && std::find(evs.begin(), evs.end(), p.ev) == evs.end()) evs.push_back(p.ev);
    for (hipEvent_t e : evs) (void)hipEventDestroy(e);
  }
  for (auto e : c->events) (void)hipEventDestroy(e);
  for (auto &kv : c->timed)
    for (auto &pr : kv.second) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  if (c->copy_stream) (void)hipStreamDestroy(c->copy_stream);
  if (c->staging_done) (void)hipEventDestroy(c->staging_done);
  if (c->staging) (void)hipHostFree(c->staging);
  if (c->base) (void)hipFree(c->base - kAlign);
  if (c->h_err) (void)hipHostFree(c->h_err);
  delete c;
}

size_t pyst_ctx_used(const pyst_ctx *c) { return c ? c->used : 0; }

pyst_status pyst_ctx_option(pyst_ctx *c, int key, int64_t value) {
  if (!c) return set_error(PYST_ERR_ARG, "pyst_ctx_option: ctx is NULL");
  switch (key) {
    case PYST_OPT_GENERIC_ONLY: c->generic_only = value != 0; return PYST_OK;
    case PYST_OPT_GROUPBY_HASH_ONLY: c->groupby_hash_only = value != 0; return PYST_OK;
    case PYST_OPT_HASH_JOIN_ONLY: c->hash_join_only = value != 0; return PYST_OK;
    case PYST_OPT_FAIL_FACT_PASS: c->fail_pass_countdown = value > 0 ? value : 0; return PYST_OK;
  }
  return set_error(PYST_ERR_ARG, "pyst_ctx_option: unknown option");
}

pyst_status pyst_ctx_timing(pyst_ctx *c, int enable) {
  if (!c) return set_error(PYST_ERR_ARG, "pyst_ctx_timing: ctx is NULL");
  c->timing = enable != 0;
  return PYST_OK;
}

pyst_status pyst_ctx_kernel_time(pyst_ctx *c, const char *name, double *total_ms, int64_t *launches) {
  if (!c || !name || !total_ms || !launches) return set_error(PYST_ERR_ARG, "pyst_ctx_kernel_time: NULL argument");
  *total_ms = 0.0;
  *launches = 0;
  auto it = c->timed.find(name);
  if (it == c->timed.end()) return PYST_OK;
  for (auto &pr : it->second) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(pr.second);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess) return hip_error(e, "hipEventElapsedTime");
    *total_ms += ms;
    ++*launches;
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  c->timed.erase(it);
  return PYST_OK;
}
size_t pyst_ctx_budget(const pyst_ctx *c) { return c ? c->budget : 0; }

pyst_status pyst_device_hbm(int device, int64_t *mem_clock_khz, int32_t *bus_bits, double *peak_gbs) {
  if (!mem_clock_khz || !bus_bits || !peak_gbs) return set_error(PYST_ERR_ARG, "pyst_device_hbm: NULL argument");
  int clock = 0, bits = 0;
  hipError_t e = hipDeviceGetAttribute(&clock, hipDeviceAttributeMemoryClockRate, device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&bits, hipDeviceAttributeMemoryBusWidth, device);
  if (e != hipSuccess) return hip_error(e, "pyst_device_hbm");
  *mem_clock_khz = clock;
  *bus_bits = bits;
  // HBM3 / HBM3E move 4 transfers a pin per reported memory clock (2.0 GHz -> 8 Gb/s on this device)
  *peak_gbs = 4.0 * static_cast<double>(clock) * 1e3 * (static_cast<double>(bits) / 8.0) / 1e9;
  return PYST_OK;
}

pyst_status pyst_ctx_check(pyst_ctx *c, hipStream_t stream) {
  if (!c) return set_error(PYST_ERR_ARG, "pyst_ctx_check: ctx is NULL");
  hipError_t e = hipMemcpyAsync(c->h_err, c->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync(error word)");
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  ctx_stream_idle(c, stream);  // what was freed on it is free for every stream now
  const uint32_t bits = *c->h_err;
  if (bits == 0) return PYST_OK;
  pyst_status st = fill_u32(c->d_err, 1, 0u, stream);
  if (st != PYST_OK) return st;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_error(e, "hipStreamSynchronize");
  return status_of_error_bits(bits);
}

}  // extern "C"

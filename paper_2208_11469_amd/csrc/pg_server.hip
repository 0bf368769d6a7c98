// Serving engine: resident sketches, vertex-pair queries, continuous batching.
//
// The memory budget is a staging arena of pinned, coherent host memory, 16
// bytes per pair slot (two IDs and the answer). Submit checks a request on the
// calling thread, reserves a contiguous range of pair slots (best fit within
// one part of the arena; no range free = not admitted now) and writes the
// pairs there itself. An engine
// thread keeps up to K batches in flight, one stream each (default priority):
// whenever a batch slot is free and requests wait, it forms one launch from as
// many of them as fit (a segment table tells each pair its request's sketch
// set, estimator, operation and arena range) and one fused kernel reads the
// pairs from the arena over the bus and writes every answer back into the
// request's range. The engine neither packs nor copies pairs: per request it
// only adds a segment, and it marks a batch's requests finished when the
// batch's event completes, so requests that arrived meanwhile start in the next
// launch. The thread that collects a request (wait, or the poll that first
// sees it finished) copies its answers into the request's output buffer and
// returns the range to the arena.
//
// Synchronisation is split so that client threads rarely meet: submitted
// requests reach the engine through a lock-free stack that it empties in one
// exchange (the engine's queue is its own); the arena (split into parts,
// each under a spinning lock), the ticket table (sharded), the
// finished/collected states and the engine's sleep each have their own lock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pg_device.h"
#include "pg_internal.h"
#include "pg_pair.h"

namespace pg {
namespace {

constexpr int kMaxSegments = 1024;  // requests per batch
constexpr int kEstSlots = 8;        // view slots per sketch set, indexed by estimator id
// Segment tables this small travel as kernel arguments (16 bytes each, 2 KiB):
// larger ones need a copy in front of the kernel on the slot's stream.
constexpr int kArgSegments = 128;
// While a batch is on the device, the next one starts only once the queue
// holds this many pairs (at most half a batch) or its oldest request has
// waited this long: each launch costs the engine thread a few microseconds,
// so under load requests gather into fewer, larger batches, and with the GPU
// idle a request starts at once.
constexpr int64_t kBusyBatchPairs = 1 << 18;
constexpr int64_t kMaxQueueWaitNs = 50000;

// Test-and-test-and-set lock for the arena's short critical sections (a few
// ordered-map operations). Under contention a blocking mutex hands over
// through sleeping threads, several microseconds per hand-over, and the
// submitting and collecting threads formed a convoy on it.
class SpinLock {
 public:
  void lock() {
    for (;;) {
      if (!f_.exchange(true, std::memory_order_acquire)) return;
      while (f_.load(std::memory_order_relaxed)) __builtin_ia32_pause();
    }
  }
  void unlock() { f_.store(false, std::memory_order_release); }

 private:
  std::atomic<bool> f_{false};
};

// One part of the staging arena: its free ranges, indexed by first slot (to
// merge neighbours) and by length (best fit), under its own lock.
struct alignas(64) ArenaPart {
  SpinLock mu;
  std::map<int64_t, int64_t> by_start;           // first slot -> length, disjoint and not adjacent
  std::set<std::pair<int64_t, int64_t>> by_len;  // (length, first slot) of the same ranges
};
// The arena has at most this many parts, each of at least four requests of
// the largest size.
constexpr int64_t kArenaParts = 16;

struct SegDesc {
  int64_t arena;  // first pair slot of its request in the arena
  int32_t begin;  // first pair of the segment in the batch (batches hold at most 2^30 pairs)
  int16_t view;   // index into the server's views (sketch * kEstSlots + estimator, below 512)
  int16_t op;     // PG_OP_CN or PG_OP_JACCARD
};
static_assert(sizeof(SegDesc) == 16, "segment descriptors are 16 bytes");

struct SegArgs {
  int32_t nseg;
  SegDesc seg[kArgSegments];  // used when nseg <= kArgSegments
};

// One lane per pair of the batch; its segment is found by binary search over
// the segment starts held in LDS. `au`, `av` and `out` are the arena (pinned
// host memory). A common-neighbour answer is the FP64 estimate in the pair's
// slot; a Jaccard answer is FP32, stored densely from the start of the
// request's range (its output buffer is float[npairs]).
__global__ __launch_bounds__(256) void k_serve_batch(const SkView* __restrict__ views, SegArgs a,
                                                     const SegDesc* __restrict__ big, const int32_t* __restrict__ au,
                                                     const int32_t* __restrict__ av, double* __restrict__ out,
                                                     int64_t total) {
  __shared__ SegDesc table[kMaxSegments];
  const int32_t nseg = a.nseg;
  const SegDesc* segs = nseg <= kArgSegments ? a.seg : big;
  for (int i = threadIdx.x; i < nseg; i += blockDim.x) table[i] = segs[i];
  __syncthreads();
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = nseg;  // last segment with begin <= e
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (table[mid].begin <= e)
        lo = mid;
      else
        hi = mid;
    }
    const SegDesc sd = table[lo];
    const SkView& s = views[sd.view];
    const int64_t j = e - sd.begin;
    const int64_t slot = sd.arena + j;
    const int32_t u = au[slot], v = av[slot];
    uint32_t raw;
    const double est = eval_pair_any(s, u, v, raw);
    if (sd.op == PG_OP_CN)
      out[slot] = est;
    else
      reinterpret_cast<float*>(out + sd.arena)[j] = (float)jaccard_of(est, s.deg[u], s.deg[v]);
  }
}

using Clock = std::chrono::steady_clock;
inline int64_t to_ns(Clock::time_point t) {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(t.time_since_epoch()).count();
}

enum State { kQueued = 0, kFinished = 1, kCollecting = 2, kCollected = 3 };

struct Request {
  uint64_t ticket = 0;
  int32_t op = 0, view = 0;
  int64_t npairs = 0;
  int64_t arena = 0;  // first pair slot
  void* out = nullptr;
  Clock::time_point t_submit, t_collected;
  std::atomic<int> state{kQueued};
  Request* next = nullptr;  // link in the submission stack
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;
  SegDesc* h_seg = nullptr;  // segment tables larger than kArgSegments, staged for d_seg
  SegDesc* d_seg = nullptr;
  std::vector<Request*> reqs;
  bool busy = false;
};

constexpr int kShards = 16;  // ticket table shards
struct TicketShard {
  std::mutex mu;
  std::unordered_map<uint64_t, Request*> map;
};

}  // namespace
}  // namespace pg

struct pg_server {
  pg_ctx* ctx = nullptr;
  const pg_graph* g = nullptr;
  std::vector<pg_sketches*> sketches;
  pg::SkView* d_views = nullptr;
  std::vector<bool> view_ok;
  pg_server_params p{};
  // staging arena: cap pair slots of pinned, coherent host memory
  int64_t cap = 0;
  int32_t* a_u = nullptr;
  int32_t* a_v = nullptr;
  double* a_out = nullptr;
  // Its free ranges are split into parts, each under its own lock: a
  // submitting thread takes from its home part first and a range returns to
  // the part that holds it, so threads seldom meet on a lock. One allocator
  // for all threads spent 1-2 us per operation in cache misses on its tree
  // nodes and 4-9 us waiting for its lock.
  std::vector<std::unique_ptr<pg::ArenaPart>> parts;
  int64_t part_len = 0;  // slots per part; the last part also holds the remainder
  std::atomic<pg::Request*> inbox{nullptr};  // submitted requests the engine has not taken yet (a stack)
  std::mutex work_mu;                        // the engine's sleep
  std::condition_variable work_cv;
  std::atomic<bool> engine_sleeping{false};
  std::mutex done_mu;                 // state changes waiters wait for
  std::condition_variable done_cv;    // a request finished (its answers are in the arena)
  std::condition_variable taken_cv;   // a request was collected
  pg::TicketShard tickets[pg::kShards];
  std::atomic<uint64_t> next_ticket{1};
  std::vector<pg::Slot> slots;
  std::thread engine;
  std::atomic<bool> stop{false};
  std::atomic<int> engine_error{PG_OK};
  std::mutex err_mu;
  std::string engine_msg;
  std::atomic<uint64_t> st_submitted{0}, st_rejected_busy{0}, st_rejected_invalid{0}, st_completed{0},
      st_batches{0}, st_pairs{0}, st_max_in_flight{0},
      st_max_batch_requests{0};
};

namespace pg {
namespace {

constexpr uint64_t kBytesPerPair = 16;

void add_free(ArenaPart& a, int64_t at, int64_t len) {
  a.by_start.emplace(at, len);
  a.by_len.emplace(len, at);
}

// Best-fit range of `len` free slots in part `a` (the shortest free range
// that holds them, lowest first slot among equals), O(log ranges); -1 if
// none. (A linear first-fit scan grew slow once small holes gathered at the
// front.) Caller holds a.mu.
int64_t part_take(ArenaPart& a, int64_t len) {
  auto it = a.by_len.lower_bound({len, INT64_MIN});
  if (it == a.by_len.end()) return -1;
  const int64_t have = it->first, at = it->second;
  a.by_len.erase(it);
  a.by_start.erase(at);
  if (have > len) add_free(a, at + len, have - len);
  return at;
}

// Return [at, at + len) to part `a`, merging with free neighbours. Caller holds a.mu.
void part_give(ArenaPart& a, int64_t at, int64_t len) {
  auto next = a.by_start.lower_bound(at);
  if (next != a.by_start.end() && next->first == at + len) {
    len += next->second;
    a.by_len.erase({next->second, next->first});
    next = a.by_start.erase(next);
  }
  if (next != a.by_start.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == at) {
      at = prev->first;
      len += prev->second;
      a.by_len.erase({prev->second, prev->first});
      a.by_start.erase(prev);
    }
  }
  add_free(a, at, len);
}

std::atomic<uint32_t> g_next_home{0};

// A range of `len` slots: from the calling thread's home part, else from the
// next part that has one; -1 if no part has a free range that long.
int64_t arena_take(pg_server* srv, int64_t len) {
  thread_local uint32_t home = g_next_home.fetch_add(1, std::memory_order_relaxed);
  const size_t P = srv->parts.size();
  for (size_t k = 0; k < P; ++k) {
    ArenaPart& a = *srv->parts[(home + k) % P];
    std::lock_guard<SpinLock> lk(a.mu);
    const int64_t at = part_take(a, len);
    if (at >= 0) return at;
  }
  return -1;
}

void arena_give(pg_server* srv, int64_t at, int64_t len) {
  const int64_t p = std::min<int64_t>(at / srv->part_len, (int64_t)srv->parts.size() - 1);
  ArenaPart& a = *srv->parts[(size_t)p];
  std::lock_guard<SpinLock> lk(a.mu);
  part_give(a, at, len);
}

TicketShard& shard_of(pg_server* srv, uint64_t ticket) { return srv->tickets[ticket % kShards]; }

void set_engine_error(pg_server* srv, int code, const std::string& msg) {
  std::lock_guard<std::mutex> lk(srv->err_mu);
  if (srv->engine_error.load() == PG_OK) {
    srv->engine_msg = msg;
    srv->engine_error.store(code);
  }
}

int engine_failure(pg_server* srv) {
  std::lock_guard<std::mutex> lk(srv->err_mu);
  return fail(srv->engine_error.load(), srv->engine_msg);
}

int slot_init(Slot& sl) {
  PG_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
  PG_HIP(hipEventCreateWithFlags(&sl.event, hipEventDisableTiming));
  PG_HIP(hipHostMalloc((void**)&sl.h_seg, sizeof(SegDesc) * kMaxSegments, hipHostMallocDefault));
  PG_TRY(palloc((void**)&sl.d_seg, sizeof(SegDesc) * kMaxSegments));
  return PG_OK;
}

void slot_free(Slot& sl) {
  if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  if (sl.h_seg) (void)hipHostFree(sl.h_seg);
  pfree(sl.d_seg);
  if (sl.event) (void)hipEventDestroy(sl.event);
  if (sl.stream) (void)hipStreamDestroy(sl.stream);
  sl = Slot();
}

// Enqueue the batch of the slot's requests: segment table (as kernel
// arguments, or one small copy when it is larger), the kernel and the event.
int launch_batch(pg_server* srv, Slot& sl) {
  int64_t total = 0;
  SegArgs a{};
  a.nseg = (int32_t)sl.reqs.size();
  int32_t i = 0;
  for (Request* r : sl.reqs) {
    const SegDesc sd{r->arena, (int32_t)total, (int16_t)r->view, (int16_t)r->op};
    if (a.nseg > kArgSegments)
      sl.h_seg[i] = sd;
    else
      a.seg[i] = sd;
    ++i;
    total += r->npairs;
  }
  if (a.nseg > kArgSegments)
    PG_HIP(hipMemcpyAsync(sl.d_seg, sl.h_seg, sizeof(SegDesc) * a.nseg, hipMemcpyHostToDevice, sl.stream));
  const unsigned grid = grid_for(total, 256, 16384);
  hipLaunchKernelGGL(k_serve_batch, dim3(grid), dim3(256), 0, sl.stream, (const SkView*)srv->d_views, a,
                     (const SegDesc*)sl.d_seg, (const int32_t*)srv->a_u, (const int32_t*)srv->a_v, srv->a_out, total);
  PG_LAUNCH_CHECK();
  PG_HIP(hipEventRecord(sl.event, sl.stream));
  return PG_OK;
}

void engine_loop(pg_server* srv) {
  (void)hipSetDevice(srv->ctx->device);
  std::deque<Request*> queue;  // the engine's own: submission order
  int64_t queued_pairs = 0;
  std::vector<Request*> taken;
  std::vector<Slot*> done;
  std::vector<hipError_t> done_status;
  const int64_t min_pairs = std::min<int64_t>(kBusyBatchPairs, srv->p.max_batch_pairs / 2);
  for (;;) {
    // new submissions: the stack holds them newest first
    if (Request* list = srv->inbox.exchange(nullptr, std::memory_order_acq_rel)) {
      taken.clear();
      for (Request* r = list; r; r = r->next) taken.push_back(r);
      for (auto it = taken.rbegin(); it != taken.rend(); ++it) {
        queue.push_back(*it);
        queued_pairs += (*it)->npairs;
      }
    }
    // batches on the device
    done.clear();
    done_status.clear();
    int inflight = 0;
    for (Slot& sl : srv->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.event);
      if (q == hipErrorNotReady) {
        ++inflight;
        continue;
      }
      done.push_back(&sl);
      done_status.push_back(q);
    }
    if (!done.empty()) {  // retire: their answers are in the arena
      {
        std::lock_guard<std::mutex> lk(srv->done_mu);
        for (size_t i = 0; i < done.size(); ++i) {
          if (done_status[i] != hipSuccess)
            set_engine_error(srv, PG_E_DEVICE, std::string("serving batch: ") + hipGetErrorString(done_status[i]));
          for (Request* r : done[i]->reqs) r->state.store(kFinished, std::memory_order_release);
          done[i]->reqs.clear();
          done[i]->busy = false;
        }
      }
      srv->done_cv.notify_all();
    }
    // start batches on free slots: at once when the GPU is idle; while batches
    // run, once the queue is large or old enough
    bool launched = false;
    for (Slot& sl : srv->slots) {
      if (sl.busy || queue.empty()) continue;
      const bool ready = inflight == 0 || queued_pairs >= min_pairs ||
                         to_ns(Clock::now()) - to_ns(queue.front()->t_submit) >= kMaxQueueWaitNs;
      if (!ready) break;
      int64_t total = 0;
      while (!queue.empty() && (int)sl.reqs.size() < kMaxSegments &&
             total + queue.front()->npairs <= srv->p.max_batch_pairs) {
        Request* r = queue.front();
        queue.pop_front();
        total += r->npairs;
        sl.reqs.push_back(r);
      }
      queued_pairs -= total;
      if (sl.reqs.size() > srv->st_max_batch_requests.load(std::memory_order_relaxed))
        srv->st_max_batch_requests.store(sl.reqs.size(), std::memory_order_relaxed);  // only this thread writes it
      sl.busy = true;
      ++inflight;
      launched = true;
      srv->st_batches.fetch_add(1, std::memory_order_relaxed);
      const int rc = launch_batch(srv, sl);
      if (rc != PG_OK) set_engine_error(srv, rc, pg_last_error());
    }
    uint64_t seen = srv->st_max_in_flight.load(std::memory_order_relaxed);
    while ((uint64_t)inflight > seen &&
           !srv->st_max_in_flight.compare_exchange_weak(seen, (uint64_t)inflight, std::memory_order_relaxed)) {
    }
    if (!done.empty() || launched) continue;
    if (inflight > 0 || !queue.empty()) {  // a batch is on the device, or the queue waits to grow
      std::this_thread::yield();
      continue;
    }
    // idle: sleep until a submission or the stop
    std::unique_lock<std::mutex> lk(srv->work_mu);
    if (srv->stop.load() && srv->inbox.load() == nullptr) break;
    srv->engine_sleeping.store(true);
    srv->work_cv.wait(lk, [&] { return srv->stop.load() || srv->inbox.load() != nullptr; });
    srv->engine_sleeping.store(false);
  }
}

// Copy a finished request's answers from the arena into its output buffer and
// return its range. The caller moved r from kFinished to kCollecting; the
// range belongs to r alone until it is returned.
void collect(pg_server* srv, Request* r) {
  if (r->op == PG_OP_CN)
    std::memcpy(r->out, srv->a_out + r->arena, sizeof(double) * (size_t)r->npairs);
  else
    std::memcpy(r->out, srv->a_out + r->arena, sizeof(float) * (size_t)r->npairs);
  arena_give(srv, r->arena, r->npairs);
  srv->st_completed.fetch_add(1, std::memory_order_relaxed);
  srv->st_pairs.fetch_add((uint64_t)r->npairs, std::memory_order_relaxed);
  {
    std::lock_guard<std::mutex> lk(srv->done_mu);
    r->t_collected = Clock::now();
    r->state.store(kCollected, std::memory_order_release);
  }
  srv->taken_cv.notify_all();
}

// Collect r if it is finished and no other thread does, else wait until
// whoever collects it is done (state kCollected). `wait_finish`: also wait
// for the batch to finish first.
void collect_or_wait(pg_server* srv, Request* r, bool wait_finish) {
  if (wait_finish && r->state.load(std::memory_order_acquire) == kQueued) {
    std::unique_lock<std::mutex> lk(srv->done_mu);
    srv->done_cv.wait(lk, [&] { return r->state.load(std::memory_order_acquire) != kQueued; });
  }
  int expected = kFinished;
  if (r->state.compare_exchange_strong(expected, kCollecting, std::memory_order_acq_rel)) {
    collect(srv, r);
  } else if (expected == kCollecting) {
    std::unique_lock<std::mutex> lk(srv->done_mu);
    srv->taken_cv.wait(lk, [&] { return r->state.load(std::memory_order_acquire) == kCollected; });
  }
}

}  // namespace
}  // namespace pg

using namespace pg;

extern "C" {

int pg_server_create(pg_ctx* ctx, const pg_graph* g, pg_sketches* const* sketches, int32_t nsketches,
                     const pg_server_params* params, pg_server** out) {
  clear_error();
  if (!ctx || !g || !out || (nsketches > 0 && !sketches)) return fail(PG_E_INVALID, "NULL argument");
  *out = nullptr;
  if (nsketches < 1 || nsketches > 64) return fail(PG_E_INVALID, "nsketches must be in [1, 64]");
  for (int i = 0; i < nsketches; ++i) {
    if (!sketches[i] || sketches[i]->g != g) return fail(PG_E_INVALID, "every sketch set must be built on the graph");
    if (sketches[i]->oriented)
      return fail(PG_E_UNSUPPORTED, "servers answer queries on N_v; an oriented sketch set sketches N+_v");
  }
  pg_server_params p{};
  if (params) p = *params;
  if (p.max_batches_in_flight <= 0) p.max_batches_in_flight = 3;
  if (p.max_pairs_per_request <= 0) p.max_pairs_per_request = 65536;
  if (p.max_batch_pairs <= 0) p.max_batch_pairs = 1 << 20;
  if (p.memory_budget_bytes == 0) p.memory_budget_bytes = 256ull << 20;
  p.max_batches_in_flight = std::min(p.max_batches_in_flight, 16);
  p.max_batch_pairs = std::min<int64_t>(std::max<int64_t>(p.max_batch_pairs, p.max_pairs_per_request), 1 << 30);
  if (p.memory_budget_bytes < kBytesPerPair) return fail(PG_E_INVALID, "memory_budget_bytes below one pair (16 bytes)");
  PG_HIP(hipSetDevice(ctx->device));
  pg_server* srv = new (std::nothrow) pg_server();
  if (!srv) return fail(PG_E_NOMEM, "host allocation failed");
  srv->ctx = ctx;
  srv->g = g;
  srv->sketches.assign(sketches, sketches + nsketches);
  srv->p = p;
  // one view per (sketch set, estimator); Bloom-filter views read the set's own tables
  std::vector<SkView> views((size_t)nsketches * kEstSlots);
  srv->view_ok.assign(views.size(), false);
  for (int i = 0; i < nsketches; ++i) {
    pg_sketches* sk = srv->sketches[i];
    for (int est = 1; est < kEstSlots; ++est) {
      if (check_estimator(sk, est) != PG_OK) continue;
      views[(size_t)i * kEstSlots + est] = make_view(sk, est);
      srv->view_ok[(size_t)i * kEstSlots + est] = true;
    }
  }
  clear_error();
  int rc = palloc((void**)&srv->d_views, sizeof(SkView) * views.size());
  if (rc == PG_OK) {
    hipError_t e = hipMemcpy(srv->d_views, views.data(), sizeof(SkView) * views.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = fail(PG_E_DEVICE, std::string("server views: ") + hipGetErrorString(e));
  }
  srv->cap = (int64_t)(p.memory_budget_bytes / kBytesPerPair);
  if (rc == PG_OK) {
    hipError_t e = hipHostMalloc((void**)&srv->a_u, sizeof(int32_t) * srv->cap, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void**)&srv->a_v, sizeof(int32_t) * srv->cap, hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostMalloc((void**)&srv->a_out, sizeof(double) * srv->cap, hipHostMallocCoherent);
    if (e != hipSuccess) rc = fail(PG_E_NOMEM, std::string("pinned staging arena: ") + hipGetErrorString(e));
  }
  if (rc == PG_OK) {
    // touch every page once now: the first CPU access to a page of this
    // mapping faults it in (about 10 us per 48 KB request range otherwise)
    std::memset(srv->a_u, 0, sizeof(int32_t) * srv->cap);
    std::memset(srv->a_v, 0, sizeof(int32_t) * srv->cap);
    std::memset(srv->a_out, 0, sizeof(double) * srv->cap);
  }
  {
    const int64_t P = std::max<int64_t>(
        1, std::min<int64_t>(kArenaParts, srv->cap / (4 * (int64_t)p.max_pairs_per_request)));
    srv->part_len = srv->cap / P;
    for (int64_t i = 0; i < P && rc == PG_OK; ++i) {
      ArenaPart* part = new (std::nothrow) ArenaPart();
      if (!part) {
        rc = fail(PG_E_NOMEM, "host allocation failed");
        break;
      }
      srv->parts.emplace_back(part);
      const int64_t b = i * srv->part_len, e = i == P - 1 ? srv->cap : b + srv->part_len;
      add_free(*part, b, e - b);
    }
  }
  srv->slots.resize((size_t)p.max_batches_in_flight);
  for (Slot& sl : srv->slots)
    if (rc == PG_OK) rc = slot_init(sl);
  if (rc != PG_OK) {
    for (Slot& sl : srv->slots) slot_free(sl);
    if (srv->a_u) (void)hipHostFree(srv->a_u);
    if (srv->a_v) (void)hipHostFree(srv->a_v);
    if (srv->a_out) (void)hipHostFree(srv->a_out);
    pfree(srv->d_views);
    delete srv;
    return rc;
  }
  srv->engine = std::thread(engine_loop, srv);
  *out = srv;
  return PG_OK;
}

int pg_server_submit(pg_server* srv, const pg_request* req, uint64_t* ticket) {
  clear_error();
  if (!srv || !req || !ticket) return fail(PG_E_INVALID, "NULL argument");
  auto invalid = [&](const char* why) {
    srv->st_rejected_invalid.fetch_add(1, std::memory_order_relaxed);
    return fail(PG_E_INVALID, why);
  };
  if (req->op != PG_OP_CN && req->op != PG_OP_JACCARD) return invalid("unknown op");
  if (req->sketch < 0 || req->sketch >= (int32_t)srv->sketches.size()) return invalid("sketch index out of range");
  if (req->estimator < 1 || req->estimator >= kEstSlots ||
      !srv->view_ok[(size_t)req->sketch * kEstSlots + req->estimator])
    return invalid("estimator does not match the sketch kind");
  if (req->npairs < 1 || req->npairs > srv->p.max_pairs_per_request) return invalid("npairs out of range");
  if (req->npairs > srv->cap) return invalid("request larger than the memory budget (16 bytes per pair)");
  if (!req->u || !req->v || !req->out) return invalid("NULL pair or output array");
  const uint32_t n = (uint32_t)srv->g->n;
  const int64_t L = req->npairs;
  uint32_t bad = 0;
  for (int64_t i = 0; i < L; ++i) bad |= (uint32_t)((uint32_t)req->u[i] >= n) | (uint32_t)((uint32_t)req->v[i] >= n);
  if (bad) return invalid("vertex ID out of range");
  if (srv->stop.load()) return fail(PG_E_INVALID, "server is stopping");
  if (srv->engine_error.load() != PG_OK) return engine_failure(srv);
  Request* r = new (std::nothrow) Request();
  if (!r) return fail(PG_E_NOMEM, "host allocation failed");
  r->arena = arena_take(srv, L);
  if (r->arena < 0) {
    srv->st_rejected_busy.fetch_add(1, std::memory_order_relaxed);
    delete r;
    return fail(PG_E_BUSY, "not admitted: no free range of the memory budget");
  }
  // the range is this request's alone: write its pairs without a lock
  std::memcpy(srv->a_u + r->arena, req->u, sizeof(int32_t) * (size_t)L);
  std::memcpy(srv->a_v + r->arena, req->v, sizeof(int32_t) * (size_t)L);
  r->op = req->op;
  r->view = req->sketch * kEstSlots + req->estimator;
  r->npairs = L;
  r->out = req->out;
  r->t_submit = Clock::now();
  r->ticket = srv->next_ticket.fetch_add(1, std::memory_order_relaxed);
  {
    TicketShard& sh = shard_of(srv, r->ticket);
    std::lock_guard<std::mutex> lk(sh.mu);
    sh.map[r->ticket] = r;
  }
  *ticket = r->ticket;
  srv->st_submitted.fetch_add(1, std::memory_order_relaxed);
  // hand it to the engine, waking it if it sleeps
  Request* head = srv->inbox.load(std::memory_order_relaxed);
  do {
    r->next = head;
  } while (!srv->inbox.compare_exchange_weak(head, r, std::memory_order_seq_cst));
  if (srv->engine_sleeping.load()) {
    std::lock_guard<std::mutex> lk(srv->work_mu);
    srv->work_cv.notify_one();
  }
  return PG_OK;
}

int pg_server_poll(pg_server* srv, uint64_t ticket, int32_t* done) {
  clear_error();
  if (!srv || !done) return fail(PG_E_INVALID, "NULL argument");
  TicketShard& sh = shard_of(srv, ticket);
  std::lock_guard<std::mutex> lk(sh.mu);  // held so that a wait on the same ticket cannot free it meanwhile
  auto it = sh.map.find(ticket);
  if (it == sh.map.end()) return fail(PG_E_INVALID, "unknown ticket");
  Request* r = it->second;
  if (r->state.load(std::memory_order_acquire) != kQueued) collect_or_wait(srv, r, false);
  *done = r->state.load(std::memory_order_acquire) == kCollected ? 1 : 0;
  if (srv->engine_error.load() != PG_OK) return engine_failure(srv);
  return PG_OK;
}

int pg_server_wait(pg_server* srv, uint64_t ticket, double* latency_ms) {
  clear_error();
  if (!srv) return fail(PG_E_INVALID, "NULL argument");
  Request* r = nullptr;
  {
    TicketShard& sh = shard_of(srv, ticket);
    std::lock_guard<std::mutex> lk(sh.mu);
    auto it = sh.map.find(ticket);
    if (it == sh.map.end()) return fail(PG_E_INVALID, "unknown ticket");
    r = it->second;
    sh.map.erase(it);  // this call owns the ticket now
  }
  collect_or_wait(srv, r, true);
  if (latency_ms) latency_ms[0] = std::chrono::duration<double, std::milli>(r->t_collected - r->t_submit).count();
  delete r;
  if (srv->engine_error.load() != PG_OK) return engine_failure(srv);
  return PG_OK;
}

int pg_server_get_stats(pg_server* srv, pg_server_stats* out) {
  clear_error();
  if (!srv || !out) return fail(PG_E_INVALID, "NULL argument");
  out->submitted = srv->st_submitted.load();
  out->rejected_busy = srv->st_rejected_busy.load();
  out->rejected_invalid = srv->st_rejected_invalid.load();
  out->completed = srv->st_completed.load();
  out->batches = srv->st_batches.load();
  out->pairs = srv->st_pairs.load();
  out->max_in_flight = srv->st_max_in_flight.load();
  out->max_batch_requests = srv->st_max_batch_requests.load();
  return PG_OK;
}

int pg_server_replay(pg_server* srv, int64_t nreq, const pg_request* reqs, const double* arrival_s,
                     int32_t max_outstanding, double* latency_ms, double* elapsed_s) {
  clear_error();
  if (!srv || (nreq > 0 && (!reqs || !latency_ms))) return fail(PG_E_INVALID, "NULL argument");
  if (nreq <= 0) return PG_OK;
  if (!arrival_s && max_outstanding < 1) return fail(PG_E_INVALID, "closed loop needs max_outstanding >= 1");
  // a few submitting and a few collecting threads: request i is submitted by
  // thread i mod S (in order of i within a thread; closed loop: the next
  // request of a shared counter) and collected by thread i mod C. The threads
  // meet only through atomics (they spin, yielding, while they wait).
  const int S = (int)std::min<int64_t>(4, nreq), C = (int)std::min<int64_t>(4, nreq);
  std::vector<std::atomic<uint64_t>> tickets((size_t)nreq);
  for (auto& t : tickets) t.store(0, std::memory_order_relaxed);
  std::vector<Clock::time_point> t_arr((size_t)nreq);
  std::atomic<int64_t> outstanding{0}, next{0};
  std::atomic<int> err{PG_OK};
  std::mutex err_m;
  std::string err_msg;
  auto set_err = [&](int rc) {
    std::lock_guard<std::mutex> lk(err_m);
    if (err.load() == PG_OK) {
      err_msg = pg_last_error();
      err.store(rc);
    }
  };
  const Clock::time_point t0 = Clock::now();
  auto submit_one = [&](int64_t i) {
    uint64_t tk = 0;
    int rc;
    while ((rc = pg_server_submit(srv, &reqs[i], &tk)) == PG_E_BUSY) std::this_thread::yield();
    if (rc != PG_OK) {
      set_err(rc);
      return false;
    }
    tickets[(size_t)i].store(tk, std::memory_order_release);
    return true;
  };
  // waiting for a time point: sleep while it is far, spin (yielding) over the
  // last stretch, so that idle load-generator threads leave the cores to the
  // threads that work
  auto wait_until = [&](Clock::time_point due) {
    for (;;) {
      const Clock::time_point now = Clock::now();
      if (now >= due) return;
      if (due - now > std::chrono::microseconds(200))
        std::this_thread::sleep_for(due - now - std::chrono::microseconds(100));
      else
        std::this_thread::yield();
    }
  };
  auto due_of = [&](int64_t i) {
    return t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
  };
  auto open_submitter = [&](int t) {
    for (int64_t i = t; i < nreq && err.load() == PG_OK; i += S) {
      const Clock::time_point due = due_of(i);
      wait_until(due);
      t_arr[(size_t)i] = due;
      if (!submit_one(i)) return;
    }
  };
  auto closed_submitter = [&]() {
    for (;;) {
      while (outstanding.load(std::memory_order_acquire) >= max_outstanding && err.load() == PG_OK)
        std::this_thread::yield();
      if (err.load() != PG_OK) return;
      const int64_t i = next.fetch_add(1);
      if (i >= nreq) return;
      outstanding.fetch_add(1);
      t_arr[(size_t)i] = Clock::now();
      if (!submit_one(i)) return;
    }
  };
  auto collector = [&](int c) {
    for (int64_t i = c; i < nreq; i += C) {
      if (arrival_s) wait_until(due_of(i));  // open loop: not submitted before its arrival
      uint64_t tk;
      while ((tk = tickets[(size_t)i].load(std::memory_order_acquire)) == 0) {
        if (err.load() != PG_OK) return;
        std::this_thread::yield();
      }
      const int rc = pg_server_wait(srv, tk, nullptr);
      latency_ms[i] = std::chrono::duration<double, std::milli>(Clock::now() - t_arr[(size_t)i]).count();
      if (rc != PG_OK) set_err(rc);
      outstanding.fetch_sub(1);
    }
  };
  std::vector<std::thread> threads;
  for (int c = 0; c < C; ++c) threads.emplace_back(collector, c);
  for (int t = 0; t < S; ++t) {
    if (arrival_s)
      threads.emplace_back(open_submitter, t);
    else
      threads.emplace_back(closed_submitter);
  }
  for (std::thread& th : threads) th.join();
  if (elapsed_s) *elapsed_s = std::chrono::duration<double>(Clock::now() - t0).count();
  if (err.load() != PG_OK) return fail(err.load(), err_msg);
  return PG_OK;
}

int pg_server_destroy(pg_server* srv) {
  clear_error();
  if (!srv) return fail(PG_E_INVALID, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(srv->work_mu);
    srv->stop.store(true);
  }
  srv->work_cv.notify_all();
  if (srv->engine.joinable()) srv->engine.join();
  for (TicketShard& sh : srv->tickets) {
    for (auto& kv : sh.map) delete kv.second;
    sh.map.clear();
  }
  for (Slot& sl : srv->slots) slot_free(sl);
  if (srv->a_u) (void)hipHostFree(srv->a_u);
  if (srv->a_v) (void)hipHostFree(srv->a_v);
  if (srv->a_out) (void)hipHostFree(srv->a_out);
  pfree(srv->d_views);
  delete srv;
  return PG_OK;
}

}  // extern "C"

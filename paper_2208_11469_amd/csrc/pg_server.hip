// Serving engine: resident sketches, vertex-pair queries, continuous batching.
//
// Submit validates a request on the host, copies its pairs and admits it if
// the byte budget allows. An engine thread keeps up to K batches in flight,
// one stream each (default priority). Whenever a batch slot is free and
// requests wait, it packs as many of them as fit into one launch: pairs go to
// the slot's pinned, coherent host buffers, a segment table tells each pair its
// request's sketch set, estimator and operation, and one fused kernel reads the
// pairs from host memory and writes every answer back there (no copy calls:
// a batch is one launch and one event). When a batch's event completes, its
// results are copied into the requests' host buffers and its slot and bytes are
// released, so requests that arrived meanwhile start in the next launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
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

constexpr int kArgSegments = 16;    // segment tables this small travel as kernel arguments

struct SegDesc {
  int64_t begin;  // first pair of the segment in the batch
  int32_t view;   // index into the server's views (sketch * kEstSlots + estimator)
  int32_t op;     // PG_OP_CN or PG_OP_JACCARD
};

struct SegArgs {
  int32_t nseg;
  SegDesc seg[kArgSegments];  // used when nseg <= kArgSegments
};

// One lane per pair; the segment is found by binary search over the batch's
// segment starts held in LDS. `pu`, `pv` and `out` are pinned host memory.
__global__ __launch_bounds__(256) void k_serve_batch(const SkView* __restrict__ views, SegArgs a,
                                                     const SegDesc* __restrict__ big, const int32_t* __restrict__ pu,
                                                     const int32_t* __restrict__ pv, int64_t total,
                                                     double* __restrict__ out) {
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
    const int32_t u = pu[e], v = pv[e];
    uint32_t raw;
    const double est = eval_pair_any(s, u, v, raw);
    out[e] = sd.op == PG_OP_CN ? est : jaccard_of(est, s.deg[u], s.deg[v]);
  }
}

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  int32_t op = 0, view = 0;
  int64_t npairs = 0;
  std::vector<int32_t> u, v;
  void* out = nullptr;
  uint64_t bytes = 0;
  Clock::time_point t_submit, t_done;
  bool done = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t event = nullptr;
  int32_t* h_u = nullptr;  // pinned, coherent: the batch kernel reads the pairs here
  int32_t* h_v = nullptr;
  double* h_out = nullptr;  // and writes the answers here
  SegDesc* h_seg = nullptr;  // segment tables larger than kArgSegments, staged for d_seg
  SegDesc* d_seg = nullptr;
  std::vector<Request*> reqs;
  bool busy = false;
};

}  // namespace
}  // namespace pg

struct pg_server {
  pg_ctx* ctx = nullptr;
  const pg_graph* g = nullptr;
  std::vector<pg_sketches*> sketches;
  pg::SkView* d_views = nullptr;
  std::vector<double*> tables;  // server-owned estimator tables (Bloom filters)
  std::vector<bool> view_ok;
  pg_server_params p{};
  std::mutex mu;
  std::condition_variable work_cv;  // engine: new requests or stop
  std::condition_variable done_cv;  // waiters: results delivered
  std::deque<pg::Request*> queue;
  std::unordered_map<uint64_t, pg::Request*> live;
  std::vector<pg::Slot> slots;
  std::thread engine;
  bool stop = false;
  int engine_error = PG_OK;
  std::string engine_msg;
  uint64_t next_ticket = 1;
  uint64_t bytes_admitted = 0;
  pg_server_stats stats{};
};

namespace pg {
namespace {

int slot_init(pg_server* srv, Slot& sl) {
  const int64_t cap = srv->p.max_batch_pairs;
  PG_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
  PG_HIP(hipEventCreateWithFlags(&sl.event, hipEventDisableTiming));
  PG_HIP(hipHostMalloc((void**)&sl.h_u, sizeof(int32_t) * cap, hipHostMallocCoherent));
  PG_HIP(hipHostMalloc((void**)&sl.h_v, sizeof(int32_t) * cap, hipHostMallocCoherent));
  PG_HIP(hipHostMalloc((void**)&sl.h_out, sizeof(double) * cap, hipHostMallocCoherent));
  PG_HIP(hipHostMalloc((void**)&sl.h_seg, sizeof(SegDesc) * kMaxSegments, hipHostMallocDefault));
  PG_TRY(palloc((void**)&sl.d_seg, sizeof(SegDesc) * kMaxSegments));
  return PG_OK;
}

void slot_free(Slot& sl) {
  if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  if (sl.h_u) (void)hipHostFree(sl.h_u);
  if (sl.h_v) (void)hipHostFree(sl.h_v);
  if (sl.h_out) (void)hipHostFree(sl.h_out);
  if (sl.h_seg) (void)hipHostFree(sl.h_seg);
  pfree(sl.d_seg);
  if (sl.event) (void)hipEventDestroy(sl.event);
  if (sl.stream) (void)hipStreamDestroy(sl.stream);
  sl = Slot();
}

// Pack requests into the slot's host buffers and enqueue the kernel and the
// event (plus one small copy when the segment table is too big for arguments).
int launch_batch(pg_server* srv, Slot& sl) {
  int64_t total = 0;
  SegArgs a{};
  a.nseg = (int32_t)sl.reqs.size();
  int32_t i = 0;
  for (Request* r : sl.reqs) {
    std::memcpy(sl.h_u + total, r->u.data(), sizeof(int32_t) * r->npairs);
    std::memcpy(sl.h_v + total, r->v.data(), sizeof(int32_t) * r->npairs);
    const SegDesc sd{total, r->view, r->op};
    sl.h_seg[i] = sd;
    if (i < kArgSegments) a.seg[i] = sd;
    ++i;
    total += r->npairs;
  }
  if (a.nseg > kArgSegments)
    PG_HIP(hipMemcpyAsync(sl.d_seg, sl.h_seg, sizeof(SegDesc) * a.nseg, hipMemcpyHostToDevice, sl.stream));
  const unsigned grid = grid_for(total, 256, 16384);
  hipLaunchKernelGGL(k_serve_batch, dim3(grid), dim3(256), 0, sl.stream, (const SkView*)srv->d_views, a,
                     (const SegDesc*)sl.d_seg, (const int32_t*)sl.h_u, (const int32_t*)sl.h_v, total, sl.h_out);
  PG_LAUNCH_CHECK();
  PG_HIP(hipEventRecord(sl.event, sl.stream));
  return PG_OK;
}

// Copy a finished batch's results to the requests' buffers.
void deliver(Slot& sl) {
  int64_t off = 0;
  for (Request* r : sl.reqs) {
    if (r->op == PG_OP_CN) {
      std::memcpy(r->out, sl.h_out + off, sizeof(double) * r->npairs);
    } else {
      float* o = (float*)r->out;
      for (int64_t i = 0; i < r->npairs; ++i) o[i] = (float)sl.h_out[off + i];
    }
    off += r->npairs;
  }
}

void engine_loop(pg_server* srv) {
  (void)hipSetDevice(srv->ctx->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    bool progressed = false;
    // retire finished batches
    for (Slot& sl : srv->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.event);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        srv->engine_error = PG_E_DEVICE;
        srv->engine_msg = std::string("serving batch: ") + hipGetErrorString(q);
      } else {
        deliver(sl);
      }
      const Clock::time_point now = Clock::now();
      for (Request* r : sl.reqs) {
        r->done = true;
        r->t_done = now;
        srv->stats.completed++;
        srv->stats.pairs += (uint64_t)r->npairs;
      }
      sl.reqs.clear();
      sl.busy = false;
      progressed = true;
      srv->done_cv.notify_all();
    }
    // start batches on free slots
    for (Slot& sl : srv->slots) {
      if (sl.busy || srv->queue.empty()) continue;
      int64_t total = 0;
      while (!srv->queue.empty() && (int)sl.reqs.size() < kMaxSegments &&
             total + srv->queue.front()->npairs <= srv->p.max_batch_pairs) {
        Request* r = srv->queue.front();
        srv->queue.pop_front();
        total += r->npairs;
        sl.reqs.push_back(r);
      }
      if (sl.reqs.empty()) continue;
      const int rc = launch_batch(srv, sl);
      if (rc != PG_OK) {
        srv->engine_error = rc;
        srv->engine_msg = pg_last_error();
      }
      sl.busy = true;
      srv->stats.batches++;
      progressed = true;
    }
    const uint64_t busy = (uint64_t)std::count_if(srv->slots.begin(), srv->slots.end(), [](const Slot& s) { return s.busy; });
    srv->stats.max_in_flight = std::max(srv->stats.max_in_flight, busy);
    const bool inflight = busy > 0;
    if (srv->stop && !inflight && srv->queue.empty()) break;
    if (!progressed) {
      if (inflight) {
        // a batch is on the device: poll again shortly
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        srv->work_cv.wait(lk, [&] { return srv->stop || !srv->queue.empty(); });
      }
    }
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
  PG_HIP(hipSetDevice(ctx->device));
  pg_server* srv = new (std::nothrow) pg_server();
  if (!srv) return fail(PG_E_NOMEM, "host allocation failed");
  srv->ctx = ctx;
  srv->g = g;
  srv->sketches.assign(sketches, sketches + nsketches);
  pg_server_params p{};
  if (params) p = *params;
  if (p.max_batches_in_flight <= 0) p.max_batches_in_flight = 3;
  if (p.max_pairs_per_request <= 0) p.max_pairs_per_request = 65536;
  if (p.max_batch_pairs <= 0) p.max_batch_pairs = 1 << 20;
  if (p.memory_budget_bytes == 0) p.memory_budget_bytes = 256ull << 20;
  p.max_batches_in_flight = std::min(p.max_batches_in_flight, 16);
  p.max_batch_pairs = std::max<int64_t>(p.max_batch_pairs, p.max_pairs_per_request);
  srv->p = p;
  // one view per (sketch set, estimator); Bloom filters get server-owned tables
  std::vector<SkView> views((size_t)nsketches * kEstSlots);
  srv->view_ok.assign(views.size(), false);
  int rc = PG_OK;
  hipStream_t s = nullptr;
  for (int i = 0; i < nsketches && rc == PG_OK; ++i) {
    pg_sketches* sk = srv->sketches[i];
    for (int est = 1; est < kEstSlots && rc == PG_OK; ++est) {
      if (check_estimator(sk, est) != PG_OK) continue;
      SkView v = make_view(sk, est);
      if (sk->kind == PG_BF) {
        double* t = nullptr;
        rc = palloc((void**)&t, sizeof(double) * (sk->size + 1));
        if (rc != PG_OK) break;
        srv->tables.push_back(t);
        rc = fill_table(t, sk->size, sk->b, est, s);
        v.table = t;
      }
      views[(size_t)i * kEstSlots + est] = v;
      srv->view_ok[(size_t)i * kEstSlots + est] = true;
    }
  }
  clear_error();
  if (rc == PG_OK) rc = palloc((void**)&srv->d_views, sizeof(SkView) * views.size());
  if (rc == PG_OK) {
    hipError_t e = hipMemcpy(srv->d_views, views.data(), sizeof(SkView) * views.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = fail(PG_E_DEVICE, std::string("server views: ") + hipGetErrorString(e));
  }
  srv->slots.resize((size_t)p.max_batches_in_flight);
  for (Slot& sl : srv->slots)
    if (rc == PG_OK) rc = slot_init(srv, sl);
  if (rc != PG_OK) {
    for (Slot& sl : srv->slots) slot_free(sl);
    for (double* t : srv->tables) pfree(t);
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
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stats.rejected_invalid++;
    return fail(PG_E_INVALID, why);
  };
  if (req->op != PG_OP_CN && req->op != PG_OP_JACCARD) return invalid("unknown op");
  if (req->sketch < 0 || req->sketch >= (int32_t)srv->sketches.size()) return invalid("sketch index out of range");
  if (req->estimator < 1 || req->estimator >= kEstSlots ||
      !srv->view_ok[(size_t)req->sketch * kEstSlots + req->estimator])
    return invalid("estimator does not match the sketch kind");
  if (req->npairs < 1 || req->npairs > srv->p.max_pairs_per_request) return invalid("npairs out of range");
  if (!req->u || !req->v || !req->out) return invalid("NULL pair or output array");
  const int32_t n = srv->g->n;
  for (int64_t i = 0; i < req->npairs; ++i)
    if ((uint32_t)req->u[i] >= (uint32_t)n || (uint32_t)req->v[i] >= (uint32_t)n)
      return invalid("vertex ID out of range");
  const uint64_t bytes = (uint64_t)req->npairs * 16;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->engine_error != PG_OK) return fail(srv->engine_error, srv->engine_msg);
    if (srv->stop) return fail(PG_E_INVALID, "server is stopping");
    if (srv->bytes_admitted + bytes > srv->p.memory_budget_bytes) {
      srv->stats.rejected_busy++;
      return fail(PG_E_BUSY, "not admitted: memory budget in use");
    }
    srv->bytes_admitted += bytes;
  }
  Request* r = new (std::nothrow) Request();
  if (!r) {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->bytes_admitted -= bytes;
    return fail(PG_E_NOMEM, "host allocation failed");
  }
  r->op = req->op;
  r->view = req->sketch * kEstSlots + req->estimator;
  r->npairs = req->npairs;
  r->u.assign(req->u, req->u + req->npairs);
  r->v.assign(req->v, req->v + req->npairs);
  r->out = req->out;
  r->bytes = bytes;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    r->ticket = srv->next_ticket++;
    srv->live[r->ticket] = r;
    srv->queue.push_back(r);
    srv->stats.submitted++;
    *ticket = r->ticket;
  }
  srv->work_cv.notify_one();
  return PG_OK;
}

int pg_server_poll(pg_server* srv, uint64_t ticket, int32_t* done) {
  clear_error();
  if (!srv || !done) return fail(PG_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->live.find(ticket);
  if (it == srv->live.end()) return fail(PG_E_INVALID, "unknown ticket");
  *done = it->second->done ? 1 : 0;
  return srv->engine_error;
}

int pg_server_wait(pg_server* srv, uint64_t ticket, double* latency_ms) {
  clear_error();
  if (!srv) return fail(PG_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->live.find(ticket);
  if (it == srv->live.end()) return fail(PG_E_INVALID, "unknown ticket");
  Request* r = it->second;
  srv->done_cv.wait(lk, [&] { return r->done; });
  if (latency_ms) latency_ms[0] = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  srv->live.erase(it);
  srv->bytes_admitted -= r->bytes;
  const int err = srv->engine_error;
  const std::string msg = srv->engine_msg;
  delete r;
  if (err != PG_OK) return fail(err, msg);
  return PG_OK;
}

int pg_server_get_stats(pg_server* srv, pg_server_stats* out) {
  clear_error();
  if (!srv || !out) return fail(PG_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->stats;
  return PG_OK;
}

int pg_server_replay(pg_server* srv, int64_t nreq, const pg_request* reqs, const double* arrival_s,
                     int32_t max_outstanding, double* latency_ms, double* elapsed_s) {
  clear_error();
  if (!srv || (nreq > 0 && (!reqs || !latency_ms))) return fail(PG_E_INVALID, "NULL argument");
  if (nreq <= 0) return PG_OK;
  if (!arrival_s && max_outstanding < 1) return fail(PG_E_INVALID, "closed loop needs max_outstanding >= 1");
  std::vector<uint64_t> tickets((size_t)nreq, 0);
  std::vector<Clock::time_point> t_arr((size_t)nreq);
  std::mutex m;
  std::condition_variable cv;
  int64_t submitted = 0, collected = 0;
  int err = PG_OK;
  std::string err_msg;
  const Clock::time_point t0 = Clock::now();
  // collector: waits for the requests in submission order
  std::thread collector([&] {
    for (int64_t i = 0; i < nreq; ++i) {
      uint64_t tk;
      {
        std::unique_lock<std::mutex> lk(m);
        cv.wait(lk, [&] { return submitted > i || err != PG_OK; });
        if (submitted <= i) return;
        tk = tickets[(size_t)i];
      }
      double lat = 0.0;
      const int rc = pg_server_wait(srv, tk, &lat);
      std::lock_guard<std::mutex> lk(m);
      if (rc != PG_OK && err == PG_OK) {
        err = rc;
        err_msg = pg_last_error();
      }
      latency_ms[i] = std::chrono::duration<double, std::milli>(Clock::now() - t_arr[(size_t)i]).count();
      ++collected;
      cv.notify_all();
    }
  });
  for (int64_t i = 0; i < nreq && err == PG_OK; ++i) {
    if (arrival_s) {
      const Clock::time_point due = t0 + std::chrono::duration_cast<Clock::duration>(
                                             std::chrono::duration<double>(arrival_s[i]));
      while (Clock::now() < due) std::this_thread::yield();
      t_arr[(size_t)i] = due;
    } else {
      std::unique_lock<std::mutex> lk(m);
      cv.wait(lk, [&] { return submitted - collected < max_outstanding || err != PG_OK; });
      t_arr[(size_t)i] = Clock::now();
    }
    uint64_t tk = 0;
    int rc;
    while ((rc = pg_server_submit(srv, &reqs[i], &tk)) == PG_E_BUSY) std::this_thread::yield();
    std::lock_guard<std::mutex> lk(m);
    if (rc != PG_OK) {
      err = rc;
      err_msg = pg_last_error();
    } else {
      tickets[(size_t)i] = tk;
      ++submitted;
    }
    cv.notify_all();
  }
  collector.join();
  if (elapsed_s) *elapsed_s = std::chrono::duration<double>(Clock::now() - t0).count();
  if (err != PG_OK) return fail(err, err_msg);
  return PG_OK;
}

int pg_server_destroy(pg_server* srv) {
  clear_error();
  if (!srv) return fail(PG_E_INVALID, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->work_cv.notify_all();
  if (srv->engine.joinable()) srv->engine.join();
  for (auto& kv : srv->live) delete kv.second;
  srv->live.clear();
  for (Slot& sl : srv->slots) slot_free(sl);
  for (double* t : srv->tables) pfree(t);
  pfree(srv->d_views);
  delete srv;
  return PG_OK;
}

}  // extern "C"

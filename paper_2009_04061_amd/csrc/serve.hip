// The serving loop: programs stay resident (loaded by the caller), sample
// batches are submitted as requests, admitted in arrival order against a
// device-memory budget, and run in batches by the batched kernels of the
// histogram, the blamer and the estimators (every kernel launch context is
// analyzed on its own, Sec. 3, so a batch is a set of independent
// profiles).  A worker thread per server forms a batch from whatever has
// been admitted whenever fewer than kMaxInflight batches are on the device,
// launches it on one of two streams in turn (consecutive batches overlap),
// and completes tickets when a batch's event has been reached.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>

#include "common.h"

namespace gpa {

constexpr int kServeStreams = 2;
constexpr size_t kMaxInflight = 4;
constexpr size_t kMaxBatch = 64;

uint64_t request_device_bytes(const gpa_program &p, uint64_t n, bool host_records) {
  const uint64_t ni = p.n_instr, ns = p.n_scopes, ne = p.n_edges;
  uint64_t b = host_records ? 8 * n : 0;
  b += n ? hist_hot_scratch_bytes(p.n_instr <= hist_hot_max_pcs() ? p.n_instr : hist_hot_max_pcs(),
                                  n)
         : 0;
  if (p.n_instr > hist_hot_max_pcs()) b += 8 * n + 16 * n;   // the partition path's payloads
  b += 100 * ni + 32;                                         // counts, issued, totals
  b += 16 * ne * p.n_blamable + 8 * ne + ni * (16 * p.n_blamable + 8 * kBlameFx + 2);   // shares, tables
  b += 88 * ni + 2 * 88 * ns + 16 * ne;                       // advise scratch
  b += 88 * ns * 2 + 8 * (uint64_t)p.tk_chunks * 16 * 2;      // chunk partials, top-k candidates
  b += 8 * ns * 23 + 16 * 16 * (uint64_t)p.n_roots;           // advice outputs
  // every block rounds up to its size class (powers of two up to 16 MiB,
  // whole MiB beyond): at most twice the size, plus the tables of the batch
  return 2 * b + (64u << 10);
}

}  // namespace gpa

using namespace gpa;

namespace {

enum ReqState { kPending = 0, kAdmitted, kDone, kFailed };

struct Request {
  uint64_t ticket = 0;
  gpa_program *prog = nullptr;
  const gpa_sample *samples = nullptr;
  uint64_t n = 0;
  bool on_device = false;
  uint64_t bytes = 0;
  ReqState state = kPending;
  gpa_status status = GPA_OK;
  std::string err;
  gpa_blame *blame = nullptr;
  gpa_advice *advice = nullptr;
};

struct Batch {
  std::vector<Request *> reqs;
  std::unique_ptr<Arena> ar;
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  unsigned long long *tot_host = nullptr;   // pinned, 4 per request
};

}  // namespace

struct gpa_server {
  uint64_t budget = 0;
  int dev = 0;
  hipStream_t streams[kServeStreams] = {nullptr, nullptr};
  int next_stream = 0;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t reserved = 0;
  std::deque<Request *> pending;
  std::vector<Batch *> inflight;
  std::unordered_map<uint64_t, Request *> live;
  std::deque<uint64_t> done_q;            // tickets finished since the last waits, in order
  std::condition_variable done_cv;        // signalled when done_q grows
  std::vector<hipEvent_t> free_events;
  std::vector<unsigned long long *> free_tot;   // pinned buffers of kMaxBatch * 4
  gpa_server_stats stats{};
};

namespace {

// launches one batch (called without the server lock; the requests are
// already admitted and owned by the batch)
void launch_batch(gpa_server *sv, Batch *bt) {
  hipStream_t s = bt->s;
  const uint32_t m = (uint32_t)bt->reqs.size();
  bt->ar.reset(new Arena(s));
  Arena &ar = *bt->ar;
  std::vector<gpa_program *> progs(m);
  std::vector<const gpa_sample *> ds(m);
  std::vector<uint64_t> n(m);
  for (uint32_t k = 0; k < m; ++k) {
    Request *r = bt->reqs[k];
    progs[k] = r->prog;
    n[k] = r->n;
    ds[k] = r->samples;
    if (r->n && !r->on_device) {
      gpa_sample *tmp = ar.get<gpa_sample>(r->n);
      GPA_HIP(hipMemcpyAsync(tmp, r->samples, r->n * sizeof(gpa_sample), hipMemcpyHostToDevice, s));
      ds[k] = tmp;
    }
  }
  unsigned long long *dtot = ar.get<unsigned long long>((size_t)m * 4);
  std::vector<gpa_blame *> b(m, nullptr);
  std::vector<gpa_advice *> a(m, nullptr);
  try {
    enqueue_attribute_batch(progs.data(), ds.data(), n.data(), m, s, ar, b.data(), dtot, false);
    for (uint32_t k = 0; k < m; ++k) a[k] = new gpa_advice(b[k]->prog);
    run_estimate_batch(b.data(), a.data(), m, 16, s, ar);
  } catch (...) {
    // no kernel of this batch may still read the handles' memory
    (void)hipStreamSynchronize(s);
    for (gpa_blame *x : b) delete x;
    for (gpa_advice *x : a) delete x;
    throw;
  }
  GPA_HIP(hipMemcpyAsync(bt->tot_host, dtot, sizeof(unsigned long long) * 4 * m,
                         hipMemcpyDeviceToHost, s));
  GPA_HIP(hipEventRecord(bt->done, s));
  for (uint32_t k = 0; k < m; ++k) {
    bt->reqs[k]->blame = b[k];
    bt->reqs[k]->advice = a[k];
  }
  (void)sv;
}

// under the lock: a batch whose event has been reached
void complete_batch(gpa_server *sv, Batch *bt, gpa_status st, const std::string &err) {
  for (size_t k = 0; k < bt->reqs.size(); ++k) {
    Request *r = bt->reqs[k];
    if (st == GPA_OK) {
      for (int q = 0; q < 4; ++q) r->blame->totals[q] = bt->tot_host[4 * k + q];
      r->state = kDone;
      sv->stats.completed += 1;
    } else {
      delete r->advice;
      delete r->blame;
      r->advice = nullptr;
      r->blame = nullptr;
      r->state = kFailed;
      r->status = st;
      r->err = err;
      sv->stats.failed += 1;
    }
    sv->reserved -= r->bytes;
    sv->done_q.push_back(r->ticket);
    gpa::program_release(r->prog);
  }
  sv->done_cv.notify_all();
  if (bt->ar) bt->ar->work_done();
  bt->ar.reset();
  sv->free_events.push_back(bt->done);
  sv->free_tot.push_back(bt->tot_host);
  delete bt;
}

void worker_main(gpa_server *sv) {
  (void)hipSetDevice(sv->dev);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // completions
    for (size_t i = 0; i < sv->inflight.size();) {
      Batch *bt = sv->inflight[i];
      const hipError_t q = hipEventQuery(bt->done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      sv->inflight.erase(sv->inflight.begin() + i);
      if (q == hipSuccess) {
        complete_batch(sv, bt, GPA_OK, "");
      } else {
        (void)hipGetLastError();
        complete_batch(sv, bt, GPA_E_DEVICE, std::string("batch failed: ") + hipGetErrorString(q));
      }
      sv->cv.notify_all();
    }
    // admission, in arrival order, while memory and batch slots allow
    Batch *bt = nullptr;
    if (sv->inflight.size() < kMaxInflight) {
      while (!sv->pending.empty() && (!bt || bt->reqs.size() < kMaxBatch)) {
        Request *r = sv->pending.front();
        if (sv->reserved + r->bytes > sv->budget) break;
        sv->pending.pop_front();
        sv->reserved += r->bytes;
        r->state = kAdmitted;
        if (!bt) bt = new Batch();
        bt->reqs.push_back(r);
      }
    }
    if (bt) {
      sv->stats.peak_reserved = std::max(sv->stats.peak_reserved, sv->reserved);
      sv->stats.batches += 1;
      sv->stats.admitted += bt->reqs.size();
      sv->stats.max_batch = std::max<uint64_t>(sv->stats.max_batch, bt->reqs.size());
      bt->s = sv->streams[sv->next_stream];
      sv->next_stream = (sv->next_stream + 1) % kServeStreams;
      bt->done = sv->free_events.back();
      sv->free_events.pop_back();
      bt->tot_host = sv->free_tot.back();
      sv->free_tot.pop_back();
      lk.unlock();
      gpa_status st = GPA_OK;
      std::string err;
      try {
        launch_batch(sv, bt);
      } catch (const Error &e) {
        st = e.code;
        err = gpa_last_error();
      } catch (...) {
        st = GPA_E_DEVICE;
        err = "unexpected failure while launching a batch";
      }
      if (st != GPA_OK) (void)hipStreamSynchronize(bt->s);
      lk.lock();
      if (st == GPA_OK) sv->inflight.push_back(bt);
      else complete_batch(sv, bt, st, err);
      continue;
    }
    if (sv->stop && sv->pending.empty() && sv->inflight.empty()) break;
    if (sv->inflight.empty()) sv->cv.wait(lk);   // woken by a submit or by stop
    else sv->cv.wait_for(lk, std::chrono::microseconds(20));
  }
}

}  // namespace

extern "C" {

gpa_status gpa_server_create(uint64_t budget_bytes, gpa_server **out) {
  if (!out || budget_bytes == 0) {
    set_error("gpa_server_create: NULL argument or zero budget");
    return GPA_E_INVALID;
  }
  *out = nullptr;
  gpa_server *sv = new (std::nothrow) gpa_server();
  if (!sv) {
    set_error("host allocation failed");
    return GPA_E_NOMEM;
  }
  sv->budget = budget_bytes;
  hipError_t e = hipGetDevice(&sv->dev);
  for (int k = 0; k < kServeStreams && e == hipSuccess; ++k)
    e = hipStreamCreateWithFlags(&sv->streams[k], hipStreamNonBlocking);
  for (size_t k = 0; k < kMaxInflight && e == hipSuccess; ++k) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) sv->free_events.push_back(ev);
    unsigned long long *t = nullptr;
    if (e == hipSuccess) e = hipHostMalloc((void **)&t, sizeof(unsigned long long) * 4 * kMaxBatch);
    if (e == hipSuccess) sv->free_tot.push_back(t);
  }
  if (e != hipSuccess) {
    set_error("gpa_server_create: %s", hipGetErrorString(e));
    for (hipStream_t s : sv->streams)
      if (s) (void)hipStreamDestroy(s);
    for (hipEvent_t ev : sv->free_events) (void)hipEventDestroy(ev);
    for (unsigned long long *t : sv->free_tot) (void)hipHostFree(t);
    delete sv;
    return GPA_E_DEVICE;
  }
  sv->worker = std::thread(worker_main, sv);
  *out = sv;
  return GPA_OK;
}

gpa_status gpa_server_submit(gpa_server *sv, gpa_program *p, const gpa_sample *samples,
                             uint64_t n, int samples_on_device, uint64_t *ticket) {
  if (!sv || !p || !ticket || (n && !samples)) {
    set_error("gpa_server_submit: NULL argument");
    return GPA_E_INVALID;
  }
  if (n >= 0x40000000ull) {
    set_error("gpa_server_submit: 2^30 samples or more");
    return GPA_E_UNSUPPORTED;
  }
  const uint64_t bytes = request_device_bytes(*p, n, !samples_on_device);
  if (bytes > sv->budget) {
    set_error("gpa_server_submit: the request needs about %llu bytes, more than the server's "
              "budget of %llu", (unsigned long long)bytes, (unsigned long long)sv->budget);
    return GPA_E_NOMEM;
  }
  Request *r = new (std::nothrow) Request();
  if (!r) {
    set_error("host allocation failed");
    return GPA_E_NOMEM;
  }
  r->prog = p;
  r->samples = samples;
  r->n = n;
  r->on_device = samples_on_device != 0;
  r->bytes = bytes;
  gpa::program_retain(p);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      gpa::program_release(p);
      delete r;
      set_error("gpa_server_submit: the server is shutting down");
      return GPA_E_STATE;
    }
    r->ticket = sv->next_ticket++;
    sv->live[r->ticket] = r;
    sv->pending.push_back(r);
    sv->stats.submitted += 1;
  }
  sv->cv.notify_all();
  *ticket = r->ticket;
  return GPA_OK;
}

gpa_status gpa_server_poll(gpa_server *sv, uint64_t ticket, gpa_blame **blame,
                           gpa_advice **advice) {
  if (!sv || !advice) {
    set_error("gpa_server_poll: NULL argument");
    return GPA_E_INVALID;
  }
  *advice = nullptr;
  if (blame) *blame = nullptr;
  Request *r = nullptr;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) {
      set_error("gpa_server_poll: unknown ticket %llu", (unsigned long long)ticket);
      return GPA_E_INVALID;
    }
    r = it->second;
    if (r->state == kPending || r->state == kAdmitted) return GPA_E_BUSY;
    sv->live.erase(it);
  }
  const gpa_status st = r->status;
  if (st != GPA_OK) {
    set_error("%s", r->err.c_str());
  } else {
    *advice = r->advice;
    if (blame) *blame = r->blame;
    else delete r->blame;
  }
  delete r;
  return st;
}

gpa_status gpa_server_wait(gpa_server *sv, uint64_t timeout_us, uint64_t *ticket) {
  if (!sv || !ticket) {
    set_error("gpa_server_wait: NULL argument");
    return GPA_E_INVALID;
  }
  std::unique_lock<std::mutex> lk(sv->mu);
  const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(timeout_us);
  for (;;) {
    // tickets already collected by a poll are skipped
    while (!sv->done_q.empty() && !sv->live.count(sv->done_q.front())) sv->done_q.pop_front();
    if (!sv->done_q.empty()) {
      *ticket = sv->done_q.front();
      sv->done_q.pop_front();
      return GPA_OK;
    }
    if (sv->done_cv.wait_until(lk, until) == std::cv_status::timeout) {
      while (!sv->done_q.empty() && !sv->live.count(sv->done_q.front())) sv->done_q.pop_front();
      if (sv->done_q.empty()) return GPA_E_BUSY;
    }
  }
}

gpa_status gpa_server_stats_get(gpa_server *sv, gpa_server_stats *st) {
  if (!sv || !st) {
    set_error("gpa_server_stats_get: NULL argument");
    return GPA_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  *st = sv->stats;
  st->reserved = sv->reserved;
  st->budget = sv->budget;
  st->queued = sv->pending.size();
  st->inflight_batches = sv->inflight.size();
  return GPA_OK;
}

void gpa_server_free(gpa_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  for (auto &kv : sv->live) {
    Request *r = kv.second;
    delete r->advice;
    delete r->blame;
    if (r->state == kPending) gpa::program_release(r->prog);
    delete r;
  }
  for (hipStream_t s : sv->streams)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t ev : sv->free_events) (void)hipEventDestroy(ev);
  for (unsigned long long *t : sv->free_tot) (void)hipHostFree(t);
  delete sv;
}

}  // extern "C"

// Continuous-batching census server.
//
// Requests carry host CSR buffers.  The server owns one device pool of
// `hbm_budget_bytes`, sub-allocated first-fit; a request is admitted when the
// head of the FIFO queue fits in the pool and a worker is free, and it holds
// its range (graph copy + histogram + build/census workspace) until it
// completes.  Each of the `max_inflight` workers drives its own HIP stream, so
// admitted requests run on the device concurrently and a request that arrives
// while others run starts as soon as memory and a worker free up.  The census
// itself is the same validated pipeline as motif_census().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

using namespace motif;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kMaxPending = 1 << 16;

size_t al(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

struct Request {
  uint64_t ticket = 0;
  int32_t k = 0, n = 0;
  int64_t m = 0;
  std::vector<int32_t> off, idx;
  uint64_t* hist_out = nullptr;
  size_t footprint = 0;
  TuningSet tune;       // taken at submit: sizes the footprint and drives the run
  bool waited = false;  // a thread is in motif_server_wait on this request
  enum State { kPending, kRunning, kDone, kCanceled } state = kPending;
  int32_t status = 0;
};

// First-fit allocator over [0, size) with coalescing.
class RangeAlloc {
 public:
  explicit RangeAlloc(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

size_t request_bytes(int32_t n, int64_t m, int32_t k, int cus, const Tuning& t) {
  const int C = motif_num_classes(k);
  return al(sizeof(int32_t) * (size_t)(n + 1)) + al(sizeof(int32_t) * (size_t)(m + 1)) + al(sizeof(uint64_t) * C) +
         al(pipeline_bytes(n, m, 1, false, k, cus, n, t));
}

}  // namespace

struct motif_server {
  int device = 0;
  int cus = 0;
  size_t budget = 0;
  int max_inflight = 1;
  char* pool = nullptr;
  RangeAlloc* ranges = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending;
  std::map<uint64_t, Request*> requests;
  uint64_t next_ticket = 1;
  bool stop = false;
  int64_t completed = 0, inflight = 0, bytes_inflight = 0, peak_bytes = 0;
  std::vector<std::thread> workers;

  void worker_main(int wid);
};

void motif_server::worker_main(int /*wid*/) {
  hipStream_t s = nullptr;
  Pipeline p;
  p.num_cus = cus;
  // a worker whose stream or status words cannot be set up still takes
  // requests and ends them with MOTIF_EDEVICE, so no waiter is left behind
  const bool ready = hipSetDevice(device) == hipSuccess && hipStreamCreate(&s) == hipSuccess &&
                     hipMalloc(&p.status, kStatusWords * sizeof(int32_t)) == hipSuccess &&
                     hipHostMalloc(&p.host_status, kStatusWords * sizeof(int32_t), hipHostMallocDefault) == hipSuccess;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    Request* r = nullptr;
    size_t off = 0;
    while (!stop) {
      // strict FIFO: only the head may start, so a large request is never starved
      if (!pending.empty() && ranges->alloc(pending.front()->footprint, &off)) {
        r = pending.front();
        pending.pop_front();
        break;
      }
      cv_work.wait(lk);
    }
    if (!r) break;
    r->state = Request::kRunning;
    ++inflight;
    bytes_inflight += (int64_t)r->footprint;
    peak_bytes = std::max(peak_bytes, bytes_inflight);
    lk.unlock();

    char* base = pool + off;
    int32_t* d_off = (int32_t*)base;
    int32_t* d_idx = (int32_t*)(base + al(sizeof(int32_t) * (size_t)(r->n + 1)));
    uint64_t* d_hist = (uint64_t*)((char*)d_idx + al(sizeof(int32_t) * (size_t)(r->m + 1)));
    const int C = motif_num_classes(r->k);
    p.arena.base = (char*)d_hist + al(sizeof(uint64_t) * C);
    p.arena.cap = r->footprint - (size_t)(p.arena.base - base);
    int32_t rc = 0;
    if (!ready) {
      rc = MOTIF_EDEVICE;
    } else if (r->n == 0) {
      std::fill(r->hist_out, r->hist_out + C, 0ull);
    } else if (hipMemcpyAsync(d_off, r->off.data(), sizeof(int32_t) * (size_t)(r->n + 1), hipMemcpyHostToDevice, s) !=
                   hipSuccess ||
               (r->m && hipMemcpyAsync(d_idx, r->idx.data(), sizeof(int32_t) * (size_t)r->m, hipMemcpyHostToDevice,
                                       s) != hipSuccess)) {
      (void)hipStreamSynchronize(s);  // a copy already enqueued ends before its buffers are released
      rc = MOTIF_EDEVICE;
    } else {
      BuildInput in{};
      in.out_off = d_off;
      in.out_idx = d_idx;
      in.n = r->n;
      in.m = r->m;
      p.tune = r->tune;  // the tuning the footprint was sized with
      rc = run_census_on(p, in, r->k, d_hist, s);
      if (rc == 0) {
        if (hipMemcpyAsync(r->hist_out, d_hist, sizeof(uint64_t) * C, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          rc = MOTIF_EDEVICE;
      }
    }
    std::vector<int32_t>().swap(r->off);
    std::vector<int32_t>().swap(r->idx);

    lk.lock();
    ranges->release(off, r->footprint);
    --inflight;
    bytes_inflight -= (int64_t)r->footprint;
    ++completed;
    r->status = rc;
    r->state = Request::kDone;
    cv_done.notify_all();
    cv_work.notify_all();
  }
  lk.unlock();
  // tear-down: errors here change nothing that a caller could act on
  if (s) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  if (p.status) (void)hipFree(p.status);
  if (p.host_status) (void)hipHostFree(p.host_status);
}

extern "C" {

int64_t motif_request_footprint(int32_t n, int64_t m, int32_t k) {
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (n < 0 || m < 0 || n >= kMaxN || m >= kMaxN) return MOTIF_EINVAL_SHAPE;
  int dev = 0;
  if (ensure_init(&dev)) return MOTIF_EDEVICE;
  return (int64_t)request_bytes(n, m, k, device_cus(dev), tuning_for_call(dev, 1, &k, false, m).k[k]);
}

motif_server_t* motif_server_create(size_t hbm_budget_bytes, int32_t max_inflight) {
  if (max_inflight < 1 || max_inflight > 64 || hbm_budget_bytes < (1u << 20)) return nullptr;
  int dev = 0;
  if (ensure_init(&dev)) return nullptr;
  motif_server* s = new motif_server();
  s->device = dev;
  s->cus = device_cus(dev);
  s->budget = hbm_budget_bytes & ~(kAlign - 1);
  s->max_inflight = max_inflight;
  if (hipMalloc(&s->pool, s->budget) != hipSuccess) {
    delete s;
    return nullptr;
  }
  s->ranges = new RangeAlloc(s->budget);
  for (int w = 0; w < max_inflight; ++w) s->workers.emplace_back(&motif_server::worker_main, s, w);
  return s;
}

int32_t motif_server_submit(motif_server_t* s, const motif_graph_t* g, int32_t k, uint64_t* hist_out_host,
                            uint64_t* ticket) {
  if (!s || !g || !hist_out_host || !ticket) return MOTIF_EINVAL_ARG;
  if (motif_num_classes(k) < 0) return MOTIF_EINVAL_K;
  if (g->n < 0 || g->m < 0 || g->n >= kMaxN || g->m >= kMaxN) return MOTIF_EINVAL_SHAPE;
  if (g->n == 0 && g->m != 0) return MOTIF_EINVAL_SHAPE;
  if ((g->n > 0 && !g->out_off) || (g->m > 0 && !g->out_idx)) return MOTIF_EINVAL_ARG;
  Request* r = new Request();
  r->k = k;
  r->n = g->n;
  r->m = g->m;
  r->hist_out = hist_out_host;
  r->tune = tuning_for_call(s->device, 1, &k, false, g->m);
  r->footprint = request_bytes(g->n, g->m, k, s->cus, r->tune.k[k]);
  if (r->footprint > s->budget) {
    delete r;
    return MOTIF_ETOOBIG;
  }
  if (g->n > 0) r->off.assign(g->out_off, g->out_off + g->n + 1);
  if (g->m > 0) r->idx.assign(g->out_idx, g->out_idx + g->m);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->pending.size() >= kMaxPending) {
    delete r;
    return MOTIF_EAGAIN;
  }
  r->ticket = s->next_ticket++;
  s->requests[r->ticket] = r;
  s->pending.push_back(r);
  *ticket = r->ticket;
  s->cv_work.notify_all();
  return 0;
}

int32_t motif_server_wait(motif_server_t* s, uint64_t ticket, int64_t timeout_us) {
  if (!s) return MOTIF_EINVAL_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return MOTIF_EINVAL_ARG;
  Request* r = it->second;
  // one waiter per ticket: the waiter that sees the request end frees it, so
  // a second concurrent waiter would read freed memory
  if (r->waited) return MOTIF_EINVAL_ARG;
  r->waited = true;
  auto done = [r] { return r->state == Request::kDone || r->state == Request::kCanceled; };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, done);
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
    r->waited = false;
    return MOTIF_ETIMEOUT;
  }
  const int32_t rc = r->state == Request::kCanceled ? MOTIF_ECANCELED : r->status;
  s->requests.erase(it);
  delete r;
  return rc;
}

int32_t motif_server_cancel(motif_server_t* s, uint64_t ticket) {
  if (!s) return MOTIF_EINVAL_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return MOTIF_EINVAL_ARG;
  Request* r = it->second;
  if (r->state != Request::kPending) return MOTIF_EAGAIN;
  s->pending.erase(std::find(s->pending.begin(), s->pending.end(), r));
  r->state = Request::kCanceled;
  s->cv_done.notify_all();
  s->cv_work.notify_all();
  return 0;
}

int32_t motif_server_stats(motif_server_t* s, int64_t* completed, int64_t* inflight, int64_t* bytes_inflight,
                           int64_t* peak_bytes) {
  if (!s) return MOTIF_EINVAL_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  if (completed) *completed = s->completed;
  if (inflight) *inflight = s->inflight;
  if (bytes_inflight) *bytes_inflight = s->bytes_inflight;
  if (peak_bytes) *peak_bytes = s->peak_bytes;
  return 0;
}

int32_t motif_server_destroy(motif_server_t* s) {
  if (!s) return MOTIF_EINVAL_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // requests still queued are cancelled; running ones finish
    for (Request* r : s->pending) r->state = Request::kCanceled;
    s->pending.clear();
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  for (auto& t : s->workers) t.join();
  (void)hipSetDevice(s->device);  // tear-down: errors change nothing a caller could act on
  (void)hipFree(s->pool);
  delete s->ranges;
  for (auto& kv : s->requests) delete kv.second;
  delete s;
  return 0;
}

}  // extern "C"

// Continuous-batching server over a resident design.
//
// Requests (host location arrays + parameters) wait in a FIFO.  A worker
// thread groups waiting requests into a batch (up to a location cap): requests
// with identical parameters, and exhaustive FP64 requests scored by Cholesky
// columns on chip whatever their design sizes, lengthscales and nuggets (the
// batch then carries those per location, and one launch of the search kernel
// serves them all, the device's workgroup dispatcher handing locations to
// compute units as they free up); it admits the batch when the device
// memory it needs (its
// inputs, outputs and prediction workspace) fits under the HBM budget and a
// stream slot is free, and launches it: upload, candidate search, local
// designs, download, all asynchronous on the slot's stream (through pinned
// staging that each slot owns from creation, so no pinned allocation happens
// per request or batch).  Batches on
// different slots overlap on the device; a request that arrives while others
// run is admitted as soon as memory and a slot free up.  A head batch that
// does not fit may be bypassed by smaller batches a bounded number of times,
// after which admission waits for it.  Completion is detected by events;
// latency runs from submit to results resident in host memory.  Locations
// are independent, so a request's results do not depend on its batch.
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
#include <string>
#include <thread>
#include <vector>

#include "lagp_internal.h"

namespace {

using clk = std::chrono::steady_clock;

constexpr int64_t BATCH_MAX_LOCATIONS = 4096;
constexpr int HEAD_BYPASS_LIMIT = 4;
constexpr size_t WAITING_MAX = 1 << 16;

struct Request {
  uint64_t ticket = 0;
  lagp_params P{};
  int64_t M = 0;
  int p = 0;
  std::vector<double> xx;  // host copy, M x p
  // results (pinned host), filled by the batch that ran the request
  double* mean = nullptr;
  double* s2 = nullptr;
  double* df = nullptr;
  int32_t* sel = nullptr;
  int32_t* status = nullptr;
  clk::time_point t_submit;
  double latency_ms = 0.0;
  bool done = false;
  int32_t rc = LAGP_OK;
};

struct Batch {
  std::vector<std::shared_ptr<Request>> reqs;
  lagp_params P{};  // (a merged batch: the largest n of its requests)
  bool merged = false;  // per-location n, d, g
  int64_t M = 0;
  size_t bytes = 0;  // device bytes held while in flight
  int slot = -1;
  void* dev = nullptr;
  char* host = nullptr;  // the slot's pinned staging: xx in, results out
  hipEvent_t ev = nullptr;
};

bool same_params(const lagp_params& a, const lagp_params& b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

void free_host(Request& r) { std::vector<double>().swap(r.xx); }

size_t io_bytes(int64_t M, int p, int n) {
  return (size_t)M * (sizeof(double) * p + 3 * sizeof(double) + sizeof(int32_t) * n + sizeof(int32_t));
}

// A merged batch's per-location parameters as staged and uploaded after the
// locations: d and g (FP64), then n (int32), padded to 8 bytes.
size_t pl_stage_bytes(int64_t M) { return ((size_t)M * (2 * sizeof(double) + sizeof(int32_t)) + 7) & ~size_t(7); }

// Pinned staging of one slot: the largest batch's locations, per-location
// parameters and results.
size_t stage_bytes(int p) {
  return io_bytes(BATCH_MAX_LOCATIONS, p, LAGP_MAX_N) + pl_stage_bytes(BATCH_MAX_LOCATIONS) + 256;
}

}  // namespace

struct lagp_server {
  const lagp_design* design = nullptr;
  size_t budget = 0;
  size_t ws_cap = 0;
  int max_inflight = 1;
  std::vector<hipStream_t> streams;
  std::vector<bool> slot_busy;
  std::vector<char*> stage;  // pinned host staging per slot

  std::mutex mu;
  std::condition_variable cv_work;  // worker wake-up
  std::condition_variable cv_done;  // fetch wake-up
  std::deque<std::shared_ptr<Request>> waiting;
  std::map<uint64_t, std::shared_ptr<Request>> tickets;
  std::vector<Batch> inflight;
  size_t bytes_in_use = 0;
  int head_bypassed = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::string worker_error;

  // stats
  std::vector<double> lat_ms;
  int64_t preds_done = 0;
  clk::time_point t_first;
  clk::time_point t_last;
  bool have_first = false;

  std::thread worker;
};

namespace {

// Per-location parameters of a merged batch: n (int32), d and g (FP64).
size_t per_location_bytes(int64_t M) { return (size_t)M * (sizeof(int32_t) + 2 * sizeof(double)); }

size_t batch_device_bytes(const lagp_server* s, const lagp_params& P, int64_t M, bool merged) {
  const int p = s->design->p;
  return io_bytes(M, p, P.n) + (merged ? per_location_bytes(M) + 256 : 0) +
         lagp::predict_workspace_bytes(s->design, &P, false, M, s->ws_cap) + 4096;
}

// Requests that may share a batch whatever their n, d and g: exhaustive FP64
// search by Cholesky columns on chip with an isotropic lengthscale.
bool mergeable(const lagp_server* s, const lagp_params& P) {
  return P.search == LAGP_SEARCH_EXHAUSTIVE && P.precision == LAGP_PREC_FP64 && P.scoring == LAGP_SCORING_CHOL &&
         P.d_len == 1 && P.snap == LAGP_SNAP_CANDIDATES && lagp::chol_onchip_shape(s->design, P.n, P.ncand);
}

bool same_batch(const lagp_server* s, const lagp_params& a, const lagp_params& b) {
  if (same_params(a, b)) return true;
  if (!mergeable(s, a) || !mergeable(s, b)) return false;
  lagp_params x = a, y = b;  // equal but for n, d and g
  x.n = y.n = 0;
  x.d[0] = y.d[0] = 0.0;
  x.g = y.g = 0.0;
  return same_params(x, y);
}

// Called with the lock held: form the next batch from the waiting queue,
// starting at position `start`.
Batch form_batch(lagp_server* s, size_t start) {
  Batch b;
  auto& head = s->waiting[start];
  b.P = head->P;
  b.merged = mergeable(s, head->P);
  for (size_t i = start; i < s->waiting.size(); ++i) {
    auto& r = s->waiting[i];
    if (!same_batch(s, r->P, head->P)) continue;
    lagp_params P = b.P;
    P.n = std::max(P.n, r->P.n);
    // the first request alone always fits (checked at submit); growth stops
    // at the location cap or the budget, so a head batch can always run
    if (!b.reqs.empty() &&
        (b.M + r->M > BATCH_MAX_LOCATIONS || batch_device_bytes(s, P, b.M + r->M, b.merged) > s->budget))
      break;
    b.P = P;
    b.reqs.push_back(r);
    b.M += r->M;
  }
  b.bytes = batch_device_bytes(s, b.P, b.M, b.merged);
  return b;
}

void remove_from_waiting(lagp_server* s, const Batch& b) {
  for (auto& r : b.reqs) {
    auto it = std::find(s->waiting.begin(), s->waiting.end(), r);
    if (it != s->waiting.end()) s->waiting.erase(it);
  }
}

// Launch an admitted batch on its slot's stream (lock not held).
int32_t launch_batch(lagp_server* s, Batch& b) {
  const int p = s->design->p, n = b.P.n;
  const int64_t M = b.M;
  hipStream_t st = s->streams[b.slot];
  const size_t xb = sizeof(double) * (size_t)M * p, db = sizeof(double) * (size_t)M,
               sb = sizeof(int32_t) * (size_t)M * n, tb = sizeof(int32_t) * (size_t)M,
               plb = b.merged ? pl_stage_bytes(M) : 0;
  // (xb + plb + 3 db + sb + tb <= stage_bytes: M <= BATCH_MAX_LOCATIONS, n <= LAGP_MAX_N)
  b.host = s->stage[b.slot];
  char* h = b.host;
  double* hx = reinterpret_cast<double*>(h);
  double* hd = reinterpret_cast<double*>(h + xb);
  double* hg = hd + M;
  int32_t* hn = reinterpret_cast<int32_t*>(hg + M);
  int64_t off = 0;
  for (auto& r : b.reqs) {
    std::memcpy(hx + off * p, r->xx.data(), sizeof(double) * r->M * p);
    if (b.merged)
      for (int64_t i = 0; i < r->M; ++i) {
        hd[off + i] = r->P.d[0];
        hg[off + i] = r->P.g;
        hn[off + i] = r->P.n;
      }
    off += r->M;
  }
  if (hipMallocAsync(&b.dev, xb + plb + 3 * db + sb + tb, st) != hipSuccess) return LAGP_ENOMEM;
  char* dv = reinterpret_cast<char*>(b.dev);
  double* dx = reinterpret_cast<double*>(dv);
  double* dd = reinterpret_cast<double*>(dv + xb);
  double* dmean = reinterpret_cast<double*>(dv + xb + plb);
  double* ds2 = dmean + M;
  double* ddf = ds2 + M;
  int32_t* dsel = reinterpret_cast<int32_t*>(ddf + M);
  int32_t* dst = dsel + (size_t)M * n;
  if (hipMemcpyAsync(dx, hx, xb + plb, hipMemcpyHostToDevice, st) != hipSuccess) return LAGP_EDEVICE;
  const lagp::PerLocation pl{reinterpret_cast<const int32_t*>(dd + 2 * M), dd, dd + M};
  int32_t rc = lagp::run_predict(s->design, dx, M, nullptr, &b.P, dmean, ds2, ddf, dsel, nullptr, dst, st, s->ws_cap,
                                 nullptr, 0, nullptr, b.merged ? &pl : nullptr);
  if (rc < 0) return rc;
  if (hipMemcpyAsync(h + xb + plb, dmean, 3 * db + sb + tb, hipMemcpyDeviceToHost, st) != hipSuccess)
    return LAGP_EDEVICE;
  if (hipFreeAsync(b.dev, st) != hipSuccess) return LAGP_EDEVICE;
  b.dev = nullptr;
  if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) return LAGP_EDEVICE;
  if (hipEventRecord(b.ev, st) != hipSuccess) return LAGP_EDEVICE;
  return LAGP_OK;
}

// Copy a finished batch's results into its requests (lock held).
void finish_batch(lagp_server* s, Batch& b, int32_t rc) {
  const int p = s->design->p, n = b.P.n;
  const int64_t M = b.M;
  const size_t xb = sizeof(double) * (size_t)M * p, plb = b.merged ? pl_stage_bytes(M) : 0;
  const double* hmean = b.host ? reinterpret_cast<const double*>(b.host + xb + plb) : nullptr;
  const double* hs2 = hmean ? hmean + M : nullptr;
  const double* hdf = hs2 ? hs2 + M : nullptr;
  const int32_t* hsel = hdf ? reinterpret_cast<const int32_t*>(hdf + M) : nullptr;
  const int32_t* hst = hsel ? hsel + (size_t)M * n : nullptr;
  const auto now = clk::now();
  int64_t off = 0;
  for (auto& r : b.reqs) {
    const int64_t m = r->M;
    r->rc = rc;
    if (rc == LAGP_OK && hmean) {
      r->mean = new (std::nothrow) double[m];
      r->s2 = new (std::nothrow) double[m];
      r->df = new (std::nothrow) double[m];
      const int rn = r->P.n;  // (a merged batch's rows hold n of the batch: the largest)
      r->sel = new (std::nothrow) int32_t[(size_t)m * rn];
      r->status = new (std::nothrow) int32_t[m];
      if (r->mean && r->s2 && r->df && r->sel && r->status) {
        std::memcpy(r->mean, hmean + off, sizeof(double) * m);
        std::memcpy(r->s2, hs2 + off, sizeof(double) * m);
        std::memcpy(r->df, hdf + off, sizeof(double) * m);
        for (int64_t i = 0; i < m; ++i)
          std::memcpy(r->sel + i * rn, hsel + (off + i) * n, sizeof(int32_t) * rn);
        std::memcpy(r->status, hst + off, sizeof(int32_t) * m);
        for (int64_t i = 0; i < m; ++i)
          if (r->status[i] != 0) r->rc = LAGP_WARN_NUMERIC;
      } else {
        r->rc = LAGP_ENOMEM;
      }
    }
    off += m;
    r->latency_ms = std::chrono::duration<double, std::milli>(now - r->t_submit).count();
    r->done = true;
    free_host(*r);
    s->lat_ms.push_back(r->latency_ms);
    s->preds_done += m;
    s->t_last = now;
  }
  (void)p;
  b.host = nullptr;  // (the slot's staging, kept for its next batch)
  if (b.ev) (void)hipEventDestroy(b.ev);
  b.ev = nullptr;
  s->bytes_in_use -= b.bytes;
  s->slot_busy[b.slot] = false;
}

void worker_main(lagp_server* s) {
  (void)hipSetDevice(s->design->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // 1. retire finished batches
    for (size_t i = 0; i < s->inflight.size();) {
      hipError_t q = hipEventQuery(s->inflight[i].ev);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      finish_batch(s, s->inflight[i], q == hipSuccess ? LAGP_OK : LAGP_EDEVICE);
      s->inflight.erase(s->inflight.begin() + i);
      s->cv_done.notify_all();
    }
    if (s->stop && s->waiting.empty() && s->inflight.empty()) break;
    // 2. admit: the head batch first; smaller later batches may bypass a
    //    blocked head a bounded number of times
    bool launched = false;
    bool head_blocked = false;  // the head batch did not fit on this pass
    for (size_t start = 0; start < s->waiting.size();) {
      int slot = -1;
      for (int k = 0; k < s->max_inflight; ++k)
        if (!s->slot_busy[k]) {
          slot = k;
          break;
        }
      if (slot < 0) break;
      Batch b = form_batch(s, start);
      if (s->bytes_in_use + b.bytes > s->budget) {
        if (start == 0 && s->head_bypassed >= HEAD_BYPASS_LIMIT) break;
        // look for a later batch with other parameters
        size_t nxt = start + 1;
        while (nxt < s->waiting.size() && same_batch(s, s->waiting[nxt]->P, s->waiting[start]->P)) ++nxt;
        if (start == 0) head_blocked = true;
        start = nxt;
        continue;
      }
      // a bypass counts only when a later batch is actually launched ahead
      // of a blocked head
      if (start == 0) s->head_bypassed = 0;
      else if (head_blocked) ++s->head_bypassed;
      remove_from_waiting(s, b);
      b.slot = slot;
      s->slot_busy[slot] = true;
      s->bytes_in_use += b.bytes;
      lk.unlock();
      const int32_t rc = launch_batch(s, b);
      lk.lock();
      if (rc != LAGP_OK) {
        // drain what was queued: the slot's staging is reused by its next batch
        (void)hipStreamSynchronize(s->streams[slot]);
        if (b.dev) (void)hipFree(b.dev);
        b.dev = nullptr;
        finish_batch(s, b, rc);
        s->cv_done.notify_all();
      } else {
        s->inflight.push_back(b);
      }
      launched = true;
      head_blocked = false;
      start = 0;
    }
    if (!launched) {
      if (s->inflight.empty() && s->waiting.empty() && !s->stop)
        s->cv_work.wait(lk);
      else
        s->cv_work.wait_for(lk, std::chrono::microseconds(50));
    }
  }
}

int32_t server_fail(int32_t code, const char* msg) {
  lagp::set_error(msg);
  return code;
}

}  // namespace

extern "C" {

int32_t lagp_server_create(const lagp_design* design, size_t hbm_budget_bytes, int32_t max_inflight,
                           lagp_server** out) {
  if (!out) return server_fail(LAGP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!design) return server_fail(LAGP_EINVAL, "design is NULL");
  if (max_inflight < 1 || max_inflight > 64) return server_fail(LAGP_EINVAL, "max_inflight must be in [1, 64]");
  if (hbm_budget_bytes < ((size_t)1 << 20)) return server_fail(LAGP_EINVAL, "hbm budget must be at least 1 MiB");
  lagp_server* s = new (std::nothrow) lagp_server();
  if (!s) return server_fail(LAGP_ENOMEM, "host allocation failed");
  s->design = design;
  s->budget = hbm_budget_bytes;
  s->max_inflight = max_inflight;
  s->ws_cap = std::max<size_t>(hbm_budget_bytes / (size_t)max_inflight, (size_t)1 << 20);
  if (hipSetDevice(design->device) != hipSuccess) {
    delete s;
    return server_fail(LAGP_EDEVICE, "hipSetDevice failed");
  }
  s->streams.resize(max_inflight, nullptr);
  s->slot_busy.assign(max_inflight, false);
  s->stage.assign(max_inflight, nullptr);
  for (int k = 0; k < max_inflight; ++k) {
    if (hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->stage[k]), stage_bytes(design->p), hipHostMallocDefault) !=
            hipSuccess) {
      for (auto st : s->streams)
        if (st) (void)hipStreamDestroy(st);
      for (auto h : s->stage)
        if (h) (void)hipHostFree(h);
      delete s;
      return server_fail(LAGP_EDEVICE, "stream or pinned staging creation failed");
    }
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return LAGP_OK;
}

int32_t lagp_server_submit(lagp_server* s, const double* XX_host, int64_t M, const lagp_params* P,
                           uint64_t* ticket) {
  if (!s || !P || !ticket) return server_fail(LAGP_EINVAL, "server, params and ticket must not be NULL");
  if (M < 1) return server_fail(LAGP_EINVAL, "M must be >= 1");
  if (!XX_host) return server_fail(LAGP_EINVAL, "XX_host is NULL");
  int32_t rc = lagp::check_predict_params(s->design, P);
  if (rc != LAGP_OK) return rc;
  if (M > BATCH_MAX_LOCATIONS) return server_fail(LAGP_EINVAL, "a request may hold at most 4096 locations");
  const size_t need = batch_device_bytes(s, *P, M, mergeable(s, *P));
  if (need > s->budget) return server_fail(LAGP_ENOMEM, "request can never fit the server's HBM budget");
  auto r = std::make_shared<Request>();
  r->P = *P;
  r->M = M;
  r->p = s->design->p;
  r->xx.assign(XX_host, XX_host + (size_t)M * r->p);
  r->t_submit = clk::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      free_host(*r);
      return server_fail(LAGP_EINVAL, "server is shutting down");
    }
    if (s->waiting.size() >= WAITING_MAX) {
      free_host(*r);
      return server_fail(LAGP_EAGAIN, "server queue is full");
    }
    r->ticket = s->next_ticket++;
    s->waiting.push_back(r);
    s->tickets[r->ticket] = r;
    if (!s->have_first) {
      s->have_first = true;
      s->t_first = r->t_submit;
    }
    *ticket = r->ticket;
  }
  s->cv_work.notify_one();
  return LAGP_OK;
}

int32_t lagp_server_poll(lagp_server* s, uint64_t ticket, int32_t* done) {
  if (!s || !done) return server_fail(LAGP_EINVAL, "server and done must not be NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return server_fail(LAGP_EINVAL, "unknown ticket");
  *done = it->second->done ? 1 : 0;
  return LAGP_OK;
}

int32_t lagp_server_fetch(lagp_server* s, uint64_t ticket, double* mean, double* s2, double* df, int32_t* sel_idx,
                          int32_t* status, double* latency_ms) {
  if (!s) return server_fail(LAGP_EINVAL, "server is NULL");
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return server_fail(LAGP_EINVAL, "unknown ticket");
    r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    s->tickets.erase(it);
  }
  const int64_t m = r->M;
  const int n = r->P.n;
  if (r->mean) {
    if (mean) std::memcpy(mean, r->mean, sizeof(double) * m);
    if (s2) std::memcpy(s2, r->s2, sizeof(double) * m);
    if (df) std::memcpy(df, r->df, sizeof(double) * m);
    if (sel_idx) std::memcpy(sel_idx, r->sel, sizeof(int32_t) * m * n);
    if (status) std::memcpy(status, r->status, sizeof(int32_t) * m);
  }
  if (latency_ms) *latency_ms = r->latency_ms;
  delete[] r->mean;
  delete[] r->s2;
  delete[] r->df;
  delete[] r->sel;
  delete[] r->status;
  r->mean = r->s2 = r->df = nullptr;
  r->sel = r->status = nullptr;
  if (r->rc < 0) return server_fail(r->rc, "request failed on the device");
  return r->rc;
}

int32_t lagp_server_stats(lagp_server* s, double* p50_ms, double* p99_ms, double* pred_per_s, int32_t reset) {
  if (!s) return server_fail(LAGP_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<double> v = s->lat_ms;
  std::sort(v.begin(), v.end());
  auto pct = [&](double q) {
    if (v.empty()) return 0.0;
    const size_t k = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
    return v[k];
  };
  if (p50_ms) *p50_ms = pct(0.50);
  if (p99_ms) *p99_ms = pct(0.99);
  if (pred_per_s) {
    const double secs = s->have_first ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
    *pred_per_s = secs > 0.0 ? (double)s->preds_done / secs : 0.0;
  }
  if (reset) {
    s->lat_ms.clear();
    s->preds_done = 0;
    s->have_first = false;
  }
  return LAGP_OK;
}

void lagp_server_destroy(lagp_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->tickets) {
    Request& r = *kv.second;
    free_host(r);
    delete[] r.mean;
    delete[] r.s2;
    delete[] r.df;
    delete[] r.sel;
    delete[] r.status;
  }
  for (auto st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  for (auto h : s->stage)
    if (h) (void)hipHostFree(h);
  delete s;
}

}  // extern "C"

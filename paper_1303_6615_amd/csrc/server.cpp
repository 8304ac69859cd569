// Serving loop over the library's C ABI: requests (one parareal solve each,
// Alg. 4) are admitted by their HBM footprint, batched by arrival and run as
// persistent batched launches on several streams, so that work admitted
// while earlier batches are still on the device overlaps with them
// (continuous batching).  One worker thread owns every context and stream;
// submit and poll only touch the request table under the server's lock.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/aparareal.h"
#include "launch.hpp"

namespace aplib {
void set_last_error(const std::string& msg);   // host.cpp: the message of aparareal_last_error
}

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kStreams = 4;         // batches in flight at once
constexpr int kMaxBatch = 64;       // requests per batched launch
constexpr int kPoolPerKey = 8;      // idle contexts kept per (N, eps, F, nu)

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Device bytes one request holds while it runs: its states at every
// iteration level (U, G: K+1 levels, F: K levels, modal FP64), the split
// averages' group sums, counters and residual parts, coefficient tables,
// its physical input/output and the job list of its launch.
size_t footprint(int N, const ap_solve_params& p) {
  const size_t KP = size_t(N / 3 + 1);
  const size_t st = 3 * KP * 16;
  const size_t Ns = size_t(p.slices), K = size_t(p.K);
  const size_t gs_bytes = p.precision == AP_PREC_FP64 ? 16 : 8;
  size_t b = st * (Ns + 1) * (2 * (K + 1) + std::max<size_t>(K, 1));
  b += 2 * (K + 1) * size_t(p.M_avg) * 3 * KP * gs_bytes;       // group sums (groups <= M)
  b += size_t(ap::pipe_counters(int(Ns), int(K))) * 4 + K * Ns * 16;   // counters, residual parts
  b += 2 * 8 * 3 * KP * 16 + size_t(p.M_avg) * KP * 24 + KP * 64; // tables
  b += 3 * size_t(N) * 8 * (Ns + 2) + K * 8;                     // u0, U_out, resid
  b += ((2 * K + 1) * Ns * size_t(2 * p.M_avg + 1)) * 20;       // job list
  return b + (size_t(1) << 16);
}

struct Request {
  unsigned long long ticket = 0;
  int N = 0;
  double eps = 0, F = 0, nu = 0;
  ap_solve_params p{};
  std::vector<double> u0, U, resid;
  size_t bytes = 0;
  Clock::time_point t_submit, t_done;
  enum { kQueued, kRunning, kDone, kFailed } state = kQueued;
  int err = AP_OK;
  std::string msg;
  // device side (worker thread only)
  ap_ctx* ctx = nullptr;
  double *d_u0 = nullptr, *d_U = nullptr, *d_r = nullptr;
};

struct Batch {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  std::vector<Request*> reqs;
  bool busy = false;
};

}  // namespace

struct ap_server {
  size_t budget = 0, used = 0;
  int max_slots = 0, running = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;                                 // submitted, not admitted
  std::map<unsigned long long, std::unique_ptr<Request>> reqs;
  unsigned long long next_ticket = 1;
  bool stop = false;
  std::thread worker;
  // worker-owned
  Batch batches[kStreams];
  std::map<std::tuple<int, double, double, double>, std::vector<ap_ctx*>> ctx_pool;
  std::multimap<size_t, void*> buf_pool;                      // free device buffers by size
  std::vector<void*> all_bufs;
  // statistics
  unsigned long long completed = 0, failed = 0, launches = 0;
  size_t peak = 0;
};

namespace {

int serve_fail(int code, const std::string& m) {
  aplib::set_last_error(m);
  return code;
}

void* take_buf(ap_server* sv, size_t bytes) {
  size_t cls = 4096;
  while (cls < bytes) cls <<= 1;
  auto it = sv->buf_pool.find(cls);
  if (it != sv->buf_pool.end()) {
    void* p = it->second;
    sv->buf_pool.erase(it);
    return p;
  }
  void* p = nullptr;
  if (hipMalloc(&p, cls) != hipSuccess) return nullptr;
  sv->all_bufs.push_back(p);
  return p;
}

void give_buf(ap_server* sv, void* p, size_t bytes) {
  if (!p) return;
  size_t cls = 4096;
  while (cls < bytes) cls <<= 1;
  sv->buf_pool.emplace(cls, p);
}

ap_ctx* take_ctx(ap_server* sv, const Request& r) {
  auto key = std::make_tuple(r.N, r.eps, r.F, r.nu);
  auto& v = sv->ctx_pool[key];
  if (!v.empty()) {
    ap_ctx* c = v.back();
    v.pop_back();
    return c;
  }
  // Batches of requests fill the GPU with independent jobs, so a coarse step
  // runs in one workgroup (AP_OPT_SPLIT 0): fewer, longer jobs, and a job
  // graph the host schedules in a few milliseconds instead of tens (values
  // are unchanged; measured 163 against 98-107 solves/s closed loop).
  ap_ctx* c = aparareal_create(r.N, r.eps, r.F, r.nu);
  if (c) (void)aparareal_set_option(c, AP_OPT_SPLIT, 0);
  return c;
}

void give_ctx(ap_server* sv, const Request& r, ap_ctx* c) {
  if (!c) return;
  auto& v = sv->ctx_pool[std::make_tuple(r.N, r.eps, r.F, r.nu)];
  if (int(v.size()) < kPoolPerKey)
    v.push_back(c);
  else
    aparareal_destroy(c);
}

void release_device(ap_server* sv, Request* r) {
  give_buf(sv, r->d_u0, 3 * size_t(r->N) * 8);
  give_buf(sv, r->d_U, size_t(r->p.slices + 1) * 3 * r->N * 8);
  give_buf(sv, r->d_r, size_t(std::max(r->p.K, 1)) * 8);
  give_ctx(sv, *r, r->ctx);
  r->d_u0 = r->d_U = r->d_r = nullptr;
  r->ctx = nullptr;
}

// Marks a request finished (under the lock) and returns its memory.
void finish(ap_server* sv, Request* r, int err, const std::string& msg) {
  std::lock_guard<std::mutex> lk(sv->mu);
  r->t_done = Clock::now();
  r->err = err;
  r->msg = msg;
  r->state = err == AP_OK ? Request::kDone : Request::kFailed;
  sv->used -= r->bytes;
  sv->running -= 1;
  if (err == AP_OK)
    sv->completed += 1;
  else
    sv->failed += 1;
  sv->cv.notify_all();
}

// Starts one batch of admitted requests (same precision) on a free stream.
void launch_batch(ap_server* sv, Batch& b, std::vector<Request*>& group) {
  std::vector<ap_batch_item> items;
  std::vector<Request*> ok;
  for (Request* r : group) {
    r->ctx = take_ctx(sv, *r);
    r->d_u0 = static_cast<double*>(take_buf(sv, 3 * size_t(r->N) * 8));
    r->d_U = static_cast<double*>(take_buf(sv, size_t(r->p.slices + 1) * 3 * r->N * 8));
    r->d_r = static_cast<double*>(take_buf(sv, size_t(std::max(r->p.K, 1)) * 8));
    if (!r->ctx || !r->d_u0 || !r->d_U || !r->d_r) {
      release_device(sv, r);
      finish(sv, r, AP_ENOMEM, "device allocation for the request failed");
      continue;
    }
    if (hipMemcpyAsync(r->d_u0, r->u0.data(), r->u0.size() * 8, hipMemcpyHostToDevice, b.stream) != hipSuccess) {
      release_device(sv, r);
      finish(sv, r, AP_EDEVICE, "input copy failed");
      continue;
    }
    items.push_back(ap_batch_item{r->ctx, r->d_u0, r->p, r->d_U, r->d_r});
    ok.push_back(r);
  }
  if (ok.empty()) return;
  const int rc = aparareal_solve_batch(items.data(), int(items.size()), b.stream);
  if (rc != AP_OK) {
    const std::string m = aparareal_last_error();
    (void)hipStreamSynchronize(b.stream);
    for (Request* r : ok) {
      release_device(sv, r);
      finish(sv, r, rc, m);
    }
    return;
  }
  (void)hipEventRecord(b.done, b.stream);
  b.reqs = ok;
  b.busy = true;
  sv->launches += 1;
}

// Copies the results of a finished batch to the requests' host buffers.
void complete_batch(ap_server* sv, Batch& b) {
  for (Request* r : b.reqs) {
    r->U.resize(size_t(r->p.slices + 1) * 3 * r->N);
    r->resid.resize(size_t(r->p.K));
    hipError_t e = hipMemcpyAsync(r->U.data(), r->d_U, r->U.size() * 8, hipMemcpyDeviceToHost, b.stream);
    if (e == hipSuccess && r->p.K > 0)
      e = hipMemcpyAsync(r->resid.data(), r->d_r, r->resid.size() * 8, hipMemcpyDeviceToHost, b.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
    int err = e == hipSuccess ? AP_OK : AP_EDEVICE;
    std::string msg = e == hipSuccess ? "" : hipGetErrorString(e);
    if (err == AP_OK)
      for (double v : r->resid)
        if (!std::isfinite(v)) {
          err = AP_ENUMERIC;
          msg = "non-finite residual (pipeline stall or numerical blow-up)";
          break;
        }
    release_device(sv, r);
    finish(sv, r, err, msg);
  }
  b.reqs.clear();
  b.busy = false;
}

void worker_main(ap_server* sv) {
  (void)hipSetDevice(sv->device);
  for (;;) {
    // finished batches
    for (Batch& b : sv->batches)
      if (b.busy && hipEventQuery(b.done) == hipSuccess) complete_batch(sv, b);
    // admit queued requests in arrival order while memory and slots allow
    std::vector<Request*> admitted;
    bool idle;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      int free_streams = 0;
      for (Batch& b : sv->batches) free_streams += b.busy ? 0 : 1;
      while (free_streams > 0 && !sv->queue.empty() && int(admitted.size()) < kMaxBatch) {
        Request* r = sv->queue.front();
        if (sv->running >= sv->max_slots || sv->used + r->bytes > sv->budget) break;
        sv->queue.pop_front();
        sv->used += r->bytes;
        sv->peak = std::max(sv->peak, sv->used);
        sv->running += 1;
        r->state = Request::kRunning;
        admitted.push_back(r);
      }
      bool any_busy = false;
      for (Batch& b : sv->batches) any_busy = any_busy || b.busy;
      if (sv->stop && sv->queue.empty() && admitted.empty() && !any_busy) return;
      idle = admitted.empty();
      if (idle) {
        // nothing to start: wait for a submission, or poll the device soon
        sv->cv.wait_for(lk, any_busy ? std::chrono::microseconds(100) : std::chrono::milliseconds(5));
        continue;
      }
    }
    // one batch per precision present, each on its own free stream
    for (int prec = 0; prec <= 1; ++prec) {
      std::vector<Request*> group;
      for (Request* r : admitted)
        if (r->p.precision == prec) group.push_back(r);
      if (group.empty()) continue;
      Batch* free_b = nullptr;
      for (Batch& b : sv->batches)
        if (!b.busy) {
          free_b = &b;
          break;
        }
      if (!free_b) {
        // every stream busy: finish one batch first
        for (;;) {
          for (Batch& b : sv->batches)
            if (b.busy && hipEventQuery(b.done) == hipSuccess) {
              complete_batch(sv, b);
              free_b = &b;
              break;
            }
          if (free_b) break;
          std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
      }
      launch_batch(sv, *free_b, group);
    }
  }
}

int check_params(int N, double eps, double F, double nu, const ap_solve_params* p) {
  if (!pow2(N) || N < 64 || N > 2048) return serve_fail(AP_EINVAL, "N must be a power of two in [64, 2048]");
  if (!(eps > 0.0) || !(F > 0.0) || !(nu >= 0.0) || !std::isfinite(eps) || !std::isfinite(F) || !std::isfinite(nu))
    return serve_fail(AP_EINVAL, "need eps > 0, F > 0, nu >= 0 (finite)");
  if (!p) return serve_fail(AP_EINVAL, "null parameters");
  if (p->precision != AP_PREC_FP32 && p->precision != AP_PREC_FP64) return serve_fail(AP_EINVAL, "bad precision");
  if (!(p->T > 0.0) || !std::isfinite(p->T) || p->slices < 1 || p->K < 0 || p->M_avg < 2 ||
      !(p->dt_fine > 0.0) || !std::isfinite(p->dt_fine) || !std::isfinite(p->T0))
    return serve_fail(AP_EINVAL, "bad solve parameters");
  if (p->T / p->slices / p->dt_fine > 1e7) return serve_fail(AP_EINVAL, "dT/dt_fine too large");
  if (size_t(2 * p->K + 1) * size_t(p->slices) > (size_t(1) << 26)) return serve_fail(AP_EINVAL, "problem too large");
  return AP_OK;
}

}  // namespace

extern "C" {

ap_server* aparareal_serve_create(size_t hbm_budget_bytes, int max_slots) {
  if (hbm_budget_bytes == 0 || max_slots < 1) {
    serve_fail(AP_EINVAL, "need a positive HBM budget and max_slots >= 1");
    return nullptr;
  }
  auto sv = std::make_unique<ap_server>();
  sv->budget = hbm_budget_bytes;
  sv->max_slots = max_slots;
  if (hipGetDevice(&sv->device) != hipSuccess) {
    serve_fail(AP_EDEVICE, "hipGetDevice failed");
    return nullptr;
  }
  for (Batch& b : sv->batches) {
    // default priority; non-blocking so that the library's synchronous table
    // uploads do not wait for running batches
    if (hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) {
      serve_fail(AP_EDEVICE, "stream creation failed");
      for (Batch& x : sv->batches) {
        if (x.stream) (void)hipStreamDestroy(x.stream);
        if (x.done) (void)hipEventDestroy(x.done);
      }
      return nullptr;
    }
  }
  ap_server* raw = sv.release();
  raw->worker = std::thread(worker_main, raw);
  return raw;
}

int aparareal_serve_submit(ap_server* sv, int N, double eps, double F, double nu, const double* u0,
                           const ap_solve_params* params, unsigned long long* ticket) {
  if (!sv) return serve_fail(AP_EINVAL, "null server");
  if (!u0 || !ticket) return serve_fail(AP_EINVAL, "null argument");
  int rc = check_params(N, eps, F, nu, params);
  if (rc) return rc;
  auto r = std::make_unique<Request>();
  r->N = N;
  r->eps = eps;
  r->F = F;
  r->nu = nu;
  r->p = *params;
  r->u0.assign(u0, u0 + 3 * size_t(N));
  r->bytes = footprint(N, *params);
  if (r->bytes > sv->budget) return serve_fail(AP_ENOMEM, "request exceeds the server's HBM budget");
  r->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stop) return serve_fail(AP_EBUSY, "server shutting down");
  r->ticket = sv->next_ticket++;
  *ticket = r->ticket;
  sv->queue.push_back(r.get());
  sv->reqs[r->ticket] = std::move(r);
  sv->cv.notify_all();
  return AP_OK;
}

int aparareal_serve_poll(ap_server* sv, unsigned long long ticket, double* U_out, double* resid, double* latency_s) {
  if (!sv) return serve_fail(AP_EINVAL, "null server");
  std::unique_ptr<Request> r;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return serve_fail(AP_ENOTFOUND, "unknown ticket");
    Request* q = it->second.get();
    if (q->state == Request::kQueued || q->state == Request::kRunning) return AP_PENDING;
    r = std::move(it->second);
    sv->reqs.erase(it);
  }
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  if (r->state == Request::kFailed) return serve_fail(r->err, r->msg);
  if (U_out) std::memcpy(U_out, r->U.data(), r->U.size() * 8);
  if (resid && !r->resid.empty()) std::memcpy(resid, r->resid.data(), r->resid.size() * 8);
  return AP_OK;
}

int aparareal_serve_stats(ap_server* sv, unsigned long long* out) {
  if (!sv || !out) return serve_fail(AP_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  out[0] = sv->completed;
  out[1] = sv->failed;
  out[2] = sv->queue.size();
  out[3] = (unsigned long long)sv->running;
  out[4] = sv->launches;
  out[5] = sv->used;
  out[6] = sv->peak;
  return AP_OK;
}

int aparareal_serve_destroy(ap_server* sv) {
  if (!sv) return serve_fail(AP_EINVAL, "null server");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv.notify_all();
  }
  if (sv->worker.joinable()) sv->worker.join();
  for (auto& kv : sv->ctx_pool)
    for (ap_ctx* c : kv.second) aparareal_destroy(c);
  for (void* p : sv->all_bufs) (void)hipFree(p);
  for (Batch& b : sv->batches) {
    (void)hipStreamDestroy(b.stream);
    (void)hipEventDestroy(b.done);
  }
  delete sv;
  return AP_OK;
}

}  // extern "C"

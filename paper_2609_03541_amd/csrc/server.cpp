// Batched serving: continuous batching of independent MBAR problems on one
// device (the C ABI declared in include/bumbar.h).
//
// Memory: one arena of hbm_budget_bytes is reserved at creation and handed
// out first-fit (256-byte aligned) to admitted requests; a request's
// footprint is its resident u_kn (if it carries one; a model request keeps
// only its coordinates, the energies being evaluated inside the kernels)
// plus inputs plus the workspace bumbar_solve asks for. Admission is strictly in arrival order: a free slot takes the
// oldest queued request as soon as its footprint fits, so a large request is
// not overtaken indefinitely. Each slot owns a HIP stream (default priority)
// and a library context; slots run in their own host threads, so the
// kernels of different problems overlap on the device while every problem is
// solved by exactly the kernels of bumbar_solve (identical results alone and
// in the mix). Latency = completion time - submission time (host clock).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "bumbar.h"
#include "bumbar_impl.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, cap) (host bookkeeping of the device arena).
class ArenaAllocator {
 public:
  explicit ArenaAllocator(size_t cap) : cap_(cap) { free_[0] = cap; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    // merge with the following and the preceding free blocks
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t peak() const { return peak_; }

 private:
  size_t cap_;
  size_t used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> size
};

struct Job {
  uint64_t ticket = 0;
  bumbar_request req{};
  size_t footprint = 0;
  size_t ws_bytes = 0;
  Clock::time_point t_submit, t_done;
  int state = BUMBAR_TICKET_QUEUED;
  int status = BUMBAR_OK;
  std::vector<double> f;
  bumbar_stats stats{};
};

}  // namespace

struct bumbar_server {
  bumbar_server_options opt{};
  char* arena = nullptr;
  std::unique_ptr<ArenaAllocator> alloc;
  std::mutex mu;
  std::condition_variable cv_admit;  // queue or memory changed
  std::condition_variable cv_done;   // a ticket finished
  std::deque<std::shared_ptr<Job>> queue;
  std::map<uint64_t, std::shared_ptr<Job>> jobs;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;  // one per slot, default priority
  std::vector<bumbar_ctx*> ctxs;
  uint64_t next_ticket = 1;
  bool stop = false;
  int64_t active = 0, peak_active = 0, completed = 0;
  // workspace sizing uses a context that is never used for work
  bumbar_ctx* sizing_ctx = nullptr;
};

namespace {

size_t footprint_of(bumbar_server* srv, const bumbar_request& r, size_t* ws_out) {
  size_t ws = 0;
  if (r.u_kn) {
    const int dq = (r.opt.binning && r.xi) ? r.d : 0;
    bumbar_query_workspace(srv->sizing_ctx, r.K, r.N, dq, &r.opt, &ws);
  } else {
    bumbar_query_workspace_model(srv->sizing_ctx, r.K, r.N, r.d, &r.opt, &ws);
  }
  *ws_out = ws;
  size_t b = 0;
  if (r.u_kn) b += align_up(sizeof(double) * (size_t)r.K * (size_t)r.N);  // resident u_kn
  if (r.xi) b += align_up(sizeof(double) * (size_t)r.N * (size_t)r.d);
  b += align_up(sizeof(int64_t) * (size_t)r.K);
  if (r.coef) b += align_up(sizeof(double) * (size_t)r.K * (size_t)(1 + 2 * r.d));
  b += align_up(sizeof(double) * (size_t)r.K);  // f
  b += align_up(ws);
  return b;
}

void run_job(bumbar_ctx* ctx, hipStream_t stream, char* base, Job& job) {
  const bumbar_request& r = job.req;
  char* p = base;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += align_up(bytes);
    return q;
  };
  double* u =
      r.u_kn ? reinterpret_cast<double*>(take(sizeof(double) * (size_t)r.K * (size_t)r.N)) : nullptr;
  double* xi = r.xi ? reinterpret_cast<double*>(take(sizeof(double) * (size_t)r.N * r.d)) : nullptr;
  int64_t* nk = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (size_t)r.K));
  double* coef =
      r.coef ? reinterpret_cast<double*>(take(sizeof(double) * (size_t)r.K * (1 + 2 * r.d)))
             : nullptr;
  double* f = reinterpret_cast<double*>(take(sizeof(double) * (size_t)r.K));
  void* ws = take(job.ws_bytes);
  hipError_t e = hipSuccess;
  if (r.u_kn)
    e = hipMemcpyAsync(u, r.u_kn, sizeof(double) * (size_t)r.K * (size_t)r.N,
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && r.xi)
    e = hipMemcpyAsync(xi, r.xi, sizeof(double) * (size_t)r.N * r.d, hipMemcpyHostToDevice,
                       stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(nk, r.N_k, sizeof(int64_t) * (size_t)r.K, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && r.coef)
    e = hipMemcpyAsync(coef, r.coef, sizeof(double) * (size_t)r.K * (1 + 2 * r.d),
                       hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) {
    job.status = BUMBAR_EDEVICE;
    return;
  }
  // a request without u_kn is solved with the energies evaluated from the
  // model inside the kernels (u_kn = NULL in bumbar_solve)
  const int dq = r.xi ? r.d : 0;
  job.stats.checks = nullptr;
  job.stats.checks_capacity = 0;
  job.status = bumbar_solve(ctx, u, BUMBAR_F64, r.K, r.N, nk, dq ? xi : nullptr, dq, r.model,
                            coef, nullptr, &r.opt, ws, job.ws_bytes, f, nullptr, nullptr,
                            &job.stats);
  job.f.assign(r.K, 0.0);
  if (hipMemcpyAsync(job.f.data(), f, sizeof(double) * r.K, hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    if (job.status == BUMBAR_OK) job.status = BUMBAR_EDEVICE;
  }
}

void worker_main(bumbar_server* srv, int slot) {
  (void)hipSetDevice(srv->opt.device);
  hipStream_t stream = srv->streams[slot];
  bumbar_ctx* ctx = srv->ctxs[slot];
  for (;;) {
    std::shared_ptr<Job> job;
    size_t off = 0;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv_admit.wait(lk, [&] {
        if (srv->stop) return true;
        if (srv->queue.empty()) return false;
        return srv->alloc->alloc(srv->queue.front()->footprint, &off);
      });
      if (srv->stop && srv->queue.empty()) break;
      if (srv->stop) {
        // drain: jobs still queued at shutdown fail without running
        for (auto& j : srv->queue) {
          j->state = BUMBAR_TICKET_FAILED;
          j->status = BUMBAR_EBUSY;
        }
        srv->queue.clear();
        srv->cv_done.notify_all();
        break;
      }
      job = srv->queue.front();
      srv->queue.pop_front();
      job->state = BUMBAR_TICKET_RUNNING;
      srv->active++;
      srv->peak_active = std::max(srv->peak_active, srv->active);
    }
    run_job(ctx, stream, srv->arena + off, *job);
    // whatever path run_job left by, no copy or kernel of this job may still
    // touch its arena block once the block is handed to another request
    if (hipStreamSynchronize(stream) != hipSuccess && job->status == BUMBAR_OK)
      job->status = BUMBAR_EDEVICE;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->alloc->release(off, job->footprint);
      job->t_done = Clock::now();
      job->state = (job->status == BUMBAR_OK || job->status == BUMBAR_ENOTCONV)
                       ? BUMBAR_TICKET_DONE
                       : BUMBAR_TICKET_FAILED;
      srv->active--;
      srv->completed++;
    }
    srv->cv_admit.notify_all();
    srv->cv_done.notify_all();
  }
}

// Frees the slots, the sizing context and the arena, then the server.
void release_slots(bumbar_server* srv) {
  for (bumbar_ctx* c : srv->ctxs) bumbar_destroy(c);
  for (hipStream_t st : srv->streams) (void)hipStreamDestroy(st);
  bumbar_destroy(srv->sizing_ctx);
  (void)hipFree(srv->arena);
  delete srv;
}

}  // namespace

extern "C" {

int bumbar_server_create(const bumbar_server_options* opt, bumbar_server** out) {
  if (!opt || !out || opt->max_active < 1 || opt->hbm_budget_bytes < kAlign) return BUMBAR_EINVAL;
  *out = nullptr;
  auto* srv = new (std::nothrow) bumbar_server();
  if (!srv) return BUMBAR_ENOMEM;
  srv->opt = *opt;
  if (hipSetDevice(opt->device) != hipSuccess) {
    delete srv;
    return BUMBAR_EDEVICE;
  }
  if (hipMalloc(&srv->arena, opt->hbm_budget_bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete srv;
    return BUMBAR_ENOMEM;
  }
  if (bumbar_create(&srv->sizing_ctx, opt->device, nullptr) != BUMBAR_OK) {
    (void)hipFree(srv->arena);
    delete srv;
    return BUMBAR_EDEVICE;
  }
  srv->alloc.reset(new ArenaAllocator(opt->hbm_budget_bytes));
  for (int i = 0; i < opt->max_active; ++i) {
    hipStream_t st = nullptr;
    bumbar_ctx* c = nullptr;
    if (hipStreamCreate(&st) != hipSuccess || bumbar_create(&c, opt->device, st) != BUMBAR_OK) {
      if (st) (void)hipStreamDestroy(st);
      (void)hipGetLastError();
      release_slots(srv);
      return BUMBAR_EDEVICE;
    }
    srv->streams.push_back(st);
    srv->ctxs.push_back(c);
  }
  for (int i = 0; i < opt->max_active; ++i) srv->workers.emplace_back(worker_main, srv, i);
  *out = srv;
  return BUMBAR_OK;
}

int bumbar_server_submit(bumbar_server* srv, const bumbar_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket || req->K <= 0 || req->N <= 0 || !req->N_k) return BUMBAR_EINVAL;
  if (!req->u_kn && (req->model == BUMBAR_MODEL_NONE || !req->xi || !req->coef))
    return BUMBAR_EINVAL;
  auto job = std::make_shared<Job>();
  job->req = *req;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return BUMBAR_EBUSY;
    // the sizing context is shared by submitting threads
    job->footprint = footprint_of(srv, *req, &job->ws_bytes);
    if (job->footprint > srv->opt.hbm_budget_bytes) return BUMBAR_ETOOBIG;
    job->t_submit = Clock::now();
    job->ticket = srv->next_ticket++;
    srv->jobs[job->ticket] = job;
    srv->queue.push_back(job);
    *ticket = job->ticket;
  }
  srv->cv_admit.notify_all();
  return BUMBAR_OK;
}

int bumbar_server_poll(bumbar_server* srv, uint64_t ticket, int* state) {
  if (!srv || !state) return BUMBAR_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(ticket);
  if (it == srv->jobs.end()) return BUMBAR_EINVAL;
  *state = it->second->state;
  return BUMBAR_OK;
}

int bumbar_server_wait(bumbar_server* srv, uint64_t ticket) {
  if (!srv) return BUMBAR_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(ticket);
  if (it == srv->jobs.end()) return BUMBAR_EINVAL;
  auto job = it->second;
  srv->cv_done.wait(lk, [&] {
    return job->state == BUMBAR_TICKET_DONE || job->state == BUMBAR_TICKET_FAILED;
  });
  return BUMBAR_OK;
}

int bumbar_server_result(bumbar_server* srv, uint64_t ticket, double* f_k_host,
                         bumbar_stats* stats, double* latency_ms, int* status) {
  if (!srv) return BUMBAR_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(ticket);
  if (it == srv->jobs.end()) return BUMBAR_EINVAL;
  const Job& j = *it->second;
  if (j.state != BUMBAR_TICKET_DONE && j.state != BUMBAR_TICKET_FAILED) return BUMBAR_EBUSY;
  if (f_k_host && !j.f.empty()) std::memcpy(f_k_host, j.f.data(), sizeof(double) * j.f.size());
  if (stats) {
    bumbar_check* c = stats->checks;
    const int cap = stats->checks_capacity;
    *stats = j.stats;
    stats->checks = c;
    stats->checks_capacity = cap;
  }
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(j.t_done - j.t_submit).count();
  if (status) *status = j.status;
  srv->jobs.erase(it);
  return BUMBAR_OK;
}

int bumbar_server_counters(bumbar_server* srv, int64_t* completed, int64_t* peak_active,
                           size_t* peak_bytes) {
  if (!srv) return BUMBAR_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (completed) *completed = srv->completed;
  if (peak_active) *peak_active = srv->peak_active;
  if (peak_bytes) *peak_bytes = srv->alloc->peak();
  return BUMBAR_OK;
}

void bumbar_server_destroy(bumbar_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_admit.notify_all();
  for (auto& t : srv->workers) t.join();
  release_slots(srv);
}

}  // extern "C"

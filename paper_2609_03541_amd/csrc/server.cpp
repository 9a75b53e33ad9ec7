// Batched serving: continuous batching of independent MBAR problems on one
// device (the C ABI declared in include/bumbar.h).
//
// Memory: one arena of hbm_budget_bytes is reserved at creation and handed
// out first-fit (256-byte aligned) to admitted requests; a request's
// footprint is its resident u_kn (uploaded, or materialised from the model;
// a model request without it keeps only its coordinates, the energies being
// evaluated inside the kernels) plus inputs plus the workspace bumbar_solve
// asks for. Admission is strictly in arrival order: a free slot takes the
// oldest queued request as soon as its footprint fits, so a large request is
// not overtaken indefinitely. Each slot owns a HIP stream (default priority)
// and a library context, and every problem is solved by exactly the kernels
// of bumbar_solve (identical results alone and in the mix). Latency =
// completion time - submission time (host clock).
//
// Driving the slots: a host thread per slot, or (caller-driven) fibers: each
// admitted solve runs on its own stack (ucontext) on the thread that calls
// bumbar_server_progress, and where bumbar_solve would block on its stream
// (ctx_wait) it swaps back to the tick, which resumes the next slot. Kernels
// of all slots stay queued on their streams meanwhile, so they overlap on the
// device exactly as with threads, but nothing advances between ticks.
//
// Fused launches (caller-driven servers with fuse = 1): a solve that reaches
// a batch of binned steps on a level small enough for one workgroup posts
// the batch's arguments instead of launching it and yields. After resuming
// every slot the tick writes all posts of the tick into a pinned work list,
// makes the fused stream wait for each posting slot's stream (an event
// recorded at the post), and replays a captured graph (copy of the work list
// to the device, then one fused kernel over all items); each posting slot's
// stream then waits for the graph's completion event before its readback.
// Two work-list buffers alternate; a buffer is rewritten only once the
// replay that last read it has completed (else the posts wait a tick).
#include <hip/hip_runtime.h>
#include <sys/mman.h>
#include <ucontext.h>

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
#include "solver_internal.h"

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

size_t dtype_bytes(int dt) { return dt == BUMBAR_F32 ? sizeof(float) : sizeof(double); }

struct Job {
  uint64_t ticket = 0;
  bumbar_request req{};
  size_t footprint = 0;
  size_t ws_bytes = 0;
  bool stored = false;     // the solve reads a resident u_kn (uploaded or materialised)
  bool xi_wide = false;    // FP32 coordinates widened here for the model evaluation
  Clock::time_point t_submit, t_done;
  int state = BUMBAR_TICKET_QUEUED;
  int status = BUMBAR_OK;
  bool mem_waited = false;  // was first in line with a slot free but no room in the arena
  std::vector<double> f;
  bumbar_stats stats{};
};

// A solve suspended on its own stack (caller-driven servers).
struct Fiber {
  ucontext_t self{}, back{};
  char* map = nullptr;  // mmap'ed region: a guard page, then the stack
  size_t map_bytes = 0;
  bool finished = true;
};

constexpr size_t kFiberStack = size_t(4) << 20;

struct Slot {
  bumbar_server* srv = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_post = nullptr;  // fused servers: recorded on the stream at a post
  bumbar_ctx* ctx = nullptr;
  // caller-driven: the job on this slot and its arena block
  std::shared_ptr<Job> job;
  size_t off = 0;
  Fiber fib;  // ucontext_t points into itself: a Slot never moves (held by pointer)
};

// A batch handed to the next fused launch; lives on the posting fiber's
// stack until the launch is queued.
struct Post {
  Slot* slot = nullptr;
  bumbar::SmallBatch a{};
  hipEvent_t done = nullptr;
  hipError_t status = hipSuccess;
  bool launched = false;
};

// One work-list buffer of the fused launches and the graphs that replay it
// (one per item count).
struct FusedBuf {
  bumbar::SmallWorkHeader* host = nullptr;  // pinned
  bumbar::SmallWorkHeader* dev = nullptr;
  hipEvent_t done = nullptr;
  bool used = false;
  std::map<int64_t, hipGraphExec_t> graphs;
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
  std::vector<std::unique_ptr<Slot>> slots;
  std::thread::id owner;  // creating thread (caller-driven calls come from it)
  uint64_t next_ticket = 1;
  bool stop = false;
  int64_t active = 0, peak_active = 0, completed = 0;
  int64_t mem_waits = 0;  // requests that waited at the head of the queue for arena room
  // workspace sizing uses a context that is never used for work
  bumbar_ctx* sizing_ctx = nullptr;
  // fused launches
  hipStream_t fstream = nullptr;  // the fused launches run here
  hipStream_t fcap = nullptr;     // graphs are captured here (nothing executes on it)
  FusedBuf fbuf[2];
  size_t fbytes = 0;  // a work-list buffer: header and max_active items
  int fgrid = 1;      // workgroups per fused kernel: min(max_active, kFusedGrid)
  int fnext = 0;
  bool fgraphs = true;  // false once capture or instantiation failed
  std::vector<Post*> posts;
  int64_t fused_launches = 0, fused_items = 0;
};

namespace {

size_t footprint_of(bumbar_server* srv, Job& job) {
  bumbar_request& r = job.req;
  job.stored = r.u_kn != nullptr || r.materialize;
  job.xi_wide = r.materialize && r.xi_dtype == BUMBAR_F32;
  // the solve gets the stored matrix's type, and FP64 coordinates where they
  // were widened here
  r.opt.u_dtype = job.stored ? r.u_dtype : BUMBAR_F64;
  r.opt.xi_dtype = job.xi_wide ? BUMBAR_F64 : r.xi_dtype;
  size_t ws = 0;
  if (job.stored) {
    const int dq = (r.opt.binning && r.xi) ? r.d : 0;
    bumbar_query_workspace(srv->sizing_ctx, r.K, r.N, dq, &r.opt, &ws);
  } else {
    bumbar_query_workspace_model(srv->sizing_ctx, r.K, r.N, r.d, &r.opt, &ws);
  }
  job.ws_bytes = ws;
  const size_t KN = (size_t)r.K * (size_t)r.N, Nd = (size_t)r.N * (size_t)r.d;
  size_t b = 0;
  if (job.stored) b += align_up(dtype_bytes(r.u_dtype) * KN);  // resident u_kn
  if (r.xi) b += align_up(dtype_bytes(r.xi_dtype) * Nd);
  if (job.xi_wide) b += align_up(sizeof(double) * Nd);
  b += align_up(sizeof(int64_t) * (size_t)r.K);
  if (r.coef) b += align_up(sizeof(double) * (size_t)r.K * (size_t)(1 + 2 * r.d));
  b += align_up(sizeof(double) * (size_t)r.K);  // f
  b += align_up(ws);
  return b;
}

// Uploads the request into its arena block, solves it and reads f back. On
// a caller-driven server this runs inside the slot's fiber: every wait on
// the stream goes through ctx_wait and so yields to the tick.
void run_job(bumbar_ctx* ctx, hipStream_t stream, char* base, Job& job) {
  const bumbar_request& r = job.req;
  char* p = base;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += align_up(bytes);
    return q;
  };
  const size_t KN = (size_t)r.K * (size_t)r.N, Nd = (size_t)r.N * (size_t)r.d;
  void* u = job.stored ? take(dtype_bytes(r.u_dtype) * KN) : nullptr;
  void* xi = r.xi ? take(dtype_bytes(r.xi_dtype) * Nd) : nullptr;
  double* xi64 = job.xi_wide ? reinterpret_cast<double*>(take(sizeof(double) * Nd)) : nullptr;
  int64_t* nk = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (size_t)r.K));
  double* coef =
      r.coef ? reinterpret_cast<double*>(take(sizeof(double) * (size_t)r.K * (1 + 2 * r.d)))
             : nullptr;
  double* f = reinterpret_cast<double*>(take(sizeof(double) * (size_t)r.K));
  void* ws = take(job.ws_bytes);
  hipError_t e = hipSuccess;
  if (r.u_kn)
    e = hipMemcpyAsync(u, r.u_kn, dtype_bytes(r.u_dtype) * KN, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && r.xi)
    e = hipMemcpyAsync(xi, r.xi, dtype_bytes(r.xi_dtype) * Nd, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(nk, r.N_k, sizeof(int64_t) * (size_t)r.K, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess && r.coef)
    e = hipMemcpyAsync(coef, r.coef, sizeof(double) * (size_t)r.K * (1 + 2 * r.d),
                       hipMemcpyHostToDevice, stream);
  const void* xs = xi;  // the coordinates the solve reads
  int xs_dtype = r.xi_dtype;
  if (e == hipSuccess && job.xi_wide) {
    e = bumbar::launch_widen_f32(stream, static_cast<const float*>(xi), (int64_t)Nd, xi64);
    xs = xi64;
    xs_dtype = BUMBAR_F64;
  }
  // a materialised request: the model evaluated once into the resident u_kn
  if (e == hipSuccess && !r.u_kn && r.materialize)
    e = bumbar::launch_model_energies(stream, r.K, r.N, r.d, r.model, coef,
                                      static_cast<const double*>(xs), u,
                                      r.u_dtype == BUMBAR_F32);
  if (e != hipSuccess) {
    job.status = BUMBAR_EDEVICE;
    return;
  }
  // a request without a stored u_kn is solved with the energies evaluated
  // from the model inside the kernels (u_kn = NULL in bumbar_solve)
  const int dq = r.xi ? r.d : 0;
  job.stats.checks = nullptr;
  job.stats.checks_capacity = 0;
  job.status = bumbar_solve(ctx, u, r.u_dtype, r.K, r.N, nk, dq ? xs : nullptr, xs_dtype, dq,
                            r.model, coef, nullptr, &r.opt, ws, job.ws_bytes, f, nullptr,
                            nullptr, &job.stats);
  job.f.assign(r.K, 0.0);
  // drain before the copy into pageable memory (it would block a fiber's thread)
  e = bumbar::ctx_wait(ctx, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(job.f.data(), f, sizeof(double) * r.K, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = bumbar::ctx_wait(ctx, stream);
  if (e != hipSuccess && job.status == BUMBAR_OK) job.status = BUMBAR_EDEVICE;
}

// Takes an arena block for the request at the head of the queue; a request
// that finds a free slot but no room is counted once (caller holds srv->mu).
bool alloc_front_locked(bumbar_server* srv, size_t* off) {
  Job& front = *srv->queue.front();
  if (srv->alloc->alloc(front.footprint, off)) return true;
  if (!front.mem_waited) {
    front.mem_waited = true;
    srv->mem_waits++;
  }
  return false;
}

// Marks a job finished and returns its arena block (caller holds srv->mu).
void finish_locked(bumbar_server* srv, Job& job, size_t off) {
  srv->alloc->release(off, job.footprint);
  job.t_done = Clock::now();
  job.state = (job.status == BUMBAR_OK || job.status == BUMBAR_ENOTCONV) ? BUMBAR_TICKET_DONE
                                                                         : BUMBAR_TICKET_FAILED;
  srv->active--;
  srv->completed++;
}

// Fails every queued job (shutdown; caller holds srv->mu).
void fail_queued_locked(bumbar_server* srv) {
  for (auto& j : srv->queue) {
    j->state = BUMBAR_TICKET_FAILED;
    j->status = BUMBAR_EBUSY;
  }
  srv->queue.clear();
}

void worker_main(bumbar_server* srv, Slot* sl) {
  (void)hipSetDevice(srv->opt.device);
  for (;;) {
    std::shared_ptr<Job> job;
    size_t off = 0;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv_admit.wait(lk, [&] {
        if (srv->stop) return true;
        if (srv->queue.empty()) return false;
        return alloc_front_locked(srv, &off);
      });
      if (srv->stop && srv->queue.empty()) break;
      if (srv->stop) {
        // drain: jobs still queued at shutdown fail without running
        fail_queued_locked(srv);
        srv->cv_done.notify_all();
        break;
      }
      job = srv->queue.front();
      srv->queue.pop_front();
      job->state = BUMBAR_TICKET_RUNNING;
      srv->active++;
      srv->peak_active = std::max(srv->peak_active, srv->active);
    }
    run_job(sl->ctx, sl->stream, srv->arena + off, *job);
    // whatever path run_job left by, no copy or kernel of this job may still
    // touch its arena block once the block is handed to another request
    if (hipStreamSynchronize(sl->stream) != hipSuccess && job->status == BUMBAR_OK)
      job->status = BUMBAR_EDEVICE;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      finish_locked(srv, *job, off);
    }
    srv->cv_admit.notify_all();
    srv->cv_done.notify_all();
  }
}

// ---- fibers (caller-driven servers) --------------------------------------

thread_local Slot* t_entering = nullptr;  // the slot whose fiber starts next

void fiber_yield(void* arg) {
  Fiber* f = static_cast<Fiber*>(arg);
  swapcontext(&f->self, &f->back);
}

void fiber_main() {
  Slot* sl = t_entering;
  try {
    run_job(sl->ctx, sl->stream, sl->srv->arena + sl->off, *sl->job);
  } catch (...) {
    sl->job->status = BUMBAR_ENOMEM;  // host allocation failed inside the solve
  }
  sl->ctx->yield = nullptr;
  sl->ctx->yield_arg = nullptr;
  sl->ctx->post_small = nullptr;
  sl->ctx->post_arg = nullptr;
  sl->fib.finished = true;
  // returning resumes uc_link, the tick that last resumed this fiber
}

bool fiber_alloc(Fiber& f) {
  const size_t page = 4096;
  f.map_bytes = kFiberStack + page;
  void* m = mmap(nullptr, f.map_bytes, PROT_READ | PROT_WRITE,
                 MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
  if (m == MAP_FAILED) return false;
  f.map = static_cast<char*>(m);
  // the lowest page stays inaccessible: a stack overflow faults on the host
  // instead of writing over other memory
  if (mprotect(f.map, page, PROT_NONE) != 0) return false;
  return true;
}

void fiber_free(Fiber& f) {
  if (f.map) munmap(f.map, f.map_bytes);
  f.map = nullptr;
}

// ctx->post_small of a fused server's fibers: queue the batch for the tick's
// fused launch, yield until it is queued, then order the slot's stream
// after it.
int post_small(void* arg, const bumbar::SmallBatch& a) {
  Slot& sl = *static_cast<Slot*>(arg);
  hipError_t e = hipEventRecord(sl.ev_post, sl.stream);
  if (e != hipSuccess) return bumbar::hip_fail(sl.ctx, e, "post event");
  Post p;
  p.slot = &sl;
  p.a = a;
  sl.srv->posts.push_back(&p);
  while (!p.launched) sl.ctx->yield(sl.ctx->yield_arg);
  if (p.status != hipSuccess) return bumbar::hip_fail(sl.ctx, p.status, "fused launch");
  e = hipStreamWaitEvent(sl.stream, p.done, 0);
  if (e != hipSuccess) return bumbar::hip_fail(sl.ctx, e, "wait for the fused launch");
  return BUMBAR_OK;
}

// The graph of buffer fb for the column-layout classes in mask: the work
// list's copy, then a fused kernel per class (nullptr if capture is off or
// fails). The copy is of the whole buffer, so the graph serves any counts.
hipGraphExec_t fused_graph(bumbar_server* srv, FusedBuf& fb, unsigned mask) {
  auto it = fb.graphs.find(mask);
  if (it != fb.graphs.end()) return it->second;
  if (!srv->fgraphs) return nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  hipError_t e = hipStreamBeginCapture(srv->fcap, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    hipError_t e1 = hipMemcpyAsync(fb.dev, fb.host, srv->fbytes, hipMemcpyHostToDevice, srv->fcap);
    if (e1 == hipSuccess) e1 = bumbar::launch_small_fused(srv->fcap, fb.dev, mask, srv->fgrid);
    e = hipStreamEndCapture(srv->fcap, &g);
    if (e == hipSuccess) e = e1;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    srv->fgraphs = false;  // launched directly from now on
    return nullptr;
  }
  fb.graphs[mask] = x;
  return x;
}

// Queues one fused launch over every post of this tick (after the slot
// resumptions); posts stay pending for a tick if the next buffer is still
// being read by an earlier launch.
void launch_fused(bumbar_server* srv) {
  if (srv->posts.empty()) return;
  FusedBuf& fb = srv->fbuf[srv->fnext];
  if (fb.used && hipEventQuery(fb.done) == hipErrorNotReady) return;
  (void)hipGetLastError();
  srv->fnext ^= 1;
  // the items grouped by column layout, in posting order within a layout
  bumbar::SmallWorkHeader& hd = *fb.host;
  bumbar::SmallBatch* items = reinterpret_cast<bumbar::SmallBatch*>(fb.host + 1);
  unsigned mask = 0u;
  int64_t n = 0;
  for (int c = 0; c < 4; ++c) {
    hd.first[c] = n;
    hd.count[c] = 0;
    for (Post* p : srv->posts)
      if (bumbar::small_class(p->a.nc) == c) {
        items[n++] = p->a;
        hd.count[c]++;
      }
    if (hd.count[c]) mask |= 1u << c;
  }
  hipError_t e = n == (int64_t)srv->posts.size() ? hipSuccess : hipErrorInvalidValue;
  for (Post* p : srv->posts)
    if (e == hipSuccess) e = hipStreamWaitEvent(srv->fstream, p->slot->ev_post, 0);
  if (e == hipSuccess) {
    hipGraphExec_t x = fused_graph(srv, fb, mask);
    if (x) {
      e = hipGraphLaunch(x, srv->fstream);
    } else {
      e = hipMemcpyAsync(fb.dev, fb.host, bumbar::small_work_bytes(n), hipMemcpyHostToDevice,
                         srv->fstream);
      if (e == hipSuccess) e = bumbar::launch_small_fused(srv->fstream, fb.dev, mask, srv->fgrid);
    }
  }
  if (e == hipSuccess) e = hipEventRecord(fb.done, srv->fstream);
  fb.used = true;
  for (Post* p : srv->posts) {
    p->done = fb.done;
    p->status = e;
    p->launched = true;
  }
  srv->posts.clear();
  srv->fused_launches++;
  srv->fused_items += n;
}

// Starts the fiber of a slot that has just been given a job.
bool fiber_start(Slot& sl) {
  Fiber& f = sl.fib;
  if (getcontext(&f.self) != 0) return false;
  f.self.uc_stack.ss_sp = f.map + 4096;
  f.self.uc_stack.ss_size = kFiberStack;
  f.self.uc_link = &f.back;
  makecontext(&f.self, fiber_main, 0);
  f.finished = false;
  sl.ctx->yield = fiber_yield;
  sl.ctx->yield_arg = &f;
  if (sl.srv->opt.fuse) {
    sl.ctx->post_small = post_small;
    sl.ctx->post_arg = &sl;
  }
  return true;
}

// Admission of a caller-driven tick: free slots take queued jobs in arrival
// order while the oldest one's footprint fits.
void admit(bumbar_server* srv) {
  std::lock_guard<std::mutex> lk(srv->mu);
  for (auto& slp : srv->slots) {
    Slot& sl = *slp;
    if (sl.job) continue;
    if (srv->queue.empty()) break;
    size_t off = 0;
    if (!alloc_front_locked(srv, &off)) break;
    sl.job = srv->queue.front();
    srv->queue.pop_front();
    sl.off = off;
    sl.job->state = BUMBAR_TICKET_RUNNING;
    srv->active++;
    srv->peak_active = std::max(srv->peak_active, srv->active);
    if (!fiber_start(sl)) {
      sl.job->status = BUMBAR_EDEVICE;
      finish_locked(srv, *sl.job, off);
      sl.job.reset();
      sl.ctx->yield = nullptr;
    }
  }
}

// Resumes every running fiber once and retires the finished ones.
int tick(bumbar_server* srv) {
  (void)hipSetDevice(srv->opt.device);
  admit(srv);
  int done = 0;
  for (auto& slp : srv->slots) {
    Slot& sl = *slp;
    if (!sl.job) continue;
    t_entering = &sl;
    swapcontext(&sl.fib.back, &sl.fib.self);
    if (!sl.fib.finished) continue;
    Job& job = *sl.job;
    if (hipStreamSynchronize(sl.stream) != hipSuccess && job.status == BUMBAR_OK)
      job.status = BUMBAR_EDEVICE;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      finish_locked(srv, job, sl.off);
    }
    sl.job.reset();
    ++done;
  }
  launch_fused(srv);
  if (done) srv->cv_done.notify_all();
  return done;
}

bool any_running(bumbar_server* srv) {
  for (auto& slp : srv->slots)
    if (slp->job) return true;
  return false;
}

// Frees the slots, the sizing context and the arena, then the server.
void release_slots(bumbar_server* srv) {
  for (auto& slp : srv->slots) {
    if (slp->ctx) bumbar_destroy(slp->ctx);
    if (slp->ev_post) (void)hipEventDestroy(slp->ev_post);
    if (slp->stream) (void)hipStreamDestroy(slp->stream);
    fiber_free(slp->fib);
  }
  if (srv->fstream) (void)hipStreamSynchronize(srv->fstream);
  for (FusedBuf& fb : srv->fbuf) {
    for (auto& g : fb.graphs) (void)hipGraphExecDestroy(g.second);
    if (fb.done) (void)hipEventDestroy(fb.done);
    if (fb.host) (void)hipHostFree(fb.host);
    if (fb.dev) (void)hipFree(fb.dev);
  }
  if (srv->fstream) (void)hipStreamDestroy(srv->fstream);
  if (srv->fcap) (void)hipStreamDestroy(srv->fcap);
  bumbar_destroy(srv->sizing_ctx);
  (void)hipFree(srv->arena);
  delete srv;
}

}  // namespace

extern "C" {

int bumbar_server_create(const bumbar_server_options* opt, bumbar_server** out) {
  if (!opt || !out || opt->max_active < 1 || opt->hbm_budget_bytes < kAlign) return BUMBAR_EINVAL;
  if (opt->fuse != 0 && (opt->fuse != 1 || !opt->caller_driven)) return BUMBAR_EINVAL;
  *out = nullptr;
  auto* srv = new (std::nothrow) bumbar_server();
  if (!srv) return BUMBAR_ENOMEM;
  srv->opt = *opt;
  srv->owner = std::this_thread::get_id();
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
    std::unique_ptr<Slot> sl(new Slot());
    sl->srv = srv;
    if (hipStreamCreate(&sl->stream) != hipSuccess ||
        (opt->fuse && hipEventCreateWithFlags(&sl->ev_post, hipEventDisableTiming) != hipSuccess) ||
        bumbar_create(&sl->ctx, opt->device, sl->stream) != BUMBAR_OK) {
      (void)hipGetLastError();
      srv->slots.push_back(std::move(sl));
      release_slots(srv);
      return BUMBAR_EDEVICE;
    }
    // the slots' streams run concurrently: no cooperative launches (two of
    // them could each hold part of the device and wait for the rest)
    sl->ctx->coop_ok = false;
    const bool fib_ok = !opt->caller_driven || fiber_alloc(sl->fib);
    srv->slots.push_back(std::move(sl));
    if (!fib_ok) {
      release_slots(srv);
      return BUMBAR_ENOMEM;
    }
  }
  if (opt->fuse) {
    // one work-list buffer holds a post of every slot
    const size_t wl = bumbar::small_work_bytes(opt->max_active);
    srv->fbytes = wl;
    srv->fgrid = std::min(opt->max_active, bumbar::kFusedGrid);
    bool ok = hipStreamCreate(&srv->fstream) == hipSuccess &&
              hipStreamCreateWithFlags(&srv->fcap, hipStreamNonBlocking) == hipSuccess;
    for (FusedBuf& fb : srv->fbuf)
      ok = ok && hipHostMalloc(reinterpret_cast<void**>(&fb.host), wl, hipHostMallocDefault) == hipSuccess &&
           hipMalloc(reinterpret_cast<void**>(&fb.dev), wl) == hipSuccess &&
           hipEventCreateWithFlags(&fb.done, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      release_slots(srv);
      return BUMBAR_EDEVICE;
    }
  }
  if (!opt->caller_driven)
    for (auto& slp : srv->slots) srv->workers.emplace_back(worker_main, srv, slp.get());
  *out = srv;
  return BUMBAR_OK;
}

int bumbar_server_submit(bumbar_server* srv, const bumbar_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket || req->K <= 0 || req->N <= 0 || !req->N_k) return BUMBAR_EINVAL;
  if ((req->u_dtype != BUMBAR_F64 && req->u_dtype != BUMBAR_F32) ||
      (req->xi_dtype != BUMBAR_F64 && req->xi_dtype != BUMBAR_F32))
    return BUMBAR_EINVAL;
  if (!req->u_kn && (req->model == BUMBAR_MODEL_NONE || !req->xi || !req->coef))
    return BUMBAR_EINVAL;
  if (req->u_kn && req->materialize) return BUMBAR_EINVAL;
  auto job = std::make_shared<Job>();
  job->req = *req;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return BUMBAR_EBUSY;
    // the sizing context is shared by submitting threads
    job->footprint = footprint_of(srv, *job);
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

int bumbar_server_progress(bumbar_server* srv, int* n_done) {
  if (n_done) *n_done = 0;
  if (!srv || !srv->opt.caller_driven || std::this_thread::get_id() != srv->owner)
    return BUMBAR_EINVAL;
  const int done = tick(srv);
  if (n_done) *n_done = done;
  return BUMBAR_OK;
}

int bumbar_server_wait(bumbar_server* srv, uint64_t ticket) {
  if (!srv) return BUMBAR_EINVAL;
  std::shared_ptr<Job> job;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    if (it == srv->jobs.end()) return BUMBAR_EINVAL;
    job = it->second;
  }
  auto finished = [&] {
    return job->state == BUMBAR_TICKET_DONE || job->state == BUMBAR_TICKET_FAILED;
  };
  if (srv->opt.caller_driven) {
    if (std::this_thread::get_id() != srv->owner) return BUMBAR_EINVAL;
    for (;;) {
      {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (finished()) return BUMBAR_OK;
      }
      if (tick(srv) == 0) std::this_thread::yield();
    }
  }
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, finished);
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
                           size_t* peak_bytes, int64_t* mem_waits) {
  if (!srv) return BUMBAR_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (completed) *completed = srv->completed;
  if (peak_active) *peak_active = srv->peak_active;
  if (peak_bytes) *peak_bytes = srv->alloc->peak();
  if (mem_waits) *mem_waits = srv->mem_waits;
  return BUMBAR_OK;
}

int bumbar_server_fused_counters(bumbar_server* srv, int64_t* launches, int64_t* items) {
  if (!srv) return BUMBAR_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (launches) *launches = srv->fused_launches;
  if (items) *items = srv->fused_items;
  return BUMBAR_OK;
}

void bumbar_server_destroy(bumbar_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    if (srv->opt.caller_driven) fail_queued_locked(srv);
  }
  if (srv->opt.caller_driven) {
    // the suspended solves hold live objects on their stacks: run them out
    while (any_running(srv))
      if (tick(srv) == 0) std::this_thread::yield();
  } else {
    srv->cv_admit.notify_all();
    for (auto& t : srv->workers) t.join();
  }
  release_slots(srv);
}

}  // extern "C"

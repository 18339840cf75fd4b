// Solve server: continuous batching of independent solve requests on one GPU.
//
// Host runtime only (no kernels of its own). Requests are admitted by their HBM
// footprint against a caller-provided device arena, and run as soon as a worker
// and memory are free, while earlier requests are still on the device:
//   * small systems (n <= 256, nrhs <= 8, no kept factors) queue for the batch
//     worker, which takes every such request waiting when it becomes free and
//     solves them with one persistent batched launch (detection, routing,
//     condition estimate and fallback per system on the device);
//   * every other request runs the single-system solve on one of the solve
//     workers, each with its own context and HIP stream, so that their kernels
//     overlap on the device;
//   * a request may keep its factorisation resident in the arena (with a copy of
//     A); later requests that name it solve new right-hand sides with the kept
//     factors only (triangular solves, or the SVD's V, U and sigma), until the
//     caller releases it.
// The method applied to each system is the adaptive solve of Section II; the
// server adds scheduling and memory management around it.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ada.h"
#include "ada_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kSmallN = 256;       // batched kernel: n <= 256
constexpr int kSmallRhs = 8;       // and nrhs <= 8
constexpr int kPlanRhs = 8;        // kept factors serve up to this many right-hand sides per request
constexpr int kMaxBatch = 16384;   // systems per batched launch
constexpr int kBatchWg = 128;      // batched launches use half the compute units; single solves get the rest
constexpr int kFastN = 1024;       // the fast-lane solve worker takes fresh solves up to this order
constexpr size_t kAlign = 256;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// first-fit allocator over [0, size) of the arena, free ranges coalesced
class Arena {
 public:
  void init(size_t size) {
    size_ = size;
    free_.clear();
    if (size) free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t& off) {
    bytes = align_up(bytes, kAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes, kAlign);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
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
  size_t size() const { return size_; }
  size_t used() const { return used_; }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

enum JobKind { JOB_BATCH = 0, JOB_SINGLE = 1, JOB_REUSE = 2 };
enum JobState { QUEUED = 0, RUNNING = 1, DONE = 2 };

struct Factor {
  uint64_t id = 0;
  int n = 0;
  size_t off = 0, bytes = 0, ws_bytes = 0;  // workspace (factors) then the copy of A
  ada_opts opts{};
  ada_result res{};
  bool busy = false;
  bool release_pending = false;
  int users = 0;  // queued or running requests that name it
};

struct Job {
  uint64_t ticket = 0;
  ada_request req{};
  int kind = JOB_SINGLE;
  int state = QUEUED;
  int rc = ADA_OK;
  std::string err;
  ada_result res{};
  uint64_t kept = 0;
  size_t off = 0, bytes = 0;
  Clock::time_point t_submit, t_start, t_done;
};

bool same_opts(const ada_opts& a, const ada_opts& b) {
  return a.no_approx == b.no_approx && a.rcond_threshold == b.rcond_threshold && a.force_general == b.force_general &&
         a.want_berr == b.want_berr && a.precision == b.precision;
}

}  // namespace

struct ada_server_s {
  int device = 0;
  char* base = nullptr;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> small_q, large_q;
  std::unordered_map<uint64_t, Job*> jobs;
  std::unordered_map<uint64_t, Factor*> factors;
  uint64_t next_ticket = 1, next_factor = 1;
  bool stop = false;
  std::vector<std::thread> threads;
  std::vector<ada_ctx> ctxs;
  std::vector<hipStream_t> streams;
  // batch worker buffers: descriptors and results (device, arena) and their pinned host mirrors
  size_t bdesc_off = 0, bres_off = 0, bwork_off = 0, bwork_bytes = 0;
  size_t reserved = 0;  // arena bytes those buffers take
  ada_desc* h_desc = nullptr;
  ada_result* h_res = nullptr;
};

namespace {

void finish(ada_server s, Job* j, int rc, const std::string& err) {
  // s->mu held
  j->rc = rc;
  j->err = err;
  j->state = DONE;
  j->t_done = Clock::now();
  s->cv_done.notify_all();
}

void batch_worker(ada_server s, int w) {
  ada_ctx ctx = s->ctxs[w];
  hipStream_t st = s->streams[w];
  (void)ctx;
  hipSetDevice(s->device);
  std::vector<Job*> batch;
  for (;;) {
    batch.clear();
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || !s->small_q.empty(); });
      if (s->stop) return;
      // every waiting small request with the options of the first (one launch takes one set of options)
      const ada_opts o0 = s->small_q.front()->req.opts;
      for (auto it = s->small_q.begin(); it != s->small_q.end() && (int)batch.size() < kMaxBatch;) {
        if (same_opts((*it)->req.opts, o0)) {
          batch.push_back(*it);
          (*it)->state = RUNNING;
          (*it)->t_start = Clock::now();
          it = s->small_q.erase(it);
        } else {
          ++it;
        }
      }
    }
    const int count = (int)batch.size();
    const double* base = reinterpret_cast<const double*>(s->base);
    for (int k = 0; k < count; ++k) {
      const ada_request& r = batch[k]->req;
      ada_desc& d = s->h_desc[k];
      d.n = r.n;
      d.nrhs = r.nrhs;
      d.lda = r.lda;
      d.ldb = r.ldb;
      d.ldx = r.ldx;
      d.pad = 0;
      // element offsets from the arena base (any sign): the kernel addresses base + offset
      d.a_off = (int64_t)(reinterpret_cast<intptr_t>(r.A) - reinterpret_cast<intptr_t>(base)) / 8;
      d.b_off = (int64_t)(reinterpret_cast<intptr_t>(r.B) - reinterpret_cast<intptr_t>(base)) / 8;
      d.x_off = (int64_t)(reinterpret_cast<intptr_t>(r.X) - reinterpret_cast<intptr_t>(base)) / 8;
    }
    ada_desc* d_desc = reinterpret_cast<ada_desc*>(s->base + s->bdesc_off);
    ada_result* d_res = reinterpret_cast<ada_result*>(s->base + s->bres_off);
    hipError_t e = hipMemcpyAsync(d_desc, s->h_desc, sizeof(ada_desc) * count, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = ada::launch_solve_batched(count, d_desc, base, base, const_cast<double*>(base), s->base + s->bwork_off,
                                    s->bwork_bytes, batch[0]->req.opts, d_res, st,
                                    ada::batched_default_shape(kBatchWg));
    if (e == hipSuccess) e = hipMemcpyAsync(s->h_res, d_res, sizeof(ada_result) * count, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    std::lock_guard<std::mutex> lk(s->mu);
    for (int k = 0; k < count; ++k) {
      Job* j = batch[k];
      if (e != hipSuccess) {
        finish(s, j, ADA_ERR_HIP, std::string("batched launch: ") + hipGetErrorString(e));
      } else {
        j->res = s->h_res[k];
        finish(s, j, j->res.status, j->res.status == ADA_OK ? "" : "batched solve reported an error status");
      }
    }
  }
}

// next request for a solve worker: first a reuse whose factors are idle (only triangular solves: it
// never waits behind factorisations), then the first fresh solve in arrival order whose workspace fits;
// a fresh solve that does not fit holds back the fresh solves behind it (no starvation of large
// requests). The fast-lane worker takes fresh solves of order <= kFastN only, so that small and medium
// requests keep moving while the other workers run long factorisations or SVD fallbacks.
Job* take_large(ada_server s, bool fast_lane) {
  for (auto it = s->large_q.begin(); it != s->large_q.end(); ++it) {
    Job* j = *it;
    if (j->kind != JOB_REUSE) continue;
    Factor* f = s->factors.at(j->req.reuse);
    if (f->busy) continue;
    f->busy = true;
    s->large_q.erase(it);
    return j;
  }
  for (auto it = s->large_q.begin(); it != s->large_q.end(); ++it) {
    Job* j = *it;
    if (j->kind == JOB_REUSE) continue;
    if (fast_lane && j->req.n > kFastN) continue;
    if (s->arena.alloc(j->bytes, j->off)) {
      s->large_q.erase(it);
      return j;
    }
    return nullptr;
  }
  return nullptr;
}

void solve_worker(ada_server s, int w) {
  const bool fast_lane = w == 1 && s->ctxs.size() > 2;  // with two or more solve workers, the first is the fast lane
  ada_ctx ctx = s->ctxs[w];
  hipStream_t st = s->streams[w];
  hipSetDevice(s->device);
  for (;;) {
    Job* j = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || (j = take_large(s, fast_lane)) != nullptr; });
      if (s->stop && !j) return;
      j->state = RUNNING;
      j->t_start = Clock::now();
    }
    const ada_request& r = j->req;
    ada_result res;
    memset(&res, 0, sizeof(res));
    int rc;
    std::string err;
    if (j->kind == JOB_REUSE) {
      Factor* f;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        f = s->factors.at(r.reuse);
      }
      const double* Ak = reinterpret_cast<const double*>(s->base + f->off + f->ws_bytes);
      rc = ada::solve_factored(ctx, f->n, r.nrhs, kPlanRhs, Ak, f->n, r.B, r.ldb, r.X, r.ldx, s->base + f->off,
                               f->ws_bytes, f->opts, f->res, &res, st);
      if (rc != ADA_OK) err = ada::last_error_string();
      std::lock_guard<std::mutex> lk(s->mu);
      f->busy = false;
      --f->users;
      j->res = res;
      if (f->release_pending && f->users == 0) {
        s->arena.release(f->off, f->bytes);
        s->factors.erase(f->id);
        delete f;
      }
      finish(s, j, rc, err);
      s->cv_work.notify_all();
      continue;
    }
    const bool keep = r.keep_factor != 0;
    const int plan = keep ? kPlanRhs : r.nrhs;
    const size_t ws = ada_workspace_size(r.n, plan, &r.opts);
    char* work = s->base + j->off;
    rc = ada::solve_internal(ctx, r.n, r.nrhs, plan, r.A, r.lda, r.B, r.ldb, r.X, r.ldx, work, ws, r.opts, &res, st,
                             keep);
    if (rc != ADA_OK) err = ada::last_error_string();
    bool kept = false;
    if (keep && rc == ADA_OK && res.route != ADA_ROUTE_NONE) {
      // the copy of A sits after the workspace; the factors stay where the solve left them
      double* Ak = reinterpret_cast<double*>(work + ws);
      hipError_t e = hipMemcpy2DAsync(Ak, (size_t)r.n * 8, r.A, (size_t)r.lda * 8, (size_t)r.n * 8, (size_t)r.n,
                                      hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      kept = e == hipSuccess;
      if (!kept) {
        rc = ADA_ERR_HIP;
        err = std::string("copy of A for the kept factors: ") + hipGetErrorString(e);
      }
    }
    std::lock_guard<std::mutex> lk(s->mu);
    j->res = res;
    if (kept) {
      Factor* f = new Factor();
      f->id = s->next_factor++;
      f->n = r.n;
      f->off = j->off;
      f->bytes = j->bytes;
      f->ws_bytes = ws;
      f->opts = r.opts;
      f->res = res;
      s->factors[f->id] = f;
      j->kept = f->id;
    } else {
      s->arena.release(j->off, j->bytes);
    }
    finish(s, j, rc, err);
    s->cv_work.notify_all();  // memory freed: waiting requests may fit now
  }
}

int fail_s(int code, const char* msg) {
  ada::set_last_error(msg);
  return code;
}

// the request's options with defaults filled in (struct_size 0 = all defaults)
bool normalized_opts(const ada_opts& in, ada_opts& o) {
  ada_opts_default(&o);
  if (in.struct_size == 0) return true;
  if (in.struct_size < sizeof(uint32_t) || in.struct_size > sizeof(ada_opts)) return false;
  memcpy(&o, &in, in.struct_size);
  o.struct_size = sizeof(ada_opts);
  return true;
}

}  // namespace

extern "C" {

int ada_server_create(ada_ctx ctx, void* arena, size_t arena_bytes, int solve_workers, ada_server* out) {
  if (!ctx || !arena || !out) return fail_s(ADA_ERR_ARG, "NULL context, arena or output pointer");
  if ((reinterpret_cast<uintptr_t>(arena) & (kAlign - 1)) != 0) return fail_s(ADA_ERR_ARG, "arena must be 256-byte aligned");
  if (solve_workers < 1 || solve_workers > 8) return fail_s(ADA_ERR_ARG, "solve_workers must be in 1..8");
  const int device = ada::context_device(ctx);
  ada_server s = new ada_server_s();
  s->device = device;
  s->base = static_cast<char*>(arena);
  s->arena.init(arena_bytes);
  // batch worker buffers
  s->bwork_bytes = ada_batched_workspace_size(kMaxBatch);
  if (!s->arena.alloc(sizeof(ada_desc) * kMaxBatch, s->bdesc_off) ||
      !s->arena.alloc(sizeof(ada_result) * kMaxBatch, s->bres_off) ||
      !s->arena.alloc(s->bwork_bytes, s->bwork_off)) {
    delete s;
    return fail_s(ADA_ERR_NOMEM, "arena too small for the batch worker's buffers");
  }
  s->reserved = s->arena.used();
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void**)&s->h_desc, sizeof(ada_desc) * kMaxBatch, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&s->h_res, sizeof(ada_result) * kMaxBatch, hipHostMallocDefault) != hipSuccess) {
    if (s->h_desc) hipHostFree(s->h_desc);
    delete s;
    return fail_s(ADA_ERR_HIP, "pinned host buffers");
  }
  const int nw = 1 + solve_workers;
  for (int w = 0; w < nw; ++w) {
    ada_ctx c = nullptr;
    hipStream_t st = nullptr;
    if (ada_create(&c, device) != ADA_OK || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      if (c) ada_destroy(c);
      for (auto& x : s->ctxs) ada_destroy(x);
      for (auto& x : s->streams) hipStreamDestroy(x);
      hipHostFree(s->h_desc);
      hipHostFree(s->h_res);
      delete s;
      return fail_s(ADA_ERR_HIP, "worker context or stream");
    }
    s->ctxs.push_back(c);
    s->streams.push_back(st);
  }
  s->threads.emplace_back(batch_worker, s, 0);
  for (int w = 1; w < nw; ++w) s->threads.emplace_back(solve_worker, s, w);
  *out = s;
  return ADA_OK;
}

void ada_server_destroy(ada_server s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->threads) t.join();
  for (size_t w = 0; w < s->ctxs.size(); ++w) {
    hipStreamSynchronize(s->streams[w]);
    hipStreamDestroy(s->streams[w]);
    ada_destroy(s->ctxs[w]);
  }
  for (auto& kv : s->jobs) delete kv.second;
  for (auto& kv : s->factors) delete kv.second;
  hipHostFree(s->h_desc);
  hipHostFree(s->h_res);
  s->cv_done.notify_all();
  delete s;
}

size_t ada_request_footprint(const ada_request* r) {
  if (!r) return 0;
  if (r->reuse) return 0;
  ada_opts o;
  if (!normalized_opts(r->opts, o)) return 0;
  if (!r->keep_factor && r->n >= 1 && r->n <= kSmallN && r->nrhs >= 1 && r->nrhs <= kSmallRhs &&
      o.precision != ADA_PREC_BF16_IR && o.extensions == 0)
    return 0;
  const int plan = r->keep_factor ? kPlanRhs : r->nrhs;
  size_t b = ada_workspace_size(r->n, plan, &o);
  if (r->keep_factor) b += align_up((size_t)r->n * r->n * 8, kAlign);
  return b;
}

int ada_submit(ada_server s, const ada_request* r, ada_ticket* out) {
  if (!s || !r || !out) return fail_s(ADA_ERR_ARG, "NULL server, request or ticket pointer");
  ada_opts o;
  if (!normalized_opts(r->opts, o)) return fail_s(ADA_ERR_ARG, "opts.struct_size is not a known size");
  if (o.layout != ADA_LAYOUT_DENSE) return fail_s(ADA_ERR_ARG, "the server takes dense input only");
  if (!r->B || !r->X || r->nrhs < 1) return fail_s(ADA_ERR_ARG, "NULL B or X, or nrhs < 1");
  const uintptr_t mis = reinterpret_cast<uintptr_t>(r->A) | reinterpret_cast<uintptr_t>(r->B) |
                        reinterpret_cast<uintptr_t>(r->X);
  if (mis & 7) return fail_s(ADA_ERR_ARG, "A, B and X must be 8-byte aligned");
  Job* j = new Job();
  j->req = *r;
  j->req.opts = o;
  j->t_submit = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (r->reuse) {
    auto it = s->factors.find(r->reuse);
    if (it == s->factors.end() || it->second->release_pending) {
      delete j;
      return fail_s(ADA_ERR_ARG, "unknown or released factor");
    }
    Factor* f = it->second;
    if (r->keep_factor || r->nrhs > kPlanRhs || r->ldb < f->n || r->ldx < f->n || (r->n && r->n != f->n)) {
      delete j;
      return fail_s(ADA_ERR_ARG, "reuse request: n must match the factor, nrhs <= 8, no keep_factor");
    }
    j->req.n = f->n;
    j->req.opts = f->opts;
    j->kind = JOB_REUSE;
    ++f->users;
  } else {
    if (!r->A || r->n < 1 || r->lda < r->n || r->ldb < r->n || r->ldx < r->n) {
      delete j;
      return fail_s(ADA_ERR_ARG, "bad n or leading dimension, or NULL A");
    }
    if (r->n > 16384) {
      delete j;
      return fail_s(ADA_ERR_ARG, "dense requests support n <= 16384");
    }
    // the batched kernel runs the paper's routes only: requests with extensions take a solve worker
    const bool small = !r->keep_factor && r->n <= kSmallN && r->nrhs <= kSmallRhs &&
                       o.precision != ADA_PREC_BF16_IR && o.extensions == 0;
    j->kind = small ? JOB_BATCH : JOB_SINGLE;
    if (!small) {
      ada_request rq = j->req;
      j->bytes = ada_request_footprint(&rq);
      if (align_up(j->bytes, kAlign) > s->arena.size() - s->reserved) {
        delete j;
        return fail_s(ADA_ERR_NOMEM, "the request's footprint exceeds the arena");
      }
    }
  }
  j->ticket = s->next_ticket++;
  s->jobs[j->ticket] = j;
  if (j->kind == JOB_BATCH) s->small_q.push_back(j);
  else s->large_q.push_back(j);
  s->cv_work.notify_all();
  *out = j->ticket;
  return ADA_OK;
}

int ada_poll_timed(ada_server s, ada_ticket t, ada_result* out, ada_factor* kept, int64_t timeout_us,
                   double* queue_us, double* total_us) {
  if (!s) return fail_s(ADA_ERR_ARG, "NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(t);
  if (it == s->jobs.end()) return fail_s(ADA_ERR_ARG, "unknown ticket (never issued, or already polled to completion)");
  Job* j = it->second;
  auto done = [&] { return j->state == DONE; };
  if (!done()) {
    if (timeout_us < 0) s->cv_done.wait(lk, done);
    else if (timeout_us > 0) s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done);
  }
  if (!done()) return ADA_PENDING;
  if (out) *out = j->res;
  if (kept) *kept = j->kept;
  if (queue_us) *queue_us = std::chrono::duration<double, std::micro>(j->t_start - j->t_submit).count();
  if (total_us) *total_us = std::chrono::duration<double, std::micro>(j->t_done - j->t_submit).count();
  const int rc = j->rc;
  if (rc != ADA_OK) ada::set_last_error(j->err);
  s->jobs.erase(it);
  delete j;
  return rc;
}

int ada_poll(ada_server s, ada_ticket t, ada_result* out, ada_factor* kept, int64_t timeout_us) {
  return ada_poll_timed(s, t, out, kept, timeout_us, nullptr, nullptr);
}

int ada_factor_release(ada_server s, ada_factor f) {
  if (!s) return fail_s(ADA_ERR_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->factors.find(f);
  if (it == s->factors.end() || it->second->release_pending) return fail_s(ADA_ERR_ARG, "unknown or released factor");
  Factor* fa = it->second;
  if (fa->users > 0) {
    fa->release_pending = true;  // freed when its last request completes
    return ADA_OK;
  }
  s->arena.release(fa->off, fa->bytes);
  s->factors.erase(it);
  delete fa;
  s->cv_work.notify_all();
  return ADA_OK;
}

int ada_server_usage(ada_server s, size_t* arena_used, int* queued, int* kept_factors) {
  if (!s) return fail_s(ADA_ERR_ARG, "NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (arena_used) *arena_used = s->arena.used();
  if (queued) *queued = (int)(s->small_q.size() + s->large_q.size());
  if (kept_factors) *kept_factors = (int)s->factors.size();
  return ADA_OK;
}

}  // extern "C"

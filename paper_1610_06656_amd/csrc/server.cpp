// Batching and serving (declared in include/smp.h): a persistent request loop
// that runs independent SMP-PCA jobs on one GPU. Each worker thread owns a
// context with its own non-blocking HIP stream (default priority) and
// workspace and runs whole jobs (smp_solve); jobs on different workers
// overlap on the device. Admission is in submission order, bounded by the
// device memory the jobs hold: the workspace every worker's context retains
// (a worker keeps its buffers between jobs) plus the inputs and outputs of the
// running jobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "smp_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Job {
  smp_params p;
  const float *A, *B;
  int64_t lda, ldb;
  double *U, *V, *sigma;
  size_t ws = 0;       // smp_workspace_size of the job
  size_t io = 0;       // bytes of its inputs and outputs
  bool done = false;
  int32_t status = SMP_OK;
  int32_t worker = -1;
  std::string error;
  Clock::time_point t_submit, t_start, t_end;
};

}  // namespace

struct smp_server {
  int device = 0;
  size_t budget = 0;   // 0: none
  std::vector<std::thread> threads;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_ready;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, Job> jobs;
  uint64_t next_id = 1;
  std::vector<size_t> held;   // per worker: workspace its context holds (while running: at least the job's)
  std::vector<smp_ctx *> ctxs;  // per worker: its context (null until created)
  size_t running_io = 0;      // inputs and outputs of the running jobs
  int running = 0;
  bool stopping = false;
  int ready = 0, init_failed = 0;
  std::string init_error;
  std::string last_error;
  smp_server_stats stats{};
};

namespace {

size_t in_use(const smp_server &s) {
  size_t t = s.running_io;
  for (size_t h : s.held) t += h;
  return t;
}

// Memory in use if job j started on worker w (whose context grows to at
// least the job's workspace).
size_t in_use_with(const smp_server &s, int w, const Job &j) {
  return in_use(s) - s.held[w] + std::max(s.held[w], j.ws) + j.io;
}

// The head of the queue may start on worker w: either nothing runs (a job
// larger than the budget runs alone) or the memory in use stays within the
// budget.
bool admissible(const smp_server &s, int w) {
  if (s.queue.empty()) return false;
  if (s.running == 0 || s.budget == 0) return true;
  return in_use_with(s, w, s.jobs.at(s.queue.front())) <= s.budget;
}

void worker_main(smp_server *s, int index) {
  hipStream_t st = nullptr;
  smp_ctx *ctx = nullptr;
  std::string err;
  if (hipSetDevice(s->device) != hipSuccess) err = "hipSetDevice failed";
  else if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) err = "hipStreamCreate failed";
  else if (smp_create(&ctx, s->device, st) != SMP_OK) err = "smp_create failed";
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!err.empty()) {
      ++s->init_failed;
      s->init_error = err;
    } else {
      s->ctxs[index] = ctx;
    }
    ++s->ready;
  }
  s->cv_ready.notify_all();
  if (!err.empty()) {
    if (st) hipStreamDestroy(st);
    return;
  }

  for (;;) {
    uint64_t id;
    Job *j;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return admissible(*s, index) || (s->stopping && s->queue.empty()); });
      if (s->queue.empty()) break;   // stopping, nothing left
      id = s->queue.front();
      s->queue.pop_front();
      j = &s->jobs.at(id);   // unordered_map references stay valid across inserts
      if (s->budget > 0 && in_use_with(*s, index, *j) > s->budget) {
        // only when nothing runs (admissible): the workspace the idle
        // workers retain is given back first, so that only a job larger than
        // the budget by itself can exceed it
        for (size_t w = 0; w < s->ctxs.size(); ++w) {
          if (s->ctxs[w] && s->held[w]) smp::ctx_release_workspace(s->ctxs[w]);
          s->held[w] = 0;
        }
      }
      s->held[index] = std::max(s->held[index], j->ws);
      s->running_io += j->io;
      ++s->running;
      s->stats.max_running = std::max<int32_t>(s->stats.max_running, s->running);
      s->stats.max_budget_in_use = std::max<int64_t>(s->stats.max_budget_in_use, (int64_t)in_use(*s));
      j->worker = index;
      j->t_start = Clock::now();
    }
    const smp_status rc = smp_solve(ctx, &j->p, j->A, j->lda, j->B, j->ldb, j->U, j->V, j->sigma);
    const std::string msg = rc == SMP_OK ? std::string() : std::string(smp_last_error(ctx));
    size_t kept = smp::ctx_workspace_bytes(ctx);
    bool release = false;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->held[index] = kept;
      s->running_io -= j->io;
      // a job that ran alone above the budget leaves more retained than the
      // budget allows: give it back before the next admission
      release = s->budget > 0 && in_use(*s) > s->budget;
    }
    if (release) {
      smp::ctx_release_workspace(ctx);
      kept = 0;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->held[index] = kept;
      j->status = rc;
      j->error = msg;
      j->t_end = Clock::now();
      j->done = true;
      --s->running;
      ++s->stats.completed;
      if (rc != SMP_OK) ++s->stats.failed;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->ctxs[index] = nullptr;
  }
  smp_destroy(ctx);
  hipStreamDestroy(st);
}

}  // namespace

extern "C" {

smp_status smp_server_create(int device, int workers, size_t hbm_budget, smp_server **out) {
  if (!out || workers < 1 || workers > 16) return SMP_ERR_INVALID_ARG;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SMP_ERR_INVALID_ARG;
  auto *s = new (std::nothrow) smp_server();
  if (!s) return SMP_ERR_OUT_OF_MEMORY;
  s->device = device;
  s->budget = hbm_budget;
  s->held.assign(workers, 0);
  s->ctxs.assign(workers, nullptr);
  s->stats.workers = workers;
  for (int i = 0; i < workers; ++i) s->threads.emplace_back(worker_main, s, i);
  {
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_ready.wait(lk, [&] { return s->ready == workers; });
  }
  if (s->init_failed) {
    smp_server_destroy(s);
    return SMP_ERR_DEVICE;
  }
  *out = s;
  return SMP_OK;
}

namespace {

smp_status make_job(const smp_params *p, const float *A, int64_t lda, const float *B, int64_t ldb, double *U,
                    double *V, double *sigma, Job &j) {
  const smp_status chk = smp_check_params(p);
  if (chk != SMP_OK) return chk;
  const bool same = (p->flags & SMP_B_IS_A) != 0 || (B == A && p->n1 == p->n2 && ldb == lda);
  if (!A || lda < p->n1 || (!same && (!B || ldb < p->n2)) || !U || !V) return SMP_ERR_INVALID_ARG;
  size_t ws = 0;
  if (smp_workspace_size(p, &ws) != SMP_OK) return SMP_ERR_INVALID_ARG;
  j.p = *p;
  j.A = A;
  j.lda = lda;
  j.B = B;
  j.ldb = ldb;
  j.U = U;
  j.V = V;
  j.sigma = sigma;
  j.ws = ws;
  j.io = (size_t)p->d * (size_t)lda * 4 + (same ? 0 : (size_t)p->d * (size_t)ldb * 4) +
         (size_t)(p->n1 + p->n2 + 1) * (size_t)p->r * 8;
  j.t_submit = Clock::now();
  return SMP_OK;
}

}  // namespace

smp_status smp_server_submit(smp_server *s, const smp_params *p, const float *A, int64_t lda, const float *B,
                             int64_t ldb, double *U, double *V, double *sigma, uint64_t *job_id) {
  if (!s || !p || !job_id) return SMP_ERR_INVALID_ARG;
  Job j;
  const smp_status mk = make_job(p, A, lda, B, ldb, U, V, sigma, j);
  if (mk != SMP_OK) return mk;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return SMP_ERR_STATE;
    const uint64_t id = s->next_id++;
    s->jobs.emplace(id, std::move(j));
    s->queue.push_back(id);
    ++s->stats.submitted;
    *job_id = id;
  }
  s->cv_work.notify_all();   // workers differ in what they can admit
  return SMP_OK;
}

smp_status smp_server_try_submit(smp_server *s, const smp_params *p, const float *A, int64_t lda, const float *B,
                                 int64_t ldb, double *U, double *V, double *sigma, uint64_t *job_id) {
  if (!s || !p || !job_id) return SMP_ERR_INVALID_ARG;
  Job j;
  const smp_status mk = make_job(p, A, lda, B, ldb, U, V, sigma, j);
  if (mk != SMP_OK) return mk;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return SMP_ERR_STATE;
    // refuse unless the job can start now: nothing waits ahead of it, a
    // worker is free, and (with a budget) some free worker can take it
    // within the budget or nothing runs at all
    bool fits = s->queue.empty() && s->running < s->stats.workers;
    if (fits && s->budget > 0 && s->running > 0) {
      fits = false;
      for (int w = 0; w < s->stats.workers && !fits; ++w) fits = in_use_with(*s, w, j) <= s->budget;
    }
    if (!fits) {
      ++s->stats.refused;
      return SMP_ERR_BUSY;
    }
    const uint64_t id = s->next_id++;
    s->jobs.emplace(id, std::move(j));
    s->queue.push_back(id);
    ++s->stats.submitted;
    *job_id = id;
  }
  s->cv_work.notify_all();
  return SMP_OK;
}

smp_status smp_server_wait(smp_server *s, uint64_t job_id, smp_job_result *res) {
  if (!s) return SMP_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return SMP_ERR_INVALID_ARG;
  const Job &j = it->second;   // references survive rehashing by concurrent submits; iterators do not
  s->cv_done.wait(lk, [&] { return j.done; });
  if (res) {
    res->status = j.status;
    res->worker = j.worker;
    res->queue_ms = ms_between(j.t_submit, j.t_start);
    res->run_ms = ms_between(j.t_start, j.t_end);
  }
  s->last_error = j.error;
  s->jobs.erase(job_id);
  return SMP_OK;
}

const char *smp_server_last_error(const smp_server *s) { return s ? s->last_error.c_str() : ""; }

smp_status smp_server_get_stats(smp_server *s, smp_server_stats *st) {
  if (!s || !st) return SMP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->stats;
  return SMP_OK;
}

void smp_server_destroy(smp_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  for (std::thread &t : s->threads)
    if (t.joinable()) t.join();
  delete s;
}

smp_status smp_solve_batch(int device, int njobs, const smp_params *p, const float *const *A, const int64_t *lda,
                           const float *const *B, const int64_t *ldb, double *const *U, double *const *V,
                           double *const *sigma, int workers, size_t hbm_budget, smp_job_result *res) {
  if (njobs < 0 || (njobs > 0 && (!p || !A || !lda || !B || !ldb || !U || !V))) return SMP_ERR_INVALID_ARG;
  if (njobs == 0) return SMP_OK;
  smp_server *s = nullptr;
  smp_status rc = smp_server_create(device, workers, hbm_budget, &s);
  if (rc != SMP_OK) return rc;
  std::vector<uint64_t> ids(njobs, 0);
  std::vector<smp_status> sub(njobs, SMP_OK);
  for (int i = 0; i < njobs; ++i)
    sub[i] = smp_server_submit(s, &p[i], A[i], lda[i], B[i], ldb[i], U[i], V[i], sigma ? sigma[i] : nullptr, &ids[i]);
  smp_status first = SMP_OK;
  for (int i = 0; i < njobs; ++i) {
    smp_job_result r{};
    if (sub[i] != SMP_OK) {
      r.status = sub[i];
      r.worker = -1;
    } else {
      smp_server_wait(s, ids[i], &r);
    }
    if (res) res[i] = r;
    if (first == SMP_OK && r.status != SMP_OK) first = (smp_status)r.status;
  }
  smp_server_destroy(s);
  return first;
}

}  // extern "C"

// A batch of independent SMP-PCA jobs in two phases (declared in
// include/smp.h as smp_solve_batch_group):
//  1. worker threads, each with its own context and non-blocking stream
//     (default priority), take the jobs in order and run Alg. 1 steps 2-4 for
//     each (sketch pass, the sample of Eq. (1) sized by one count, the
//     estimates of Eq. (2)), keeping each job's sample, estimates and squared
//     column norms of A in memory of its own;
//  2. one context runs Alg. 2 for all of them with smp_waltmin_group: one
//     launch per step for every group of jobs with the same launch sequence
//     (optionally one HIP graph per group), instead of the ~50 dependent
//     launches of each job's own WAltMin.
// Every job's result is bit for bit what smp_solve gives for it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "smp_internal.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// A job's state between the two phases: its sample with the estimates, and
// the squared column norms of A (the trim of Alg. 2 reads them).
struct Held {
  smp_params q{};
  smp_omega om{};
  float *na2 = nullptr;
  std::vector<void *> allocs;
  int32_t status = SMP_OK;
  int32_t worker = -1;
  Clock::time_point t_start, t_end;
  void release() {
    for (void *p : allocs) hipFree(p);
    allocs.clear();
  }
  // the job's share of the batch arena (bytes at `at`, `left` of them free);
  // a share too small (a sample beyond its bound) falls back to hipMalloc
  char *at = nullptr;
  size_t left = 0;
  template <typename T>
  T *alloc(int64_t count) {
    const size_t b = ((size_t)std::max<int64_t>(1, count) * sizeof(T) + 255) / 256 * 256;
    if (b <= left) {
      T *out = reinterpret_cast<T *>(at);
      at += b;
      left -= b;
      return out;
    }
    void *p = nullptr;
    if (hipMalloc(&p, b) != hipSuccess) {
      hipGetLastError();
      return nullptr;
    }
    allocs.push_back(p);
    return static_cast<T *>(p);
  }
};

// Bytes a job's sample, estimates and norms take at most (the bound on |Omega|
// that smp_workspace_size uses): allocated once for the whole batch, since
// hipMalloc per job would serialise the workers.
size_t held_bytes(const smp_params &p) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const double m = p.m;
  const int64_t cap = (int64_t)std::min<double>((double)p.n1 * (double)p.n2,
                                                (p.flags & SMP_SAMPLE_MULTINOMIAL) ? (double)smp::mn_draw_bound(p.n1, m)
                                                                                   : m + 6.0 * std::sqrt(m) + 64.0);
  const bool split = p.omega_mode == SMP_OMEGA_SPLIT;
  return al(p.n1 * 4) + al((p.n1 + 1) * 8) + al((p.n2 + 1) * 8) + 2 * al(cap * 4) + 4 * al(cap * 8) +
         (split ? 2 * al(cap) : 0);
}

// Grows a worker's scratch buffer of sketches and norms.
struct Scratch {
  void *p = nullptr;
  size_t bytes = 0;
  bool ensure(size_t need) {
    if (need <= bytes) return true;
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, need) != hipSuccess) {
      hipGetLastError();
      return false;
    }
    bytes = need;
    return true;
  }
};

size_t al(size_t b) { return (b + 255) / 256 * 256; }

// Steps 2-4 of one job on ctx (the caller synchronises ctx's stream).
smp_status prepare(smp_ctx *ctx, Scratch &sc, const smp_params &p, const float *A, int64_t lda, const float *B,
                   int64_t ldb, Held &h) {
  smp_params q = p;
  if (B == A && p.n1 == p.n2 && ldb == lda) q.flags |= SMP_B_IS_A;
  const bool same = (q.flags & SMP_B_IS_A) != 0;
  const int64_t n1 = q.n1, n2 = q.n2, k = q.k;
  if (!sc.ensure(al(n1 * k * 4) + al(n2 * k * 4) + al(n2 * 4))) return SMP_ERR_OUT_OF_MEMORY;
  char *c = static_cast<char *>(sc.p);
  float *At = reinterpret_cast<float *>(c);
  float *Bt = reinterpret_cast<float *>(c + al(n1 * k * 4));
  float *nb2 = reinterpret_cast<float *>(c + al(n1 * k * 4) + al(n2 * k * 4));
  h.na2 = h.alloc<float>(n1);
  int64_t *rp = h.alloc<int64_t>(n1 + 1), *cp = h.alloc<int64_t>(n2 + 1);
  if (!h.na2 || !rp || !cp) return SMP_ERR_OUT_OF_MEMORY;
  smp_status s = smp_sketch(ctx, &q, A, lda, same ? nullptr : B, ldb, At, same ? nullptr : Bt, h.na2,
                            same ? nullptr : nb2);
  if (s != SMP_OK) return s;
  const float *nb = same ? h.na2 : nb2;
  const bool split = q.omega_mode == SMP_OMEGA_SPLIT;
  smp_omega om{};
  om.n1 = n1;
  om.n2 = n2;
  om.row_ptr = rp;
  om.col_ptr = cp;
  auto carve_entries = [&](int64_t cap) {
    om.cap = cap;
    om.col_idx = h.alloc<int32_t>(cap);
    om.row_idx = h.alloc<int32_t>(cap);
    om.w_csr = h.alloc<double>(cap);
    om.w_csc = h.alloc<double>(cap);
    om.mt_csr = h.alloc<double>(cap);
    om.mt_csc = h.alloc<double>(cap);
    om.sub_csr = split ? h.alloc<uint8_t>(cap) : nullptr;
    om.sub_csc = split ? h.alloc<uint8_t>(cap) : nullptr;
    return om.col_idx && om.row_idx && om.w_csr && om.w_csc && om.mt_csr && om.mt_csc &&
           (!split || (om.sub_csr && om.sub_csc));
  };
  // the rest of the job's share holds the entry arrays at the bound on |Omega|
  const size_t per = 2 * 4 + 4 * 8 + (split ? 2 : 0);
  if (!carve_entries((int64_t)(h.left / per > 2048 ? h.left / per - 2048 : 1))) return SMP_ERR_OUT_OF_MEMORY;
  s = smp_sample(ctx, &q, h.na2, nb, &om);
  if (s == SMP_ERR_CAPACITY) {   // beyond the bound: arrays of the exact size
    const int64_t nnz = om.nnz;
    if (!carve_entries(nnz)) return SMP_ERR_OUT_OF_MEMORY;
    s = smp_sample(ctx, &q, h.na2, nb, &om);
  }
  if (s != SMP_OK) return s;
  s = smp_estimate(ctx, &q, At, same ? At : Bt, h.na2, nb, &om);
  if (s != SMP_OK) return s;
  h.q = q;
  h.om = om;
  return SMP_OK;   // the worker synchronises its stream
}

}  // namespace

extern "C" {

smp_status smp_solve_batch_group(int device, int njobs, const smp_params *p, const float *const *A,
                                 const int64_t *lda, const float *const *B, const int64_t *ldb, double *const *U,
                                 double *const *V, double *const *sigma, int workers, int graph,
                                 smp_job_result *res) {
  if (njobs < 0 || (njobs > 0 && (!p || !A || !lda || !B || !ldb || !U || !V))) return SMP_ERR_INVALID_ARG;
  if (njobs == 0) return SMP_OK;
  if (workers < 1) workers = 1;
  if (workers > 32) workers = 32;
  std::vector<Held> held(njobs);
  const Clock::time_point t0 = Clock::now();
  if (hipSetDevice(device) != hipSuccess) return SMP_ERR_DEVICE;
  size_t arena_bytes = 0;
  std::vector<size_t> share(njobs);
  for (int j = 0; j < njobs; ++j) arena_bytes += (share[j] = held_bytes(p[j]));
  void *arena = nullptr;
  if (hipMalloc(&arena, std::max<size_t>(256, arena_bytes)) != hipSuccess) {
    hipGetLastError();
    arena = nullptr;   // every job then allocates its own
  } else {
    char *c = static_cast<char *>(arena);
    for (int j = 0; j < njobs; ++j) {
      held[j].at = c;
      held[j].left = share[j];
      c += share[j];
    }
  }
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int w = 0; w < std::min(workers, njobs); ++w) {
    th.emplace_back([&, w] {
      if (hipSetDevice(device) != hipSuccess) return;
      hipStream_t st = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
      smp_ctx *ctx = nullptr;
      if (smp_create(&ctx, device, st) != SMP_OK) {
        hipStreamDestroy(st);
        return;
      }
      Scratch sc;
      for (int j; (j = next.fetch_add(1)) < njobs;) {
        Held &h = held[j];
        h.worker = w;
        h.t_start = Clock::now();
        h.status = prepare(ctx, sc, p[j], A[j], lda[j], B[j], ldb[j], h);
        hipStreamSynchronize(st);
        h.t_end = Clock::now();
      }
      if (sc.p) hipFree(sc.p);
      smp_destroy(ctx);
      hipStreamDestroy(st);
    });
  }
  for (auto &t : th) t.join();
  for (int j = 0; j < njobs; ++j)
    if (held[j].worker < 0) held[j].status = SMP_ERR_DEVICE;   // no worker could start

  // phase 2: the WAltMin of every job that got this far, grouped
  std::vector<int> ok;
  for (int j = 0; j < njobs; ++j)
    if (held[j].status == SMP_OK) ok.push_back(j);
  smp_status group_status = SMP_OK;
  if (!ok.empty()) {
    smp_ctx *ctx = nullptr;
    group_status = smp_create(&ctx, device, nullptr);
    if (group_status == SMP_OK) {
      std::vector<smp_params> gp;
      std::vector<smp_omega> go;
      std::vector<const float *> gn;
      std::vector<double *> gu, gv, gs;
      for (int j : ok) {
        gp.push_back(held[j].q);
        go.push_back(held[j].om);
        gn.push_back(held[j].na2);
        gu.push_back(U[j]);
        gv.push_back(V[j]);
        gs.push_back(sigma ? sigma[j] : nullptr);
      }
      group_status = smp_waltmin_group(ctx, (int)ok.size(), gp.data(), go.data(), gn.data(), gu.data(), gv.data(),
                                       gs.data(), graph);
      smp_destroy(ctx);
    }
    for (int j : ok) held[j].status = group_status;
  }
  const Clock::time_point t_end = Clock::now();
  smp_status first = SMP_OK;
  for (int j = 0; j < njobs; ++j) {
    if (res) {
      res[j].status = held[j].status;
      res[j].worker = held[j].worker;
      res[j].queue_ms = held[j].worker >= 0 ? ms_between(t0, held[j].t_start) : 0.0;
      res[j].run_ms = held[j].worker >= 0 ? ms_between(held[j].t_start, t_end) : 0.0;
    }
    if (first == SMP_OK && held[j].status != SMP_OK) first = (smp_status)held[j].status;
    held[j].release();
  }
  if (arena) hipFree(arena);
  return first;
}

}  // extern "C"

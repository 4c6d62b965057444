// C-ABI of the SMP-PCA hot path (declared in include/smp.h): argument
// validation, library workspace, and the stage orchestration of Alg. 1
// (sketch -> sample -> estimate -> WAltMin) on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "smp_internal.hpp"

using smp::SketchPlan;

namespace {

constexpr int kMaxK = 4096;
constexpr int kMaxR = 32;

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};

thread_local std::string g_err_no_ctx;

smp_status fail(smp_ctx *ctx, smp_status s, const std::string &msg) {
  if (ctx) ctx->last_error = msg;
  else g_err_no_ctx = msg;
  return s;
}

smp_status hip_fail(smp_ctx *ctx, hipError_t e, const char *where) {
  return fail(ctx, SMP_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define SMP_HIP(ctx, expr)                                   \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr); \
  } while (0)

std::string check(const smp_params *p) {
  if (!p) return "params is NULL";
  if (p->d < 1 || p->n1 < 1 || p->n2 < 1) return "d, n1, n2 must be >= 1";
  if (p->k < 1 || p->k > kMaxK) return "k must be in [1, 4096]";
  if (p->r < 1 || p->r > kMaxR || p->r > p->n1 || p->r > p->n2) return "r must be in [1, min(n1, n2, 32)]";
  if (p->T < 0 || p->T > 1000) return "T must be in [0, 1000]";
  if (p->T > 127 && p->omega_mode == SMP_OMEGA_SPLIT) return "SPLIT mode needs 2T+1 <= 255 subsets";
  if (!(p->m > 0.0) || !std::isfinite(p->m)) return "m must be a finite positive number";
  if (p->prec != SMP_PREC_FP32 && p->prec != SMP_PREC_BF16 && p->prec != SMP_PREC_FP8) return "unknown precision";
  if (p->omega_mode != SMP_OMEGA_REUSE && p->omega_mode != SMP_OMEGA_SPLIT) return "unknown omega_mode";
  if (p->init_iters < 0 || p->init_iters > 1000) return "init_iters must be in [0, 1000]";
  if (p->reserved != 0) return "reserved must be 0";
  if (p->flags & ~(uint32_t)(SMP_B_IS_A | SMP_SAMPLE_MULTINOMIAL | SMP_SKETCH_SRHT)) return "unknown flags";
  if ((p->flags & SMP_SKETCH_SRHT) && p->prec != SMP_PREC_FP32) return "the SRHT sketch is FP32 only";
  if ((p->flags & SMP_B_IS_A) && p->n1 != p->n2) return "SMP_B_IS_A needs n1 == n2";
  if ((p->flags & SMP_SAMPLE_MULTINOMIAL) && p->m > 1e12) return "m too large for the multinomial sampler";
  if ((p->n1 + 1) * 4 > INT32_MAX || p->n2 > INT32_MAX / 4) return "n1, n2 too large for int32 entry indices";
  return "";
}

// Rows one FP32 accumulator of the FP32 pass sums at most. Summing N random-
// sign products in FP32 leaves a relative error of about 2^-24 sqrt(N / 8)
// (the 16x16x4 MFMA adds 4 products per accumulation); 32,768 rows keep it
// near 4e-6, below the 1e-5 per-column bound, whatever d is.
constexpr int64_t kFp32RowsPerSplit = 32768;

// Number of d-splits S of the sketch pass. The kt * tiles * S workgroups of a
// launch run in ceil(total / slots) rounds on the slots the device holds at
// once; each launch writes (and, after the first, reads back) the S partial
// sketches, and the reduction reads them once. A stored-Pi pass makes one
// launch per Pi window of w = pi_window_rows rows, the other passes one launch
// over all d rows (w = d). S minimises (streaming time with the last round's
// idle slots) + (partial traffic), both relative to one perfectly balanced
// read of the input:
//   cost(S) = rounds * slots / total + 2 S kpad / w,
// with at least 256 rows per split and, for the FP32 pass, at most
// kFp32RowsPerSplit.
// The sketch pass a parameter set selects: the SRHT (SMP_SKETCH_SRHT) or the
// Gaussian pass in the given operand precision.
SketchPlan plan_for(const smp_params *p) {
  if (p->flags & SMP_SKETCH_SRHT) {
    SketchPlan pl = smp::sketch_plan_srht(p->k);
    pl.d = p->d;
    return pl;
  }
  SketchPlan pl = smp::sketch_plan(p->k, p->prec);
  pl.ntot = p->n1 + p->n2;   // the FP8 fragment pass sizes its window by the columns
  return pl;
}

// Rows one launch covers: one stored-Pi window, else all d rows.
int64_t launch_rows(const SketchPlan &pl, int64_t d) {
  return pl.pi_stored ? std::min<int64_t>(d, smp::pi_window_rows(pl)) : d;
}

// The admissible split counts [smin, smax] of a Gaussian pass.
void split_range(const SketchPlan &pl, int64_t d, int64_t &smin, int64_t &smax) {
  const int64_t wrows = launch_rows(pl, d);
  smin = pl.prec == SMP_PREC_FP32 ? (d + kFp32RowsPerSplit - 1) / kFp32RowsPerSplit : 1;
  smax = std::max<int64_t>(smin, std::min<int64_t>(256, wrows / std::max(256, 2 * pl.kc)));
}

int choose_splits(const SketchPlan &pl, int64_t d, int64_t n1, int64_t n2) {
  if (pl.srht) return smp::srht_splits(pl, d, n1, n2);
  const int64_t tiles = (n1 + pl.ncol_tile - 1) / pl.ncol_tile + (n2 + pl.ncol_tile - 1) / pl.ncol_tile;
  const int64_t per = (int64_t)pl.kt * tiles;
  const int64_t slots = smp::sketch_slots(pl);
  const int64_t wrows = launch_rows(pl, d);
  int64_t smin, smax;
  split_range(pl, d, smin, smax);
  if (const char *e = getenv("SMP_SKETCH_SPLITS")) {   // tuning override
    const long v = strtol(e, nullptr, 10);
    if (v >= 1) return (int)std::max<int64_t>(smin, std::min<int64_t>(v, smax));
  }
  int best = (int)smin;
  double best_cost = 1e300;
  for (int64_t S = smin; S <= smax; ++S) {
    const int64_t total = per * S;
    const int64_t rounds = (total + slots - 1) / slots;
    const double cost = (double)(rounds * slots) / (double)total + 2.0 * (double)S * pl.kpad / (double)wrows;
    if (cost < best_cost - 1e-12) {
      best_cost = cost;
      best = (int)S;
    }
  }
  return best;
}

smp::TuneKey tune_key(const smp_params *p, const SketchPlan &pl, int64_t n2) {
  return smp::TuneKey{p->prec, (p->flags & SMP_SKETCH_SRHT) ? 1 : 0, p->k, p->n1, n2, launch_rows(pl, p->d)};
}

// While smp_tune_sketch times a candidate on this thread, it replaces the table.
thread_local const smp::TuneChoice *t_trial = nullptr;

// The launch shape of the sketch pass for a parameter set (n2 = 0 when B is
// A): the plan, with the BF16 chunk cap that the tuning table or the trial
// under measurement gives, and the row splits, tuned or from the cost model.
void launch_shape(const smp_params *p, int64_t n2, SketchPlan &pl, int &S) {
  pl = plan_for(p);
  smp::TuneChoice c{};
  const bool have = t_trial ? (c = *t_trial, true) : smp::tune_lookup(tune_key(p, pl, n2), c);
  if (have && !pl.srht) {
    if (c.cap > 0 && pl.prec == SMP_PREC_BF16 && pl.pi_stored) {
      const SketchPlan q = smp::sketch_plan_bf16(p->k, c.cap);
      if (q.kernel && q.kernel_clamp && q.kernel_scalar) pl = q;
    }
    int64_t smin, smax;
    split_range(pl, p->d, smin, smax);
    S = (int)std::max<int64_t>(smin, std::min<int64_t>(smax, c.splits));
    return;
  }
  S = choose_splits(pl, p->d, p->n1, n2);
}

smp_status ensure(smp_ctx *ctx, Buf &b, size_t bytes) {
  if (b.bytes >= bytes) return SMP_OK;
  if (b.p) {
    hipStreamSynchronize(ctx->stream);
    hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (bytes == 0) return SMP_OK;
  if (hipMalloc(&b.p, bytes) != hipSuccess) {
    hipGetLastError();
    return fail(ctx, SMP_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  return SMP_OK;
}

size_t al(size_t b) { return (b + 255) / 256 * 256; }

enum Stage { kStSketch = 0, kStFinish = 1, kStSample = 2, kStEstimate = 3, kStWaltmin = 4 };

bool timed(const smp_ctx *ctx, int s) { return ctx->timing == 1 || (ctx->timing == 2 && s == kStSketch); }

void mark(smp_ctx *ctx, Stage s, bool end) {
  if (!timed(ctx, s)) return;
  hipEventRecord(ctx->events[2 * s + (end ? 1 : 0)], ctx->stream);
  if (end) ctx->recorded[s] = true;
}

template <typename T>
T *take(char *&c, size_t count) {
  T *o = reinterpret_cast<T *>(c);
  c += al(count * sizeof(T));
  return o;
}

}  // namespace

struct smp_sketch_state {
  smp_ctx *ctx;
  smp_params p;
  SketchPlan plan;
  int S;
  float *part;
  double *npart;
  void *pi = nullptr;    // stored-Pi scratch of the largest push so far
  size_t pi_bytes = 0;
  bool ended;
};

// ---- allocation-free estimate: its scratch in a file-scope device array -----
// na, nb (sketch-column norms) and sa, sb (data-column norms), FP64, for at
// most kNoAllocMaxCols = n1 + n2 columns: 2 * 2^20 doubles = 16 MiB on every
// device the library runs on, held until the process ends. Every call on a
// device shares that device's copy; the kernels write every entry they read,
// so nothing is cleared between calls.
namespace {
constexpr int64_t kNoAllocMaxCols = int64_t(1) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) double scratch[2 * kNoAllocMaxCols];

// The device address of `scratch` on the current device (which is `device`),
// looked up once per device. The array's name is only a host-side stand-in.
static hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

static void *scratch_for(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

struct smp_ctx_bufs {
  Buf sketch, samplews, head, omega, est, wm, mn, base, sparse, tune, group, skgroup;
};

namespace {
smp_ctx_bufs &bufs(smp_ctx *ctx);
}

extern "C" {

const char *smp_status_str(smp_status s) {
  switch (s) {
    case SMP_OK: return "ok";
    case SMP_ERR_INVALID_ARG: return "invalid argument";
    case SMP_ERR_OUT_OF_MEMORY: return "out of device memory";
    case SMP_ERR_DEVICE: return "device error";
    case SMP_ERR_NUMERIC: return "numeric error";
    case SMP_ERR_CAPACITY: return "buffer capacity exceeded";
    case SMP_ERR_STATE: return "call out of order";
    case SMP_ERR_BUSY: return "admission refused (busy)";
  }
  return "unknown status";
}

const char *smp_last_error(const smp_ctx *ctx) { return ctx ? ctx->last_error.c_str() : g_err_no_ctx.c_str(); }

smp_status smp_check_params(const smp_params *p) {
  const std::string m = check(p);
  if (!m.empty()) return fail(nullptr, SMP_ERR_INVALID_ARG, m);
  return SMP_OK;
}

smp_status smp_create(smp_ctx **ctx, int device, void *hip_stream) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
    return fail(nullptr, SMP_ERR_INVALID_ARG, "no such HIP device");
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, SMP_ERR_DEVICE, "hipSetDevice failed");
  smp_ctx *c = new (std::nothrow) smp_ctx();
  if (!c) return fail(nullptr, SMP_ERR_OUT_OF_MEMORY, "host allocation failed");
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipHostMalloc((void **)&c->host_pinned, 8 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return fail(nullptr, SMP_ERR_OUT_OF_MEMORY, "hipHostMalloc failed");
  }
  const hipError_t se = scratch_setup(device);   // with `device` current (set above)
  if (se != hipSuccess) {
    hipGetLastError();
    hipHostFree(c->host_pinned);
    delete c;
    return fail(nullptr, SMP_ERR_DEVICE, std::string("scratch symbol lookup failed: ") + hipGetErrorString(se));
  }
  c->ws = new smp_ctx_bufs();
  static std::once_flag tune_env;   // SMP_TUNE_FILE: a tuning file written by smp_tune_save
  std::call_once(tune_env, [] {
    if (const char *f = getenv("SMP_TUNE_FILE")) smp::tune_load(f);   // a missing or bad file leaves the table empty
  });
  *ctx = c;
  return SMP_OK;
}

void smp_destroy(smp_ctx *ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  auto *b = static_cast<smp_ctx_bufs *>(ctx->ws);
  if (b) {
    for (Buf *x : {&b->sketch, &b->samplews, &b->head, &b->omega, &b->est, &b->wm, &b->mn, &b->base, &b->sparse, &b->tune, &b->group})
      if (x->p) hipFree(x->p);
    delete b;
  }
  if (ctx->host_pinned) hipHostFree(ctx->host_pinned);
  for (hipEvent_t &e : ctx->events)
    if (e) hipEventDestroy(e);
  smp::blas_destroy(ctx->blas);
  delete ctx;
}

smp_status smp_set_stream(smp_ctx *ctx, void *hip_stream) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return SMP_OK;
}

smp_status smp_set_timing(smp_ctx *ctx, int enable) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  if (enable < 0 || enable > 2) return fail(ctx, SMP_ERR_INVALID_ARG, "timing level must be 0, 1 or 2");
  if (enable && !ctx->events[0])
    for (hipEvent_t &e : ctx->events) SMP_HIP(ctx, hipEventCreate(&e));
  ctx->timing = enable;
  for (bool &r : ctx->recorded) r = false;   // no stage of an earlier setting is reported
  return SMP_OK;
}

smp_status smp_stage_times(smp_ctx *ctx, float *ms, int n) {
  if (!ctx || !ms || n < 0) return fail(ctx, SMP_ERR_INVALID_ARG, "ctx or ms is NULL");
  for (int s = 0; s < 5 && s < n; ++s) {
    ms[s] = 0.0f;
    if (timed(ctx, s) && ctx->recorded[s]) {
      SMP_HIP(ctx, hipEventSynchronize(ctx->events[2 * s + 1]));
      SMP_HIP(ctx, hipEventElapsedTime(&ms[s], ctx->events[2 * s], ctx->events[2 * s + 1]));
    }
  }
  return SMP_OK;
}

smp_status smp_workspace_size(const smp_params *p, size_t *bytes) {
  const std::string m = check(p);
  if (!m.empty()) return fail(nullptr, SMP_ERR_INVALID_ARG, m);
  if (!bytes) return fail(nullptr, SMP_ERR_INVALID_ARG, "bytes is NULL");
  SketchPlan pl = plan_for(p);
  const int64_t nt = p->n1 + p->n2, k = p->k;
  size_t s = 0;
  // sketch partials, for B given and for B = A (smp_solve treats B == A as SMP_B_IS_A)
  for (const int64_t n2 : {p->n2, int64_t(0)}) {
    if (n2 == 0 && p->n1 != p->n2) continue;
    int S = 0;
    launch_shape(p, n2, pl, S);
    const int slots = smp::sketch_slots_total(pl, S);
    s = std::max(s, al((size_t)slots * (p->n1 + n2) * pl.kpad * 4) + al((size_t)slots * (p->n1 + n2) * 8));
  }
  s += al(smp::sketch_pi_bytes(pl, p->d));                                  // stored-Pi window of the one-shot pass
  s += al(nt * k * 4) + al(nt * 4);                                       // sketches + norms
  s += al(64) + al(nt * 8) + al((nt / 256 + 4) * 8) + al((nt + 2) * 8);   // sampling
  const bool multi = (p->flags & SMP_SAMPLE_MULTINOMIAL) != 0;
  if (multi) s += al(smp::mn_ws_bytes(p->n1, p->n2, p->m));               // multinomial draws and sorts
  const double nnz = std::min<double>((double)p->n1 * (double)p->n2,
                                      multi ? (double)smp::mn_draw_bound(p->n1, p->m)
                                            : p->m + 6.0 * std::sqrt(p->m) + 64.0);
  s += 2 * al((size_t)(p->n1 + p->n2 + 2) * 8) + (size_t)(nnz * (4 + 8 + 8 + 1) * 2) + 8 * 256;  // omega
  s += 2 * al(nt * 8);                                                    // estimate
  s += smp::waltmin_ws_bytes(p->n1, p->n2, p->r, (int64_t)nnz);
  *bytes = s;
  return SMP_OK;
}

smp_status smp_pi_fill(smp_ctx *ctx, const smp_params *p, int64_t l0, int64_t nrows, float *out) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  if (l0 < 0 || nrows < 0 || l0 + nrows > p->d) return fail(ctx, SMP_ERR_INVALID_ARG, "rows out of [0, d)");
  if (nrows > 0 && !out) return fail(ctx, SMP_ERR_INVALID_ARG, "out is NULL");
  if (nrows == 0) return SMP_OK;
  SMP_HIP(ctx, smp::pi_fill(l0, nrows, p->k, p->seed, out, ctx->stream));
  return SMP_OK;
}

// ---- sketch launch-shape tuning ------------------------------------------------------

smp_status smp_tune_sketch(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B,
                           int64_t ldb, int32_t *cap, int32_t *splits, double *ms) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  if (p->flags & SMP_SKETCH_SRHT) return fail(ctx, SMP_ERR_INVALID_ARG, "tuning covers the Gaussian passes");
  const bool same = (p->flags & SMP_B_IS_A) != 0;
  if (!A || lda < p->n1 || (!same && (!B || ldb < p->n2)))
    return fail(ctx, SMP_ERR_INVALID_ARG, "A/B is NULL or leading dimension too small");
  const int64_t n2 = same ? 0 : p->n2;
  const SketchPlan base = plan_for(p);
  // time the pass on the rows of (up to) four launches, so that the launches
  // after the first (which add into the partials of the ones before) weigh in
  // as they do in a long pass; the choice applies to every launch of the shape
  const int64_t wrows = launch_rows(base, p->d);
  smp_params q = *p;
  q.d = std::min<int64_t>(p->d, 4 * wrows);
  if (q.prec == SMP_PREC_FP8 && q.d != p->d) q.d = q.d / 32 * 32;
  const double launches = (double)((q.d + wrows - 1) / wrows);
  smp_ctx_bufs &b = bufs(ctx);
  const size_t ob = al(p->n1 * (size_t)p->k * 4) + al(n2 * (size_t)p->k * 4) + al(p->n1 * 4) + al(n2 * 4);
  smp_status s = ensure(ctx, b.tune, ob);
  if (s != SMP_OK) return s;
  char *c = static_cast<char *>(b.tune.p);
  float *At = take<float>(c, p->n1 * p->k);
  float *Bt = take<float>(c, n2 * p->k);
  float *na2 = take<float>(c, p->n1);
  float *nb2 = take<float>(c, n2);
  std::vector<int> caps = {0};
  if (base.prec == SMP_PREC_BF16 && base.pi_stored) caps = {13, 16};
  int64_t smin, smax;
  split_range(base, q.d, smin, smax);
  std::vector<int64_t> cands;
  for (int64_t v : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256})
    if (v >= smin && v <= smax) cands.push_back(v);
  if (cands.empty()) cands.push_back(smin);
  // each candidate's cost: the launch (Pi window, main and tail launches) plus
  // the reduction of its partials spread over the launches of a whole pass
  const int saved_timing = ctx->timing;
  s = smp_set_timing(ctx, 1);
  if (s != SMP_OK) return s;
  const double share = (double)q.d / (double)p->d;
  smp::TuneChoice best{0, 0, 1e300};
  smp_status rs = SMP_OK;
  for (int cp : caps) {
    for (int64_t sv : cands) {
      const smp::TuneChoice trial{cp, (int)sv, 0.0};
      t_trial = &trial;
      double t[6];
      for (int rep = 0; rep < 6 && rs == SMP_OK; ++rep) {   // one warm-up, five timed
        rs = smp_sketch(ctx, &q, A, lda, same ? nullptr : B, ldb, At, same ? nullptr : Bt, na2, same ? nullptr : nb2);
        float st[5] = {0, 0, 0, 0, 0};
        if (rs == SMP_OK) rs = smp_stage_times(ctx, st, 5);
        t[rep] = ((double)st[0] + share * (double)st[1]) / launches;
      }
      t_trial = nullptr;
      if (rs != SMP_OK) break;
      std::sort(t + 1, t + 6);
      if (t[3] < best.ms) best = smp::TuneChoice{cp, (int)sv, t[3]};
    }
    if (rs != SMP_OK) break;
  }
  smp_set_timing(ctx, saved_timing);
  if (rs != SMP_OK) return rs;
  smp::tune_store(tune_key(p, base, n2), best);
  if (cap) *cap = best.cap;
  if (splits) *splits = best.splits;
  if (ms) *ms = best.ms;
  return SMP_OK;
}

smp_status smp_tune_lookup(const smp_params *p, int32_t *cap, int32_t *splits) {
  const std::string m = check(p);
  if (!m.empty()) return fail(nullptr, SMP_ERR_INVALID_ARG, m);
  if (!cap || !splits) return fail(nullptr, SMP_ERR_INVALID_ARG, "cap or splits is NULL");
  const SketchPlan pl = plan_for(p);
  smp::TuneChoice c{};
  if (!smp::tune_lookup(tune_key(p, pl, (p->flags & SMP_B_IS_A) ? 0 : p->n2), c)) c = smp::TuneChoice{0, 0, 0.0};
  *cap = c.cap;
  *splits = c.splits;
  return SMP_OK;
}

smp_status smp_tune_save(const char *path) {
  if (!path) return fail(nullptr, SMP_ERR_INVALID_ARG, "path is NULL");
  const std::string e = smp::tune_save(path);
  return e.empty() ? SMP_OK : fail(nullptr, SMP_ERR_INVALID_ARG, e);
}

smp_status smp_tune_load(const char *path) {
  if (!path) return fail(nullptr, SMP_ERR_INVALID_ARG, "path is NULL");
  const std::string e = smp::tune_load(path);
  return e.empty() ? SMP_OK : fail(nullptr, SMP_ERR_INVALID_ARG, e);
}

void smp_tune_clear(void) { smp::tune_clear(); }

smp_status smp_sketch_begin(smp_ctx *ctx, const smp_params *p, smp_sketch_state **st) {
  if (!ctx || !st) return fail(ctx, SMP_ERR_INVALID_ARG, "ctx or st is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  auto *s = new (std::nothrow) smp_sketch_state();
  if (!s) return fail(ctx, SMP_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->ctx = ctx;
  s->p = *p;
  launch_shape(p, (p->flags & SMP_B_IS_A) ? 0 : p->n2, s->plan, s->S);
  const int64_t n2 = (p->flags & SMP_B_IS_A) ? 0 : p->n2;
  const int64_t nt = p->n1 + n2;
  const int slots = smp::sketch_slots_total(s->plan, s->S);
  const size_t pb = (size_t)slots * nt * s->plan.kpad * sizeof(float);
  const size_t nb = (size_t)slots * nt * sizeof(double);
  if (hipMalloc((void **)&s->part, pb) != hipSuccess || hipMalloc((void **)&s->npart, nb) != hipSuccess) {
    hipGetLastError();
    if (s->part) hipFree(s->part);
    delete s;
    return fail(ctx, SMP_ERR_OUT_OF_MEMORY, "sketch state allocation failed");
  }
  SMP_HIP(ctx, hipMemsetAsync(s->part, 0, pb, ctx->stream));
  SMP_HIP(ctx, hipMemsetAsync(s->npart, 0, nb, ctx->stream));
  s->ended = false;
  *st = s;
  return SMP_OK;
}

smp_status smp_sketch_push(smp_ctx *ctx, smp_sketch_state *st, const float *A_rows, int64_t lda, const float *B_rows,
                           int64_t ldb, int64_t row0, int64_t nrows) {
  if (!ctx || !st) return fail(ctx, SMP_ERR_INVALID_ARG, "ctx or st is NULL");
  if (st->ended) return fail(ctx, SMP_ERR_STATE, "push after end");
  const smp_params &p = st->p;
  const bool same = (p.flags & SMP_B_IS_A) != 0;
  if (row0 < 0 || nrows < 0 || row0 + nrows > p.d) return fail(ctx, SMP_ERR_INVALID_ARG, "rows out of [0, d)");
  if (nrows == 0) return SMP_OK;
  if (!A_rows || lda < p.n1) return fail(ctx, SMP_ERR_INVALID_ARG, "A is NULL or lda < n1");
  if (p.prec == SMP_PREC_FP8 && (row0 % 32 != 0 || (nrows % 32 != 0 && row0 + nrows != p.d)))
    return fail(ctx, SMP_ERR_INVALID_ARG, "FP8 pushes must cover whole 32-row scaling blocks");
  if (!same && (!B_rows || ldb < p.n2)) return fail(ctx, SMP_ERR_INVALID_ARG, "B is NULL or ldb < n2");
  const size_t need = smp::sketch_pi_bytes(st->plan, nrows);
  if (need > st->pi_bytes) {   // grow the stored-Pi scratch (earlier pushes may still read the old one)
    SMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (st->pi) hipFree(st->pi);
    st->pi = nullptr;
    st->pi_bytes = 0;
    if (hipMalloc(&st->pi, need) != hipSuccess) {
      hipGetLastError();
      st->pi = nullptr;
      return fail(ctx, SMP_ERR_OUT_OF_MEMORY, "stored-Pi scratch allocation failed");
    }
    st->pi_bytes = need;
  }
  SMP_HIP(ctx, smp::sketch_push(st->plan, A_rows, lda, p.n1, same ? nullptr : B_rows, ldb, same ? 0 : p.n2, row0,
                                nrows, p.k, p.seed, st->S, true, st->part, st->npart, st->pi, ctx->stream));
  return SMP_OK;
}

smp_status smp_sketch_end(smp_ctx *ctx, smp_sketch_state *st, float *At, float *Bt, float *na2, float *nb2) {
  if (!ctx || !st) return fail(ctx, SMP_ERR_INVALID_ARG, "ctx or st is NULL");
  const smp_params &p = st->p;
  const bool same = (p.flags & SMP_B_IS_A) != 0;
  if (!At || !na2) return fail(ctx, SMP_ERR_INVALID_ARG, "At or na2 is NULL");
  if (!same && (!Bt || !nb2)) return fail(ctx, SMP_ERR_INVALID_ARG, "Bt or nb2 is NULL");
  const int64_t n2 = same ? 0 : p.n2;
  SMP_HIP(ctx, smp::sketch_finish(st->plan, st->part, st->npart, smp::sketch_slots_total(st->plan, st->S), p.n1, n2,
                                  p.k, At, same ? nullptr : Bt, na2,
                                  same ? nullptr : nb2, ctx->stream));
  if (same) {
    if (Bt && Bt != At)
      SMP_HIP(ctx, hipMemcpyAsync(Bt, At, (size_t)p.n1 * p.k * 4, hipMemcpyDeviceToDevice, ctx->stream));
    if (nb2 && nb2 != na2)
      SMP_HIP(ctx, hipMemcpyAsync(nb2, na2, (size_t)p.n1 * 4, hipMemcpyDeviceToDevice, ctx->stream));
  }
  st->ended = true;
  return SMP_OK;
}

void smp_sketch_free(smp_sketch_state *st) {
  if (!st) return;
  hipStreamSynchronize(st->ctx->stream);
  hipFree(st->part);
  hipFree(st->npart);
  if (st->pi) hipFree(st->pi);
  delete st;
}

// ---- entry pushes (f4): triples in any order ------------------------------------------

static smp_status push_entries(smp_ctx *ctx, smp_sketch_state *st, int which, const smp::SparseIn &in) {
  if (!ctx || !st) return fail(ctx, SMP_ERR_INVALID_ARG, "ctx or st is NULL");
  if (st->ended) return fail(ctx, SMP_ERR_STATE, "push after end");
  const smp_params &p = st->p;
  const bool same = (p.flags & SMP_B_IS_A) != 0;
  if (which != SMP_MAT_A && which != SMP_MAT_B) return fail(ctx, SMP_ERR_INVALID_ARG, "which must be SMP_MAT_A or SMP_MAT_B");
  if (same && which == SMP_MAT_B) return fail(ctx, SMP_ERR_INVALID_ARG, "B is A (SMP_B_IS_A): push the entries as A");
  if (p.prec == SMP_PREC_FP8)
    return fail(ctx, SMP_ERR_INVALID_ARG,
                "entry pushes need an FP32, BF16 or SRHT sketch (FP8 scales need whole 32-row blocks of a column)");
  if (in.nnz < 0 || in.nnz > INT32_MAX) return fail(ctx, SMP_ERR_INVALID_ARG, "nnz must be in [0, 2^31)");
  if (in.nnz == 0) return SMP_OK;
  if (!in.cols || !in.vals || (!in.rows && !in.row_ptr)) return fail(ctx, SMP_ERR_INVALID_ARG, "an entry array is NULL");
  const int64_t n = which == SMP_MAT_A ? p.n1 : p.n2;
  if (!smp::sparse_key_fits(p.d, n)) return fail(ctx, SMP_ERR_INVALID_ARG, "d * (n + 1) must be below 2^64");
  // the context's scratch, grown to the largest push (pushes run in stream order)
  smp_ctx_bufs &b = bufs(ctx);
  const smp_status s = ensure(ctx, b.sparse, smp::sparse_ws_bytes(in.nnz, n, st->plan.kpad));
  if (s != SMP_OK) return s;
  const int64_t off = which == SMP_MAT_B ? p.n1 : 0;
  auto *res = reinterpret_cast<smp::SpStatus *>(ctx->host_pinned);
  SMP_HIP(ctx, smp::sparse_prepare(st->plan, in, p.d, n, b.sparse.p, res, ctx->stream));
  if (res->bad_index) return fail(ctx, SMP_ERR_INVALID_ARG, "an entry's row or column index is out of range");
  if (res->bad_ptr) return fail(ctx, SMP_ERR_INVALID_ARG, "row_ptr must start at 0, end at nnz and not decrease");
  if (res->dup) return fail(ctx, SMP_ERR_INVALID_ARG, "an entry (row, column) occurs more than once in the push");
  const smp::SpStatus prep = *res;
  mark(ctx, kStSketch, false);   // stage [0]: the accumulation kernels of this push
  SMP_HIP(ctx, smp::sparse_accumulate(st->plan, in, p.d, n, p.k, p.seed, st->part + off * st->plan.kpad,
                                      st->npart + off, b.sparse.p, prep, ctx->stream));
  mark(ctx, kStSketch, true);
  return SMP_OK;
}

smp_status smp_sketch_push_coo(smp_ctx *ctx, smp_sketch_state *st, int which, const int64_t *rows,
                               const int32_t *cols, const float *vals, int64_t nnz) {
  smp::SparseIn in;
  in.rows = rows;
  in.cols = cols;
  in.vals = vals;
  in.nnz = nnz;
  if (nnz > 0 && !rows) return fail(ctx, SMP_ERR_INVALID_ARG, "rows is NULL");
  return push_entries(ctx, st, which, in);
}

smp_status smp_sketch_push_csr(smp_ctx *ctx, smp_sketch_state *st, int which, int64_t row0, int64_t nrows,
                               const int64_t *row_ptr, const int32_t *cols, const float *vals, int64_t nnz) {
  if (st && (row0 < 0 || nrows < 0 || row0 + nrows > st->p.d))
    return fail(ctx, SMP_ERR_INVALID_ARG, "rows out of [0, d)");
  if (nrows == 0 && nnz != 0) return fail(ctx, SMP_ERR_INVALID_ARG, "entries given for zero rows");
  if (nnz > 0 && !row_ptr) return fail(ctx, SMP_ERR_INVALID_ARG, "row_ptr is NULL");
  smp::SparseIn in;
  in.row_ptr = row_ptr;
  in.row0 = row0;
  in.nrows = nrows;
  in.cols = cols;
  in.vals = vals;
  in.nnz = nnz;
  return push_entries(ctx, st, which, in);
}

smp_status smp_sketch_group(smp_ctx *ctx, int njobs, const smp_params *p, const float *const *A,
                            const int64_t *lda, const float *const *B, const int64_t *ldb, float *const *At,
                            float *const *Bt, float *const *na2, float *const *nb2) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  if (njobs < 0 || njobs > 65535) return fail(ctx, SMP_ERR_INVALID_ARG, "njobs outside [0, 65535]");
  if (njobs == 0) return SMP_OK;
  if (!p || !A || !lda || !B || !ldb || !At || !Bt || !na2 || !nb2)
    return fail(ctx, SMP_ERR_INVALID_ARG, "an argument array is NULL");
  std::vector<smp::GroupSketchJob> jobs(njobs);
  for (int j = 0; j < njobs; ++j) {
    const std::string m = check(&p[j]);
    const std::string pre = "job " + std::to_string(j) + ": ";
    if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, pre + m);
    if (p[j].prec != SMP_PREC_BF16) return fail(ctx, SMP_ERR_INVALID_ARG, pre + "smp_sketch_group runs BF16 jobs only");
    if (p[j].flags & SMP_SKETCH_SRHT) return fail(ctx, SMP_ERR_INVALID_ARG, pre + "the SRHT sketch is not grouped");
    const bool same = (p[j].flags & SMP_B_IS_A) != 0;
    if (!A[j] || lda[j] < p[j].n1) return fail(ctx, SMP_ERR_INVALID_ARG, pre + "A is NULL or lda < n1");
    if (!same && (!B[j] || ldb[j] < p[j].n2)) return fail(ctx, SMP_ERR_INVALID_ARG, pre + "B is NULL or ldb < n2");
    if (!At[j] || !na2[j] || (!same && (!Bt[j] || !nb2[j])))
      return fail(ctx, SMP_ERR_INVALID_ARG, pre + "output pointer is NULL");
    jobs[j] = smp::GroupSketchJob{A[j], same ? nullptr : B[j], lda[j], same ? 0 : ldb[j], p[j].n1,
                                  same ? p[j].n1 : p[j].n2, p[j].d, (int)p[j].k, p[j].seed,
                                  At[j], Bt[j], na2[j], nb2[j]};
  }
  const size_t need = smp::bf16_group_scratch_bytes(jobs.data(), njobs);
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.skgroup, need);
  if (s != SMP_OK) return s;
  SMP_HIP(ctx, smp::bf16_sketch_group(jobs.data(), njobs, b.skgroup.p, b.skgroup.bytes, ctx->stream));
  return SMP_OK;
}

smp_status smp_sketch(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B, int64_t ldb,
                      float *At, float *Bt, float *na2, float *nb2) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  const bool same = (p->flags & SMP_B_IS_A) != 0;
  if (!A || lda < p->n1) return fail(ctx, SMP_ERR_INVALID_ARG, "A is NULL or lda < n1");
  if (!same && (!B || ldb < p->n2)) return fail(ctx, SMP_ERR_INVALID_ARG, "B is NULL or ldb < n2");
  if (!At || !na2 || (!same && (!Bt || !nb2))) return fail(ctx, SMP_ERR_INVALID_ARG, "output pointer is NULL");
  // the one-shot pass keeps its partials in the context's workspace
  const int64_t n2 = same ? 0 : p->n2;   // B = A: only A's column tiles run
  SketchPlan pl;
  int S = 0;
  launch_shape(p, n2, pl, S);
  const int64_t nt = p->n1 + n2;
  const int slots = smp::sketch_slots_total(pl, S);
  const size_t pb = al((size_t)slots * nt * pl.kpad * 4), nb = al((size_t)slots * nt * 8);
  const size_t pib = al(smp::sketch_pi_bytes(pl, p->d));
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.sketch, pb + nb + pib);
  if (s != SMP_OK) return s;
  float *part = static_cast<float *>(b.sketch.p);
  double *npart = reinterpret_cast<double *>(static_cast<char *>(b.sketch.p) + pb);
  void *pi = pib ? static_cast<char *>(b.sketch.p) + pb + nb : nullptr;
  for (bool &r : ctx->recorded) r = false;
  mark(ctx, kStSketch, false);
  SMP_HIP(ctx, smp::sketch_push(pl, A, lda, p->n1, same ? nullptr : B, ldb, n2, 0, p->d, p->k, p->seed, S, false,
                                part, npart, pi, ctx->stream));
  mark(ctx, kStSketch, true);
  mark(ctx, kStFinish, false);
  SMP_HIP(ctx, smp::sketch_finish(pl, part, npart, slots, p->n1, n2, p->k, At, same ? nullptr : Bt, na2,
                                  same ? nullptr : nb2, ctx->stream));
  mark(ctx, kStFinish, true);
  if (same) {
    if (Bt && Bt != At)
      SMP_HIP(ctx, hipMemcpyAsync(Bt, At, (size_t)p->n1 * p->k * 4, hipMemcpyDeviceToDevice, ctx->stream));
    if (nb2 && nb2 != na2)
      SMP_HIP(ctx, hipMemcpyAsync(nb2, na2, (size_t)p->n1 * 4, hipMemcpyDeviceToDevice, ctx->stream));
  }
  return SMP_OK;
}

// The sampler's scratch (per-entry probabilities alpha, beta, the F totals,
// block sums and counts) in the context's buffer; carved the same way on every
// call, so a fill pass can follow a count pass made by an earlier call.
static smp_status sample_ws(smp_ctx *ctx, int64_t n1, int64_t n2, smp::SampleWs &ws) {
  const int64_t nt = n1 + n2;
  smp_ctx_bufs &b = bufs(ctx);
  const size_t need = al(64) + al(n1 * 8) + al(n2 * 8) + al((nt / 256 + 4) * 8) + al((nt + 2) * 8);
  smp_status s = ensure(ctx, b.samplews, need);
  if (s != SMP_OK) return s;
  char *c = static_cast<char *>(b.samplews.p);
  ws.stats = take<double>(c, 8);
  ws.alpha = take<double>(c, n1);
  ws.beta = take<double>(c, n2);
  ws.blocks = take<double>(c, nt / 256 + 4);
  ws.cnt = take<int64_t>(c, nt + 2);
  return SMP_OK;
}

// The multinomial sampler's scratch in the context's buffer (carved the same
// way on every call, like sample_ws).
static smp_status mn_ws(smp_ctx *ctx, int64_t n1, int64_t n2, double m, smp::MnWs &w) {
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.mn, smp::mn_ws_bytes(n1, n2, m));
  if (s != SMP_OK) return s;
  smp::mn_ws_carve(b.mn.p, n1, n2, m, w);
  return SMP_OK;
}

// The fill pass of the sampler selected by p->flags, after its count pass.
static hipError_t sample_fill_any(smp_ctx *ctx, const smp_params *p, const smp::SampleWs &ws, const smp_omega &om) {
  const int split = p->omega_mode == SMP_OMEGA_SPLIT ? 1 : 0;
  if (p->flags & SMP_SAMPLE_MULTINOMIAL) {
    smp::MnWs mws;
    smp::mn_ws_carve(bufs(ctx).mn.p, p->n1, p->n2, p->m, mws);
    return smp::mn_fill(ws, mws, p->n1, p->n2, p->m, p->seed, p->T, split, om, ctx->stream);
  }
  return smp::sample_fill(ws, p->n1, p->n2, p->m, p->seed, p->T, split, om, ctx->stream);
}

smp_status smp_sample(smp_ctx *ctx, const smp_params *p, const float *na2, const float *nb2, smp_omega *om) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  if (!na2 || !nb2 || !om) return fail(ctx, SMP_ERR_INVALID_ARG, "na2, nb2 or om is NULL");
  if (om->n1 != p->n1 || om->n2 != p->n2) return fail(ctx, SMP_ERR_INVALID_ARG, "om grid differs from params");
  if (!om->row_ptr || !om->col_ptr || (om->cap > 0 && (!om->col_idx || !om->w_csr || !om->row_idx || !om->w_csc)))
    return fail(ctx, SMP_ERR_INVALID_ARG, "om index or weight array is NULL");
  const bool split = p->omega_mode == SMP_OMEGA_SPLIT;
  if (split && om->cap > 0 && (!om->sub_csr || !om->sub_csc))
    return fail(ctx, SMP_ERR_INVALID_ARG, "SPLIT mode needs sub_csr and sub_csc");
  const int64_t n1 = p->n1, n2 = p->n2;
  const bool multi = (p->flags & SMP_SAMPLE_MULTINOMIAL) != 0;
  smp::SampleWs ws;
  smp_status s = sample_ws(ctx, n1, n2, ws);
  if (s != SMP_OK) return s;
  smp::MnWs mws;
  if (multi && (s = mn_ws(ctx, n1, n2, p->m, mws)) != SMP_OK) return s;
  SMP_HIP(ctx, smp::sample_prepare(na2, nb2, n1, n2, ws, ctx->stream));
  if (multi) {
    SMP_HIP(ctx, smp::mn_count(ws, mws, n1, n2, p->m, p->seed, om->row_ptr, ctx->stream));
    SMP_HIP(ctx, hipMemcpyAsync(ctx->host_pinned + 1, mws.doff + n1, 8, hipMemcpyDeviceToHost, ctx->stream));
  } else {
    SMP_HIP(ctx, smp::sample_count(ws, n1, n2, p->m, p->seed, om->row_ptr, om->col_ptr, ws.cnt, ctx->stream));
    SMP_HIP(ctx, hipMemcpyAsync(ctx->host_pinned + 1, om->col_ptr + n2, 8, hipMemcpyDeviceToHost, ctx->stream));
  }
  SMP_HIP(ctx, hipMemcpyAsync(ctx->host_pinned, om->row_ptr + n1, 8, hipMemcpyDeviceToHost, ctx->stream));
  SMP_HIP(ctx, hipMemcpyAsync(ctx->host_pinned + 2, ws.stats + 4, 8, hipMemcpyDeviceToHost, ctx->stream));
  SMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  double nonfinite = 0.0;
  std::memcpy(&nonfinite, ctx->host_pinned + 2, sizeof(double));
  if (nonfinite != 0.0)
    return fail(ctx, SMP_ERR_NUMERIC, "non-finite input: ||A||_F^2 or ||B||_F^2 is not finite (NaN or Inf in A or B)");
  const int64_t nnz = ctx->host_pinned[0];
  if (multi) {
    if (ctx->host_pinned[1] > mws.dmax || nnz > ctx->host_pinned[1])
      return fail(ctx, SMP_ERR_DEVICE, "multinomial draws exceed their bound");
  } else if (nnz != ctx->host_pinned[1]) {
    return fail(ctx, SMP_ERR_DEVICE, "row and column listings disagree on |Omega|");
  }
  om->nnz = nnz;
  if (nnz > om->cap)
    return fail(ctx, SMP_ERR_CAPACITY, "|Omega| = " + std::to_string(nnz) + " exceeds cap " + std::to_string(om->cap));
  SMP_HIP(ctx, sample_fill_any(ctx, p, ws, *om));
  return SMP_OK;
}

smp_status smp_estimate(smp_ctx *ctx, const smp_params *p, const float *At, const float *Bt, const float *na2,
                        const float *nb2, smp_omega *om) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  if (!At || !Bt || !na2 || !nb2 || !om) return fail(ctx, SMP_ERR_INVALID_ARG, "input pointer is NULL");
  if (om->n1 != p->n1 || om->n2 != p->n2) return fail(ctx, SMP_ERR_INVALID_ARG, "om grid differs from params");
  if (om->nnz > 0 && (!om->mt_csr || !om->mt_csc)) return fail(ctx, SMP_ERR_INVALID_ARG, "mt arrays are NULL");
  const int64_t n1 = p->n1, n2 = p->n2;
  const bool same = At == Bt && na2 == nb2;
  smp_ctx_bufs &b = bufs(ctx);
  const size_t need = 2 * al(n1 * 8) + 2 * al(n2 * 8);
  smp_status s = ensure(ctx, b.est, need);
  if (s != SMP_OK) return s;
  char *c = static_cast<char *>(b.est.p);
  double *na = take<double>(c, n1);
  double *nb = take<double>(c, n2);
  double *sa = take<double>(c, n1);
  double *sb = take<double>(c, n2);
  if (same) {
    nb = na;
    sb = sa;
  }
  SMP_HIP(ctx, smp::estimate_run(At, Bt, na2, nb2, n1, n2, p->k, na, nb, sa, sb, *om, ctx->stream));
  return SMP_OK;
}

smp_status smp_estimate_noalloc(smp_ctx *ctx, const smp_params *p, const float *At, const float *Bt,
                                const float *na2, const float *nb2, smp_omega *om) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  if (!At || !Bt || !na2 || !nb2 || !om) return fail(ctx, SMP_ERR_INVALID_ARG, "input pointer is NULL");
  if (om->n1 != p->n1 || om->n2 != p->n2) return fail(ctx, SMP_ERR_INVALID_ARG, "om grid differs from params");
  if (om->nnz > 0 && (!om->mt_csr || !om->mt_csc)) return fail(ctx, SMP_ERR_INVALID_ARG, "mt arrays are NULL");
  const int64_t n1 = p->n1, n2 = p->n2;
  if (n1 + n2 > kNoAllocMaxCols)
    return fail(ctx, SMP_ERR_CAPACITY, "n1 + n2 = " + std::to_string(n1 + n2) +
                                           " exceeds the allocation-free limit of " + std::to_string(kNoAllocMaxCols));
  double *base = static_cast<double *>(scratch_for(ctx->device));
  if (!base) return fail(ctx, SMP_ERR_DEVICE, "no scratch address for this device");
  const bool same = At == Bt && na2 == nb2;
  double *na = base, *nb = base + n1, *sa = base + n1 + n2, *sb = base + 2 * n1 + n2;
  if (same) {
    nb = na;
    sb = sa;
  }
  SMP_HIP(ctx, smp::estimate_run(At, Bt, na2, nb2, n1, n2, p->k, na, nb, sa, sb, *om, ctx->stream));
  return SMP_OK;
}

// WAltMin on the context's workspace; fa: F_A already on the device (the
// sampler's, in the same summation order), or null to sum it from na2.
static smp_status waltmin_call(smp_ctx *ctx, const smp_params *p, const smp_omega *om, const float *na2, double *U,
                               double *V, double *sigma, const double *fa) {
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.wm, smp::waltmin_ws_bytes(p->n1, p->n2, p->r, om->nnz));
  if (s != SMP_OK) return s;
  SMP_HIP(ctx, smp::waltmin_run(*p, *om, na2, U, V, sigma, b.wm.p, ctx->stream, fa));
  return SMP_OK;
}

smp_status smp_waltmin(smp_ctx *ctx, const smp_params *p, const smp_omega *om, const float *na2, double *U, double *V,
                       double *sigma) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  if (!om || !na2 || !U || !V) return fail(ctx, SMP_ERR_INVALID_ARG, "input or output pointer is NULL");
  if (om->n1 != p->n1 || om->n2 != p->n2) return fail(ctx, SMP_ERR_INVALID_ARG, "om grid differs from params");
  if (p->omega_mode == SMP_OMEGA_SPLIT && om->nnz > 0 && (!om->sub_csr || !om->sub_csc))
    return fail(ctx, SMP_ERR_INVALID_ARG, "SPLIT mode needs sub_csr and sub_csc");
  return waltmin_call(ctx, p, om, na2, U, V, sigma, nullptr);
}

smp_status smp_waltmin_group(smp_ctx *ctx, int njobs, const smp_params *p, const smp_omega *om,
                             const float *const *na2, double *const *U, double *const *V, double *const *sigma,
                             int graph) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  if (njobs < 0) return fail(ctx, SMP_ERR_INVALID_ARG, "njobs < 0");
  if (njobs == 0) return SMP_OK;
  if (!p || !om || !na2 || !U || !V) return fail(ctx, SMP_ERR_INVALID_ARG, "an array argument is NULL");
  size_t total = 0;
  std::vector<size_t> wsz(njobs);
  for (int j = 0; j < njobs; ++j) {
    const std::string m = check(&p[j]);
    if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, "job " + std::to_string(j) + ": " + m);
    if (!na2[j] || !U[j] || !V[j]) return fail(ctx, SMP_ERR_INVALID_ARG, "job " + std::to_string(j) + ": NULL pointer");
    if (om[j].n1 != p[j].n1 || om[j].n2 != p[j].n2)
      return fail(ctx, SMP_ERR_INVALID_ARG, "job " + std::to_string(j) + ": om grid differs from params");
    if (p[j].omega_mode == SMP_OMEGA_SPLIT && om[j].nnz > 0 && (!om[j].sub_csr || !om[j].sub_csc))
      return fail(ctx, SMP_ERR_INVALID_ARG, "job " + std::to_string(j) + ": SPLIT mode needs sub_csr and sub_csc");
    wsz[j] = al(smp::waltmin_ws_bytes(p[j].n1, p[j].n2, p[j].r, om[j].nnz));
    total += wsz[j];
  }
  const size_t tb = al(smp::waltmin_group_table_bytes(njobs, p, om));
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.group, total + tb);
  if (s != SMP_OK) return s;
  std::vector<void *> ws(njobs);
  char *c = static_cast<char *>(b.group.p);
  for (int j = 0; j < njobs; ++j) {
    ws[j] = c;
    c += wsz[j];
  }
  SMP_HIP(ctx, smp::waltmin_group_run(njobs, p, om, na2, U, V, sigma, ws.data(), nullptr, c, graph, ctx->stream));
  SMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return SMP_OK;
}

static smp_status solve_after_sketch(smp_ctx *ctx, const smp_params &q, const float *At, const float *Bt,
                                     const float *na2, const float *nb2, int64_t *rp, int64_t *cp, double *U,
                                     double *V, double *sigma);

smp_status smp_solve(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B, int64_t ldb,
                     double *U, double *V, double *sigma) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string msg = check(p);
  if (!msg.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, msg);
  smp_params q = *p;
  if (B == A && p->n1 == p->n2 && ldb == lda) q.flags |= SMP_B_IS_A;
  const bool same = (q.flags & SMP_B_IS_A) != 0;
  if (!A || lda < q.n1 || (!same && (!B || ldb < q.n2)))
    return fail(ctx, SMP_ERR_INVALID_ARG, "A/B is NULL or leading dimension too small");
  if (!U || !V) return fail(ctx, SMP_ERR_INVALID_ARG, "U or V is NULL");
  const int64_t n1 = q.n1, n2 = q.n2, k = q.k;
  smp_ctx_bufs &b = bufs(ctx);

  // sketches, norms and the listing offsets; the entry arrays are sized after counting
  const size_t head = al(n1 * k * 4) + al(n2 * k * 4) + al(n1 * 4) + al(n2 * 4) + al((n1 + 2) * 8) + al((n2 + 2) * 8);
  smp_status s = ensure(ctx, b.head, head);
  if (s != SMP_OK) return s;
  char *hc = static_cast<char *>(b.head.p);
  float *At = take<float>(hc, n1 * k);
  float *Bt = take<float>(hc, n2 * k);
  float *na2 = take<float>(hc, n1);
  float *nb2 = take<float>(hc, n2);
  int64_t *rp = take<int64_t>(hc, n1 + 2);
  int64_t *cp = take<int64_t>(hc, n2 + 2);
  s = smp_sketch(ctx, &q, A, lda, B, ldb, At, Bt, na2, nb2);
  if (s != SMP_OK) return s;
  return solve_after_sketch(ctx, q, At, same ? At : Bt, na2, same ? na2 : nb2, rp, cp, U, V, sigma);
}

// Alg. 1 steps 3-5 from the sketches and norms: sampling, estimates, WAltMin.
static smp_status solve_after_sketch(smp_ctx *ctx, const smp_params &q, const float *At, const float *Bt,
                                     const float *na2, const float *nb2, int64_t *rp, int64_t *cp, double *U,
                                     double *V, double *sigma) {
  const int64_t n1 = q.n1, n2 = q.n2;
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s;
  // Omega: count first (one readback), then size the entry arrays exactly
  smp_omega om{};
  om.n1 = n1;
  om.n2 = n2;
  om.cap = 0;
  om.row_ptr = rp;
  om.col_ptr = cp;
  mark(ctx, kStSample, false);
  s = smp_sample(ctx, &q, na2, nb2, &om);
  if (s != SMP_OK && s != SMP_ERR_CAPACITY) return s;
  const int64_t nnz = om.nnz;
  const bool split = q.omega_mode == SMP_OMEGA_SPLIT;
  const size_t ent = 2 * (al(nnz * 4) + al(nnz * 8) + al(nnz * 8) + (split ? al(nnz) : 0));
  s = ensure(ctx, b.omega, std::max<size_t>(ent, 256));
  if (s != SMP_OK) return s;
  char *c = static_cast<char *>(b.omega.p);
  om.cap = nnz;
  om.col_idx = take<int32_t>(c, nnz);
  om.w_csr = take<double>(c, nnz);
  om.mt_csr = take<double>(c, nnz);
  om.row_idx = take<int32_t>(c, nnz);
  om.w_csc = take<double>(c, nnz);
  om.mt_csc = take<double>(c, nnz);
  om.sub_csr = split ? take<uint8_t>(c, nnz) : nullptr;
  om.sub_csc = split ? take<uint8_t>(c, nnz) : nullptr;
  if (nnz > 0) {
    // the counting call above left alpha, beta and the listings' pointers in
    // place: only the fill pass remains
    smp::SampleWs ws;
    s = sample_ws(ctx, n1, n2, ws);
    if (s != SMP_OK) return s;
    SMP_HIP(ctx, sample_fill_any(ctx, &q, ws, om));
  }
  mark(ctx, kStSample, true);
  mark(ctx, kStEstimate, false);
  s = smp_estimate(ctx, &q, At, Bt, na2, nb2, &om);
  if (s != SMP_OK) return s;
  mark(ctx, kStEstimate, true);
  mark(ctx, kStWaltmin, false);
  {
    smp::SampleWs sws;   // the sampler's F_A (stats[0]) is the trim's
    s = sample_ws(ctx, n1, n2, sws);
    if (s != SMP_OK) return s;
    s = waltmin_call(ctx, &q, &om, na2, U, V, sigma, sws.stats);
  }
  if (s != SMP_OK) return s;
  mark(ctx, kStWaltmin, true);
  SMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return SMP_OK;
}

smp_status smp_solve_sketched(smp_ctx *ctx, const smp_params *p, const float *At, const float *Bt, const float *na2,
                              const float *nb2, double *U, double *V, double *sigma) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string msg = check(p);
  if (!msg.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, msg);
  const bool same = (p->flags & SMP_B_IS_A) != 0;
  if (!At || !na2 || (!same && (!Bt || !nb2))) return fail(ctx, SMP_ERR_INVALID_ARG, "a sketch or norm pointer is NULL");
  if (!U || !V) return fail(ctx, SMP_ERR_INVALID_ARG, "U or V is NULL");
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.head, al((p->n1 + 2) * 8) + al((p->n2 + 2) * 8));
  if (s != SMP_OK) return s;
  char *hc = static_cast<char *>(b.head.p);
  int64_t *rp = take<int64_t>(hc, p->n1 + 2);
  int64_t *cp = take<int64_t>(hc, p->n2 + 2);
  return solve_after_sketch(ctx, *p, At, same ? At : Bt, na2, same ? na2 : nb2, rp, cp, U, V, sigma);
}

// ---- comparison methods (Section 4) -------------------------------------------------

smp_status smp_svd_sketch(smp_ctx *ctx, const smp_params *p, const float *At, const float *Bt, double *U, double *V,
                          double *sigma) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  if (!At || !Bt || !U || !V) return fail(ctx, SMP_ERR_INVALID_ARG, "input or output pointer is NULL");
  if (p->r > p->k) return fail(ctx, SMP_ERR_INVALID_ARG, "r must not exceed k (A~^T B~ has rank <= k)");
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.base, smp::svd_sketch_ws_bytes(p->n1, p->n2, p->k, p->r));
  if (s != SMP_OK) return s;
  const int iters = p->init_iters > 0 ? p->init_iters : 8;
  SMP_HIP(ctx, smp::svd_sketch_run(At, Bt, p->n1, p->n2, p->k, p->r, iters, p->seed, U, V, sigma, b.base.p,
                                   ctx->stream));
  return SMP_OK;
}

smp_status smp_solve_svd_sketch(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B,
                                int64_t ldb, double *U, double *V, double *sigma) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string msg = check(p);
  if (!msg.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, msg);
  smp_params q = *p;
  if (B == A && p->n1 == p->n2 && ldb == lda) q.flags |= SMP_B_IS_A;
  const bool same = (q.flags & SMP_B_IS_A) != 0;
  if (!A || lda < q.n1 || (!same && (!B || ldb < q.n2)))
    return fail(ctx, SMP_ERR_INVALID_ARG, "A/B is NULL or leading dimension too small");
  if (!U || !V) return fail(ctx, SMP_ERR_INVALID_ARG, "U or V is NULL");
  const int64_t n1 = q.n1, n2 = q.n2, k = q.k;
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.head, al(n1 * k * 4) + al(n2 * k * 4) + al(n1 * 4) + al(n2 * 4));
  if (s != SMP_OK) return s;
  char *hc = static_cast<char *>(b.head.p);
  float *At = take<float>(hc, n1 * k);
  float *Bt = take<float>(hc, n2 * k);
  float *na2 = take<float>(hc, n1);
  float *nb2 = take<float>(hc, n2);
  s = smp_sketch(ctx, &q, A, lda, B, ldb, At, Bt, na2, nb2);
  if (s != SMP_OK) return s;
  s = smp_svd_sketch(ctx, &q, At, same ? At : Bt, U, V, sigma);
  if (s != SMP_OK) return s;
  SMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return SMP_OK;
}

smp_status smp_column_norms(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B,
                            int64_t ldb, float *na2, float *nb2) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  const bool same = (p->flags & SMP_B_IS_A) != 0;
  if (!A || lda < p->n1 || !na2) return fail(ctx, SMP_ERR_INVALID_ARG, "A or na2 is NULL or lda < n1");
  if (!same && (!B || ldb < p->n2 || !nb2)) return fail(ctx, SMP_ERR_INVALID_ARG, "B or nb2 is NULL or ldb < n2");
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.est, smp::norms_ws_bytes(p->n1, same ? p->n1 : p->n2));
  if (s != SMP_OK) return s;
  double *part = static_cast<double *>(b.est.p);
  SMP_HIP(ctx, smp::column_norms(A, lda, p->d, p->n1, na2, part, ctx->stream));
  if (same) {
    if (nb2 && nb2 != na2)
      SMP_HIP(ctx, hipMemcpyAsync(nb2, na2, (size_t)p->n1 * 4, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    SMP_HIP(ctx, smp::column_norms(B, ldb, p->d, p->n2, nb2, part, ctx->stream));
  }
  return SMP_OK;
}

smp_status smp_exact_entries(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B,
                             int64_t ldb, smp_omega *om) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string m = check(p);
  if (!m.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, m);
  const bool same = (p->flags & SMP_B_IS_A) != 0;
  if (same) {
    B = A;
    ldb = lda;
  }
  if (!A || !B || lda < p->n1 || ldb < p->n2 || !om) return fail(ctx, SMP_ERR_INVALID_ARG, "A, B or om is NULL");
  if (lda > INT32_MAX || ldb > INT32_MAX) return fail(ctx, SMP_ERR_INVALID_ARG, "leading dimension too large");
  if (om->n1 != p->n1 || om->n2 != p->n2) return fail(ctx, SMP_ERR_INVALID_ARG, "om grid differs from params");
  if (om->nnz > 0 && (!om->mt_csr || !om->mt_csc)) return fail(ctx, SMP_ERR_INVALID_ARG, "mt arrays are NULL");
  if (!ctx->blas && smp::blas_create(&ctx->blas) != hipSuccess) {
    ctx->blas = nullptr;
    return fail(ctx, SMP_ERR_DEVICE, "rocBLAS handle creation failed");
  }
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.base, smp::exact_entries_ws_bytes(p->n1, p->n2));
  if (s != SMP_OK) return s;
  SMP_HIP(ctx, smp::exact_entries(ctx->blas, A, lda, B, ldb, p->d, p->n1, p->n2, *om, b.base.p, ctx->stream));
  return SMP_OK;
}

smp_status smp_lela(smp_ctx *ctx, const smp_params *p, const float *A, int64_t lda, const float *B, int64_t ldb,
                    double *U, double *V, double *sigma) {
  if (!ctx) return fail(nullptr, SMP_ERR_INVALID_ARG, "ctx is NULL");
  const std::string msg = check(p);
  if (!msg.empty()) return fail(ctx, SMP_ERR_INVALID_ARG, msg);
  smp_params q = *p;
  if (B == A && p->n1 == p->n2 && ldb == lda) q.flags |= SMP_B_IS_A;
  const bool same = (q.flags & SMP_B_IS_A) != 0;
  if (!A || lda < q.n1 || (!same && (!B || ldb < q.n2)))
    return fail(ctx, SMP_ERR_INVALID_ARG, "A/B is NULL or leading dimension too small");
  if (!U || !V) return fail(ctx, SMP_ERR_INVALID_ARG, "U or V is NULL");
  const int64_t n1 = q.n1, n2 = q.n2;
  smp_ctx_bufs &b = bufs(ctx);
  smp_status s = ensure(ctx, b.head, al(n1 * 4) + al(n2 * 4) + al((n1 + 2) * 8) + al((n2 + 2) * 8));
  if (s != SMP_OK) return s;
  char *hc = static_cast<char *>(b.head.p);
  float *na2 = take<float>(hc, n1);
  float *nb2 = take<float>(hc, n2);
  int64_t *rp = take<int64_t>(hc, n1 + 2);
  int64_t *cp = take<int64_t>(hc, n2 + 2);
  // pass 1: column norms, then the sample of Eq. (1)
  s = smp_column_norms(ctx, &q, A, lda, B, ldb, na2, same ? na2 : nb2);
  if (s != SMP_OK) return s;
  smp_omega om{};
  om.n1 = n1;
  om.n2 = n2;
  om.row_ptr = rp;
  om.col_ptr = cp;
  s = smp_sample(ctx, &q, na2, same ? na2 : nb2, &om);
  if (s != SMP_OK && s != SMP_ERR_CAPACITY) return s;
  const int64_t nnz = om.nnz;
  const bool split = q.omega_mode == SMP_OMEGA_SPLIT;
  s = ensure(ctx, b.omega, std::max<size_t>(2 * (al(nnz * 4) + al(nnz * 8) + al(nnz * 8) + (split ? al(nnz) : 0)), 256));
  if (s != SMP_OK) return s;
  char *c = static_cast<char *>(b.omega.p);
  om.cap = nnz;
  om.col_idx = take<int32_t>(c, nnz);
  om.w_csr = take<double>(c, nnz);
  om.mt_csr = take<double>(c, nnz);
  om.row_idx = take<int32_t>(c, nnz);
  om.w_csc = take<double>(c, nnz);
  om.mt_csc = take<double>(c, nnz);
  om.sub_csr = split ? take<uint8_t>(c, nnz) : nullptr;
  om.sub_csc = split ? take<uint8_t>(c, nnz) : nullptr;
  smp::SampleWs ws;
  if (nnz > 0) {
    s = sample_ws(ctx, n1, n2, ws);
    if (s != SMP_OK) return s;
    SMP_HIP(ctx, sample_fill_any(ctx, &q, ws, om));
  }
  // pass 2: the exact entries on the sample, then WAltMin on them
  s = smp_exact_entries(ctx, &q, A, lda, same ? A : B, same ? lda : ldb, &om);
  if (s != SMP_OK) return s;
  s = sample_ws(ctx, n1, n2, ws);
  if (s != SMP_OK) return s;
  s = waltmin_call(ctx, &q, &om, na2, U, V, sigma, ws.stats);
  if (s != SMP_OK) return s;
  SMP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return SMP_OK;
}

}  // extern "C"

namespace {
smp_ctx_bufs &bufs(smp_ctx *ctx) { return *static_cast<smp_ctx_bufs *>(ctx->ws); }
}  // namespace

namespace smp {

size_t ctx_workspace_bytes(const smp_ctx *ctx) {
  const auto *b = static_cast<const smp_ctx_bufs *>(ctx->ws);
  size_t s = 0;
  for (const Buf *x : {&b->sketch, &b->samplews, &b->head, &b->omega, &b->est, &b->wm, &b->mn, &b->base})
    s += x->bytes;
  return s;
}

void ctx_release_workspace(smp_ctx *ctx) {
  auto *b = static_cast<smp_ctx_bufs *>(ctx->ws);
  hipStreamSynchronize(ctx->stream);
  for (Buf *x : {&b->sketch, &b->samplews, &b->head, &b->omega, &b->est, &b->wm, &b->mn, &b->base}) {
    if (x->p) hipFree(x->p);
    x->p = nullptr;
    x->bytes = 0;
  }
}

}  // namespace smp

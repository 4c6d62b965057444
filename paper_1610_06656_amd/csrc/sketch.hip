// The single pass of SMP-PCA (Alg. 1 step 2; Section 2 "Step 1"):
//   A~ = Pi A, B~ = Pi B (Pi k x d, i.i.d. N(0, 1/k)) and ||A_i||^2, ||B_j||^2,
// as one streaming split-K GEMM on the FP32 matrix cores of gfx950.
//
// Work decomposition. A workgroup of W waves owns
//   * a tile of 16*W*NV data columns of A or B (each lane holds NV adjacent
//     columns of one row, loaded with one vector load),
//   * a chunk of MT*16 sketch rows (k = 400 runs as two chunks of 13 m-tiles),
//   * one of S contiguous row ranges of the d rows (split-K).
// It streams its rows in chunks of KC. For every chunk the workgroup
// regenerates the MT*16 x KC block of Pi it needs from the Philox counter
// spec into LDS (Pi is never stored in HBM; rows past the range end get zero
// Pi entries) and feeds the data rows straight from HBM into
// v_mfma_f32_16x16x4_f32 as the B operand: lane (q, ph) of a wave supplies row
// ph of each 4-row K step for its NV columns, so n-tile v of the MFMA sees
// column (base + q*NV + v). The squared column norms are accumulated from the
// same registers with per-lane compensated (Kahan) FP32 sums. The S row ranges
// write FP32 partial sketches and FP64 partial norms; sketch_finish reduces
// them in a fixed order (deterministic, no atomics).
//
// Workgroups that read the same data tile (same column tile and row range,
// different sketch-row chunk) get consecutive logical ids placed on the same
// XCD, so the second read of the tile hits that XCD's L2.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "sketch_common.hpp"
#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {

namespace {

// Pi block for sketch rows [c0, c0 + 16 MT) and data rows [lg, lg + KC) into
// LDS as z (unscaled N(0,1)), layout P[row][c]. Every thread makes CPT Philox
// calls (4 sketch rows each); the calls past MT*64 only pad the trip count and
// land in a scratch slot. Sketch rows c >= k and data rows past the first
// `valid` of the block are zero.
template <int MT, int W, int KC>
__device__ __forceinline__ void gen_pi(float *P, int tid, uint64_t seed, uint64_t lg, int64_t valid, int c0, int k) {
  constexpr int kThreads = 64 * W;
  constexpr int MR = MT * 16, PST = MR + 4;
  constexpr int NCALL = MT * 4 * KC;
  constexpr int CPT = (NCALL + kThreads - 1) / kThreads;
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    const int idx = tid + u * kThreads;
    const int lr = idx / (MT * 4);
    const int cb = idx - lr * (MT * 4);
    const int c = c0 + cb * 4;
    float4 z = normals4(stream_call(seed, kTagPi, lg + (uint64_t)lr, (uint32_t)(c >> 2)));
    const bool rv = lr < valid;
    z.x = rv && c + 0 < k ? z.x : 0.f;
    z.y = rv && c + 1 < k ? z.y : 0.f;
    z.z = rv && c + 2 < k ? z.z : 0.f;
    z.w = rv && c + 3 < k ? z.w : 0.f;
    const int slot = (NCALL % kThreads == 0 || idx < NCALL) ? lr * PST + cb * 4 : KC * PST + tid * 4;
    *reinterpret_cast<float4 *>(&P[slot]) = z;
  }
}

template <int MT, int NV, int W, int KC, bool FULL>
__device__ __forceinline__ void sketch_loop(const SkArgs &g, const SkWork &w, int64_t col, int c0, float *P0,
                                            float *P1, v4f (&acc)[MT][NV], float (&ksum)[NV], float (&kcmp)[NV]) {
  constexpr int MR = MT * 16, PST = MR + 4;
  constexpr int NST = KC / 4;   // MFMA K steps per chunk
  const int tid = threadIdx.x;
  const int lane = tid & 63, q = lane & 15, ph = lane >> 4;
  const int64_t row_last = w.lend - 1;

  float xv[NST][NV];
#pragma unroll
  for (int st = 0; st < NST; ++st) sk_load_row<NV, FULL, true>(w.X, w.ld, w.n, w.lbeg + 4 * st + ph, row_last, col, xv[st]);
  gen_pi<MT, W, KC>(P0, tid, g.seed, (uint64_t)(g.row0 + w.lbeg), w.lend - w.lbeg, c0, g.k);

  int buf = 0;
  for (int64_t l = w.lbeg; l < w.lend; l += KC) {
    __syncthreads();   // Pi of this chunk is complete; the other buffer is free
    float *Pc = buf ? P1 : P0;
    float *Pn = buf ? P0 : P1;
    // prefetch the next chunk's rows and build its Pi block while this one is multiplied
    float xn[NST][NV];
#pragma unroll
    for (int st = 0; st < NST; ++st)
      sk_load_row<NV, FULL, true>(w.X, w.ld, w.n, l + KC + 4 * st + ph, row_last, col, xn[st]);
    gen_pi<MT, W, KC>(Pn, tid, g.seed, (uint64_t)(g.row0 + l + KC), w.lend - (l + KC), c0, g.k);

#pragma unroll
    for (int st = 0; st < NST; ++st) {
      const bool rv = l + 4 * st + ph <= row_last;   // rows past the split end re-read row_last
#pragma unroll
      for (int v = 0; v < NV; ++v) kahan_add(ksum[v], kcmp[v], rv ? xv[st][v] * xv[st][v] : 0.0f);
    }
#pragma unroll
    for (int st = 0; st < NST; ++st) {
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        const float af = Pc[(4 * st + ph) * PST + 16 * i + q];
#pragma unroll
        for (int v = 0; v < NV; ++v)
          acc[i][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, xv[st][v], acc[i][v], 0, 0, 0);
      }
    }
#pragma unroll
    for (int st = 0; st < NST; ++st)
#pragma unroll
      for (int v = 0; v < NV; ++v) xv[st][v] = xn[st][v];
    buf ^= 1;
  }
}

template <int MT, int NV, int W, int KC>
__global__ __launch_bounds__(64 * W) void sketch_kernel(SkArgs g) {
  constexpr int kThreads = 64 * W;
  constexpr int MR = MT * 16;          // sketch rows per workgroup
  constexpr int PST = MR + 4;          // LDS row stride (floats)
  constexpr int PBUF = KC * PST + kThreads * 4;   // one Pi block + a scratch slot per thread
  __shared__ __attribute__((aligned(16))) float P[2 * PBUF];

  SkWork w;
  if (!sk_decode(g, w)) return;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int q = lane & 15, ph = lane >> 4;
  const int64_t tile_col = (int64_t)w.tile * (16 * W * NV);
  const int64_t col = tile_col + wave * (16 * NV) + q * NV;
  const int c0 = w.kc * MT * 16;

  v4f acc[MT][NV];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[i][v] = v4f{0.f, 0.f, 0.f, 0.f};
  float ksum[NV], kcmp[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) ksum[v] = kcmp[v] = 0.0f;

  if (w.lbeg < w.lend) {   // an empty split still stores its zero partials
    if (w.vec_ok && tile_col + 16 * W * NV <= w.n)
      sketch_loop<MT, NV, W, KC, true>(g, w, col, c0, P, P + PBUF, acc, ksum, kcmp);
    else
      sketch_loop<MT, NV, W, KC, false>(g, w, col, c0, P, P + PBUF, acc, ksum, kcmp);
  }
  sk_epilogue<MT, NV>(g, w, col, c0, ph, acc, ksum, kcmp);
}

using KernelPtr = void (*)(SkArgs);

template <int NV, int W, int KC, int MT>
struct KTable {
  static void fill(KernelPtr *t) {
    t[MT] = sketch_kernel<MT, NV, W, KC>;
    KTable<NV, W, KC, MT - 1>::fill(t);
  }
};
template <int NV, int W, int KC>
struct KTable<NV, W, KC, 0> {
  static void fill(KernelPtr *) {}
};

// Instantiated shapes, keyed by (nv, waves, chunk rows); each table is
// indexed by mt up to the largest that keeps two waves per SIMD.
struct ShapeTable {
  int nv, waves, kc, max_mt;
  KernelPtr t[26];
};

ShapeTable *shape_tables(int &count) {
  static ShapeTable tabs[] = {
      {2, 4, 16, 25, {}}, {4, 4, 16, 12, {}}, {2, 8, 16, 13, {}}, {4, 8, 16, 7, {}}, {2, 8, 32, 13, {}},
  };
  // function-local statics initialise once, also under concurrent first calls
  static const bool init = [] {
    KTable<2, 4, 16, 25>::fill(tabs[0].t);
    KTable<4, 4, 16, 12>::fill(tabs[1].t);
    KTable<2, 8, 16, 13>::fill(tabs[2].t);
    KTable<4, 8, 16, 7>::fill(tabs[3].t);
    KTable<2, 8, 32, 13>::fill(tabs[4].t);
    return true;
  }();
  (void)init;
  count = (int)(sizeof(tabs) / sizeof(tabs[0]));
  return tabs;
}

KernelPtr kernel_for(int nv, int mt, int waves, int kc) {
  int count = 0;
  ShapeTable *tabs = shape_tables(count);
  for (int i = 0; i < count; ++i)
    if (tabs[i].nv == nv && tabs[i].waves == waves && tabs[i].kc == kc && mt >= 1 && mt <= tabs[i].max_mt)
      return tabs[i].t[mt];
  return nullptr;
}

__global__ void sketch_finish_kernel(const float *__restrict__ part, const double *__restrict__ npart, int S,
                                     int64_t ntot, int64_t n1, int k, int kpad, double scale, float *At,
                                     float *Bt, float *na2, float *nb2) {
  const int64_t colx = blockIdx.y;
  const int64_t ncol = ntot;
  for (int64_t colv = colx; colv < ncol; colv += gridDim.y) {
    const bool isb = colv >= n1;
    float *dst = isb ? Bt : At;
    const int64_t cl = isb ? colv - n1 : colv;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < k; c += gridDim.x * blockDim.x) {
      double acc = 0.0;
      for (int s = 0; s < S; ++s) acc += (double)part[((int64_t)s * ntot + colv) * kpad + c];
      if (dst) dst[cl * k + c] = (float)(acc * scale);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      double acc = 0.0;
      for (int s = 0; s < S; ++s) acc += npart[(int64_t)s * ntot + colv];
      float *nd = isb ? nb2 : na2;
      if (nd) nd[cl] = (float)acc;
    }
  }
}

__global__ void pi_fill_kernel(int64_t l0, int64_t nrows, int k, uint64_t seed, double scale, float *out) {
  const int nb4 = (k + 3) / 4;
  const int64_t total = nrows * nb4;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lr = idx / nb4;
    const int cb = (int)(idx - lr * nb4);
    const float4 z = normals4(stream_call(seed, kTagPi, (uint64_t)(l0 + lr), (uint32_t)cb));
    const float zz[4] = {z.x, z.y, z.z, z.w};
    for (int u = 0; u < 4; ++u) {
      const int c = cb * 4 + u;
      if (c < k) out[lr * k + c] = (float)((double)zz[u] * scale);
    }
  }
}

}  // namespace

// Tile shape. A workgroup of `waves` waves covers 16*waves*nv columns (nv
// adjacent columns per lane) and mt m-tiles of 16 sketch rows; all its waves
// share one Pi block. The accumulators take mt*nv*4 VGPRs per lane; two waves
// per SIMD (the occupancy that overlaps one wave's Pi generation with another
// wave's MFMAs) leave room for mt*nv <= 28. Wider column tiles regenerate each
// Pi element for fewer tiles (less VALU) but split k into more chunks, which
// re-read their data tile (from L2). SMP_SKETCH_TILE="nv,mt[,waves[,kc]]"
// overrides the choice (for tuning sweeps); kc is the number of data rows per
// streaming chunk.
static SketchPlan sketch_plan_fp32(int k) {
  SketchPlan p{};
  p.prec = SMP_PREC_FP32;
  p.mt_total = (k + 15) / 16;
  int nv = 2, cap = 13, waves = 8, kc = 32;
  if (const char *e = getenv("SMP_SKETCH_TILE")) {
    int env[4] = {0, 0, 4, 16};
    const int got = sscanf(e, "%d,%d,%d,%d", &env[0], &env[1], &env[2], &env[3]);
    if (got >= 2 && kernel_for(env[0], env[1], env[2], env[3])) {
      nv = env[0];
      cap = env[1];
      waves = env[2];
      kc = env[3];
    }
  }
  p.nv = nv;
  p.waves = waves;
  p.kc = kc;
  p.kt = (p.mt_total + cap - 1) / cap;
  p.mt = (p.mt_total + p.kt - 1) / p.kt;
  p.ncol_tile = 16 * waves * p.nv;
  p.kpad = p.mt_total * 16;
  p.kernel = reinterpret_cast<void *>(kernel_for(nv, p.mt, waves, kc));
  return p;
}

SketchPlan sketch_plan(int k, int prec) {
  return prec == SMP_PREC_BF16 ? sketch_plan_bf16(k) : prec == SMP_PREC_FP8 ? sketch_plan_fp8(k) : sketch_plan_fp32(k);
}

int sketch_slots(const SketchPlan &pl) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    cus = 256;
  if (!pl.kernel || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<KernelPtr>(pl.kernel),
                                                                 64 * pl.waves, 0) != hipSuccess)
    per_cu = 1;
  hipGetLastError();
  return std::max(1, cus) * std::max(1, per_cu);
}

hipError_t sketch_push(const SketchPlan &pl, const float *A, int64_t lda, int64_t n1, const float *B, int64_t ldb,
                       int64_t n2, int64_t row0, int64_t rows, int k, uint64_t seed, int S, bool accumulate,
                       float *part, double *npart, void *pi_buf, hipStream_t st) {
  if (rows < 0) return hipErrorInvalidValue;
  if (pl.srht) return srht_push(pl, A, lda, n1, B, ldb, n2, pl.d, row0, rows, k, seed, S, accumulate, part, npart, st);
  if (pl.frag)
    return fp8_frag_push(pl, A, lda, n1, B, ldb, n2, rows, k, seed, row0, S, accumulate, part, npart, pi_buf, st);
  if (pl.pi_stored && rows > 0 && !pi_buf) return hipErrorInvalidValue;
  SkArgs g{};
  const int nct = pl.ncol_tile;
  // vector loads of e elements per lane need an aligned base, a leading
  // dimension and a column count that are multiples of e
  auto aligned = [](const float *X, int64_t ld, int64_t n, int e) {
    const int vb = 4 * e;
    return ld % e == 0 && n % e == 0 && ((uintptr_t)X % (vb > 16 ? 16 : vb)) == 0;
  };
  auto vec_ok = [&](const float *X, int64_t ld, int64_t n) { return aligned(X, ld, n, pl.nv); };
  g.a = SkMat{A, lda, n1, 0, (int)((n1 + nct - 1) / nct), (int)vec_ok(A, lda, n1)};
  if (B) {
    g.b = SkMat{B, ldb, n2, n1, (int)((n2 + nct - 1) / nct), (int)vec_ok(B, ldb, n2)};
  } else {
    g.b = SkMat{nullptr, 0, 0, n1, 0, 1};
  }
  g.ntot = n1 + n2;
  g.k = k;
  g.kpad = pl.kpad;
  g.kt = pl.kt;
  g.mt_total = pl.mt_total;
  g.accumulate = accumulate ? 1 : 0;
  g.seed = seed;
  g.part = part;
  g.npart = npart;
  // stored Pi: pi_buf holds the Pi fragments of the launch's own rows (one window)
  auto launch = [&](KernelPtr kern, int64_t r0, int64_t nrows, int splits, int64_t rps, int s_base, int extra = 0,
                    int unit = 0) {
    g.row0 = r0;
    g.pi = pl.pi_stored ? pi_buf : nullptr;
    g.rows = nrows;
    g.S = splits;
    g.rows_per_split = rps;
    g.split_extra = extra;
    g.split_unit = unit;
    g.s_base = s_base;
    const int64_t nlog = (int64_t)g.kt * (g.a.ntiles + g.b.ntiles) * splits;
    const int64_t grid = (nlog + 7) / 8 * 8;
    const float *Xa = g.a.X, *Xb = g.b.X;
    g.a.X = Xa + (r0 - row0) * lda;   // the kernels index rows from the launch's first row
    if (Xb) g.b.X = Xb + (r0 - row0) * ldb;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * pl.waves), 0, st, g);
    g.a.X = Xa;
    g.b.X = Xb;
    return hipGetLastError();
  };

  if (pl.prec == SMP_PREC_FP32) {
    if (rows == 0) return hipSuccess;
    KernelPtr kern = reinterpret_cast<KernelPtr>(pl.kernel);
    if (!kern) return hipErrorInvalidValue;
    int64_t rps = (rows + S - 1) / S;
    rps = (rps + pl.kc - 1) / pl.kc * pl.kc;
    return launch(kern, row0, rows, S, rps, 0);
  }

  // BF16 / FP8: main launches over S splits holding every whole block (the
  // first nblk mod S splits one block more than the others), and a tail launch
  // (one split, clamped) for the rows past the last whole block, into partial
  // slot S. The tail launch also runs with no rows, so that a one-shot pass
  // stores zeros in that slot.
  //
  // Stored Pi is drawn one window of at most pi_window_rows(pl) rows at a
  // time, just before the launch that reads it: the whole blocks are cut into
  // nwin windows of equal size (the first nblk mod nwin one block longer),
  // each one Pi draw plus one main launch; the first window's launch stores
  // the partials of a one-shot pass, every later one adds into them.
  // the widest loads the inputs allow: vec_elems (paired 16-byte loads), nv, or scalar
  const bool vec = g.a.vec_ok && g.b.vec_ok;
  const int ve = pl.vec_elems > pl.nv ? pl.vec_elems : pl.nv;
  const bool wide = vec && (ve == pl.nv || (aligned(A, lda, n1, ve) && (!B || aligned(B, ldb, n2, ve))));
  const bool narrow = vec && !wide && pl.kernel_v2 && pl.kernel_v2_clamp;
  KernelPtr kmain = reinterpret_cast<KernelPtr>(wide ? pl.kernel : narrow ? pl.kernel_v2 : pl.kernel_scalar);
  KernelPtr ktail = reinterpret_cast<KernelPtr>(wide ? pl.kernel_clamp : narrow ? pl.kernel_v2_clamp : pl.kernel_scalar);
  if (!kmain || !ktail) return hipErrorInvalidValue;
  const int64_t nblk = rows / pl.kc;
  const int64_t main_rows = nblk * pl.kc;
  const int64_t wblk = pl.pi_stored ? pi_window_rows(pl) / pl.kc : nblk;
  const int64_t nwin = nblk == 0 ? 0 : (nblk + wblk - 1) / wblk;
  hipError_t e = hipSuccess;
  if (nblk == 0 && !accumulate) {   // with no whole block the one-shot pass still stores zero partials
    if ((e = launch(kmain, row0, 0, S, 0, 0, 0, pl.kc)) != hipSuccess) return e;
  }
  for (int64_t w = 0; w < nwin; ++w) {
    const int64_t wb0 = w * (nblk / nwin) + std::min<int64_t>(w, nblk % nwin);
    const int64_t wbn = nblk / nwin + (w < nblk % nwin ? 1 : 0);
    const int64_t r0 = row0 + wb0 * pl.kc;
    if (pl.pi_stored && (e = pi_store(pl, seed, r0, wbn * pl.kc, k, pi_buf, st)) != hipSuccess) return e;
    g.accumulate = (accumulate || w > 0) ? 1 : 0;
    if ((e = launch(kmain, r0, wbn * pl.kc, S, wbn / S * pl.kc, 0, (int)(wbn % S), pl.kc)) != hipSuccess) return e;
  }
  const int64_t tail = rows - main_rows;
  if (tail == 0 && accumulate) return hipSuccess;
  if (pl.pi_stored && tail > 0 && (e = pi_store(pl, seed, row0 + main_rows, tail, k, pi_buf, st)) != hipSuccess)
    return e;
  g.accumulate = accumulate ? 1 : 0;
  return launch(ktail, row0 + main_rows, tail, 1, (tail + pl.kc - 1) / pl.kc * pl.kc, S);
}

hipError_t sketch_finish(const SketchPlan &pl, const float *part, const double *npart, int S, int64_t n1,
                         int64_t n2, int k, float *At, float *Bt, float *na2, float *nb2, hipStream_t st) {
  const int64_t ntot = n1 + n2;
  const int bx = (k + 255) / 256;
  const unsigned gy = (unsigned)std::min<int64_t>(ntot, 65535);
  hipLaunchKernelGGL(sketch_finish_kernel, dim3(bx, gy), dim3(256), 0, st, part, npart, S, ntot, n1, k, pl.kpad,
                     1.0 / std::sqrt((double)k), At, Bt, na2, nb2);
  return hipGetLastError();
}

// Bytes of Pi fragments per data row of a stored-Pi pass (BF16: 32 B per
// m-tile, FP8: 16 B per m-tile).
static int64_t pi_row_bytes(const SketchPlan &pl) { return (int64_t)pl.mt_total * pl.pi_frag_bytes / pl.pi_rows; }

int64_t pi_window_rows(const SketchPlan &pl) {
  if (!pl.pi_stored) return 0;
  if (pl.frag) return fp8_frag_window_rows(pl);
  int64_t cap = kPiWindowBytes;
  if (const char *e = getenv("SMP_PI_WINDOW_MB")) {   // tuning override
    const long v = strtol(e, nullptr, 10);
    if (v >= 1 && v <= 4096) cap = (int64_t)v << 20;
  }
  const int64_t rows = cap / pi_row_bytes(pl) / pl.kc * pl.kc;
  return std::max<int64_t>(rows, pl.kc);
}

size_t sketch_pi_bytes(const SketchPlan &pl, int64_t rows) {
  if (!pl.pi_stored || rows <= 0) return 0;
  if (pl.frag) return fp8_frag_bytes(pl, rows);
  const int64_t wr = std::min<int64_t>((rows + pl.pi_rows - 1) / pl.pi_rows * pl.pi_rows, pi_window_rows(pl));
  return (size_t)(wr / pl.pi_rows) * (size_t)pl.mt_total * (size_t)pl.pi_frag_bytes;
}

hipError_t pi_store(const SketchPlan &pl, uint64_t seed, int64_t r0, int64_t rows, int k, void *buf,
                    hipStream_t st) {
  if (!pl.pi_stored || rows <= 0) return hipSuccess;
  return pl.prec == SMP_PREC_FP8 ? pi_store_fp8(pl, seed, r0, rows, k, buf, st)
                                 : pi_store_bf16(pl, seed, r0, rows, k, buf, st);
}

hipError_t pi_fill(int64_t l0, int64_t nrows, int k, uint64_t seed, float *out, hipStream_t st) {
  const int64_t total = nrows * ((k + 3) / 4);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
  hipLaunchKernelGGL(pi_fill_kernel, dim3(grid), dim3(256), 0, st, l0, nrows, k, seed, 1.0 / std::sqrt((double)k),
                     out);
  return hipGetLastError();
}

}  // namespace smp

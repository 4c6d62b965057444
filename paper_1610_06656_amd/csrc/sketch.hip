// The single pass of SMP-PCA (Alg. 1 step 2; Section 2 "Step 1"):
//   A~ = Pi A, B~ = Pi B (Pi k x d, i.i.d. N(0, 1/k)) and ||A_i||^2, ||B_j||^2,
// as one streaming split-K GEMM on the FP32 matrix cores of gfx950.
//
// Work decomposition. A workgroup (4 waves) owns
//   * a tile of 64*NV data columns of A or B (each lane holds NV adjacent
//     columns of one row, loaded with one vector load),
//   * a chunk of MT*16 sketch rows (all of k when k <= 400 with NV = 2),
//   * one of S contiguous row ranges of the d rows (split-K).
// It streams its rows in chunks of 16. For every chunk the workgroup
// regenerates the MT*16 x 16 block of Pi it needs from the Philox counter
// spec into LDS (Pi is never stored in HBM), and feeds the data rows straight
// from HBM into v_mfma_f32_16x16x4_f32 as the B operand: lane (q, ph) of a
// wave supplies row ph of each 4-row K step for its NV columns, so n-tile v of
// the MFMA sees column (base + q*NV + v). The squared column norms are
// accumulated from the same registers with per-lane compensated (Kahan) FP32
// sums. The S row ranges write FP32 partial sketches and FP64 partial norms;
// sketch_finish reduces them in a fixed order (deterministic, no atomics).
//
// Workgroups that read the same data tile (same column tile and row range,
// different sketch-row chunk) get consecutive logical ids placed on the same
// XCD, so the second read of the tile hits that XCD's L2.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

namespace {


struct SkMat {
  const float *X;
  int64_t ld, n, col_base;
  int ntiles, vec_ok;
};

struct SkArgs {
  SkMat a, b;
  int64_t row0, rows, rows_per_split, ntot;
  int k, kpad, kt, mt_total, S;
  uint64_t seed;
  float *part;
  double *npart;
};

// NV columns of one row into registers. FULL: the whole tile is inside the
// matrix and vector loads are aligned, so the load is unconditional (the row
// index is clamped into the row range and the value zeroed when it is out).
template <int NV, bool FULL>
__device__ __forceinline__ void load_row(const float *X, int64_t ld, int64_t n, int64_t row, int64_t row_last,
                                         int64_t col, bool vec_ok, float (&out)[NV]) {
  const bool row_ok = row <= row_last;
  if constexpr (FULL) {
    const float *p = X + (row_ok ? row : row_last) * ld + col;
    if constexpr (NV == 2) {
      const v2f t = __builtin_nontemporal_load(reinterpret_cast<const v2f *>(p));
      out[0] = t[0]; out[1] = t[1];
    } else {
#pragma unroll
      for (int h = 0; h < NV / 4; ++h) {
        const v4f t = __builtin_nontemporal_load(reinterpret_cast<const v4f *>(p) + h);
        out[4 * h + 0] = t[0]; out[4 * h + 1] = t[1]; out[4 * h + 2] = t[2]; out[4 * h + 3] = t[3];
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = row_ok ? out[v] : 0.0f;
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = 0.0f;
    if (!row_ok || col >= n) return;
    const float *p = X + row * ld + col;
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (col + v < n) out[v] = p[v];
  }
}

// Pi block for sketch rows [c0, c0 + 16 MT) and data rows [lg, lg + KC) into
// LDS as z (unscaled N(0,1)), layout P[row][c]. Every thread makes CPT Philox
// calls (4 sketch rows each); the calls past MT*64 only pad the trip count and
// land in a scratch slot. Rows c >= k are zero.
template <int MT, int W, int KC>
__device__ __forceinline__ void gen_pi(float *P, int tid, uint64_t seed, uint64_t lg, int c0, int k) {
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
    z.x = c + 0 < k ? z.x : 0.f;
    z.y = c + 1 < k ? z.y : 0.f;
    z.z = c + 2 < k ? z.z : 0.f;
    z.w = c + 3 < k ? z.w : 0.f;
    const int slot = (NCALL % kThreads == 0 || idx < NCALL) ? lr * PST + cb * 4 : KC * PST + tid * 4;
    *reinterpret_cast<float4 *>(&P[slot]) = z;
  }
}

template <int MT, int NV, int W, int KC, bool FULL>
__device__ __forceinline__ void sketch_loop(const SkArgs &g, const float *X, int64_t ld, int64_t n, bool vec_ok,
                                            int64_t lbeg, int64_t lend, int64_t col, int c0, float *P0, float *P1,
                                            v4f (&acc)[MT][NV], float (&ksum)[NV], float (&kcmp)[NV]) {
  constexpr int MR = MT * 16, PST = MR + 4;
  constexpr int NST = KC / 4;   // MFMA K steps per chunk
  const int tid = threadIdx.x;
  const int lane = tid & 63, q = lane & 15, ph = lane >> 4;
  const int64_t row_last = lend - 1;

  float xv[NST][NV];
#pragma unroll
  for (int st = 0; st < NST; ++st) load_row<NV, FULL>(X, ld, n, lbeg + 4 * st + ph, row_last, col, vec_ok, xv[st]);
  gen_pi<MT, W, KC>(P0, tid, g.seed, (uint64_t)(g.row0 + lbeg), c0, g.k);

  int buf = 0;
  for (int64_t l = lbeg; l < lend; l += KC) {
    __syncthreads();   // Pi of this chunk is complete; the other buffer is free
    float *Pc = buf ? P1 : P0;
    float *Pn = buf ? P0 : P1;
    // prefetch the next chunk's rows and build its Pi block while this one is multiplied
    float xn[NST][NV];
#pragma unroll
    for (int st = 0; st < NST; ++st)
      load_row<NV, FULL>(X, ld, n, l + KC + 4 * st + ph, row_last, col, vec_ok, xn[st]);
    gen_pi<MT, W, KC>(Pn, tid, g.seed, (uint64_t)(g.row0 + l + KC), c0, g.k);

#pragma unroll
    for (int st = 0; st < NST; ++st)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const float x = xv[st][v];
        const float y = x * x - kcmp[v];
        const float t = ksum[v] + y;
        kcmp[v] = (t - ksum[v]) - y;
        ksum[v] = t;
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

  // ---- XCD-aware decode of the workgroup id (grid size is a multiple of 8)
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int logical = (b & 7) * (nb >> 3) + (b >> 3);
  const int ntl = g.a.ntiles + g.b.ntiles;
  const int nlog = g.kt * ntl * g.S;
  if (logical >= nlog) return;
  const int kc = logical % g.kt;
  const int rest = logical / g.kt;
  int tile = rest % ntl;
  const int s = rest / ntl;
  const bool isb = tile >= g.a.ntiles;
  if (isb) tile -= g.a.ntiles;
  const float *X = isb ? g.b.X : g.a.X;
  const int64_t ld = isb ? g.b.ld : g.a.ld;
  const int64_t n = isb ? g.b.n : g.a.n;
  const int64_t col_base = isb ? g.b.col_base : g.a.col_base;
  const bool vec_ok = isb ? g.b.vec_ok : g.a.vec_ok;

  const int64_t lbeg = (int64_t)s * g.rows_per_split;
  const int64_t lend = min(g.rows, lbeg + g.rows_per_split);
  if (lbeg >= lend) return;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int q = lane & 15, ph = lane >> 4;
  const int64_t tile_col = (int64_t)tile * (16 * W * NV);
  const int64_t col = tile_col + wave * (16 * NV) + q * NV;
  const int mt0 = kc * MT;            // first m-tile of this workgroup
  const int c0 = mt0 * 16;

  v4f acc[MT][NV];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[i][v] = v4f{0.f, 0.f, 0.f, 0.f};
  float ksum[NV], kcmp[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) ksum[v] = kcmp[v] = 0.0f;

  const bool full = vec_ok && tile_col + 16 * W * NV <= n;
  if (full)
    sketch_loop<MT, NV, W, KC, true>(g, X, ld, n, vec_ok, lbeg, lend, col, c0, P, P + PBUF, acc, ksum, kcmp);
  else
    sketch_loop<MT, NV, W, KC, false>(g, X, ld, n, vec_ok, lbeg, lend, col, c0, P, P + PBUF, acc, ksum, kcmp);

  // ---- epilogue: partial sketches (FP32) and partial squared norms (FP64)
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double nrm = (double)ksum[v] - (double)kcmp[v];
    nrm += __shfl_xor(nrm, 16, 64);
    nrm += __shfl_xor(nrm, 32, 64);
    const int64_t c_ = col + v;
    if (c_ < n && ph == 0 && kc == 0) {
      double *dst = g.npart + (int64_t)s * g.ntot + col_base + c_;
      *dst += nrm;
    }
  }
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    if (mt0 + i < g.mt_total) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int64_t c_ = col + v;
        if (c_ < n) {
          float *dst = g.part + ((int64_t)s * g.ntot + col_base + c_) * g.kpad + c0 + 16 * i + 4 * ph;
          float4 old = *reinterpret_cast<float4 *>(dst);
          old.x += acc[i][v][0];
          old.y += acc[i][v][1];
          old.z += acc[i][v][2];
          old.w += acc[i][v][3];
          *reinterpret_cast<float4 *>(dst) = old;
        }
      }
    }
  }
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
  static bool init = false;
  if (!init) {
    KTable<2, 4, 16, 25>::fill(tabs[0].t);
    KTable<4, 4, 16, 12>::fill(tabs[1].t);
    KTable<2, 8, 16, 13>::fill(tabs[2].t);
    KTable<4, 8, 16, 7>::fill(tabs[3].t);
    KTable<2, 8, 32, 13>::fill(tabs[4].t);
    init = true;
  }
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
SketchPlan sketch_plan(int k) {
  SketchPlan p;
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
  return p;
}

hipError_t sketch_push(const SketchPlan &pl, const float *A, int64_t lda, int64_t n1, const float *B, int64_t ldb,
                       int64_t n2, int64_t row0, int64_t rows, int k, uint64_t seed, int S, float *part,
                       double *npart, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  KernelPtr kern = kernel_for(pl.nv, pl.mt, pl.waves, pl.kc);
  if (!kern) return hipErrorInvalidValue;
  SkArgs g{};
  const int nct = pl.ncol_tile;
  const int vb = 4 * pl.nv;   // bytes of one lane's vector load
  g.a = SkMat{A, lda, n1, 0, (int)((n1 + nct - 1) / nct),
              (int)(lda % pl.nv == 0 && ((uintptr_t)A % (vb > 16 ? 16 : vb)) == 0)};
  if (B) {
    g.b = SkMat{B, ldb, n2, n1, (int)((n2 + nct - 1) / nct),
                (int)(ldb % pl.nv == 0 && ((uintptr_t)B % (vb > 16 ? 16 : vb)) == 0)};
  } else {
    g.b = SkMat{nullptr, 0, 0, n1, 0, 0};
  }
  g.row0 = row0;
  g.rows = rows;
  g.S = S;
  int64_t rps = (rows + S - 1) / S;
  rps = (rps + pl.kc - 1) / pl.kc * pl.kc;
  g.rows_per_split = rps;
  g.ntot = n1 + n2;
  g.k = k;
  g.kpad = pl.kpad;
  g.kt = pl.kt;
  g.mt_total = pl.mt_total;
  g.seed = seed;
  g.part = part;
  g.npart = npart;
  const int64_t nlog = (int64_t)g.kt * (g.a.ntiles + g.b.ntiles) * S;
  const int64_t grid = (nlog + 7) / 8 * 8;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64 * pl.waves), 0, st, g);
  return hipGetLastError();
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

hipError_t pi_fill(int64_t l0, int64_t nrows, int k, uint64_t seed, float *out, hipStream_t st) {
  const int64_t total = nrows * ((k + 3) / 4);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
  hipLaunchKernelGGL(pi_fill_kernel, dim3(grid), dim3(256), 0, st, l0, nrows, k, seed, 1.0 / std::sqrt((double)k),
                     out);
  return hipGetLastError();
}

}  // namespace smp

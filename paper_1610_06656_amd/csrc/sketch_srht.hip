// The single pass with the subsampled randomized Hadamard transform as the
// sketching matrix (Section 4, "Spark implementation": the paper's own choice,
// O(n d log d) work, no Gaussian draws):
//   Pi[c, l] = sigma_l (-1)^popcount(rho_c & l) / sqrt(k),
// sigma_l = +-1 (bit 0 of the Philox word of (row 0, column l), tag 7), rho_c
// a row of the D x D Walsh-Hadamard matrix drawn uniformly with replacement
// (the low log2(D) bits of the word of (row 0, column c), tag 8), D the
// smallest power of two >= d. The 1/sqrt(k) is applied by the reduction.
//
// Work decomposition: rows are cut into chunks of C = 512 global rows
// (q = l / C, t = l mod C). With rho = (rho_hi, rho_lo) split the same way,
//   (Pi A)[c, i] sqrt(k) = sum_q (-1)^popcount(rho_hi & q) Y_q[rho_lo, i],
//   Y_q = H_C (sigma .* A[chunk q, i])   (the length-C Walsh-Hadamard transform).
// A workgroup (256 threads) owns 32 columns, a range of chunks (split-K) and a
// block of up to 8 ACC sketch rows. Per chunk:
//  1. thread (column col, group g) loads rows g + 8 m (m < 64) of its column,
//     times sigma (drawn once per chunk into LDS), and runs the six butterfly
//     stages on row bits 3..8 in registers; the squared norms of the unsigned
//     values are summed on the way (FP64);
//  2. the values go through LDS to the layout "rows 64 g + 0..63", where the
//     three stages on row bits 0..2 run in registers;
//  3. Y_q goes back to LDS and thread (col, g) adds +-Y_q[rho_lo(c)] into its
//     ACC accumulators, c = c0 + g + 8 j.
// The partial sums per split go to the same partial slots as the other passes
// (sketch_finish reduces them in a fixed order). Rows outside the launch's
// range read as zero, so pushes may start and end anywhere (the transform is
// linear: partial chunks of two pushes add up to the whole chunk's share).
#include <algorithm>

#include "sketch_common.hpp"
#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {
namespace {

constexpr int kC = 512;       // chunk rows
constexpr int kW = 32;        // columns per workgroup
constexpr int kXS = kW + 1;   // LDS row stride (floats)

struct SrhtArgs {
  SkMat a, b;
  int64_t row0, rows;      // the launch's global rows [row0, row0 + rows)
  int64_t q_first;         // first chunk touched by the launch
  int64_t chunks_per_split;
  int64_t ntot;
  int k, kpad, kt, S, s_base, accumulate, dbits;
  uint64_t seed;
  float *part;
  double *npart;
};

template <int ACC>
__global__ __launch_bounds__(256) void srht_kernel(SrhtArgs g) {
  __shared__ float X[kC * kXS];
  __shared__ float sig[kC];
  __shared__ int rho_lo[8 * ACC];
  __shared__ int rho_hi[8 * ACC];
  __shared__ double nred[256];

  const int ntl = g.a.ntiles + g.b.ntiles;
  const int logical = blockIdx.x;
  const int kc = logical % g.kt;
  const int rest = logical / g.kt;
  int tile = rest % ntl;
  const int s = rest / ntl;
  if (s >= g.S) return;
  const bool isb = tile >= g.a.ntiles;
  if (isb) tile -= g.a.ntiles;
  const SkMat &mat = isb ? g.b : g.a;
  const int tid = threadIdx.x, col_l = tid & 31, grp = tid >> 5;
  const int64_t col = (int64_t)tile * kW + col_l;
  const bool col_ok = col < mat.n;
  const int64_t colc = col_ok ? col : mat.n - 1;
  const int c0 = kc * 8 * ACC;

  // this block's sketch rows: rho split into the chunk bits and the rest
  for (int u = tid; u < 8 * ACC; u += 256) {
    const int c = c0 + u;
    const uint32_t r = c < g.k ? (stream_word(g.seed, kTagSrhtRow, 0ull, (uint64_t)c) & ((g.dbits >= 32 ? 0u : (1u << g.dbits)) - 1u))
                               : 0u;
    rho_lo[u] = (int)(r & (kC - 1));
    rho_hi[u] = (int)(r >> 9);
  }
  float acc[ACC];
#pragma unroll
  for (int j = 0; j < ACC; ++j) acc[j] = 0.0f;
  double nrm = 0.0;

  const int64_t q_end_all = (g.row0 + g.rows + kC - 1) / kC;
  const int64_t qb = g.q_first + (int64_t)s * g.chunks_per_split;
  const int64_t qe = std::min<int64_t>(q_end_all, qb + g.chunks_per_split);
  const int64_t lo = g.row0, hi = g.row0 + g.rows;   // global rows of this launch
  for (int64_t q = qb; q < qe; ++q) {
    const int64_t l0 = q * kC;
    __syncthreads();   // the previous chunk's LDS reads are done
    for (int u = tid; u < kC / 4; u += 256) {
      const u32x4 w = stream_call(g.seed, kTagSrhtSign, 0ull, (uint32_t)((l0 >> 2) + u));
      sig[4 * u + 0] = (w.x & 1u) ? -1.0f : 1.0f;
      sig[4 * u + 1] = (w.y & 1u) ? -1.0f : 1.0f;
      sig[4 * u + 2] = (w.z & 1u) ? -1.0f : 1.0f;
      sig[4 * u + 3] = (w.w & 1u) ? -1.0f : 1.0f;
    }
    __syncthreads();
    // 1. rows grp + 8 m: load, sign, norms, butterflies on row bits 3..8
    float v[64];
#pragma unroll
    for (int m = 0; m < 64; ++m) {
      const int64_t l = l0 + grp + 8 * m;
      const bool ok = l >= lo && l < hi;
      const int64_t lr = ok ? l - g.row0 : 0;   // the launch's matrices start at row0
      const float x = mat.X[lr * mat.ld + colc];
      const float xv = (ok && col_ok) ? x : 0.0f;
      nrm = fma((double)xv, (double)xv, nrm);
      v[m] = xv * sig[grp + 8 * m];
    }
#pragma unroll
    for (int b = 0; b < 6; ++b) {
#pragma unroll
      for (int m = 0; m < 64; ++m) {
        if (!(m & (1 << b))) {
          const float x0 = v[m], x1 = v[m | (1 << b)];
          v[m] = x0 + x1;
          v[m | (1 << b)] = x0 - x1;
        }
      }
    }
    // 2. through LDS to rows 64 grp + 0..63; butterflies on row bits 0..2
#pragma unroll
    for (int m = 0; m < 64; ++m) X[(grp + 8 * m) * kXS + col_l] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 64; ++m) v[m] = X[(64 * grp + m) * kXS + col_l];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
#pragma unroll
      for (int m = 0; m < 64; ++m) {
        if (!(m & (1 << b))) {
          const float x0 = v[m], x1 = v[m | (1 << b)];
          v[m] = x0 + x1;
          v[m | (1 << b)] = x0 - x1;
        }
      }
    }
    __syncthreads();   // every thread has read its rows before Y_q is written
#pragma unroll
    for (int m = 0; m < 64; ++m) X[(64 * grp + m) * kXS + col_l] = v[m];
    __syncthreads();
    // 3. the sampled rows of Y_q, with the sign of the chunk's Hadamard factor
    const int qlow = (int)(q & 0x7fffffff);
#pragma unroll
    for (int j = 0; j < ACC; ++j) {
      const int u = grp + 8 * j;
      const float y = X[rho_lo[u] * kXS + col_l];
      acc[j] += (__builtin_popcount(rho_hi[u] & qlow) & 1) ? -y : y;
    }
  }

  // partial sums of this split: sketch rows c0 + grp + 8 j, norms (from the
  // first sketch-row block only, summed over the 8 row groups)
  const int64_t slot = g.s_base + s;
  if (col_ok) {
    float *dst = g.part + (slot * g.ntot + mat.col_base + col) * g.kpad;
#pragma unroll
    for (int j = 0; j < ACC; ++j) {
      const int c = c0 + grp + 8 * j;
      if (c < g.kpad) dst[c] = g.accumulate ? dst[c] + acc[j] : acc[j];
    }
  }
  nred[tid] = nrm;
  __syncthreads();
  if (grp == 0 && kc == 0 && col_ok) {
    double t = 0.0;
    for (int u = 0; u < 8; ++u) t += nred[col_l + 32 * u];
    double *nd = g.npart + slot * g.ntot + mat.col_base + col;
    *nd = g.accumulate ? *nd + t : t;
  }
}

using KPtr = void (*)(SrhtArgs);

KPtr srht_kernel_for(int acc) {
  switch (acc) {
    case 4: return srht_kernel<4>;
    case 8: return srht_kernel<8>;
    case 16: return srht_kernel<16>;
    case 32: return srht_kernel<32>;
    case 64: return srht_kernel<64>;
    default: return srht_kernel<128>;
  }
}

}  // namespace

// Plan: sketch rows per workgroup 8 ACC (ACC a power of two from 4 to 128,
// the smallest that holds k, else 128 and kt = ceil(k / 1024) blocks).
SketchPlan sketch_plan_srht(int k) {
  SketchPlan p{};
  p.prec = SMP_PREC_FP32;
  p.srht = 1;
  p.mt_total = (k + 15) / 16;
  p.kpad = p.mt_total * 16;
  int acc = 4;
  while (acc < 128 && 8 * acc < k) acc *= 2;
  p.mt = acc;                                  // accumulators per thread
  p.kt = (k + 8 * acc - 1) / (8 * acc);
  p.waves = 4;
  p.kc = kC;
  p.nv = 1;
  p.ncol_tile = kW;
  p.kernel = reinterpret_cast<void *>(srht_kernel_for(acc));
  return p;
}

// Splits: about two workgroups per CU over the column tiles and sketch-row
// blocks, at least one chunk per split.
int srht_splits(const SketchPlan &pl, int64_t d, int64_t n1, int64_t n2) {
  const int64_t tiles = (n1 + kW - 1) / kW + (n2 + kW - 1) / kW;
  const int64_t per = tiles * pl.kt;
  const int64_t chunks = (d + kC - 1) / kC;
  const int64_t want = (512 + per - 1) / per;
  return (int)std::max<int64_t>(1, std::min<int64_t>({want, chunks, 256}));
}

hipError_t srht_push(const SketchPlan &pl, const float *A, int64_t lda, int64_t n1, const float *B, int64_t ldb,
                     int64_t n2, int64_t d, int64_t row0, int64_t rows, int k, uint64_t seed, int S, bool accumulate,
                     float *part, double *npart, hipStream_t st) {
  if (rows <= 0 && accumulate) return hipSuccess;
  SrhtArgs g{};
  g.a = SkMat{A, lda, n1, 0, (int)((n1 + kW - 1) / kW), 1};
  g.b = B ? SkMat{B, ldb, n2, n1, (int)((n2 + kW - 1) / kW), 1} : SkMat{nullptr, 0, 0, n1, 0, 1};
  g.row0 = row0;
  g.rows = rows;
  g.q_first = row0 / kC;
  const int64_t q_last = rows > 0 ? (row0 + rows - 1) / kC : g.q_first - 1;
  const int64_t nq = q_last - g.q_first + 1;
  g.chunks_per_split = std::max<int64_t>(1, (nq + S - 1) / S);
  g.ntot = n1 + n2;
  g.k = k;
  g.kpad = pl.kpad;
  g.kt = pl.kt;
  g.S = S;
  g.s_base = 0;
  g.accumulate = accumulate ? 1 : 0;
  int dbits = 0;
  while ((int64_t(1) << dbits) < d) ++dbits;
  g.dbits = dbits;
  g.seed = seed;
  g.part = part;
  g.npart = npart;
  const int64_t grid = (int64_t)pl.kt * (g.a.ntiles + g.b.ntiles) * S;
  hipLaunchKernelGGL(reinterpret_cast<KPtr>(pl.kernel), dim3((unsigned)grid), dim3(256), 0, st, g);
  return hipGetLastError();
}

}  // namespace smp

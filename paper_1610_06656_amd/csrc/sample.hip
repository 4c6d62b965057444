// Biased entrywise sampling of SMP-PCA (Eq. (1); Alg. 1 step 3; Alg. 2 steps 2-3).
//
//   q_ij = m (||A_i||^2/(2 n2 ||A||_F^2) + ||B_j||^2/(2 n1 ||B||_F^2)),  q^ = min(1, q)
//   (i, j) in Omega independently with probability q^,  w_ij = 1/q^_ij
//
// Every (i, j) gets one 32-bit Philox word (tag 2); the entry is kept iff
// word < floor(q^ 2^32). q^ is evaluated in binary64 one operation at a time
// (no contraction) in a fixed order, so the decision depends only on the FP32
// squared norms: F_A is summed sequentially inside blocks of 256 indices and
// then sequentially over the block sums, den_A = (2 n2) F_A, alpha_i =
// na2_i/den_A, q = m (alpha_i + beta_j).
//
// Omega is produced twice, as a row-major listing (CSR, for the U half-steps)
// and a column-major listing (CSC, for the V half-steps). Each listing is
// built by a count pass, an exclusive scan and a fill pass that re-draws the
// same coins and compacts them in index order with wave ballots, so both
// listings are sorted and identical as sets, with no atomics.
#include <algorithm>

#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {
namespace {

constexpr double kTwo32 = 4294967296.0;

// out[b] = x[256 b] + x[256 b + 1] + ... in index order (binary64, no
// contraction), for x1 (blocks 0 .. nb1-1 of the grid's work) and then x2
// into out2. One workgroup per block of 256 indices: the block is staged in
// LDS with one load per thread, then summed by one thread.
__global__ __launch_bounds__(256) void block_sums_kernel(const float *__restrict__ x1, int64_t n1,
                                                         double *__restrict__ out1, const float *__restrict__ x2,
                                                         int64_t n2, double *__restrict__ out2) {
#pragma clang fp contract(off)
  __shared__ float v[256];
  const int64_t nb1 = (n1 + 255) / 256, nb = nb1 + (n2 + 255) / 256;
  for (int64_t bb = blockIdx.x; bb < nb; bb += gridDim.x) {
    const bool first = bb < nb1;
    const float *x = first ? x1 : x2;
    const int64_t n = first ? n1 : n2, b = first ? bb : bb - nb1;
    const int64_t i = b * 256 + threadIdx.x;
    v[threadIdx.x] = i < n ? x[i] : 0.0f;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int cnt = (int)std::min<int64_t>(256, n - b * 256);
      double s = 0.0;
      for (int u = 0; u < cnt; ++u) s = s + (double)v[u];
      (first ? out1 : out2)[b] = s;
    }
    __syncthreads();
  }
}

inline unsigned block_sums_grid(int64_t n1, int64_t n2) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n1 + 255) / 256 + (n2 + 255) / 256, 65536));
}

__global__ void totals_kernel(const double *__restrict__ ba, int64_t nba, const double *__restrict__ bb,
                              int64_t nbb, int64_t n1, int64_t n2, double *__restrict__ stats) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double fa = 0.0, fb = 0.0;
  for (int64_t b = 0; b < nba; ++b) fa = fa + ba[b];
  for (int64_t b = 0; b < nbb; ++b) fb = fb + bb[b];
  stats[0] = fa;
  stats[1] = fb;
  stats[2] = (2.0 * (double)n2) * fa;
  stats[3] = (2.0 * (double)n1) * fb;
}

// alpha_i = na2_i / den_A, beta_j = nb2_j / den_B. Every workgroup forms
// F_A, F_B and the denominators from the block sums itself, exactly as
// totals_kernel does (sequential over the blocks), and workgroup 0 stores them
// in stats[0..3], with stats[4] = 1 when F_A or F_B is not finite.
__global__ void marginals_kernel(const float *__restrict__ na2, const float *__restrict__ nb2, int64_t n1,
                                 int64_t n2, const double *__restrict__ ba, int64_t nba,
                                 const double *__restrict__ bb, int64_t nbb, double *__restrict__ stats,
                                 double *__restrict__ alpha, double *__restrict__ beta) {
#pragma clang fp contract(off)
  __shared__ double den[2];
  if (threadIdx.x == 0) {
    double fa = 0.0, fb = 0.0;
    for (int64_t b = 0; b < nba; ++b) fa = fa + ba[b];
    for (int64_t b = 0; b < nbb; ++b) fb = fb + bb[b];
    const double da = (2.0 * (double)n2) * fa, db = (2.0 * (double)n1) * fb;
    den[0] = da;
    den[1] = db;
    if (blockIdx.x == 0) {
      stats[0] = fa;
      stats[1] = fb;
      stats[2] = da;
      stats[3] = db;
      // a NaN or infinite entry of A or B (or a squared norm that overflows
      // FP32) leaves a total that is not finite: flag it for the host
      stats[4] = (__builtin_isfinite(fa) && __builtin_isfinite(fb)) ? 0.0 : 1.0;
    }
  }
  __syncthreads();
  const double den_a = den[0], den_b = den[1];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n1 + n2;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n1)
      alpha[i] = den_a > 0.0 ? (double)na2[i] / den_a : 0.0;
    else
      beta[i - n1] = den_b > 0.0 ? (double)nb2[i - n1] / den_b : 0.0;
  }
}

// q^ and the keep decision for one entry.
__device__ __forceinline__ bool coin_keep(double alpha_i, double beta_j, double m, uint32_t x, double &qhat) {
#pragma clang fp contract(off)
  const double q = m * (alpha_i + beta_j);
  qhat = q < 1.0 ? q : 1.0;
  const uint64_t thr = (uint64_t)(qhat * kTwo32);
  return (uint64_t)x < thr;
}

__device__ __forceinline__ uint32_t word_of(const u32x4 &w, int u) {
  return u == 0 ? w.x : (u == 1 ? w.y : (u == 2 ? w.z : w.w));
}

__device__ __forceinline__ uint8_t subset_of(uint32_t y, int T) {
  return (uint8_t)(((uint64_t)y * (uint64_t)(2 * T + 1)) >> 32);
}

// One wave per row i: number of kept entries in the row.
__global__ void count_rows_kernel(const double *__restrict__ alpha, const double *__restrict__ beta, int64_t n1,
                                  int64_t n2, double m, uint64_t seed, int64_t *__restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n1) return;
  const double ai = alpha[i];
  const int64_t nb4 = (n2 + 3) / 4;
  int64_t c = 0;
  for (int64_t jb = lane; jb < nb4; jb += 64) {
    const u32x4 w = stream_call(seed, kTagSample, (uint64_t)i, (uint32_t)jb);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t j = jb * 4 + u;
      double qh;
      if (j < n2 && coin_keep(ai, beta[j], m, word_of(w, u), qh)) ++c;
    }
  }
  c = wave_sum(c);
  if (lane == 0) cnt[i] = c;
}

// One wave per column j.
__global__ void count_cols_kernel(const double *__restrict__ alpha, const double *__restrict__ beta, int64_t n1,
                                  int64_t n2, double m, uint64_t seed, int64_t *__restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t j = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= n2) return;
  const double bj = beta[j];
  int64_t c = 0;
  for (int64_t i = lane; i < n1; i += 64) {
    const u32x4 w = stream_call(seed, kTagSample, (uint64_t)i, (uint32_t)(j >> 2));
    double qh;
    if (coin_keep(alpha[i], bj, m, word_of(w, (int)(j & 3)), qh)) ++c;
  }
  c = wave_sum(c);
  if (lane == 0) cnt[j] = c;
}

// Exclusive scan of cnt[0..n) into ptr[0..n] by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void scan_kernel(const int64_t *__restrict__ cnt, int64_t n,
                                                    int64_t *__restrict__ ptr) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b = t * per, e = std::min<int64_t>(n, b + per);
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  // inclusive scan of the 1024 partial counts (Hillis-Steele)
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t add = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int64_t i = b; i < e; ++i) {
    ptr[i] = run;
    run += cnt[i];
  }
  if (e == n && b < e) ptr[n] = run;
  if (n == 0 && t == 0) ptr[0] = 0;
}

__device__ __forceinline__ int64_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// One wave per row: compacts the kept entries of row i in increasing j.
__global__ void fill_rows_kernel(const double *__restrict__ alpha, const double *__restrict__ beta, int64_t n1,
                                 int64_t n2, double m, uint64_t seed, int T, int split,
                                 const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx,
                                 double *__restrict__ w_out, uint8_t *__restrict__ sub_out) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n1) return;
  const double ai = alpha[i];
  const int64_t nb4 = (n2 + 3) / 4;
  int64_t base = row_ptr[i];
  for (int64_t jb0 = 0; jb0 < nb4; jb0 += 64) {
    const int64_t jb = jb0 + lane;
    bool keep[4] = {false, false, false, false};
    double qh[4] = {1.0, 1.0, 1.0, 1.0};
    u32x4 sw{0, 0, 0, 0};
    if (jb < nb4) {
      const u32x4 w = stream_call(seed, kTagSample, (uint64_t)i, (uint32_t)jb);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t j = jb * 4 + u;
        keep[u] = j < n2 && coin_keep(ai, beta[j], m, word_of(w, u), qh[u]);
      }
      if (split) sw = stream_call(seed, kTagSplit, (uint64_t)i, (uint32_t)jb);
    }
    const int mine = (int)keep[0] + (int)keep[1] + (int)keep[2] + (int)keep[3];
    // inclusive scan of `mine` over the wave (lane order = increasing j)
    int incl = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    int64_t pos = base + incl - mine;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (keep[u]) {
        col_idx[pos] = (int32_t)(jb * 4 + u);
        w_out[pos] = 1.0 / qh[u];
        if (split) sub_out[pos] = subset_of(word_of(sw, u), T);
        ++pos;
      }
    }
    base += total;
  }
}

// One wave per column: compacts the kept entries of column j in increasing i.
__global__ void fill_cols_kernel(const double *__restrict__ alpha, const double *__restrict__ beta, int64_t n1,
                                 int64_t n2, double m, uint64_t seed, int T, int split,
                                 const int64_t *__restrict__ col_ptr, int32_t *__restrict__ row_idx,
                                 double *__restrict__ w_out, uint8_t *__restrict__ sub_out) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const int64_t j = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= n2) return;
  const double bj = beta[j];
  int64_t base = col_ptr[j];
  for (int64_t i0 = 0; i0 < n1; i0 += 64) {
    const int64_t i = i0 + lane;
    bool keep = false;
    double qh = 1.0;
    if (i < n1) {
      const u32x4 w = stream_call(seed, kTagSample, (uint64_t)i, (uint32_t)(j >> 2));
      keep = coin_keep(alpha[i], bj, m, word_of(w, (int)(j & 3)), qh);
    }
    const uint64_t mask = __ballot(keep);
    if (keep) {
      const int64_t pos = base + lanes_below(mask);
      row_idx[pos] = (int32_t)i;
      w_out[pos] = 1.0 / qh;
      if (split) {
        const u32x4 sw = stream_call(seed, kTagSplit, (uint64_t)i, (uint32_t)(j >> 2));
        sub_out[pos] = subset_of(word_of(sw, (int)(j & 3)), T);
      }
    }
    base += __popcll(mask);
  }
}

inline unsigned grid_for(int64_t items, int per_block) {
  return (unsigned)std::max<int64_t>(1, (items + per_block - 1) / per_block);
}

}  // namespace

hipError_t sample_prepare(const float *na2, const float *nb2, int64_t n1, int64_t n2, SampleWs &ws,
                          hipStream_t st) {
  const int64_t nba = (n1 + 255) / 256, nbb = (n2 + 255) / 256;
  hipLaunchKernelGGL(block_sums_kernel, dim3(block_sums_grid(n1, n2)), dim3(256), 0, st, na2, n1, ws.blocks, nb2, n2,
                     ws.blocks + nba);
  hipLaunchKernelGGL(marginals_kernel, dim3(grid_for(n1 + n2, 256)), dim3(256), 0, st, na2, nb2, n1, n2, ws.blocks,
                     nba, ws.blocks + nba, nbb, ws.stats, ws.alpha, ws.beta);
  return hipGetLastError();
}

hipError_t sample_count(const SampleWs &ws, int64_t n1, int64_t n2, double m, uint64_t seed, int64_t *row_ptr,
                        int64_t *col_ptr, int64_t *scan_tmp, hipStream_t st) {
  hipLaunchKernelGGL(count_rows_kernel, dim3(grid_for(n1, 4)), dim3(256), 0, st, ws.alpha, ws.beta, n1, n2, m, seed,
                     scan_tmp);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, scan_tmp, n1, row_ptr);
  hipLaunchKernelGGL(count_cols_kernel, dim3(grid_for(n2, 4)), dim3(256), 0, st, ws.alpha, ws.beta, n1, n2, m, seed,
                     scan_tmp + n1);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, scan_tmp + n1, n2, col_ptr);
  return hipGetLastError();
}

hipError_t sample_fill(const SampleWs &ws, int64_t n1, int64_t n2, double m, uint64_t seed, int T, int split,
                       const smp_omega &om, hipStream_t st) {
  hipLaunchKernelGGL(fill_rows_kernel, dim3(grid_for(n1, 4)), dim3(256), 0, st, ws.alpha, ws.beta, n1, n2, m, seed,
                     T, split, om.row_ptr, om.col_idx, om.w_csr, om.sub_csr);
  hipLaunchKernelGGL(fill_cols_kernel, dim3(grid_for(n2, 4)), dim3(256), 0, st, ws.alpha, ws.beta, n1, n2, m, seed,
                     T, split, om.col_ptr, om.row_idx, om.w_csc, om.sub_csc);
  return hipGetLastError();
}

// Sum of x[0..n) in the fixed order (sequential in blocks of 256, then over
// the block sums) into out[0]; out must hold 4 doubles.
hipError_t fixed_total(const float *x, int64_t n, double *blocks, double *out, hipStream_t st) {
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(block_sums_kernel, dim3(block_sums_grid(n, 0)), dim3(256), 0, st, x, n, blocks,
                     (const float *)nullptr, (int64_t)0, (double *)nullptr);
  hipLaunchKernelGGL(totals_kernel, dim3(1), dim3(64), 0, st, blocks, nb, blocks, (int64_t)0, n, n, out);
  return hipGetLastError();
}

}  // namespace smp

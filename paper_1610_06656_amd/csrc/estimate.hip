// Rescaled-JL estimates on the sampled entries (Eq. (2); Alg. 1 step 4):
//
//   M~(i,j) = ||A_i|| ||B_j|| <A~_i, B~_j> / (||A~_i|| ||B~_j||)
//
// computed only for (i, j) in Omega. A prologue computes, once per column, the
// sketch norm ||A~_i|| and s_i = ||A_i|| = sqrt(na2_i), both FP64. The dot
// product of the FP32 sketch columns is accumulated in FP64 (every FP32 x FP32
// product is exact in FP64), the cosine is clamped to [-1, 1], and
// M~ = s_i s_j cos. A column with a zero norm (data or sketch) gives M~ = 0.
//
// Two ways to evaluate the sampled dot products, both writing bit-identical
// values into the CSR and CSC listings:
//  * dense tiles (Omega covers at least 1/32 of the grid): a workgroup
//    computes a 64 x 64 block of A~^T B~ on the FP64 matrix cores
//    (v_mfma_f64_16x16x4f64, FP32 sketch entries widened exactly) and writes
//    the estimates of the sampled entries of that block, found by binary
//    search in each row's (column's) sorted listing;
//  * gather (sparse grids): one wave per row of the CSR listing (resp. column
//    of the CSC listing), a quarter-wave of 16 lanes per entry, lane u of the
//    quarter summing components u, u+16, ...; the CSR and CSC kernels share
//    the lane split and reduction tree.
#include <algorithm>

#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {
namespace {

// One wave per sketch column: sn = ||S_i|| (FP64), s = sqrt(nrm2) (0 if either is 0).
__global__ void column_scale_kernel(const float *__restrict__ S, const float *__restrict__ nrm2, int64_t n, int k,
                                    double *__restrict__ sn, double *__restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n) return;
  const float *src = S + i * k;
  double ss = 0.0;
  for (int c = lane; c < k; c += 64) ss += (double)src[c] * (double)src[c];
  ss = wave_sum(ss);
  const double nv = (double)nrm2[i];
  const bool ok = ss > 0.0 && nv > 0.0;
  if (lane == 0) {
    sn[i] = ok ? sqrt(ss) : 0.0;
    scale[i] = ok ? sqrt(nv) : 0.0;
  }
}

__device__ __forceinline__ double dot16(const float *__restrict__ a, const float *__restrict__ b, int k, int u) {
  double acc = 0.0;
  for (int c = u; c < k; c += 16) acc = fma((double)a[c], (double)b[c], acc);
  acc += __shfl_xor(acc, 8, 64);
  acc += __shfl_xor(acc, 4, 64);
  acc += __shfl_xor(acc, 2, 64);
  acc += __shfl_xor(acc, 1, 64);
  return acc;
}

__device__ __forceinline__ double rescaled(double si, double sj, double ni, double nj, double dot) {
  const double den = ni * nj;
  if (!(den > 0.0)) return 0.0;
  const double cosv = fmin(1.0, fmax(-1.0, dot / den));
  return (si * sj) * cosv;
}

// Entries of row i: (i, idx[e]) for e in [ptr[i], ptr[i+1]).
__global__ void estimate_rows_kernel(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                     const float *__restrict__ At, const float *__restrict__ Bt,
                                     const double *__restrict__ na, const double *__restrict__ nb,
                                     const double *__restrict__ sa, const double *__restrict__ sb, int64_t n_out,
                                     int k, double *__restrict__ mt) {
  const int lane = threadIdx.x & 63;
  const int quarter = lane >> 4, u = lane & 15;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n_out) return;
  const int64_t e0 = ptr[i], e1 = ptr[i + 1];
  const float *a = At + i * k;
  // each quarter-wave walks its own entries; the shuffles stay inside the quarter
  for (int64_t e = e0 + quarter; e < e1; e += 4) {
    const int64_t j = idx[e];
    const double d = dot16(a, Bt + j * (int64_t)k, k, u);
    if (u == 0) mt[e] = rescaled(sa[i], sb[j], na[i], nb[j], d);
  }
}

// Entries of column j: (idx[e], j) for e in [ptr[j], ptr[j+1]).
__global__ void estimate_cols_kernel(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                     const float *__restrict__ At, const float *__restrict__ Bt,
                                     const double *__restrict__ na, const double *__restrict__ nb,
                                     const double *__restrict__ sa, const double *__restrict__ sb, int64_t n_out,
                                     int k, double *__restrict__ mt) {
  const int lane = threadIdx.x & 63;
  const int quarter = lane >> 4, u = lane & 15;
  const int64_t j = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= n_out) return;
  const int64_t e0 = ptr[j], e1 = ptr[j + 1];
  const float *b = Bt + j * k;
  for (int64_t e = e0 + quarter; e < e1; e += 4) {
    const int64_t i = idx[e];
    const double d = dot16(At + i * (int64_t)k, b, k, u);
    if (u == 0) mt[e] = rescaled(sa[i], sb[j], na[i], nb[j], d);
  }
}

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kTS = 64, kKCH = 32;

__device__ __forceinline__ int64_t lower_bound_idx(const int32_t *__restrict__ a, int64_t lo, int64_t hi, int64_t key) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// One 64 x 64 block of A~^T B~ per workgroup, then the estimates of the
// block's sampled entries.
//  * Products: 32-wide chunks of the sketch rows staged in LDS (FP32), four
//    waves each owning a 32 x 32 quadrant on v_mfma_f64_16x16x4f64; every
//    thread loads its share of chunk c + 1 into registers (clamped,
//    unconditional loads, masked afterwards) while chunk c is multiplied.
//  * The staging tiles and the FP64 dot block share one LDS buffer (33 KB),
//    so four workgroups fit on a CU.
//  * Epilogue: threads 0..63 find the entries of rows i0.. (CSR) and threads
//    64..127 those of columns j0.. (CSC) whose other index falls in the block
//    (binary search in the sorted listings) and cache the rows' and columns'
//    norms in LDS; after a prefix sum over the 64 + 64 counts the block's
//    entries are spread over all 256 threads, four in flight per thread.
__global__ __launch_bounds__(256, 4) void estimate_tiles_kernel(
    const float *__restrict__ At, const float *__restrict__ Bt, int64_t n1, int64_t n2, int k,
    const double *__restrict__ na, const double *__restrict__ nb, const double *__restrict__ sa,
    const double *__restrict__ sb, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const int64_t *__restrict__ cp, const int32_t *__restrict__ ri, double *__restrict__ mt_csr,
    double *__restrict__ mt_csc) {
  constexpr int LD = kKCH + 1;
  __shared__ double smem[kTS * (kTS + 1)];
  __shared__ double r_s[kTS], r_n[kTS], c_s[kTS], c_n[kTS];
  __shared__ int64_t lo_r[kTS], lo_c[kTS];
  __shared__ int pre_r[kTS + 1], pre_c[kTS + 1];
  float *sA = reinterpret_cast<float *>(smem);
  float *sB = sA + kTS * LD;
  double (*dot)[kTS + 1] = reinterpret_cast<double (*)[kTS + 1]>(smem);
  const int64_t i0 = (int64_t)blockIdx.y * kTS, j0 = (int64_t)blockIdx.x * kTS;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wm = wave >> 1, wn = wave & 1;   // 32 x 32 quadrant of the block
  const int m = lane & 15, kk = lane >> 4;
  // this thread's staging elements: rows (t >> 5) + 8 u, sketch row c0 + (t & 31)
  const int cc = t & 31, rr0 = t >> 5;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
  float pa[8], pb[8];
  auto fetch = [&](int c0) {
    const int c = c0 + cc < k ? c0 + cc : k - 1;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = i0 + rr0 + 8 * u, j = j0 + rr0 + 8 * u;
      pa[u] = At[(i < n1 ? i : n1 - 1) * k + c];
      pb[u] = Bt[(j < n2 ? j : n2 - 1) * k + c];
    }
  };
  fetch(0);
  for (int c0 = 0; c0 < k; c0 += kKCH) {
    const bool cok = c0 + cc < k;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int rr = rr0 + 8 * u;
      sA[rr * LD + cc] = (cok && i0 + rr < n1) ? pa[u] : 0.0f;
      sB[rr * LD + cc] = (cok && j0 + rr < n2) ? pb[u] : 0.0f;
    }
    __syncthreads();
    if (c0 + kKCH < k) fetch(c0 + kKCH);
#pragma unroll
    for (int ks = 0; ks < kKCH; ks += 4) {
      const double a0 = sA[(wm * 32 + m) * LD + ks + kk], a1 = sA[(wm * 32 + 16 + m) * LD + ks + kk];
      const double b0 = sB[(wn * 32 + m) * LD + ks + kk], b1 = sB[(wn * 32 + 16 + m) * LD + ks + kk];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  // v_mfma_f64_16x16x4f64 leaves D[4*j + t/16][t%16] in register j of lane t
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) dot[wm * 32 + 16 * a + 4 * jj + kk][wn * 32 + 16 * b + m] = acc[a][b][jj];
  if (t < kTS) {
    const int64_t i = i0 + t;
    int64_t lo = 0, cnt = 0;
    double s_ = 0.0, n_ = 0.0;
    if (i < n1) {
      const int64_t end = rp[i + 1];
      lo = lower_bound_idx(ci, rp[i], end, j0);
      cnt = lower_bound_idx(ci, lo, end, j0 + kTS) - lo;
      s_ = sa[i];
      n_ = na[i];
    }
    lo_r[t] = lo;
    pre_r[t + 1] = (int)cnt;
    r_s[t] = s_;
    r_n[t] = n_;
  } else if (t < 2 * kTS) {
    const int u = t - kTS;
    const int64_t j = j0 + u;
    int64_t lo = 0, cnt = 0;
    double s_ = 0.0, n_ = 0.0;
    if (j < n2) {
      const int64_t end = cp[j + 1];
      lo = lower_bound_idx(ri, cp[j], end, i0);
      cnt = lower_bound_idx(ri, lo, end, i0 + kTS) - lo;
      s_ = sb[j];
      n_ = nb[j];
    }
    lo_c[u] = lo;
    pre_c[u + 1] = (int)cnt;
    c_s[u] = s_;
    c_n[u] = n_;
  }
  __syncthreads();
  if (t == 0) {
    pre_r[0] = 0;
    for (int u = 0; u < kTS; ++u) pre_r[u + 1] += pre_r[u];
  } else if (t == 64) {
    pre_c[0] = 0;
    for (int u = 0; u < kTS; ++u) pre_c[u + 1] += pre_c[u];
  }
  __syncthreads();
  // entry f of the block's listing: owner r = the last with pre[r] <= f
  auto owner = [](const int *pre, int f) {
    int lo = 0, hi = kTS;   // pre[lo] <= f < pre[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pre[mid] <= f) lo = mid;
      else hi = mid;
    }
    return lo;
  };
  const int tot_r = pre_r[kTS], tot_c = pre_c[kTS];
  for (int f0 = 0; f0 < tot_r; f0 += 4 * 256) {
    int64_t e[4];
    int r[4], jj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = min(f0 + q * 256 + t, tot_r - 1);
      r[q] = owner(pre_r, f);
      e[q] = lo_r[r[q]] + (f - pre_r[r[q]]);
      jj[q] = ci[e[q]];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (f0 + q * 256 + t < tot_r) {
        const int cj = (int)(jj[q] - j0);
        mt_csr[e[q]] = rescaled(r_s[r[q]], c_s[cj], r_n[r[q]], c_n[cj], dot[r[q]][cj]);
      }
    }
  }
  for (int f0 = 0; f0 < tot_c; f0 += 4 * 256) {
    int64_t e[4];
    int c[4], ii[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = min(f0 + q * 256 + t, tot_c - 1);
      c[q] = owner(pre_c, f);
      e[q] = lo_c[c[q]] + (f - pre_c[c[q]]);
      ii[q] = ri[e[q]];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (f0 + q * 256 + t < tot_c) {
        const int ri_ = (int)(ii[q] - i0);
        mt_csc[e[q]] = rescaled(r_s[ri_], c_s[c[q]], r_n[ri_], c_n[c[q]], dot[ri_][c[q]]);
      }
    }
  }
}

inline unsigned waves_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 3) / 4); }

}  // namespace

hipError_t estimate_run(const float *At, const float *Bt, const float *na2, const float *nb2, int64_t n1,
                        int64_t n2, int k, double *na, double *nb, double *sa, double *sb, const smp_omega &om,
                        hipStream_t st) {
  hipLaunchKernelGGL(column_scale_kernel, dim3(waves_grid(n1)), dim3(256), 0, st, At, na2, n1, k, na, sa);
  if (nb != na)
    hipLaunchKernelGGL(column_scale_kernel, dim3(waves_grid(n2)), dim3(256), 0, st, Bt, nb2, n2, k, nb, sb);
  const bool dense = (double)om.nnz * 32.0 >= (double)n1 * (double)n2;
  if (om.nnz > 0 && dense) {
    const dim3 grid((unsigned)((n2 + kTS - 1) / kTS), (unsigned)((n1 + kTS - 1) / kTS));
    hipLaunchKernelGGL(estimate_tiles_kernel, grid, dim3(256), 0, st, At, Bt, n1, n2, k, na, nb, sa, sb, om.row_ptr,
                       om.col_idx, om.col_ptr, om.row_idx, om.mt_csr, om.mt_csc);
  } else if (om.nnz > 0) {
    hipLaunchKernelGGL(estimate_rows_kernel, dim3(waves_grid(n1)), dim3(256), 0, st, om.row_ptr, om.col_idx, At, Bt,
                       na, nb, sa, sb, n1, k, om.mt_csr);
    hipLaunchKernelGGL(estimate_cols_kernel, dim3(waves_grid(n2)), dim3(256), 0, st, om.col_ptr, om.row_idx, At, Bt,
                       na, nb, sa, sb, n2, k, om.mt_csc);
  }
  return hipGetLastError();
}

}  // namespace smp

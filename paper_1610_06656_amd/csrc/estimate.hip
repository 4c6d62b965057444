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
// The estimate is a gather-dot over the sampled entries: one wave per row of
// the CSR listing (resp. column of the CSC listing), a quarter-wave of 16
// lanes per entry, lane u of the quarter summing components u, u+16, ... The
// CSR and CSC kernels use the same lane split and reduction tree, so the two
// listings carry bit-identical M~ values.
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

inline unsigned waves_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 3) / 4); }

}  // namespace

hipError_t estimate_run(const float *At, const float *Bt, const float *na2, const float *nb2, int64_t n1,
                        int64_t n2, int k, double *na, double *nb, double *sa, double *sb, const smp_omega &om,
                        hipStream_t st) {
  hipLaunchKernelGGL(column_scale_kernel, dim3(waves_grid(n1)), dim3(256), 0, st, At, na2, n1, k, na, sa);
  if (nb != na)
    hipLaunchKernelGGL(column_scale_kernel, dim3(waves_grid(n2)), dim3(256), 0, st, Bt, nb2, n2, k, nb, sb);
  if (om.nnz > 0) {
    hipLaunchKernelGGL(estimate_rows_kernel, dim3(waves_grid(n1)), dim3(256), 0, st, om.row_ptr, om.col_idx, At, Bt,
                       na, nb, sa, sb, n1, k, om.mt_csr);
    hipLaunchKernelGGL(estimate_cols_kernel, dim3(waves_grid(n2)), dim3(256), 0, st, om.col_ptr, om.row_idx, At, Bt,
                       na, nb, sa, sb, n2, k, om.mt_csc);
  }
  return hipGetLastError();
}

}  // namespace smp

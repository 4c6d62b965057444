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
//  * gather (sparse grids): one wave per row of the CSR listing holds A~_i in
//    registers and forms the dot products of its entries (two B~_j loads in
//    flight, FP64 per-lane sums, a wave reduction); the CSC listing then
//    copies each entry's value from the CSR listing (binary search for j in
//    row i), so the two listings hold the same values.
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

__device__ __forceinline__ double rescaled(double si, double sj, double ni, double nj, double dot) {
  const double den = ni * nj;
  if (!(den > 0.0)) return 0.0;
  const double cosv = fmin(1.0, fmax(-1.0, dot / den));
  return (si * sj) * cosv;
}

// A sketch column of k FP32 values spread over a wave: lane t holds 4 M values,
// component 256 m + 4 t + q (VEC: one 16-byte load per m, k a multiple of 4)
// or 64 (4 m + q) + t (scalar loads); components >= k read as 0.
template <int M, bool VEC>
__device__ __forceinline__ void load_col(const float *__restrict__ src, int k, int lane, float (&v)[4 * M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    if (VEC) {
      const int c = 256 * m + 4 * lane;
      const float4 x = c < k ? *reinterpret_cast<const float4 *>(src + c) : make_float4(0.f, 0.f, 0.f, 0.f);
      v[4 * m + 0] = x.x;
      v[4 * m + 1] = x.y;
      v[4 * m + 2] = x.z;
      v[4 * m + 3] = x.w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 64 * (4 * m + q) + lane;
        v[4 * m + q] = c < k ? src[c] : 0.0f;
      }
    }
  }
}

template <int M>
__device__ __forceinline__ double dot_wave(const float (&a)[4 * M], const float (&b)[4 * M]) {
  double acc = 0.0;
#pragma unroll
  for (int x = 0; x < 4 * M; ++x) acc = fma((double)a[x], (double)b[x], acc);
  return wave_sum(acc);
}

// Gather path, one wave per row i of the CSR listing: A~_i stays in registers,
// the B~_j of two entries are loaded together (one for k > 2048), each dot
// product is a per-lane
// FP64 sum and a wave reduction (a fixed order).
template <int M, bool VEC>
__global__ __launch_bounds__(256) void estimate_rows_kernel(const int64_t *__restrict__ ptr,
                                                            const int32_t *__restrict__ idx,
                                                            const float *__restrict__ At, const float *__restrict__ Bt,
                                                            const double *__restrict__ na,
                                                            const double *__restrict__ nb,
                                                            const double *__restrict__ sa,
                                                            const double *__restrict__ sb, int64_t n1, int k,
                                                            double *__restrict__ mt) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n1) return;
  const int64_t e0 = ptr[i], e1 = ptr[i + 1];
  if (e0 >= e1) return;
  float a[4 * M];
  load_col<M, VEC>(At + i * (int64_t)k, k, lane, a);
  const double si = sa[i], ni = na[i];
  int64_t e = e0;
  for (; M <= 8 && e + 1 < e1; e += 2) {   // k > 2048: one entry at a time (registers)
    const int64_t j0 = idx[e], j1 = idx[e + 1];
    float b0[4 * M], b1[4 * M];
    load_col<M, VEC>(Bt + j0 * (int64_t)k, k, lane, b0);
    load_col<M, VEC>(Bt + j1 * (int64_t)k, k, lane, b1);
    const double d0 = dot_wave<M>(a, b0), d1 = dot_wave<M>(a, b1);
    if (lane == 0) {
      mt[e] = rescaled(si, sb[j0], ni, nb[j0], d0);
      mt[e + 1] = rescaled(si, sb[j1], ni, nb[j1], d1);
    }
  }
  for (; e < e1; ++e) {
    const int64_t j0 = idx[e];
    float b0[4 * M];
    load_col<M, VEC>(Bt + j0 * (int64_t)k, k, lane, b0);
    const double d0 = dot_wave<M>(a, b0);
    if (lane == 0) mt[e] = rescaled(si, sb[j0], ni, nb[j0], d0);
  }
}

// The CSC listing's estimates from the CSR listing: one wave per column j, a
// lane per entry (i, j), whose CSR position is found by binary search for j
// in row i's sorted columns.
__global__ __launch_bounds__(256) void estimate_csc_copy_kernel(const int64_t *__restrict__ cp,
                                                                const int32_t *__restrict__ ri,
                                                                const int64_t *__restrict__ rp,
                                                                const int32_t *__restrict__ ci, int64_t n2,
                                                                const double *__restrict__ mt_csr,
                                                                double *__restrict__ mt_csc) {
  const int lane = threadIdx.x & 63;
  const int64_t j = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= n2) return;
  for (int64_t e = cp[j] + lane; e < cp[j + 1]; e += 64) {
    const int64_t i = ri[e];
    int64_t lo = rp[i], hi = rp[i + 1] - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ci[mid] < j) lo = mid + 1;
      else hi = mid;
    }
    mt_csc[e] = mt_csr[lo];
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
    const int M = k <= 256 ? 1 : k <= 512 ? 2 : k <= 1024 ? 4 : k <= 2048 ? 8 : 16;
    const bool vec = k % 4 == 0;
    const dim3 g(waves_grid(n1)), b(256);
#define SMP_ROWS(MM, VV)                                                                                            \
  hipLaunchKernelGGL((estimate_rows_kernel<MM, VV>), g, b, 0, st, om.row_ptr, om.col_idx, At, Bt, na, nb, sa, sb, \
                     n1, k, om.mt_csr)
    switch (M * 2 + (vec ? 1 : 0)) {
      case 3: SMP_ROWS(1, true); break;
      case 2: SMP_ROWS(1, false); break;
      case 5: SMP_ROWS(2, true); break;
      case 4: SMP_ROWS(2, false); break;
      case 9: SMP_ROWS(4, true); break;
      case 8: SMP_ROWS(4, false); break;
      case 17: SMP_ROWS(8, true); break;
      case 16: SMP_ROWS(8, false); break;
      case 33: SMP_ROWS(16, true); break;
      default: SMP_ROWS(16, false); break;
    }
#undef SMP_ROWS
    hipLaunchKernelGGL(estimate_csc_copy_kernel, dim3(waves_grid(n2)), dim3(256), 0, st, om.col_ptr, om.row_idx,
                       om.row_ptr, om.col_idx, n2, om.mt_csr, om.mt_csc);
  }
  return hipGetLastError();
}

}  // namespace smp

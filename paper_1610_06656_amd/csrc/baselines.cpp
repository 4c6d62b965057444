// The comparison methods of the paper (Section 1 footnote; Section 4):
//
// * SVD(A~^T B~): the top-r SVD of the product of the two sketches of Alg. 1
//   step 2, without the rescaling of Eq. (2) (svd_sketch_run in waltmin.hip).
// * LELA, the two-pass method: pass 1 the column norms, the sample of Eq. (1),
//   pass 2 the exact entries (A^T B)_ij on the sample, then WAltMin (Alg. 2)
//   on those entries. Here pass 2 is a plain library GEMM (rocBLAS SGEMM of
//   A^T B over chunks of 65,536 rows, each chunk's FP32 product added into an
//   FP64 accumulator) followed by a gather into both listings of Omega.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>

#include "smp_internal.hpp"

namespace smp {
namespace {

inline unsigned blocks_for(int64_t items, int per) {
  return (unsigned)std::max<int64_t>(1, (items + per - 1) / per);
}

// part[b][j] = sum over the rows of block b of X[l][j]^2 (FP64); thread per column.
__global__ __launch_bounds__(256) void norms_partial_kernel(const float *__restrict__ X, int64_t ld, int64_t d,
                                                            int64_t n, int64_t rpb, double *__restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const int64_t l0 = (int64_t)blockIdx.y * rpb, l1 = std::min<int64_t>(d, l0 + rpb);
  double s = 0.0;
  for (int64_t l = l0; l < l1; ++l) {
    const double v = (double)X[l * ld + j];
    s = fma(v, v, s);
  }
  part[(int64_t)blockIdx.y * n + j] = s;
}

__global__ void norms_reduce_kernel(const double *__restrict__ part, int nblk, int64_t n, float *__restrict__ out) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * n + j];
    out[j] = (float)s;
  }
}

// acc (FP64) += c (FP32), or acc = c for the first chunk.
__global__ void accumulate_kernel(const float *__restrict__ c, int64_t n, int first, double *__restrict__ acc) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    acc[x] = first ? (double)c[x] : acc[x] + (double)c[x];
}

// mt of every entry of both listings from C = A^T B (column-major n1 x n2).
__global__ void gather_csr_kernel(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
                                  int64_t n1, const double *__restrict__ C, double *__restrict__ mt) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n1) return;
  for (int64_t e = row_ptr[i] + lane; e < row_ptr[i + 1]; e += 64) mt[e] = C[(int64_t)col_idx[e] * n1 + i];
}

__global__ void gather_csc_kernel(const int64_t *__restrict__ col_ptr, const int32_t *__restrict__ row_idx,
                                  int64_t n1, int64_t n2, const double *__restrict__ C, double *__restrict__ mt) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n2) return;
  for (int64_t e = col_ptr[j] + lane; e < col_ptr[j + 1]; e += 64) mt[e] = C[j * n1 + row_idx[e]];
}

constexpr int kNormBlocks = 64;
constexpr int64_t kGemmChunk = 65536;

}  // namespace

size_t norms_ws_bytes(int64_t n1, int64_t n2) {
  return (size_t)kNormBlocks * (size_t)std::max(n1, n2) * 8;
}

hipError_t column_norms(const float *X, int64_t ld, int64_t d, int64_t n, float *out, double *part, hipStream_t st) {
  const int nblk = (int)std::min<int64_t>(kNormBlocks, std::max<int64_t>(1, d / 1024));
  const int64_t rpb = (d + nblk - 1) / nblk;
  hipLaunchKernelGGL(norms_partial_kernel, dim3(blocks_for(n, 256), (unsigned)nblk), dim3(256), 0, st, X, ld, d, n,
                     rpb, part);
  hipLaunchKernelGGL(norms_reduce_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, part, nblk, n, out);
  return hipGetLastError();
}

size_t exact_entries_ws_bytes(int64_t n1, int64_t n2) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  return al((size_t)n1 * n2 * 4) + al((size_t)n1 * n2 * 8);
}

hipError_t exact_entries(void *blas, const float *A, int64_t lda, const float *B, int64_t ldb, int64_t d, int64_t n1,
                         int64_t n2, const smp_omega &om, void *ws, hipStream_t st) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  float *C32 = static_cast<float *>(ws);
  double *C = reinterpret_cast<double *>(static_cast<char *>(ws) + al((size_t)n1 * n2 * 4));
  rocblas_handle h = static_cast<rocblas_handle>(blas);
  if (rocblas_set_stream(h, st) != rocblas_status_success) return hipErrorUnknown;
  const float one = 1.0f, zero = 0.0f;
  const int64_t nn = n1 * n2;
  for (int64_t l0 = 0; l0 < d; l0 += kGemmChunk) {
    const int64_t kc = std::min<int64_t>(kGemmChunk, d - l0);
    // row-major A (d x n1, lda) is column-major n1 x d with leading dimension lda: C = A^T B = Acm Bcm^T
    const rocblas_status s =
        rocblas_sgemm(h, rocblas_operation_none, rocblas_operation_transpose, (rocblas_int)n1, (rocblas_int)n2,
                      (rocblas_int)kc, &one, A + l0 * lda, (rocblas_int)lda, B + l0 * ldb, (rocblas_int)ldb, &zero,
                      C32, (rocblas_int)n1);
    if (s != rocblas_status_success) return hipErrorUnknown;
    hipLaunchKernelGGL(accumulate_kernel, dim3(blocks_for(nn, 256 * 8)), dim3(256), 0, st, C32, nn, l0 == 0 ? 1 : 0,
                       C);
  }
  if (om.nnz > 0) {
    hipLaunchKernelGGL(gather_csr_kernel, dim3(blocks_for(n1, 4)), dim3(256), 0, st, om.row_ptr, om.col_idx, n1, C,
                       om.mt_csr);
    hipLaunchKernelGGL(gather_csc_kernel, dim3(blocks_for(n2, 4)), dim3(256), 0, st, om.col_ptr, om.row_idx, n1, n2,
                       C, om.mt_csc);
  }
  return hipGetLastError();
}

hipError_t blas_create(void **blas) {
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) return hipErrorUnknown;
  *blas = h;
  return hipSuccess;
}

void blas_destroy(void *blas) {
  if (blas) rocblas_destroy_handle(static_cast<rocblas_handle>(blas));
}

}  // namespace smp

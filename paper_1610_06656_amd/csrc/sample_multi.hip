// Row-wise multinomial sampling of Omega (Appendix D, "Sampling"): instead of
// one coin per grid entry (Alg. 1 step 3, O(n1 n2)), row i makes c_i draws
// with replacement from its share of Eq. (1),
//   m_i = sum_j q_ij = m (||A_i||^2 / (2 ||A||_F^2) + 1 / (2 n1)),  q~_ij = q_ij / m_i,
// each located by binary search over the row's CDF, which is a linear function
// of the column index plus a prefix sum shared by every row, so a row costs
// O(m_i log n2) after O(n1 + n2) set-up.
//
// Definitions (the same integers on every side, so Omega is reproducible bit
// for bit):
//   a_i = floor(alpha_i 2^52), b_j = floor(beta_j 2^52) from the binary64
//   marginals of Eq. (1) (sample_prepare); Bcum_j = b_0 + ... + b_j;
//   CDF_i(j) = (j + 1) a_i + Bcum_j;  total_i = CDF_i(n2 - 1) < 2^53;
//   m_i = m (total_i 2^-52); c_i = floor(m_i) + [x_i < floor(frac(m_i) 2^32)],
//   x_i = word 0 of Philox (tag 5, row i, block 0) (randomised rounding);
//   draw k of row i: u = 64-bit uniform from Philox (tag 6, row i, block
//   k/2), words (0,1) for even k and (2,3) for odd k, high word first;
//   t = floor(u total_i / 2^64); column = smallest j with CDF_i(j) > t;
//   an entry drawn N_ij times is kept once with w_ij = N_ij / q_ij,
//   q_ij = m ((a_i + b_j) 2^-52), so that E[w_ij 1{(i,j) in Omega}] = 1.
//
// GPU layout of the work: one thread per draw writes the key (i << bj) | j;
// an LSD radix sort (stable ranks from wave ballots, no atomics on the
// output order) puts the keys in row-major order; one wave per row merges
// equal keys into the CSR listing; a second sort of the entries by
// (j << bi) | i gives the CSC listing, whose weights are copied from the CSR
// entry found by binary search. Every step is deterministic.
#include <algorithm>

#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {
namespace {

constexpr uint32_t kTagRowCount = 5, kTagDraw = 6;

inline unsigned blocks_for(int64_t items, int per) {
  return (unsigned)std::max<int64_t>(1, (items + per - 1) / per);
}

inline int bits_for(int64_t n) {   // bits of n - 1 (0 for n <= 1)
  int b = 0;
  while (b < 63 && (int64_t(1) << b) < n) ++b;
  return b;
}

__device__ __forceinline__ int64_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---- the sampler ------------------------------------------------------------------

__global__ void mn_weights_kernel(const double *__restrict__ alpha, const double *__restrict__ beta, int64_t n1,
                                  int64_t n2, uint64_t *__restrict__ a, int64_t *__restrict__ b) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n1 + n2;
       x += (int64_t)gridDim.x * blockDim.x) {
    // alpha, beta >= 0 and < 1: the products by 2^52 are exact, the conversions floor them
    if (x < n1) {
      const double v = alpha[x] * 0x1p52;
      a[x] = v >= 0.0 && v < 0x1p53 ? (uint64_t)v : 0;
    } else {
      const double v = beta[x - n1] * 0x1p52;
      b[x - n1] = v >= 0.0 && v < 0x1p53 ? (int64_t)v : 0;
    }
  }
}

// c_i (randomised rounding of m_i) and total_i; bptr is the exclusive scan of
// b, so Bcum_{n2-1} = bptr[n2].
__global__ void mn_counts_kernel(const uint64_t *__restrict__ a, const int64_t *__restrict__ bptr, int64_t n1,
                                 int64_t n2, double m, uint64_t seed, uint64_t *__restrict__ tot,
                                 int64_t *__restrict__ cnt) {
#pragma clang fp contract(off)
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n1; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t t = (uint64_t)n2 * a[i] + (uint64_t)bptr[n2];
    double mi = m * ((double)t * 0x1p-52);
    if (!(mi >= 0.0) || !(mi < 0x1p62)) mi = 0.0;   // only reached with non-finite input (reported by the host)
    const double fl = __builtin_floor(mi);
    const uint64_t thr = (uint64_t)((mi - fl) * 4294967296.0);
    const uint32_t x = stream_call(seed, kTagRowCount, (uint64_t)i, 0u).x;
    tot[i] = t;
    cnt[i] = (int64_t)fl + ((uint64_t)x < thr ? 1 : 0);
  }
}

// One thread per draw p < min(doff[n1], dmax): its row i (the last row with
// doff[i] <= p), its 64-bit uniform, its column by binary search.
__global__ void mn_draws_kernel(const uint64_t *__restrict__ a, const int64_t *__restrict__ bptr,
                                const uint64_t *__restrict__ tot, const int64_t *__restrict__ doff, int64_t n1,
                                int64_t n2, int64_t dmax, uint64_t seed, int bj, uint64_t *__restrict__ keys) {
  const int64_t D = std::min<int64_t>(doff[n1], dmax);
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < D; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n1 - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (doff[mid] <= p) lo = mid;
      else hi = mid - 1;
    }
    const int64_t i = lo, k = p - doff[i];
    const u32x4 w = stream_call(seed, kTagDraw, (uint64_t)i, (uint32_t)(k >> 1));
    const uint64_t u = (k & 1) ? (((uint64_t)w.z << 32) | w.w) : (((uint64_t)w.x << 32) | w.y);
    const uint64_t t = __umul64hi(u, tot[i]);
    const uint64_t ai = a[i];
    int64_t jl = 0, jh = n2 - 1;
    while (jl < jh) {
      const int64_t mid = (jl + jh) >> 1;
      const uint64_t cdf = (uint64_t)(mid + 1) * ai + (uint64_t)bptr[mid + 1];
      if (cdf > t) jh = mid;
      else jl = mid + 1;
    }
    keys[p] = ((uint64_t)i << bj) | (uint64_t)jl;
  }
}

// One wave per row: distinct keys in the row's (sorted) draw segment.
__global__ void mn_distinct_count_kernel(const uint64_t *__restrict__ keys, const int64_t *__restrict__ doff,
                                         int64_t n1, int64_t dmax, int64_t *__restrict__ dcnt) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n1) return;
  const int64_t b = std::min<int64_t>(doff[i], dmax), e = std::min<int64_t>(doff[i + 1], dmax);
  int64_t c = 0;
  for (int64_t p0 = b; p0 < e; p0 += 64) {
    const int64_t p = p0 + lane;
    const bool head = p < e && (p == b || keys[p] != keys[p - 1]);
    c += __popcll(__ballot(head));
  }
  if (lane == 0) dcnt[i] = c;
}

__device__ __forceinline__ uint8_t mn_subset(uint64_t seed, int64_t i, int64_t j, int T) {
  const u32x4 w = stream_call(seed, kTagSplit, (uint64_t)i, (uint32_t)(j >> 2));
  const int u = (int)(j & 3);
  const uint32_t y = u == 0 ? w.x : (u == 1 ? w.y : (u == 2 ? w.z : w.w));
  return (uint8_t)(((uint64_t)y * (uint64_t)(2 * T + 1)) >> 32);
}

// One wave per row: the row's distinct entries in increasing j with
// w = N_ij / q_ij (N_ij: the length of the key's run, found by binary search
// for its end).
__global__ void mn_fill_rows_kernel(const uint64_t *__restrict__ keys, const int64_t *__restrict__ doff,
                                    const uint64_t *__restrict__ a, const int64_t *__restrict__ b, int64_t n1,
                                    int64_t dmax, double m, uint64_t seed, int T, int split, uint64_t jmask,
                                    const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx,
                                    double *__restrict__ w_out, uint8_t *__restrict__ sub_out) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n1) return;
  const int64_t s0 = std::min<int64_t>(doff[i], dmax), e = std::min<int64_t>(doff[i + 1], dmax);
  const uint64_t ai = a[i];
  int64_t base = row_ptr[i];
  for (int64_t p0 = s0; p0 < e; p0 += 64) {
    const int64_t p = p0 + lane;
    const uint64_t key = p < e ? keys[p] : 0;
    const bool head = p < e && (p == s0 || key != keys[p - 1]);
    const uint64_t mask = __ballot(head);
    if (head) {
      int64_t lo = p + 1, hi = e;   // first index in (p, e] whose key differs
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] == key) lo = mid + 1;
        else hi = mid;
      }
      const int64_t j = (int64_t)(key & jmask);
      const double q = m * ((double)(ai + (uint64_t)b[j]) * 0x1p-52);
      const int64_t pos = base + lanes_below(mask);
      col_idx[pos] = (int32_t)j;
      w_out[pos] = (double)(lo - p) / q;
      if (split) sub_out[pos] = mn_subset(seed, i, j, T);
    }
    base += __popcll(mask);
  }
}

// CSC keys (j << bi) | i of the CSR entries.
__global__ void mn_csc_keys_kernel(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
                                   int64_t n1, int64_t cap, int bi, uint64_t *__restrict__ ckeys) {
  const int64_t nnz = std::min<int64_t>(row_ptr[n1], cap);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n1 - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (row_ptr[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    ckeys[e] = ((uint64_t)(uint32_t)col_idx[e] << bi) | (uint64_t)lo;
  }
}

// col_ptr[j] = first sorted CSC key with column >= j (binary search); col_ptr[n2] = nnz.
__global__ void mn_col_ptr_kernel(const uint64_t *__restrict__ ckeys, const int64_t *__restrict__ row_ptr, int64_t n1,
                                  int64_t n2, int64_t cap, int bi, int64_t *__restrict__ col_ptr) {
  const int64_t nnz = std::min<int64_t>(row_ptr[n1], cap);
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= n2; j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t target = (uint64_t)j << bi;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ckeys[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    col_ptr[j] = j == n2 ? nnz : lo;
  }
}

// CSC entry e: its row, and the weight (and subset) of the same entry in the
// CSR listing, found by binary search for j in row i.
__global__ void mn_fill_cols_kernel(const uint64_t *__restrict__ ckeys, const int64_t *__restrict__ row_ptr,
                                    const int32_t *__restrict__ col_idx, const double *__restrict__ w_csr,
                                    const uint8_t *__restrict__ sub_csr, int64_t n1, int64_t cap, int bi, int split,
                                    int32_t *__restrict__ row_idx, double *__restrict__ w_csc,
                                    uint8_t *__restrict__ sub_csc) {
  const int64_t nnz = std::min<int64_t>(row_ptr[n1], cap);
  const uint64_t imask = bi >= 64 ? ~0ull : ((1ull << bi) - 1);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = ckeys[e];
    const int64_t i = (int64_t)(key & imask);
    const int32_t j = (int32_t)(key >> bi);
    int64_t lo = row_ptr[i], hi = row_ptr[i + 1] - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (col_idx[mid] < j) lo = mid + 1;
      else hi = mid;
    }
    row_idx[e] = (int32_t)i;
    w_csc[e] = w_csr[lo];
    if (split) sub_csc[e] = sub_csr[lo];
  }
}

}  // namespace

// ---- host side ----------------------------------------------------------------------

int64_t mn_draw_bound(int64_t n1, double m) {
  // sum_i c_i <= sum_i m_i + n1 and sum_i m_i <= m (1 + n 2^-52) (each
  // total_i is a floor of its exact value): a margin of 1e-9 m covers it
  return (int64_t)(m * (1.0 + 1e-9)) + n1 + 16;
}

size_t mn_ws_bytes(int64_t n1, int64_t n2, double m) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  return al(n1 * 8) * 4 + al((n1 + 1) * 8) + al(n2 * 8) + al((n2 + 1) * 8) +
         sort_ws_bytes(mn_draw_bound(n1, m), false, std::max(n1, n2));
}

void mn_ws_carve(void *base, int64_t n1, int64_t n2, double m, MnWs &w) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  char *c = static_cast<char *>(base);
  auto take = [&](size_t bytes) {
    void *p = c;
    c += al(bytes);
    return p;
  };
  w.dmax = mn_draw_bound(n1, m);
  w.a = static_cast<uint64_t *>(take(n1 * 8));
  w.tot = static_cast<uint64_t *>(take(n1 * 8));
  w.cnt = static_cast<int64_t *>(take(n1 * 8));
  w.dcnt = static_cast<int64_t *>(take(n1 * 8));
  w.doff = static_cast<int64_t *>(take((n1 + 1) * 8));
  w.b = static_cast<int64_t *>(take(n2 * 8));
  w.bptr = static_cast<int64_t *>(take((n2 + 1) * 8));
  sort_ws_carve(c, w.dmax, false, std::max(n1, n2), w.srt);
}

hipError_t mn_count(const SampleWs &ws, const MnWs &w, int64_t n1, int64_t n2, double m, uint64_t seed,
                    int64_t *row_ptr, hipStream_t st) {
  hipError_t e;
  hipLaunchKernelGGL(mn_weights_kernel, dim3(blocks_for(n1 + n2, 256)), dim3(256), 0, st, ws.alpha, ws.beta, n1, n2,
                     w.a, w.b);
  if ((e = scan_exclusive(w.srt, w.b, n2, w.bptr, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(mn_counts_kernel, dim3(blocks_for(n1, 256)), dim3(256), 0, st, w.a, w.bptr, n1, n2, m, seed,
                     w.tot, w.cnt);
  if ((e = scan_exclusive(w.srt, w.cnt, n1, w.doff, st)) != hipSuccess) return e;
  const int bi = bits_for(n1), bj = bits_for(n2);
  hipLaunchKernelGGL(mn_draws_kernel, dim3(blocks_for(w.dmax, 256)), dim3(256), 0, st, w.a, w.bptr, w.tot, w.doff, n1,
                     n2, w.dmax, seed, bj, w.srt.keys0);
  if ((e = radix_sort(w.srt, w.doff + n1, bi + bj, st)) != hipSuccess) return e;
  const uint64_t *sorted = radix_result(w.srt, bi + bj);
  hipLaunchKernelGGL(mn_distinct_count_kernel, dim3(blocks_for(n1, 4)), dim3(256), 0, st, sorted, w.doff, n1, w.dmax,
                     w.dcnt);
  return scan_exclusive(w.srt, w.dcnt, n1, row_ptr, st);
}

hipError_t mn_fill(const SampleWs &ws, const MnWs &w, int64_t n1, int64_t n2, double m, uint64_t seed, int T,
                   int split, const smp_omega &om, hipStream_t st) {
  (void)ws;
  const int bi = bits_for(n1), bj = bits_for(n2);
  // the draw keys sorted by mn_count sit where its passes left them
  const uint64_t *sorted = radix_result(w.srt, bi + bj);
  const uint64_t jmask = bj >= 64 ? ~0ull : ((1ull << bj) - 1);
  hipLaunchKernelGGL(mn_fill_rows_kernel, dim3(blocks_for(n1, 4)), dim3(256), 0, st, sorted, w.doff, w.a, w.b, n1,
                     w.dmax, m, seed, T, split, jmask, om.row_ptr, om.col_idx, om.w_csr, om.sub_csr);
  // CSC: sort the entries by (column, row); the draw keys are no longer needed
  hipLaunchKernelGGL(mn_csc_keys_kernel, dim3(blocks_for(om.cap, 256)), dim3(256), 0, st, om.row_ptr, om.col_idx, n1,
                     om.cap, bi, w.srt.keys0);
  const hipError_t e = radix_sort(w.srt, om.row_ptr + n1, bi + bj, st);
  if (e != hipSuccess) return e;
  const uint64_t *cs = radix_result(w.srt, bi + bj);
  hipLaunchKernelGGL(mn_col_ptr_kernel, dim3(blocks_for(n2 + 1, 256)), dim3(256), 0, st, cs, om.row_ptr, n1, n2,
                     om.cap, bi, om.col_ptr);
  hipLaunchKernelGGL(mn_fill_cols_kernel, dim3(blocks_for(om.cap, 256)), dim3(256), 0, st, cs, om.row_ptr, om.col_idx,
                     om.w_csr, om.sub_csr, n1, om.cap, bi, split, om.row_idx, om.w_csc, om.sub_csc);
  return hipGetLastError();
}

}  // namespace smp

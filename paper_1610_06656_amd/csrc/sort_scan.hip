// Exclusive scans of int64 counts and a stable LSD radix sort of uint64 keys
// (8 bits per pass) with an optional uint32 payload. Used by the multinomial
// sampler (draw keys, then the CSC listing) and by the entry-wise sketch
// (entries grouped by column). Everything here is deterministic: the scans
// add integers, and a key's place in each pass comes from the digit counts
// of the tiles before it and from wave ballots inside its tile, never from
// the order in which atomics land.
#include <algorithm>

#include "smp_internal.hpp"

namespace smp {
namespace {

constexpr int kChunk = 4096;   // elements per workgroup of the scans
constexpr int kTile = 1024;    // keys per workgroup of the radix sort (4 rounds of 256)

__device__ __forceinline__ int64_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---- scan_exclusive: chunk sums, a one-workgroup scan of the chunk sums, then
// each chunk's own scan offset by its chunk's sum -------------------------------

__global__ __launch_bounds__(256) void chunk_sums_kernel(const int64_t *__restrict__ in, int64_t n,
                                                         int64_t *__restrict__ sums) {
  __shared__ int64_t red[256];
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  int64_t s = 0;
#pragma unroll
  for (int u = 0; u < kChunk / 256; ++u) {
    const int64_t i = base + u * 256 + threadIdx.x;
    s += i < n ? in[i] : 0;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// Exclusive scan of cnt[0..n) into ptr[0..n] by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void small_scan_kernel(const int64_t *__restrict__ cnt, int64_t n,
                                                          int64_t *__restrict__ ptr) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b = t * per, e = std::min<int64_t>(n, b + per);
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
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
  if (t == 1023) ptr[n] = part[1023];
}

__global__ __launch_bounds__(256) void chunk_scan_kernel(const int64_t *__restrict__ in, int64_t n,
                                                         const int64_t *__restrict__ off, int64_t *__restrict__ out) {
  __shared__ int64_t part[256];
  constexpr int PER = kChunk / 256;
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)t * PER;
  int64_t v[PER];
  int64_t s = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    v[u] = base + u < n ? in[base + u] : 0;
    s += v[u];
  }
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int64_t add = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int64_t run = off[blockIdx.x] + part[t] - s;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (base + u < n) out[base + u] = run;
    run += v[u];
  }
  if (blockIdx.x == gridDim.x - 1 && t == 255) out[n] = off[blockIdx.x] + part[255];
}

// ---- radix sort -----------------------------------------------------------------
// n_dev: the number of keys on the device, clamped to nmax (the buffers'
// size; the grid covers nmax).

__global__ __launch_bounds__(256) void rs_hist_kernel(const uint64_t *__restrict__ keys, const int64_t *__restrict__ n_dev,
                                                      int64_t nmax, int shift, int64_t ntiles,
                                                      int64_t *__restrict__ hist) {
  __shared__ int cnt[256];
  const int64_t n = std::min<int64_t>(*n_dev, nmax);
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int r = 0; r < kTile / 256; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(int)((keys[i] >> shift) & 255u)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];   // digit-major
}

// Each key goes to (offset of its digit in this tile) + (keys of the same
// digit before it in the tile). Items are taken in index order (round r,
// wave w, lane l -> index r*256 + 64 w + l); ranks inside a wave come from
// eight ballots (the lanes whose digit matches bit by bit), per-wave digit
// counts from the group's lowest lane, prefix over (round, wave) per digit.
// PAY: the payload word of each key moves with it.
template <bool PAY>
__global__ __launch_bounds__(256) void rs_scatter_kernel(const uint64_t *__restrict__ in, uint64_t *__restrict__ out,
                                                         const uint32_t *__restrict__ pin, uint32_t *__restrict__ pout,
                                                         const int64_t *__restrict__ n_dev, int64_t nmax, int shift,
                                                         int64_t ntiles, const int64_t *__restrict__ hoff) {
  constexpr int R = kTile / 256;
  __shared__ int cnt[R][4][256];
  const int64_t n = std::min<int64_t>(*n_dev, nmax);
  const int tid = threadIdx.x, wave = tid >> 6;
  int *flat = &cnt[0][0][0];
#pragma unroll
  for (int u = 0; u < R * 4; ++u) flat[u * 256 + tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  uint64_t key[R];
  uint32_t pay[R];
  int dg[R], rank[R];
  bool val[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = base + r * 256 + tid;
    val[r] = i < n;
    key[r] = val[r] ? in[i] : 0;
    pay[r] = PAY && val[r] ? pin[i] : 0u;
    dg[r] = (int)((key[r] >> shift) & 255u);
    uint64_t mask = __ballot(val[r]);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dg[r] >> b) & 1;
      const uint64_t bal = __ballot(bit);
      mask &= bit ? bal : ~bal;
    }
    rank[r] = (int)lanes_below(mask);
    if (val[r] && rank[r] == 0) cnt[r][wave][dg[r]] = __popcll(mask);
  }
  __syncthreads();
  int run = 0;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int c = cnt[r][w][tid];
      cnt[r][w][tid] = run;
      run += c;
    }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (val[r]) {
      const int64_t pos = hoff[(int64_t)dg[r] * ntiles + blockIdx.x] + cnt[r][wave][dg[r]] + rank[r];
      out[pos] = key[r];
      if (PAY) pout[pos] = pay[r];
    }
}

inline size_t al(size_t b) { return (b + 255) / 256 * 256; }
inline int64_t scan_chunks(int64_t n) { return (n + 1 + kChunk - 1) / kChunk; }

}  // namespace

int64_t radix_tiles(int64_t nmax) { return std::max<int64_t>(1, (nmax + kTile - 1) / kTile); }

size_t sort_ws_bytes(int64_t nmax, bool payload, int64_t scan_n) {
  const int64_t hn = 256 * radix_tiles(nmax);
  const int64_t sc = scan_chunks(std::max<int64_t>(hn, scan_n));
  return 2 * al(nmax * 8) + (payload ? 2 * al(nmax * 4) : 0) + al(hn * 8) + al((hn + 1) * 8) + al(sc * 8) +
         al((sc + 1) * 8);
}

void *sort_ws_carve(void *base, int64_t nmax, bool payload, int64_t scan_n, SortWs &w) {
  char *c = static_cast<char *>(base);
  auto take = [&](size_t bytes) {
    void *p = c;
    c += al(bytes);
    return p;
  };
  w.nmax = nmax;
  w.ntiles = radix_tiles(nmax);
  const int64_t hn = 256 * w.ntiles;
  w.scan_n = std::max<int64_t>(hn, scan_n);
  const int64_t sc = scan_chunks(w.scan_n);
  w.keys0 = static_cast<uint64_t *>(take(nmax * 8));
  w.keys1 = static_cast<uint64_t *>(take(nmax * 8));
  w.vals0 = payload ? static_cast<uint32_t *>(take(nmax * 4)) : nullptr;
  w.vals1 = payload ? static_cast<uint32_t *>(take(nmax * 4)) : nullptr;
  w.hist = static_cast<int64_t *>(take(hn * 8));
  w.hoff = static_cast<int64_t *>(take((hn + 1) * 8));
  w.csum = static_cast<int64_t *>(take(sc * 8));
  w.coff = static_cast<int64_t *>(take((sc + 1) * 8));
  return c;
}

hipError_t scan_exclusive(const SortWs &w, const int64_t *in, int64_t n, int64_t *out, hipStream_t st) {
  if (n > w.scan_n) return hipErrorInvalidValue;
  const int64_t nb = std::max<int64_t>(1, (n + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(chunk_sums_kernel, dim3((unsigned)nb), dim3(256), 0, st, in, n, w.csum);
  hipLaunchKernelGGL(small_scan_kernel, dim3(1), dim3(1024), 0, st, w.csum, nb, w.coff);
  hipLaunchKernelGGL(chunk_scan_kernel, dim3((unsigned)nb), dim3(256), 0, st, in, n, w.coff, out);
  return hipGetLastError();
}

hipError_t radix_sort(const SortWs &w, const int64_t *n_dev, int bits, hipStream_t st) {
  uint64_t *src = w.keys0, *dst = w.keys1;
  uint32_t *psrc = w.vals0, *pdst = w.vals1;
  const bool pay = w.vals0 != nullptr;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(rs_hist_kernel, dim3((unsigned)w.ntiles), dim3(256), 0, st, src, n_dev, w.nmax, shift,
                       w.ntiles, w.hist);
    const hipError_t e = scan_exclusive(w, w.hist, 256 * w.ntiles, w.hoff, st);
    if (e != hipSuccess) return e;
    if (pay)
      hipLaunchKernelGGL(rs_scatter_kernel<true>, dim3((unsigned)w.ntiles), dim3(256), 0, st, src, dst, psrc, pdst,
                         n_dev, w.nmax, shift, w.ntiles, w.hoff);
    else
      hipLaunchKernelGGL(rs_scatter_kernel<false>, dim3((unsigned)w.ntiles), dim3(256), 0, st, src, dst, psrc, pdst,
                         n_dev, w.nmax, shift, w.ntiles, w.hoff);
    std::swap(src, dst);
    std::swap(psrc, pdst);
  }
  return hipGetLastError();
}

}  // namespace smp

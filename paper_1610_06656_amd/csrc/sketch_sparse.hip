// The sketch of a matrix given entry by entry, in any order (Section 1: the
// entries of A and B may arrive in an arbitrary order, as in streaming logs;
// Section 3, "Computation Complexity": step 1 costs O(nnz(A) k + nnz(B) k)).
//
// A push hands over triples (l, i, v) (COO, or CSR rows row0 .. row0+nrows-1)
// of one matrix; every (l, i) occurs at most once over the stream. The push
// adds X~[:, i] += v Pi[:, l] and ||X_i||^2 += v^2 into the streaming sketch
// state (partial slot 0, the same buffers the dense pushes add into), so
// dense row blocks and entry pushes mix freely.
//
// Steps of a push:
//  1. key = (i << dbits) | l per entry, payload = its index; indices out of
//     range raise a flag (and become the sentinel column n);
//  2. stable LSD radix sort of the keys: entries grouped by column, rows
//     increasing inside a column, whatever the arrival order;
//  3. column offsets by binary search; a repeated key raises a flag; each
//     column is cut into segments of at most kSeg entries; one readback of
//     the flags and counts (nothing has touched the state yet, so a bad push
//     leaves it as it was);
//  4. one workgroup per segment: staged entries in LDS, each thread owns
//     4 Q sketch rows and adds v Pi[c, l] for every entry (the Gaussian Pi
//     regenerated from the counter: one Philox call per 4 sketch rows and
//     entry; BF16: Z and v rounded to bfloat16, exact products; SRHT:
//     +-v from sigma_l and popcount(rho_c & l)). Columns of one segment add
//     straight into the state; longer columns write per-segment partials;
//  5. one workgroup per (long column, 256 sketch rows) adds its segments'
//     partials in segment order. Every sum has a fixed order: the result does
//     not depend on the arrival order or on the timing of the launch.
#include <algorithm>

#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {
namespace {

constexpr int kSeg = 512;   // entries per segment (one workgroup)

inline int bits_for(int64_t n) {   // bits of n - 1 (0 for n <= 1)
  int b = 0;
  while (b < 63 && (int64_t(1) << b) < n) ++b;
  return b;
}

inline unsigned blocks_for(int64_t items, int per) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + per - 1) / per, 1 << 20));
}

inline size_t al(size_t b) { return (b + 255) / 256 * 256; }

// ---- 1. keys ---------------------------------------------------------------------

__global__ void sp_keys_coo_kernel(const int64_t *__restrict__ rows, const int32_t *__restrict__ cols, int64_t nnz,
                                   int64_t d, int64_t n, int dbits, uint64_t *__restrict__ keys,
                                   uint32_t *__restrict__ pay, SpStatus *__restrict__ st) {
  if (blockIdx.x == 0 && threadIdx.x == 0) st->nnz = nnz;
  bool bad = false;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t l = rows[e];
    int64_t i = cols[e];
    if (l < 0 || l >= d || i < 0 || i >= n) {
      bad = true;
      l = 0;
      i = n;
    }
    keys[e] = ((uint64_t)i << dbits) | (uint64_t)l;
    pay[e] = (uint32_t)e;
  }
  if (bad) st->bad_index = 1;
}

// CSR rows row0 .. row0 + nrows - 1: entry e's row is the last r with
// row_ptr[r] <= e (in [0, nrows) whatever row_ptr holds, so the reads stay in
// bounds); row_ptr must start at 0, end at nnz and not decrease.
__global__ void sp_keys_csr_kernel(const int64_t *__restrict__ row_ptr, int64_t nrows, int64_t row0,
                                   const int32_t *__restrict__ cols, int64_t nnz, int64_t n, int dbits,
                                   uint64_t *__restrict__ keys, uint32_t *__restrict__ pay,
                                   SpStatus *__restrict__ st) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0) {
    st->nnz = nnz;
    if (row_ptr[0] != 0 || row_ptr[nrows] != nnz) st->bad_ptr = 1;
  }
  bool badp = false, bad = false;
  for (int64_t r = tid; r < nrows; r += stride)
    if (row_ptr[r] > row_ptr[r + 1]) badp = true;
  for (int64_t e = tid; e < nnz; e += stride) {
    int64_t lo = 0, hi = nrows - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (row_ptr[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    int64_t l = row0 + lo;
    int64_t i = cols[e];
    if (i < 0 || i >= n) {
      bad = true;
      l = 0;
      i = n;
    }
    keys[e] = ((uint64_t)i << dbits) | (uint64_t)l;
    pay[e] = (uint32_t)e;
  }
  if (badp) st->bad_ptr = 1;
  if (bad) st->bad_index = 1;
}

// ---- 3. column offsets, repeats, segments ------------------------------------------

// col_ptr[c] = first sorted key with column >= c, for c <= n (c = n: the
// sentinel column of bad entries, so col_ptr[n] counts the valid ones).
__global__ void sp_col_ptr_kernel(const uint64_t *__restrict__ keys, const SpStatus *__restrict__ st, int64_t n,
                                  int dbits, int64_t *__restrict__ col_ptr) {
  const int64_t nnz = st->nnz;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c <= n; c += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t target = (uint64_t)c << dbits;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (keys[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    col_ptr[c] = lo;
  }
}

__global__ void sp_repeats_kernel(const uint64_t *__restrict__ keys, SpStatus *__restrict__ st) {
  const int64_t nnz = st->nnz;
  bool dup = false;
  for (int64_t p = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
    if (keys[p] == keys[p - 1]) dup = true;
  if (dup) st->dup = 1;
}

// Per column: segments, segments kept as partials (columns of two or more),
// and whether it is such a long column.
__global__ void sp_seg_count_kernel(const int64_t *__restrict__ col_ptr, int64_t n, int64_t *__restrict__ segc,
                                    int64_t *__restrict__ msc, int64_t *__restrict__ mcc) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t cnt = col_ptr[c + 1] - col_ptr[c];
    const int64_t ns = (cnt + kSeg - 1) / kSeg;
    segc[c] = ns;
    msc[c] = ns >= 2 ? ns : 0;
    mcc[c] = ns >= 2 ? 1 : 0;
  }
}

__global__ void sp_long_list_kernel(const int64_t *__restrict__ mcc, const int64_t *__restrict__ mc_ptr, int64_t n,
                                    int64_t *__restrict__ mlist) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
    if (mcc[c]) mlist[mc_ptr[c]] = c;
}

__global__ void sp_totals_kernel(const int64_t *__restrict__ seg_ptr, const int64_t *__restrict__ ms_ptr,
                                 const int64_t *__restrict__ mc_ptr, int64_t n, SpStatus *__restrict__ st) {
  if (threadIdx.x == 0) {
    st->nseg = seg_ptr[n];
    st->nms = ms_ptr[n];
    st->nlong = mc_ptr[n];
  }
}

// ---- 4. the segment sketch ----------------------------------------------------------

enum { kGauss = 0, kGaussBf16 = 1, kSrht = 2 };

struct SpArgs {
  const uint64_t *keys;
  const uint32_t *pay;
  const float *vals;
  const int64_t *col_ptr, *seg_ptr, *ms_ptr;
  int64_t n;
  int dbits;          // key: (column << dbits) | row
  int k, kpad, K4;    // sketch rows; K4 = ceil(k / 4) Philox calls per entry
  int TG, G;          // threads per entry group, groups per workgroup
  int hbits;          // SRHT: log2 of the Hadamard size
  uint64_t seed;
  float *part;        // slot 0 of this matrix's columns: [n][kpad]
  double *npart;      // [n]
  float *ms;          // per-segment partials of long columns: [nms][kpad]
  double *msn;        // [nms]
};

__device__ __forceinline__ float bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// Workgroup s: segment s. Thread t = TG g + u (g < G) owns the sketch rows
// 4 (u + TG q) + 0..3, q < Q, and takes the segment's entries g, g + G, ...
template <int KIND, int Q>
__global__ __launch_bounds__(256) void sp_sketch_kernel(SpArgs a) {
  __shared__ uint32_t s_lo[256], s_hi[256];
  __shared__ float s_v[256];
  __shared__ float s_red[256 * 4];   // groups 1 .. G-1 (G > 1 only when Q = 1)
  __shared__ double s_n[256];
  const int t = threadIdx.x;
  const int64_t s = blockIdx.x;
  int64_t lo = 0, hi = a.n - 1;   // the last column whose first segment is <= s
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (a.seg_ptr[mid] <= s) lo = mid;
    else hi = mid - 1;
  }
  const int64_t c = lo, j = s - a.seg_ptr[c];
  const int64_t cb = a.col_ptr[c], ce = a.col_ptr[c + 1];
  const int64_t b = cb + j * kSeg, e = std::min<int64_t>(ce, b + kSeg);
  const int g = t / a.TG, u = t - g * a.TG;
  const bool active = g < a.G;

  float acc[4 * Q];
#pragma unroll
  for (int x = 0; x < 4 * Q; ++x) acc[x] = 0.0f;
  uint32_t rho[KIND == kSrht ? 4 * Q : 1];
  if (KIND == kSrht) {
    const uint32_t hmask = a.hbits >= 32 ? 0xffffffffu : ((1u << a.hbits) - 1u);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int cc = 4 * (u + a.TG * q) + r;
        rho[4 * q + r] = cc < a.k ? (stream_word(a.seed, kTagSrhtRow, 0ull, (uint64_t)cc) & hmask) : 0u;
      }
  }
  const uint64_t lmask = a.dbits >= 64 ? ~0ull : ((1ull << a.dbits) - 1);
  double nrm = 0.0;
  for (int64_t p0 = b; p0 < e; p0 += 256) {
    const int nb = (int)std::min<int64_t>(256, e - p0);
    __syncthreads();   // the previous batch is consumed
    if (t < nb) {
      const uint64_t l = a.keys[p0 + t] & lmask;
      float v = a.vals[a.pay[p0 + t]];
      nrm = fma((double)v, (double)v, nrm);
      if (KIND == kSrht && (stream_word(a.seed, kTagSrhtSign, 0ull, l) & 1u)) v = -v;
      if (KIND == kGaussBf16) v = bf16_rne(v);
      s_lo[t] = (uint32_t)l;
      s_hi[t] = (uint32_t)(l >> 32);
      s_v[t] = v;
    }
    __syncthreads();
    if (active)
      for (int x = g; x < nb; x += a.G) {
        const uint64_t l = ((uint64_t)s_hi[x] << 32) | s_lo[x];
        const float v = s_v[x];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int c4 = u + a.TG * q;
          if (c4 < a.K4) {
            if (KIND == kSrht) {
#pragma unroll
              for (int r = 0; r < 4; ++r)
                acc[4 * q + r] += (__popc(rho[4 * q + r] & (uint32_t)l) & 1) ? -v : v;
            } else {
              float4 z = normals4(stream_call(a.seed, kTagPi, l, (uint32_t)c4));
              if (KIND == kGaussBf16) {
                z.x = bf16_rne(z.x);
                z.y = bf16_rne(z.y);
                z.z = bf16_rne(z.z);
                z.w = bf16_rne(z.w);
              }
              acc[4 * q + 0] = fmaf(v, z.x, acc[4 * q + 0]);
              acc[4 * q + 1] = fmaf(v, z.y, acc[4 * q + 1]);
              acc[4 * q + 2] = fmaf(v, z.z, acc[4 * q + 2]);
              acc[4 * q + 3] = fmaf(v, z.w, acc[4 * q + 3]);
            }
          }
        }
      }
  }
  // groups 1 .. G-1 hand their sums to group 0, which adds them in group order
  if (a.G > 1) {
    if (active && g > 0)
#pragma unroll
      for (int x = 0; x < 4; ++x) s_red[((g - 1) * a.TG + u) * 4 + x] = acc[x];
    __syncthreads();
    if (g == 0)
      for (int h = 1; h < a.G; ++h)
#pragma unroll
        for (int x = 0; x < 4; ++x) acc[x] += s_red[((h - 1) * a.TG + u) * 4 + x];
  }
  s_n[t] = nrm;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) s_n[t] += s_n[t + off];
    __syncthreads();
  }
  const bool one = ce - cb <= kSeg;
  const int64_t mi = one ? 0 : a.ms_ptr[c] + j;
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int c4 = u + a.TG * q;
      if (c4 < a.K4) {
        float4 o;
        o.x = 4 * c4 + 0 < a.k ? acc[4 * q + 0] : 0.0f;
        o.y = 4 * c4 + 1 < a.k ? acc[4 * q + 1] : 0.0f;
        o.z = 4 * c4 + 2 < a.k ? acc[4 * q + 2] : 0.0f;
        o.w = 4 * c4 + 3 < a.k ? acc[4 * q + 3] : 0.0f;
        if (one) {
          float4 *dst = reinterpret_cast<float4 *>(a.part + c * (int64_t)a.kpad) + c4;
          const float4 old = *dst;
          *dst = make_float4(old.x + o.x, old.y + o.y, old.z + o.z, old.w + o.w);
        } else {
          reinterpret_cast<float4 *>(a.ms + mi * (int64_t)a.kpad)[c4] = o;
        }
      }
    }
  }
  if (t == 0) {
    if (one) a.npart[c] += s_n[0];
    else a.msn[mi] = s_n[0];
  }
}

// ---- 5. long columns: the segments' partials in segment order ------------------------
__global__ __launch_bounds__(256) void sp_long_reduce_kernel(const int64_t *__restrict__ mlist,
                                                             const int64_t *__restrict__ seg_ptr,
                                                             const int64_t *__restrict__ ms_ptr,
                                                             const float *__restrict__ ms,
                                                             const double *__restrict__ msn, int k, int kpad,
                                                             float *__restrict__ part, double *__restrict__ npart) {
  const int64_t c = mlist[blockIdx.x];
  const int64_t ns = seg_ptr[c + 1] - seg_ptr[c], base = ms_ptr[c];
  const int f = blockIdx.y * 256 + threadIdx.x;
  if (f < k) {
    float sum = 0.0f;
    for (int64_t j = 0; j < ns; ++j) sum += ms[(base + j) * kpad + f];
    part[c * (int64_t)kpad + f] += sum;
  }
  if (blockIdx.y == 0 && threadIdx.x == 0) {
    double sn = 0.0;
    for (int64_t j = 0; j < ns; ++j) sn += msn[base + j];
    npart[c] += sn;
  }
}

struct SpWs {
  SortWs srt;
  int64_t *col_ptr, *segc, *msc, *mcc, *seg_ptr, *ms_ptr, *mc_ptr, *mlist;
  float *ms;
  double *msn;
  SpStatus *st;
};

int64_t long_partials_bound(int64_t nnz) { return 2 * (nnz / kSeg) + 1; }

void sp_carve(void *base, int64_t nnz, int64_t n, int kpad, SpWs &w) {
  char *c = static_cast<char *>(sort_ws_carve(base, std::max<int64_t>(1, nnz), true, n + 1, w.srt));
  auto take = [&](size_t bytes) {
    void *p = c;
    c += al(bytes);
    return p;
  };
  w.col_ptr = static_cast<int64_t *>(take((n + 1) * 8));
  w.segc = static_cast<int64_t *>(take(n * 8));
  w.msc = static_cast<int64_t *>(take(n * 8));
  w.mcc = static_cast<int64_t *>(take(n * 8));
  w.seg_ptr = static_cast<int64_t *>(take((n + 1) * 8));
  w.ms_ptr = static_cast<int64_t *>(take((n + 1) * 8));
  w.mc_ptr = static_cast<int64_t *>(take((n + 1) * 8));
  w.mlist = static_cast<int64_t *>(take(n * 8));
  const int64_t nms = long_partials_bound(nnz);
  w.ms = static_cast<float *>(take((size_t)nms * kpad * 4));
  w.msn = static_cast<double *>(take(nms * 8));
  w.st = static_cast<SpStatus *>(take(sizeof(SpStatus)));
}

template <int KIND>
hipError_t launch_sketch(const SpArgs &a, int Q, int64_t nseg, hipStream_t st) {
  const dim3 grid((unsigned)nseg), block(256);
  switch (Q) {
    case 1: hipLaunchKernelGGL((sp_sketch_kernel<KIND, 1>), grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL((sp_sketch_kernel<KIND, 2>), grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL((sp_sketch_kernel<KIND, 4>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

size_t sparse_ws_bytes(int64_t nnz, int64_t n, int kpad) {
  const int64_t nms = long_partials_bound(nnz);
  return sort_ws_bytes(std::max<int64_t>(1, nnz), true, n + 1) + al((n + 1) * 8) * 4 + al(n * 8) * 4 +
         al((size_t)nms * kpad * 4) + al(nms * 8) + al(sizeof(SpStatus));
}

bool sparse_key_fits(int64_t d, int64_t n) { return bits_for(d) + bits_for(n + 1) <= 64; }

hipError_t sparse_prepare(const SketchPlan &pl, const SparseIn &in, int64_t d, int64_t n, void *ws, SpStatus *result,
                          hipStream_t st) {
  *result = SpStatus{};
  if (in.nnz == 0) return hipSuccess;
  SpWs w;
  sp_carve(ws, in.nnz, n, pl.kpad, w);
  const int dbits = bits_for(d), kbits = dbits + bits_for(n + 1);
  hipError_t e;
  if ((e = hipMemsetAsync(w.st, 0, sizeof(SpStatus), st)) != hipSuccess) return e;
  if (in.row_ptr)
    hipLaunchKernelGGL(sp_keys_csr_kernel, dim3(blocks_for(std::max(in.nnz, in.nrows), 256)), dim3(256), 0, st,
                       in.row_ptr, in.nrows, in.row0, in.cols, in.nnz, n, dbits, w.srt.keys0, w.srt.vals0, w.st);
  else
    hipLaunchKernelGGL(sp_keys_coo_kernel, dim3(blocks_for(in.nnz, 256)), dim3(256), 0, st, in.rows, in.cols, in.nnz,
                       d, n, dbits, w.srt.keys0, w.srt.vals0, w.st);
  if ((e = radix_sort(w.srt, &w.st->nnz, kbits, st)) != hipSuccess) return e;
  const uint64_t *keys = radix_result(w.srt, kbits);
  hipLaunchKernelGGL(sp_col_ptr_kernel, dim3(blocks_for(n + 1, 256)), dim3(256), 0, st, keys, w.st, n, dbits,
                     w.col_ptr);
  hipLaunchKernelGGL(sp_repeats_kernel, dim3(blocks_for(in.nnz, 256)), dim3(256), 0, st, keys, w.st);
  hipLaunchKernelGGL(sp_seg_count_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, w.col_ptr, n, w.segc, w.msc,
                     w.mcc);
  if ((e = scan_exclusive(w.srt, w.segc, n, w.seg_ptr, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(w.srt, w.msc, n, w.ms_ptr, st)) != hipSuccess) return e;
  if ((e = scan_exclusive(w.srt, w.mcc, n, w.mc_ptr, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(sp_long_list_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, w.mcc, w.mc_ptr, n, w.mlist);
  hipLaunchKernelGGL(sp_totals_kernel, dim3(1), dim3(64), 0, st, w.seg_ptr, w.ms_ptr, w.mc_ptr, n, w.st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(result, w.st, sizeof(SpStatus), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
  if (result->nms > long_partials_bound(in.nnz)) return hipErrorInvalidValue;   // cannot happen (bound proved)
  return hipSuccess;
}

hipError_t sparse_accumulate(const SketchPlan &pl, const SparseIn &in, int64_t d, int64_t n, int k, uint64_t seed,
                             float *part, double *npart, void *ws, const SpStatus &prep, hipStream_t st) {
  if (in.nnz == 0 || prep.nseg <= 0 || prep.bad_index || prep.bad_ptr || prep.dup) return hipSuccess;
  SpWs w;
  sp_carve(ws, in.nnz, n, pl.kpad, w);
  const int dbits = bits_for(d), kbits = dbits + bits_for(n + 1);
  const uint64_t *keys = radix_result(w.srt, kbits);
  const uint32_t *pay = radix_payload(w.srt, kbits);
  const SpStatus *result = &prep;
  hipError_t e;
  SpArgs a{};
  a.keys = keys;
  a.pay = pay;
  a.vals = in.vals;
  a.col_ptr = w.col_ptr;
  a.seg_ptr = w.seg_ptr;
  a.ms_ptr = w.ms_ptr;
  a.n = n;
  a.dbits = dbits;
  a.k = k;
  a.kpad = pl.kpad;
  a.K4 = (k + 3) / 4;
  const int Q = a.K4 <= 256 ? 1 : (a.K4 <= 512 ? 2 : 4);
  a.TG = std::min(256, 64 * ((a.K4 + 64 * Q - 1) / (64 * Q)));
  a.G = 256 / a.TG;
  int hb = 0;
  while ((int64_t(1) << hb) < d) ++hb;
  a.hbits = hb;
  a.seed = seed;
  a.part = part;
  a.npart = npart;
  a.ms = w.ms;
  a.msn = w.msn;
  if (pl.srht) e = launch_sketch<kSrht>(a, Q, result->nseg, st);
  else if (pl.prec == SMP_PREC_BF16) e = launch_sketch<kGaussBf16>(a, Q, result->nseg, st);
  else e = launch_sketch<kGauss>(a, Q, result->nseg, st);
  if (e != hipSuccess) return e;
  if (result->nlong > 0)
    hipLaunchKernelGGL(sp_long_reduce_kernel, dim3((unsigned)result->nlong, (unsigned)((k + 255) / 256)), dim3(256),
                       0, st, w.mlist, w.seg_ptr, w.ms_ptr, w.ms, w.msn, k, pl.kpad, part, npart);
  return hipGetLastError();
}

}  // namespace smp

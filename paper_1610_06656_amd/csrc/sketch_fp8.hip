// FP8 variant of the single pass of SMP-PCA (Alg. 1 step 2; Section 2
// "Step 1"): A~ = Pi A, B~ = Pi B with the GEMM operands in FP8 E4M3 (OCP)
// on the block-scaled matrix cores of gfx950 (v_mfma_scale_f32_16x16x128_f8f6f4,
// FP32 accumulation). Pi is rounded to E4M3 as is (|z| < 6 needs no scale);
// every data column is scaled per block of 32 consecutive rows by a power of
// two 2^e (E8M0), the smallest with max|x| <= 448 * 2^e over the block, and
// x 2^-e is rounded to E4M3 (round to nearest even). The block scales are the
// instruction's B-operand scales, so the product needs no extra arithmetic.
// The squared column norms use the unrounded FP32 data (compensated sums), as
// in the FP32 and BF16 passes.
//
// One MFMA consumes 128 data rows (its K). The instruction's operand layout:
// byte e of lane t (t = 16 g + q) holds K index 64 (e / 16) + 16 g + e % 16 of
// row/column q, and the scale in lane t applies to row/column q over the K
// block [32 g, 32 g + 32). Data row j of a 128-row block is K index j, so lane
// (q, g) loads rows 16 g .. 16 g + 15 and 64 + 16 g .. 64 + 16 g + 15 of its
// column; the 32-row scaling block b is spread over lane groups 2 (b % 2) and
// 2 (b % 2) + 1 and its scale must reach group b: the lanes take the maximum
// of their half-block exponents with lane t ^ 16 (the exponent is monotone in
// the magnitude) and groups 1 and 2 then swap one exponent (lane t ^ 48).
// Per workgroup (8 waves) and block of 128 rows:
//  * Pi block: MT*16 sketch rows x 128 rows of E4M3 bytes in LDS, sketch-row
//    major (a lane's 32 bytes are two 16-byte reads); each thread makes MT
//    Philox calls per block (4 sketch rows of one data row each), generated
//    for the next block while this one is multiplied (double buffer);
//  * data: the next block's 32 rows x NV columns per lane are loaded (vector
//    loads from a uniform base plus a 32-bit lane offset) while this block is
//    multiplied, then reduced to their block exponents, scaled and converted.
// As in the BF16 pass, the main launch covers whole 128-row blocks and a
// clamping launch takes the rows left over (rows past the end are excluded
// from the maxima and the norms, and meet zero Pi entries).
#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "sketch_common.hpp"
#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {

typedef int v8i __attribute__((ext_vector_type(8)));

namespace {

constexpr int KP8 = 128;              // data rows per block = K of one MFMA
constexpr int PST8 = KP8 + 16;        // bytes per sketch row in LDS (16-byte pad)

template <int NV>
struct RowT8 {
  typedef float type __attribute__((ext_vector_type(NV)));
};
template <int NV>
using Row8 = typename RowT8<NV>::type;

// Four E4M3 bytes (round to nearest even) from a..d, a in bits 0..7.
__device__ __forceinline__ int cvt4(float a, float b, float c, float d) {
  return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false), true);
}

// Pi block for sketch rows [c0, c0 + 16 MT) x data rows [lg, lg + 128) as E4M3
// bytes, byte (c - c0) * PST8 + row. Thread t makes MT calls: data row
// t % 128, sketch rows 4 ((t / 128) + 4 u) .. +3. Sketch rows c >= k and data
// rows past the first `valid` are zero.
template <int MT>
__device__ __forceinline__ void gen_pi_fp8(uint8_t *P, int tid, uint64_t seed, uint64_t lg, int64_t valid, int c0,
                                           int k, bool edge) {
  const int row = tid % KP8;
  const int cb0 = tid / KP8;
  const bool rv = row < valid;
#pragma unroll
  for (int u = 0; u < MT; ++u) {
    const int cl = 4 * (cb0 + 4 * u);
    const int c = c0 + cl;
    float4 z = normals4(stream_call(seed, kTagPi, lg + (uint64_t)row, (uint32_t)(c >> 2)));
    if (edge) {
      z.x = rv && c + 0 < k ? z.x : 0.f;
      z.y = rv && c + 1 < k ? z.y : 0.f;
      z.z = rv && c + 2 < k ? z.z : 0.f;
      z.w = rv && c + 3 < k ? z.w : 0.f;
    }
    const int w = cvt4(z.x, z.y, z.z, z.w);
    uint8_t *dst = P + cl * PST8 + row;
    dst[0] = (uint8_t)w;
    dst[PST8] = (uint8_t)(w >> 8);
    dst[2 * PST8] = (uint8_t)(w >> 16);
    dst[3 * PST8] = (uint8_t)(w >> 24);
  }
}

// Offset of the lane's e-th row (e < 32) from its first row 16 g.
__device__ __forceinline__ constexpr int row_of(int e) { return e < 16 ? e : e + 48; }

// Rows rel + 16 g + row_of(e) (relative to the split) of the lane's NV columns.
template <int NV, bool VEC, bool CLAMP>
__device__ __forceinline__ void load_block(const SkWork &w, const float *base, uint32_t lane_off, uint32_t ld,
                                           int64_t nrows, int64_t rel, int g, int64_t col, Row8<NV> (&x)[32]) {
  if constexpr (VEC) {
    if (!CLAMP || rel + KP8 <= nrows) {
      const float *bs = base + (size_t)rel * ld;
#pragma unroll
      for (int e = 0; e < 32; ++e)
        x[e] = *reinterpret_cast<const Row8<NV> *>(bs + (size_t)row_of(e) * ld + lane_off);
    } else {
      const int64_t last = nrows - 1;
#pragma unroll
      for (int e = 0; e < 32; ++e) {
        const int64_t r = rel + 16 * g + row_of(e);
        x[e] = *reinterpret_cast<const Row8<NV> *>(base + (r <= last ? r : last) * (int64_t)ld + col);
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < 32; ++e) {
      const int64_t r = w.lbeg + rel + 16 * g + row_of(e);
#pragma unroll
      for (int v = 0; v < NV; ++v) x[e][v] = 0.0f;
      if (r < w.lend && col < w.n) {
        const float *p = w.X + r * w.ld + col;
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (col + v < w.n) x[e][v] = p[v];
      }
    }
  }
}

// Exponent of the E8M0 scale of a (half) block with largest magnitude amax:
// the smallest e with amax <= 448 * 2^e, i.e. with amax = m 2^F (0.5 <= m < 1),
// e = F - 9, plus 1 when m > 0.875 (448 = 0.875 * 2^9); clamped to [-127, 127].
// An all-zero half gives -127 so that the pair maximum is the other half's.
__device__ __forceinline__ int scale_exp(float amax) {
  if (!(amax > 0.0f)) return -127;
  const int ex = __builtin_amdgcn_frexp_expf(amax) - 9 + (__builtin_amdgcn_frexp_mantf(amax) > 0.875f ? 1 : 0);
  return ex < -127 ? -127 : (ex > 127 ? 127 : ex);
}

// Block exponents, E8M0 scale bytes, E4M3 conversion (B operands) and squared
// norms of the 32 rows a lane holds (first row `row`, lane group g). Rows past
// row_last (CLAMP only) count as 0. NV <= 2: the exponents of all NV columns
// travel in one 32-bit word per exchange.
template <int NV, bool NORM, bool CLAMP>
__device__ __forceinline__ void prep_block(const Row8<NV> (&x)[32], int64_t row, int64_t row_last, int g,
                                           v8i (&b)[NV], int (&sb)[NV], float (&ksum)[NV], float (&kcmp)[NV],
                                           bool valid = true) {
  static_assert(NV <= 2, "exponent packing holds two columns");
  uint32_t pk = 0;   // byte 2v + h: biased exponent of half h of column v
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    float a0 = 0.0f, a1 = 0.0f, s2 = 0.0f;
#pragma unroll
    for (int e = 0; e < 32; ++e) {
      const float xv = (!CLAMP || row + row_of(e) <= row_last) ? x[e][v] : 0.0f;
      if (e < 16) a0 = __builtin_fmaxf(a0, __builtin_fabsf(xv));
      else a1 = __builtin_fmaxf(a1, __builtin_fabsf(xv));
      if constexpr (NORM) s2 = __builtin_fmaf(xv, xv, s2);
    }
    if constexpr (NORM) kahan_add(ksum[v], kcmp[v], valid ? s2 : 0.0f);
    pk |= (uint32_t)(scale_exp(a0) + 127) << (16 * v);
    pk |= (uint32_t)(scale_exp(a1) + 127) << (16 * v + 8);
  }
  // whole 32-row blocks: maximum with the partner half in lane t ^ 16
  const uint32_t po = (uint32_t)__shfl_xor((int)pk, 16);
  uint32_t full = 0;
#pragma unroll
  for (int h = 0; h < 2 * NV; ++h) {
    const uint32_t m0 = (pk >> (8 * h)) & 0xffu, m1 = (po >> (8 * h)) & 0xffu;
    full |= (m0 > m1 ? m0 : m1) << (8 * h);
  }
  // lane group g holds the scale of block g: groups 0 and 3 own it (first and
  // second half respectively); group 1 takes the first-half exponent of group
  // 2, group 2 the second-half exponent of group 1
  const uint32_t send = g == 1 ? full >> 8 : full;   // byte 2v: what the partner needs
  const uint32_t got = (uint32_t)__shfl_xor((int)send, 48);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int e0 = (int)((full >> (16 * v)) & 0xffu) - 127;
    const int e1 = (int)((full >> (16 * v + 8)) & 0xffu) - 127;
    const uint32_t mine = g == 0 ? (full >> (16 * v)) : g == 3 ? (full >> (16 * v + 8)) : (got >> (16 * v));
    sb[v] = (int)(mine & 0xffu);
#pragma unroll
    for (int d = 0; d < 8; ++d) {
      const int ex = d < 4 ? e0 : e1;
      float y[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int e = 4 * d + h;
        const float xv = (!CLAMP || row + row_of(e) <= row_last) ? x[e][v] : 0.0f;
        y[h] = __builtin_amdgcn_ldexpf(xv, -ex);
      }
      b[v][d] = cvt4(y[0], y[1], y[2], y[3]);
    }
  }
}

template <int MT, int NV>
__device__ __forceinline__ void mfma_block(const v8i (&b)[NV], const int (&sb)[NV], const uint8_t *Pc, int q, int g,
                                           v4f (&acc)[MT][NV]) {
  v8i a[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const uint8_t *src = Pc + (16 * i + q) * PST8 + 16 * g;
    const int4 lo = *reinterpret_cast<const int4 *>(src);
    const int4 hi = *reinterpret_cast<const int4 *>(src + 64);
    a[i] = v8i{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int v = 0; v < NV; ++v)
      acc[i][v] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[i], b[v], acc[i][v], 0, 0, 0, 127, 0, sb[v]);
}

template <int MT, int NV, bool VEC, bool CLAMP, bool NORM>
__device__ __forceinline__ void loop_fp8(const SkArgs &g, const SkWork &w, int64_t col, int c0, uint8_t *P0,
                                         uint8_t *P1, v4f (&acc)[MT][NV], float (&ksum)[NV], float (&kcmp)[NV]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, q = lane & 15, gq = lane >> 4;
  const int64_t row_last = w.lend - 1;
  const bool kedge = c0 + 16 * MT > g.k;
  const int64_t lcol = VEC ? (col < w.n - NV ? col : w.n - NV) : col;
  const float *base = w.X + w.lbeg * w.ld;
  const uint32_t ld = (uint32_t)w.ld;
  const uint32_t lane_off = (uint32_t)(16 * gq) * ld + (uint32_t)lcol;
  const int64_t nrows = w.lend - w.lbeg;

  Row8<NV> raw[32];
  v8i b[NV];
  int sb[NV];
  load_block<NV, VEC, CLAMP>(w, base, lane_off, ld, nrows, 0, gq, lcol, raw);
  gen_pi_fp8<MT>(P0, tid, g.seed, (uint64_t)(g.row0 + w.lbeg), nrows, c0, g.k, kedge || (CLAMP && nrows < KP8));
  prep_block<NV, NORM, CLAMP>(raw, w.lbeg + 16 * gq, row_last, gq, b, sb, ksum, kcmp);

  int buf = 0;
  for (int64_t l = w.lbeg; l < w.lend; l += KP8) {
    __syncthreads();   // Pi of this block is complete; the other buffer is free
    const uint8_t *Pc = buf ? P1 : P0;
    uint8_t *Pn = buf ? P0 : P1;
    const bool more = l + KP8 < w.lend;
    const bool next = CLAMP || more;   // without CLAMP a load past the split would leave it
    const int64_t rel = l - w.lbeg + KP8;
    if (next) load_block<NV, VEC, CLAMP>(w, base, lane_off, ld, nrows, rel, gq, lcol, raw);
    __builtin_amdgcn_sched_barrier(0);
    if (more)
      gen_pi_fp8<MT>(Pn, tid, g.seed, (uint64_t)(g.row0 + l + KP8), w.lend - (l + KP8), c0, g.k,
                     kedge || (CLAMP && w.lend - (l + KP8) < KP8));
    mfma_block<MT, NV>(b, sb, Pc, q, gq, acc);
    __builtin_amdgcn_sched_barrier(0);
    if (next) prep_block<NV, NORM, CLAMP>(raw, w.lbeg + rel + 16 * gq, row_last, gq, b, sb, ksum, kcmp);
    buf ^= 1;
  }
}

template <int MT, int NV, bool VEC, bool CLAMP>
__global__ __launch_bounds__(512) void sketch_fp8_kernel(SkArgs g) {
  constexpr int W = 8;
  constexpr int PBUF = MT * 16 * PST8;   // bytes of one Pi block
  __shared__ __attribute__((aligned(16))) uint8_t P[2 * PBUF];

  SkWork w;
  if (!sk_decode(g, w)) return;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int q = lane & 15, gq = lane >> 4;
  const int64_t tile_col = (int64_t)w.tile * (16 * W * NV);
  const int64_t col = tile_col + wave * (16 * NV) + q * NV;
  const int c0 = w.kc * MT * 16;

  v4f acc[MT][NV];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[i][v] = v4f{0.f, 0.f, 0.f, 0.f};
  float ksum[NV], kcmp[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) ksum[v] = kcmp[v] = 0.0f;

  if (w.lbeg < w.lend) {   // an empty split still stores its zero partials
    if (w.kc == 0) loop_fp8<MT, NV, VEC, CLAMP, true>(g, w, col, c0, P, P + PBUF, acc, ksum, kcmp);
    else loop_fp8<MT, NV, VEC, CLAMP, false>(g, w, col, c0, P, P + PBUF, acc, ksum, kcmp);
  }
  sk_epilogue<MT, NV>(g, w, col, c0, gq, acc, ksum, kcmp);
}

// ---------------------------------------------------------------------------
// Stored-Pi variant (as for BF16): Pi is drawn once per push, rounded to
// E4M3, into fragments of the A operand of one MFMA: 128-byte unit
// (b * mt_total + i) * 16 + ... holds, for lane t = 16 g + q, the 32 bytes of
// sketch row 16 i + q at the data rows 128 b + 16 g + (0..15) and
// 128 b + 64 + 16 g + (0..15) (b: 128-row block from the push's first row);
// a fragment is 2 KiB. Each workgroup (8 waves) then owns 16*8*NV columns and a
// chunk of up to MT m-tiles; per 128-row step every lane loads its 32 rows x NV
// columns and each wave copies its share of the chunk's fragments, one step
// ahead, into registers; the fragments go to LDS and the rows are
// scaled and converted after the step's MFMAs. The steady-state loop has no
// data-dependent branches (see the BF16 stored-Pi pass).
typedef uint32_t v4u8 __attribute__((ext_vector_type(4)));
constexpr int kPiUnit8 = 128;   // 16-byte units per 2 KiB fragment

__global__ __launch_bounds__(256) void pi_store_fp8_kernel(uint64_t seed, int64_t r0, int64_t nrows, int k,
                                                           int mt_total, int64_t frags, v4u8 *__restrict__ out) {
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (u >= frags * 16) return;
  const int64_t frag = u >> 4;
  const int sub = (int)(u & 15);
  const int g = sub >> 2, q4 = sub & 3;
  const int i = (int)(frag % mt_total);
  const int64_t blk = frag / mt_total;
  const int c = 16 * i + 4 * q4;
  float z[32][4];
#pragma unroll
  for (int e = 0; e < 32; ++e) {
    const int64_t l = 128 * blk + 16 * g + (e < 16 ? e : e + 48);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (l < nrows && c < k) v = normals4(stream_call(seed, kTagPi, (uint64_t)(r0 + l), (uint32_t)(c >> 2)));
    z[e][0] = v.x;
    z[e][1] = c + 1 < k ? v.y : 0.f;
    z[e][2] = c + 2 < k ? v.z : 0.f;
    z[e][3] = c + 3 < k ? v.w : 0.f;
  }
  v4u8 *dst = out + frag * kPiUnit8 + 2 * (16 * g + 4 * q4);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t dw[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) dw[m] = (uint32_t)cvt4(z[4 * m][j], z[4 * m + 1][j], z[4 * m + 2][j], z[4 * m + 3][j]);
    dst[2 * j] = v4u8{dw[0], dw[1], dw[2], dw[3]};
    dst[2 * j + 1] = v4u8{dw[4], dw[5], dw[6], dw[7]};
  }
}

template <int MT, int NV, bool VEC, bool CLAMP, bool NORM, int D>
__device__ __forceinline__ void loop_fp8_stored(const SkArgs &g, const SkWork &w, int64_t col, int i0, int mv,
                                                v4u8 *L, v4f (&acc)[MT][NV], float (&ksum)[NV], float (&kcmp)[NV]) {
  constexpr int W = 8;
  constexpr int CPW = (MT + W - 1) / W;
  constexpr int LT = CPW * W;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int gq = lane >> 4;
  const int64_t row_last = w.lend - 1;
  const int64_t lcol = VEC ? (col < w.n - NV ? col : w.n - NV) : col;
  const float *base = w.X + w.lbeg * w.ld;
  const uint32_t ld = (uint32_t)w.ld;
  const uint32_t lane_off = (uint32_t)(16 * gq) * ld + (uint32_t)lcol;
  const int64_t nrows = w.lend - w.lbeg;
  const v4u8 *pi = reinterpret_cast<const v4u8 *>(g.pi) + (int64_t)i0 * kPiUnit8 + 2 * lane;
  const int64_t fstride = (int64_t)g.mt_total * kPiUnit8;
  const int64_t blk0 = w.lbeg / KP8;
  const int64_t nsteps = (nrows + KP8 - 1) / KP8;

  Row8<NV> raw[D][32];
  v4u8 pst[D][CPW][2];
  v8i b[NV];
  int sb[NV];
  auto issue = [&](int set, int64_t t) {   // t < nsteps; every load is unconditional
    load_block<NV, VEC, CLAMP>(w, base, lane_off, ld, nrows, KP8 * t, gq, lcol, raw[set]);
    const v4u8 *src = pi + (blk0 + t) * fstride;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int i = wave + W * j;
      const v4u8 *f = src + (i < mv ? i : mv - 1) * kPiUnit8;
      pst[set][j][0] = f[0];
      pst[set][j][1] = f[1];
    }
  };
  auto land = [&](int set, int64_t t) {   // Pi of step t into LDS buffer t % 2, its rows from register set `set`
    const bool valid = t < nsteps;
    v4u8 *Ld = L + (t & 1) * (LT * kPiUnit8);
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int i = wave + W * j;
      const bool keep = valid && i < mv;
      Ld[i * kPiUnit8 + 2 * lane] = keep ? pst[set][j][0] : v4u8{0u, 0u, 0u, 0u};
      Ld[i * kPiUnit8 + 2 * lane + 1] = keep ? pst[set][j][1] : v4u8{0u, 0u, 0u, 0u};
    }
    prep_block<NV, NORM, CLAMP>(raw[set], w.lbeg + KP8 * t + 16 * gq, row_last, gq, b, sb, ksum, kcmp, valid);
  };
  // fragments read from LDS two m-tiles at a time, the next pair issued before
  // this pair's MFMAs (all MT at once would hold 8 MT registers)
  auto frag = [&](const v4u8 *Lc, int i) {
    const v4u8 lo = Lc[i * kPiUnit8 + 2 * lane], hi = Lc[i * kPiUnit8 + 2 * lane + 1];
    return v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
  };
  auto multiply = [&](const v4u8 *Lc) {
    constexpr int G = 2, NG = (MT + G - 1) / G;
    v8i a[2][G];
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (j < MT) a[0][j] = frag(Lc, j);
#pragma unroll
    for (int gr = 0; gr < NG; ++gr) {
      if (gr + 1 < NG) {
#pragma unroll
        for (int j = 0; j < G; ++j)
          if ((gr + 1) * G + j < MT) a[(gr + 1) & 1][j] = frag(Lc, (gr + 1) * G + j);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const int i = gr * G + j;
        if (i < MT) {
#pragma unroll
          for (int v = 0; v < NV; ++v)
            acc[i][v] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[gr & 1][j], b[v], acc[i][v], 0, 0, 0, 127,
                                                                         0, sb[v]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };

#pragma unroll
  for (int d = 0; d < D; ++d) issue(d, d < nsteps ? d : nsteps - 1);
  land(0, 0);
  for (int64_t t0 = 0; t0 < nsteps; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int64_t t = t0 + d;
      __syncthreads();   // step t's fragments are in LDS buffer t % 2; buffer (t + 1) % 2 is no longer read
      issue(d, t + D < nsteps ? t + D : nsteps - 1);
      __builtin_amdgcn_sched_barrier(0);
      multiply(L + (t & 1) * (LT * kPiUnit8));
      __builtin_amdgcn_sched_barrier(0);
      land((d + 1) % D, t + 1);
    }
  }
}

template <int MT, int NV, bool VEC, bool CLAMP>
__global__ __launch_bounds__(512) void sketch_fp8_stored_kernel(SkArgs g) {
  constexpr int D = 1;   // one 128-row step of loads in flight
  constexpr int LT = (MT + 7) / 8 * 8;
  __shared__ __attribute__((aligned(16))) v4u8 L[2 * LT * kPiUnit8];

  SkWork w;
  if (!sk_decode(g, w)) return;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int q = lane & 15, gq = lane >> 4;
  const int64_t col = (int64_t)w.tile * (16 * 8 * NV) + wave * (16 * NV) + q * NV;
  const int i0 = w.kc * MT;
  const int mv = g.mt_total - i0 < MT ? g.mt_total - i0 : MT;

  v4f acc[MT][NV];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[i][v] = v4f{0.f, 0.f, 0.f, 0.f};
  float ksum[NV], kcmp[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) ksum[v] = kcmp[v] = 0.0f;

  if (w.lbeg < w.lend) {
    if (w.kc == 0) loop_fp8_stored<MT, NV, VEC, CLAMP, true, D>(g, w, col, i0, mv, L, acc, ksum, kcmp);
    else loop_fp8_stored<MT, NV, VEC, CLAMP, false, D>(g, w, col, i0, mv, L, acc, ksum, kcmp);
  }
  sk_epilogue<MT, NV>(g, w, col, i0 * 16, gq, acc, ksum, kcmp);
}

using KernelPtr = void (*)(SkArgs);

// ---------------------------------------------------------------------------
// Fragment pass (the default for k > 416). The stored-Pi pass above reads the
// FP32 data once per sketch-row chunk (4 bytes per value each time) and
// converts it in every chunk; here each window of rows is first quantised
// once, by a streaming kernel, into the B operands of
// v_mfma_scale_f32_16x16x128_f8f6f4: E4M3 bytes in the operand's lane order,
// 2 KiB per 128-row block and 16-column n-tile, stored as two 1 KiB halves
// (bytes 0-15 of every lane, then bytes 16-31) so that the quantiser writes
// whole lines and the GEMM reads 1 KiB per load instruction; with them the
// E8M0 scales (the same per column and 32-row block as above) and the
// columns' squared norms. The GEMM then reads one byte per value per chunk,
// and its tiles hold 2 n-tiles per wave (256 columns per workgroup) and up to
// 16 m-tiles.

constexpr int kQuantBlocks32 = 4;    // 32-row blocks per quantising thread (one 128-row block)

struct QArgs {
  const float *A, *B;   // the window's first row (B null: A only)
  int64_t lda, ldb, n1, n2;
  int64_t rows;         // rows of the window; rows past them (to the last whole block) quantise as zeros
  int nblk;             // 128-row blocks of the window
  int nt16, ntA16;      // n-tiles in all (A's first, then B's) and A's
  int rq;               // 32-row blocks per thread
  uint8_t *frag;        // [nblk][nt16][2 halves][64 lanes][16 B]
  uint8_t *scale;       // [nblk][nt16][16 columns q][4 32-row blocks g]: the scale of operand lane (q, g)
  double *nscr;         // [gridDim.y][nt16 * 16] squared norms of the thread's rows
};

// Thread: one column (of the n-tile space, A's then B's) and rq consecutive
// 32-row blocks. Block j (rows 32 j .. 32 j + 31) is 32-row block gp = j % 4
// of 128-row block j / 4, i.e. K indices 32 gp + i of the operand: its rows
// i < 16 are bytes 16 (gp / 2) + i of lane (q, 2 (gp % 2)) (half gp / 2 of
// the fragment), rows i >= 16 the same bytes of lane (q, 2 (gp % 2) + 1), and
// its scale is the byte of lane (q, gp), stored at 4 q + gp (a thread covers
// one 128-row block, so it writes its column's four scales as one word).
// Loads are unconditional (clamped row and column, masked after).
__global__ __launch_bounds__(256) void quantize_fp8_kernel(QArgs a) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= (int64_t)a.nt16 * 16) return;
  const int nt = (int)(c >> 4), q = (int)(c & 15);
  const bool isb = nt >= a.ntA16;
  const int64_t mc = isb ? c - (int64_t)a.ntA16 * 16 : c;
  const int64_t nm = isb ? a.n2 : a.n1;
  const bool cv = mc < nm;
  const float *X = isb ? a.B : a.A;
  const int64_t ld = isb ? a.ldb : a.lda;
  const float *xc = X + (cv ? mc : nm - 1);
  const int64_t last = a.rows - 1;
  const int j0 = (int)blockIdx.y * a.rq;
  const int j1 = j0 + a.rq < 4 * a.nblk ? j0 + a.rq : 4 * a.nblk;
  static_assert(kQuantBlocks32 == 4, "a thread covers one 128-row block");
  double s2 = 0.0;
  uint32_t sc4 = 0;   // byte gp: the scale of 32-row block gp
  // block j + 1's rows are requested before block j is converted
  float xn[32];
  auto load = [&](int j, float (&x)[32]) {
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const int64_t r = (int64_t)j * 32 + i;
      x[i] = xc[(r <= last ? r : last) * ld];
    }
  };
  if (j0 < j1) load(j0, xn);
  for (int j = j0; j < j1; ++j) {
    float x[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) x[i] = xn[i];
    load(j + 1 < j1 ? j + 1 : j, xn);
    float amax = 0.0f;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const bool ok = cv && (int64_t)j * 32 + i <= last;
      x[i] = ok ? x[i] : 0.0f;
      amax = __builtin_fmaxf(amax, __builtin_fabsf(x[i]));
      s2 = __builtin_fma((double)x[i], (double)x[i], s2);
    }
    const int ex = scale_exp(amax);
    uint32_t wv[8];
#pragma unroll
    for (int h = 0; h < 8; ++h)
      wv[h] = (uint32_t)cvt4(__builtin_amdgcn_ldexpf(x[4 * h], -ex), __builtin_amdgcn_ldexpf(x[4 * h + 1], -ex),
                             __builtin_amdgcn_ldexpf(x[4 * h + 2], -ex), __builtin_amdgcn_ldexpf(x[4 * h + 3], -ex));
    const int blk = j >> 2, gp = j & 3;
    const int64_t fb = (int64_t)blk * a.nt16 + nt;
    uint8_t *f = a.frag + fb * 2048 + 1024 * (gp >> 1);
    const int g0 = 2 * (gp & 1);
    *reinterpret_cast<v4u8 *>(f + (16 * g0 + q) * 16) = v4u8{wv[0], wv[1], wv[2], wv[3]};
    *reinterpret_cast<v4u8 *>(f + (16 * (g0 + 1) + q) * 16) = v4u8{wv[4], wv[5], wv[6], wv[7]};
    sc4 |= (uint32_t)(ex + 127) << (8 * gp);
  }
  if (j0 < j1)
    *reinterpret_cast<uint32_t *>(a.scale + ((int64_t)(j0 >> 2) * a.nt16 + nt) * 64 + 4 * q) = sc4;
  a.nscr[(int64_t)blockIdx.y * a.nt16 * 16 + c] = s2;
}

// The window's squared norms into the pass's norm partials: column c of
// [A B] sums the quantising threads' partials (one per 128-row block): 16
// threads per column each sum every 16th partial in order, and the 16 sums
// are added in a fixed order (deterministic). The first window of a one-shot
// pass stores the result (and zeros in the other split slots), later windows
// and streaming pushes add.
constexpr int kNormSlices = 16;
__global__ __launch_bounds__(256) void fp8_norm_reduce_kernel(const double *__restrict__ nscr, int ny, int nt16,
                                                              int ntA16, int64_t n1, int64_t ntot, int S,
                                                              int accumulate, double *__restrict__ npart) {
  __shared__ double part[kNormSlices][256 / kNormSlices];
  const int cl = threadIdx.x % (256 / kNormSlices), sl = threadIdx.x / (256 / kNormSlices);
  const int64_t c = (int64_t)blockIdx.x * (256 / kNormSlices) + cl;
  const bool cv = c < ntot;
  const int64_t pc = !cv ? 0 : c < n1 ? c : (int64_t)ntA16 * 16 + (c - n1);
  const int64_t stride = (int64_t)nt16 * 16;
  double s = 0.0;
  if (cv)
    for (int y = sl; y < ny; y += kNormSlices) s += nscr[(int64_t)y * stride + pc];
  part[sl][cl] = s;
  __syncthreads();
  if (sl != 0 || !cv) return;
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < kNormSlices; ++u) t += part[u][cl];
  if (accumulate) {
    npart[c] += t;
  } else {
    npart[c] = t;
    for (int k = 1; k < S; ++k) npart[(int64_t)k * ntot + c] = 0.0;
  }
}

// Per 128-row step: each wave loads its two n-tiles' B operands and scale
// bytes and its share of the chunk's Pi fragments one step ahead; the Pi
// fragments go through LDS (double buffer), the B operands stay in registers.
// Steps past the end re-load the last step and multiply zero operands.
template <int MT>
__device__ __forceinline__ void loop_fp8_frag(const SkArgs &g, const SkWork &w, int nt0, int ntlast, int i0, int mv,
                                              v4u8 *L, v4f (&acc)[MT][2]) {
  constexpr int W = 8, NV = 2;
  constexpr int CPW = (MT + W - 1) / W;
  constexpr int LT = CPW * W;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const v4u8 *pi = reinterpret_cast<const v4u8 *>(g.pi) + (int64_t)i0 * kPiUnit8 + 2 * lane;
  const int64_t fstride = (int64_t)g.mt_total * kPiUnit8;
  const int64_t blk0 = w.lbeg / KP8;
  const int64_t nsteps = (w.lend - w.lbeg + KP8 - 1) / KP8;
  const v4u8 *df = reinterpret_cast<const v4u8 *>(g.dfrag) + lane;   // half h of lane t: unit 64 h + t
  const uint8_t *ds = g.dscale + 4 * (lane & 15) + (lane >> 4);   // lane (q, g): byte 4 q + g
  int ntv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int t = nt0 + 2 * wave + v;   // past the matrix: its last n-tile (those columns are never stored)
    ntv[v] = t < ntlast ? t : ntlast;
  }
  v4u8 rawb[NV][2];
  uint32_t raws[NV];
  v4u8 pst[CPW][2];
  v8i b[NV];
  int sb[NV];
  auto issue = [&](int64_t t) {   // t < nsteps; every load is unconditional
    const int64_t blk = blk0 + t;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t fb = blk * g.nt16 + ntv[v];
      rawb[v][0] = df[fb * 128];
      rawb[v][1] = df[fb * 128 + 64];
      raws[v] = ds[fb * 64];
    }
    const v4u8 *src = pi + blk * fstride;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int i = wave + W * j;
      const v4u8 *f = src + (i < mv ? i : mv - 1) * kPiUnit8;
      pst[j][0] = f[0];
      pst[j][1] = f[1];
    }
  };
  auto land = [&](int64_t t) {   // step t's Pi into LDS buffer t % 2, its B operands into b
    const bool valid = t < nsteps;
    v4u8 *Ld = L + (t & 1) * (LT * kPiUnit8);
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int i = wave + W * j;
      const bool keep = valid && i < mv;
      Ld[i * kPiUnit8 + 2 * lane] = keep ? pst[j][0] : v4u8{0u, 0u, 0u, 0u};
      Ld[i * kPiUnit8 + 2 * lane + 1] = keep ? pst[j][1] : v4u8{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const v4u8 lo = valid ? rawb[v][0] : v4u8{0u, 0u, 0u, 0u}, hi = valid ? rawb[v][1] : v4u8{0u, 0u, 0u, 0u};
      b[v] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      sb[v] = (int)(raws[v] & 0xffu);
    }
  };
  auto frag = [&](const v4u8 *Lc, int i) {
    const v4u8 lo = Lc[i * kPiUnit8 + 2 * lane], hi = Lc[i * kPiUnit8 + 2 * lane + 1];
    return v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
  };
  auto multiply = [&](const v4u8 *Lc) {
    constexpr int G = 2, NG = (MT + G - 1) / G;
    v8i a[2][G];
#pragma unroll
    for (int j = 0; j < G; ++j)
      if (j < MT) a[0][j] = frag(Lc, j);
#pragma unroll
    for (int gr = 0; gr < NG; ++gr) {
      if (gr + 1 < NG) {
#pragma unroll
        for (int j = 0; j < G; ++j)
          if ((gr + 1) * G + j < MT) a[(gr + 1) & 1][j] = frag(Lc, (gr + 1) * G + j);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const int i = gr * G + j;
        if (i < MT) {
#pragma unroll
          for (int v = 0; v < NV; ++v)
            acc[i][v] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[gr & 1][j], b[v], acc[i][v], 0, 0, 0, 127,
                                                                         0, sb[v]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  issue(0);
  land(0);
  for (int64_t t = 0; t < nsteps; ++t) {
    __syncthreads();   // step t's fragments are in LDS buffer t % 2; buffer (t + 1) % 2 is no longer read
    issue(t + 1 < nsteps ? t + 1 : nsteps - 1);
    __builtin_amdgcn_sched_barrier(0);
    multiply(L + (t & 1) * (LT * kPiUnit8));
    __builtin_amdgcn_sched_barrier(0);
    land(t + 1);
  }
}

template <int MT>
__global__ __launch_bounds__(512) void sketch_fp8_frag_kernel(SkArgs g) {
  constexpr int LT = (MT + 7) / 8 * 8;
  __shared__ __attribute__((aligned(16))) v4u8 L[2 * LT * kPiUnit8];

  SkWork w;
  if (!sk_decode(g, w)) return;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int q = lane & 15, gq = lane >> 4;
  const bool isb = w.col_base != 0;   // B's columns follow A's n1 >= 1 columns
  const int ntm0 = isb ? g.ntA16 : 0, ntml = isb ? g.nt16 - 1 : g.ntA16 - 1;
  const int nt0 = ntm0 + w.tile * 16;
  const int64_t col = (int64_t)w.tile * 256 + wave * 32 + q;   // n-tile v of the wave: columns col + 16 v
  const int i0 = w.kc * MT;
  const int mv = g.mt_total - i0 < MT ? g.mt_total - i0 : MT;

  v4f acc[MT][2];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int v = 0; v < 2; ++v) acc[i][v] = v4f{0.f, 0.f, 0.f, 0.f};
  const float ksum[2] = {0.f, 0.f}, kcmp[2] = {0.f, 0.f};

  if (w.lbeg < w.lend) loop_fp8_frag<MT>(g, w, nt0, ntml, i0, mv, L, acc);
  sk_epilogue<MT, 2, 16, false>(g, w, col, i0 * 16, gq, acc, ksum, kcmp);
}

constexpr int kFragMaxMt8 = 16;

template <int MT>
struct KTab8F {
  static void fill(KernelPtr *t) {
    t[MT] = sketch_fp8_frag_kernel<MT>;
    KTab8F<MT - 1>::fill(t);
  }
};
template <>
struct KTab8F<0> {
  static void fill(KernelPtr *) {}
};

KernelPtr fp8_frag_kernel_for(int mt) {
  static KernelPtr t[kFragMaxMt8 + 1];
  static const bool init = [] {
    KTab8F<kFragMaxMt8>::fill(t);
    return true;
  }();
  (void)init;
  return mt >= 1 && mt <= kFragMaxMt8 ? t[mt] : nullptr;
}


template <int NV, int MT>
struct KTab8 {
  static void fill(KernelPtr *t, KernelPtr *tc, KernelPtr *ts) {
    t[MT] = sketch_fp8_kernel<MT, NV, true, false>;
    tc[MT] = sketch_fp8_kernel<MT, NV, true, true>;
    ts[MT] = sketch_fp8_kernel<MT, NV, false, true>;
    KTab8<NV, MT - 1>::fill(t, tc, ts);
  }
};
template <int NV>
struct KTab8<NV, 0> {
  static void fill(KernelPtr *, KernelPtr *, KernelPtr *) {}
};

struct Shape8 {
  int nv, max_mt;
  KernelPtr t[9], tc[9], ts[9];
};

Shape8 *shapes8(int &count) {
  // the largest mt of each shape is the largest whose main kernel stays in
  // registers (no scratch) at two waves per SIMD
  static Shape8 tabs[] = {{2, 3, {}, {}, {}}, {1, 8, {}, {}, {}}};
  // function-local statics initialise once, also under concurrent first calls
  static const bool init = [] {
    KTab8<2, 3>::fill(tabs[0].t, tabs[0].tc, tabs[0].ts);
    KTab8<1, 8>::fill(tabs[1].t, tabs[1].tc, tabs[1].ts);
    return true;
  }();
  (void)init;
  count = (int)(sizeof(tabs) / sizeof(tabs[0]));
  return tabs;
}

template <int NV, int MT>
struct KTab8S {
  static void fill(KernelPtr *t, KernelPtr *tc, KernelPtr *ts) {
    t[MT] = sketch_fp8_stored_kernel<MT, NV, true, false>;
    tc[MT] = sketch_fp8_stored_kernel<MT, NV, true, true>;
    ts[MT] = sketch_fp8_stored_kernel<MT, NV, false, true>;
    KTab8S<NV, MT - 1>::fill(t, tc, ts);
  }
};
template <int NV>
struct KTab8S<NV, 0> {
  static void fill(KernelPtr *, KernelPtr *, KernelPtr *) {}
};

constexpr int kStoredMaxMt8 = 13;

KernelPtr fp8_stored_kernel_for(int mt, int variant) {
  static KernelPtr t[kStoredMaxMt8 + 1], tc[kStoredMaxMt8 + 1], ts[kStoredMaxMt8 + 1];
  static const bool init = [] {
    KTab8S<1, kStoredMaxMt8>::fill(t, tc, ts);
    return true;
  }();
  (void)init;
  if (mt < 1 || mt > kStoredMaxMt8) return nullptr;
  return variant == 0 ? t[mt] : variant == 1 ? tc[mt] : ts[mt];
}

// variant 0: vector loads over whole blocks; 1: vector loads, clamped; 2: scalar loads, clamped
KernelPtr fp8_kernel_for(int nv, int mt, int variant) {
  int count = 0;
  Shape8 *t = shapes8(count);
  for (int i = 0; i < count; ++i)
    if (t[i].nv == nv && mt >= 1 && mt <= t[i].max_mt)
      return variant == 0 ? t[i].t[mt] : variant == 1 ? t[i].tc[mt] : t[i].ts[mt];
  return nullptr;
}

}  // namespace

// Regenerating pass: 8 waves x 16 x nv columns, at most `cap` m-tiles per
// workgroup. SMP_SKETCH_TILE_FP8="nv,mt" overrides the tile (tuning sweeps).
static SketchPlan sketch_plan_fp8_regen(int k) {
  SketchPlan p{};
  p.prec = SMP_PREC_FP8;
  p.mt_total = (k + 15) / 16;
  int nv = 2, cap = 3;
  if (const char *e = getenv("SMP_SKETCH_TILE_FP8")) {
    int env[2] = {0, 0};
    if (sscanf(e, "%d,%d", &env[0], &env[1]) == 2 && fp8_kernel_for(env[0], env[1], 0)) {
      nv = env[0];
      cap = env[1];
    }
  }
  p.nv = nv;
  p.waves = 8;
  p.kc = KP8;
  p.kt = (p.mt_total + cap - 1) / cap;
  p.mt = (p.mt_total + p.kt - 1) / p.kt;
  p.ncol_tile = 16 * 8 * nv;
  p.kpad = p.mt_total * 16;
  p.kernel = reinterpret_cast<void *>(fp8_kernel_for(nv, p.mt, 0));
  p.kernel_clamp = reinterpret_cast<void *>(fp8_kernel_for(nv, p.mt, 1));
  p.kernel_scalar = reinterpret_cast<void *>(fp8_kernel_for(nv, p.mt, 2));
  return p;
}

// Fragment pass (the default): the data quantised window by window into MFMA
// operands, then 256-column tiles (two n-tiles per wave) of up to 16 m-tiles.
static SketchPlan sketch_plan_fp8_frag(int k) {
  SketchPlan p{};
  p.prec = SMP_PREC_FP8;
  p.pi_stored = 1;
  p.frag = 1;
  p.pi_rows = KP8;
  p.pi_frag_bytes = kPiUnit8 * 16;
  p.mt_total = (k + 15) / 16;
  p.nv = 2;
  p.waves = 8;
  p.kc = KP8;
  p.kt = (p.mt_total + kFragMaxMt8 - 1) / kFragMaxMt8;
  p.mt = (p.mt_total + p.kt - 1) / p.kt;
  p.ncol_tile = 16 * 8 * 2;
  p.kpad = p.mt_total * 16;
  p.kernel = reinterpret_cast<void *>(fp8_frag_kernel_for(p.mt));
  p.kernel_clamp = p.kernel;    // the fragment pass has no separate tail launch
  p.kernel_scalar = p.kernel;   // nor alignment variants (the quantisation reads any layout)
  return p;
}

// The stored-Pi pass converts the data in every chunk (128-column tiles, one
// column per lane, up to 13 m-tiles per workgroup): it reads the FP32 data
// ceil(k / 208) times, the fragment pass once plus one byte per value per
// chunk of 256 sketch rows. The fragment pass is the default from three
// stored-pass chunks (k > 416: 16.5 against 25.2 ms at d = 10^6, n = 8,192,
// k = 1,024), the stored-Pi pass below (1.31 against 1.35 ms at d = 200,000,
// n = 4,000, k = 400). SMP_SKETCH_FP8_STORED=0 selects the regenerating pass
// above, =1 the stored-Pi pass, =2 the fragment pass.
SketchPlan sketch_plan_fp8(int k) {
  const int mt_total = (k + 15) / 16;
  bool frag = mt_total > 2 * kStoredMaxMt8;
  if (const char *e = getenv("SMP_SKETCH_FP8_STORED")) {
    if (e[0] == '0' && e[1] == 0) return sketch_plan_fp8_regen(k);
    frag = e[0] == '2' && e[1] == 0;
  }
  if (frag) return sketch_plan_fp8_frag(k);
  SketchPlan p{};
  p.prec = SMP_PREC_FP8;
  p.pi_stored = 1;
  p.pi_rows = KP8;
  p.pi_frag_bytes = kPiUnit8 * 16;
  p.mt_total = (k + 15) / 16;
  p.nv = 1;
  p.waves = 8;
  p.kc = KP8;
  p.kt = (p.mt_total + kStoredMaxMt8 - 1) / kStoredMaxMt8;
  p.mt = (p.mt_total + p.kt - 1) / p.kt;
  p.ncol_tile = 16 * 8;
  p.kpad = p.mt_total * 16;
  p.kernel = reinterpret_cast<void *>(fp8_stored_kernel_for(p.mt, 0));
  p.kernel_clamp = reinterpret_cast<void *>(fp8_stored_kernel_for(p.mt, 1));
  p.kernel_scalar = reinterpret_cast<void *>(fp8_stored_kernel_for(p.mt, 2));
  return p;
}

// ---- fragment pass: the window and its scratch -------------------------------
// Scratch of one window of wr rows (wr / 128 blocks), each part 256-byte
// aligned: the Pi fragments (mt_total x 2 KiB per block), the data fragments
// and scales ((2 KiB + 64 B) per block and n-tile), and the per-thread norm
// partials (one row of nt16 x 16 FP64 values per 32 x 32 rows). nt16 is
// bounded by ntot / 16 + 2 (A's and B's n-tiles).
namespace {
int64_t frag_nt16_max(const SketchPlan &pl) { return pl.ntot / 16 + 2; }
size_t al256(size_t b) { return (b + 255) / 256 * 256; }
struct FragLayout {
  size_t pi, data, scale, nscr, total;
};
FragLayout frag_layout(const SketchPlan &pl, int64_t wr) {
  const int64_t nblk = (wr + KP8 - 1) / KP8, nt = frag_nt16_max(pl);
  const int64_t ny = (4 * nblk + kQuantBlocks32 - 1) / kQuantBlocks32;
  FragLayout f;
  f.pi = 0;
  f.data = al256((size_t)nblk * pl.mt_total * 2048);
  f.scale = f.data + al256((size_t)nblk * nt * 2048);
  f.nscr = f.scale + al256((size_t)nblk * nt * 64);
  f.total = f.nscr + al256((size_t)ny * nt * 16 * 8);
  return f;
}
}  // namespace

int64_t fp8_frag_window_rows(const SketchPlan &pl) {
  int64_t cap = kFragWindowBytes;
  if (const char *e = getenv("SMP_PI_WINDOW_MB")) {   // tuning override (as for the Pi windows)
    const long v = strtol(e, nullptr, 10);
    if (v >= 1 && v <= 4096) cap = (int64_t)v << 20;
  }
  const int64_t nt = frag_nt16_max(pl);
  const int64_t per_blk = (int64_t)pl.mt_total * 2048 + nt * (2048 + 64) + nt * 16 * 8 * 4 / kQuantBlocks32;
  return std::max<int64_t>(1, cap / per_blk) * KP8;
}

size_t fp8_frag_bytes(const SketchPlan &pl, int64_t rows) {
  if (rows <= 0) return 0;
  const int64_t wr = std::min<int64_t>((rows + KP8 - 1) / KP8 * KP8, fp8_frag_window_rows(pl));
  return frag_layout(pl, wr).total;
}

hipError_t fp8_frag_push(const SketchPlan &pl, const float *A, int64_t lda, int64_t n1, const float *B, int64_t ldb,
                         int64_t n2, int64_t rows, int k, uint64_t seed, int64_t row0, int S, bool accumulate,
                         float *part, double *npart, void *buf, hipStream_t st) {
  const KernelPtr kern = reinterpret_cast<KernelPtr>(pl.kernel);
  if (!kern) return hipErrorInvalidValue;
  if (rows > 0 && !buf) return hipErrorInvalidValue;
  const int ntA16 = (int)((n1 + 15) / 16), nt16 = ntA16 + (int)((n2 + 15) / 16);
  if (nt16 > frag_nt16_max(pl)) return hipErrorInvalidValue;   // the scratch was sized for fewer columns
  const int64_t ntot = n1 + n2;
  const int64_t wr = fp8_frag_window_rows(pl);
  const FragLayout lay = frag_layout(pl, std::min<int64_t>((rows + KP8 - 1) / KP8 * KP8, wr));
  char *cb = static_cast<char *>(buf);
  SkArgs g{};
  g.a = SkMat{A, lda, n1, 0, (int)((n1 + pl.ncol_tile - 1) / pl.ncol_tile), 1};
  g.b = B ? SkMat{B, ldb, n2, n1, (int)((n2 + pl.ncol_tile - 1) / pl.ncol_tile), 1}
          : SkMat{nullptr, 0, 0, n1, 0, 1};
  g.ntot = ntot;
  g.k = k;
  g.kpad = pl.kpad;
  g.kt = pl.kt;
  g.mt_total = pl.mt_total;
  g.seed = seed;
  g.part = part;
  g.npart = npart;
  g.S = S;
  g.split_unit = KP8;
  g.s_base = 0;
  g.nt16 = nt16;
  g.ntA16 = ntA16;
  const int64_t nlog = (int64_t)g.kt * (g.a.ntiles + g.b.ntiles) * S;
  const unsigned grid = (unsigned)((nlog + 7) / 8 * 8);
  const int64_t nwin = rows == 0 ? 1 : (rows + wr - 1) / wr;   // a one-shot pass with no rows still stores zeros
  for (int64_t w = 0; w < nwin; ++w) {
    const int64_t r0 = w * wr, wrows = std::min<int64_t>(wr, rows - r0);
    const int nblk = (int)((wrows + KP8 - 1) / KP8);
    const bool acc = accumulate || w > 0;
    if (nblk == 0 && accumulate) break;
    int ny = 0;
    if (nblk > 0) {
      hipError_t e = pi_store_fp8(pl, seed, row0 + r0, wrows, k, cb + lay.pi, st);
      if (e != hipSuccess) return e;
      QArgs q{A + r0 * lda, B ? B + r0 * ldb : nullptr, lda, ldb, n1, n2, wrows, nblk, nt16, ntA16, kQuantBlocks32,
              reinterpret_cast<uint8_t *>(cb + lay.data), reinterpret_cast<uint8_t *>(cb + lay.scale),
              reinterpret_cast<double *>(cb + lay.nscr)};
      ny = (4 * nblk + kQuantBlocks32 - 1) / kQuantBlocks32;
      hipLaunchKernelGGL(quantize_fp8_kernel, dim3((unsigned)((nt16 * 16 + 255) / 256), (unsigned)ny), dim3(256), 0,
                         st, q);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(fp8_norm_reduce_kernel, dim3((unsigned)((ntot + 15) / 16)), dim3(256), 0, st,
                       reinterpret_cast<const double *>(cb + lay.nscr), ny, nt16, ntA16, n1, ntot, S, acc ? 1 : 0,
                       npart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    g.row0 = row0 + r0;
    g.rows = (int64_t)nblk * KP8;
    g.rows_per_split = (int64_t)(nblk / S) * KP8;
    g.split_extra = nblk % S;
    g.accumulate = acc ? 1 : 0;
    g.pi = cb + lay.pi;
    g.dfrag = cb + lay.data;
    g.dscale = reinterpret_cast<const uint8_t *>(cb + lay.scale);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * pl.waves), 0, st, g);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t pi_store_fp8(const SketchPlan &pl, uint64_t seed, int64_t r0, int64_t rows, int k, void *buf,
                        hipStream_t st) {
  const int64_t frags = (rows + KP8 - 1) / KP8 * pl.mt_total;
  const int64_t grid = (frags * 16 + 255) / 256;
  hipLaunchKernelGGL(pi_store_fp8_kernel, dim3((unsigned)grid), dim3(256), 0, st, seed, r0, rows, k, pl.mt_total,
                     frags, static_cast<v4u8 *>(buf));
  return hipGetLastError();
}

}  // namespace smp

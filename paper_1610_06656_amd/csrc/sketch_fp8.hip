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
                                           v8i (&b)[NV], int (&sb)[NV], float (&ksum)[NV], float (&kcmp)[NV]) {
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
    if constexpr (NORM) kahan_add(ksum[v], kcmp[v], s2);
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

using KernelPtr = void (*)(SkArgs);

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

// Tile: 8 waves x 16 x nv columns, at most `cap` m-tiles per workgroup.
// SMP_SKETCH_TILE_FP8="nv,mt" overrides it (tuning sweeps).
SketchPlan sketch_plan_fp8(int k) {
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

}  // namespace smp

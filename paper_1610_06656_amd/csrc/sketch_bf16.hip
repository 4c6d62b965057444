// BF16 variant of the single pass of SMP-PCA (Alg. 1 step 2; Section 2
// "Step 1"): A~ = Pi A, B~ = Pi B with the GEMM operands rounded to BF16
// (round to nearest even) and FP32 accumulation on v_mfma_f32_16x16x32_bf16;
// the squared column norms come from the unrounded FP32 data with compensated
// sums, exactly as in the FP32 pass. The paper fixes no arithmetic precision;
// the Pi entries are the same N(0,1) draws as in the FP32 pass (same Philox
// counters), each rounded to BF16, so the two passes differ only by rounding.
//
// Structure. Each workgroup (8 waves) owns a tile of 16*8*NV data columns, a
// chunk of MT*16 sketch rows and one of S row splits, and regenerates the Pi
// block it needs (Pi is never stored). Per block of KP = 128 data rows:
//  * Pi block: MT*16 sketch rows x KP data rows as BF16 in LDS, sketch-row
//    major, so the 8 consecutive data rows one MFMA lane needs are one 16-byte
//    read. Each thread makes MT Philox calls per block (4 sketch rows of one
//    data row each), spread over the block's four K steps so that they overlap
//    the MFMAs; the next block is generated while this one is multiplied
//    (double buffer).
//  * Data: per MFMA K step of 32 rows, lane (q, g) loads rows 8g..8g+7 of its
//    NV adjacent columns (one vector load per row, addressed from a uniform
//    base plus one 32-bit offset), one step ahead of use; the rows are
//    converted with v_cvt_pk_bf16_f32 as they arrive.
// The main launch covers whole blocks only, so its hot loop has no row masks;
// the rows left over go to a second, clamping launch into one more partial
// slot. The kt workgroups of one data tile sit on one XCD with consecutive
// ids, so their re-reads of the tile are served by that XCD's L2.
//
// What bounds it (measured with rocprofv3 counters at d = 200,000,
// n1 = n2 = 2,000, k = 400): the per-CU vector-memory path, which carries
// every data tile kt times, and the VALU that regenerates Pi; the matrix cores
// are about 20% busy.
#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "sketch_common.hpp"
#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

namespace {

constexpr int kStep = 32;   // data rows per v_mfma_f32_16x16x32_bf16

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  const v2bf p = __builtin_convertvector((v2f){lo, hi}, v2bf);
  return __builtin_bit_cast(uint32_t, p);
}

// Part of a Pi block: sketch rows [c0, c0 + 16 MT) x data rows [lg, lg + KP)
// into LDS as BF16, element (c - c0) * (2 PSTW) + row. Thread t makes the
// calls u in [U0, U1) of its MT: data row t % KP, sketch rows
// 4 ((t / KP) + 4 u) .. +3, stored as four 16-bit LDS writes (adjacent lanes
// hold adjacent rows, so a wave writes 128 contiguous bytes per sketch row).
// Sketch rows c >= k and data rows past the first `valid` of the block are
// zero; `edge` says whether either can occur in this block (a uniform flag,
// so full blocks skip the masking).
template <int MT, int W, int U0, int U1>
__device__ __forceinline__ void gen_pi_bf16(uint32_t *P, int tid, uint64_t seed, uint64_t lg, int64_t valid, int c0,
                                            int k, bool edge) {
  constexpr int KP = 16 * W;
  constexpr int PST16 = KP + 8;   // bf16 elements per sketch row
  const int row = tid % KP;
  const int cb0 = tid / KP;
  const bool rv = row < valid;
  uint16_t *P16 = reinterpret_cast<uint16_t *>(P);
#pragma unroll
  for (int u = U0; u < U1; ++u) {
    const int cl = 4 * (cb0 + 4 * u);   // first sketch row of the call, relative to c0
    const int c = c0 + cl;
    float4 z = normals4(stream_call(seed, kTagPi, lg + (uint64_t)row, (uint32_t)(c >> 2)));
    if (edge) {
      z.x = rv && c + 0 < k ? z.x : 0.f;
      z.y = rv && c + 1 < k ? z.y : 0.f;
      z.z = rv && c + 2 < k ? z.z : 0.f;
      z.w = rv && c + 3 < k ? z.w : 0.f;
    }
    const uint32_t p01 = pack_bf16(z.x, z.y), p23 = pack_bf16(z.z, z.w);
    uint16_t *dst = P16 + cl * PST16 + row;
    dst[0] = (uint16_t)p01;
    dst[PST16] = (uint16_t)(p01 >> 16);
    dst[2 * PST16] = (uint16_t)p23;
    dst[3 * PST16] = (uint16_t)(p23 >> 16);
  }
}

// NV adjacent FP32 values of one data row, held as one vector register tuple.
template <int NV>
struct RowT {
  typedef float type __attribute__((ext_vector_type(NV)));
};
template <int NV>
using Row = typename RowT<NV>::type;

// NV adjacent columns of one data row (clamping as in sk_load_row: a row past
// row_last reads row_last again; the caller zeroes its Pi entries).
template <int NV, bool FULL>
__device__ __forceinline__ Row<NV> load_rowv(const float *X, int64_t ld, int64_t n, int64_t row, int64_t row_last,
                                             int64_t col) {
  const bool row_ok = row <= row_last;
  Row<NV> r;
  if constexpr (FULL) {
    r = *reinterpret_cast<const Row<NV> *>(X + (row_ok ? row : row_last) * ld + col);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) r[v] = 0.0f;
    if (row_ok && col < n) {
      const float *p = X + row * ld + col;
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (col + v < n) r[v] = p[v];
    }
  }
  return r;
}

template <int NV>
__device__ __forceinline__ void convert_step(const Row<NV> (&x)[8], v8bf (&b)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = pack_bf16(x[2 * e][v], x[2 * e + 1][v]);
    typedef uint32_t v4u __attribute__((ext_vector_type(4)));
    b[v] = __builtin_bit_cast(v8bf, (v4u){w[0], w[1], w[2], w[3]});
  }
}

// One K step: norms of the unrounded rows, BF16 conversion, MT x NV MFMAs.
// The rows of one K step as they arrive: their squared norms (rows past
// row_last, re-reads of row_last that meet zero Pi entries, are left out) and
// their BF16 packing into the MFMA B operands.
template <int NV, bool NORM, bool CLAMP>
__device__ __forceinline__ void finish_rows(const Row<NV> (&x)[8], int64_t row, int64_t row_last, v8bf (&b)[NV],
                                            float (&ksum)[NV], float (&kcmp)[NV]) {
  if constexpr (NORM) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float s8 = 0.0f;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        s8 = (!CLAMP || row + e <= row_last) ? __builtin_fmaf(x[e][v], x[e][v], s8) : s8;
      kahan_add(ksum[v], kcmp[v], s8);
    }
  }
  convert_step<NV>(x, b);
}

// All MT Pi fragments of the step are read from LDS before the first MFMA,
// so the LDS latency is paid once per step rather than once per m-tile.
template <int MT, int NV, int PSTW>
__device__ __forceinline__ void mfma_step(const v8bf (&b)[NV], const uint32_t *Pst, int q, v4f (&acc)[MT][NV]) {
  v8bf a[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) a[i] = *reinterpret_cast<const v8bf *>(Pst + (16 * i + q) * PSTW);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[i][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[v], acc[i][v], 0, 0, 0);
}

// Addressing of a workgroup's rows: a uniform base (its first row) plus one
// 32-bit element offset per lane, so the loads take the SGPR-base +
// VGPR-offset form and no per-row 64-bit address stays live. The host keeps
// every split below 2^31 elements.
struct RowAddr {
  const float *base;   // row lbeg, column 0 (uniform)
  uint32_t lane_off;   // (8 gq) * ld + column of this lane's first vector
  uint32_t ld;
  int64_t nrows;       // rows of the split
};

// Rows rel + 8 gq + e (e < 8, relative to lbeg) of the lane's NV columns.
// CLAMP: rows past the split re-read its last row (their Pi entries are zero
// and the norms leave them out); without CLAMP every row read is inside the
// split (the main launch covers whole blocks only).
template <int NV, bool VEC, bool CLAMP>
__device__ __forceinline__ void load_step(const SkWork &w, const RowAddr &ra, int64_t rel, int gq, int64_t col,
                                          Row<NV> (&x)[8]) {
  if constexpr (VEC) {
    if (!CLAMP || rel + kStep <= ra.nrows) {   // uniform: the whole step is inside the split
      const float *bs = ra.base + (size_t)rel * ra.ld;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        x[e] = *reinterpret_cast<const Row<NV> *>(bs + (size_t)e * ra.ld + ra.lane_off);
    } else {
      const int64_t last = ra.nrows - 1;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t r = rel + 8 * gq + e;
        x[e] = *reinterpret_cast<const Row<NV> *>(ra.base + (r <= last ? r : last) * (int64_t)ra.ld + col);
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      x[e] = load_rowv<NV, false>(w.X, w.ld, w.n, w.lbeg + rel + 8 * gq + e, w.lend - 1, col);
  }
}

// One K step of a block, software-pipelined: issue the loads of the next
// step, generate this step's share of the next block's Pi, multiply this
// step (its rows were converted at the end of the previous step), then
// convert the next step's rows once they arrive. The scheduling barriers keep
// that order (left free, the compiler sinks the loads next to their use and
// the latency is exposed every step).
template <int MT, int NV, int W, int GS, bool VEC, bool CLAMP, bool NORM, int ST>
__device__ __forceinline__ void block_step(const SkArgs &g, const SkWork &w, const RowAddr &ra, int64_t l,
                                           int64_t row_last, int64_t col, int c0, const uint32_t *Pc, uint32_t *Pn,
                                           bool more, bool edge_next, Row<NV> (&raw)[8], v8bf (&b)[NV],
                                           v4f (&acc)[MT][NV], float (&ksum)[NV], float (&kcmp)[NV]) {
  constexpr int KP = 16 * W;
  constexpr int PSTW = KP / 2 + 4;
  constexpr int NSTEP = KP / kStep;
  const int tid = threadIdx.x;
  const int lane = tid & 63, q = lane & 15, gq = lane >> 4;
  const int64_t rel = l - w.lbeg + kStep * (ST + 1);   // next step, relative to the split
  const int64_t rn = w.lbeg + rel + 8 * gq;            // first row of this lane in the next step
  // the last step of a split's last block has no next step (without CLAMP it would read past the split)
  const bool next = CLAMP || ST + 1 < NSTEP || more;
  if (next) load_step<NV, VEC, CLAMP>(w, ra, rel, gq, col, raw);
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (ST < GS) {
    if (more)
      gen_pi_bf16<MT, W, ST * MT / GS, (ST + 1) * MT / GS>(Pn, tid, g.seed, (uint64_t)(g.row0 + l + KP),
                                                          w.lend - (l + KP), c0, g.k, edge_next);
  }
  mfma_step<MT, NV, PSTW>(b, Pc + (kStep / 2) * ST + 4 * gq, q, acc);
  __builtin_amdgcn_sched_barrier(0);
  if (next) finish_rows<NV, NORM, CLAMP>(raw, rn, row_last, b, ksum, kcmp);
}

// VEC: every lane loads its NV columns with one aligned vector load; lanes
// past the last column load the last vector again (their results are not
// stored). Otherwise every element is loaded on its own, guarded.
template <int MT, int NV, int W, int GS, bool VEC, bool CLAMP, bool NORM>
__device__ __forceinline__ void loop_bf16(const SkArgs &g, const SkWork &w, int64_t col, int c0, uint32_t *P0,
                                          uint32_t *P1, v4f (&acc)[MT][NV], float (&ksum)[NV], float (&kcmp)[NV]) {
  constexpr int KP = 16 * W;
  static_assert(KP / kStep == 4, "four K steps per Pi block");
  const int tid = threadIdx.x;
  const int gq = (tid & 63) >> 4;
  const int64_t row_last = w.lend - 1;
  const bool kedge = c0 + 16 * MT > g.k;   // the chunk has padding sketch rows
  const int64_t lcol = VEC ? (col < w.n - NV ? col : w.n - NV) : col;

  RowAddr ra;
  ra.base = w.X + w.lbeg * w.ld;
  ra.ld = (uint32_t)w.ld;
  ra.lane_off = (uint32_t)(8 * gq) * ra.ld + (uint32_t)lcol;
  ra.nrows = w.lend - w.lbeg;
  Row<NV> raw[8];
  v8bf b[NV];
  load_step<NV, VEC, CLAMP>(w, ra, 0, gq, lcol, raw);
  gen_pi_bf16<MT, W, 0, MT>(P0, tid, g.seed, (uint64_t)(g.row0 + w.lbeg), w.lend - w.lbeg, c0, g.k,
                            kedge || (CLAMP && w.lend - w.lbeg < KP));
  finish_rows<NV, NORM, CLAMP>(raw, w.lbeg + 8 * gq, row_last, b, ksum, kcmp);

  int buf = 0;
  for (int64_t l = w.lbeg; l < w.lend; l += KP) {
    __syncthreads();   // Pi of this block is complete; the other buffer is free
    const uint32_t *Pc = buf ? P1 : P0;
    uint32_t *Pn = buf ? P0 : P1;
    const bool more = l + KP < w.lend;
    const bool edge_next = kedge || (CLAMP && w.lend - (l + KP) < KP);
    block_step<MT, NV, W, GS, VEC, CLAMP, NORM, 0>(g, w, ra, l, row_last, lcol, c0, Pc, Pn, more, edge_next, raw, b, acc, ksum, kcmp);
    block_step<MT, NV, W, GS, VEC, CLAMP, NORM, 1>(g, w, ra, l, row_last, lcol, c0, Pc, Pn, more, edge_next, raw, b, acc, ksum, kcmp);
    block_step<MT, NV, W, GS, VEC, CLAMP, NORM, 2>(g, w, ra, l, row_last, lcol, c0, Pc, Pn, more, edge_next, raw, b, acc, ksum, kcmp);
    block_step<MT, NV, W, GS, VEC, CLAMP, NORM, 3>(g, w, ra, l, row_last, lcol, c0, Pc, Pn, more, edge_next, raw, b, acc, ksum, kcmp);
    buf ^= 1;
  }
}

// VEC: vector loads (see loop_bf16). CLAMP: the launch may hold partial blocks
// (rows past a split's end are clamped and masked); the main launch of a pass
// covers whole blocks only and runs without.
template <int MT, int NV, int W, int GS, bool VEC, bool CLAMP>
__global__ __launch_bounds__(64 * W) void sketch_bf16_kernel(SkArgs g) {
  constexpr int KP = 16 * W;
  constexpr int PSTW = KP / 2 + 4;
  constexpr int PBUF = MT * 16 * PSTW;   // dwords of one Pi block
  __shared__ __attribute__((aligned(16))) uint32_t P[2 * PBUF];

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
    if (w.kc == 0) loop_bf16<MT, NV, W, GS, VEC, CLAMP, true>(g, w, col, c0, P, P + PBUF, acc, ksum, kcmp);
    else loop_bf16<MT, NV, W, GS, VEC, CLAMP, false>(g, w, col, c0, P, P + PBUF, acc, ksum, kcmp);
  }
  sk_epilogue<MT, NV>(g, w, col, c0, gq, acc, ksum, kcmp);
}

using KernelPtr = void (*)(SkArgs);

template <int NV, int W, int GS, int MT>
struct KTab {
  static void fill(KernelPtr *t, KernelPtr *tc, KernelPtr *ts) {
    t[MT] = sketch_bf16_kernel<MT, NV, W, GS, true, false>;
    tc[MT] = sketch_bf16_kernel<MT, NV, W, GS, true, true>;
    ts[MT] = sketch_bf16_kernel<MT, NV, W, GS, false, true>;
    KTab<NV, W, GS, MT - 1>::fill(t, tc, ts);
  }
};
template <int NV, int W, int GS>
struct KTab<NV, W, GS, 0> {
  static void fill(KernelPtr *, KernelPtr *, KernelPtr *) {}
};

// gs: the K steps of a block over which the next block's Pi generation is
// spread (fewer steps: more independent Philox chains in flight per step)
struct Shape {
  int nv, waves, gs, max_mt;
  KernelPtr t[14];    // vector loads, whole blocks
  KernelPtr tc[14];   // vector loads, clamped partial blocks
  KernelPtr ts[14];   // guarded scalar loads, clamped
};

Shape *shapes(int &count) {
  // (nv, waves, largest mt that keeps the kernel in registers without scratch)
  // the largest mt of each shape is the largest whose main kernel stays in
  // registers (no scratch) at two waves per SIMD
  static Shape tabs[] = {{4, 8, 4, 4, {}, {}, {}}, {2, 8, 4, 12, {}, {}, {}}};
  // function-local statics initialise once, also under concurrent first calls
  static const bool init = [] {
    KTab<4, 8, 4, 4>::fill(tabs[0].t, tabs[0].tc, tabs[0].ts);
    KTab<2, 8, 4, 12>::fill(tabs[1].t, tabs[1].tc, tabs[1].ts);
    return true;
  }();
  (void)init;
  count = (int)(sizeof(tabs) / sizeof(tabs[0]));
  return tabs;
}

// variant 0: vector loads over whole blocks; 1: vector loads, clamped; 2: scalar loads, clamped
KernelPtr bf16_kernel_for(int nv, int mt, int waves, int gs, int variant) {
  int count = 0;
  Shape *t = shapes(count);
  for (int i = 0; i < count; ++i)
    if (t[i].nv == nv && t[i].waves == waves && t[i].gs == gs && mt >= 1 && mt <= t[i].max_mt)
      return variant == 0 ? t[i].t[mt] : variant == 1 ? t[i].tc[mt] : t[i].ts[mt];
  return nullptr;
}

}  // namespace

// Tile choice. Two per-CU resources bound the pass: the vector-memory path
// (every byte of a data tile passes each CU's L1 once per sketch-row chunk,
// so its load grows with kt) and the VALU that regenerates Pi (which grows
// with the number of column tiles, i.e. shrinks with the tile width). The
// accumulators (mt * nv * 4 VGPRs per lane) cap width x chunk. Measured at
// d = 200,000, n1 = n2 = 2,000, k = 400: 512-column tiles of 4 m-tiles
// (kt = 7) are the fastest; for larger k the 256-column tiles of up to 12
// m-tiles keep kt lower. SMP_SKETCH_TILE_BF16="nv,mt[,waves[,gs]]" overrides
// the choice (tuning sweeps).
SketchPlan sketch_plan_bf16(int k) {
  SketchPlan p{};
  p.prec = SMP_PREC_BF16;
  p.mt_total = (k + 15) / 16;
  int nv = 4, cap = 4, waves = 8, gs = 4;
  if (p.mt_total > 28) {
    nv = 2;
    cap = 12;
  }
  if (const char *e = getenv("SMP_SKETCH_TILE_BF16")) {
    int env[4] = {0, 0, 8, 4};
    const int got = sscanf(e, "%d,%d,%d,%d", &env[0], &env[1], &env[2], &env[3]);
    if (got >= 2 && bf16_kernel_for(env[0], env[1], env[2], env[3], 0)) {
      nv = env[0];
      cap = env[1];
      waves = env[2];
      gs = env[3];
    }
  }
  p.nv = nv;
  p.waves = waves;
  p.kc = 16 * waves;
  p.kt = (p.mt_total + cap - 1) / cap;
  p.mt = (p.mt_total + p.kt - 1) / p.kt;
  p.ncol_tile = 16 * waves * nv;
  p.kpad = p.mt_total * 16;
  p.kernel = reinterpret_cast<void *>(bf16_kernel_for(nv, p.mt, waves, gs, 0));
  p.kernel_clamp = reinterpret_cast<void *>(bf16_kernel_for(nv, p.mt, waves, gs, 1));
  p.kernel_scalar = reinterpret_cast<void *>(bf16_kernel_for(nv, p.mt, waves, gs, 2));
  return p;
}

}  // namespace smp

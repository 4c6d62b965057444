// BF16 variant of the single pass of SMP-PCA (Alg. 1 step 2; Section 2
// "Step 1"): A~ = Pi A, B~ = Pi B with the GEMM operands rounded to BF16
// (round to nearest even) and FP32 accumulation on v_mfma_f32_16x16x32_bf16;
// the squared column norms come from the unrounded FP32 data with compensated
// sums, exactly as in the FP32 pass. The paper fixes no arithmetic precision;
// the Pi entries are the same N(0,1) draws as in the FP32 pass (same Philox
// counters), each rounded to BF16, so the two passes differ only by rounding.
//
// Two passes share this file.
//
// Stored-Pi pass (the default). Pi is drawn once per push (one Philox call per
// four sketch rows of a data row) into a scratch buffer in the MFMA A-operand
// order, and the pass is a split-K GEMM over it: each workgroup (8 waves, two
// per SIMD) owns 16*8*NV = 256 columns, a chunk of up to 16 m-tiles and one of
// S row splits. Per K step of 32 rows every lane loads its 8 rows x NV
// columns and each wave copies its share of the chunk's 1 KiB Pi fragments
// into an LDS buffer, D steps ahead of use; the wave then multiplies all
// m-tiles of the chunk for its 16*NV columns. At d = 200,000, n1 = n2 = 2,000,
// k = 400 (kt = 2 chunks) the per-CU vector L1 is what bounds it: about 100
// misses in flight per CU at 600-800 cycles of L2 latency, i.e. about 19
// bytes per clock per CU, for 2.8 bytes of L1 fill per byte of data (the data
// read by both chunks, Pi read by each of the 16 column tiles). A wider tile
// or a single chunk would cut that ratio, but the accumulators of 256
// columns x 400 sketch rows fill the register file (400 of the 512 registers
// per lane at one wave per SIMD), and the compiler then shuttles them between
// AGPRs and VGPRs every step.
//
// Regenerating pass (SMP_SKETCH_BF16_STORED=0; needs no scratch). Each
// workgroup (8 waves) owns a tile of 16*8*NV data columns, a chunk of MT*16
// sketch rows and one of S row splits, and regenerates the Pi block it needs.
// Per block of KP = 128 data rows:
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
#include <functional>
#include <vector>

#include "sketch_common.hpp"
#include "smp_device.hpp"
#include "smp_internal.hpp"

namespace smp {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

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

// Unaligned inputs: one 4-byte load per value from a clamped row and column,
// all unconditional (a row past the split reads its last row, whose Pi
// entries are zero there and which the norms leave out; a column past n reads
// column n - 1 into an accumulator that is never stored). Offsets are 32-bit
// from the split's first row (the host keeps every split below 2^31 elements).
template <int NV>
__device__ __forceinline__ void load_step_clamped(const RowAddr &ra, int64_t rel, int gq, const uint32_t (&c)[NV],
                                                  Row<NV> (&x)[8]) {
  const int64_t last = ra.nrows - 1;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t r = rel + 8 * gq + e;
    const uint32_t ro = (uint32_t)(r <= last ? r : last) * ra.ld;
#pragma unroll
    for (int v = 0; v < NV; ++v) x[e][v] = ra.base[ro + c[v]];
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
__device__ __forceinline__ void sketch_bf16_body(const SkArgs &g, const SkWork &w) {
  constexpr int KP = 16 * W;
  constexpr int PSTW = KP / 2 + 4;
  constexpr int PBUF = MT * 16 * PSTW;   // dwords of one Pi block
  __shared__ __attribute__((aligned(16))) uint32_t P[2 * PBUF];

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

template <int MT, int NV, int W, int GS, bool VEC, bool CLAMP>
__global__ __launch_bounds__(64 * W) void sketch_bf16_kernel(SkArgs g) {
  SkWork w;
  if (!sk_decode(g, w)) return;
  sketch_bf16_body<MT, NV, W, GS, VEC, CLAMP>(g, w);
}

// Grouped form: the launch of many jobs' passes at once (blockIdx.y = job,
// its arguments and its own grid size from a device table; grid.x is the
// largest of the jobs' grids). Workgroup b of a job is its workgroup b of a
// launch of its own, decoded over the job's grid, so each job's work keeps the
// XCD spread of a launch of its own; the surplus workgroups of smaller jobs
// exit at once.
template <int MT, int NV, int W, int GS, bool VEC, bool CLAMP>
__global__ __launch_bounds__(64 * W) void sketch_bf16_group_kernel(const SkJob *__restrict__ jobs) {
  const int grid = jobs[blockIdx.y].grid;
  if ((int)blockIdx.x >= grid) return;
  const SkArgs g = jobs[blockIdx.y].g;   // uniform: held in scalar registers like kernel arguments
  SkWork w;
  if (!sk_decode_in(g, w, (int)blockIdx.x, grid)) return;
  sketch_bf16_body<MT, NV, W, GS, VEC, CLAMP>(g, w);
}

using KernelPtr = void (*)(SkArgs);

using GroupKernelPtr = void (*)(const SkJob *);

template <int NV, int W, int GS, int MT>
struct KTab {
  static void fill(KernelPtr *t, KernelPtr *tc, KernelPtr *ts, GroupKernelPtr *gt, GroupKernelPtr *gtc,
                   GroupKernelPtr *gts) {
    t[MT] = sketch_bf16_kernel<MT, NV, W, GS, true, false>;
    tc[MT] = sketch_bf16_kernel<MT, NV, W, GS, true, true>;
    ts[MT] = sketch_bf16_kernel<MT, NV, W, GS, false, true>;
    gt[MT] = sketch_bf16_group_kernel<MT, NV, W, GS, true, false>;
    gtc[MT] = sketch_bf16_group_kernel<MT, NV, W, GS, true, true>;
    gts[MT] = sketch_bf16_group_kernel<MT, NV, W, GS, false, true>;
    KTab<NV, W, GS, MT - 1>::fill(t, tc, ts, gt, gtc, gts);
  }
};
template <int NV, int W, int GS>
struct KTab<NV, W, GS, 0> {
  static void fill(KernelPtr *, KernelPtr *, KernelPtr *, GroupKernelPtr *, GroupKernelPtr *, GroupKernelPtr *) {}
};

// gs: the K steps of a block over which the next block's Pi generation is
// spread (fewer steps: more independent Philox chains in flight per step)
struct Shape {
  int nv, waves, gs, max_mt;
  KernelPtr t[14];    // vector loads, whole blocks
  KernelPtr tc[14];   // vector loads, clamped partial blocks
  KernelPtr ts[14];   // guarded scalar loads, clamped
  GroupKernelPtr gt[14], gtc[14], gts[14];   // the same three as grouped launches
};

Shape *shapes(int &count) {
  // (nv, waves, largest mt that keeps the kernel in registers without scratch)
  // the largest mt of each shape is the largest whose main kernel stays in
  // registers (no scratch) at two waves per SIMD
  static Shape tabs[] = {{4, 8, 4, 4, {}, {}, {}, {}, {}, {}}, {2, 8, 4, 12, {}, {}, {}, {}, {}, {}}};
  // function-local statics initialise once, also under concurrent first calls
  static const bool init = [] {
    KTab<4, 8, 4, 4>::fill(tabs[0].t, tabs[0].tc, tabs[0].ts, tabs[0].gt, tabs[0].gtc, tabs[0].gts);
    KTab<2, 8, 4, 12>::fill(tabs[1].t, tabs[1].tc, tabs[1].ts, tabs[1].gt, tabs[1].gtc, tabs[1].gts);
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

// the grouped kernel of the same shape and variant as a plan's kernel
GroupKernelPtr bf16_group_kernel_for(int nv, int mt, int waves, int gs, int variant) {
  int count = 0;
  Shape *t = shapes(count);
  for (int i = 0; i < count; ++i)
    if (t[i].nv == nv && t[i].waves == waves && t[i].gs == gs && mt >= 1 && mt <= t[i].max_mt)
      return variant == 0 ? t[i].gt[mt] : variant == 1 ? t[i].gtc[mt] : t[i].gts[mt];
  return nullptr;
}

// ---------------------------------------------------------------------------
// Stored-Pi variant. Pi is drawn once per pass (one Philox call per four sketch
// rows of a data row, as above) into a buffer laid out in the A-operand order
// of v_mfma_f32_16x16x32_bf16, and the pass itself is a split-K GEMM that
// streams that buffer through LDS. Every workgroup then covers all m-tiles of
// its chunk for 16*8*NV columns, so a data tile crosses the CU's vector-memory
// path once per chunk instead of once per 4-tile chunk, and no column tile
// repeats the Philox work.
//
// Buffer layout: 16-byte unit (b * mt_total + i) * 64 + t holds, for lane
// t = 16 g + q, the BF16 entries of sketch row 16 i + q at the data rows
// 32 b + 8 g + (0..7) of the pass (b: 32-row block from the pass's first
// row). One (b, i) pair is 1 KiB, the operand of one MFMA.

constexpr int kPiUnit = 64;   // 16-byte units per (block, m-tile) fragment

// Thread u of the grid fills lanes 16 g + 4 q4 + (0..3) of fragment u / 16
// (g, q4 from u % 16): eight Philox calls (rows 32 b + 8 g + e, sketch rows
// 16 i + 4 q4 .. +3) and four 16-byte stores that are contiguous across the
// 16 threads of one fragment. Rows past nrows and sketch rows >= k are zero.
__global__ __launch_bounds__(256) void pi_store_bf16_kernel(uint64_t seed, int64_t r0, int64_t nrows, int k,
                                                            int mt_total, int64_t frags, v4u *__restrict__ out) {
  const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (u >= frags * 16) return;
  const int64_t frag = u >> 4;
  const int sub = (int)(u & 15);
  const int g = sub >> 2, q4 = sub & 3;
  const int i = (int)(frag % mt_total);
  const int64_t blk = frag / mt_total;
  const int c = 16 * i + 4 * q4;
  float z[8][4];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t l = 32 * blk + 8 * g + e;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (l < nrows && c < k) v = normals4(stream_call(seed, kTagPi, (uint64_t)(r0 + l), (uint32_t)(c >> 2)));
    z[e][0] = v.x;
    z[e][1] = c + 1 < k ? v.y : 0.f;
    z[e][2] = c + 2 < k ? v.z : 0.f;
    z[e][3] = c + 3 < k ? v.w : 0.f;
  }
  v4u *dst = out + frag * kPiUnit + 16 * g + 4 * q4;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    dst[j] = v4u{pack_bf16(z[0][j], z[1][j]), pack_bf16(z[2][j], z[3][j]), pack_bf16(z[4][j], z[5][j]),
                 pack_bf16(z[6][j], z[7][j])};
}

// One K step of the stored-Pi pass: MT x NV MFMAs whose A fragments are read
// from LDS in groups of G, the next group's reads issued before this group's
// products so that the LDS latency overlaps the matrix cores.
template <int MT, int NV, int G>
__device__ __forceinline__ void mfma_step_stored(const v8bf (&b)[NV], const v4u *Lc, int lane, v4f (&acc)[MT][NV]) {
  constexpr int NG = (MT + G - 1) / G;
  v8bf a[2][G];
#pragma unroll
  for (int j = 0; j < G; ++j)
    if (j < MT) a[0][j] = __builtin_bit_cast(v8bf, Lc[j * kPiUnit + lane]);
#pragma unroll
  for (int gr = 0; gr < NG; ++gr) {
    if (gr + 1 < NG) {
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const int i = (gr + 1) * G + j;
        if (i < MT) a[(gr + 1) & 1][j] = __builtin_bit_cast(v8bf, Lc[i * kPiUnit + lane]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const int i = gr * G + j;
      if (i < MT) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
          acc[i][v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[gr & 1][j], b[v], acc[i][v], 0, 0, 0);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Per K step t of 32 rows: issue the data loads and the Pi fragment loads of
// step t + D into register set t % D (D steps of loads in flight, so that one
// workgroup per CU covers the memory latency), multiply step t (Pi from LDS
// buffer t % D), then store step t + 1's fragments into LDS buffer
// (t + 1) % D and convert its rows. Wave w copies fragments w, w + W, ... of
// the chunk (one 1 KiB fragment per load instruction). Fragments of m-tiles
// past the chunk's valid ones are stored as zeros, so every wave runs the same
// MT x NV products.
//
// The loop body has no data-dependent branches: the steps run in whole groups
// of D, prefetches past the last step re-load the last step, and steps past
// the end land zero Pi fragments and add nothing to the norms. (With the
// issue and the landing under conditions, the compiler cannot prove that a
// register set's previous loads have completed and waits for every load in
// flight before reusing it, which serialises the prefetch.)
// Paired 16-byte row loads (nv = 2). Lanes q and q + 8 of a row group
// (q < 8) own the four adjacent columns 4q .. 4q + 3 of the wave's 32 (lane q
// the first two, lane q + 8 the last two); lane q loads those four columns of
// the group's even rows, lane q + 8 of its odd rows, so that every load is 16
// bytes wide (half as many load instructions as one 8-byte load per row) and
// lanes 0-7 and 8-15 each read one whole 128-byte line. Unpacking swaps the
// halves between the two lanes (DPP rotation by 8 within the 16-lane row)
// and leaves each lane its own two columns of all 8 rows, exactly the values
// the 8-byte loads give.
struct PairAddr {
  const float *base;   // row lbeg, column 0 (uniform)
  uint32_t lane_off;   // (8 gq + parity) * ld + first of the pair's four columns
  uint32_t ld;
  uint32_t pcol;       // first of the pair's four columns (clamped into the matrix)
  int64_t nrows;       // rows of the split
};

template <bool CLAMP>
__device__ __forceinline__ void load_pair_step(const PairAddr &pa, int64_t rel, int gq, int par, v4f (&y)[4]) {
  if (!CLAMP || rel + kStep <= pa.nrows) {   // uniform: the whole step is inside the split
    const float *bs = pa.base + (size_t)rel * pa.ld;
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] = *reinterpret_cast<const v4f *>(bs + (size_t)(2 * i) * pa.ld + pa.lane_off);
  } else {
    const int64_t last = pa.nrows - 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = rel + 8 * gq + 2 * i + par;
      y[i] = *reinterpret_cast<const v4f *>(pa.base + (r <= last ? r : last) * (int64_t)pa.ld + pa.pcol);
    }
  }
}

__device__ __forceinline__ float swap_pair(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x128, 0xF, 0xF, false));
}

__device__ __forceinline__ void unpack_pair_step(const v4f (&y)[4], int par, Row<2> (&x)[8]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const float a = y[i][v], c = y[i][2 + v];
      const float recv = swap_pair(par ? a : c);
      x[2 * i][v] = par ? recv : a;
      x[2 * i + 1][v] = par ? c : recv;
    }
}

template <int NV, bool NORM, bool CLAMP>
__device__ __forceinline__ void finish_rows_if(const Row<NV> (&x)[8], int64_t row, int64_t row_last, bool valid,
                                               v8bf (&b)[NV], float (&ksum)[NV], float (&kcmp)[NV]) {
  if constexpr (NORM) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float s8 = 0.0f;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        s8 = (!CLAMP || row + e <= row_last) ? __builtin_fmaf(x[e][v], x[e][v], s8) : s8;
      kahan_add(ksum[v], kcmp[v], valid ? s8 : 0.0f);
    }
  }
  convert_step<NV>(x, b);
}

template <int MT, int NV, int G, int W, int D, bool VEC, bool CLAMP, bool NORM, bool PAIRED>
__device__ __forceinline__ void loop_bf16_stored(const SkArgs &g, const SkWork &w, int64_t col, int i0, int mv,
                                                 v4u *L, v4f (&acc)[MT][NV], float (&ksum)[NV], float (&kcmp)[NV]) {
  static_assert(D >= 2, "step t + 1 lands in another LDS buffer than the one step t reads");
  constexpr int CPW = (MT + W - 1) / W;
  constexpr int LT = CPW * W;   // m-tile slots per LDS buffer
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, gq = lane >> 4;
  const int64_t row_last = w.lend - 1;
  const int64_t lcol = VEC ? (col < w.n - NV ? col : w.n - NV) : col;
  const v4u *pi = reinterpret_cast<const v4u *>(g.pi) + (int64_t)i0 * kPiUnit + lane;
  const int64_t fstride = (int64_t)g.mt_total * kPiUnit;   // units per 32-row block
  const int64_t blk0 = w.lbeg / kStep;
  const int64_t nsteps = (w.lend - w.lbeg + kStep - 1) / kStep;

  RowAddr ra;
  ra.base = w.X + w.lbeg * w.ld;
  ra.ld = (uint32_t)w.ld;
  ra.lane_off = (uint32_t)(8 * gq) * ra.ld + (uint32_t)lcol;
  ra.nrows = w.lend - w.lbeg;
  constexpr bool PAIR = VEC && NV == 2 && PAIRED;   // paired 16-byte loads (the host then requires 4-element alignment)
  const int par = (lane >> 3) & 1;
  PairAddr pa;
  if constexpr (PAIR) {
    const int64_t pc = col - 2 * par;   // the even lane's column: the pair's first
    pa.base = ra.base;
    pa.ld = ra.ld;
    pa.pcol = (uint32_t)(pc < w.n - 4 ? pc : w.n - 4);
    pa.lane_off = (uint32_t)(8 * gq + par) * pa.ld + pa.pcol;
    pa.nrows = ra.nrows;
  }
  uint32_t ccol[NV];   // unaligned inputs: the lane's columns, clamped into the matrix
#pragma unroll
  for (int v = 0; v < NV; ++v) ccol[v] = (uint32_t)(col + v < w.n ? col + v : w.n - 1);
  Row<NV> raw[PAIR ? 1 : D][8];
  v4f rawp[PAIR ? D : 1][4];
  v4u pst[D][CPW];
  v8bf b[NV];
  auto issue = [&](int set, int64_t t) {   // t < nsteps; every load is unconditional (see above)
    if constexpr (PAIR) load_pair_step<CLAMP>(pa, kStep * t, gq, par, rawp[set]);
    else if constexpr (VEC) load_step<NV, VEC, CLAMP>(w, ra, kStep * t, gq, lcol, raw[set]);
    else load_step_clamped<NV>(ra, kStep * t, gq, ccol, raw[set]);
    const v4u *src = pi + (blk0 + t) * fstride;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int i = wave + W * j;
      pst[set][j] = src[(i < mv ? i : mv - 1) * kPiUnit];
    }
  };
  auto land = [&](int set, int64_t t) {   // step t's loads: Pi into LDS buffer `set`, rows into b
    const bool valid = t < nsteps;
    v4u *Ld = L + set * (LT * kPiUnit);
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int i = wave + W * j;   // tiles mv .. LT-1 get zeros (the padding m-tiles stay zero)
      Ld[i * kPiUnit + lane] = (valid && i < mv) ? pst[set][j] : v4u{0u, 0u, 0u, 0u};
    }
    if constexpr (PAIR) {
      Row<NV> x[8];
      unpack_pair_step(rawp[set], par, x);
      finish_rows_if<NV, NORM, CLAMP>(x, w.lbeg + kStep * t + 8 * gq, row_last, valid, b, ksum, kcmp);
    } else {
      finish_rows_if<NV, NORM, CLAMP>(raw[set], w.lbeg + kStep * t + 8 * gq, row_last, valid, b, ksum, kcmp);
    }
  };

#pragma unroll
  for (int d = 0; d < D; ++d) issue(d, d < nsteps ? d : nsteps - 1);
  land(0, 0);
  for (int64_t t0 = 0; t0 < nsteps; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int64_t t = t0 + d;
      __syncthreads();   // step t's fragments are in LDS; buffer (t + 1) % D is no longer read
      issue(d, t + D < nsteps ? t + D : nsteps - 1);
      __builtin_amdgcn_sched_barrier(0);
      mfma_step_stored<MT, NV, G>(b, L + d * (LT * kPiUnit), lane, acc);
      __builtin_amdgcn_sched_barrier(0);
      land((d + 1) % D, t + 1);
    }
  }
}

template <int MT, int NV, int G, int W, int D, bool VEC, bool CLAMP, bool PAIRED>
__global__ __launch_bounds__(64 * W) void sketch_bf16_stored_kernel(SkArgs g) {
  constexpr int LT = (MT + W - 1) / W * W;
  __shared__ __attribute__((aligned(16))) v4u L[D * LT * kPiUnit];

  SkWork w;
  if (!sk_decode(g, w)) return;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int q = lane & 15, gq = lane >> 4;
  // the lane's NV columns (paired loads: lanes q and q + 8 own columns 4q .. 4q + 3 of the wave's 32)
  constexpr bool PAIR = VEC && NV == 2 && PAIRED;
  const int64_t col = (int64_t)w.tile * (16 * W * NV) + wave * (16 * NV) + (PAIR ? (q & 7) * 4 + (q >> 3) * 2 : q * NV);
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
    if (w.kc == 0) loop_bf16_stored<MT, NV, G, W, D, VEC, CLAMP, true, PAIRED>(g, w, col, i0, mv, L, acc, ksum, kcmp);
    else loop_bf16_stored<MT, NV, G, W, D, VEC, CLAMP, false, PAIRED>(g, w, col, i0, mv, L, acc, ksum, kcmp);
  }
  sk_epilogue<MT, NV>(g, w, col, i0 * 16, gq, acc, ksum, kcmp);
}

// t, tc: vector loads (paired 16-byte loads at nv = 2), whole blocks and
// clamped; t2, tc2: one nv-wide vector load per row (inputs aligned to nv but
// not to 4 elements); ts: guarded scalar loads.
template <int NV, int G, int W, int D, int MT, int MT0>
struct KTabS {
  static void fill(KernelPtr *t, KernelPtr *tc, KernelPtr *ts, KernelPtr *t2, KernelPtr *tc2) {
    t[MT] = sketch_bf16_stored_kernel<MT, NV, G, W, D, true, false, true>;
    tc[MT] = sketch_bf16_stored_kernel<MT, NV, G, W, D, true, true, true>;
    ts[MT] = sketch_bf16_stored_kernel<MT, NV, G, W, D, false, true, true>;
    if constexpr (NV == 2) {
      t2[MT] = sketch_bf16_stored_kernel<MT, NV, G, W, D, true, false, false>;
      tc2[MT] = sketch_bf16_stored_kernel<MT, NV, G, W, D, true, true, false>;
    }
    KTabS<NV, G, W, D, MT - 1, MT0>::fill(t, tc, ts, t2, tc2);
  }
};
template <int NV, int G, int W, int D, int MT0>
struct KTabS<NV, G, W, D, MT0, MT0> {
  static void fill(KernelPtr *, KernelPtr *, KernelPtr *, KernelPtr *, KernelPtr *) {}
};

struct ShapeS {
  int nv, waves, depth, max_mt;
  KernelPtr t[33], tc[33], ts[33], t2[33], tc2[33];
};

ShapeS *shapes_stored(int &count) {
  // nv 2, 8 waves (two per SIMD), up to 16 m-tiles: 256 columns x 256 sketch
  // rows, 242 VGPRs at 16 m-tiles
  static ShapeS tabs[] = {{2, 8, 2, 16, {}, {}, {}, {}, {}}};
  static const bool init = [] {
    KTabS<2, 2, 8, 2, 16, 0>::fill(tabs[0].t, tabs[0].tc, tabs[0].ts, tabs[0].t2, tabs[0].tc2);
    return true;
  }();
  (void)init;
  count = (int)(sizeof(tabs) / sizeof(tabs[0]));
  return tabs;
}

KernelPtr bf16_stored_kernel_for(int nv, int waves, int depth, int mt, int variant) {
  int count = 0;
  ShapeS *t = shapes_stored(count);
  for (int i = 0; i < count; ++i)
    if (t[i].nv == nv && t[i].waves == waves && t[i].depth == depth && mt >= 1 && mt <= t[i].max_mt && t[i].t[mt])
      return variant == 0   ? t[i].t[mt]
             : variant == 1 ? t[i].tc[mt]
             : variant == 2 ? t[i].ts[mt]
             : variant == 3 ? t[i].t2[mt]
                            : t[i].tc2[mt];
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
static SketchPlan sketch_plan_bf16_regen(int k) {
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

// Stored-Pi plan: tiles of 16 * waves * nv columns, at most `cap` m-tiles per
// workgroup, `depth` K steps of loads in flight.
// SMP_SKETCH_BF16_STORED="nv,waves,depth,cap" picks the shape, "0" selects
// the regenerating pass above.
SketchPlan sketch_plan_bf16(int k, int cap_in) {
  // up to 16 m-tiles per chunk: at k = 1,024 every data tile is read by 4
  // chunks instead of 5 with 13 (22.8 -> 19.8 ms at d = 10^6, n = 8,192);
  // one wave per SIMD with the accumulators in AGPRs (nv 4, 4 waves) was
  // slower (21.7 ms): it spills and leaves less latency hidden
  int nv = 2, waves = 8, depth = 2, cap = cap_in >= 1 && cap_in <= 16 ? cap_in : 16;
  if (const char *e = getenv("SMP_SKETCH_BF16_STORED")) {
    int env[4] = {0, 0, 0, 0};
    const int got = sscanf(e, "%d,%d,%d,%d", &env[0], &env[1], &env[2], &env[3]);
    if (got == 1 && env[0] == 0) return sketch_plan_bf16_regen(k);
    if (got == 4 && bf16_stored_kernel_for(env[0], env[1], env[2], env[3], 0)) {
      nv = env[0];
      waves = env[1];
      depth = env[2];
      cap = env[3];
    }
  }
  SketchPlan p{};
  p.prec = SMP_PREC_BF16;
  p.pi_stored = 1;
  p.pi_rows = kStep;
  p.pi_frag_bytes = kPiUnit * 16;
  p.mt_total = (k + 15) / 16;
  p.nv = nv;
  p.vec_elems = nv == 2 ? 4 : nv;   // nv 2 loads 16 bytes per lane (paired rows)
  p.waves = waves;
  p.kc = kStep;
  p.kt = (p.mt_total + cap - 1) / cap;
  p.mt = (p.mt_total + p.kt - 1) / p.kt;
  p.ncol_tile = 16 * waves * nv;
  p.kpad = p.mt_total * 16;
  p.kernel = reinterpret_cast<void *>(bf16_stored_kernel_for(nv, waves, depth, p.mt, 0));
  p.kernel_clamp = reinterpret_cast<void *>(bf16_stored_kernel_for(nv, waves, depth, p.mt, 1));
  p.kernel_scalar = reinterpret_cast<void *>(bf16_stored_kernel_for(nv, waves, depth, p.mt, 2));
  if (p.vec_elems > nv) {
    p.kernel_v2 = reinterpret_cast<void *>(bf16_stored_kernel_for(nv, waves, depth, p.mt, 3));
    p.kernel_v2_clamp = reinterpret_cast<void *>(bf16_stored_kernel_for(nv, waves, depth, p.mt, 4));
  }
  return p;
}

// ---- grouped sketch of many jobs ---------------------------------------------
// Each job: its own regenerating BF16 plan, S splits of at least 64 whole
// blocks each (at most 16), a main launch over the whole blocks and a tail
// launch (one split, clamped) over the rest into partial slot S, exactly as a
// pass of its own would run them; the grouping only puts the jobs whose
// launches use the same kernel into one launch.
namespace {
struct GroupJobShape {
  SketchPlan pl;
  int S;
  int64_t n2e;   // B's columns in the pass (0 for B = A)
  size_t part_bytes, npart_bytes;
};
size_t al256(size_t b) { return (b + 255) / 256 * 256; }
GroupJobShape group_job_shape(const GroupSketchJob &j) {
  GroupJobShape s;
  s.pl = sketch_plan_bf16_regen(j.k);
  const int64_t nblk = j.d / s.pl.kc;
  s.S = (int)std::max<int64_t>(1, std::min<int64_t>(16, nblk / 64));
  s.n2e = j.B ? j.n2 : 0;
  const int64_t nt = j.n1 + s.n2e;
  s.part_bytes = al256((size_t)(s.S + 1) * nt * s.pl.kpad * 4);
  s.npart_bytes = al256((size_t)(s.S + 1) * nt * 8);
  return s;
}
}  // namespace

size_t bf16_group_scratch_bytes(const GroupSketchJob *jobs, int njobs) {
  size_t b = al256((size_t)2 * std::max(njobs, 1) * sizeof(SkJob));
  for (int i = 0; i < njobs; ++i) {
    const GroupJobShape s = group_job_shape(jobs[i]);
    b += s.part_bytes + s.npart_bytes;
  }
  return b;
}

hipError_t bf16_sketch_group(const GroupSketchJob *jobs, int njobs, void *scratch, size_t scratch_bytes,
                             hipStream_t st) {
  if (njobs <= 0) return hipSuccess;
  if (njobs > 65535 || !scratch || scratch_bytes < bf16_group_scratch_bytes(jobs, njobs)) return hipErrorInvalidValue;
  char *cb = static_cast<char *>(scratch);
  SkJob *dtab = reinterpret_cast<SkJob *>(cb);
  size_t off = al256((size_t)2 * njobs * sizeof(SkJob));
  auto aligned = [](const float *X, int64_t ld, int64_t n, int e) {
    const int vb = 4 * e;
    return ld % e == 0 && n % e == 0 && ((uintptr_t)X % (vb > 16 ? 16 : vb)) == 0;
  };
  std::vector<SkJob> tab(2 * (size_t)njobs);   // main launches, then tail launches
  std::vector<GroupKernelPtr> kern(2 * (size_t)njobs);
  std::vector<GroupJobShape> shape(njobs);
  std::vector<float *> parts(njobs);
  std::vector<double *> nparts(njobs);
  for (int i = 0; i < njobs; ++i) {
    const GroupSketchJob &j = jobs[i];
    const GroupJobShape sh = group_job_shape(j);
    shape[i] = sh;
    const SketchPlan &pl = sh.pl;
    parts[i] = reinterpret_cast<float *>(cb + off);
    nparts[i] = reinterpret_cast<double *>(cb + off + sh.part_bytes);
    off += sh.part_bytes + sh.npart_bytes;
    const int nct = pl.ncol_tile;
    SkArgs g{};
    g.a = SkMat{j.A, j.lda, j.n1, 0, (int)((j.n1 + nct - 1) / nct), (int)aligned(j.A, j.lda, j.n1, pl.nv)};
    g.b = j.B ? SkMat{j.B, j.ldb, j.n2, j.n1, (int)((j.n2 + nct - 1) / nct), (int)aligned(j.B, j.ldb, j.n2, pl.nv)}
              : SkMat{nullptr, 0, 0, j.n1, 0, 1};
    g.ntot = j.n1 + sh.n2e;
    g.k = j.k;
    g.kpad = pl.kpad;
    g.kt = pl.kt;
    g.mt_total = pl.mt_total;
    g.accumulate = 0;
    g.seed = j.seed;
    g.part = parts[i];
    g.npart = nparts[i];
    const bool vec = g.a.vec_ok && g.b.vec_ok;
    const int64_t nblk = j.d / pl.kc, main_rows = nblk * pl.kc, tail = j.d - main_rows;
    // main launch: the whole blocks over S splits (with no whole block it still stores zero partials)
    SkJob m{g, 0};
    m.g.row0 = 0;
    m.g.rows = main_rows;
    m.g.S = sh.S;
    m.g.rows_per_split = nblk / sh.S * pl.kc;
    m.g.split_extra = (int)(nblk % sh.S);
    m.g.split_unit = pl.kc;
    m.g.s_base = 0;
    m.grid = (int)(((int64_t)pl.kt * (g.a.ntiles + g.b.ntiles) * sh.S + 7) / 8 * 8);
    // tail launch: the rows past the last whole block, one split, into slot S
    SkJob t{g, 0};
    t.g.row0 = main_rows;
    t.g.rows = tail;
    t.g.S = 1;
    t.g.rows_per_split = (tail + pl.kc - 1) / pl.kc * pl.kc;
    t.g.split_extra = 0;
    t.g.split_unit = 0;
    t.g.s_base = sh.S;
    t.g.a.X = j.A + main_rows * j.lda;
    if (j.B) t.g.b.X = j.B + main_rows * j.ldb;
    t.grid = (int)(((int64_t)pl.kt * (g.a.ntiles + g.b.ntiles) + 7) / 8 * 8);
    kern[i] = bf16_group_kernel_for(pl.nv, pl.mt, pl.waves, 4, vec ? 0 : 2);
    kern[njobs + i] = bf16_group_kernel_for(pl.nv, pl.mt, pl.waves, 4, vec ? 1 : 2);
    if (!kern[i] || !kern[njobs + i] || pl.waves != 8) return hipErrorInvalidValue;
    tab[i] = m;
    tab[njobs + i] = t;
  }
  // order each half of the table by kernel, so that a launch's jobs are contiguous
  std::vector<int> order(2 * (size_t)njobs);
  for (int i = 0; i < 2 * njobs; ++i) order[i] = i;
  auto by_kernel = [&](int a, int b) {
    const bool ta = a >= njobs, tb = b >= njobs;
    if (ta != tb) return tb;   // main launches first
    if (kern[a] != kern[b]) return std::less<const void *>()(reinterpret_cast<const void *>(kern[a]),
                                                            reinterpret_cast<const void *>(kern[b]));
    return a < b;
  };
  std::sort(order.begin(), order.end(), by_kernel);
  std::vector<SkJob> sorted(2 * (size_t)njobs);
  for (int i = 0; i < 2 * njobs; ++i) sorted[i] = tab[order[i]];
  hipError_t e = hipMemcpyAsync(dtab, sorted.data(), sorted.size() * sizeof(SkJob), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;   // the host table is freed on return
  for (int i0 = 0; i0 < 2 * njobs;) {
    int i1 = i0 + 1;
    while (i1 < 2 * njobs && (order[i1] >= njobs) == (order[i0] >= njobs) && kern[order[i1]] == kern[order[i0]]) ++i1;
    int gx = 8;
    for (int i = i0; i < i1; ++i) gx = std::max(gx, sorted[i].grid);
    hipLaunchKernelGGL(kern[order[i0]], dim3((unsigned)gx, (unsigned)(i1 - i0)), dim3(64 * 8), 0, st,
                       static_cast<const SkJob *>(dtab + i0));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    i0 = i1;
  }
  for (int i = 0; i < njobs; ++i) {
    const GroupSketchJob &j = jobs[i];
    const GroupJobShape &sh = shape[i];
    if ((e = sketch_finish(sh.pl, parts[i], nparts[i], sh.S + 1, j.n1, sh.n2e, j.k, j.At, j.B ? j.Bt : nullptr,
                           j.na2, j.B ? j.nb2 : nullptr, st)) != hipSuccess)
      return e;
    if (!j.B) {
      if (j.Bt && j.Bt != j.At &&
          (e = hipMemcpyAsync(j.Bt, j.At, (size_t)j.n1 * j.k * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return e;
      if (j.nb2 && j.nb2 != j.na2 &&
          (e = hipMemcpyAsync(j.nb2, j.na2, (size_t)j.n1 * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return e;
    }
  }
  return hipSuccess;
}

hipError_t pi_store_bf16(const SketchPlan &pl, uint64_t seed, int64_t r0, int64_t rows, int k, void *buf,
                         hipStream_t st) {
  const int64_t frags = (rows + kStep - 1) / kStep * pl.mt_total;
  const int64_t grid = (frags * 16 + 255) / 256;
  hipLaunchKernelGGL(pi_store_bf16_kernel, dim3((unsigned)grid), dim3(256), 0, st, seed, r0, rows, k, pl.mt_total,
                     frags, static_cast<v4u *>(buf));
  return hipGetLastError();
}

}  // namespace smp

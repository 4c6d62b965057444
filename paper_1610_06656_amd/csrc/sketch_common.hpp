// Pieces shared by the FP32, BF16 and FP8 sketch kernels (Alg. 1 step 2): the
// launch arguments, the XCD-aware work decode, the data-row loads and the
// split-K epilogue.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smp {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));

struct SkMat {
  const float *X;
  int64_t ld, n, col_base;
  int ntiles, vec_ok;
};

struct SkArgs {
  SkMat a, b;
  int64_t row0, rows, rows_per_split, ntot;
  int k, kpad, kt, mt_total, S;
  int split_extra;  // splits 0 .. split_extra-1 hold split_unit rows more than rows_per_split
  int split_unit;
  int s_base;       // partial slot of split 0
  int accumulate;   // 1: add into the partials (streaming pushes); 0: store them (one-shot pass)
  uint64_t seed;
  const void *pi;   // stored-Pi passes: the fragments of the launch's first 32-row block (else null)
  // FP8 fragment pass: the data as MFMA B operands (2 KiB per 128-row block and
  // 16-column n-tile, blocks from the launch's first row), their E8M0 scales
  // (64 B per block and n-tile) and the n-tile counts (A's, then B's)
  const void *dfrag;
  const uint8_t *dscale;
  int nt16, ntA16;
  float *part;      // [S][ntot][kpad]
  double *npart;    // [S][ntot]
};

// One workgroup's share of the pass.
struct SkWork {
  const float *X;
  int64_t ld, n, col_base;
  bool vec_ok;
  int tile;   // column tile within its matrix
  int kc;     // sketch-row chunk
  int s;      // row split
  int64_t lbeg, lend;
};

// Workgroup b of a grid whose size is a multiple of 8 runs on XCD b % 8. The
// logical id keeps consecutive ids on one XCD, and the kt workgroups that
// read the same data tile (same column tile and split, different sketch-row
// chunk) have consecutive logical ids, so their reads of that tile meet in the
// XCD's L2. Returns false for the padding workgroups. sk_decode_in decodes
// workgroup b of a grid of nb (a multiple of 8) given explicitly (a job of a
// grouped launch), sk_decode the launch's own.
__device__ __forceinline__ bool sk_decode_in(const SkArgs &g, SkWork &w, int b, int nb) {
  const int logical = (b & 7) * (nb >> 3) + (b >> 3);
  const int ntl = g.a.ntiles + g.b.ntiles;
  if (logical >= g.kt * ntl * g.S) return false;
  w.kc = logical % g.kt;
  const int rest = logical / g.kt;
  int tile = rest % ntl;
  w.s = rest / ntl;
  const bool isb = tile >= g.a.ntiles;
  if (isb) tile -= g.a.ntiles;
  w.tile = tile;
  const SkMat &m = isb ? g.b : g.a;
  w.X = m.X;
  w.ld = m.ld;
  w.n = m.n;
  w.col_base = m.col_base;
  w.vec_ok = m.vec_ok != 0;
  const int longer = w.s < g.split_extra;
  w.lbeg = (int64_t)w.s * g.rows_per_split + (int64_t)(longer ? w.s : g.split_extra) * g.split_unit;
  const int64_t span = g.rows_per_split + (longer ? g.split_unit : 0);
  w.lend = w.lbeg + span < g.rows ? w.lbeg + span : g.rows;
  return true;
}

__device__ __forceinline__ bool sk_decode(const SkArgs &g, SkWork &w) {
  return sk_decode_in(g, w, (int)blockIdx.x, (int)gridDim.x);
}

// One job of a grouped launch: its arguments and the grid of a launch of its
// own (a multiple of 8).
struct SkJob {
  SkArgs g;
  int grid;
};

// NV adjacent columns of one data row into registers. FULL: the whole tile is
// inside the matrix and the vector loads are aligned, so the load is
// unconditional: a row past row_last reads row_last again, and the caller
// gives such rows a zero Pi entry and leaves them out of the norms (zeroing
// the loaded values here would make every load wait for its data at once).
// Otherwise each element is loaded only when inside the matrix (else 0).
// NT marks the loads nontemporal (streamed past the caches).
template <int NV, bool FULL, bool NT = false>
__device__ __forceinline__ void sk_load_row(const float *X, int64_t ld, int64_t n, int64_t row, int64_t row_last,
                                            int64_t col, float (&out)[NV]) {
  const bool row_ok = row <= row_last;
  if constexpr (FULL) {
    const float *p = X + (row_ok ? row : row_last) * ld + col;
    if constexpr (NV == 2) {
      const v2f t = NT ? __builtin_nontemporal_load(reinterpret_cast<const v2f *>(p)) : *reinterpret_cast<const v2f *>(p);
      out[0] = t[0];
      out[1] = t[1];
    } else {
#pragma unroll
      for (int h = 0; h < NV / 4; ++h) {
        const v4f t = NT ? __builtin_nontemporal_load(reinterpret_cast<const v4f *>(p) + h)
                         : *(reinterpret_cast<const v4f *>(p) + h);
        out[4 * h + 0] = t[0];
        out[4 * h + 1] = t[1];
        out[4 * h + 2] = t[2];
        out[4 * h + 3] = t[3];
      }
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = 0.0f;
    if (!row_ok || col >= n) return;
    const float *p = X + row * ld + col;
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (col + v < n) out[v] = p[v];
  }
}

// Compensated (Kahan) accumulation of one FP32 term.
__device__ __forceinline__ void kahan_add(float &sum, float &comp, float term) {
  const float y = term - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

// Split-K epilogue. acc[i][v] holds, in lane (q, ph), the sketch rows
// c0 + 16 i + 4 ph + (0..3) of data column col + v (the 16x16 MFMA output
// layout). Partial norms come from the sketch-row chunk 0 workgroup only.
// Column v of the lane is col + VS * v. NORMS = false leaves the norm
// partials alone (a pass whose norms come from elsewhere).
template <int MT, int NV, int VS = 1, bool NORMS = true>
__device__ __forceinline__ void sk_epilogue(const SkArgs &g, const SkWork &w, int64_t col, int c0, int ph,
                                            const v4f (&acc)[MT][NV], const float (&ksum)[NV],
                                            const float (&kcmp)[NV]) {
  const int mt0 = c0 / 16;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double nrm = (double)ksum[v] - (double)kcmp[v];
    nrm += __shfl_xor(nrm, 16, 64);
    nrm += __shfl_xor(nrm, 32, 64);
    const int64_t c_ = col + VS * v;
    if (NORMS && c_ < w.n && ph == 0 && w.kc == 0) {
      double *dst = g.npart + (int64_t)(g.s_base + w.s) * g.ntot + w.col_base + c_;
      *dst = g.accumulate ? *dst + nrm : nrm;
    }
  }
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    if (mt0 + i < g.mt_total) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int64_t c_ = col + VS * v;
        if (c_ < w.n) {
          float *dst = g.part + ((int64_t)(g.s_base + w.s) * g.ntot + w.col_base + c_) * g.kpad + c0 + 16 * i + 4 * ph;
          float4 val = make_float4(acc[i][v][0], acc[i][v][1], acc[i][v][2], acc[i][v][3]);
          if (g.accumulate) {
            const float4 old = *reinterpret_cast<float4 *>(dst);
            val.x += old.x;
            val.y += old.y;
            val.z += old.z;
            val.w += old.w;
          }
          *reinterpret_cast<float4 *>(dst) = val;
        }
      }
    }
  }
}

}  // namespace smp

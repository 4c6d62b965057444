// Device-side building blocks for the SMP-PCA kernels (gfx950, wave64).
//
// * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): the counter-based
//   generator behind every random draw of the method: the Gaussian sketching
//   matrix Pi of Alg. 1 step 2 and the entry coins of Alg. 1 step 3.
// * Box-Muller (1958) from two 24-bit uniforms.
// * wave64 reductions.
//
// Stream layout ("counter spec"): key = (seed mod 2^32, seed >> 32); the
// counter of a call is (col_block, row mod 2^32, tag, row >> 32) and the call
// serves columns 4*col_block .. 4*col_block+3 of that row. Pi uses row = l (the
// d index) and col = c (the sketch row); the coins use row = i, col = j.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smp {

enum : uint32_t {
  kTagPi = 1, kTagSample = 2, kTagSplit = 3, kTagInit = 4,
  kTagSrhtSign = 7, kTagSrhtRow = 8   // the SRHT's signs sigma_l and Hadamard rows rho_c (row 0, column l or c)
};

struct u32x4 {
  uint32_t x, y, z, w;
};

// a ^ b ^ c in one instruction: gfx950's three-input bitwise op with the
// truth table 0x96 (the output bit is set when an odd number of inputs are).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// Ten Philox-4x32 rounds. Round r uses the key (k0 + r*0x9E3779B9, k1 + r*0xBB67AE85).
__device__ __forceinline__ u32x4 philox10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = u32x4{xor3(hi1, c.y, k0), lo1, xor3(hi0, c.w, k1), lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ u32x4 stream_call(uint64_t seed, uint32_t tag, uint64_t row, uint32_t col_block) {
  return philox10(u32x4{col_block, (uint32_t)row, tag, (uint32_t)(row >> 32)}, (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

// The word the counter spec assigns to (row, col): lane col mod 4 of the call
// (col / 4, row).
__device__ __forceinline__ uint32_t stream_word(uint64_t seed, uint32_t tag, uint64_t row, uint64_t col) {
  const u32x4 w = stream_call(seed, tag, row, (uint32_t)(col >> 2));
  const int u = (int)(col & 3);
  return u == 0 ? w.x : (u == 1 ? w.y : (u == 2 ? w.z : w.w));
}

// Box-Muller pair: u = ((a>>8)+1) 2^-24 in (0,1], phi = (b>>8) 2^-24 in [0,1),
// rad = sqrt(-2 ln u); returns rad*cos(2 pi phi), rad*sin(2 pi phi).
// Uses the hardware transcendentals: v_log_f32 (log2), v_sqrt_f32, and
// v_sin_f32 / v_cos_f32, whose argument is in revolutions, so phi is passed
// as is.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& zc, float& zs) {
  const float u = (float)((a >> 8) + 1u) * 0x1p-24f;
  const float phi = (float)(b >> 8) * 0x1p-24f;
  const float rad = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u));  // -2 ln 2 log2 u
  zc = rad * __builtin_amdgcn_cosf(phi);
  zs = rad * __builtin_amdgcn_sinf(phi);
}

// The four N(0,1) variates of one Philox call, in lane order 0..3.
__device__ __forceinline__ float4 normals4(u32x4 w) {
  float4 z;
  box_muller(w.x, w.y, z.x, z.y);
  box_muller(w.z, w.w, z.z, z.w);
  return z;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace smp

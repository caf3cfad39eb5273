// FP64 matrix-core helpers for gfx950 (v_mfma_f64_16x16x4_f64).
//
// Operand layout of one 16x16x4 step (wavefront of 64 lanes, l = lane id):
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[l / 16 + 4 * i][l % 16] in accumulator i = 0..3
#pragma once
#include <hip/hip_runtime.h>

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ inline f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline int lane_id() { return threadIdx.x & 63; }

// row of accumulator i held by lane l in a 16x16 f64 result tile
__device__ inline int mfma_row(int l, int i) { return (l >> 4) + 4 * i; }

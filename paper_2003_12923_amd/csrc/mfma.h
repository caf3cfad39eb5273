// Matrix-core helpers for gfx950: v_mfma_f64_16x16x4_f64 and
// v_mfma_f32_16x16x4_f32 (one 16x16 block, K = 4, one operand value per lane).
//
// Operand layout of one 16x16x4 step (wavefront of 64 lanes, l = lane id), both types:
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
// Result layout (accumulator i = 0..3 of lane l holds D[row][l % 16]):
//   f64: row = l / 16 + 4 i        f32: row = 4 (l / 16) + i
#pragma once
#include <hip/hip_runtime.h>

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline f32x4 mfma16x16x4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <class T> struct MfmaAcc;
template <> struct MfmaAcc<double> { typedef f64x4 type; };
template <> struct MfmaAcc<float> { typedef f32x4 type; };

__device__ inline int lane_id() { return threadIdx.x & 63; }

// row of accumulator i held by lane l in a 16x16 result tile
__device__ inline int mfma_row(int l, int i) { return (l >> 4) + 4 * i; }

template <class T> __device__ inline int mfma_row_t(int l, int i);
template <> __device__ inline int mfma_row_t<double>(int l, int i) { return (l >> 4) + 4 * i; }
template <> __device__ inline int mfma_row_t<float>(int l, int i) { return 4 * (l >> 4) + i; }

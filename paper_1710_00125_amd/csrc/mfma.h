// Matrix-core helpers for gfx950: V_MFMA_F64_16X16X4_F64,
// V_MFMA_F32_16X16X4_F32 and V_MFMA_F32_16X16X32_BF16.
//
// Operand layouts of one 16 x 16 x K step (64 lanes):
//   A fragment (16 x K): lane l holds A(l % 16, k) for the k of group l / 16
//   B fragment (K x 16): lane l holds B(k, l % 16) for the same k group
//   C/D (16 x 16), element v of lane l:
//     FP64:          C(l / 16 + 4 v, l % 16)
//     FP32 and BF16: C(4 (l / 16) + v, l % 16)
// For K = 4 the k of lane l is l / 16; for the BF16 step (K = 32) lane l
// holds the eight consecutive k = 8 (l / 16) + e.  The accumulator layouts
// were established with probes on the hardware.
#pragma once

#include <hip/hip_runtime.h>

typedef double rcp_d4 __attribute__((ext_vector_type(4)));
typedef float rcp_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 rcp_bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ rcp_d4 mfma16x16x4(double a, double b, rcp_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ rcp_f4 mfma16x16x4(float a, float b, rcp_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ rcp_f4 mfma16x16x32(rcp_bf8 a, rcp_bf8 b, rcp_f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int frag_row(int lane) { return lane & 15; }   // A: row
__device__ __forceinline__ int frag_k(int lane) { return lane >> 4; }     // A, B: k (K = 4)
__device__ __forceinline__ int frag_col(int lane) { return lane & 15; }   // B: column
__device__ __forceinline__ int acc_row(int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ int acc_row_f32(int lane, int v) { return 4 * (lane >> 4) + v; }
__device__ __forceinline__ int acc_col(int lane) { return lane & 15; }

// accumulator type and row map by element type
template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  typedef rcp_d4 type;
  static __device__ __forceinline__ int row(int lane, int v) { return acc_row(lane, v); }
};
template <>
struct MfmaAcc<float> {
  typedef rcp_f4 type;
  static __device__ __forceinline__ int row(int lane, int v) { return acc_row_f32(lane, v); }
};

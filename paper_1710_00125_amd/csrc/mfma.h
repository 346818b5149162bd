// FP64 matrix-core helpers: V_MFMA_F64_16X16X4_F64 on gfx950.
//
// Operand layouts of one 16x16x4 step (64 lanes):
//   A fragment (16 x 4): lane l holds A(l % 16, l / 16)
//   B fragment (4 x 16): lane l holds B(l / 16, l % 16)
//   C/D (16 x 16):       lane l, element v holds C(l / 16 + 4 v, l % 16)
// (the accumulator layout was established with a probe on the hardware)
#pragma once

#include <hip/hip_runtime.h>

typedef double rcp_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ rcp_d4 mfma16x16x4(double a, double b, rcp_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int frag_row(int lane) { return lane & 15; }   // A: row
__device__ __forceinline__ int frag_k(int lane) { return lane >> 4; }     // A, B: k
__device__ __forceinline__ int frag_col(int lane) { return lane & 15; }   // B: column
__device__ __forceinline__ int acc_row(int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ __forceinline__ int acc_col(int lane) { return lane & 15; }

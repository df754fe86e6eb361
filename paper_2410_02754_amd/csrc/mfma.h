// MFMA wrappers and accumulator layout of the gfx950 16x16x4 matrix instructions
// shared by the cell, Gram and rotation kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace chfsi {


typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <class T> struct Vec4;
template <> struct Vec4<double> { typedef d4 type; };
template <> struct Vec4<float> { typedef f4 type; };

// Row (within the 16x16 tile) of accumulator element j held by `lane`; the
// column is lane % 16.  The two 16x16x4 MFMAs distribute rows differently on
// gfx950: FP32 gives lane/16 groups of four consecutive rows, FP64 interleaves
// (row = lane/16 + 4 j).  Verified on the device with known operands.
template <class T> __device__ __forceinline__ int acc_row(int lane, int j);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int j) { return 4 * (lane >> 4) + j; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int j) { return (lane >> 4) + 4 * j; }

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

#define LAUNCH_CHECK() CHFSI_HIP(hipGetLastError())

}  // namespace chfsi

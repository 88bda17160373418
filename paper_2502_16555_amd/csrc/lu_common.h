// Device helpers shared by the LU kernels: MFMA tile conventions, XCD-aware
// block mapping and 16-byte vector types.  Each translation unit gets its own
// copies (internal linkage).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace bte {
namespace {

using f64x4 = double __attribute__((ext_vector_type(4)));
using f32x4 = float __attribute__((ext_vector_type(4)));

constexpr int kXcd = 8;  // XCDs of an MI355X; workgroups are dealt to them round-robin

// MFMA 16x16x4 tiles: operand lanes hold A[i = lane%16][k = lane/16] and
// B[k = lane/16][j = lane%16]; result item t of lane l holds D[row(l, t)][l%16]
// with row = 4*(l/16) + t for f32 and row = l/16 + 4*t for f64 (measured).
template <typename T>
struct Mma;
template <>
struct Mma<double> {
  using acc = f64x4;
  __device__ static inline acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int t) { return lk + 4 * t; }
};
template <>
struct Mma<float> {
  using acc = f32x4;
  __device__ static inline acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int t) { return 4 * lk + t; }
};

// Block id -> (matrix, item) such that all items of a matrix run on one XCD.
__device__ inline void xcd_map(int bid, int items, int nmat, int* mat, int* item) {
  const int xcd = bid % kXcd, j = bid / kXcd;
  *mat = xcd + kXcd * (j / items);
  *item = j % items;
}

inline int xcd_grid(int items, int nmat) { return kXcd * items * ((nmat + kXcd - 1) / kXcd); }

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  using type = float4;
  static constexpr int per = 4;
};
template <>
struct Vec4<double> {
  using type = double2;
  static constexpr int per = 2;
};
// FP16 storage of factors that only precondition (the Krylov solver's bins)
using half8 = _Float16 __attribute__((ext_vector_type(8)));
template <>
struct Vec4<_Float16> {
  using type = half8;
  static constexpr int per = 8;
};

}  // namespace
}  // namespace bte

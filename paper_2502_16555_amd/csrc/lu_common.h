// Device helpers shared by the LU kernels: MFMA tile conventions, XCD-aware
// block mapping and 16-byte vector types.  Each translation unit gets its own
// copies (internal linkage).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "internal.h"

namespace bte {
namespace {

using f64x4 = double __attribute__((ext_vector_type(4)));
using f32x4 = float __attribute__((ext_vector_type(4)));
using f64x2 = double __attribute__((ext_vector_type(2)));

constexpr int kXcd = 8;  // XCDs of an MI355X; workgroups are dealt to them round-robin

// Non-temporal 16-byte load of data read once (the solves' factors, a
// trailing update's old tile), so that it does not displace what is reused.
template <typename V>
__device__ inline V ntload(const V* p) {
  using I = int __attribute__((ext_vector_type(sizeof(V) / 4)));
  return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const I*>(p)));
}

// f(integral_constant<int, I>) for I in the sequence, in order: loop bodies
// whose indices must be compile-time constants (register arrays, unrolled
// steps) without relying on the unroller
template <int... I, class F>
__device__ __forceinline__ void static_for(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}

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

// Wavefront reductions through DPP lane permutations (quad swaps, half-row and
// row mirrors) inside each row of 16 lanes, then the four row results by lane
// reads: no LDS round trip on the pivot search's critical path.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(b), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
__device__ inline double readlane_f64(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
// maximum over the wavefront of values that are never NaN; uniform result
__device__ inline double wave_max(double v) {
  double o = dpp_f64<0xB1>(v);  // quad_perm [1,0,3,2]
  v = o > v ? o : v;
  o = dpp_f64<0x4E>(v);         // quad_perm [2,3,0,1]
  v = o > v ? o : v;
  o = dpp_f64<0x141>(v);        // row_half_mirror
  v = o > v ? o : v;
  o = dpp_f64<0x140>(v);        // row_mirror
  v = o > v ? o : v;
  const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16), r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
  const double m0 = r1 > r0 ? r1 : r0, m1 = r3 > r2 ? r3 : r2;
  return m1 > m0 ? m1 : m0;
}
// maximum over the wavefront of 64-bit unsigned keys; uniform result
template <int CTRL>
__device__ inline unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(v >> 32), CTRL, 0xF, 0xF, false);
  return (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) | static_cast<unsigned>(lo);
}
__device__ inline unsigned long long readlane_u64(unsigned long long v, int l) {
  const unsigned lo = __builtin_amdgcn_readlane(static_cast<int>(v), l);
  const unsigned hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), l);
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}
__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
  unsigned long long o = dpp_u64<0xB1>(v);
  v = o > v ? o : v;
  o = dpp_u64<0x4E>(v);
  v = o > v ? o : v;
  o = dpp_u64<0x141>(v);
  v = o > v ? o : v;
  o = dpp_u64<0x140>(v);
  v = o > v ? o : v;
  const unsigned long long r0 = readlane_u64(v, 0), r1 = readlane_u64(v, 16), r2 = readlane_u64(v, 32),
                           r3 = readlane_u64(v, 48);
  const unsigned long long m0 = r1 > r0 ? r1 : r0, m1 = r3 > r2 ? r3 : r2;
  return m1 > m0 ? m1 : m0;
}
__device__ inline int wave_min(int v) {
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

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

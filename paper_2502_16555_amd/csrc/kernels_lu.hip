// Velocity-space step V(dt): the Nx decoupled dense systems of
// eq. (vspace_batched_system),  (I - dt (n0 C + E_i A)) F*_i = F_i,  solved by a
// batched right-looking blocked LU factorization with partial pivoting.
//
// Storage: one row-major npad x npad matrix per collocation point (npad = n
// rounded up to the panel width, padded with identity).  Interchanges are
// applied "as you go": a panel's interchanges are applied to that panel and
// to the trailing columns only, so the solve applies P_1, L_1^-1, P_2, L_2^-1,
// ..., U^-1 in that order (A = P_1^T L_1 P_2^T L_2 ... U).
//
// Per panel k0 (width kNB):
//   k_panel      one 512-thread block per matrix: partial pivoting (max |a|,
//                ties to the lowest row), elimination of 8/16-column sub-panels
//                held in registers, in-panel updates of the remaining columns;
//   k_swap_trsm  interchanges + U12 = L11^-1 A12 on 64-column chunks;
//   k_update     A22 -= L21 U12 as a batched MFMA GEMM (64 x 64 tiles, K = kNB).
// Mixed precision (FP32 factors) refines in FP64: r = b - A x with A applied
// from the FP64 operators (the residual is the operator action of
// Alg. vspace_action), x += LU^-1 r, until max|r| <= rtol max|b|.
#include <climits>
#include <cmath>

#include "internal.h"

namespace bte {
namespace {

using f64x4 = double __attribute__((ext_vector_type(4)));
using f32x4 = float __attribute__((ext_vector_type(4)));

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

constexpr int kPermStride = 2 * kMaxSwapRows + 1;

// ---------------------------------------------------------------------------
// Matrix formation: LU[x] = I - dt (n0_x C + E_x A), identity on the padding.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_form(T* __restrict__ LU, const double* __restrict__ C,
                                              const double* __restrict__ Aop, const double* __restrict__ E,
                                              const double* __restrict__ n0x, const int* __restrict__ status,
                                              double dt, int n, int npad) {
  const int x = blockIdx.y;
  const int r = blockIdx.x;  // one block per row
  const double e = E[x], nn = n0x[x];
  T* row = LU + ((size_t)x * npad + r) * npad;
  if (r < n) {
    const double* cr = C + (size_t)r * n;
    const double* ar = Aop + (size_t)r * n;
    for (int c = threadIdx.x; c < npad; c += blockDim.x) {
      double v = (c < n) ? -dt * (nn * cr[c] + e * ar[c]) : 0.0;
      if (c == r) v += 1.0;
      row[c] = static_cast<T>(v);
    }
  } else {
    for (int c = threadIdx.x; c < npad; c += blockDim.x) row[c] = static_cast<T>(c == r ? 1.0 : 0.0);
  }
}

// ---------------------------------------------------------------------------
// Panel factorization (rows k0.., columns k0..k0+kNB-1), one block per matrix.
// ---------------------------------------------------------------------------
template <typename T, int RPT, int IB>
__global__ __launch_bounds__(kPanelThreads) void k_panel(T* __restrict__ LU, int* __restrict__ piv,
                                                         int* __restrict__ perm, int* __restrict__ status, int npad,
                                                         int k0) {
  constexpr int NW = kPanelThreads / 64;
  const int mat = blockIdx.x;
  T* A = LU + (size_t)mat * npad * npad;
  int* ip = piv + (size_t)mat * npad;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  __shared__ double s_val[NW];
  __shared__ int s_idx[NW];
  __shared__ int s_p;
  __shared__ T s_row[2][IB];
  __shared__ T s_L11[IB][IB + 1];
  __shared__ T s_U[IB][kNB];
  __shared__ int s_sw[IB];
  __shared__ int s_R[2 * IB];
  __shared__ int s_src[2 * IB];
  __shared__ int s_nR;
  __shared__ int s_any;
  __shared__ int s_lab[kMaxSwapRows];
  bool singular = false;

  for (int sp = 0; sp < kNB / IB; ++sp) {
    const int c0 = k0 + sp * IB;
    T a[RPT][IB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = c0 + tid + q * kPanelThreads;
#pragma unroll
      for (int j = 0; j < IB; ++j) a[q][j] = (r < npad) ? A[(size_t)r * npad + c0 + j] : T(0);
    }
#pragma clang loop unroll(full)
    for (int j = 0; j < IB; ++j) {
      const int c = c0 + j;
      double best = -1.0;
      int bi = INT_MAX;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = c0 + tid + q * kPanelThreads;
        if (r >= c && r < npad) {
          const double v = fabs(static_cast<double>(a[q][j]));
          if (v > best) {
            best = v;
            bi = r;
          }
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        s_val[wid] = best;
        s_idx[wid] = bi;
      }
      __syncthreads();
      if (wid == 0) {
        double v = (lane < NW) ? s_val[lane] : -1.0;
        int i = (lane < NW) ? s_idx[lane] : INT_MAX;
        for (int off = NW / 2; off > 0; off >>= 1) {
          const double ov = __shfl_xor(v, off);
          const int oi = __shfl_xor(i, off);
          if (ov > v || (ov == v && oi < i)) {
            v = ov;
            i = oi;
          }
        }
        if (lane == 0) s_p = i;
      }
      __syncthreads();
      const int p = s_p;
      // row c is owned by thread j (q = 0); exchange rows c and p through LDS
      if (tid == j) {
#pragma unroll
        for (int jj = 0; jj < IB; ++jj) s_row[0][jj] = a[0][jj];
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        if (c0 + tid + q * kPanelThreads == p) {
#pragma unroll
          for (int jj = 0; jj < IB; ++jj) s_row[1][jj] = a[q][jj];
        }
      }
      __syncthreads();
      if (p != c) {
        if (tid == j) {
#pragma unroll
          for (int jj = 0; jj < IB; ++jj) a[0][jj] = s_row[1][jj];
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          if (c0 + tid + q * kPanelThreads == p) {
#pragma unroll
            for (int jj = 0; jj < IB; ++jj) a[q][jj] = s_row[0][jj];
          }
        }
      }
      const T pv = s_row[1][j];
      if (tid == 0) {
        ip[c] = p;
        s_sw[j] = p;
      }
      if (pv == T(0)) singular = true;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = c0 + tid + q * kPanelThreads;
        if (r > c && r < npad && pv != T(0)) {
          const T l = a[q][j] / pv;
          a[q][j] = l;
#pragma unroll
          for (int jj = 0; jj < IB; ++jj)
            if (jj > j) a[q][jj] -= l * s_row[1][jj];
        }
      }
      __syncthreads();
    }
    // write the factored sub-panel back
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = c0 + tid + q * kPanelThreads;
      if (r < npad) {
#pragma unroll
        for (int j = 0; j < IB; ++j) A[(size_t)r * npad + c0 + j] = a[q][j];
      }
    }
    if (tid < IB) {
#pragma unroll
      for (int j = 0; j < IB; ++j) s_L11[tid][j] = a[0][j];
    }
    // permutation of the rows touched by this sub-panel's interchanges
    if (tid == 0) {
      int nR = IB, any = 0;
      int* lab = s_lab;
      for (int t = 0; t < IB; ++t) {
        s_R[t] = c0 + t;
        lab[t] = t;
      }
      for (int j = 0; j < IB; ++j) {
        const int p = s_sw[j];
        int ip2;
        if (p < c0 + IB) {
          ip2 = p - c0;
        } else {
          ip2 = -1;
          for (int t = IB; t < nR; ++t)
            if (s_R[t] == p) ip2 = t;
          if (ip2 < 0) {
            ip2 = nR;
            s_R[nR] = p;
            lab[nR] = nR;
            ++nR;
          }
        }
        if (ip2 != j) {
          any = 1;
          const int tmp = lab[j];
          lab[j] = lab[ip2];
          lab[ip2] = tmp;
        }
      }
      for (int t = 0; t < nR; ++t) s_src[t] = s_R[lab[t]];
      s_nR = nR;
      s_any = any;
    }
    __syncthreads();
    // apply the interchanges to the other columns of the panel (rows >= c0)
    if (s_any) {
      const int nR = s_nR;
      constexpr int NOC = kNB - IB;
      T vb[(NOC * 2 * IB + kPanelThreads - 1) / kPanelThreads];
#pragma unroll
      for (int u = 0; u < (NOC * 2 * IB + kPanelThreads - 1) / kPanelThreads; ++u) {
        const int e = tid + u * kPanelThreads;
        if (e < NOC * nR) {
          const int t = e / NOC, cc = e % NOC;
          const int col = (cc < sp * IB) ? k0 + cc : k0 + IB + cc;
          vb[u] = A[(size_t)s_src[t] * npad + col];
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < (NOC * 2 * IB + kPanelThreads - 1) / kPanelThreads; ++u) {
        const int e = tid + u * kPanelThreads;
        if (e < NOC * nR) {
          const int t = e / NOC, cc = e % NOC;
          const int col = (cc < sp * IB) ? k0 + cc : k0 + IB + cc;
          if (s_src[t] != s_R[t]) A[(size_t)s_R[t] * npad + col] = vb[u];
        }
      }
      __syncthreads();
    }
    // update the remaining columns of the panel
    const int nrest = k0 + kNB - c0 - IB;
    if (nrest > 0) {
      if (tid < nrest) {
        const int col = c0 + IB + tid;
        for (int j = 0; j < IB; ++j) s_U[j][tid] = A[(size_t)(c0 + j) * npad + col];
        for (int j = 1; j < IB; ++j) {
          T v = s_U[j][tid];
          for (int i = 0; i < j; ++i) v -= s_L11[j][i] * s_U[i][tid];
          s_U[j][tid] = v;
        }
        for (int j = 0; j < IB; ++j) A[(size_t)(c0 + j) * npad + col] = s_U[j][tid];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = c0 + tid + q * kPanelThreads;
        if (r >= c0 + IB && r < npad) {
          T* row = A + (size_t)r * npad + c0 + IB;
          for (int cc = 0; cc < nrest; ++cc) {
            T s = row[cc];
#pragma unroll
            for (int j = 0; j < IB; ++j) s -= a[q][j] * s_U[j][cc];
            row[cc] = s;
          }
        }
      }
      __syncthreads();
    }
  }
  if (singular && tid == 0) atomicOr(status, kStSingular);
  // permutation of the whole panel (for the trailing columns)
  if (tid == 0) {
    int* pm = perm + (size_t)mat * kPermStride;
    int* R = pm + 1;
    int* src = pm + 1 + kMaxSwapRows;
    int* lab = s_lab;
    int nR = kNB;
    for (int t = 0; t < kNB; ++t) {
      R[t] = k0 + t;
      lab[t] = t;
    }
    for (int j = 0; j < kNB; ++j) {
      const int p = ip[k0 + j];
      int i2;
      if (p < k0 + kNB) {
        i2 = p - k0;
      } else {
        i2 = -1;
        for (int t = kNB; t < nR; ++t)
          if (R[t] == p) i2 = t;
        if (i2 < 0) {
          i2 = nR;
          R[nR] = p;
          lab[nR] = nR;
          ++nR;
        }
      }
      const int tmp = lab[j];
      lab[j] = lab[i2];
      lab[i2] = tmp;
    }
    for (int t = 0; t < nR; ++t) src[t] = R[lab[t]];
    pm[0] = nR;
  }
}

// ---------------------------------------------------------------------------
// Interchanges and U12 = L11^-1 A12 for one 64-column chunk right of the panel.
// One wavefront per chunk; every lane owns one column (no cross-lane hazards).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void k_swap_trsm(T* __restrict__ LU, const int* __restrict__ perm, int npad, int k0) {
  const int mat = blockIdx.y;
  T* A = LU + (size_t)mat * npad * npad;
  const int col = k0 + kNB + blockIdx.x * 64 + threadIdx.x;
  const int* pm = perm + (size_t)mat * kPermStride;
  const int nR = pm[0];
  const int* R = pm + 1;
  const int* src = pm + 1 + kMaxSwapRows;
  __shared__ T sL[kNB][kNB + 1];
  __shared__ T sX[kNB][64];
  __shared__ T sE[kNB][64];
  for (int e = threadIdx.x; e < kNB * kNB; e += 64) {
    const int r = e / kNB, c = e % kNB;
    sL[r][c] = A[(size_t)(k0 + r) * npad + k0 + c];
  }
  const bool active = col < npad;
  if (active) {
    for (int t = 0; t < nR; ++t) {
      const T v = A[(size_t)src[t] * npad + col];
      if (t < kNB) sX[t][threadIdx.x] = v;
      else sE[t - kNB][threadIdx.x] = v;
    }
    for (int t = kNB; t < nR; ++t)
      if (src[t] != R[t]) A[(size_t)R[t] * npad + col] = sE[t - kNB][threadIdx.x];
  }
  __syncthreads();
  if (active) {
    for (int j = 1; j < kNB; ++j) {
      T s = sX[j][threadIdx.x];
      for (int i = 0; i < j; ++i) s -= sL[j][i] * sX[i][threadIdx.x];
      sX[j][threadIdx.x] = s;
    }
    for (int j = 0; j < kNB; ++j) A[(size_t)(k0 + j) * npad + col] = sX[j][threadIdx.x];
  }
}

// ---------------------------------------------------------------------------
// Trailing update A22 -= L21 U12, 64 x 64 output tiles, K = kNB, MFMA 16x16x4.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_update(T* __restrict__ LU, int npad, int k0) {
  const int mat = blockIdx.y;
  const int mt = (npad - k0 - kNB) / 64;
  const int ti = blockIdx.x / mt, tj = blockIdx.x % mt;
  T* A = LU + (size_t)mat * npad * npad;
  const int r0 = k0 + kNB + ti * 64, c0 = k0 + kNB + tj * 64;
  __shared__ T sA[64][kNB + 1];
  __shared__ T sB[kNB][64 + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB;
    sA[r][c] = A[(size_t)(r0 + r) * npad + k0 + c];
  }
  for (int e = tid; e < kNB * 64; e += 256) {
    const int r = e / 64, c = e % 64;
    sB[r][c] = A[(size_t)(k0 + r) * npad + c0 + c];
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  typename Mma<T>::acc acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = typename Mma<T>::acc{0, 0, 0, 0};
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 4
  for (int k = 0; k < kNB; k += 4) {
    T av[2], bv[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) av[bi] = sA[wr + bi * 16 + li][k + lk];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) bv[bj] = sB[k + lk][wc + bj * 16 + li];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = Mma<T>::step(av[bi], bv[bj], acc[bi][bj]);
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int r = r0 + wr + bi * 16 + Mma<T>::row(lk, it);
        const int c = c0 + wc + bj * 16 + li;
        T* p = A + (size_t)r * npad + c;
        *p = *p - acc[bi][bj][it];
      }
}

// ---------------------------------------------------------------------------
// Solve with the factors (one block per matrix), FP64 right-hand side.
// transpose = 0: x = U^-1 L_m^-1 P_m ... L_1^-1 P_1 b
// transpose = 1: y = P_1^T L_1^-T ... P_m^T L_m^-T U^-T c
// ---------------------------------------------------------------------------
template <typename T, int TRANSPOSE>
__global__ __launch_bounds__(256) void k_solve(const T* __restrict__ LU, const int* __restrict__ piv,
                                               const double* __restrict__ Bin, double* __restrict__ Xout,
                                               const int* __restrict__ status, int accumulate, int check_done,
                                               int npad) {
  if (check_done && status[1]) return;
  extern __shared__ double sb[];        // [npad] right-hand side / solution
  __shared__ double sT[kNB][kNB + 1];   // diagonal block
  __shared__ double sacc[4][kNB];
  const int mat = blockIdx.x;
  const T* A = LU + (size_t)mat * npad * npad;
  const int* ip = piv + (size_t)mat * npad;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double* b = Bin + (size_t)mat * npad;
  for (int i = tid; i < npad; i += 256) sb[i] = b[i];
  __syncthreads();
  const int np = npad / kNB;
  if (!TRANSPOSE) {
    for (int p = 0; p < np; ++p) {
      const int k0 = p * kNB;
      if (tid == 0) {
        for (int j = 0; j < kNB; ++j) {
          const int q = ip[k0 + j];
          if (q != k0 + j) {
            const double t = sb[k0 + j];
            sb[k0 + j] = sb[q];
            sb[q] = t;
          }
        }
      }
      for (int e = tid; e < kNB * kNB; e += 256) sT[e / kNB][e % kNB] = A[(size_t)(k0 + e / kNB) * npad + k0 + e % kNB];
      __syncthreads();
      if (w == 0) {  // unit lower triangular solve of the diagonal block
        double v = sb[k0 + lane];
        for (int i = 0; i < kNB - 1; ++i) {
          const double xi = __shfl(v, i);
          if (lane > i) v -= sT[lane][i] * xi;
        }
        sb[k0 + lane] = v;
      }
      __syncthreads();
      // b[r] -= L[r][k0:k0+64] y  for r >= k0 + 64
      const double y = sb[k0 + lane];
      for (int r = k0 + kNB + w; r < npad; r += 4) {
        double s = static_cast<double>(A[(size_t)r * npad + k0 + lane]) * y;
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) sb[r] -= s;
      }
      __syncthreads();
    }
    for (int p = np - 1; p >= 0; --p) {
      const int k0 = p * kNB;
      // rhs_j = b_j - sum_{c >= k0+64} U[k0+j][c] x_c
      for (int j = w; j < kNB; j += 4) {
        const T* row = A + (size_t)(k0 + j) * npad;
        double s = 0.0;
        for (int c = k0 + kNB + lane; c < npad; c += 64) s += static_cast<double>(row[c]) * sb[c];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) sacc[0][j] = s;
      }
      for (int e = tid; e < kNB * kNB; e += 256) sT[e / kNB][e % kNB] = A[(size_t)(k0 + e / kNB) * npad + k0 + e % kNB];
      __syncthreads();
      if (w == 0) {
        double v = sb[k0 + lane] - sacc[0][lane];
        for (int i = kNB - 1; i >= 0; --i) {
          if (lane == i) v = v / sT[i][i];
          const double xi = __shfl(v, i);
          if (lane < i) v -= sT[lane][i] * xi;
        }
        sb[k0 + lane] = v;
      }
      __syncthreads();
    }
  } else {
    // z = U^-T c: forward over panels; U^T is lower triangular
    for (int p = 0; p < np; ++p) {
      const int k0 = p * kNB;
      // acc_j = sum_{i < k0} U[i][k0+j] z_i
      double s = 0.0;
      for (int i = w; i < k0; i += 4) s += static_cast<double>(A[(size_t)i * npad + k0 + lane]) * sb[i];
      sacc[w][lane] = s;
      for (int e = tid; e < kNB * kNB; e += 256) sT[e / kNB][e % kNB] = A[(size_t)(k0 + e / kNB) * npad + k0 + e % kNB];
      __syncthreads();
      if (w == 0) {
        double v = sb[k0 + lane] - (sacc[0][lane] + sacc[1][lane] + sacc[2][lane] + sacc[3][lane]);
        for (int i = 0; i < kNB; ++i) {
          if (lane == i) v = v / sT[i][i];
          const double xi = __shfl(v, i);
          if (lane > i) v -= sT[i][lane] * xi;  // (U^T)[lane][i] = U[i][lane]
        }
        sb[k0 + lane] = v;
      }
      __syncthreads();
    }
    // for p = m..1: z <- L_p^-T z, then z <- P_p^T z
    for (int p = np - 1; p >= 0; --p) {
      const int k0 = p * kNB;
      double s = 0.0;
      for (int r = k0 + kNB + w; r < npad; r += 4) s += static_cast<double>(A[(size_t)r * npad + k0 + lane]) * sb[r];
      sacc[w][lane] = s;
      for (int e = tid; e < kNB * kNB; e += 256) sT[e / kNB][e % kNB] = A[(size_t)(k0 + e / kNB) * npad + k0 + e % kNB];
      __syncthreads();
      if (w == 0) {
        double v = sb[k0 + lane] - (sacc[0][lane] + sacc[1][lane] + sacc[2][lane] + sacc[3][lane]);
        for (int i = kNB - 1; i >= 0; --i) {
          const double xi = __shfl(v, i);
          if (lane < i) v -= sT[i][lane] * xi;  // (L^T)[lane][i] = L[i][lane], unit diagonal
        }
        sb[k0 + lane] = v;
      }
      __syncthreads();
      if (tid == 0) {
        for (int j = kNB - 1; j >= 0; --j) {
          const int q = ip[k0 + j];
          if (q != k0 + j) {
            const double t = sb[k0 + j];
            sb[k0 + j] = sb[q];
            sb[q] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  double* xo = Xout + (size_t)mat * npad;
  for (int i = tid; i < npad; i += 256) xo[i] = accumulate ? xo[i] + sb[i] : sb[i];
}

__global__ void k_pad(const double* __restrict__ F, double* __restrict__ Bp, int n, int npad, int nx) {
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (size_t)nx * npad;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t x = idx / npad;
    const int j = static_cast<int>(idx % npad);
    Bp[idx] = (j < n) ? F[x * n + j] : 0.0;
  }
}

__global__ void k_unpad(const double* __restrict__ Bp, double* __restrict__ F, int n, int npad, int nx) {
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < (size_t)nx * n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t x = idx / n;
    const int j = static_cast<int>(idx % n);
    F[idx] = Bp[x * npad + j];
  }
}

// ---------------------------------------------------------------------------
// FP64 residual R = B - X + dt n0_x (X C^T) + dt E_x (X A^T)  (TRANSPOSE: C, A)
// rows = collocation points, 32 x 64 output tiles, MFMA f64 16x16x4.
// ---------------------------------------------------------------------------
__device__ inline void atomic_max_pos(unsigned long long* p, double v) {
  atomicMax(p, static_cast<unsigned long long>(__double_as_longlong(v)));
}

template <int TRANSPOSE>
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ Bv, const double* __restrict__ Xv,
                                                  double* __restrict__ Rv, const double* __restrict__ C,
                                                  const double* __restrict__ Aop, const double* __restrict__ E,
                                                  const double* __restrict__ n0x, unsigned long long* __restrict__ rmax,
                                                  unsigned long long* __restrict__ bmax, const int* __restrict__ status,
                                                  double dt, int n, int npad, int nx) {
  if (status[1]) return;
  constexpr int BM = 32, BN = 64, BK = 64;
  __shared__ double sX[BM][BK + 1];
  __shared__ double sC[BN][BK + 1];
  __shared__ double sA[BN][BK + 1];
  const int x0 = blockIdx.y * BM, i0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 accC[2], accA[2];
  for (int b = 0; b < 2; ++b) accC[b] = accA[b] = f64x4{0, 0, 0, 0};
  for (int k0 = 0; k0 < n; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      const int r = e / BK, c = e % BK;
      sX[r][c] = (x0 + r < nx && k0 + c < n) ? Xv[(size_t)(x0 + r) * npad + k0 + c] : 0.0;
    }
    for (int e = tid; e < BN * BK; e += 256) {
      const int r = e / BK, c = e % BK;
      const int i = i0 + r, k = k0 + c;
      double cv = 0.0, av = 0.0;
      if (i < n && k < n) {
        const size_t o = TRANSPOSE ? (size_t)k * n + i : (size_t)i * n + k;
        cv = C[o];
        av = Aop[o];
      }
      sC[r][c] = cv;
      sA[r][c] = av;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < BK; k += 4) {
      const double bc = sC[w * 16 + li][k + lk];
      const double ba = sA[w * 16 + li][k + lk];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const double ax = sX[b * 16 + li][k + lk];
        accC[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, bc, accC[b], 0, 0, 0);
        accA[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, ba, accA[b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int x = x0 + b * 16 + Mma<double>::row(lk, it);
      const int i = i0 + w * 16 + li;
      if (x < nx && i < n) {
        const size_t o = (size_t)x * npad + i;
        const double bv = Bv[o];
        const double r = bv - Xv[o] + dt * n0x[x] * accC[b][it] + dt * E[x] * accA[b][it];
        Rv[o] = r;
        atomic_max_pos(&rmax[x], fabs(r));
        atomic_max_pos(&bmax[x], fabs(bv));
      }
    }
}

// status[1] = done flag, status[2] = sweeps used; resid[0] = max_x |r|/|b|
__global__ void k_refine_check(unsigned long long* __restrict__ rmax, unsigned long long* __restrict__ bmax,
                               int* __restrict__ status, double* __restrict__ resid, double rtol, int sweep,
                               int final_sweep, int nx) {
  if (status[1]) return;
  __shared__ double red[256];
  double worst = 0.0;
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    const double r = __longlong_as_double(static_cast<long long>(rmax[x]));
    const double b = __longlong_as_double(static_cast<long long>(bmax[x]));
    const double q = (b > 0.0) ? r / b : (r > 0.0 ? INFINITY : 0.0);
    worst = fmax(worst, (q == q) ? q : INFINITY);
    rmax[x] = 0ull;
    bmax[x] = 0ull;
  }
  red[threadIdx.x] = worst;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    resid[0] = red[0];
    status[2] = sweep;
    if (red[0] <= rtol) status[1] = 1;
    else if (final_sweep) atomicOr(status, kStNoConv);
  }
}

__global__ void k_reset_refine(unsigned long long* rmax, unsigned long long* bmax, int* status, int nx) {
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    rmax[x] = 0ull;
    bmax[x] = 0ull;
  }
  if (threadIdx.x == 0) {
    status[1] = 0;
    status[2] = 0;
  }
}

// grad_scal[op] += dt sum_x n0_x mu_x^T C^(op) F*_x  and  grad_E[x] = dt mu_x^T A F*_x.
// Tiled like the residual: out[x][i] = sum_k F*[x][k] M[i][k] (MFMA f64), then the
// epilogue contracts with mu[x][i].  Grid: (n/64, ceil(nx/32), n_params + 1).
__global__ __launch_bounds__(256) void k_adjoint_grads(const double* __restrict__ Mu, const double* __restrict__ Fs,
                                                       const double* __restrict__ Csb, const double* __restrict__ Aop,
                                                       const double* __restrict__ n0x, double* __restrict__ gscal,
                                                       double* __restrict__ gE, double dt, int n, int nx, int nparams) {
  constexpr int BM = 32, BN = 64, BK = 64;
  const int op = blockIdx.z;
  const double* M = (op < nparams) ? Csb + (size_t)op * n * n : Aop;
  __shared__ double sX[BM][BK + 1];
  __shared__ double sM[BN][BK + 1];
  __shared__ double sRed[BM];
  const int x0 = blockIdx.y * BM, i0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (tid < BM) sRed[tid] = 0.0;
  f64x4 acc[2] = {f64x4{0, 0, 0, 0}, f64x4{0, 0, 0, 0}};
  for (int k0 = 0; k0 < n; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      const int r = e / BK, c = e % BK;
      sX[r][c] = (x0 + r < nx && k0 + c < n) ? Fs[(size_t)(x0 + r) * n + k0 + c] : 0.0;
    }
    for (int e = tid; e < BN * BK; e += 256) {
      const int r = e / BK, c = e % BK;
      sM[r][c] = (i0 + r < n && k0 + c < n) ? M[(size_t)(i0 + r) * n + k0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < BK; k += 4) {
      const double bm = sM[w * 16 + li][k + lk];
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(sX[b * 16 + li][k + lk], bm, acc[b], 0, 0, 0);
    }
    __syncthreads();
  }
  // contract with mu and reduce over i within the block
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int xl = b * 16 + Mma<double>::row(lk, it);
      const int x = x0 + xl;
      const int i = i0 + w * 16 + li;
      double v = (x < nx && i < n) ? Mu[(size_t)x * n + i] * acc[b][it] : 0.0;
      // reduce over the 16 lanes sharing this x (same lk)
      for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (li == 0 && x < nx) atomicAdd(&sRed[xl], v);
    }
  __syncthreads();
  if (tid == 0) {
    double total = 0.0;
    for (int xl = 0; xl < BM; ++xl) {
      const int x = x0 + xl;
      if (x >= nx) break;
      if (op < nparams) total += dt * n0x[x] * sRed[xl];
      else atomicAdd(&gE[x], dt * sRed[xl]);
    }
    if (op < nparams) atomicAdd(&gscal[op], total);
  }
}

template <typename T>
void factor_impl(const DevOps& d, hipStream_t s, LuTimer* tm) {
  T* LU = static_cast<T*>(d.lu);
  dim3 gform(d.npad, d.nx_total);
  k_form<T><<<gform, 256, 0, s>>>(LU, d.Cord, d.Aord, d.E, d.n0x, d.status, d.dt, d.n, d.npad);
  const int np = d.npad / kNB;
  if (tm) tm->used = 0;
  for (int p = 0; p < np; ++p) {
    const int k0 = p * kNB;
    const bool rec = tm && p < tm->max_panels;
    if (rec) (void)hipEventRecord(tm->ev[2 * tm->max_panels + 2 * p], s);
    constexpr int IB = sizeof(T) == 8 ? 8 : 16;  // register sub-panel width (VGPR budget of 512 threads)
    if (d.npad <= kPanelThreads) k_panel<T, 1, IB><<<d.nx_total, kPanelThreads, 0, s>>>(LU, d.piv, d.perm, d.status, d.npad, k0);
    else if (d.npad <= 2 * kPanelThreads) k_panel<T, 2, IB><<<d.nx_total, kPanelThreads, 0, s>>>(LU, d.piv, d.perm, d.status, d.npad, k0);
    else k_panel<T, 4, IB><<<d.nx_total, kPanelThreads, 0, s>>>(LU, d.piv, d.perm, d.status, d.npad, k0);  // npad <= 2048
    const int rest = d.npad - k0 - kNB;
    if (rest > 0) {
      dim3 gs(rest / 64, d.nx_total);
      k_swap_trsm<T><<<gs, 64, 0, s>>>(LU, d.perm, d.npad, k0);
      if (rec) {
        (void)hipEventRecord(tm->ev[2 * tm->max_panels + 2 * p + 1], s);
        (void)hipEventRecord(tm->ev[2 * p], s);
      }
      const int mt = rest / 64;
      dim3 gu(mt * mt, d.nx_total);
      k_update<T><<<gu, 256, 0, s>>>(LU, d.npad, k0);
      if (rec) (void)hipEventRecord(tm->ev[2 * p + 1], s);
    } else if (rec) {
      (void)hipEventRecord(tm->ev[2 * tm->max_panels + 2 * p + 1], s);
      (void)hipEventRecord(tm->ev[2 * p], s);
      (void)hipEventRecord(tm->ev[2 * p + 1], s);
    }
    if (rec) tm->used = p + 1;
  }
}

}  // namespace

void launch_lu_factor(const DevOps& d, int precision, hipStream_t s, LuTimer* timer) {
  if (precision == 0) factor_impl<double>(d, s, timer);
  else factor_impl<float>(d, s, timer);
}

void launch_lu_solve(const DevOps& d, int precision, bool transpose, const double* Bin, double* Xout, bool accumulate,
                     bool check_done, hipStream_t s) {
  const size_t sh = sizeof(double) * d.npad;
  if (precision == 0) {
    const double* LU = static_cast<const double*>(d.lu);
    if (transpose) k_solve<double, 1><<<d.nx_total, 256, sh, s>>>(LU, d.piv, Bin, Xout, d.status, accumulate, check_done, d.npad);
    else k_solve<double, 0><<<d.nx_total, 256, sh, s>>>(LU, d.piv, Bin, Xout, d.status, accumulate, check_done, d.npad);
  } else {
    const float* LU = static_cast<const float*>(d.lu);
    if (transpose) k_solve<float, 1><<<d.nx_total, 256, sh, s>>>(LU, d.piv, Bin, Xout, d.status, accumulate, check_done, d.npad);
    else k_solve<float, 0><<<d.nx_total, 256, sh, s>>>(LU, d.piv, Bin, Xout, d.status, accumulate, check_done, d.npad);
  }
}

void launch_pad_rows(const DevOps& d, const double* F, double* Bp, hipStream_t s) {
  k_pad<<<1024, 256, 0, s>>>(F, Bp, d.n, d.npad, d.nx_total);
}

void launch_unpad_rows(const DevOps& d, const double* Bp, double* F, hipStream_t s) {
  k_unpad<<<1024, 256, 0, s>>>(Bp, F, d.n, d.npad, d.nx_total);
}

void launch_residual(const DevOps& d, bool transpose, hipStream_t s) {
  dim3 g((d.n + 63) / 64, (d.nx_total + 31) / 32);
  if (transpose)
    k_residual<1><<<g, 256, 0, s>>>(d.B, d.X, d.R, d.Cord, d.Aord, d.E, d.n0x, d.rmax, d.bmax, d.status, d.dt, d.n,
                                    d.npad, d.nx_total);
  else
    k_residual<0><<<g, 256, 0, s>>>(d.B, d.X, d.R, d.Cord, d.Aord, d.E, d.n0x, d.rmax, d.bmax, d.status, d.dt, d.n,
                                    d.npad, d.nx_total);
}

void launch_refine_check(const DevOps& d, double rtol, int sweep, bool final_sweep, hipStream_t s) {
  k_refine_check<<<1, 256, 0, s>>>(d.rmax, d.bmax, d.status, d.resid, rtol, sweep, final_sweep ? 1 : 0, d.nx_total);
}

void launch_reset_refine(const DevOps& d, hipStream_t s) {
  k_reset_refine<<<1, 256, 0, s>>>(d.rmax, d.bmax, d.status, d.nx_total);
}

void launch_adjoint_grads(const DevOps& d, double* grad_scal, double* grad_E, hipStream_t s) {
  dim3 g((d.n + 63) / 64, (d.nx_total + 31) / 32, d.n_params + 1);
  k_adjoint_grads<<<g, 256, 0, s>>>(d.mu, d.Fs, d.Csb, d.Aord, d.n0x, grad_scal, grad_E, d.dt, d.n, d.nx_total,
                                    d.n_params);
}

}  // namespace bte

// Velocity-space step in Hessenberg form (the harmonic-basis systems
// (B - s A_h) u = b of eq. (vspace_batched_system), s = dt E_x, reduced once per
// discharge to u = Q (I - s H)^-1 W b with H upper Hessenberg; see hessenberg.cpp):
//   k_mat_apply   Out[x] = M In[x] for the points of one discharge (W, then Q):
//                 32 points x 64 outputs per block, MFMA f64 16x16x4;
//   k_hess_solve  (I - s H) z = y, one block per point, in O(n^2): Givens
//                 rotations of columns (k-1, k), k = n-1 .. 1, turn G = I - s H
//                 into an upper triangular R = G Z; column k of R is final once
//                 formed, so the back substitution R w = y runs alongside and R is
//                 never stored; then z = Z w.
#include <cmath>

#include "internal.h"

namespace bte {
namespace {

using f64x4 = double __attribute__((ext_vector_type(4)));

// Result row of item t of lane group lk for MFMA f64 16x16x4 (measured layout).
__device__ inline int f64_row(int lk, int t) { return lk + 4 * t; }

// Out[x][i] = sum_k M[i][k] In[x][k], x in [x0, x0 + nx), rows of length ld.
// Grid: (ceil(n / 64), ceil(nx / 32)).
__global__ __launch_bounds__(256) void k_mat_apply(const double* __restrict__ M, const double* __restrict__ In,
                                                   double* __restrict__ Out, int n, int ld, int x0, int nx) {
  constexpr int BM = 32, BN = 64, BK = 64;
  __shared__ double sX[BM][BK + 1];
  __shared__ double sM[BN][BK + 1];
  const int xb = blockIdx.y * BM, i0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[2] = {f64x4{0, 0, 0, 0}, f64x4{0, 0, 0, 0}};
  for (int k0 = 0; k0 < n; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      const int r = e / BK, c = e % BK;
      sX[r][c] = (xb + r < nx && k0 + c < n) ? In[(size_t)(x0 + xb + r) * ld + k0 + c] : 0.0;
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
      for (int b = 0; b < 2; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(sX[b * 16 + li][k + lk], bm, acc[b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int xl = xb + b * 16 + f64_row(lk, it);
      const int i = i0 + w * 16 + li;
      if (xl < nx && i < n) Out[(size_t)(x0 + xl) * ld + i] = acc[b][it];
    }
}

constexpr int kHessThreads = 256;

// (I - s H) z = y for one point per block; H column-major (n x n, upper
// Hessenberg), y and z rows of length ld.  Thread t holds rows t + q NT of the
// current column of G Z, of y and of the next D columns of G (loaded D steps ahead).
template <int RPT>
__global__ __launch_bounds__(kHessThreads) void k_hess_solve(const double* __restrict__ Hc,
                                                             const size_t* __restrict__ h_off,
                                                             const int* __restrict__ x_disc,
                                                             const double* __restrict__ E, double dt,
                                                             const double* __restrict__ Y, double* __restrict__ Z,
                                                             int n, int ld, int* __restrict__ status) {
  constexpr int NT = kHessThreads;
  const int x = blockIdx.x, tid = threadIdx.x;
  const double* H = Hc + h_off[x_disc[x]];
  const double s = dt * E[x];
  __shared__ double s_c[kMaxRows], s_s[kMaxRows], s_w[kMaxRows];
  __shared__ double s_bc[2][3];
  // columns of H in flight, raw (the transform to G = I - s H is applied where a
  // column is used, so that no instruction waits on a load before then): slot u
  // holds column k - 1 for the steps k = n - 1 - u (mod D), D steps ahead of use
  constexpr int D = 8;
  double cur[RPT], y[RPT], hq[D][RPT];
  auto load_h = [&](double (&dst)[RPT], int c) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + q * NT;
      dst[q] = (r <= c + 1 && r < n) ? H[(size_t)c * n + r] : 0.0;
    }
  };
  // entry (r, c) of G from the raw H entry h
  auto gval = [&](int r, int c, double h) { return (r == c ? 1.0 : 0.0) - s * h; };
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = tid + q * NT;
    y[q] = (r < n) ? Y[(size_t)x * ld + r] : 0.0;
  }
  load_h(cur, n - 1);
#pragma unroll
  for (int q = 0; q < RPT; ++q) cur[q] = gval(tid + q * NT, n - 1, cur[q]);
#pragma unroll
  for (int u = 0; u < D; ++u)
    if (n - 2 - u >= 0) load_h(hq[u], n - 2 - u);
  bool bad = false;
  for (int kb = n - 1; kb >= 1; kb -= D) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int k = kb - u;
      if (k < 1) break;
      const int par = k & 1;
      double g[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) g[q] = gval(tid + q * NT, k - 1, hq[u][q]);
      if (tid == k % NT) {
        // rows k of column k-1 (a) and of the current column k (b): the rotation
        // that zeroes row k of the new column k-1; R[k][k] = hypot(a, b)
        const int qk = k / NT;
        double a = 0.0, b = 0.0, yk = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q)
          if (q == qk) {
            a = g[q];
            b = cur[q];
            yk = y[q];
          }
        const double rr = hypot(a, b);
        const double ri = 1.0 / rr;
        const double c = rr > 0.0 ? b * ri : 1.0, sg = rr > 0.0 ? a * ri : 0.0;
        const double wk = yk * ri;
        if (rr == 0.0) bad = true;
        s_bc[par][0] = c;
        s_bc[par][1] = sg;
        s_bc[par][2] = wk;
        s_c[k] = c;
        s_s[k] = sg;
        s_w[k] = wk;
      }
      __syncthreads();
      const double c = s_bc[par][0], sg = s_bc[par][1], wk = s_bc[par][2];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = tid + q * NT;
        if (r < k) {
          const double rk = c * cur[q] + sg * g[q];   // column k of R
          y[q] -= rk * wk;
          cur[q] = -sg * cur[q] + c * g[q];           // the new column k-1
        }
      }
      if (k - 1 - D >= 0) load_h(hq[u], k - 1 - D);    // for the step k - D
    }
  }
  if (tid == 0) {
    const double r0 = cur[0];
    if (r0 == 0.0) bad = true;
    s_w[0] = y[0] / r0;
    // z = Z_{n-1} ... Z_1 w, Z_k acting on entries (k-1, k): a running carry t
    double t = s_w[0];
    for (int k = 1; k < n; ++k) {
      const double c = s_c[k], sg = s_s[k], wk = s_w[k];
      s_w[k - 1] = c * t + sg * wk;
      t = -sg * t + c * wk;
    }
    s_w[n - 1] = t;
    if (!(fabs(t) <= 1.0e300)) atomicOr(status, kStNonFinite);
  }
  if (bad) atomicOr(status, kStSingular);
  __syncthreads();
  for (int r = tid; r < ld; r += NT) Z[(size_t)x * ld + r] = (r < n) ? s_w[r] : 0.0;
}

}  // namespace

void launch_mat_apply(const double* M, const double* In, double* Out, int n, int ld, int x0, int nx, hipStream_t s) {
  if (nx <= 0) return;
  dim3 g((n + 63) / 64, (nx + 31) / 32);
  k_mat_apply<<<g, 256, 0, s>>>(M, In, Out, n, ld, x0, nx);
}

void launch_hess_solve(const DevOps& d, const double* Hc, const size_t* h_off, int n, int ld, const double* Y,
                       double* Z, hipStream_t s) {
  const int rpt = (n + kHessThreads - 1) / kHessThreads;
  if (rpt <= 1)
    k_hess_solve<1><<<d.nx_total, kHessThreads, 0, s>>>(Hc, h_off, d.x_disc, d.E, d.dt, Y, Z, n, ld, d.status);
  else if (rpt <= 2)
    k_hess_solve<2><<<d.nx_total, kHessThreads, 0, s>>>(Hc, h_off, d.x_disc, d.E, d.dt, Y, Z, n, ld, d.status);
  else if (rpt <= 4)
    k_hess_solve<4><<<d.nx_total, kHessThreads, 0, s>>>(Hc, h_off, d.x_disc, d.E, d.dt, Y, Z, n, ld, d.status);
  else
    k_hess_solve<8><<<d.nx_total, kHessThreads, 0, s>>>(Hc, h_off, d.x_disc, d.E, d.dt, Y, Z, n, ld, d.status);
}

}  // namespace bte

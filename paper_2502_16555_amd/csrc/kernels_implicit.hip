// Pieces of the fully implicit electron step (eq. bte_fully_implicit) that the
// semi-implicit kernels do not already provide: the forward spatial operator
// A_x F D_x^T in the speed eigenbasis, the wall rows of the implicit system,
// and the vector kernels of the Newton-Krylov driver (batched dot products with
// deterministic two-stage sums, linear combinations).
#include <stdexcept>

#include "internal.h"

namespace bte {
namespace {

constexpr int kThreads = 256;
constexpr int kDotBlocks = 256;

// Y_ia <- lambda_i cos(theta_a) D_x Y_ia for every mode of every discharge
// (mode-major Y of the X step: the modes of discharge d at Y + x_off[d] n, one
// row of nx_d per mode); A_x = U Lambda U^-1 (x) diag(cos theta).  D_x is read
// column-major (entry (x, k) at k nx + x), so that a load over the threads' x is
// one coalesced row of D_x^T, and each loaded entry serves the MB modes of the
// block; every output takes its products in ascending k.
template <int MB>
__global__ __launch_bounds__(kThreads) void k_x_fwd(double* __restrict__ Y, const double* __restrict__ DT,
                                                    const size_t* __restrict__ dx_off, const double* __restrict__ lam,
                                                    const double* __restrict__ mu, const int* __restrict__ x_off,
                                                    const int* __restrict__ nx_of, int nth, int n) {
  extern __shared__ double sy[];   // [MB][nx]
  const int o0 = blockIdx.x * MB, d = blockIdx.y;
  const int nx = nx_of[d], nm = min(MB, n - o0);
  double* y0 = Y + (size_t)x_off[d] * n;
  for (int m = 0; m < MB; ++m)
    for (int j = threadIdx.x; j < nx; j += blockDim.x) sy[m * nx + j] = m < nm ? y0[(size_t)(o0 + m) * nx + j] : 0.0;
  __syncthreads();
  const double* D = DT + dx_off[d];
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    double acc[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) acc[m] = 0.0;
#pragma unroll 8
    for (int k = 0; k < nx; ++k) {
      const double dk = D[(size_t)k * nx + x];
#pragma unroll
      for (int m = 0; m < MB; ++m) acc[m] += dk * sy[m * nx + k];
    }
#pragma unroll
    for (int m = 0; m < MB; ++m) {
      if (m < nm) {
        const int o = o0 + m;
        y0[(size_t)o * nx + x] = lam[o / nth] * mu[o % nth] * acc[m];
      }
    }
  }
}

// out = X at the inflow entries (x = 0 for cos theta > 0, x = L for cos theta < 0)
__global__ __launch_bounds__(kThreads) void k_wall_rows(double* __restrict__ out, const double* __restrict__ X,
                                                        const int* __restrict__ x_disc, const int* __restrict__ x_off,
                                                        const int* __restrict__ nx_of, const double* __restrict__ mu,
                                                        int nth, int n) {
  const int x = blockIdx.x, d = x_disc[x];
  const int xl = x - x_off[d], nx = nx_of[d];
  if (xl != 0 && xl != nx - 1) return;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const double m = mu[e % nth];
    if ((xl == 0 && m > 0.0) || (xl == nx - 1 && m < 0.0)) out[(size_t)x * n + e] = X[(size_t)x * n + e];
  }
}

// partial[b][v] = sum over block b's slice of w . V_v   (v < nvec, V_v = V + v stride)
__global__ __launch_bounds__(kThreads) void k_dots(const double* __restrict__ w, const double* __restrict__ V,
                                                   int nvec, size_t stride, size_t N, double* __restrict__ partial) {
  __shared__ double red[kThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int v = 0; v < nvec; ++v) {
    const double* vv = V + (size_t)v * stride;
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x)
      s += w[i] * vv[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) red[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int u = 0; u < kThreads / 64; ++u) t += red[u];
      partial[(size_t)blockIdx.x * nvec + v] = t;
    }
    __syncthreads();
  }
}

// y = beta y + sum_v coef[v] V_v
__global__ __launch_bounds__(kThreads) void k_comb(double* __restrict__ y, double beta, const double* __restrict__ V,
                                                   const double* __restrict__ coef, int nvec, size_t stride,
                                                   size_t N) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
    double s = (beta == 0.0) ? 0.0 : beta * y[i];
    for (int v = 0; v < nvec; ++v) s += coef[v] * V[(size_t)v * stride + i];
    y[i] = s;
  }
}

// The Gram-Schmidt coefficients of one pass from k_dots' partial sums, summed
// over the blocks in block order (the same order on every call): h[v] = t_v
// (first pass) or h[v] + t_v (second pass), coef[v] = -t_v for k_comb.
__global__ __launch_bounds__(kThreads) void k_gs_reduce(const double* __restrict__ partial, int nvec, int nb,
                                                        int accumulate, double* __restrict__ h,
                                                        double* __restrict__ coef) {
  for (int v = threadIdx.x; v < nvec; v += blockDim.x) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += partial[(size_t)b * nvec + v];
    h[v] = accumulate ? h[v] + t : t;
    coef[v] = -t;
  }
}

// *h = sqrt of k_dots' single partial sums (w . w), summed in block order
__global__ __launch_bounds__(64) void k_norm_reduce(const double* __restrict__ partial, int nb,
                                                    double* __restrict__ h) {
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += partial[b];
    *h = sqrt(t);
  }
}

// y = y / *h where *h > 0 (else y is left as it is)
__global__ __launch_bounds__(kThreads) void k_scale_inv(double* __restrict__ y, const double* __restrict__ h,
                                                        size_t N) {
  const double hv = *h;
  if (!(hv > 0.0)) return;
  const double a = 1.0 / hv;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * y[i];
}

// y = a y + b x
__global__ __launch_bounds__(kThreads) void k_axpby(double* __restrict__ y, const double* __restrict__ x, double a,
                                                    double b, size_t N) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x)
    y[i] = a * y[i] + b * x[i];
}

}  // namespace

void launch_x_forward(const DevOps& d, hipStream_t s) {
  // eight modes per block: their rows take at most 64 KB of LDS (Nx <= 1024)
  constexpr int MB = 8;
  if ((size_t)MB * d.max_nx * sizeof(double) > 65536) throw std::invalid_argument("Nx above 1024");
  dim3 g((d.n + MB - 1) / MB, d.nd);
  k_x_fwd<MB><<<g, kThreads, sizeof(double) * MB * d.max_nx, s>>>(d.Y, d.dxT, d.p_off, d.lam, d.mu_th, d.x_off,
                                                                   d.nx_of, d.nth, d.n);
}

void launch_wall_rows(const DevOps& d, double* out, const double* X, hipStream_t s) {
  k_wall_rows<<<d.nx_total, kThreads, 0, s>>>(out, X, d.x_disc, d.x_off, d.nx_of, d.mu_th, d.nth, d.n);
}

int dot_blocks() { return kDotBlocks; }

void launch_dots(const double* w, const double* V, int nvec, size_t stride, size_t N, double* partial,
                 hipStream_t s) {
  k_dots<<<kDotBlocks, kThreads, 0, s>>>(w, V, nvec, stride, N, partial);
}

void launch_comb(double* y, double beta, const double* V, const double* coef, int nvec, size_t stride, size_t N,
                 hipStream_t s) {
  k_comb<<<1024, kThreads, 0, s>>>(y, beta, V, coef, nvec, stride, N);
}

void launch_gs_reduce(const double* partial, int nvec, int accumulate, double* h, double* coef, hipStream_t s) {
  k_gs_reduce<<<1, kThreads, 0, s>>>(partial, nvec, kDotBlocks, accumulate, h, coef);
}

void launch_norm_reduce(const double* partial, double* h, hipStream_t s) {
  k_norm_reduce<<<1, 64, 0, s>>>(partial, kDotBlocks, h);
}

void launch_scale_inv(double* y, const double* h, size_t N, hipStream_t s) {
  k_scale_inv<<<1024, kThreads, 0, s>>>(y, h, N);
}

void launch_axpby(double* y, const double* x, double a, double b, size_t N, hipStream_t s) {
  k_axpby<<<1024, kThreads, 0, s>>>(y, x, a, b, N);
}

}  // namespace bte

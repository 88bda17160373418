// Spatial advection X(dt/2) (Alg. bte_spatial_adv of the paper), the field
// E^{1/2} (eq. bte_semi_implicit_efield), the moments (eq. hybrid_discrete_c and
// the k_i definition of the hybrid model) and the Maxwellian initial state.
//
// X(dt/2):  Y = (U^-1 (x) I) F      -> mode-major Y[i][a][x] (x contiguous)
//           Y_ia <- Q_ia Y_ia        (HBM-bound batched GEMV; Q streamed once per
//                                     ordinate pair thanks to Q(-mu) = J Q(mu) J)
//           F = (U (x) I) Y
#include <cmath>

#include "internal.h"

namespace bte {
namespace {

constexpr int kThreads = 256;

__device__ inline bool finite_d(double v) { return (v - v) == 0.0; }

// Y_d[i][a][xl] = sum_k Uinv[i][k] F[x][k][a]   (one block per global x)
__global__ __launch_bounds__(kThreads) void k_x_to_modes(const double* __restrict__ F, double* __restrict__ Y,
                                                         const double* __restrict__ W, const int* __restrict__ x_disc,
                                                         const int* __restrict__ x_off, const int* __restrict__ nx_of,
                                                         int nr, int nth, int transposeW, int* __restrict__ status) {
  extern __shared__ double sm[];
  const int x = blockIdx.x;
  const int n = nr * nth;
  double* f = sm;
  double* w = sm + n;
  bool bad = false;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double v = F[(size_t)x * n + j];
    bad |= !finite_d(v);
    f[j] = v;
  }
  for (int j = threadIdx.x; j < nr * nr; j += blockDim.x) {
    // transposeW: use W^T (the X^T path contracts with U^T)
    int r = j / nr, c = j % nr;
    w[j] = transposeW ? W[c * nr + r] : W[j];
  }
  if (bad) atomicOr(status, kStNonFinite);
  __syncthreads();
  const int d = x_disc[x];
  const int nx = nx_of[d];
  const int xl = x - x_off[d];
  double* Yd = Y + (size_t)x_off[d] * n;
  for (int o = threadIdx.x; o < n; o += blockDim.x) {
    const int i = o / nth, a = o % nth;
    double s = 0.0;
    for (int k = 0; k < nr; ++k) s += w[i * nr + k] * f[k * nth + a];
    Yd[(size_t)o * nx + xl] = s;
  }
}

// F[x][k][a] = sum_i W[k][i] Y_d[i][a][xl]
__global__ __launch_bounds__(kThreads) void k_modes_to_x(const double* __restrict__ Y, double* __restrict__ F,
                                                         const double* __restrict__ W, const int* __restrict__ x_disc,
                                                         const int* __restrict__ x_off, const int* __restrict__ nx_of,
                                                         int nr, int nth, int transposeW) {
  extern __shared__ double sm[];
  const int x = blockIdx.x;
  const int n = nr * nth;
  const int d = x_disc[x];
  const int nx = nx_of[d];
  const int xl = x - x_off[d];
  const double* Yd = Y + (size_t)x_off[d] * n;
  double* z = sm;
  double* w = sm + n;
  for (int j = threadIdx.x; j < n; j += blockDim.x) z[j] = Yd[(size_t)j * nx + xl];
  for (int j = threadIdx.x; j < nr * nr; j += blockDim.x) {
    int r = j / nr, c = j % nr;
    w[j] = transposeW ? W[c * nr + r] : W[j];
  }
  __syncthreads();
  for (int o = threadIdx.x; o < n; o += blockDim.x) {
    const int k = o / nth, a = o % nth;
    double s = 0.0;
    for (int i = 0; i < nr; ++i) s += w[k * nr + i] * z[i * nth + a];
    F[(size_t)x * n + o] = s;
  }
}

// Batched Chebyshev-system application for one (eigen-speed i, ordinate pair).
// Qt holds Q_{i,a} transposed (Qt[c][r] = Q[r][c]) for the ordinates with cos > 0;
// the mirrored ordinate uses Q(-mu) y = J Q(mu) J y.  transpose=1 applies Q^T.
// Q is read once per half-step (537 MB at C2 in FP64) by non-temporal loads.
template <typename QT, int TRANSPOSE>
__global__ __launch_bounds__(kThreads) void k_advect(double* __restrict__ Y, const QT* __restrict__ Qt,
                                                     const size_t* __restrict__ q_off, const int* __restrict__ x_off,
                                                     const int* __restrict__ nx_of, int nr, int nth) {
  extern __shared__ double sy[];
  const int m = blockIdx.x;
  const int d = blockIdx.y;
  const int nh = nth / 2;
  const int i = m / nh, h = m % nh;
  const int nx = nx_of[d];
  const int n = nr * nth;
  double* Yd = Y + (size_t)x_off[d] * n;
  double* yp = Yd + (size_t)(i * nth + nh + h) * nx;
  double* yn = Yd + (size_t)(i * nth + nh - 1 - h) * nx;
  const QT* Q = Qt + q_off[d] + (size_t)m * nx * nx;
  for (int c = threadIdx.x; c < nx; c += blockDim.x) {
    sy[c] = yp[c];
    sy[nx + c] = yn[nx - 1 - c];
  }
  __syncthreads();
  if (!TRANSPOSE) {
    // out[r] = sum_c Q[r][c] y[c] = sum_c Qt[c][r] y[c]: coalesced over r
    for (int r = threadIdx.x; r < nx; r += blockDim.x) {
      double ap = 0.0, an = 0.0;
#pragma unroll 8
      for (int c = 0; c < nx; ++c) {
        const double q = static_cast<double>(__builtin_nontemporal_load(&Q[(size_t)c * nx + r]));
        ap += q * sy[c];
        an += q * sy[nx + c];
      }
      yp[r] = ap;
      yn[nx - 1 - r] = an;
    }
  } else {
    // out[c] = sum_r Q[r][c] y[r] = sum_r Qt[c][r] y[r]: one wavefront per output c
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int c = wid; c < nx; c += nw) {
      double ap = 0.0, an = 0.0;
      for (int r = lane; r < nx; r += 64) {
        const double q = static_cast<double>(__builtin_nontemporal_load(&Q[(size_t)c * nx + r]));
        ap += q * sy[r];
        an += q * sy[nx + r];
      }
      for (int off = 32; off > 0; off >>= 1) {
        ap += __shfl_xor(ap, off);
        an += __shfl_xor(an, off);
      }
      if (lane == 0) {
        yp[c] = ap;
        yn[nx - 1 - c] = an;
      }
    }
  }
}

// Poisson field over all points: rhs[x] = -(e/eps0)(n_i - u^T F) at interior
// points, the electrode voltage / 0 at the walls (one wavefront per point);
// then E[x] = (P_d rhs_d)[x] (one wavefront per point, lanes along P's row).
__global__ __launch_bounds__(kThreads) void k_field_rhs(double t_half, double freq, double V0,
                                                        const double* __restrict__ Fh, const double* __restrict__ ni,
                                                        double* __restrict__ rhs, const int* __restrict__ x_disc,
                                                        const int* __restrict__ x_off, const int* __restrict__ nx_of,
                                                        const double* __restrict__ mom, int nx_total, int n) {
  const int x = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (x >= nx_total) return;
  const int d = x_disc[x], xl = x - x_off[d];
  const double kE = 1.602176634e-19, kEps0 = 8.8541878128e-12, kPi = 3.14159265358979323846;
  const double* f = Fh + (size_t)x * n;
  double s = 0.0;
  for (int c = lane; c < n; c += 64) s += mom[c] * f[c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) {
    double v = -(kE / kEps0) * (ni[x] - s);
    if (xl == 0) v = V0 * sin(2.0 * kPi * freq * t_half);
    if (xl == nx_of[d] - 1) v = 0.0;
    rhs[x] = v;
  }
}

__global__ __launch_bounds__(kThreads) void k_field_apply(const double* __restrict__ rhs, double* __restrict__ E,
                                                          const int* __restrict__ x_disc,
                                                          const int* __restrict__ x_off, const int* __restrict__ nx_of,
                                                          const double* __restrict__ P,
                                                          const size_t* __restrict__ p_off, int nx_total) {
  const int x = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (x >= nx_total) return;
  const int d = x_disc[x], x0 = x_off[d], nx = nx_of[d], j = x - x0;
  const double* row = P + p_off[d] + (size_t)j * nx;
  double s = 0.0;
  for (int c = lane; c < nx; c += 64) s += row[c] * rhs[x0 + c];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) E[x] = s;
}

// E^{1/2} for the specified modes (one block per discharge).
__global__ __launch_bounds__(kThreads) void k_field(int mode, double t_half, double freq, double a1, double V0,
                                                    const double* __restrict__ Fh, const double* __restrict__ Eg,
                                                    const double* __restrict__ ni, double* __restrict__ E,
                                                    const int* __restrict__ x_off, const int* __restrict__ nx_of,
                                                    const double* __restrict__ E0_of, const double* __restrict__ xhat,
                                                    const double* __restrict__ mom, const double* __restrict__ P,
                                                    const size_t* __restrict__ p_off, int n) {
  const int d = blockIdx.x;
  const int x0 = x_off[d], nx = nx_of[d];
  const double kPi = 3.14159265358979323846;
  if (mode == 0 || mode == 1 || mode == 2) {
    const double s = (mode == 1) ? sin(2.0 * kPi * freq * t_half) : 1.0;
    for (int j = threadIdx.x; j < nx; j += blockDim.x) {
      const int x = x0 + j;
      E[x] = (mode == 2) ? Eg[x] : (mode == 0 ? E0_of[d] : E0_of[d] * s * (1.0 + a1 * xhat[x]));
    }
  }
  // Poisson (mode 3) runs as k_field_rhs and k_field_apply
}

// gE0[d] += sum_{x in d} gE[x] dE_x/dE0_d
__global__ void k_field_dE0(int mode, double t_half, double freq, double a1, const double* __restrict__ gE,
                            double* __restrict__ gE0, const int* __restrict__ x_off, const int* __restrict__ nx_of,
                            const double* __restrict__ xhat) {
  const int d = blockIdx.x;
  const double kPi = 3.14159265358979323846;
  const double s = (mode == 1) ? sin(2.0 * kPi * freq * t_half) : 1.0;
  double acc = 0.0;
  for (int j = threadIdx.x; j < nx_of[d]; j += blockDim.x) {
    const int x = x_off[d] + j;
    acc += gE[x] * (mode == 1 ? s * (1.0 + a1 * xhat[x]) : 1.0);
  }
  __shared__ double red[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    gE0[d] += t;
  }
}

__device__ inline void block_sum3(double& a, double& b, double& c, double* red) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
    c += __shfl_xor(c, off);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
    red[3 * wid] = a;
    red[3 * wid + 1] = b;
    red[3 * wid + 2] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
  for (int w = 0; w < nw; ++w) {
    a += red[3 * w];
    b += red[3 * w + 1];
    c += red[3 * w + 2];
  }
}

// Moments per x: n_e = u.F, mean energy = e.F / n_e, k_i = k.F / n_e
__global__ __launch_bounds__(kThreads) void k_moments(const double* __restrict__ F, const double* __restrict__ mom,
                                                      double* __restrict__ out, int n, int nx_total) {
  __shared__ double red[3 * (kThreads / 64)];
  const int x = blockIdx.x;
  const double* f = F + (size_t)x * n;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double v = f[j];
    a += mom[j] * v;
    b += mom[n + j] * v;
    c += mom[2 * n + j] * v;
  }
  block_sum3(a, b, c, red);
  if (threadIdx.x == 0) {
    out[x] = a;
    out[nx_total + x] = (a != 0.0) ? b / a : 0.0;
    out[2 * nx_total + x] = (a != 0.0) ? c / a : 0.0;
  }
}

// lam[x] += g0 u + g1 (e - ebar u)/ne + g2 (k - kbar u)/ne
__global__ __launch_bounds__(kThreads) void k_moments_vjp(const double* __restrict__ F, const double* __restrict__ mom,
                                                          const double* __restrict__ g, double* __restrict__ lam, int n,
                                                          int nx_total) {
  __shared__ double red[3 * (kThreads / 64)];
  const int x = blockIdx.x;
  const double* f = F + (size_t)x * n;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double v = f[j];
    a += mom[j] * v;
    b += mom[n + j] * v;
    c += mom[2 * n + j] * v;
  }
  block_sum3(a, b, c, red);
  const double g0 = g[x], g1 = g[nx_total + x], g2 = g[2 * nx_total + x];
  const double inv = (a != 0.0) ? 1.0 / a : 0.0;
  const double eb = b * inv, kb = c * inv;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double u = mom[j];
    lam[(size_t)x * n + j] += g0 * u + g1 * (mom[n + j] - eb * u) * inv + g2 * (mom[2 * n + j] - kb * u) * inv;
  }
}

__global__ void k_maxwellian(const double* __restrict__ ne, const double* __restrict__ coeff, double* __restrict__ F,
                             int nr, int nth, int nx_total) {
  const size_t n = (size_t)nr * nth;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n * nx_total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t x = idx / n;
    const int k = static_cast<int>((idx % n) / nth);
    F[idx] = ne[x] * coeff[k];
  }
}

}  // namespace

void launch_x_to_modes(const DevOps& d, const double* F, hipStream_t s) {
  const size_t sh = sizeof(double) * (d.n + d.nr * d.nr);
  k_x_to_modes<<<d.nx_total, kThreads, sh, s>>>(F, d.Y, d.Uinv, d.x_disc, d.x_off, d.nx_of, d.nr, d.nth, 0, d.status);
}

void launch_x_to_modes_T(const DevOps& d, const double* F, hipStream_t s) {
  const size_t sh = sizeof(double) * (d.n + d.nr * d.nr);
  k_x_to_modes<<<d.nx_total, kThreads, sh, s>>>(F, d.Y, d.U, d.x_disc, d.x_off, d.nx_of, d.nr, d.nth, 1, d.status);
}

void launch_modes_to_x(const DevOps& d, double* F, hipStream_t s) {
  const size_t sh = sizeof(double) * (d.n + d.nr * d.nr);
  k_modes_to_x<<<d.nx_total, kThreads, sh, s>>>(d.Y, F, d.U, d.x_disc, d.x_off, d.nx_of, d.nr, d.nth, 0);
}

void launch_modes_to_x_T(const DevOps& d, double* F, hipStream_t s) {
  const size_t sh = sizeof(double) * (d.n + d.nr * d.nr);
  k_modes_to_x<<<d.nx_total, kThreads, sh, s>>>(d.Y, F, d.Uinv, d.x_disc, d.x_off, d.nx_of, d.nr, d.nth, 1);
}

void launch_advect(const DevOps& d, bool fp32, bool transpose, hipStream_t s, const double* Qt) {
  dim3 grid(d.nr * d.nh, d.nd);
  const size_t sh = sizeof(double) * 2 * d.max_nx;
  if (Qt) {   // other FP64 inverses in the layout of d.Qt (forward only)
    k_advect<double, 0><<<grid, kThreads, sh, s>>>(d.Y, Qt, d.q_off, d.x_off, d.nx_of, d.nr, d.nth);
  } else if (fp32) {
    if (transpose) k_advect<float, 1><<<grid, kThreads, sh, s>>>(d.Y, d.Qt32, d.q_off, d.x_off, d.nx_of, d.nr, d.nth);
    else k_advect<float, 0><<<grid, kThreads, sh, s>>>(d.Y, d.Qt32, d.q_off, d.x_off, d.nx_of, d.nr, d.nth);
  } else {
    if (transpose) k_advect<double, 1><<<grid, kThreads, sh, s>>>(d.Y, d.Qt, d.q_off, d.x_off, d.nx_of, d.nr, d.nth);
    else k_advect<double, 0><<<grid, kThreads, sh, s>>>(d.Y, d.Qt, d.q_off, d.x_off, d.nx_of, d.nr, d.nth);
  }
}

void launch_field(const DevOps& d, int mode, double t_half, double freq, double a1, double V0, const double* Fh,
                  const double* E_given, const double* ni, double* E, hipStream_t s, double* rhs) {
  if (mode == 3) {
    if (!rhs) rhs = d.field_rhs;
    const int gb = (d.nx_total + kThreads / 64 - 1) / (kThreads / 64);
    k_field_rhs<<<gb, kThreads, 0, s>>>(t_half, freq, V0, Fh, ni, rhs, d.x_disc, d.x_off, d.nx_of, d.mom,
                                        d.nx_total, d.n);
    k_field_apply<<<gb, kThreads, 0, s>>>(rhs, E, d.x_disc, d.x_off, d.nx_of, d.poisson, d.p_off,
                                          d.nx_total);
    return;
  }
  k_field<<<d.nd, kThreads, 0, s>>>(mode, t_half, freq, a1, V0, Fh, E_given, ni, E, d.x_off, d.nx_of, d.E0_of,
                                    d.xhat, d.mom, d.poisson, d.p_off, d.n);
}

void launch_field_dE0(const DevOps& d, int mode, double t_half, double freq, double a1, const double* gE, double* gE0,
                      hipStream_t s) {
  k_field_dE0<<<d.nd, kThreads, 0, s>>>(mode, t_half, freq, a1, gE, gE0, d.x_off, d.nx_of, d.xhat);
}

void launch_moments(const DevOps& d, const double* F, double* out, hipStream_t s) {
  k_moments<<<d.nx_total, kThreads, 0, s>>>(F, d.mom, out, d.n, d.nx_total);
}

void launch_moments_vjp(const DevOps& d, const double* F, const double* gbar, double* lam, hipStream_t s) {
  k_moments_vjp<<<d.nx_total, kThreads, 0, s>>>(F, d.mom, gbar, lam, d.n, d.nx_total);
}

void launch_maxwellian(const DevOps& d, const double* ne, const double* coeff, double* F, hipStream_t s) {
  const size_t total = (size_t)d.n * d.nx_total;
  const int blocks = static_cast<int>(std::min<size_t>((total + kThreads - 1) / kThreads, 65535));
  k_maxwellian<<<blocks, kThreads, 0, s>>>(ne, coeff, F, d.nr, d.nth, d.nx_total);
}

}  // namespace bte

// Heavies' update of the hybrid model (eq. fluid_step): for every discharge,
//   (n_i^{n+1} - n_i^n)/dt + D_x J_i(E^n, n_i^{n+1}) = (k_i^T F^n) n0 (u^T F^n),
//   J_i = mu_i n_i E - D_i D_x n_i   (eq. hybrid_cnt_a_flux), E = E^n frozen,
// on the CGL collocation points, with the drift outflow condition at the two
// walls (eq. fl_ion_bc, outward normal: J_i . n = n_i max(0, mu_i E . n), no
// inflow) in place of the equation at the wall nodes.  The constant ion
// coefficients are those of the table of modeling parameters (n0 mu_i and
// n0 D_i).  One Nx x Nx dense system per discharge, formed and solved by
// Gaussian elimination with partial pivoting in one block per discharge.
#include <cfloat>
#include <climits>

#include "internal.h"
#include "lu_common.h"

namespace bte {
namespace {

constexpr double kIonN0Mu = 4.65e21;  // n0 mu_i [1/(V m s)]
constexpr double kIonN0D = 2.07e20;   // n0 D_i [1/(m s)]
constexpr int kIonThreads = 256;

// M (column-major, Nx x Nx per discharge) and b of the ion system.  Interior
// rows: I/dt + D_x diag(mu E) - D D_x^2; wall rows: the outflow condition,
// scaled to the size of the interior rows (1/dt) -- an equilibration that does
// not change the solution; b = n_i/dt + n0 (k_i weights . F), 0 at the walls.
__global__ __launch_bounds__(kIonThreads) void k_ion_form(const double* __restrict__ F, const double* __restrict__ ni,
                                                          const double* __restrict__ E, const double* __restrict__ Dx,
                                                          const double* __restrict__ D2,
                                                          const double* __restrict__ kiw,
                                                          const double* __restrict__ n0_of,
                                                          const int* __restrict__ x_off, const int* __restrict__ nx_of,
                                                          const size_t* __restrict__ m_off, double* __restrict__ M,
                                                          double* __restrict__ b, double dt, int n) {
  const int d = blockIdx.x, N = nx_of[d], x0 = x_off[d];
  const double n0 = n0_of[d], mu = kIonN0Mu / n0, D = kIonN0D / n0;
  const double* dx = Dx + m_off[d];   // row-major
  const double* d2 = D2 + m_off[d];
  double* A = M + m_off[d];
  const double e0 = E[x0], eL = E[x0 + N - 1];
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int r = e % N, c = e / N;
    double v;
    if (r == 0) {
      v = D * dx[c] + (c == 0 ? -mu * e0 - fmax(0.0, -mu * e0) : 0.0);
    } else if (r == N - 1) {
      v = -D * dx[(size_t)(N - 1) * N + c] + (c == N - 1 ? mu * eL - fmax(0.0, mu * eL) : 0.0);
    } else {
      v = (r == c ? 1.0 / dt : 0.0) + dx[(size_t)r * N + c] * (mu * E[x0 + c]) - D * d2[(size_t)r * N + c];
    }
    A[e] = v;
  }
  // right-hand side: one wavefront per point
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = w; j < N; j += nw) {
    const double* f = F + (size_t)(x0 + j) * n;
    double s = 0.0;
    for (int c = lane; c < n; c += 64) s += kiw[c] * f[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) b[x0 + j] = (j == 0 || j == N - 1) ? 0.0 : ni[x0 + j] / dt + n0 * s;
  }
  __syncthreads();
  // equilibration of the two wall rows (wavefront 0: row 0, wavefront 1: row N-1)
  if (w < 2) {
    const int r = (w == 0) ? 0 : N - 1;
    double m = 0.0;
    for (int c = lane; c < N; c += 64) m = fmax(m, fabs(A[(size_t)c * N + r]));
    m = wave_max(m);
    const double sc = (m > 0.0) ? 1.0 / (dt * m) : 1.0;
    for (int c = lane; c < N; c += 64) A[(size_t)c * N + r] *= sc;
  }
}

// Gaussian elimination with partial pivoting (max |a|, ties to the lowest row)
// on [M | b] of one discharge, then back substitution; out = n_i^{n+1}.  Per
// column: the pivot by wavefront reductions, the interchange, the multipliers
// and the pivot row staged in LDS, and the trailing update by a 64-row x
// 16-column thread grid (coalesced down the columns); four barriers.
constexpr int kIonSolveThreads = 1024;
__global__ __launch_bounds__(kIonSolveThreads) void k_ion_solve(double* __restrict__ M, double* __restrict__ b,
                                                                double* __restrict__ out,
                                                                const int* __restrict__ x_off,
                                                                const int* __restrict__ nx_of,
                                                                const size_t* __restrict__ m_off,
                                                                int* __restrict__ status) {
  constexpr int NT = kIonSolveThreads, NW = NT / 64;
  const int d = blockIdx.x, N = nx_of[d], x0 = x_off[d];
  double* A = M + m_off[d];
  double* r = b + x0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  extern __shared__ double s_dyn[];
  double* s_l = s_dyn;        // [N] multipliers of the current column
  double* s_u = s_dyn + N;    // [N + 1] pivot row (and its right-hand side)
  __shared__ double s_val[NW];
  __shared__ int s_idx[NW];
  bool singular = false, nonfinite = false;
  for (int k = 0; k < N; ++k) {
    // (a) pivot
    double best = -1.0;
    int bi = INT_MAX;
    for (int i = k + tid; i < N; i += NT) {
      const double v = fabs(A[(size_t)k * N + i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    const double wm = wave_max(best);
    const int wr = wave_min(best == wm ? bi : INT_MAX);
    if (lane == 0) {
      s_val[w] = wm;
      s_idx[w] = wr;
    }
    __syncthreads();
    int p = INT_MAX;
    {
      double v = -1.0;
      for (int u = 0; u < NW; ++u)
        if (s_val[u] > v || (s_val[u] == v && s_idx[u] < p)) {
          v = s_val[u];
          p = s_idx[u];
        }
    }
    if (p == INT_MAX) p = k;  // a column of NaNs keeps row k
    // (b) interchange of rows k and p over columns k.. and the right-hand side
    if (p != k) {
      for (int j = k + tid; j <= N; j += NT) {
        double* x = (j < N) ? A + (size_t)j * N : r;
        const double t = x[k];
        x[k] = x[p];
        x[p] = t;
      }
    }
    __syncthreads();
    // (c) multipliers and the pivot row into LDS
    const double pv = A[(size_t)k * N + k];
    if (pv == 0.0) singular = true;
    if (!(fabs(pv) <= DBL_MAX)) nonfinite = true;
    const int m = N - k - 1;
    for (int i = tid; i < m; i += NT) {
      const double l = (pv != 0.0) ? A[(size_t)k * N + k + 1 + i] / pv : 0.0;
      A[(size_t)k * N + k + 1 + i] = l;
      s_l[i] = l;
    }
    for (int j = tid; j <= m; j += NT) s_u[j] = (j < m) ? A[(size_t)(k + 1 + j) * N + k] : r[k];
    __syncthreads();
    // (d) trailing update of [M | b] (column m of the grid is b)
    {
      const int ti = tid & 63, tj = tid >> 6;
      for (int j = tj; j <= m; j += NW) {
        double* x = (j < m) ? A + (size_t)(k + 1 + j) * N + k + 1 : r + k + 1;
        const double u = s_u[j];
        for (int i = ti; i < m; i += 64) x[i] -= s_l[i] * u;
      }
    }
    __syncthreads();
  }
  // back substitution U x = b
  for (int k = N - 1; k >= 0; --k) {
    const double xk = r[k] / A[(size_t)k * N + k];
    for (int i = tid; i < k; i += NT) r[i] -= A[(size_t)k * N + i] * xk;
    __syncthreads();
    if (tid == 0) r[k] = xk;
  }
  __syncthreads();
  for (int i = tid; i < N; i += NT) out[x0 + i] = r[i];
  if (singular && tid == 0) atomicOr(status, kStSingular);
  if (nonfinite && tid == 0) atomicOr(status, kStNonFinite);
}

}  // namespace

void launch_ion_update(const DevOps& d, const double* F, const double* ni_in, double* ni_out, hipStream_t s) {
  k_ion_form<<<d.nd, kIonThreads, 0, s>>>(F, ni_in, d.ion_E, d.dx, d.dx2, d.mom + 2 * (size_t)d.n, d.n0_of,
                                          d.x_off, d.nx_of, d.p_off, d.ion_M, d.ion_b, d.dt, d.n);
  const size_t sh = (size_t)(2 * d.max_nx + 1) * sizeof(double);
  k_ion_solve<<<d.nd, kIonSolveThreads, sh, s>>>(d.ion_M, d.ion_b, ni_out, d.x_off, d.nx_of, d.p_off, d.status);
}

}  // namespace bte

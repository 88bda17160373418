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
#include <mutex>
#include <type_traits>

#include "internal.h"
#include "lu_common.h"

namespace bte {
namespace {

constexpr double kIonN0Mu = 4.65e21;  // n0 mu_i [1/(V m s)]
constexpr double kIonN0D = 2.07e20;   // n0 D_i [1/(m s)]
constexpr int kIonThreads = 256;

// M (column-major, Nx x Nx per discharge) and b of the ion system.  Interior
// rows: I/dt + D_x diag(mu E) - D D_x^2; wall rows: the outflow condition (the
// solve scales them to the size of the interior rows, 1/dt -- an equilibration
// that does not change the solution); b = n_i/dt + n0 (k_i weights . F), 0 at
// the walls.  Each block forms 8 columns (all rows, from the column-major
// copies of D_x and D_x^2, so that reads and writes run down the columns) and
// the right-hand sides of the same 8 points.
constexpr int kIonFormCols = 8;
__global__ __launch_bounds__(kIonThreads) void k_ion_form(const double* __restrict__ F, const double* __restrict__ ni,
                                                          const double* __restrict__ E, const double* __restrict__ DxT,
                                                          const double* __restrict__ D2T,
                                                          const double* __restrict__ kiw,
                                                          const double* __restrict__ n0_of,
                                                          const int* __restrict__ x_off, const int* __restrict__ nx_of,
                                                          const size_t* __restrict__ m_off, double* __restrict__ M,
                                                          double* __restrict__ b, double dt, int n) {
  const int d = blockIdx.y, N = nx_of[d], x0 = x_off[d];
  const int cb = blockIdx.x * kIonFormCols;
  if (cb >= N) return;
  const int ce = min(N, cb + kIonFormCols);
  const double n0 = n0_of[d], mu = kIonN0Mu / n0, D = kIonN0D / n0;
  const double* dx = DxT + m_off[d];   // column-major: dx[c * N + r] = (D_x)_{rc}
  const double* d2 = D2T + m_off[d];
  double* A = M + m_off[d];
  const double e0 = E[x0], eL = E[x0 + N - 1];
  for (int e = threadIdx.x; e < (ce - cb) * N; e += blockDim.x) {
    const int c = cb + e / N, r = e % N;
    const size_t o = (size_t)c * N + r;
    double v;
    if (r == 0) {
      v = D * dx[o] + (c == 0 ? -mu * e0 - fmax(0.0, -mu * e0) : 0.0);
    } else if (r == N - 1) {
      v = -D * dx[o] + (c == N - 1 ? mu * eL - fmax(0.0, mu * eL) : 0.0);
    } else {
      v = (r == c ? 1.0 / dt : 0.0) + dx[o] * (mu * E[x0 + c]) - D * d2[o];
    }
    A[o] = v;
  }
  // right-hand sides: one wavefront per point
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = cb + w; j < ce; j += nw) {
    const double* f = F + (size_t)(x0 + j) * n;
    double s = 0.0;
    for (int c = lane; c < n; c += 64) s += kiw[c] * f[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) b[x0 + j] = (j == 0 || j == N - 1) ? 0.0 : ni[x0 + j] / dt + n0 * s;
  }
}

constexpr int kIonSolveThreads = 1024;
// Gaussian elimination with partial pivoting (max |a|, ties to the lowest row)
// on [M | b] of one discharge in one block, blocked: panels of W columns factored in LDS
// (pivot, interchange, multipliers and the panel's own update per column, all
// on the LDS copy), then for the columns outside the panel and b the panel's
// interchanges as one gather / scatter, U12 by substitution with the panel's
// unit lower block, and one rank-W update of the trailing matrix and b.  The
// trailing matrix is read and written once per panel instead of once per
// column; the pivots (max |a|, ties to the lowest row) are those of the
// unblocked kernel.
template <int W>
__global__ __launch_bounds__(kIonSolveThreads) void k_ion_solve_blk(double* __restrict__ M, double* __restrict__ b,
                                                                    double* __restrict__ out,
                                                                    const int* __restrict__ x_off,
                                                                    const int* __restrict__ nx_of,
                                                                    const size_t* __restrict__ m_off,
                                                                    int* __restrict__ status, int ldp, double dt) {
  constexpr int NT = kIonSolveThreads, NW = NT / 64;
  const int d = blockIdx.x, N = nx_of[d], x0 = x_off[d];
  double* A = M + m_off[d];
  double* r = b + x0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  extern __shared__ double s_dyn[];
  double* sP = s_dyn;              // [W][ldp]: the panel, column-major (rows 0..N-1)
  double* sU = s_dyn + W * ldp;    // [ldp + 1][W]: U12 rows of every column outside the panel, and of b
  __shared__ double s_val[NW];
  __shared__ int s_idx[NW];
  __shared__ int s_piv[W];
  __shared__ int s_R[2 * W], s_src[2 * W];
  __shared__ int s_nR;
  bool singular = false, nonfinite = false;
  auto col = [&](int c) { return c < N ? A + (size_t)c * N : r; };   // column N is b
  // equilibration of the two wall rows (wavefront 0: row 0, wavefront 1: row
  // N-1) to the size of the interior rows; their right-hand sides are 0
  if (w < 2) {
    const int rr = (w == 0) ? 0 : N - 1;
    double m = 0.0;
    for (int c = lane; c < N; c += 64) m = fmax(m, fabs(A[(size_t)c * N + rr]));
    m = wave_max(m);
    const double sc = (m > 0.0) ? 1.0 / (dt * m) : 1.0;
    for (int c = lane; c < N; c += 64) A[(size_t)c * N + rr] *= sc;
  }
  __syncthreads();
  for (int k0 = 0; k0 < N; k0 += W) {
    const int wd = min(W, N - k0);
    // (1) the panel into LDS and its factorization there
    for (int e = tid; e < wd * N; e += NT) {
      const int j = e / N, i = e % N;
      if (i >= k0) sP[j * ldp + i] = A[(size_t)(k0 + j) * N + i];
    }
    __syncthreads();
    for (int j = 0; j < wd; ++j) {
      const int c = k0 + j;
      double* pc = sP + j * ldp;
      double best = -1.0;
      int bi = INT_MAX;
      for (int i = c + tid; i < N; i += NT) {
        const double v = fabs(pc[i]);
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
      if (p == INT_MAX) p = c;  // a column of NaNs keeps row c
      if (p != c && tid < wd) {
        double* q = sP + tid * ldp;
        const double t = q[c];
        q[c] = q[p];
        q[p] = t;
      }
      if (tid == 0) s_piv[j] = p;
      __syncthreads();
      const double pv = pc[c];
      if (pv == 0.0) singular = true;
      if (!(fabs(pv) <= DBL_MAX)) nonfinite = true;
      for (int i = c + 1 + tid; i < N; i += NT) pc[i] = (pv != 0.0) ? pc[i] / pv : 0.0;
      __syncthreads();
      // the panel's columns to the right of c
      const int m = N - c - 1, nr = wd - j - 1;
      for (int e = tid; e < m * nr; e += NT) {
        const int i = c + 1 + e % m, jj = j + 1 + e / m;
        sP[jj * ldp + i] -= pc[i] * sP[jj * ldp + c];
      }
      __syncthreads();
    }
    for (int e = tid; e < wd * N; e += NT) {
      const int j = e / N, i = e % N;
      if (i >= k0) A[(size_t)(k0 + j) * N + i] = sP[j * ldp + i];
    }
    // (2) the panel's interchanges as a list of touched rows and their sources
    if (tid == 0) {
      int nR = wd;
      for (int t = 0; t < wd; ++t) {
        s_R[t] = k0 + t;
        s_src[t] = k0 + t;
      }
      for (int j = 0; j < wd; ++j) {
        const int a = k0 + j, pj = s_piv[j];
        if (pj == a) continue;
        int ia = -1, ip = -1;
        for (int t = 0; t < nR; ++t) {
          if (s_R[t] == a) ia = t;
          if (s_R[t] == pj) ip = t;
        }
        if (ip < 0) {
          ip = nR++;
          s_R[ip] = pj;
          s_src[ip] = pj;
        }
        const int tmp = s_src[ia];
        s_src[ia] = s_src[ip];
        s_src[ip] = tmp;
      }
      s_nR = nR;
    }
    __syncthreads();
    // (3) the interchanges on every column outside the panel and on b: all
    // reads, then all writes
    const int nR = s_nR, nc = N + 1 - wd;
    // at most 2 W touched rows of at most NMAX + 1 columns (NMAX the largest Nx
    // this panel width is launched for)
    constexpr int NMAX = W == 32 ? 256 : (W == 16 ? 512 : 1024);
    constexpr int NV = (2 * W * (NMAX + 1) + NT - 1) / NT;
    double v[NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = tid + u * NT;
      if (e < nR * nc) {
        const int t = e % nR, cc = e / nR, cg = cc < k0 ? cc : cc + wd;
        v[u] = col(cg)[s_src[t]];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = tid + u * NT;
      if (e < nR * nc) {
        const int t = e % nR, cc = e / nR, cg = cc < k0 ? cc : cc + wd;
        if (s_src[t] != s_R[t]) col(cg)[s_R[t]] = v[u];
      }
    }
    __syncthreads();
    // (4) U12 = L11^-1 A12 for the columns after the panel and b (thread per column)
    const int c1 = k0 + wd, ncols = N + 1 - c1;
    for (int cc = tid; cc < ncols; cc += NT) {
      double* q = col(c1 + cc);
      double x[W];
#pragma unroll
      for (int t = 0; t < W; ++t) x[t] = t < wd ? q[k0 + t] : 0.0;
#pragma unroll
      for (int t = 1; t < W; ++t)
#pragma unroll
        for (int k = 0; k < t; ++k)
          if (t < wd) x[t] -= sP[k * ldp + k0 + t] * x[k];
#pragma unroll
      for (int t = 0; t < W; ++t)
        if (t < wd) {
          q[k0 + t] = x[t];
          sU[cc * W + t] = x[t];
        }
    }
    __syncthreads();
    // (5) rank-wd update of the trailing matrix and b: lanes down the rows,
    // wavefronts across the columns
    const int mr = N - c1;
    for (int cc = w; cc < ncols; cc += NW) {
      double* q = col(c1 + cc);
      const double* u = sU + cc * W;
      for (int i = c1 + lane; i < N; i += 64) {
        double s = 0.0;
        for (int t = 0; t < wd; ++t) s += sP[t * ldp + i] * u[t];
        q[i] -= s;
      }
    }
    (void)mr;
    __syncthreads();
  }
  // back substitution U x = b by blocks of 16 rows from the bottom, b in LDS:
  // one wavefront solves a block (values passed by lane reads), then every
  // thread subtracts the block's columns from the rows above, in the same
  // order as a column-by-column substitution
  constexpr int BS = 16;
  double* sr = sU;   // the U12 staging is free now; (ldp + 1) W >= N doubles
  for (int i = tid; i < N; i += NT) sr[i] = r[i];
  __syncthreads();
  for (int b1 = N; b1 > 0; b1 -= BS) {
    const int b0 = max(0, b1 - BS), nb = b1 - b0;
    if (w == 0) {
      const bool own = lane < nb;
      double v = own ? sr[b0 + lane] : 0.0;
      double u[BS];
#pragma unroll
      for (int t = 0; t < BS; ++t) u[t] = (own && t < nb && t >= lane) ? A[(size_t)(b0 + t) * N + b0 + lane] : 0.0;
#pragma unroll
      for (int t = BS - 1; t >= 0; --t) {
        if (t < nb) {
          if (lane == t) v = v / u[t];
          const double xt = readlane_f64(v, t);
          if (lane < t) v -= u[t] * xt;
        }
      }
      if (own) sr[b0 + lane] = v;
    }
    __syncthreads();
    for (int i = tid; i < b0; i += NT) {
      double ri = sr[i];
      for (int j = b1 - 1; j >= b0; --j) ri -= A[(size_t)j * N + i] * sr[j];
      sr[i] = ri;
    }
    __syncthreads();
  }
  for (int i = tid; i < N; i += NT) out[x0 + i] = sr[i];
  if (singular && tid == 0) atomicOr(status, kStSingular);
  if (nonfinite && tid == 0) atomicOr(status, kStNonFinite);
}

}  // namespace

void launch_ion_update_ws(const DevOps& d, const double* F, const double* ni_in, double* ni_out, double* M, double* b,
                          const double* E, hipStream_t s) {
  const dim3 gf((d.max_nx + kIonFormCols - 1) / kIonFormCols, d.nd);
  k_ion_form<<<gf, kIonThreads, 0, s>>>(F, ni_in, E, d.dxT, d.dx2, d.mom + 2 * (size_t)d.n, d.n0_of, d.x_off,
                                        d.nx_of, d.p_off, M, b, d.dt, d.n);
  // blocked elimination, panel width by the largest Nx (two W x Nx tiles of LDS)
  const int ldp = d.max_nx + 1;
  auto blk = [&](auto wc) {
    constexpr int W = decltype(wc)::value;
    const size_t sh = (size_t)(W * ldp + (ldp + 1) * W) * sizeof(double);
    k_ion_solve_blk<W><<<d.nd, kIonSolveThreads, sh, s>>>(M, b, ni_out, d.x_off, d.nx_of, d.p_off, d.status, ldp,
                                                         d.dt);
  };
  if (d.max_nx <= 512) blk(std::integral_constant<int, 16>{});
  else blk(std::integral_constant<int, 8>{});
}

void launch_ion_update(const DevOps& d, const double* F, const double* ni_in, double* ni_out, hipStream_t s) {
  launch_ion_update_ws(d, F, ni_in, ni_out, d.ion_M, d.ion_b, d.ion_E, s);
}

// Scratch of the allocation-free ion step: one copy per GPU, alive until the
// process ends.  Host code never uses the array's name as an address; it takes
// the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kIonScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t ion_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    double* p = nullptr;
    e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace bte

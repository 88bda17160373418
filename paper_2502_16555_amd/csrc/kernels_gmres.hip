// Krylov form of the velocity-space step (the paper's own V solver): the Nx
// systems of eq. (vspace_batched_system) solved by restarted GMRES, batched
// over the collocation points (one Krylov space per point), right-
// preconditioned with the field-binned operators of the velocity-space
// preconditioner (Alg. vspace_action_precon): the field range (-E0, E0) is
// split into Nc bins and H_p = (I - dt (n0 C + s_p A))^-1 with s_p the bin
// centre.  H_p is applied as the triangular solves of its LU factors (factored
// once per setup by the batched LU), so each point only needs the index of its
// bin (set once per step from the field).
//
// Per iteration: z = H_{w(x)} v_j (k_solve with the bin map), w = M z (MFMA
// operator action, Alg. vspace_action), then this file's k_gmres_arnoldi: two
// passes of classical Gram-Schmidt against v_0..v_j (one block per point),
// the new basis vector, and the Givens rotation of the Hessenberg column with
// the point's convergence test.  Converged points stop updating (flags), so the
// host issues a fixed sequence of launches with no synchronization.
#include <cmath>

#include "internal.h"

namespace bte {
namespace {

constexpr int kThreads = 256;

__device__ inline double block_sum(double v, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int u = 0; u < kThreads / 64; ++u) t += red[u];
  return t;
}

// bin of every point: p = clamp(floor((u(E) - S0) / width)) with u(E) = E, or
// asinh(E / scale) for bins graded towards zero field; factor set of its
// discharge d: d * nbins + p
__global__ void k_bin_map(const double* __restrict__ E, const int* __restrict__ x_disc, int* __restrict__ mat_of,
                          double S0, double width, double scale, int nbins, int nx) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  const double u = (scale > 0.0) ? asinh(E[x] / scale) : E[x];
  const double f = floor((u - S0) / width);
  int p = (f == f) ? static_cast<int>(fmin(fmax(f, 0.0), static_cast<double>(nbins - 1))) : 0;
  mat_of[x] = x_disc[x] * nbins + p;
}

// Start of a cycle: r = b - M x in R.  beta = ||r||, v_0 = r / beta, g = beta e_0;
// on the first cycle also ||b|| (the reference of the relative tolerance).  A
// point whose residual already meets the tolerance is marked converged; inact
// records the points that take no part in this cycle.
__global__ __launch_bounds__(kThreads) void k_gmres_init(const double* __restrict__ R, const double* __restrict__ B,
                                                         double* __restrict__ V0, double* __restrict__ g,
                                                         double* __restrict__ bnorm, int* __restrict__ conv,
                                                         int* __restrict__ inact, int* __restrict__ kcount,
                                                         int* __restrict__ ktot, double* __restrict__ rest,
                                                         double rtol, int first, int npad, int m) {
  __shared__ double red[kThreads / 64];
  const int x = blockIdx.x, tid = threadIdx.x;
  const double* r = R + (size_t)x * npad;
  double s = 0.0, sb = 0.0;
  for (int i = tid; i < npad; i += kThreads) {
    s += r[i] * r[i];
    if (first) sb += B[(size_t)x * npad + i] * B[(size_t)x * npad + i];
  }
  const double beta = sqrt(block_sum(s, red));
  double bn = 0.0;
  if (first) bn = sqrt(block_sum(sb, red));
  if (tid == 0) {
    if (first) {
      bnorm[x] = bn;
      conv[x] = 0;
      ktot[x] = 0;
    }
    kcount[x] = 0;
  }
  __syncthreads();
  const double ref = first ? bn : bnorm[x];
  const bool before = first ? false : (conv[x] != 0);   // converged in an earlier cycle
  const bool done = before || !(beta > rtol * ref);
  if (tid == 0) {
    conv[x] = done ? 1 : 0;
    inact[x] = done ? 1 : 0;
    g[(size_t)x * (m + 1)] = beta;
    // residual estimate: only points taking part (R is not formed for the others)
    if (!before) rest[x] = beta / (ref > 0.0 ? ref : 1.0);
  }
  const double inv = (beta > 0.0) ? 1.0 / beta : 0.0;
  double* v = V0 + (size_t)x * npad;
  for (int i = tid; i < npad; i += kThreads) v[i] = done ? 0.0 : r[i] * inv;
}

// Iteration j: W holds M z_j.  Orthogonalize against v_0..v_j (classical
// Gram-Schmidt, twice), v_{j+1} = w / ||w||, then the Givens update of column j
// of the point's Hessenberg matrix and the residual estimate |g_{j+1}|.
__global__ __launch_bounds__(kThreads) void k_gmres_arnoldi(double* __restrict__ W, double* __restrict__ V,
                                                            double* __restrict__ H, double* __restrict__ cs,
                                                            double* __restrict__ sn, double* __restrict__ g,
                                                            const double* __restrict__ bnorm, int* __restrict__ conv,
                                                            int* __restrict__ kcount, int* __restrict__ ktot,
                                                            double* __restrict__ rest, double rtol, int j, int nxt,
                                                            int npad, int m) {
  const int x = blockIdx.x, tid = threadIdx.x;
  if (conv[x]) return;
  __shared__ double red[kThreads / 64];
  __shared__ double hcol[64];
  double* w = W + (size_t)x * npad;
  const size_t vs = (size_t)nxt * npad;      // stride between basis vectors
  const double* vx = V + (size_t)x * npad;
  if (tid <= j) hcol[tid] = 0.0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = 0; i <= j; ++i) {            // h_i = <w, v_i>
      const double* vi = vx + (size_t)i * vs;
      double s = 0.0;
      for (int e = tid; e < npad; e += kThreads) s += w[e] * vi[e];
      s = block_sum(s, red);
      if (tid == 0) hcol[i] += s;
      __syncthreads();
      for (int e = tid; e < npad; e += kThreads) w[e] -= s * vi[e];
      __syncthreads();
    }
  }
  double s = 0.0;
  for (int e = tid; e < npad; e += kThreads) s += w[e] * w[e];
  const double hn = sqrt(block_sum(s, red));
  const double inv = (hn > 0.0) ? 1.0 / hn : 0.0;
  double* vn = V + (size_t)(j + 1) * vs + (size_t)x * npad;
  for (int e = tid; e < npad; e += kThreads) vn[e] = w[e] * inv;
  if (tid == 0) {
    double* Hx = H + (size_t)x * (m + 1) * m;   // column-major (m+1) x m
    double* c = cs + (size_t)x * m;
    double* sx = sn + (size_t)x * m;
    double* gx = g + (size_t)x * (m + 1);
    double col[65];
    for (int i = 0; i <= j; ++i) col[i] = hcol[i];
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {             // previous rotations
      const double a = c[i] * col[i] + sx[i] * col[i + 1];
      col[i + 1] = -sx[i] * col[i] + c[i] * col[i + 1];
      col[i] = a;
    }
    const double r = hypot(col[j], col[j + 1]);
    const double cj = (r > 0.0) ? col[j] / r : 1.0, sj = (r > 0.0) ? col[j + 1] / r : 0.0;
    c[j] = cj;
    sx[j] = sj;
    col[j] = r;
    col[j + 1] = 0.0;
    for (int i = 0; i <= j + 1; ++i) Hx[(size_t)j * (m + 1) + i] = col[i];
    const double gj = gx[j];
    gx[j] = cj * gj;
    gx[j + 1] = -sj * gj;
    kcount[x] = j + 1;
    ktot[x] += 1;
    rest[x] = fabs(gx[j + 1]) / (bnorm[x] > 0.0 ? bnorm[x] : 1.0);
    if (!(fabs(gx[j + 1]) > rtol * bnorm[x]) || hn == 0.0) conv[x] = 1;
  }
}

// End of a cycle: y = R^-1 g (the rotated Hessenberg matrix, k x k) and
// Z = V_k y for the points that took part in the cycle.
__global__ __launch_bounds__(kThreads) void k_gmres_combine(const double* __restrict__ V, const double* __restrict__ H,
                                                            const double* __restrict__ g,
                                                            const int* __restrict__ inact,
                                                            const int* __restrict__ kcount, double* __restrict__ Z,
                                                            int nxt, int npad, int m) {
  const int x = blockIdx.x, tid = threadIdx.x;
  if (inact[x]) return;
  __shared__ double y[64];
  const int k = kcount[x];
  if (tid == 0) {
    const double* Hx = H + (size_t)x * (m + 1) * m;
    const double* gx = g + (size_t)x * (m + 1);
    for (int i = k - 1; i >= 0; --i) {
      double t = gx[i];
      for (int l = i + 1; l < k; ++l) t -= Hx[(size_t)l * (m + 1) + i] * y[l];
      const double d = Hx[(size_t)i * (m + 1) + i];
      y[i] = (d != 0.0) ? t / d : 0.0;
    }
  }
  __syncthreads();
  const size_t vs = (size_t)nxt * npad;
  double* z = Z + (size_t)x * npad;
  for (int e = tid; e < npad; e += kThreads) {
    double t = 0.0;
    for (int i = 0; i < k; ++i) t += V[(size_t)i * vs + (size_t)x * npad + e] * y[i];
    z[e] = t;
  }
}

// Status: any point not converged after the last cycle -> no convergence (a
// non-finite estimate -> non-finite); resid[0] = max_x of the points' last
// relative residual estimates, status[2] = the largest iteration count.
__global__ void k_gmres_status(const int* __restrict__ conv, const int* __restrict__ ktot,
                               const double* __restrict__ rest, int* __restrict__ status, double* __restrict__ resid,
                               int nx) {
  __shared__ double red[256];
  __shared__ int redi[256];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double worst = 0.0;
  int it = 0;
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    const double est = rest[x];
    worst = fmax(worst, (est == est) ? est : INFINITY);
    it = max(it, ktot[x]);
    if (!conv[x]) bad = 1;
  }
  red[threadIdx.x] = worst;
  redi[threadIdx.x] = it;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
      redi[threadIdx.x] = max(redi[threadIdx.x], redi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    resid[0] = red[0];
    status[2] = redi[0];
    if (bad) atomicOr(status, kStNoConv);
    if (!(red[0] <= 1.0e300)) atomicOr(status, kStNonFinite);
  }
}

}  // namespace

void launch_bin_map(const DevOps& d, const GmresOps& q, hipStream_t s) {
  k_bin_map<<<(d.nx_total + 255) / 256, 256, 0, s>>>(d.E, d.x_disc, q.mat_of, q.S0, q.width, q.scale, q.nbins,
                                                      d.nx_total);
}

void launch_gmres_init(const DevOps& d, const GmresOps& q, bool first, hipStream_t s) {
  k_gmres_init<<<d.nx_total, kThreads, 0, s>>>(q.R, d.B, q.V, q.g, q.bnorm, q.conv, q.inact, q.kcount, q.ktot,
                                               q.rest, q.rtol, first ? 1 : 0, d.npad, q.m);
}

void launch_gmres_arnoldi(const DevOps& d, const GmresOps& q, int j, hipStream_t s) {
  k_gmres_arnoldi<<<d.nx_total, kThreads, 0, s>>>(q.W, q.V, q.H, q.cs, q.sn, q.g, q.bnorm, q.conv, q.kcount,
                                                  q.ktot, q.rest, q.rtol, j, d.nx_total, d.npad, q.m);
}

void launch_gmres_combine(const DevOps& d, const GmresOps& q, hipStream_t s) {
  k_gmres_combine<<<d.nx_total, kThreads, 0, s>>>(q.V, q.H, q.g, q.inact, q.kcount, q.Z, d.nx_total, d.npad, q.m);
}

void launch_gmres_status(const DevOps& d, const GmresOps& q, hipStream_t s) {
  k_gmres_status<<<1, 256, 0, s>>>(q.conv, q.ktot, q.rest, d.status, d.resid, d.nx_total);
}

}  // namespace bte

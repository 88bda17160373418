// FP64 refinement of the mixed-precision V step and the adjoint gradient
// contractions.  The residual r = b - (I - dt (n0 C + E A)) x is the operator
// action of Alg. vspace_action of the paper evaluated in FP64 with MFMA f64;
// the refinement x += LU^-1 r repeats until max|r| <= rtol max|b| (a device
// flag stops the remaining sweeps without a host synchronization).
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace bte {
namespace {

using f64x4 = double __attribute__((ext_vector_type(4)));

// Result row of item t of lane group lk for MFMA f64 16x16x4 (measured layout).
__device__ inline int f64_row(int lk, int t) { return lk + 4 * t; }

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

// Ordinates <-> harmonics of every point: harmonic coefficients
// Bh[l * nr + k] = sum_a TS[l][a] F[k][a] (P_S of eq. (proj_ops), l-major, padded
// rows of npad, l < nl) and back.  With nl = nth, P_O P_S = I and the way back is
// F[k][a] = sum_l TO[a][l] Xh[l * nr + k] (P_O).  With nl < nth the operator part
// of the V system has rank nr nl, (I - P_O K P_S)^-1 = I - P_O P_S + P_O (I - K)^-1 P_S
// (T_S T_O = I_nl), so the way back adds the solution's harmonic change to the
// state: F[k][a] += sum_l TO[a][l] (Xh - Bh)[l * nr + k].
__global__ __launch_bounds__(256) void k_to_harm(const double* __restrict__ F, const double* __restrict__ TS,
                                                 double* __restrict__ Bh, int nr, int nth, int nl, int npad) {
  extern __shared__ double sh[];
  const int n = nr * nth, x = blockIdx.x;
  double* sF = sh;
  double* sT = sh + n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) sF[i] = F[(size_t)x * n + i];
  for (int i = threadIdx.x; i < nl * nth; i += blockDim.x) sT[i] = TS[i];
  __syncthreads();
  for (int o = threadIdx.x; o < npad; o += blockDim.x) {
    double v = 0.0;
    if (o < nr * nl) {
      const int l = o / nr, k = o % nr;
      for (int a = 0; a < nth; ++a) v += sT[l * nth + a] * sF[k * nth + a];
    }
    Bh[(size_t)x * npad + o] = v;
  }
}

__global__ __launch_bounds__(256) void k_from_harm(const double* __restrict__ Xh, const double* __restrict__ Bh,
                                                   const double* __restrict__ TO, double* __restrict__ F, int nr,
                                                   int nth, int nl, int npad) {
  extern __shared__ double sh[];
  const int n = nr * nth, nhm = nr * nl, x = blockIdx.x;
  const bool reduced = nl < nth;
  double* sX = sh;
  double* sT = sh + nhm;
  for (int i = threadIdx.x; i < nhm; i += blockDim.x)
    sX[i] = reduced ? Xh[(size_t)x * npad + i] - Bh[(size_t)x * npad + i] : Xh[(size_t)x * npad + i];
  for (int i = threadIdx.x; i < nth * nl; i += blockDim.x) sT[i] = TO[i];
  __syncthreads();
  for (int o = threadIdx.x; o < n; o += blockDim.x) {
    const int k = o / nth, a = o % nth;
    double v = 0.0;
    for (int l = 0; l < nl; ++l) v += sT[a * nl + l] * sX[l * nr + k];
    F[(size_t)x * n + o] = reduced ? F[(size_t)x * n + o] + v : v;
  }
}

// ---------------------------------------------------------------------------
// FP64 residual R = B - X + dt n0_x (X C^T) + dt E_x (X A^T)  (TRANSPOSE: C, A)
// rows = collocation points, 32 x 64 output tiles, MFMA f64 16x16x4; eight
// wavefronts per tile, each 16 points x 16 outputs, two per SIMD so that one
// wave's LDS reads overlap the other's products.
// ---------------------------------------------------------------------------
// MODE 0: the refinement residual above, with the per-point maxima (skipped once
// the refinement is done); MODE 1: R = B - M X only; MODE 2: R = M X (operator
// action of Alg. vspace_action, for the Krylov solver); MODE 3: R = B - dt E (X A^T)
// (the field-coupling term of the fully implicit Jacobian, eq. 1dbte_jac_action).
constexpr int kResThreads = 512;

template <int TRANSPOSE, int MODE = 0>
__global__ __launch_bounds__(kResThreads) void k_residual(const double* __restrict__ Bv, const double* __restrict__ Xv,
                                                  double* __restrict__ Rv, const double* __restrict__ C,
                                                  const double* __restrict__ Aop, const double* __restrict__ E,
                                                  const double* __restrict__ n0x, unsigned long long* __restrict__ rmax,
                                                  unsigned long long* __restrict__ bmax,
                                                  unsigned long long* __restrict__ xmax, const int* __restrict__ status,
                                                  double dt, int n, int npad, int nx, const int* __restrict__ skip) {
  if (MODE == 0 && status[1]) return;
  constexpr int BM = 32, BN = 64, BK = 64;
  if (MODE != 0 && skip) {  // points already converged need no operator action
    bool all = true;
    for (int u = 0; u < BM; ++u) {
      const int x = blockIdx.y * BM + u;
      if (x < nx && !skip[x]) all = false;
    }
    if (all) return;
  }
  constexpr int NT = kResThreads;
  constexpr int LX = BM * BK / NT, LO = BN * BK / NT;  // loads per thread and tile
  __shared__ double sX[BM][BK + 1];
  __shared__ double sC[BN][BK + 1];
  __shared__ double sA[BN][BK + 1];
  __shared__ unsigned long long s_rm[4][BM], s_bm[4][BM], s_xm[4][BM];
  const int x0 = blockIdx.y * BM, i0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = (tid >> 6) & 3, b = tid >> 8;   // outputs 16 w.., points 16 b..
  const int li = lane & 15, lk = lane >> 4;
  // operator element e of a tile: row r (output index i), column c (k); the
  // transposed form walks i fastest so that its loads stay coalesced
  auto op_rc = [&](int e, int* r, int* c) {
    if (TRANSPOSE) {
      *r = e % BN;
      *c = e / BN;
    } else {
      *r = e / BK;
      *c = e % BK;
    }
  };
  double px[LX], pc[LO], pa[LO];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < LX; ++u) {
      const int e = tid + NT * u, r = e / BK, c = e % BK;
      px[u] = (x0 + r < nx && k0 + c < n) ? Xv[(size_t)(x0 + r) * npad + k0 + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < LO; ++u) {
      int r, c;
      op_rc(tid + NT * u, &r, &c);
      const int i = i0 + r, k = k0 + c;
      double cv = 0.0, av = 0.0;
      if (i < n && k < n) {
        const size_t o = TRANSPOSE ? (size_t)k * n + i : (size_t)i * n + k;
        cv = C[o];
        av = Aop[o];
      }
      pc[u] = cv;
      pa[u] = av;
    }
  };
  f64x4 accC = f64x4{0, 0, 0, 0}, accA = f64x4{0, 0, 0, 0};
  fetch(0);
  for (int k0 = 0; k0 < n; k0 += BK) {
#pragma unroll
    for (int u = 0; u < LX; ++u) {
      const int e = tid + NT * u;
      sX[e / BK][e % BK] = px[u];
    }
#pragma unroll
    for (int u = 0; u < LO; ++u) {
      int r, c;
      op_rc(tid + NT * u, &r, &c);
      sC[r][c] = pc[u];
      sA[r][c] = pa[u];
    }
    __syncthreads();
    if (k0 + BK < n) fetch(k0 + BK);  // next tile in flight during the products
#pragma unroll 4
    for (int k = 0; k < BK; k += 4) {
      const double bc = sC[w * 16 + li][k + lk];
      const double ba = sA[w * 16 + li][k + lk];
      const double ax = sX[b * 16 + li][k + lk];
      accC = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, bc, accC, 0, 0, 0);
      accA = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, ba, accA, 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue: residual, then max |r| and max |b| per point, reduced over the
  // block before one atomic per point (bit patterns of non-negative doubles
  // order like the values, and a NaN orders above +inf)
  {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int xl = b * 16 + f64_row(lk, it);
      const int x = x0 + xl;
      const int i = i0 + w * 16 + li;
      unsigned long long rb = 0ull, bb = 0ull, xb = 0ull;
      if (MODE != 0) {
        if (x < nx && i < n) {
          const size_t o = (size_t)x * npad + i;
          if (MODE == 3) {
            Rv[o] = Bv[o] - dt * E[x] * accA[it];
          } else {
            const double mx = Xv[o] - dt * n0x[x] * accC[it] - dt * E[x] * accA[it];
            Rv[o] = (MODE == 1) ? Bv[o] - mx : mx;
          }
        }
        continue;
      }
      if (x < nx && i < n) {
        const size_t o = (size_t)x * npad + i;
        const double bv = Bv[o], xv = Xv[o];
        const double r = bv - xv + dt * n0x[x] * accC[it] + dt * E[x] * accA[it];
        Rv[o] = r;
        rb = static_cast<unsigned long long>(__double_as_longlong(fabs(r)));
        bb = static_cast<unsigned long long>(__double_as_longlong(fabs(bv)));
        xb = static_cast<unsigned long long>(__double_as_longlong(fabs(xv)));
      }
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const unsigned long long orb = __shfl_xor(rb, off), obb = __shfl_xor(bb, off), oxb = __shfl_xor(xb, off);
        rb = orb > rb ? orb : rb;
        bb = obb > bb ? obb : bb;
        xb = oxb > xb ? oxb : xb;
      }
      if (li == 0) {
        s_rm[w][xl] = rb;
        s_bm[w][xl] = bb;
        s_xm[w][xl] = xb;
      }
    }
  }
  if (MODE != 0) return;
  __syncthreads();
  if (tid < BM && x0 + tid < nx) {
    unsigned long long rb = 0ull, bb = 0ull, xb = 0ull;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      rb = s_rm[u][tid] > rb ? s_rm[u][tid] : rb;
      bb = s_bm[u][tid] > bb ? s_bm[u][tid] : bb;
      xb = s_xm[u][tid] > xb ? s_xm[u][tid] : xb;
    }
    atomicMax(&rmax[x0 + tid], rb);
    atomicMax(&bmax[x0 + tid], bb);
    atomicMax(&xmax[x0 + tid], xb);
  }
}

// Stop test of the refinement: the normwise backward error of every point,
//   eta_x = max|r_x| / (||M_x|| max|x_x| + max|b_x|),
// with ||M_x|| <= 1 + dt (n0_x ||C|| + |E_x| ||A||) in the norm that matches
// max-norms of the vectors (inf-norm for M, 1-norm for M^T).  The residual's own
// FP64 rounding is of order sqrt(n) eps ||M|| |x|, so a bound relative to |b|
// alone is unreachable once dt |E| ||A|| grows; eta is not.
// status[1] = done flag, status[2] = sweeps used; resid[0] = max_x eta_x.
__global__ void k_refine_check(unsigned long long* __restrict__ rmax, unsigned long long* __restrict__ bmax,
                               unsigned long long* __restrict__ xmax, const double* __restrict__ E,
                               const double* __restrict__ n0x, double dt, double cnorm, double anorm,
                               int* __restrict__ status, double* __restrict__ resid, double rtol, int sweep,
                               int final_sweep, int nx) {
  if (status[1]) return;
  __shared__ double red[256];
  double worst = 0.0;
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    const double r = __longlong_as_double(static_cast<long long>(rmax[x]));
    const double b = __longlong_as_double(static_cast<long long>(bmax[x]));
    const double xm = __longlong_as_double(static_cast<long long>(xmax[x]));
    const double mn = 1.0 + dt * (n0x[x] * cnorm + fabs(E[x]) * anorm);
    const double den = mn * xm + b;
    const double q = (den > 0.0) ? r / den : (r > 0.0 ? INFINITY : 0.0);
    worst = fmax(worst, (q == q) ? q : INFINITY);
    rmax[x] = 0ull;
    bmax[x] = 0ull;
    xmax[x] = 0ull;
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

__global__ void k_reset_refine(unsigned long long* rmax, unsigned long long* bmax, unsigned long long* xmax,
                               int* status, int nx) {
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    rmax[x] = 0ull;
    bmax[x] = 0ull;
    xmax[x] = 0ull;
  }
  if (threadIdx.x == 0) {
    status[1] = 0;
    status[2] = 0;
  }
}

// grad_scal[op] += dt sum_x n0_x mu_x^T C^(op) F*_x  and  grad_E[x] = dt mu_x^T A F*_x.
// Tiled like the residual: out[x][i] = sum_k F*[x][k] M[i][k] (MFMA f64), then the
// epilogue contracts with mu[x][i].  Grid: (gx = n/64, gy = ceil(nx/32), n_params + 1).
// Every block writes its partial sums to slots of its own (no atomics), and
// k_adjoint_reduce adds the slots in a fixed order, so the gradients are the same
// bit for bit from run to run:
//   pscal[(op * gy + by) * gx + bx]  = dt sum_{x in block} n0_x (mu_x . out_x)   (op < n_params)
//   pE[x * gx + bx]                  = dt (mu_x . out_x) over the block's i range  (op = n_params)
__global__ __launch_bounds__(256) void k_adjoint_grads(const double* __restrict__ Mu, const double* __restrict__ Fs,
                                                       const double* __restrict__ Csb, const double* __restrict__ Aop,
                                                       const double* __restrict__ n0x, double* __restrict__ pscal,
                                                       double* __restrict__ pE, double dt, int n, int nx, int nparams) {
  constexpr int BM = 32, BN = 64, BK = 64;
  const int op = blockIdx.z;
  const double* M = (op < nparams) ? Csb + (size_t)op * n * n : Aop;
  __shared__ double sX[BM][BK + 1];
  __shared__ double sM[BN][BK + 1];
  __shared__ double sRed[4][BM];
  const int x0 = blockIdx.y * BM, i0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
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
  // contract with mu: each wave reduces its 16 rows i for each of the 32 points
  // (lanes of the same lk hold one point) and writes one slot per point
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int xl = b * 16 + f64_row(lk, it);
      const int x = x0 + xl;
      const int i = i0 + w * 16 + li;
      double v = (x < nx && i < n) ? Mu[(size_t)x * n + i] * acc[b][it] : 0.0;
      for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (li == 0) sRed[w][xl] = v;
    }
  __syncthreads();
  const size_t gx = gridDim.x, gy = gridDim.y;
  if (op < nparams) {
    if (tid == 0) {
      double total = 0.0;
      for (int xl = 0; xl < BM && x0 + xl < nx; ++xl)
        total += dt * n0x[x0 + xl] * (((sRed[0][xl] + sRed[1][xl]) + sRed[2][xl]) + sRed[3][xl]);
      pscal[((size_t)op * gy + blockIdx.y) * gx + blockIdx.x] = total;
    }
  } else if (tid < BM && x0 + tid < nx) {
    pE[(size_t)(x0 + tid) * gx + blockIdx.x] =
        dt * (((sRed[0][tid] + sRed[1][tid]) + sRed[2][tid]) + sRed[3][tid]);
  }
}

// Second pass: gscal[op] += sum over the (by, bx) slots, gE[x] = sum over bx,
// both in ascending slot order.
__global__ void k_adjoint_reduce(const double* __restrict__ pscal, const double* __restrict__ pE,
                                 double* __restrict__ gscal, double* __restrict__ gE, int nparams, int nx, int gx,
                                 int gy) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nparams) {
    const double* p = pscal + (size_t)t * gy * gx;
    double s = 0.0;
    for (int q = 0; q < gx * gy; ++q) s += p[q];
    gscal[t] += s;
  } else if (t < nparams + nx) {
    const int x = t - nparams;
    const double* p = pE + (size_t)x * gx;
    double s = 0.0;
    for (int q = 0; q < gx; ++q) s += p[q];
    gE[x] = s;
  }
}

}  // namespace

void launch_to_harm(const DevOps& d, int nl, int npad_h, const double* F, const double* TS, double* Bh,
                    hipStream_t s) {
  const size_t sh = (size_t)(d.n + nl * d.nth) * sizeof(double);
  k_to_harm<<<d.nx_total, 256, sh, s>>>(F, TS, Bh, d.nr, d.nth, nl, npad_h);
}

void launch_from_harm(const DevOps& d, int nl, int npad_h, const double* Xh, const double* Bh, const double* TO,
                      double* F, hipStream_t s) {
  const size_t sh = (size_t)(d.nr * nl + nl * d.nth) * sizeof(double);
  k_from_harm<<<d.nx_total, 256, sh, s>>>(Xh, Bh, TO, F, d.nr, d.nth, nl, npad_h);
}

void launch_pad_rows(const DevOps& d, const double* F, double* Bp, hipStream_t s) {
  k_pad<<<1024, 256, 0, s>>>(F, Bp, d.n, d.npad, d.nx_total);
}

void launch_unpad_rows(const DevOps& d, const double* Bp, double* F, hipStream_t s) {
  k_unpad<<<1024, 256, 0, s>>>(Bp, F, d.n, d.npad, d.nx_total);
}

void launch_apply(const DevOps& d, int mode, const double* B, const double* X, double* R, const int* skip,
                  hipStream_t s) {
  dim3 g((d.n + 63) / 64, (d.nx_total + 31) / 32);
  if (mode == 1)
    k_residual<0, 1><<<g, kResThreads, 0, s>>>(B, X, R, d.Cord, d.Aord, d.E, d.n0x, d.rmax, d.bmax, d.xmax, d.status, d.dt,
                                       d.n, d.npad, d.nx_total, skip);
  else
    k_residual<0, 2><<<g, kResThreads, 0, s>>>(B, X, R, d.Cord, d.Aord, d.E, d.n0x, d.rmax, d.bmax, d.xmax, d.status, d.dt,
                                       d.n, d.npad, d.nx_total, skip);
}

void launch_apply_field(const DevOps& d, int mode, const double* B, const double* X, double* R, const double* E,
                        hipStream_t s) {
  dim3 g((d.n + 63) / 64, (d.nx_total + 31) / 32);
  if (mode == 3)
    k_residual<0, 3><<<g, kResThreads, 0, s>>>(B, X, R, d.Cord, d.Aord, E, d.n0x, d.rmax, d.bmax, d.xmax, d.status, d.dt,
                                       d.n, d.npad, d.nx_total, nullptr);
  else
    k_residual<0, 2><<<g, kResThreads, 0, s>>>(B, X, R, d.Cord, d.Aord, E, d.n0x, d.rmax, d.bmax, d.xmax, d.status, d.dt,
                                       d.n, d.npad, d.nx_total, nullptr);
}

void launch_residual(const DevOps& d, bool transpose, hipStream_t s) {
  dim3 g((d.n + 63) / 64, (d.nx_total + 31) / 32);
  if (transpose)
    k_residual<1><<<g, kResThreads, 0, s>>>(d.B, d.X, d.R, d.Cord, d.Aord, d.E, d.n0x, d.rmax, d.bmax, d.xmax, d.status, d.dt, d.n,
                                    d.npad, d.nx_total, nullptr);
  else
    k_residual<0><<<g, kResThreads, 0, s>>>(d.B, d.X, d.R, d.Cord, d.Aord, d.E, d.n0x, d.rmax, d.bmax, d.xmax, d.status, d.dt, d.n,
                                    d.npad, d.nx_total, nullptr);
}

namespace {
__global__ void k_fill(double* __restrict__ p, double v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
}  // namespace

void launch_fill(double* p, double v, size_t n, hipStream_t s) {
  if (n == 0) return;
  const int blocks = static_cast<int>(std::min<size_t>((n + 255) / 256, 1024));
  k_fill<<<blocks, 256, 0, s>>>(p, v, n);
}

void launch_refine_check(const DevOps& d, bool transpose, double rtol, int sweep, bool final_sweep, hipStream_t s) {
  k_refine_check<<<1, 256, 0, s>>>(d.rmax, d.bmax, d.xmax, d.E, d.n0x, d.dt, transpose ? d.c_one : d.c_inf,
                                   transpose ? d.a_one : d.a_inf, d.status, d.resid, rtol, sweep, final_sweep ? 1 : 0,
                                   d.nx_total);
}

void launch_reset_refine(const DevOps& d, hipStream_t s) {
  k_reset_refine<<<1, 256, 0, s>>>(d.rmax, d.bmax, d.xmax, d.status, d.nx_total);
}

void launch_adjoint_grads(const DevOps& d, double* grad_scal, double* grad_E, hipStream_t s) {
  const int gx = (d.n + 63) / 64, gy = (d.nx_total + 31) / 32;
  dim3 g(gx, gy, d.n_params + 1);
  double* pE = d.adj_part + (size_t)d.n_params * gx * gy;
  k_adjoint_grads<<<g, 256, 0, s>>>(d.mu, d.Fs, d.Csb, d.Aord, d.n0x, d.adj_part, pE, d.dt, d.n, d.nx_total,
                                    d.n_params);
  const int tot = d.n_params + d.nx_total;
  k_adjoint_reduce<<<(tot + 255) / 256, 256, 0, s>>>(d.adj_part, pE, grad_scal, grad_E, d.n_params, d.nx_total, gx,
                                                     gy);
}

}  // namespace bte

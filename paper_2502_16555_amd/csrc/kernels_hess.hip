// Velocity-space step in Hessenberg form (the harmonic-basis systems
// (B - s A_h) u = b of eq. (vspace_batched_system), s = dt E_x, reduced once per
// discharge to u = Q (I - s H)^-1 W b with H upper Hessenberg; see hessenberg.cpp):
//   k_mat_apply   Out[x] = M In[x] for the points of one discharge (W, then Q):
//                 32 points x 64 outputs per block, MFMA f64 16x16x4, K through
//                 double-buffered LDS;
//   k_hess_solve  (I - s H) z = y, one block per point, in O(n^2): Givens
//                 rotations of columns (k-1, k), k = n-1 .. 1, turn G = I - s H
//                 into an upper triangular R = G Z; column k of R is final once
//                 formed, so the back substitution R w = y runs alongside and R is
//                 never stored; then z = Z w.
#include <cmath>
#include <type_traits>
#include <utility>

#include "internal.h"
#include "lu_common.h"

namespace bte {
namespace {


// Result row of item t of lane group lk for MFMA f64 16x16x4 (measured layout).
__device__ inline int f64_row(int lk, int t) { return lk + 4 * t; }

// Out[x][i] = sum_k M[i][k] In[x][k], x in [x0, x0 + nx), i < n; M, In and Out
// rows of length ld (M zero from column n on).  Block: 32 points x 64 outputs,
// each wave two 16 x 16 MFMA tiles; K in chunks of 64 through two LDS buffers,
// the next chunk's 16-byte global loads in flight while the current one is
// multiplied.  Grid: (ceil(n / 64), ceil(nx / 32)); the blocks of one XCD
// (block id mod 8) share their rows of M.
constexpr int kMaBM = 32, kMaBN = 64, kMaBK = 64;
constexpr int kMaLds = kMaBK + 1;   // odd row stride: the fragment reads are conflict-free
constexpr int kMaALoads = kMaBM * kMaBK / 2 / 256, kMaBLoads = kMaBN * kMaBK / 2 / 256;

__global__ __launch_bounds__(256) void k_mat_apply(const double* __restrict__ M, const double* __restrict__ In,
                                                   double* __restrict__ Out, int n, int ld, int x0, int nx) {
  constexpr int BM = kMaBM, BN = kMaBN, BK = kMaBK, LDL = kMaLds;
  extern __shared__ double lds[];
  double* sX = lds;                      // [2][BM][LDL]
  double* sM = lds + 2 * BM * LDL;       // [2][BN][LDL]
  const int xb = blockIdx.y * BM, i0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  f64x2 ra[kMaALoads], rb[kMaBLoads];
  auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < kMaALoads; ++t) {
      const int e = tid + 256 * t, r = e / (BK / 2), k = k0 + 2 * (e % (BK / 2));
      f64x2 v = {0.0, 0.0};
      if (xb + r < nx && k < n) {
        v = *reinterpret_cast<const f64x2*>(In + (size_t)(x0 + xb + r) * ld + k);
        if (k + 1 >= n) v[1] = 0.0;
      }
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < kMaBLoads; ++t) {
      const int e = tid + 256 * t, r = e / (BK / 2), k = k0 + 2 * (e % (BK / 2));
      f64x2 v = {0.0, 0.0};
      if (i0 + r < n && k < n) v = *reinterpret_cast<const f64x2*>(M + (size_t)(i0 + r) * ld + k);
      rb[t] = v;
    }
  };
  auto store = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < kMaALoads; ++t) {
      const int e = tid + 256 * t, r = e / (BK / 2), c = 2 * (e % (BK / 2));
      double* d = sX + (buf * BM + r) * LDL + c;
      d[0] = ra[t][0];
      d[1] = ra[t][1];
    }
#pragma unroll
    for (int t = 0; t < kMaBLoads; ++t) {
      const int e = tid + 256 * t, r = e / (BK / 2), c = 2 * (e % (BK / 2));
      double* d = sM + (buf * BN + r) * LDL + c;
      d[0] = rb[t][0];
      d[1] = rb[t][1];
    }
  };
  f64x4 acc[2] = {f64x4{0, 0, 0, 0}, f64x4{0, 0, 0, 0}};
  const int nch = (n + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) load((c + 1) * BK);
    const double* xa = sX + buf * BM * LDL;
    const double* mb = sM + (buf * BN + w * 16 + li) * LDL + lk;
#pragma unroll
    for (int k = 0; k < BK; k += 4) {
      const double bm = mb[k];
#pragma unroll
      for (int b = 0; b < 2; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[(b * 16 + li) * LDL + k + lk], bm, acc[b], 0, 0, 0);
    }
    if (c + 1 < nch) store(buf ^ 1);
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
constexpr int kHessRing = 8;   // columns of H in flight per thread (fewer measured slower)
constexpr int kHessSeg = 2 * kHessThreads;      // rows per pair index (two per thread)

// row pairs per thread for an order-n solve
int hess_pairs(int n) {
  const int p = (n + kHessSeg - 1) / kHessSeg;
  return p <= 1 ? 1 : p <= 2 ? 2 : 4;
}

// two consecutive rows of one column, read by one 16-byte load
struct alignas(16) Pair {
  double x, y;
};

template <int E>
__device__ __forceinline__ double& el(Pair& v) {
  if constexpr (E == 0) return v.x; else return v.y;
}

// (I - s H) z = y for one point per block.  Rows are taken in reverse, j = n-1-r.
// Thread t holds the row pairs j = 2t + {0, 1} + SEG p, p < P, of y, of the
// running column of G Z and of the next D columns of H (raw, loaded D steps
// ahead as one 16-byte load per pair).  The step with owner row k = n-1-j (the
// rotation of columns k-1, k) acts only on rows j' >= j, so during the steps
// j in [S SEG, (S+1) SEG) only pairs p >= S are live: the loop runs per S with
// S a compile-time constant and touches no other pair.  Rows before the owner
// (j' < j: rows r > k, whose part of the solve is done) are updated too, without
// effect: nothing reads them again.
//
// The steps go two at a time: rows j, j+1 (j even) are one pair of one lane,
// which forms both rotations from its own entries and publishes them together;
// after one barrier every lane applies the two in turn.  With G = I - s H the
// update of a row by the rotation (c, sg, w) of a step whose fresh column has
// the raw entry h in that row is
//     y <- y - w c x + (w sg s) h,   x <- -sg x - (c s) h,
// plus c (to x) and -w sg (to y) on the column's diagonal row.
template <int P>
__global__ __launch_bounds__(kHessThreads) void k_hess_solve(const double* __restrict__ Hr,
                                                             const size_t* __restrict__ h_off,
                                                             const int* __restrict__ x_disc,
                                                             const double* __restrict__ E, double dt,
                                                             const double* __restrict__ Y, double* __restrict__ Z,
                                                             int n, int ld, int* __restrict__ status) {
  constexpr int NT = kHessThreads, D = kHessRing, SEG = kHessSeg, LDC = P * NT;   // column stride in pairs
  const int x = blockIdx.x, tid = threadIdx.x;
  // this thread's pairs of column 0
  const Pair* H = reinterpret_cast<const Pair*>(Hr + h_off[x_disc[x]]) + tid;
  const double s = dt * E[x];
  // rotation k at entry kOff + k (the no-op steps have k = 1 - D .. 0)
  constexpr int kOff = D;
  __shared__ double s_c[kOff + kMaxRows], s_s[kOff + kMaxRows], s_w[kOff + kMaxRows];
  Pair cur[P], y[P], hq[D][P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int j = 2 * tid + SEG * p;
    y[p].x = (j < n) ? Y[(size_t)x * ld + (n - 1 - j)] : 0.0;
    y[p].y = (j + 1 < n) ? Y[(size_t)x * ld + (n - 2 - j)] : 0.0;
    // column n-1 of G = I - s H; its diagonal entry is row j = 0
    const Pair h = H[(size_t)(n - 1) * LDC + p * NT];
    cur[p].x = fma(-s, h.x, j == 0 ? 1.0 : 0.0);
    cur[p].y = -s * h.y;
  }
#pragma unroll
  for (int u = 0; u < D; ++u) {
    const int c = max(n - 2 - u, 0);   // column k-1 of the step j = u
#pragma unroll
    for (int p = 0; p < P; ++p) hq[u][p] = H[(size_t)c * LDC + p * NT];
  }
  bool bad = false;
  // Rotation jn (owner row kn = n-1-jn), which zeroes row kn of the new column
  // kn-1: a = G[kn][kn-1] (sub-diagonal), b of the running column, yv of y.
  // 1/hypot(a, b) from the hardware estimate and two Newton steps.  Steps past
  // the last (jn >= n-1) are no-ops: c = 0, s = -1, w = 0 leave y and the
  // running column as they are.
  auto form = [&](int jn, double a, double b, double yv, double& rc, double& rs, double& rw)
      __attribute__((always_inline)) {
    const bool fake = jn >= n - 1;
    const double xx = fma(a, a, b * b);
    double ri = __builtin_amdgcn_rsq(xx);
    ri = fma(0.5 * ri, fma(-xx * ri, ri, 1.0), ri);
    ri = fma(0.5 * ri, fma(-xx * ri, ri, 1.0), ri);
    const bool z = !(xx > 0.0);
    bad |= z && !fake;
    rc = fake ? 0.0 : z ? 1.0 : b * ri;
    rs = fake ? -1.0 : z ? 0.0 : a * ri;
    rw = (fake || z) ? 0.0 : yv * ri;
  };
  // Rotations jn, jn+1 (jn even) by the lane holding that pair (cv, yv), with
  // the raw entries h0 of step jn's fresh column and h1 of step jn+1's: row jn+1
  // is the diagonal of the first, the sub-diagonal of the second.
  auto form2 = [&](int jn, const Pair& cv, const Pair& yv, const Pair& h0, const Pair& h1)
      __attribute__((always_inline)) {
    double c0, s0, w0, c1, s1, w1;
    form(jn, -s * h0.x, cv.x, yv.x, c0, s0, w0);
    const double g = fma(-s, h0.y, 1.0);
    const double r1 = c0 * cv.y + s0 * g;
    const double b1 = -s0 * cv.y + c0 * g;
    const double y1 = yv.y - r1 * w0;
    form(jn + 1, -s * h1.y, b1, y1, c1, s1, w1);
    const int kn = n - 1 - jn;
    s_c[kOff + kn] = c0;
    s_s[kOff + kn] = s0;
    s_w[kOff + kn] = w0;
    s_c[kOff + kn - 1] = c1;
    s_s[kOff + kn - 1] = s1;
    s_w[kOff + kn - 1] = w1;
  };
  // steps 0 and 1: rows 0, 1 are pair 0 of thread 0
  if (tid == 0) form2(0, cur[0], y[0], hq[0][0], hq[1][0]);
  static_for(std::make_integer_sequence<int, P>{}, [&](auto sc) __attribute__((always_inline)) {
    constexpr int S = decltype(sc)::value;
    const int jlo = S * SEG, jhi = min(jlo + SEG, n - 1);   // the steps j = 0 .. n-2
    for (int jb = jlo; jb < jhi; jb += D) {
      static_for(std::make_integer_sequence<int, D / 2>{}, [&](auto uc) __attribute__((always_inline)) {
        // steps j, j+1 with slots U, U+1 of the ring; the no-op steps past the
        // last keep the final block free of exits
        constexpr int U = 2 * decltype(uc)::value, U2 = (U + 2) % D, U3 = (U + 3) % D;
        const int j = jb + U;
        const int k = n - 1 - j;
        __syncthreads();
        const double c0 = s_c[kOff + k], sg0 = s_s[kOff + k], w0 = s_w[kOff + k];
        const double c1 = s_c[kOff + k - 1], sg1 = s_s[kOff + k - 1], w1 = s_w[kOff + k - 1];
        const double wc0 = w0 * c0, ws0 = w0 * sg0, cs0 = c0 * s, wss0 = ws0 * s;
        const double wc1 = w1 * c1, ws1 = w1 * sg1, cs1 = c1 * s, wss1 = ws1 * s;
        // the diagonal of step j's column, row j+1, is the second row of the
        // owner's pair; it matters only when that row is the last (j+1 = n-1)
        const bool dJ = 2 * tid + 1 + SEG * S == j + 1;
        auto rot = [&](Pair& cv, Pair& yv, const Pair& h0, const Pair& h1, bool own)
            __attribute__((always_inline)) {
          yv.x = fma(wss0, h0.x, fma(-wc0, cv.x, yv.x));
          yv.y = fma(wss0, h0.y, fma(-wc0, cv.y, yv.y));
          cv.x = fma(-sg0, cv.x, -cs0 * h0.x);
          cv.y = fma(-sg0, cv.y, -cs0 * h0.y);
          if (own) {
            cv.y += dJ ? c0 : 0.0;
            yv.y -= dJ ? ws0 : 0.0;
          }
          yv.x = fma(wss1, h1.x, fma(-wc1, cv.x, yv.x));
          yv.y = fma(wss1, h1.y, fma(-wc1, cv.y, yv.y));
          cv.x = fma(-sg1, cv.x, -cs1 * h1.x);
          cv.y = fma(-sg1, cv.y, -cs1 * h1.y);
        };
        // The diagonal of step j+1's column is row j+2, the first of the next
        // owner's pair (pair S, or pair S+1 when j+2 starts it).
        rot(cur[S], y[S], hq[U][S], hq[U + 1][S], true);
        const bool dS = 2 * tid + SEG * S == j + 2;
        cur[S].x += dS ? c1 : 0.0;
        y[S].x -= dS ? ws1 : 0.0;
        // the next two rotations, by the lane holding rows j+2, j+3 in pair S
        if (tid == ((j + 2 - jlo) >> 1)) form2(j + 2, cur[S], y[S], hq[U2][S], hq[U3][S]);
#pragma unroll
        for (int p = S + 1; p < P; ++p) rot(cur[p], y[p], hq[U][p], hq[U + 1][p], false);
        if constexpr (S + 1 < P) {
          const bool dN = 2 * tid + SEG * (S + 1) == j + 2;
          cur[S + 1].x += dN ? c1 : 0.0;
          y[S + 1].x -= dN ? ws1 : 0.0;
        }
        // the columns for the steps j + D, j + 1 + D (clamped in the last steps:
        // loaded, never used)
        const int cn0 = max(k - 1 - D, 0), cn1 = max(k - 2 - D, 0);
#pragma unroll
        for (int p = S; p < P; ++p) {
          hq[U][p] = H[(size_t)cn0 * LDC + p * NT];
          hq[U + 1][p] = H[(size_t)cn1 * LDC + p * NT];
        }
      });
    }
    // the first two rotations of pair S+1 (rows (S+1) SEG + {0, 1}: thread 0)
    if constexpr (S + 1 < P) {
      constexpr int jn = (S + 1) * SEG;
      if (jn < n - 1 && tid == 0) form2(jn, cur[S + 1], y[S + 1], hq[jn % D][S + 1], hq[(jn + 1) % D][S + 1]);
    }
  });
  // row 0 (j = n-1): R[0][0] and w_0, then z = Z_{n-1} ... Z_1 w, Z_k acting on
  // entries (k-1, k), by a running carry on the lane that holds row 0
  if (tid == ((n - 1) % SEG) >> 1) {
    const int p0 = (n - 1) / SEG, e0 = (n - 1) & 1;
    __shared__ double s_fin[4];
#pragma unroll
    for (int p = 0; p < P; ++p)
      if (p == p0) {
        s_fin[0] = cur[p].x;
        s_fin[1] = cur[p].y;
        s_fin[2] = y[p].x;
        s_fin[3] = y[p].y;
      }
    const double r0 = s_fin[e0], y0 = s_fin[2 + e0];
    if (r0 == 0.0) bad = true;
    double t = y0 / r0;
    for (int k = 1; k < n; ++k) {
      const double c = s_c[kOff + k], sg = s_s[kOff + k], wk = s_w[kOff + k];
      s_w[kOff + k - 1] = c * t + sg * wk;
      t = -sg * t + c * wk;
    }
    s_w[kOff + n - 1] = t;
    if (!(fabs(t) <= 1.0e300)) atomicOr(status, kStNonFinite);
  }
  if (bad) atomicOr(status, kStSingular);
  __syncthreads();
  for (int r = tid; r < ld; r += NT) Z[(size_t)x * ld + r] = (r < n) ? s_w[kOff + r] : 0.0;
}

}  // namespace

void launch_mat_apply(const double* M, const double* In, double* Out, int n, int ld, int x0, int nx, hipStream_t s) {
  if (nx <= 0) return;
  constexpr size_t lds = (size_t)2 * (kMaBM + kMaBN) * kMaLds * sizeof(double);
  static const bool attr = [] {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mat_apply),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess;
  }();
  (void)attr;
  dim3 g((n + kMaBN - 1) / kMaBN, (nx + kMaBM - 1) / kMaBM);
  k_mat_apply<<<g, 256, lds, s>>>(M, In, Out, n, ld, x0, nx);
}

int hess_col_stride(int n) { return hess_pairs(n) * kHessSeg; }

void launch_hess_solve(const DevOps& d, const double* Hr, const size_t* h_off, int n, int ld, const double* Y,
                       double* Z, hipStream_t s) {
  switch (hess_pairs(n)) {
    case 1:
      k_hess_solve<1><<<d.nx_total, kHessThreads, 0, s>>>(Hr, h_off, d.x_disc, d.E, d.dt, Y, Z, n, ld, d.status);
      break;
    case 2:
      k_hess_solve<2><<<d.nx_total, kHessThreads, 0, s>>>(Hr, h_off, d.x_disc, d.E, d.dt, Y, Z, n, ld, d.status);
      break;
    default:
      k_hess_solve<4><<<d.nx_total, kHessThreads, 0, s>>>(Hr, h_off, d.x_disc, d.E, d.dt, Y, Z, n, ld, d.status);
  }
}

}  // namespace bte

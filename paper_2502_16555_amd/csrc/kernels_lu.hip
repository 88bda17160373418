// Velocity-space step V(dt): the Nx decoupled dense systems of
// eq. (vspace_batched_system),  (I - dt (n0 C + E_i A)) F*_i = F_i,  solved by a
// batched right-looking blocked LU factorization with partial pivoting.
//
// Storage: one column-major npad x npad matrix per collocation point (npad = n
// rounded up to the panel width kNB = 128, padded with identity), so panel
// columns, interchanges and the column-oriented solves are all unit-stride.
// Interchanges are applied "as you go": a panel's interchanges reach that
// panel and the trailing columns only, so the solve applies P_1, L_1^-1, P_2,
// L_2^-1, ..., U^-1 in that order (A = P_1^T L_1 P_2^T L_2 ... U).
//
// Per panel k0:
//   k_panel   one 512-thread block per matrix (256 for short panels): partial
//             pivoting (max |a|, ties to the lowest row) over register-resident
//             sub-panels of 8 or 16 columns, left-looking across
//             the sub-panels, and the panel's row permutation for the
//             trailing columns;
//   k_dinv    one block per matrix: inverses of the 16 x 16 diagonal blocks of
//             the panel's unit lower block L11;
//   k_l11inv  four blocks per matrix: L11^-1 by blocked substitution on the
//             identity (16-row blocks, each two MFMA products);
//   k_u12     per 128 trailing columns: the panel's interchanges and
//             U12 = L11^-1 P A12 as one MFMA product (K = 128) -- the
//             substitution's sequential 16-row steps are paid once per panel
//             in k_l11inv instead of once per column block;
//   k_update  A22 -= L21 U12: 128 x 128 MFMA tiles, K = 128 (or 256, two
//             panels; up to 512, four) in double-buffered LDS chunks; blocks of
//             one matrix are kept on one XCD so that L21 and U12 stay in that
//             XCD's L2.
// Dense systems take the panels in pairs: panel p updates panel p+1's columns
// at once, its update of the columns beyond is deferred, and after panel p+1
// one K = 256 update applies both (A22 read and written once per two panels).
// For panel p+1, k_u12pre, k_move_down and k_perm_lp (below) take the place of
// k_u12's gather.  Panel p+1's interchanges then also reach panel p's L
// columns, so the solve applies P_p P_{p+1} before L_p and L_{p+1}
// (A = ... P_p^T P_{p+1}^T L' ...).
// Statically pivoted FP32 factors (the mixed precisions' default) take no
// interchanges: each panel is k_diag_static (the 128 x 128 diagonal block's
// factors, U11^-1, L11^-1 and the inverses of L11's diagonal blocks, in
// place of k_panel, k_dinv and k_l11inv) and k_l21_mfma (L21 = A21 U11^-1),
// and k_move_down and k_perm_lp have nothing to move (see below).  Their
// panels go in groups of four: after each of a group's first three panels,
// one k_update launch over an L-shaped tile set applies the group's panels so
// far (K = 128 j) to the next panel's columns and to its top rows beyond it
// (in place: the top rows are the panel's own), and after the group's last
// panel one K = 512 update applies all four to the columns beyond the group
// (A22 read and written once per four panels).
#include <algorithm>
#include <cfloat>
#include <climits>
#include <limits>
#include <type_traits>
#include <cmath>

#include "internal.h"
#include "lu_common.h"

namespace bte {
namespace {

constexpr int NB = kNB;

// ---------------------------------------------------------------------------
// Matrix formation, column c of points x0..x0+xpb-1: I - dt (n0_x C + E_x A) with
// identity padding.  CT/AT hold C^T and A^T row-major, i.e. the columns of C
// and A contiguously; a block reads its column of each once and writes it into
// xpb matrices with 16-byte streaming stores.  The blocks of one column run
// together on one XCD, so that the column comes from HBM once and from that
// XCD's L2 for the others, and the launch is bound by the writes.  part 0
// forms columns c_lo.. whole; part 1 columns below split whole and the first
// split rows of the others; part 2 (c_lo = split) the rest, rows from split.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_form(T* __restrict__ LU, const double* __restrict__ CT,
                                              const double* __restrict__ AT, const double* __restrict__ E,
                                              const double* __restrict__ n0x, double dt, int n, int npad, int nmat,
                                              int xpb, int kl, int ku, int* __restrict__ mirror, int do_mirror,
                                              int c_lo, int part, int split) {
  constexpr int CH = kMaxRows / 1024;  // 4-row groups per thread
  const int tid = threadIdx.x;
  int c, xb;
  xcd_map(blockIdx.x, (nmat + xpb - 1) / xpb, npad - c_lo, &c, &xb);
  c += c_lo;
  if (c >= npad) return;
  const int x0 = xb * xpb, x1 = min(nmat, x0 + xpb);
  // banded factors (lower / upper bandwidth kl / ku, kl > 0): only rows
  // [r_lo, r_hi) of column c are ever read, from the U rows of the first panel
  // whose trailing columns reach c to the last L row of c's own panel
  int r_lo = 0, r_hi = npad;
  if (kl > 0) {
    const int kp = c / NB * NB;
    r_lo = max(0, (kp - kl - ku) / NB * NB - NB);
    r_hi = min(npad, (kp + NB + kl + NB - 1) / NB * NB);
  }
  if (part == 1 && c >= split) r_hi = min(r_hi, split);
  if (part == 2) r_lo = max(r_lo, split);
  double cv[CH][4], av[CH][4];
#pragma unroll
  for (int ch = 0; ch < CH; ++ch)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = 4 * tid + 1024 * ch + u;
      const bool in = c < n && r < n;
      cv[ch][u] = in ? CT[(size_t)c * n + r] : 0.0;
      av[ch][u] = in ? AT[(size_t)c * n + r] : 0.0;
    }
  for (int x = x0; x < x1; ++x) {
    // static pivoting (do_mirror): a point with E < 0 is formed with |E|, the
    // matrix of its angularly mirrored system (ordinates theta -> pi - theta in
    // every speed block: M(-E) = J M(E) J), whose unpivoted factors stay as well
    // conditioned as those of a positive field; the solves mirror their vectors
    double e = E[x];
    const double nn = n0x[x];
    const bool mx = do_mirror && e < 0.0;
    if (mirror && c == 0 && tid == 0) mirror[x] = mx ? 1 : 0;   // the flags follow the factors
    if (mx) e = -e;
    T* col = LU + ((size_t)x * npad + c) * npad;
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
      const int r0 = 4 * tid + 1024 * ch;
      if (r0 >= r_lo && r0 < r_hi) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = static_cast<T>(-dt * (nn * cv[ch][u] + e * av[ch][u]) + (r0 + u == c ? 1.0 : 0.0));
        // FP32: streaming (non-temporal) stores, most columns are read back only by
        // a later panel or update (measured 0.87 ms against 0.99 ms at C2); FP64
        // columns keep ordinary stores (streaming ones measured twice as slow)
        if constexpr (sizeof(T) == 4) {
          __builtin_nontemporal_store(f32x4{v[0], v[1], v[2], v[3]}, reinterpret_cast<f32x4*>(col + r0));
        } else {
          *reinterpret_cast<double2*>(col + r0) = make_double2(v[0], v[1]);
          *reinterpret_cast<double2*>(col + r0 + 2) = make_double2(v[2], v[3]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Panel factorization: rows k0.., columns k0..k0+NB-1, one block per matrix,
// left-looking over sub-panels of IB columns: a sub-panel's columns receive
// the updates of all earlier sub-panels when they are loaded (their L read in
// chunks of CB columns with the next chunk in flight, the sub-panel's U rows
// from LDS), are factored in registers, and then only their U rows of the rest
// of the panel are formed.  The tall part of the panel is read once per
// sub-panel as L rather than read and written by a right-looking update, which
// halves the traffic of a 2048-row panel (1.4x faster FP32, 1.6x FP64, with the
// same products in the same order, hence the same bits).
// ---------------------------------------------------------------------------
template <typename T, int NT, int RPT, int IB, int CB>
__global__ __launch_bounds__(NT) void k_panel(T* __restrict__ LU, int* __restrict__ piv,
                                                         int* __restrict__ perm, int* __restrict__ status, int npad,
                                                         int k0, int rend) {
  // rows >= rend are zero in the panel columns (banded systems) and take no part
  static_assert(IB % CB == 0 || CB % IB == 0, "the L chunk and the sub-panel width must nest");
  constexpr int NW = NT / 64;
  const int mat = blockIdx.x;
  T* A = LU + (size_t)mat * npad * npad;
  int* ip = piv + (size_t)mat * npad;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  __shared__ double s_val[2][NW];
  __shared__ int s_idx[2][NW];
  __shared__ unsigned long long s_key[2][NW];
  __shared__ T s_row[2][1][IB];
  __shared__ T s_cand[2][NW][IB];
  __shared__ T s_L11[IB][IB + 1];
  __shared__ T s_U[IB][NB];
  __shared__ int s_sw[IB];
  __shared__ int s_piv[NB];
  __shared__ int s_R[2 * IB];
  __shared__ int s_src[2 * IB];
  __shared__ int s_lab[kMaxSwapRows];
  __shared__ int s_pos[kMaxRows];
  __shared__ int s_nR, s_any, s_cnt[2];
  __shared__ T s_Ut[NB][IB];       // U rows (k0..c0) of the sub-panel's columns
  __shared__ T s_Lr[IB][NB + 1];   // L of the sub-panel's top rows, earlier columns
  bool singular = false, nonfinite = false;

  for (int sp = 0; sp < NB / IB; ++sp) {
    const int c0 = k0 + sp * IB;
    T a[RPT][IB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = c0 + tid + q * NT;
#pragma unroll
      for (int j = 0; j < IB; ++j) a[q][j] = (r < rend) ? A[(size_t)(c0 + j) * npad + r] : T(0);
    }
    {
      // a -= L[rows, k0:c0] U[k0:c0, sub-panel]: L in chunks of CB columns with
      // the next chunk's loads in flight (a chunk wider than the sub-panel may
      // end past column c0: those loads and products are skipped)
      const int nk = c0 - k0;
      if (nk > 0) {
        for (int e = tid; e < nk * IB; e += NT) {
          const int m = e % nk, j = e / nk;
          s_Ut[m][j] = A[(size_t)(c0 + j) * npad + k0 + m];
        }
        __syncthreads();
        T lv[RPT][CB], ln[RPT][CB];
        auto ldl = [&](T (&dst)[RPT][CB], int m0) {
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            const int r = c0 + tid + q * NT;
#pragma unroll
            for (int u = 0; u < CB; ++u)
              dst[q][u] = (r < rend && (IB % CB == 0 || m0 + u < nk)) ? A[(size_t)(k0 + m0 + u) * npad + r] : T(0);
          }
        };
        ldl(lv, 0);
        for (int m0 = 0; m0 < nk; m0 += CB) {
          if (m0 + CB < nk) ldl(ln, m0 + CB);
#pragma unroll
          for (int u = 0; u < CB; ++u) {
            if (CB % IB == 0 && CB > IB && m0 + u >= nk) break;   // last chunk of a wide CB
            T uj[IB];
#pragma unroll
            for (int j = 0; j < IB; ++j) uj[j] = s_Ut[m0 + u][j];
#pragma unroll
            for (int q = 0; q < RPT; ++q)
#pragma unroll
              for (int j = 0; j < IB; ++j) a[q][j] -= lv[q][u] * uj[j];
          }
#pragma unroll
          for (int q = 0; q < RPT; ++q)
#pragma unroll
            for (int u = 0; u < CB; ++u) lv[q][u] = ln[q][u];
        }
      }
    }
#pragma clang loop unroll(full)
    for (int j = 0; j < IB; ++j) {
      const int c = c0 + j;
      double best = -1.0;
      int bi = INT_MAX;
      // FP32: one 64-bit key per candidate, the bits of |a| (monotone for
      // non-negative floats) over ~row, so that a single maximum picks the
      // largest |a| and, among equal ones, the lowest row; 0 = no candidate
      // (NaN or outside the panel's rows)
      unsigned long long key = 0;
      if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = c0 + tid + q * NT;
          const float av = fabsf(a[q][j]);
          if (r >= c && r < rend && av == av) {
            const unsigned long long k =
                (static_cast<unsigned long long>(__float_as_uint(av)) << 32) | static_cast<unsigned>(~r);
            key = k > key ? k : key;
          }
        }
        key = wave_max_u64(key);
        bi = key ? static_cast<int>(~static_cast<unsigned>(key)) : INT_MAX;
      } else {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = c0 + tid + q * NT;
          if (r >= c && r < rend) {
            const double v = fabs(static_cast<double>(a[q][j]));
            if (v > best) {
              best = v;
              bi = r;
            }
          }
        }
        const double wm = wave_max(best);
        bi = wave_min(best == wm ? bi : INT_MAX);
        best = wm;
      }
      // One barrier per column: every wavefront publishes its partial maximum
      // together with the row it belongs to, thread j publishes row c; after the
      // barrier every thread reduces the partials to the same pivot p and finds
      // both rows of the interchange in LDS.  The buffers alternate with the
      // column parity: one is rewritten two columns later, when every thread has
      // passed the barrier of the column in between and finished reading it.
      const int par = j & 1;
      if (lane == 0) {
        if constexpr (sizeof(T) == 4) {
          s_key[par][wid] = key;
        } else {
          s_val[par][wid] = best;
          s_idx[par][wid] = bi;
        }
      }
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        if (c0 + tid + q * NT == bi) {
#pragma unroll
          for (int jj = 0; jj < IB; ++jj) s_cand[par][wid][jj] = a[q][jj];
        }
      }
      if (tid == j) {  // row c is owned by thread j (q = 0)
#pragma unroll
        for (int jj = 0; jj < IB; ++jj) s_row[par][0][jj] = a[0][jj];
      }
      __syncthreads();
      int p = INT_MAX, pw = 0;
      if constexpr (sizeof(T) == 4) {
        unsigned long long km = 0;
#pragma unroll
        for (int u = 0; u < NW; ++u) {
          const unsigned long long ok = s_key[par][u];
          if (ok > km) {
            km = ok;
            pw = u;
          }
        }
        if (km) p = static_cast<int>(~static_cast<unsigned>(km));
      } else {
        double v = -1.0;
#pragma unroll
        for (int u = 0; u < NW; ++u) {
          const double ov = s_val[par][u];
          const int oi = s_idx[par][u];
          if (ov > v || (ov == v && oi < p)) {
            v = ov;
            p = oi;
            pw = u;
          }
        }
      }
      // a column of NaNs has no candidate: keep row c (every index stays in
      // range whatever the data) and report the non-finite value
      const T* prow = s_cand[par][pw];
      if (p == INT_MAX) {
        p = c;
        prow = s_row[par][0];
      }
      if (p != c) {
        if (tid == j) {
#pragma unroll
          for (int jj = 0; jj < IB; ++jj) a[0][jj] = prow[jj];
        }
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          if (c0 + tid + q * NT == p) {
#pragma unroll
            for (int jj = 0; jj < IB; ++jj) a[q][jj] = s_row[par][0][jj];
          }
        }
      }
      const T pv = prow[j];
      if (tid == 0) {  // pivots stay in LDS until the panel ends: a global store
        s_piv[c - k0] = p;  // here would make every later barrier wait for it
        s_sw[j] = p;
      }
      if (pv == T(0)) singular = true;
      if (!(fabs(static_cast<double>(pv)) <= DBL_MAX)) nonfinite = true;
      // multipliers by the reciprocal of the pivot (division for subnormal
      // pivots); the pivot is the same in every lane, so a scalar branch keeps
      // the divisions off the common path
      const bool by_rcp = fabs(pv) >= std::numeric_limits<T>::min();
      const T rp = T(1) / pv;
      auto rank1 = [&](auto use_rcp) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = c0 + tid + q * NT;
          if (r > c && r < rend && pv != T(0)) {
            const T x = a[q][j];
            const T l = decltype(use_rcp)::value ? x * rp : x / pv;
#pragma unroll
            for (int jj = 0; jj < IB; ++jj) {
              const T upd = a[q][jj] - l * prow[jj];
              a[q][jj] = (jj > j) ? upd : (jj == j ? l : a[q][jj]);
            }
          }
        }
      };
      if (__builtin_amdgcn_readfirstlane(static_cast<int>(by_rcp))) rank1(std::true_type{});
      else rank1(std::false_type{});
    }
    __syncthreads();
    // write the factored sub-panel back (coalesced: consecutive threads, consecutive rows)
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = c0 + tid + q * NT;
      if (r < rend) {
#pragma unroll
        for (int j = 0; j < IB; ++j) A[(size_t)(c0 + j) * npad + r] = a[q][j];
      }
    }
    if (tid < IB) {
#pragma unroll
      for (int j = 0; j < IB; ++j) s_L11[tid][j] = a[0][j];
    }
    // permutation of the rows touched by this sub-panel's interchanges: rows
    // c0..c0+IB-1 and the distinct pivot rows below, each traced back through
    // the interchanges (last first) to the row its content comes from
    __syncthreads();
    if (wid == 0) {
      int p = 0;
      bool own = false;
      if (lane < IB) {
        p = s_sw[lane];
        own = p >= c0 + IB;
        for (int jj = 0; jj < lane; ++jj)
          if (s_sw[jj] == p) own = false;
      }
      const unsigned long long m = __ballot(own);
      const int rank = __popcll(m & ((1ull << lane) - 1ull));
      if (lane < IB) s_R[lane] = c0 + lane;
      if (own) s_R[IB + rank] = p;
      if (lane == 0) s_nR = IB + __popcll(m);
    }
    __syncthreads();
    if (tid < s_nR) {
      int x = s_R[tid];
      for (int jj = IB - 1; jj >= 0; --jj) {
        const int pj = s_sw[jj], cj = c0 + jj;
        x = (x == cj) ? pj : (x == pj ? cj : x);
      }
      s_src[tid] = x;
    }
    if (tid == 0) {
      int any = 0;
      for (int jj = 0; jj < IB; ++jj) any |= s_sw[jj] != c0 + jj;
      s_any = any;
    }
    __syncthreads();
    // apply the interchanges to the other columns of the panel (rows >= c0)
    if (s_any) {
      const int nR = s_nR;
      constexpr int NOC = NB - IB;
      constexpr int NV = (NOC * 2 * IB + NT - 1) / NT;
      T vb[NV];
#pragma unroll
      for (int u = 0; u < NV; ++u) {
        const int e = tid + u * NT;
        if (e < NOC * nR) {
          const int t = e % nR, cc = e / nR;
          const int col = (cc < sp * IB) ? k0 + cc : k0 + IB + cc;
          vb[u] = A[(size_t)col * npad + s_src[t]];
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NV; ++u) {
        const int e = tid + u * NT;
        if (e < NOC * nR) {
          const int t = e % nR, cc = e / nR;
          const int col = (cc < sp * IB) ? k0 + cc : k0 + IB + cc;
          if (s_src[t] != s_R[t]) A[(size_t)col * npad + s_R[t]] = vb[u];
        }
      }
      __syncthreads();
    }
    // the sub-panel's U rows of the remaining columns of the panel
    const int nrest = k0 + NB - c0 - IB;
    if (nrest > 0) {
      // U rows c0..c0+IB-1 of the rest: first the updates of the earlier
      // sub-panels (their L rows staged in LDS, U read down each column in
      // chunks of 8), then the sub-panel's own unit lower block
      const int nk = c0 - k0;
      for (int e = tid; e < IB * nk; e += NT) {
        const int i = e % IB, m = e / IB;
        s_Lr[i][m] = A[(size_t)(k0 + m) * npad + c0 + i];
      }
      __syncthreads();
      for (int e = tid; e < IB * nrest; e += NT) {
        const int i = e % IB, cc = e / IB;
        const T* colp = A + (size_t)(c0 + IB + cc) * npad;
        T v = colp[c0 + i];
        for (int m0 = 0; m0 < nk; m0 += 8) {
          T uv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) uv[u] = colp[k0 + m0 + u];
#pragma unroll
          for (int u = 0; u < 8; ++u) v -= s_Lr[i][m0 + u] * uv[u];
        }
        s_U[i][cc] = v;
      }
      __syncthreads();
      if (tid < nrest) {
        T* colp = A + (size_t)(c0 + IB + tid) * npad;
        for (int j = 1; j < IB; ++j) {
          T v = s_U[j][tid];
          for (int i = 0; i < j; ++i) v -= s_L11[j][i] * s_U[i][tid];
          s_U[j][tid] = v;
        }
        for (int j = 0; j < IB; ++j) colp[c0 + j] = s_U[j][tid];
      }
      __syncthreads();
    }
  }
  if (singular && tid == 0) atomicOr(status, kStSingular);
  if (nonfinite && tid == 0) atomicOr(status, kStNonFinite);
  // pivots out, then the permutation of the whole panel for the trailing columns:
  // the panel's rows and the distinct pivot rows below it in the order of their
  // first selection, with their sources traced back as above
  __syncthreads();
  for (int t = tid; t < NB; t += NT) ip[k0 + t] = s_piv[t];
  for (int r = k0 + NB + tid; r < rend; r += NT) s_pos[r] = INT_MAX;
  __syncthreads();
  if (tid < NB) {
    const int p = s_piv[tid];
    if (p >= k0 + NB) atomicMin(&s_pos[p], tid);
  }
  __syncthreads();
  unsigned long long om = 0;
  int orank = 0, pown = 0;
  bool own = false;
  if (tid < NB) {
    pown = s_piv[tid];
    own = pown >= k0 + NB && s_pos[pown] == tid;
    om = __ballot(own);
    orank = __popcll(om & ((1ull << lane) - 1ull));
    if (lane == 0) s_cnt[wid] = __popcll(om);
    s_lab[tid] = k0 + tid;
  }
  __syncthreads();
  const int nRf = NB + s_cnt[0] + s_cnt[1];
  if (own) s_lab[NB + orank + (wid == 1 ? s_cnt[0] : 0)] = pown;
  __syncthreads();
  int* pm = perm + ((size_t)mat * kMaxPanels + k0 / NB) * kPermStride;
  for (int t = tid; t < nRf; t += NT) {
    int x = s_lab[t];
    for (int j = NB - 1; j >= 0; --j) {
      const int pj = s_piv[j], cj = k0 + j;
      x = (x == cj) ? pj : (x == pj ? cj : x);
    }
    pm[1 + t] = s_lab[t];
    pm[1 + kMaxSwapRows + t] = x;
  }
  if (tid == 0) pm[0] = nRf;
}

// ---------------------------------------------------------------------------
// Static pivoting (FP32 factors): the panel without row interchanges.  A pivot
// smaller than tau = 2^-20 max|A11| is replaced by tau with its sign (static
// pivoting, as in Li and Demmel's SuperLU_DIST); the FP64 refinement that
// follows every FP32 solve works with the unperturbed matrix.  Pivots and
// permutations are written as the identity, so that the U12, update and solve
// kernels apply them as no-ops.
//   k_diag_static  one 256-thread block per matrix, the 128 x 128 diagonal
//                  block in LDS: A11 = L11 U11 by 16-column steps (a panel
//                  factored by one wavefront in registers, its U12 rows by
//                  forward substitution, the trailing update on MFMA); then
//                  X = U11^-1 by 16 x 16 blocks in LDS (the diagonal blocks,
//                  then seven levels of off-diagonal blocks); X goes row-major
//                  into the matrix's linv slot after L11's inverses, and the
//                  inverses of L11's eight diagonal blocks (k_dinv's output)
//                  are formed beside those of U11's, by the other 128 threads,
//                  and L11^-1 (k_l11inv's output) by the same levels after X;
//   k_l21_mfma     L21 = A21 X for 128 rows per block: one MFMA product (K =
//                  128, the zero blocks of X skipped), A21 straight from HBM.
// ---------------------------------------------------------------------------
constexpr float kStaticPivotRel = 9.5367431640625e-07f;   // 2^-20

__global__ __launch_bounds__(256) void k_diag_static(float* __restrict__ LU, float* __restrict__ linv,
                                                     int* __restrict__ piv, int* __restrict__ perm,
                                                     int* __restrict__ status, int npad, int k0) {
  const int mat = blockIdx.x;
  float* A = LU + (size_t)mat * npad * npad;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // LDS: two 128 x 132 regions and the level sums.  During the factorization
  // the block sits column-major in the second region (sA[c][r]) and the first
  // holds the current step's MFMA operands; afterwards the first holds U11
  // row-major (sU) and the second X = U11^-1 transposed (sXT).
  __shared__ __align__(16) float sU[NB][NB + 4];
  __shared__ __align__(16) float sXT[NB][NB + 4];
  __shared__ float sT[8][16][17];   // a level's sums, per block
  __shared__ __align__(16) float sL11[2][16][20];   // rows as 16-byte vectors, per step parity
  __shared__ float sYd[8][16][16];                // inverses of L11's diagonal blocks
  __shared__ float s_red[4];
  float (*sA)[NB + 4] = sXT;
  constexpr int LQ = NB + 16;   // operand rows: lanes li + 16 lk fall on distinct banks
  // per step parity p: rows 32 p .. 32 p + 15 hold -L[r][c0 + k] (k = row),
  // rows 32 p + 16 .. 32 p + 31 U[c0 + k][c]
  float (*sLt)[LQ] = reinterpret_cast<float (*)[LQ]>(&sU[0][0]);
  float m = 0.0f;
  bool nonfinite = false;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = tid + 256 * u, c = e >> 5, r4 = (e & 31) * 4;
    const float4 v = *reinterpret_cast<const float4*>(A + (size_t)(k0 + c) * npad + k0 + r4);
    *reinterpret_cast<float4*>(&sA[c][r4]) = v;
    const float w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float av = fabsf(w4[q]);
      nonfinite |= !(av <= FLT_MAX);
      m = fmaxf(m, av);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (lane == 0) s_red[wid] = m;
  __syncthreads();
  const float tau = fmaxf(fmaxf(fmaxf(s_red[0], s_red[1]), fmaxf(s_red[2], s_red[3])) * kStaticPivotRel, FLT_MIN);
  // ---- A11 = L11 U11 by 16-column steps c0 = 16 kb: wavefront 0 factors the
  // step's panel (rows c0.., two per lane) in registers, each pivot row passed
  // on by lane reads, with no barrier; then U12 = L11^-1 A12 for the step's 16
  // rows (a thread per column) and A22 -= L21 U12 on MFMA in 16 x 16 tiles:
  // first the tiles of the next step's panel columns, then the others on
  // wavefronts 1-3 while wavefront 0 factors that panel (the staging buffers
  // alternate with the step).
  auto panel = [&](int kb) __attribute__((always_inline)) {
    const int c0 = 16 * kb;
    float (*sLtb)[LQ] = sLt + 32 * (kb & 1);
    float (*sL11b)[20] = sL11[kb & 1];
    const int ra = c0 + lane, rb = c0 + 64 + lane;
    const bool va = ra < NB, vb = rb < NB;
    float p[16], q[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) p[j] = q[j] = 0.0f;
    if (va) {
#pragma unroll
      for (int j = 0; j < 16; ++j) p[j] = sA[c0 + j][ra];
    }
    if (vb) {
#pragma unroll
      for (int j = 0; j < 16; ++j) q[j] = sA[c0 + j][rb];
    }
    // the lane tests stay inside the loop (hoisted, they would take 32 SGPRs)
    int lv = lane;
    asm volatile("" : "+v"(lv));
    const bool two = c0 + 64 < NB;   // a second row per lane
    static_for(std::make_integer_sequence<int, 16>(), [&](auto jc) __attribute__((always_inline)) {
      constexpr int j = decltype(jc)::value;
      float pv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(p[j]), j));
      if (!(fabsf(pv) >= tau)) pv = pv < 0.0f ? -tau : tau;   // also a NaN pivot (reported above)
      const float rp = __builtin_amdgcn_rcpf(pv);
      float u[16];
#pragma unroll
      for (int c = j + 1; c < 16; ++c) u[c] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(p[c]), j));
      // first half: lane j holds the pivot row; rows above it keep their U
      // entries (a zero multiplier leaves them exactly)
      const bool below = lv > j;
      const float l = p[j] * rp;
      const float lm = below ? l : 0.0f;
      p[j] = below ? l : (lv == j ? pv : p[j]);
#pragma unroll
      for (int c = j + 1; c < 16; ++c) p[c] = fmaf(-lm, u[c], p[c]);
      if (two) {
        const float l2 = q[j] * rp;
        q[j] = l2;
#pragma unroll
        for (int c = j + 1; c < 16; ++c) q[c] = fmaf(-l2, u[c], q[c]);
      }
    });
    // the panel in place; L21 (negated) and L11 staged for the products
    if (va) {
#pragma unroll
      for (int j = 0; j < 16; ++j) sA[c0 + j][ra] = p[j];
      if (lane >= 16) {
#pragma unroll
        for (int j = 0; j < 16; ++j) sLtb[j][ra] = -p[j];
      } else {
#pragma unroll
        for (int j = 0; j < 16; ++j) sL11b[lane][j] = p[j];
      }
    }
    if (vb) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        sA[c0 + j][rb] = q[j];
        sLtb[j][rb] = -q[j];
      }
    }
  };
  // A22 tile (rows r0.., columns cc..) -= L21 U12 of step kb
  auto tile = [&](int kb, int r0, int cc) __attribute__((always_inline)) {
    float (*sLtb)[LQ] = sLt + 32 * (kb & 1);
    float (*sUtb)[LQ] = sLt + 32 * (kb & 1) + 16;
    const float4 cv = *reinterpret_cast<const float4*>(&sA[cc + li][r0 + 4 * lk]);
    f32x4 acc = {cv.x, cv.y, cv.z, cv.w};
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4)
      acc = Mma<float>::step(sLtb[4 * q4 + lk][r0 + li], sUtb[4 * q4 + lk][cc + li], acc);
    *reinterpret_cast<float4*>(&sA[cc + li][r0 + 4 * lk]) = make_float4(acc[0], acc[1], acc[2], acc[3]);
  };
  if (wid == 0) panel(0);
  __syncthreads();
  for (int kb = 0; kb < NB / 16; ++kb) {
    const int c0 = 16 * kb;
    float (*sL11b)[20] = sL11[kb & 1];
    float (*sUtb)[LQ] = sLt + 32 * (kb & 1) + 16;
    const int ncol = NB - c0 - 16;
    if (tid < ncol) {   // U12 column c by forward substitution with the unit lower L11
      const int c = c0 + 16 + tid;
      float x[16];
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const float4 v = *reinterpret_cast<const float4*>(&sA[c][c0 + 4 * q4]);
        x[4 * q4] = v.x;
        x[4 * q4 + 1] = v.y;
        x[4 * q4 + 2] = v.z;
        x[4 * q4 + 3] = v.w;
      }
#pragma unroll
      for (int i = 1; i < 16; ++i) {
        float lr[16];
#pragma unroll
        for (int j4 = 0; j4 < i; j4 += 4) {
          const float4 v = *reinterpret_cast<const float4*>(&sL11b[i][j4]);
          lr[j4] = v.x;
          lr[j4 + 1] = v.y;
          lr[j4 + 2] = v.z;
          lr[j4 + 3] = v.w;
        }
#pragma unroll
        for (int j = 0; j < i; ++j) x[i] = fmaf(-lr[j], x[j], x[i]);
      }
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
        *reinterpret_cast<float4*>(&sA[c][c0 + 4 * q4]) = make_float4(x[4 * q4], x[4 * q4 + 1], x[4 * q4 + 2], x[4 * q4 + 3]);
#pragma unroll
      for (int i = 0; i < 16; ++i) sUtb[i][c] = x[i];
    }
    __syncthreads();
    const int nt = ncol / 16;
    if (nt > 0) {
      for (int t = wid; t < nt; t += 4) tile(kb, c0 + 16 + 16 * t, c0 + 16);
      __syncthreads();
      if (wid == 0) {
        panel(kb + 1);
      } else {
        for (int t = wid - 1; t < nt * (nt - 1); t += 3) tile(kb, c0 + 16 + 16 * (t % nt), c0 + 32 + 16 * (t / nt));
      }
      __syncthreads();
    }
  }
  // the factors to the matrix; pivots and permutation as the identity
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = tid + 256 * u, c = e >> 5, r4 = (e & 31) * 4;
    *reinterpret_cast<float4*>(A + (size_t)(k0 + c) * npad + k0 + r4) = *reinterpret_cast<const float4*>(&sA[c][r4]);
  }
  if (tid < NB) {
    piv[(size_t)mat * npad + k0 + tid] = k0 + tid;
    int* pm = perm + ((size_t)mat * kMaxPanels + k0 / NB) * kPermStride;
    pm[1 + tid] = k0 + tid;
    pm[1 + kMaxSwapRows + tid] = k0 + tid;
    if (tid == 0) pm[0] = NB;
  }
  // ---- X = U11^-1 by 16 x 16 blocks (X upper triangular, kept transposed in
  // LDS, XT[col][row]): the diagonal blocks X_bb = U_bb^-1 by back substitution,
  // then by levels d = 1..7 the blocks X_{a,a+d} = -X_aa sum_{m=a+1}^{a+d}
  // U_am X_{m,a+d}; the blocks of one level are independent.  U11 goes
  // row-major into sU, the strict lower parts of L11's diagonal blocks into sT
  // (which the levels use only later), then sXT is cleared.
#pragma unroll
  for (int u = 0; u < 4; ++u) {   // 4 x 4 blocks, transposed in registers
    const int i4 = 4 * (tid & 31), j4 = 4 * (tid >> 5) + 32 * u;
    float w[4][4];   // w[jj][ii] = A[i4 + ii][j4 + jj]
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const float4 v = *reinterpret_cast<const float4*>(&sA[j4 + jj][i4]);
      w[jj][0] = v.x;
      w[jj][1] = v.y;
      w[jj][2] = v.z;
      w[jj][3] = v.w;
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int i = i4 + ii;
      float o[4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) o[jj] = w[jj][ii];   // L's strict lower part rides below U
      *reinterpret_cast<float4*>(&sU[i][j4]) = make_float4(o[0], o[1], o[2], o[3]);
      if ((i >> 4) == (j4 >> 4)) {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          if (i > j4 + jj) sT[i >> 4][i & 15][(j4 + jj) & 15] = w[jj][ii];
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < NB * NB / 4; e += 256)
    *reinterpret_cast<float4*>(&sXT[e >> 5][(e & 31) * 4]) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  __syncthreads();
  if (tid < NB) {   // thread (b, c): column c of X_bb
    const int b = tid >> 4, c = tid & 15, o = 16 * b;
    float xv[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      float v = (i == c) ? 1.0f : 0.0f;
#pragma unroll
      for (int m2 = i + 1; m2 < 16; ++m2) v = fmaf(-sU[o + i][o + m2], xv[m2], v);
      xv[i] = v / sU[o + i][o + i];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) sXT[o + c][o + i] = xv[i];
  } else {          // thread (b, c): column c of L_bb^-1 (unit lower) by forward substitution
    const int b = (tid - NB) >> 4, c = tid & 15;
    float x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = (r == c) ? 1.0f : 0.0f;
#pragma unroll
    for (int r = 1; r < 16; ++r)
#pragma unroll
      for (int k = 0; k < r; ++k) x[r] -= sT[b][r][k] * x[k];
    float* out = linv + (size_t)mat * kLinvElems + b * 256;   // [b][r][c] row-major
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      out[r * 16 + c] = x[r];
      sYd[b][r][c] = x[r];
    }
  }
  __syncthreads();
  // levels on MFMA, the blocks of a level spread over the wavefronts: T_ab into
  // sT (lane (li, lk) holds rows 4 lk.. of column li), then X_{ab,b} = -X_aa T_ab
  // from sT, written transposed
  for (int d = 1; d < 8; ++d) {
    for (int ab = wid; ab + d < 8; ab += 4) {
      const int b = ab + d;
      f32x4 t = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int m2 = ab + 1; m2 <= b; ++m2)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
          t = Mma<float>::step(sU[16 * ab + li][16 * m2 + 4 * q4 + lk], sXT[16 * b + li][16 * m2 + 4 * q4 + lk], t);
#pragma unroll
      for (int it = 0; it < 4; ++it) sT[ab][4 * lk + it][li] = t[it];
    }
    __syncthreads();
    for (int ab = wid; ab + d < 8; ab += 4) {
      const int b = ab + d;
      f32x4 x = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
        x = Mma<float>::step(sXT[16 * ab + 4 * q4 + lk][16 * ab + li], sT[ab][4 * q4 + lk][li], x);
      *reinterpret_cast<float4*>(&sXT[16 * b + li][16 * ab + 4 * lk]) = make_float4(-x[0], -x[1], -x[2], -x[3]);
    }
    __syncthreads();
  }
  // X row-major: 4 x 4 blocks transposed in registers
  float* xo = linv + (size_t)mat * kLinvElems + kLinvXOff;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k4 = 4 * (tid & 31), c4 = 4 * (tid >> 5) + 32 * u;
    float4 v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = *reinterpret_cast<const float4*>(&sXT[c4 + j][k4]);
    *reinterpret_cast<float4*>(xo + (size_t)(k4 + 0) * NB + c4) = make_float4(v[0].x, v[1].x, v[2].x, v[3].x);
    *reinterpret_cast<float4*>(xo + (size_t)(k4 + 1) * NB + c4) = make_float4(v[0].y, v[1].y, v[2].y, v[3].y);
    *reinterpret_cast<float4*>(xo + (size_t)(k4 + 2) * NB + c4) = make_float4(v[0].z, v[1].z, v[2].z, v[3].z);
    *reinterpret_cast<float4*>(xo + (size_t)(k4 + 3) * NB + c4) = make_float4(v[0].w, v[1].w, v[2].w, v[3].w);
  }
  // ---- Y = L11^-1 (in place of k_l11inv) by the same levels: Y_bb from sYd,
  // then Y_{a+d,a} = -Y_{a+d,a+d} sum_{m=a}^{a+d-1} L_{a+d,m} Y_{m,a}, with L's
  // strict lower part in sU and Y kept transposed in the X region (zeros above
  // its diagonal); Y leaves column-major after the diagonal-block inverses
  __syncthreads();
  for (int e = tid; e < NB * NB / 4; e += 256) {   // YT row k: Y_bb's column k mod 16 in block b, zeros elsewhere
    const int k = e >> 5, i4 = (e & 31) * 4, b = k >> 4;
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if ((i4 >> 4) == b) {
      const int r = i4 & 15, c = k & 15;
      v = make_float4(sYd[b][r][c], sYd[b][r + 1][c], sYd[b][r + 2][c], sYd[b][r + 3][c]);
    }
    *reinterpret_cast<float4*>(&sXT[k][i4]) = v;
  }
  __syncthreads();
  for (int d = 1; d < 8; ++d) {
    for (int a = wid; a + d < 8; a += 4) {
      const int r = a + d;
      f32x4 t = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int m2 = a; m2 < r; ++m2)
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
          t = Mma<float>::step(sU[16 * r + li][16 * m2 + 4 * q4 + lk], sXT[16 * a + li][16 * m2 + 4 * q4 + lk], t);
#pragma unroll
      for (int it = 0; it < 4; ++it) sT[a][4 * lk + it][li] = t[it];
    }
    __syncthreads();
    for (int a = wid; a + d < 8; a += 4) {
      const int r = a + d;
      f32x4 x = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4)
        x = Mma<float>::step(sXT[16 * r + 4 * q4 + lk][16 * r + li], sT[a][4 * q4 + lk][li], x);
      *reinterpret_cast<float4*>(&sXT[16 * a + li][16 * r + 4 * lk]) = make_float4(-x[0], -x[1], -x[2], -x[3]);
    }
    __syncthreads();
  }
  float* yo = linv + (size_t)mat * kLinvElems + 8 * 256;   // column-major: (i, k) at k NB + i
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = tid + 256 * u, k = e >> 5, i4 = (e & 31) * 4;
    *reinterpret_cast<float4*>(yo + (size_t)k * NB + i4) = *reinterpret_cast<const float4*>(&sXT[k][i4]);
  }
  if (__syncthreads_or(nonfinite) && tid == 0) atomicOr(status, kStNonFinite);
}

__global__ __launch_bounds__(256, 2) void k_l21_mfma(float* __restrict__ LU, const float* __restrict__ linv,
                                                     int npad, int k0, int ntiles, int nmat) {
  int mat, tile;
  xcd_map(blockIdx.x, ntiles, nmat, &mat, &tile);
  if (mat >= nmat) return;
  float* A = LU + (size_t)mat * npad * npad;
  constexpr int LD = NB + 16;   // B fragment reads: lanes (li, lk) on banks li + 16 lk (64 banks)
  __shared__ __align__(16) float sX[NB][LD];
  const int r0 = k0 + NB + tile * NB;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // this wave's rows of A21 (32 w + 16 rb + li), all of K, into registers
  float av[32][2];
#pragma unroll
  for (int q = 0; q < 32; ++q)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) av[q][rb] = A[(size_t)(k0 + 4 * q + lk) * npad + r0 + 32 * w + 16 * rb + li];
  // X into LDS: every load issued before the first store (one wait, not sixteen)
  const float4* xs = reinterpret_cast<const float4*>(linv + (size_t)mat * kLinvElems + kLinvXOff);
  float4 xr[NB * NB / 4 / 256];
#pragma unroll
  for (int u = 0; u < NB * NB / 4 / 256; ++u) xr[u] = xs[tid + 256 * u];
#pragma unroll
  for (int u = 0; u < NB * NB / 4 / 256; ++u) {
    const int e = tid + 256 * u, rw = e / (NB / 4), q = e % (NB / 4);
    *reinterpret_cast<float4*>(&sX[rw][4 * q]) = xr[u];
  }
  __syncthreads();
  using Acc = Mma<float>::acc;
  Acc acc[2][8];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) acc[rb][cb] = Acc{0, 0, 0, 0};
  // X is upper triangular: column block cb takes the K rows 0 .. 16 cb + 15
#pragma unroll
  for (int q = 0; q < 32; ++q)
#pragma unroll
    for (int cb = q / 4; cb < 8; ++cb) {
      const float bv = sX[4 * q + lk][16 * cb + li];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) acc[rb][cb] = Mma<float>::step(av[q][rb], bv, acc[rb][cb]);
    }
  // every A21 entry of these rows is in registers: L21 goes out in place
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 8; ++cb)
      *reinterpret_cast<float4*>(A + (size_t)(k0 + 16 * cb + li) * npad + r0 + 32 * w + 16 * rb + 4 * lk) =
          make_float4(acc[rb][cb][0], acc[rb][cb][1], acc[rb][cb][2], acc[rb][cb][3]);
}

// ---------------------------------------------------------------------------
// Inverses of the eight 16 x 16 unit lower diagonal blocks of the panel's L11
// (one block of 128 threads per matrix; thread = one column of one block, by
// forward substitution in registers).  Output: the first 8 x 256 elements of
// the matrix's kLinvElems slot, [b][r][c] row-major.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(128) void k_dinv(const T* __restrict__ LU, T* __restrict__ dinv, int npad, int k0) {
  __shared__ T sD[8][16][17];
  const int mat = blockIdx.x, tid = threadIdx.x;
  const T* A = LU + (size_t)mat * npad * npad;
  for (int e = tid; e < 8 * 256; e += 128) {
    const int b = e >> 8, c = (e >> 4) & 15, r = e & 15;
    sD[b][r][c] = A[(size_t)(k0 + 16 * b + c) * npad + k0 + 16 * b + r];
  }
  __syncthreads();
  const int b = tid >> 4, c = tid & 15;
  T x[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = (r == c) ? T(1) : T(0);
#pragma unroll
  for (int r = 1; r < 16; ++r)
#pragma unroll
    for (int k = 0; k < r; ++k) x[r] -= sD[b][r][k] * x[k];
  T* out = dinv + (size_t)mat * kLinvElems + b * 256;
#pragma unroll
  for (int r = 0; r < 16; ++r) out[r * 16 + c] = x[r];
}

// ---------------------------------------------------------------------------
// L11^-1 by blocked forward substitution on the identity, 32 columns per block
// (two wavefronts, one 16-column MFMA block each): by 16-row blocks I,
//   T_I = E_I - sum_{J<I} L_IJ Y_J,   Y_I = X_II T_I   (two MFMA products),
// with X_II the inverse of the diagonal block (k_dinv) and the next block row
// of L11 prefetched into registers while the current one is in use.  The four
// blocks of a matrix write L11^-1 column-major after the diagonal-block
// inverses in the matrix's kLinvElems slot.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(128) void k_l11inv(const T* __restrict__ LU, T* __restrict__ linv, int npad, int k0,
                                                int nmat) {
  constexpr int CT = 32, LDB = CT + 4, LDL = NB + 4;
  int mat, ct;
  xcd_map(blockIdx.x, NB / CT, nmat, &mat, &ct);
  if (mat >= nmat) return;
  const T* A = LU + (size_t)mat * npad * npad;
  __shared__ T sB[NB][LDB];
  __shared__ T sLr[16][LDL];   // block row I of L11: rows 16I.., columns 0..16I+15
  __shared__ T sX[16][17];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const T* Xg = linv + (size_t)mat * kLinvElems;
  // register prefetch of one block row of L11 (16 x up to 128) and its X_II
  T pl[16], px[2];
  auto fetch = [&](int I) {
    const int ncol = 16 * I + 16;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 128 * u, c = e >> 4, r = e & 15;
      pl[u] = (c < ncol) ? A[(size_t)(k0 + c) * npad + k0 + 16 * I + r] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) px[u] = Xg[I * 256 + tid + 128 * u];
  };
  auto put = [&]() {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = tid + 128 * u;
      sLr[e & 15][e >> 4] = pl[u];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int e = tid + 128 * u;
      sX[e >> 4][e & 15] = px[u];
    }
  };
  fetch(0);
  for (int e = tid; e < NB * CT; e += 128) {
    const int k = e % NB, j = e / NB;
    sB[k][j] = (k == ct * CT + j) ? T(1) : T(0);
  }
  put();
  __syncthreads();
  const int col = 16 * w + li;
  for (int I = 0; I < NB / 16; ++I) {
    const int r0 = 16 * I;
    if (I + 1 < NB / 16) fetch(I + 1);
    if (I > 0) {
      typename Mma<T>::acc acc = typename Mma<T>::acc{0, 0, 0, 0};
      for (int k = 0; k < r0; k += 4) acc = Mma<T>::step(sLr[li][k + lk], sB[k + lk][col], acc);
#pragma unroll
      for (int it = 0; it < 4; ++it) sB[r0 + Mma<T>::row(lk, it)][col] -= acc[it];
      __syncthreads();
    }
    typename Mma<T>::acc u = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 16; k += 4) u = Mma<T>::step(sX[li][k + lk], sB[r0 + k + lk][col], u);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < 4; ++it) sB[r0 + Mma<T>::row(lk, it)][col] = u[it];
    if (I + 1 < NB / 16) put();
    __syncthreads();
  }
  T* out = linv + (size_t)mat * kLinvElems + 8 * 256;
  for (int e = tid; e < NB * CT; e += 128) {
    const int k = e % NB, j = e / NB;
    out[(size_t)(ct * CT + j) * NB + k] = sB[k][j];
  }
}

// ---------------------------------------------------------------------------
// The panel's interchanges and U12 = L11^-1 P A12 as one MFMA product per
// 128-column tile, with the explicit L11^-1 of k_l11inv (the blocks of its
// zero upper triangle skipped): the tile of
// P A12 is gathered (rows src[k] of the original columns) chunk by chunk into
// double-buffered LDS as the K operand (or read as vectors from W, below),
// L11^-1 (column-major, read by all tiles of the matrix from L2)
// as the row operand; four wavefronts of 64 x 64, the result written through
// LDS down whole columns.  The
// rows that the interchanges move below the panel are read first (each thread
// stages its own elements) and written after the last chunk, when every read
// of the tile's columns has been made.
// ---------------------------------------------------------------------------
template <typename T, bool FROM_W = false>
__global__ __launch_bounds__(256, 2) void k_u12(T* __restrict__ LU, const T* __restrict__ linv,
                                               const int* __restrict__ perm, T* __restrict__ xscr, int npad, int k0,
                                               int nct, int nmat) {
  using V = typename Vec4<T>::type;
  constexpr int PER = Vec4<T>::per;
  // LDS rows of the K chunk (64 banks of 4 bytes).  FP32: a pitch of 144 puts
  // an operand read (lanes li + 16 lk, rows k + lk) on 64 distinct banks; the
  // transposed stores of the K operand write column j of row r at j ^ SW(r),
  // SW(r) = 16 ((r / 4) mod 4) for the vectors of W (16 columns, rows 4 q + m)
  // and 4 ((r / 4) mod 4) for the gather (4 columns, rows k), which keeps them
  // conflict-free as well; SW is uniform over a wave at each k step.
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int KC = 16, LD = F32 ? 128 + 16 : 128 + 4;
  auto sw = [](int r) { return F32 ? (FROM_W ? 16 : 4) * ((r >> 2) & 3) : 0; };
  int mat, ct;
  xcd_map(blockIdx.x, nct, nmat, &mat, &ct);
  if (mat >= nmat) return;
  T* A = LU + (size_t)mat * npad * npad;
  const T* Li = linv + (size_t)mat * kLinvElems + 8 * 256;
  const int c0 = k0 + NB + ct * 128;
  const int* pm = perm + ((size_t)mat * kMaxPanels + k0 / NB) * kPermStride;
  const int nR = pm[0];
  const int* R = pm + 1;
  const int* src = pm + 1 + kMaxSwapRows;
  constexpr int LE = 64 + 1;                      // epilogue: a pass of 64 rows, column-major
  static_assert(128 * LE <= 4 * KC * LD, "an epilogue pass fits in the operand buffers");
  static_assert(PER == 2 || PER == 4, "4 rows of W are one or two vectors");
  __shared__ __align__(16) T smem[4 * KC * LD];   // the operand chunks, then the epilogue passes
  T (*sA)[KC][LD] = reinterpret_cast<T (*)[KC][LD]>(smem);
  T (*sB)[KC][LD] = reinterpret_cast<T (*)[KC][LD]>(smem + 2 * KC * LD);
  __shared__ int s_src[NB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wc = (w & 1) * 64;
  // L11^-1 is lower triangular: row block b (rows 16 b .. 16 b + 15) takes the
  // K chunks 0..b only.  The two wave rows own the row blocks {0, 3, 4, 7} and
  // {1, 2, 5, 6}, 18 of the 36 nonzero block products each.
  const int rsel = __builtin_amdgcn_readfirstlane(tid >> 7);
  int rowb[4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi) rowb[bi] = 4 * (bi >> 1) + ((bi & 1) ? 3 - rsel : rsel);
  if (tid < NB) s_src[tid] = src[tid];
  // FROM_W: the tile of P A12 is already gathered (and updated) in xscr as
  // W[col][k], and the interchanges' other rows are already moved
  const int nx = FROM_W ? 0 : nR - NB;
  T* xs = xscr + ((size_t)mat * npad + c0) * NB;
  for (int e = tid; e < nx * 128; e += 256) {
    const int t = NB + e % nx, j = e / nx;
    xs[(size_t)j * NB + (t - NB)] = A[(size_t)(c0 + j) * npad + src[t]];
  }
  __syncthreads();
  constexpr int NA = KC * 128 / PER / 256;   // vectors of L11^-1 per thread and chunk
  constexpr int NBS = KC * 128 / 256;        // B elements per thread and chunk
  V ra[NA];
  T rb[NBS];
  auto load = [&](int kk) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + u * 256;
      const int k = e / (128 / PER), i = (e % (128 / PER)) * PER;
      ra[u] = *reinterpret_cast<const V*>(Li + (size_t)(kk + k) * NB + i);
    }
    if constexpr (FROM_W) {
      // W is k-contiguous: rows kk + 4 q .. + 3 of column j as one or two vectors
#pragma unroll
      for (int u = 0; u < NBS / 4; ++u) {
        const int e = tid + u * 256;
        const int q = e % (KC / 4), j = e / (KC / 4);
#pragma unroll
        for (int h = 0; h < 4 / PER; ++h) {
          const V v = *reinterpret_cast<const V*>(xs + (size_t)j * NB + kk + 4 * q + h * PER);
          const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
          for (int m = 0; m < PER; ++m) rb[4 * u + h * PER + m] = pv[m];
        }
      }
    } else {
      // the gather: 16 lanes read rows src[kk..kk+15] of one column
#pragma unroll
      for (int u = 0; u < NBS; ++u) {
        const int e = tid + u * 256;
        const int k = e % KC, j = e / KC;
        rb[u] = A[(size_t)(c0 + j) * npad + s_src[kk + k]];
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + u * 256;
      const int k = e / (128 / PER), i = (e % (128 / PER)) * PER;
      const T* v = reinterpret_cast<const T*>(&ra[u]);
#pragma unroll
      for (int m = 0; m < PER; ++m) sA[buf][k][i + m] = v[m];
    }
    if constexpr (FROM_W) {
#pragma unroll
      for (int u = 0; u < NBS / 4; ++u) {
        const int e = tid + u * 256;
        const int q = e % (KC / 4), j = e / (KC / 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) sB[buf][4 * q + i][j ^ sw(4 * q + i)] = rb[4 * u + i];
      }
    } else {
#pragma unroll
      for (int u = 0; u < NBS; ++u) {
        const int e = tid + u * 256;
        sB[buf][e % KC][(e / KC) ^ sw(e % KC)] = rb[u];
      }
    }
  };
  typename Mma<T>::acc acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = typename Mma<T>::acc{0, 0, 0, 0};
  load(0);
  store(0);
  __syncthreads();
  constexpr int NCH = NB / KC;
  for (int ch = 0; ch < NCH; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < NCH) load((ch + 1) * KC);
#pragma unroll
    for (int k = 0; k < KC; k += 4) {
      T av[4], bv[4];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) av[bi] = sA[buf][k + lk][rowb[bi] * 16 + li];
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) bv[bj] = sB[buf][k + lk][(wc + bj * 16 + li) ^ sw(k)];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) {
        if (ch <= rowb[bi]) {  // KC = 16: chunk ch is row block ch of the K range
#pragma unroll
          for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = Mma<T>::step(av[bi], bv[bj], acc[bi][bj]);
        }
      }
    }
    if (ch + 1 < NCH) {
      store(buf ^ 1);
      __syncthreads();
    }
  }
  // every gather of the tile's columns was consumed before the last barrier.
  // The tile goes out through LDS in two passes of 64 rows (row blocks 4 h ..
  // 4 h + 3, which are bi = 2 h, 2 h + 1 of both wave rows), so that each
  // thread writes whole vectors down a column.
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
    T(*sE)[LE] = reinterpret_cast<T(*)[LE]>(smem);
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const int bi = 2 * h + bb;
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
#pragma unroll
        for (int it = 0; it < 4; ++it)
          sE[wc + bj * 16 + li][rowb[bi] * 16 - 64 * h + Mma<T>::row(lk, it)] = acc[bi][bj][it];
    }
    __syncthreads();
    constexpr int VPC = 64 / PER;   // vectors per column of a pass
#pragma unroll
    for (int u = 0; u < 128 * VPC / 256; ++u) {
      const int e = tid + u * 256;
      const int col = e / VPC, r = (e % VPC) * PER;
      V v;
      T* pv = reinterpret_cast<T*>(&v);
#pragma unroll
      for (int m = 0; m < PER; ++m) pv[m] = sE[col][r + m];
      *reinterpret_cast<V*>(A + (size_t)(c0 + col) * npad + k0 + 64 * h + r) = v;
    }
  }
  for (int e = tid; e < nx * 128; e += 256) {
    const int t = NB + e % nx, j = e / nx;
    if (src[t] != R[t]) A[(size_t)(c0 + j) * npad + R[t]] = xs[(size_t)j * NB + (t - NB)];
  }
}

// ---------------------------------------------------------------------------
// Panels in pairs (p at kp, p+1 at k1 = kp + NB): panel p's update reaches panel
// p+1's columns at once, and is deferred for the columns beyond, where one
// K = 256 update then applies both panels.  Panel p+1's U12 needs its top rows
// (after the interchanges of panel p+1) with panel p's update applied; these
// kernels form them and keep the deferred update consistent:
//   k_u12pre     W[col][k] = A[src[k]][col] - sum_i L_p[src[k]][i] U_p[i][col]
//                for the 128 rows src[k] that the interchanges of panel p+1
//                bring to its top block: one MFMA product per 128-column tile,
//                the gathered rows of L_p as the row operand; into xscr, which
//                k_u12<T, true> then takes in place of its gather;
//   k_move_down  the interchanges' other rows, A[R[t]] = A[src[t]] (t >= 128):
//                contents only ever leave the top block downwards, so every
//                source is a top-block row, not yet overwritten by U12;
//   k_perm_lp    the interchanges applied to panel p's L columns as well, so
//                that each row's deferred update moves with it; the solve then
//                applies P_{p+1} before L_p (A = P_p^T P_{p+1}^T L' U per pair).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256, 2) void k_u12pre(T* __restrict__ LU, const int* __restrict__ perm,
                                                T* __restrict__ xscr, int npad, int k1, int nct, int nmat,
                                                int ident, int kj) {
  using V = typename Vec4<T>::type;
  constexpr int PER = Vec4<T>::per;
  // FP32 operand layout as in k_u12 (the U_p stores are W's pattern)
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int KC = 16, LD = F32 ? 128 + 16 : 128 + 4;
  auto sw = [](int r) { return F32 ? 16 * ((r >> 2) & 3) : 0; };
  int mat, ct;
  xcd_map(blockIdx.x, nct, nmat, &mat, &ct);
  if (mat >= nmat) return;
  T* A = LU + (size_t)mat * npad * npad;
  // the deferred updates of the kj panels before this one (a pair's first
  // panel: kj = 1; in groups of four, up to 3): K = 128 kj from column kp
  const int kp = k1 - kj * NB;
  const int c0 = k1 + NB + ct * 128;
  const int* src = perm + ((size_t)mat * kMaxPanels + k1 / NB) * kPermStride + 1 + kMaxSwapRows;
  __shared__ __align__(16) T smem[4 * KC * LD];   // the operand chunks, then the passes of W
  T (*sA)[KC][LD] = reinterpret_cast<T (*)[KC][LD]>(smem);
  T (*sB)[KC][LD] = reinterpret_cast<T (*)[KC][LD]>(smem + 2 * KC * LD);
  __shared__ int s_src[NB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  // ident: statically pivoted factors, whose top rows are the panel's own (the
  // identity that the diagonal kernel records too), so that this kernel need
  // not wait for it
  if (tid < NB) s_src[tid] = ident ? k1 + tid : src[tid];
  __syncthreads();
  constexpr int NAS = KC * 128 / 256;         // gathered L_p elements per thread and chunk
  constexpr int NBV = KC * 128 / PER / 256;   // U_p vectors per thread and chunk
  T ra[NAS];
  V rb[NBV];
  auto load = [&](int kk) {
#pragma unroll
    for (int u = 0; u < NAS; ++u) {
      const int e = tid + u * 256;
      ra[u] = A[(size_t)(kp + kk + e / 128) * npad + s_src[e % 128]];
    }
#pragma unroll
    for (int u = 0; u < NBV; ++u) {
      const int e = tid + u * 256;
      const int j = e / (KC / PER), k = (e % (KC / PER)) * PER;
      rb[u] = *reinterpret_cast<const V*>(A + (size_t)(c0 + j) * npad + kp + kk + k);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NAS; ++u) {
      const int e = tid + u * 256;
      sA[buf][e / 128][e % 128] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NBV; ++u) {
      const int e = tid + u * 256;
      const int j = e / (KC / PER), k = (e % (KC / PER)) * PER;
      const T* v = reinterpret_cast<const T*>(&rb[u]);
#pragma unroll
      for (int m = 0; m < PER; ++m) sB[buf][k + m][j ^ sw(k + m)] = v[m];
    }
  };
  typename Mma<T>::acc acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = typename Mma<T>::acc{0, 0, 0, 0};
  load(0);
  store(0);
  __syncthreads();
  const int NCH = kj * (NB / KC);
  for (int ch = 0; ch < NCH; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < NCH) load((ch + 1) * KC);
#pragma unroll
    for (int k = 0; k < KC; k += 4) {
      T av[4], bv[4];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) av[bi] = sA[buf][k + lk][wr + bi * 16 + li];
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) bv[bj] = sB[buf][k + lk][(wc + bj * 16 + li) ^ sw(k)];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = Mma<T>::step(av[bi], bv[bj], acc[bi][bj]);
    }
    if (ch + 1 < NCH) {
      store(buf ^ 1);
      __syncthreads();
    }
  }
  // W = A[src rows] - acc, through LDS in two passes of 64 rows (a wave row's
  // tile each), so that the gathered reads and the vector stores of W run down
  // the columns
  T* xs = xscr + ((size_t)mat * npad + c0) * NB;
  constexpr int LE = 64 + 1;
  static_assert(128 * LE <= 4 * KC * LD, "a pass of the tile fits in the operand buffers");
  T(*sC)[LE] = reinterpret_cast<T(*)[LE]>(smem);
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    __syncthreads();
    if (wr == 64 * pass) {
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
          for (int it = 0; it < 4; ++it) sC[wc + bj * 16 + li][bi * 16 + Mma<T>::row(lk, it)] = acc[bi][bj][it];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 128 * 64 / 4 / 256; ++u) {
      const int e = tid + u * 256;
      const int n = e / 16, rr = (e % 16) * 4, m = pass * 64 + rr;
      const T* cp = A + (size_t)(c0 + n) * npad;
      T v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = cp[s_src[m + i]] - sC[n][rr + i];
#pragma unroll
      for (int h = 0; h < 4 / PER; ++h) {
        V o;
        T* po = reinterpret_cast<T*>(&o);
#pragma unroll
        for (int q = 0; q < PER; ++q) po[q] = v[h * PER + q];
        *reinterpret_cast<V*>(xs + (size_t)n * NB + m + h * PER) = o;
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_move_down(T* __restrict__ LU, const int* __restrict__ perm, int npad,
                                                   int k1, int nct, int nmat) {
  int mat, ct;
  xcd_map(blockIdx.x, nct, nmat, &mat, &ct);
  if (mat >= nmat) return;
  T* A = LU + (size_t)mat * npad * npad;
  const int c0 = k1 + NB + ct * 128;
  const int* pm = perm + ((size_t)mat * kMaxPanels + k1 / NB) * kPermStride;
  const int nx = pm[0] - NB;
  const int* R = pm + 1;
  const int* src = pm + 1 + kMaxSwapRows;
  for (int e = threadIdx.x; e < nx * 128; e += 256) {
    const int t = NB + e % nx, j = e / nx;
    if (src[t] != R[t]) A[(size_t)(c0 + j) * npad + R[t]] = A[(size_t)(c0 + j) * npad + src[t]];
  }
}

// panel p's L columns, rows R[t] <- src[t] for every t (16 columns per block:
// all reads before the block's writes)
template <typename T>
__global__ __launch_bounds__(256) void k_perm_lp(T* __restrict__ LU, const int* __restrict__ perm, int npad, int k1,
                                                 int nmat) {
  int mat, cg;
  xcd_map(blockIdx.x, NB / 16, nmat, &mat, &cg);
  if (mat >= nmat) return;
  T* A = LU + (size_t)mat * npad * npad;
  const int kp = k1 - NB;
  const int* pm = perm + ((size_t)mat * kMaxPanels + k1 / NB) * kPermStride;
  const int nR = pm[0];
  const int* R = pm + 1;
  const int* src = pm + 1 + kMaxSwapRows;
  constexpr int NV = kMaxSwapRows * 16 / 256;
  T v[NV];
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int e = threadIdx.x + u * 256;
    if (e < nR * 16) v[u] = A[(size_t)(kp + 16 * cg + e / nR) * npad + src[e % nR]];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    const int e = threadIdx.x + u * 256;
    if (e < nR * 16 && src[e % nR] != R[e % nR]) A[(size_t)(kp + 16 * cg + e / nR) * npad + R[e % nR]] = v[u];
  }
}

// ---------------------------------------------------------------------------
// One wavefront's triangular solve with a 128 x 128 diagonal block staged in
// LDS; v0 / v1 hold rows lane / 64 + lane and each solved value is passed on by
// a lane read.  FWD: ascending (lower triangular), else descending (upper);
// SCALE: a value is multiplied by the reciprocal of its diagonal entry (s_rc)
// before it is passed on (non-unit diagonal); TR: the block is used
// transposed.  The staged block holds only the strict triangle that the chain
// reads, with zeros elsewhere, so every step updates all rows without a mask
// (a finished row gets exactly zero).  A scaled row keeps its unscaled value
// to the end and is multiplied once after the chain, giving the same product
// as scaling it at its own step.  For FP32 and FP16 factors the entries the
// chain needs are read from LDS in chunks of 4 pivots with the next chunk in
// flight, so that the sequential chain does not wait on an LDS read at every
// step; the two halves of the block are separate loops, so that the register
// holding the current pivot is known at compile time and the half of the rows
// that a half of the pivots cannot reach is skipped.
// ---------------------------------------------------------------------------
template <typename T, bool FWD, bool SCALE, bool TR, int H>
__device__ __attribute__((always_inline)) inline void diag_half(const T (*sD)[NB + 1], const double* s_rc,
                                                                int lane, double& v0, double& v1) {
  // pivots 64 H .. 64 H + 63, whose values live in v0 (H = 0) or v1 (H = 1);
  // the entries of 4 pivots are in registers while those of the next 4 load
  constexpr int CH = 4;
  constexpr int base = 64 * H;
  constexpr bool R0 = FWD ? H == 0 : true;   // rows 0 .. 63 below / above these pivots
  constexpr bool R1 = FWD ? true : H == 1;   // rows 64 .. 127
  T c0[CH], c1[CH], n0[CH], n1[CH];
  double q[CH], nq[CH];
  auto ld = [&](T (&a)[CH], T (&b)[CH], double (&r)[CH], int i0) {
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (R0) a[u] = TR ? sD[i0 + u][lane] : sD[lane][i0 + u];
      if (R1) b[u] = TR ? sD[i0 + u][64 + lane] : sD[64 + lane][i0 + u];
      if (SCALE) r[u] = s_rc[i0 + u];
    }
  };
  ld(c0, c1, q, base + (FWD ? 0 : 64 - CH));
  for (int k = 0; k < 64 / CH; ++k) {
    const int i0 = base + (FWD ? k * CH : 64 - CH - k * CH);
    if (k + 1 < 64 / CH) ld(n0, n1, nq, FWD ? i0 + CH : i0 - CH);
#pragma unroll
    for (int uu = 0; uu < CH; ++uu) {
      const int u = FWD ? uu : CH - 1 - uu;
      double xi = readlane_f64(H ? v1 : v0, i0 + u - base);
      if constexpr (SCALE) xi *= q[u];
      if constexpr (R0) v0 -= static_cast<double>(c0[u]) * xi;
      if constexpr (R1) v1 -= static_cast<double>(c1[u]) * xi;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      c0[u] = n0[u];
      c1[u] = n1[u];
      q[u] = nq[u];
    }
  }
}

template <typename T, bool FWD, bool SCALE, bool TR>
__device__ __attribute__((always_inline)) inline void diag_chain(const T (*sD)[NB + 1], const double* s_rc,
                                                                 int lane, double& v0, double& v1) {
  if constexpr (sizeof(T) == 8) {
    // FP64: one loop, unrolled by 4 (prefetched chunks spill next to the strip)
#pragma unroll 4
    for (int k = 0; k < NB; ++k) {
      const int i = FWD ? k : NB - 1 - k;
      const double l0 = TR ? sD[i][lane] : sD[lane][i];
      const double l1 = TR ? sD[i][64 + lane] : sD[64 + lane][i];
      double xi = (i < 64) ? readlane_f64(v0, i) : readlane_f64(v1, i - 64);
      if constexpr (SCALE) xi *= s_rc[i];
      v0 -= l0 * xi;
      v1 -= l1 * xi;
    }
  } else if constexpr (FWD) {
    diag_half<T, FWD, SCALE, TR, 0>(sD, s_rc, lane, v0, v1);
    diag_half<T, FWD, SCALE, TR, 1>(sD, s_rc, lane, v0, v1);
  } else {
    diag_half<T, FWD, SCALE, TR, 1>(sD, s_rc, lane, v0, v1);
    diag_half<T, FWD, SCALE, TR, 0>(sD, s_rc, lane, v0, v1);
  }
  if constexpr (SCALE) {
    v0 *= s_rc[lane];
    v1 *= s_rc[64 + lane];
  }
}

// ---------------------------------------------------------------------------
// Solve with the factors (one 1024-thread block per matrix), FP64 right-hand side.
// transpose = 0: x = U^-1 L_m^-1 P_m ... L_1^-1 P_1 b
// transpose = 1: y = P_1^T L_1^-T ... P_m^T L_m^-T U^-T c
// Diagonal blocks are staged in LDS and solved by one wavefront (two rows per
// lane); the off-diagonal strips are applied column-oriented (thread per row)
// or, for the transposed factors, as per-column dot products (wave per column).
// The next diagonal block is loaded into registers before the strip that
// precedes its use, so that its loads travel with the strip's; a panel's
// gather / scatter is skipped when the panel interchanges no rows (always,
// for statically pivoted factors).
// ---------------------------------------------------------------------------
template <typename T, int TRANSPOSE>
__global__ __launch_bounds__(1024) void k_solve(const T* __restrict__ LU, const int* __restrict__ piv,
                                                const int* __restrict__ perm, const double* __restrict__ Bin,
                                                double* __restrict__ Xout,
                                                const int* __restrict__ status, int accumulate, int check_done,
                                                int npad, const int* __restrict__ mat_of,
                                                const int* __restrict__ skip, int band_lo, int band_up, int paired,
                                                const int* __restrict__ mirror, int n, int nth) {
  if (check_done && status[1]) return;
  // right-hand side / solution row: the block; factors: that row's own matrix,
  // or the one mat_of names (a shared factorization, e.g. a preconditioner bin)
  const int row = blockIdx.x;
  if (skip && skip[row]) return;
  __shared__ double sb[kMaxRows];
  __shared__ T sD[NB][NB + 1];
  __shared__ double s_rc[NB];
  __shared__ int s_nr[kMaxPanels];
  __shared__ double s_part[sizeof(T) < 8 ? 512 * Vec4<T>::per : 1];
  const int mat = mat_of ? mat_of[row] : row;
  const T* A = LU + (size_t)mat * npad * npad;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr int NWV = 1024 / 64;
  const double* b = Bin + (size_t)row * npad;
  // factors of the mirrored matrix: the right-hand side comes in mirrored and
  // the solution goes out mirrored (ordinate theta -> nth-1-theta of each speed)
  const bool mir = mirror && mirror[mat];
  auto src = [&](int i) { return (mir && i < n) ? (i / nth) * nth + (nth - 1 - i % nth) : i; };
  for (int i = tid; i < npad; i += 1024) sb[i] = b[src(i)];
  const int np = npad / NB;
  const int* pmat = perm + (size_t)mat * kMaxPanels * kPermStride;
  if (tid < np) s_nr[tid] = pmat[(size_t)tid * kPermStride];   // rows each panel's interchanges move
  // sb[r] -= sum_j A[r][k0 + j] sb[k0 + j] for rows r in [r_lo, r_hi): each
  // thread takes a 16-byte vector of consecutive rows (4 FP32 / 2 FP64) and keeps
  // JB column loads in flight (16 FP32, 8 FP64 and FP16: 16 FP64 loads spilled); FP32 and FP16 split the 128 columns between the
  // two halves of the block and add the halves through LDS
  auto strip = [&](int k0, int r_lo, int r_hi) {
    using V = typename Vec4<T>::type;
    constexpr int PER = Vec4<T>::per;
    constexpr int H = sizeof(T) < 8 ? 2 : 1;    // column groups
    constexpr int CW = NB / H, JB = sizeof(T) == 4 ? 16 : 8, TPG = 1024 / H;
    const int grp = tid / TPG, lt = tid % TPG;
    for (int r0 = r_lo; r0 < r_hi; r0 += TPG * PER) {
      const int r = r0 + lt * PER;
      const bool v = r < r_hi;
      double acc[PER];
#pragma unroll
      for (int m = 0; m < PER; ++m) acc[m] = 0.0;
      for (int jb = 0; jb < CW; jb += JB) {
        V x[JB];
#pragma unroll
        for (int u = 0; u < JB; ++u) {
          const int c = k0 + grp * CW + jb + u;
          if (v) x[u] = ntload(reinterpret_cast<const V*>(A + (size_t)c * npad + r));
        }
#pragma unroll
        for (int u = 0; u < JB; ++u) {
          const double bj = sb[k0 + grp * CW + jb + u];
          const T* e = reinterpret_cast<const T*>(&x[u]);
#pragma unroll
          for (int m = 0; m < PER; ++m) acc[m] += static_cast<double>(e[m]) * bj;
        }
      }
      if (H == 2) {
        if (grp == 1 && v) {
#pragma unroll
          for (int m = 0; m < PER; ++m) s_part[lt * PER + m] = acc[m];
        }
        __syncthreads();
        if (grp == 0 && v) {
#pragma unroll
          for (int m = 0; m < PER; ++m) sb[r + m] -= acc[m] + s_part[lt * PER + m];
        }
        __syncthreads();
      } else if (v) {
#pragma unroll
        for (int m = 0; m < PER; ++m) sb[r + m] -= acc[m];
      }
    }
  };
  // diagonal block of the panel at k0: loads into registers, then LDS stores
  // of the strict triangle the chain reads (lower: L; upper: U, whose
  // diagonal goes to s_rc as reciprocals), zeros elsewhere
  constexpr int NS = NB * NB / 1024;
  T dv[NS];
  auto load_diag = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = tid + 1024 * u;
      dv[u] = A[(size_t)(k0 + e / NB) * npad + k0 + e % NB];
    }
  };
  auto store_diag = [&](bool upper) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int e = tid + 1024 * u;
      const int r = e % NB, c = e / NB;
      if (upper && r == c) s_rc[r] = 1.0 / static_cast<double>(dv[u]);
      sD[r][c] = (upper ? r < c : r > c) ? dv[u] : T(0);
    }
  };
  // the panel's interchanges as one gather / scatter over its rows (INV: the
  // inverse), skipped when the panel moves no rows
  auto permute = [&](int q, bool inv) {
    const int nR = s_nr[q];
    if (nR == 0) return;
    const int* pm = pmat + (size_t)q * kPermStride;
    double pv = 0.0;
    if (tid < nR) pv = sb[pm[1 + (inv ? 0 : kMaxSwapRows) + tid]];
    __syncthreads();
    if (tid < nR) sb[pm[1 + (inv ? kMaxSwapRows : 0) + tid]] = pv;
    __syncthreads();
  };
  // wave 0 solves the panel's rows of sb with the staged block
  auto chain = [&](int k0, auto fwd, auto scale, auto tr) {
    if (w == 0) {
      double v0 = sb[k0 + lane], v1 = sb[k0 + 64 + lane];
      diag_chain<T, decltype(fwd)::value, decltype(scale)::value, decltype(tr)::value>(sD, s_rc, lane, v0, v1);
      sb[k0 + lane] = v0;
      sb[k0 + 64 + lane] = v1;
    }
  };
  using Yes = std::true_type;
  using No = std::false_type;
  load_diag(0);
  __syncthreads();
  if (!TRANSPOSE) {
    for (int p = 0; p < np; ++p) {
      const int k0 = p * NB;
      // P_p (a pair's first panel applies P_{p+1} too, its second none)
      const bool first = paired && p % 2 == 0 && p + 2 < np;
      const bool second = paired && p % 2 == 1 && p + 1 < np;
      store_diag(false);
      if (!second) permute(p, false);
      if (first) permute(p + 1, false);
      __syncthreads();
      chain(k0, Yes(), No(), No());   // unit lower triangular diagonal block
      __syncthreads();
      if (p + 1 < np) load_diag(k0 + NB);   // the last panel's block serves U too
      // banded factors: L below a panel reaches band_lo rows
      strip(k0, k0 + NB, band_lo > 0 ? min(npad, (k0 + NB + band_lo + NB - 1) / NB * NB) : npad);
      __syncthreads();
    }
    for (int p = np - 1; p >= 0; --p) {
      const int k0 = p * NB;
      store_diag(true);
      __syncthreads();
      chain(k0, No(), Yes(), No());   // upper triangular diagonal block
      __syncthreads();
      if (p > 0) load_diag(k0 - NB);
      // banded factors: U has upper bandwidth band_up (kl + ku with the fill of
      // the interchanges)
      strip(k0, band_up > 0 ? max(0, (k0 - band_up) / NB * NB) : 0, k0);
      __syncthreads();
    }
  } else {
    // z = U^-T c, forward over panels (U^T is lower triangular)
    for (int p = 0; p < np; ++p) {
      const int k0 = p * NB;
      store_diag(true);
      __syncthreads();
      chain(k0, Yes(), Yes(), Yes());
      __syncthreads();
      if (p + 1 < np) load_diag(k0 + NB);   // the last panel's block serves L^T too
      // c[col] -= sum_j U[k0+j][col] z_j for col >= k0 + NB (wave per column)
      for (int col = k0 + NB + w; col < npad; col += NWV) {
        const T* cp = A + (size_t)col * npad + k0;
        double s = static_cast<double>(cp[lane]) * sb[k0 + lane] +
                   static_cast<double>(cp[64 + lane]) * sb[k0 + 64 + lane];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) sb[col] -= s;
      }
      __syncthreads();
    }
    // for p = m..1: z <- L_p^-T z, then z <- P_p^T z
    for (int p = np - 1; p >= 0; --p) {
      const int k0 = p * NB;
      if (p < np - 1) load_diag(k0);
      // z_j -= sum_{r >= k0+NB} L[r][k0+j] z_r (wave per column j)
      for (int j = w; j < NB; j += NWV) {
        const T* cp = A + (size_t)(k0 + j) * npad;
        double s = 0.0;
        for (int r = k0 + NB + lane; r < npad; r += 64) s += static_cast<double>(cp[r]) * sb[r];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) sb[k0 + j] -= s;
      }
      store_diag(false);
      __syncthreads();
      chain(k0, No(), No(), Yes());   // L11^T is unit upper triangular
      __syncthreads();
      // P_p^T: inverse of the panel's gather / scatter (a pair's first panel
      // applies P_{p+1}^T then P_p^T, its second none)
      const bool first = paired && p % 2 == 0 && p + 2 < np;
      const bool second = paired && p % 2 == 1 && p + 1 < np;
      if (!second) {
        if (first) permute(p + 1, true);
        permute(p, true);
      }
      __syncthreads();
    }
  }
  double* xo = Xout + (size_t)row * npad;
  for (int i = tid; i < npad; i += 1024) xo[i] = accumulate ? xo[i] + sb[src(i)] : sb[src(i)];
}

template <typename T>
void factor_impl(const DevOps& d, hipStream_t s, LuTimer* tm, int m0, int nmat, int bf16_terms,
                 const LuLookAhead* la) {
  const size_t np2 = (size_t)d.npad * d.npad;
  T* LU = static_cast<T*>(d.lu) + (size_t)m0 * np2;
  T* xs = static_cast<T*>(d.xscr) + (size_t)m0 * d.npad * NB;
  T* li = static_cast<T*>(d.linv) + (size_t)m0 * kLinvElems;  // inverses of L11 and its diagonal blocks
  int* piv = d.piv + (size_t)m0 * d.npad;
  int* perm = d.perm + (size_t)m0 * kMaxPanels * kPermStride;
  const int xpb = d.form_xpb > 0 ? d.form_xpb : (sizeof(T) == 4 ? 8 : 16);   // matrices per formation block
  const int np = d.npad / NB;
  const bool stat = std::is_same<T, float>::value && d.static_piv;
  const bool pairs = lu_paired(d);
  auto form = [&](hipStream_t st, int c_lo, int part) {
    const dim3 gform(xcd_grid((nmat + xpb - 1) / xpb, d.npad - c_lo));
    k_form<T><<<gform, 256, 0, st>>>(LU, d.CordT, d.AordT, d.E + m0, d.n0x + m0, d.dt, d.n, d.npad, nmat, xpb,
                                     d.band_kl, d.band_ku, d.mirror ? d.mirror + m0 : nullptr,
                                     (std::is_same<T, float>::value && d.static_piv && d.mirror) ? 1 : 0, c_lo,
                                     part, 2 * NB);
  };
  // formation overlap (optional; statically pivoted dense pairs): the first
  // pair reads only columns and rows below 2 NB until its K = 256 update, so
  // the rest of the matrix is formed on the side stream meanwhile, and that
  // update waits (measured slower at n = 2048: the two share HBM and the CUs)
  // statically pivoted dense factors in groups of four panels (lu_pairs 2):
  // the updates of a group's panels on the columns beyond the group are
  // deferred to one K = 512 update
  const bool quads = stat && d.lu_pairs == 2 && d.band_kl == 0 && np >= 4;
  const bool fsplit = !quads && stat && pairs && la && la->form_overlap && la->side && np >= 4 && d.band_kl == 0;
  if (fsplit) {
    (void)hipEventRecord(la->form_ev[0], s);
    (void)hipStreamWaitEvent(la->side, la->form_ev[0], 0);
    form(la->side, 2 * NB, 2);
    (void)hipEventRecord(la->form_ev[1], la->side);
    form(s, 0, 1);
  } else {
    form(s, 0, 0);
  }
  const int P = tm ? tm->max_panels : 0;
  if (tm) {
    tm->used = 0;
    tm->launches = 0;
  }
  // timer event pair `slot` of panel p (slots: update, panel, remaining update, U12)
  auto mark = [&](int slot, int p, int end, hipStream_t st) {
    (void)hipEventRecord(tm->ev[2 * P * slot + 2 * p + end], st);
  };
  constexpr int IB = sizeof(T) == 8 ? 8 : 16;   // register sub-panel width (VGPR budget of 512 threads)
  const int kind = sizeof(T) == 8 ? 0 : (bf16_terms == 1 ? 2 : (bf16_terms == 3 ? 3 : 1));
  // K chunk of the trailing update (launch shape only: the K order is the same):
  // the default 16, or the alternative 8 (FP64) / 32 (FP32)
  const bool alt_kc = d.update_kc == (sizeof(T) == 8 ? 8 : 32);
  // banded systems (lower / upper bandwidth kl / ku): the rows below a panel end
  // kl below it; partial pivoting widens the upper band to kl + ku
  const int kl = d.band_kl, ku = d.band_ku;
  auto round_up = [](int v) { return (v + NB - 1) / NB * NB; };
  // panels in pairs (dense systems, `pairs` above): panel p's update of the
  // columns beyond panel p+1 is deferred and applied with panel p+1's in one
  // K = 256 update, which reads and writes A22 half as often; the last two
  // panels go singly
  auto panel = [&](int k0, int rend) {
    const int rows = rend - k0;
    constexpr int NT = kPanelThreads;  // 512 threads holding up to 4 rows each
    // block shape and L chunk by panel height (measured): short panels (the
    // last ones, banded systems) take four wavefronts, which have the larger
    // register budget
    // (FP64: chunks of 16 L columns on the shortest panels, which keeps the
    // latency-bound left-looking update to half as many round trips, and
    // 16-column sub-panels where the registers allow, which halves the L
    // re-reads; the sub-panel width does not change the result, every element
    // takes its products in column order either way)
    constexpr bool F64 = sizeof(T) == 8;
    if (rows <= NT / 2) {
      k_panel<T, NT / 2, 1, IB, F64 ? 16 : 8><<<nmat, NT / 2, 0, s>>>(LU, piv, perm, d.status, d.npad, k0, rend);
    } else if (rows <= NT) {
      k_panel<T, NT / 2, 2, 16, 8><<<nmat, NT / 2, 0, s>>>(LU, piv, perm, d.status, d.npad, k0, rend);
    } else if (rows <= 2 * NT) {
      k_panel<T, NT, 2, 16, F64 ? 4 : 8><<<nmat, NT, 0, s>>>(LU, piv, perm, d.status, d.npad, k0, rend);
    } else {
      k_panel<T, NT, 4, IB, F64 ? 4 : 8><<<nmat, NT, 0, s>>>(LU, piv, perm, d.status, d.npad, k0, rend);
    }
  };
  auto update = [&](int k0, int mtr, int mtc, int kd) {
    launch_update(kind, LU, d.npad, k0, mtr, mtc, 0, nmat, alt_kc, s, kd);
    if (tm) ++tm->launches;
  };
  // statically pivoted FP32 panels: the diagonal block and L21 (on stream st)
  auto static_panel = [&](int k0, int rend, hipStream_t st) {
    if constexpr (std::is_same<T, float>::value) {
      k_diag_static<<<nmat, 256, 0, st>>>(LU, li, piv, perm, d.status, d.npad, k0);
      const int nt = (rend - k0 - NB) / NB;   // row tiles of L21 (rend, k0 multiples of 128)
      if (nt > 0) k_l21_mfma<<<xcd_grid(nt, nmat), 256, 0, st>>>(LU, li, d.npad, k0, nt, nmat);
    }
  };
  if (quads) {
    // panel p at position j of its group (g0 = p - j): its columns and its top
    // rows beyond it received the group's earlier panels' updates (one K = 128 j
    // update in place after panel p-1 over the column block and the row block;
    // with no interchanges the top rows are the panel's own), so its U12 comes
    // straight from its rows; after it, either the next panel gets the updates
    // of panels g0..p the same way, or, after the group's last panel, the
    // columns beyond the group get all four (K = 512).  A group that does not
    // fit at the end takes single panels.
    for (int p = 0; p < np; ++p) {
      const int k0 = p * NB;
      const int g0 = p / 4 * 4;
      const bool full = g0 + 4 <= np;
      const int j = full ? p - g0 : 0;
      const bool rec = tm && p < P;
      if (rec) mark(1, p, 0, s);
      static_panel(k0, d.npad, s);
      const int rest = d.npad - k0 - NB;
      const int nct = rest / 128;
      if (rec) {
        mark(1, p, 1, s);
        mark(2, p, 0, s);
        mark(2, p, 1, s);
        mark(3, p, 0, s);
      }
      if (rest > 0) k_u12<T><<<xcd_grid(nct, nmat), 256, 0, s>>>(LU, li, perm, xs, d.npad, k0, nct, nmat);
      if (rec) {
        mark(3, p, 1, s);
        mark(0, p, 0, s);
      }
      const int mtr = rest / 128;
      if (mtr > 0) {
        if (full && j < 3) {
          // the next panel's columns, and its top rows beyond it (first tile row)
          launch_update(kind, LU, d.npad, g0 * NB, mtr, 1, 0, nmat, alt_kc, s, (j + 1) * NB, nct - 1);
          if (tm) ++tm->launches;
        } else if (full) {
          update(g0 * NB, mtr, nct, 4 * NB);       // the columns beyond the group
        } else {
          update(k0, mtr, nct, NB);
        }
      }
      if (rec) {
        mark(0, p, 1, s);
        tm->used = p + 1;
      }
    }
    return;
  }
  const bool ahead = stat && la && la->look_ahead && la->side && la->ev && np <= kMaxPanels;
  bool done_ahead[kMaxPanels] = {};   // panel already factored on the side stream
  for (int p = 0; p < np; ++p) {
    const int k0 = p * NB;
    const bool rec = tm && p < P;
    const bool first = pairs && p % 2 == 0 && p + 2 < np;   // first panel of a pair
    const bool second = pairs && p % 2 == 1 && p + 1 < np;  // second panel of a pair
    if (rec) mark(1, p, 0, s);
    const int rend = kl > 0 ? std::min(d.npad, round_up(k0 + NB + kl)) : d.npad;
    const int cend = kl > 0 ? std::min(d.npad, round_up(k0 + NB + kl + ku)) : d.npad;
    const int rest = cend - k0 - NB;
    if (stat) {
      if (done_ahead[p]) (void)hipStreamWaitEvent(s, la->ev[2 * p + 1], 0);
      else static_panel(k0, rend, s);
    } else {
      panel(k0, rend);
    }
    if (rest > 0 && !stat) k_dinv<T><<<nmat, 128, 0, s>>>(LU, li, d.npad, k0);   // (k_diag_static makes them)
    if (rec) {
      mark(1, p, 1, s);
      mark(2, p, 0, s);
      mark(2, p, 1, s);
      mark(3, p, 0, s);
    }
    const int nct = rest / 128;  // U12 tiles of 128 columns
    if (rest > 0 && !stat) k_l11inv<T><<<xcd_grid(NB / 32, nmat), 128, 0, s>>>(LU, li, d.npad, k0, nmat);   // (k_diag_static forms L11^-1)
    if (second) {
      // this panel's U12 from its top rows with panel p-1's deferred update,
      // the interchanges' other rows moved down, panel p-1's L rows permuted
      // (statically pivoted panels interchange no rows: nothing to move)
      k_u12pre<T><<<xcd_grid(nct, nmat), 256, 0, s>>>(LU, perm, xs, d.npad, k0, nct, nmat, 0, 1);
      if (!stat) k_move_down<T><<<xcd_grid(nct, nmat), 256, 0, s>>>(LU, perm, d.npad, k0, nct, nmat);
      k_u12<T, true><<<xcd_grid(nct, nmat), 256, 0, s>>>(LU, li, perm, xs, d.npad, k0, nct, nmat);
      if (!stat) k_perm_lp<T><<<xcd_grid(NB / 16, nmat), 256, 0, s>>>(LU, perm, d.npad, k0, nmat);
    } else if (rest > 0) {
      k_u12<T><<<xcd_grid(nct, nmat), 256, 0, s>>>(LU, li, perm, xs, d.npad, k0, nct, nmat);
    }
    if (rec) {
      mark(3, p, 1, s);
      mark(0, p, 0, s);
    }
    const int mtr = rest > 0 ? (rend - k0 - NB) / 128 : 0;
    // with the look-ahead, an update that reaches the next panel takes that
    // panel's tile column first; the panel then factors on the side stream
    // while the other tile columns update on this one
    auto update_ahead = [&](int ku0, int kd) {
      const int kn = k0 + NB, rn = kl > 0 ? std::min(d.npad, round_up(kn + NB + kl)) : d.npad;
      launch_update(kind, LU, d.npad, ku0, mtr, 1, 0, nmat, alt_kc, s, kd);
      (void)hipEventRecord(la->ev[2 * (p + 1)], s);
      (void)hipStreamWaitEvent(la->side, la->ev[2 * (p + 1)], 0);
      static_panel(kn, rn, la->side);
      (void)hipEventRecord(la->ev[2 * (p + 1) + 1], la->side);
      done_ahead[p + 1] = true;
      if (nct > 1) launch_update(kind, LU, d.npad, ku0, mtr, nct - 1, 1, nmat, alt_kc, s, kd);
      if (tm) tm->launches += nct > 1 ? 2 : 1;
    };
    if (fsplit && p == 1) (void)hipStreamWaitEvent(s, la->form_ev[1], 0);   // the rest of the matrix is formed
    if (first) {
      update(k0, mtr, 1, NB);                    // the next panel's columns only
    } else if (second) {
      if (ahead && mtr > 0 && nct >= 1) update_ahead(k0 - NB, 2 * NB);
      else update(k0 - NB, mtr, nct, 2 * NB);    // both panels, the columns beyond
    } else if (mtr > 0) {
      if (ahead && nct >= 1 && p + 1 < np) update_ahead(k0, NB);
      else update(k0, mtr, nct, NB);
    }
    if (rec) {
      mark(0, p, 1, s);
      tm->used = p + 1;
    }
  }
}

}  // namespace

void launch_lu_factor(const DevOps& d, int precision, hipStream_t s, LuTimer* timer, int m0, int count,
                      const LuLookAhead* la) {
  if (count < 0) count = d.nx_total - m0;
  if (count <= 0) return;
  // precision: 0 FP64, 1 FP32, 2 FP32 with a bf16 update, 3 FP32 with a split (3-term) bf16 update
  if (precision == 0) factor_impl<double>(d, s, timer, m0, count, 0, nullptr);
  else factor_impl<float>(d, s, timer, m0, count, precision == 2 ? 1 : (precision == 3 ? 3 : 0), la);
}

namespace {
__global__ void k_to_half(const float* __restrict__ src, _Float16* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = static_cast<_Float16>(src[i]);
}
}  // namespace

void launch_to_half(const float* src, void* dst, size_t n, hipStream_t s) {
  k_to_half<<<4096, 256, 0, s>>>(src, static_cast<_Float16*>(dst), n);
}

void launch_lu_solve(const DevOps& d, int precision, bool transpose, const double* Bin, double* Xout, bool accumulate,
                     bool check_done, hipStream_t s) {
  launch_lu_solve_mapped(d, precision, transpose, nullptr, nullptr, d.nx_total, Bin, Xout, accumulate, check_done, s);
}

void launch_lu_solve_mapped(const DevOps& f, int precision, bool transpose, const int* mat_of, const int* skip,
                            int nrows, const double* Bin, double* Xout, bool accumulate, bool check_done,
                            hipStream_t s) {
  // the mirror flags of the FP32 factors, set at their formation
  const int* mir = (precision != 0 && precision != kFactorsFp16) ? f.mirror : nullptr;
  if (precision == 0) {
    const double* LU = static_cast<const double*>(f.lu);
    if (transpose)
      k_solve<double, 1><<<nrows, 1024, 0, s>>>(LU, f.piv, f.perm, Bin, Xout, f.status, accumulate, check_done, f.npad, mat_of, skip, f.band_kl, f.band_kl > 0 ? f.band_kl + f.band_ku : 0, lu_paired(f) ? 1 : 0, mir, f.n, f.nth);
    else
      k_solve<double, 0><<<nrows, 1024, 0, s>>>(LU, f.piv, f.perm, Bin, Xout, f.status, accumulate, check_done, f.npad, mat_of, skip, f.band_kl, f.band_kl > 0 ? f.band_kl + f.band_ku : 0, lu_paired(f) ? 1 : 0, mir, f.n, f.nth);
  } else if (precision == kFactorsFp16) {
    const _Float16* LU = static_cast<const _Float16*>(f.lu);
    if (transpose)
      k_solve<_Float16, 1><<<nrows, 1024, 0, s>>>(LU, f.piv, f.perm, Bin, Xout, f.status, accumulate, check_done, f.npad, mat_of, skip, f.band_kl, f.band_kl > 0 ? f.band_kl + f.band_ku : 0, lu_paired(f) ? 1 : 0, mir, f.n, f.nth);
    else
      k_solve<_Float16, 0><<<nrows, 1024, 0, s>>>(LU, f.piv, f.perm, Bin, Xout, f.status, accumulate, check_done, f.npad, mat_of, skip, f.band_kl, f.band_kl > 0 ? f.band_kl + f.band_ku : 0, lu_paired(f) ? 1 : 0, mir, f.n, f.nth);
  } else {
    const float* LU = static_cast<const float*>(f.lu);
    if (transpose)
      k_solve<float, 1><<<nrows, 1024, 0, s>>>(LU, f.piv, f.perm, Bin, Xout, f.status, accumulate, check_done, f.npad, mat_of, skip, f.band_kl, f.band_kl > 0 ? f.band_kl + f.band_ku : 0, lu_paired(f) ? 1 : 0, mir, f.n, f.nth);
    else
      k_solve<float, 0><<<nrows, 1024, 0, s>>>(LU, f.piv, f.perm, Bin, Xout, f.status, accumulate, check_done, f.npad, mat_of, skip, f.band_kl, f.band_kl > 0 ? f.band_kl + f.band_ku : 0, lu_paired(f) ? 1 : 0, mir, f.n, f.nth);
  }
}

}  // namespace bte

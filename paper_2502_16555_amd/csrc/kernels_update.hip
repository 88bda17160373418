// Trailing update of the batched LU: A22 -= L21 U12 for every matrix, 128 x 128
// tiles on MFMA (FP64, FP32, or FP32 storage with bf16 operands).  The tile's
// old values are read and written once (the LDS-staged epilogue), L21 and U12
// are read once per tile; blocks of one matrix stay on one XCD so that its L21
// and U12 come from that XCD's L2.
#include "internal.h"
#include "lu_common.h"

namespace bte {
namespace {

constexpr int NB = kNB;

// ---------------------------------------------------------------------------
// Epilogue of a 128 x 128 update tile: A[r0.., c0..] -= acc.  The accumulators
// (MFMA result layout) go through LDS (the K-chunk buffers, at least 64 KB) so
// that the read-modify-write of the tile runs down whole columns with 16-byte
// accesses; FP64 tiles take two passes of 64 rows.
// ---------------------------------------------------------------------------
// FP32 tiles: the old values of the tile, in the epilogue's layout, loaded
// before the last K chunk so that their latency hides behind its products.
constexpr int kPreV = 128 * 128 / 4 / 256;  // float4 per thread
__device__ inline void tile_prefetch(const float* __restrict__ A, int npad, int r0, int c0, float4 (&pre)[kPreV]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < kPreV; ++u) {
    const int e = tid + u * 256;
    const int col = e / 32, rr = (e % 32) * 4;
    pre[u] = *reinterpret_cast<const float4*>(A + (size_t)(c0 + col) * npad + r0 + rr);
  }
}

template <typename T, bool HASPRE = false, typename Acc, int NPRE = 1>
__device__ inline void update_epilogue(T* __restrict__ A, int npad, int r0, int c0, const Acc (&acc)[4][4],
                                       void* lds, const float4 (&pre)[NPRE]) {
  using V = typename Vec4<T>::type;
  constexpr int PER = Vec4<T>::per;
  constexpr int P = sizeof(T) / 4;       // passes
  constexpr int RP = 128 / P;            // rows per pass
  constexpr int LDC = RP + 4 / P;        // 16-byte aligned column stride
  T* sC = static_cast<T*>(lds);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
#pragma unroll
  for (int pass = 0; pass < P; ++pass) {
    __syncthreads();
    if (wr / RP == pass || P == 1) {
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
          for (int it = 0; it < 4; ++it)
            sC[(wc + bj * 16 + li) * LDC + wr - pass * RP + bi * 16 + Mma<T>::row(lk, it)] = acc[bi][bj][it];
    }
    __syncthreads();
    constexpr int NV = 128 * RP / PER / 256;
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = tid + u * 256;
      const int col = e / (RP / PER), rr = (e % (RP / PER)) * PER;
      V* p = reinterpret_cast<V*>(A + (size_t)(c0 + col) * npad + r0 + pass * RP + rr);
      V o;
      if constexpr (HASPRE) o = pre[u];
      else o = *p;
      const V a = *reinterpret_cast<const V*>(sC + col * LDC + rr);
      T* po = reinterpret_cast<T*>(&o);
      const T* pa = reinterpret_cast<const T*>(&a);
#pragma unroll
      for (int m = 0; m < PER; ++m) po[m] -= pa[m];
      *p = o;
    }
  }
}

// ---------------------------------------------------------------------------
// BF16 trailing update (FP32 storage and accumulation): L21 and U12 are
// rounded to bf16 on their way to LDS, hi = bf16(a), lo = bf16(a - hi); the
// product takes hi*hi (NTERMS = 1) or hi*hi + hi*lo + lo*hi (NTERMS = 3) with
// MFMA f32_16x16x32_bf16.  Operands of that instruction: lane l holds 8
// consecutive k of row l%16 (A) and of column l%16 (B), k = 8 (l/16) + e; the
// result has the FP32 16x16x4 layout.  LDS holds the chunk k-contiguous per row
// of L21 and per column of U12 so that each operand is one 16-byte read.
// ---------------------------------------------------------------------------
using bf16x8 = __bf16 __attribute__((ext_vector_type(8)));

template <int NTERMS, int KD>
__global__ __launch_bounds__(256) void k_update_bf16(float* __restrict__ LU, int npad, int k0, int mtr, int mtc,
                                                     int tj0, int nmat, int lrow) {
  constexpr int KC = 32;
  constexpr int LDK = KC + 8;               // bf16 per row, padded (80 bytes)
  constexpr int NH = (NTERMS == 1) ? 1 : 2;  // hi (and lo) copies
  int mat, tile;
  xcd_map(blockIdx.x, mtr * mtc + lrow, nmat, &mat, &tile);
  if (mat >= nmat) return;
  // mtr x mtc tiles, then lrow more in the first tile row (columns mtc ..)
  const bool band = tile >= mtr * mtc;
  const int ti = band ? 0 : tile % mtr, tj = band ? mtc + (tile - mtr * mtc) : tile / mtr;
  float* A = LU + (size_t)mat * npad * npad;
  const int r0 = k0 + KD + ti * 128, c0 = k0 + KD + (tj0 + tj) * 128;
  // [L21/U12][buffer][hi/lo][row or column][k], or the epilogue's 128 x 132 floats
  constexpr int OPER_BYTES = 2 * 2 * NH * 128 * LDK * 2;
  constexpr int EPI_BYTES = 128 * 132 * 4;
  constexpr int LDS_BYTES = OPER_BYTES > EPI_BYTES ? OPER_BYTES : EPI_BYTES;
  __shared__ __align__(16) unsigned char smem[LDS_BYTES];
  __bf16* sL = reinterpret_cast<__bf16*>(smem);                  // [2][NH][128][LDK]
  __bf16* sU = sL + 2 * NH * 128 * LDK;                          // [2][NH][128][LDK]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  // staging: thread t owns row/column t % 128 and k range 16 (t / 128) .. +16
  const int own = tid & 127, kh = (tid >> 7) * 16;
  float ra[16], rb[16];
  auto load = [&](int kk) {
#pragma unroll
    for (int k = 0; k < 16; ++k) ra[k] = A[(size_t)(k0 + kk + kh + k) * npad + r0 + own];
    const float4* pu = reinterpret_cast<const float4*>(A + (size_t)(c0 + own) * npad + k0 + kk + kh);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = pu[q];
      rb[4 * q] = v.x;
      rb[4 * q + 1] = v.y;
      rb[4 * q + 2] = v.z;
      rb[4 * q + 3] = v.w;
    }
  };
  auto store = [&](int buf) {
    __bf16* dl = sL + ((size_t)buf * NH * 128 + own) * LDK + kh;
    __bf16* du = sU + ((size_t)buf * NH * 128 + own) * LDK + kh;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const __bf16 hl = static_cast<__bf16>(ra[k]), hu = static_cast<__bf16>(rb[k]);
      dl[k] = hl;
      du[k] = hu;
      if (NH == 2) {
        dl[128 * LDK + k] = static_cast<__bf16>(ra[k] - static_cast<float>(hl));
        du[128 * LDK + k] = static_cast<__bf16>(rb[k] - static_cast<float>(hu));
      }
    }
  };
  f32x4 acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = f32x4{0, 0, 0, 0};
  load(0);
  store(0);
  __syncthreads();
  constexpr int NCH = KD / KC;
  float4 pre[kPreV];
  for (int ch = 0; ch < NCH; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < NCH) load((ch + 1) * KC);
    else tile_prefetch(A, npad, r0, c0, pre);
    bf16x8 ah[4], bh[4], al[4], bl[4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      const __bf16* src = sL + ((size_t)buf * NH * 128 + wr + bi * 16 + li) * LDK + 8 * lk;
      ah[bi] = *reinterpret_cast<const bf16x8*>(src);
      if (NH == 2) al[bi] = *reinterpret_cast<const bf16x8*>(src + 128 * LDK);
    }
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      const __bf16* src = sU + ((size_t)buf * NH * 128 + wc + bj * 16 + li) * LDK + 8 * lk;
      bh[bj] = *reinterpret_cast<const bf16x8*>(src);
      if (NH == 2) bl[bj] = *reinterpret_cast<const bf16x8*>(src + 128 * LDK);
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) {
        if (NTERMS == 3) {
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[bi], bh[bj], acc[bi][bj], 0, 0, 0);
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[bi], bl[bj], acc[bi][bj], 0, 0, 0);
        }
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[bi], bh[bj], acc[bi][bj], 0, 0, 0);
      }
    if (ch + 1 < NCH) {
      store(buf ^ 1);
      __syncthreads();
    }
  }
  update_epilogue<float, true>(A, npad, r0, c0, acc, smem, pre);
}

// ---------------------------------------------------------------------------
// Trailing update A22 -= L21 U12: 128 x 128 tiles, K = KD (one panel, 128, or
// two, 256) in chunks of KC staged
// through double-buffered LDS, four wavefronts of 64 x 64 (4 x 4 MFMA blocks).
// The epilogue goes through LDS in P passes of 128 / P rows, which bounds the
// LDS of a block by the K-chunk buffers and lets MINB blocks share a CU; the
// old values of the first NPP passes are loaded before the last K chunk, those
// of every later pass before its accumulators are staged, so that their
// latency hides behind the products or the staging.
// ---------------------------------------------------------------------------
template <typename T, int KC, int P, int MINB, int NPP, int KD>
__global__ __launch_bounds__(256, MINB) void k_update(T* __restrict__ LU, int npad, int k0, int mtr, int mtc, int tj0,
                                                      int nmat, int lrow) {
  using V = typename Vec4<T>::type;
  constexpr int PER = Vec4<T>::per;
  // LDS rows of the K chunk (64 banks of 4 bytes).  FP32: a pitch of 144 puts
  // an operand read (lanes li + 16 lk, rows k + lk, 16 columns) on 64 distinct
  // banks, and U12's transposed stores (16 columns, rows 4 q + m) write column
  // j of row r at j ^ SW(r), SW(r) = 16 ((r / 4) mod 4), so that the four q
  // fall on different banks too; the swizzle is uniform over a wave at each
  // k step of the product, whose reads take column block bj ^ (k / 4 mod 4).
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int LD = F32 ? 128 + 16 : 128 + 4;
  auto sw = [](int r) { return F32 ? 16 * ((r >> 2) & 3) : 0; };
  constexpr int RP = 128 / P;
  constexpr int LDC = RP + 4 / (sizeof(T) / 4);
  int mat, tile;
  xcd_map(blockIdx.x, mtr * mtc + lrow, nmat, &mat, &tile);
  if (mat >= nmat) return;
  // mtr x mtc tiles, then lrow more in the first tile row (columns mtc ..)
  const bool band = tile >= mtr * mtc;
  const int ti = band ? 0 : tile % mtr, tj = band ? mtc + (tile - mtr * mtc) : tile / mtr;
  T* A = LU + (size_t)mat * npad * npad;
  const int r0 = k0 + KD + ti * 128, c0 = k0 + KD + (tj0 + tj) * 128;
  constexpr int OPER = 2 * 2 * KC * LD;
  constexpr int EPI = 128 * LDC;
  __shared__ __align__(16) T smem[OPER > EPI ? OPER : EPI];
  T (*sA)[KC][LD] = reinterpret_cast<T (*)[KC][LD]>(smem);
  T (*sB)[KC][LD] = reinterpret_cast<T (*)[KC][LD]>(smem + 2 * KC * LD);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  constexpr int NA = KC * 128 / PER / 256, NBV = KC * 128 / PER / 256;
  V ra[NA], rb[NBV];
  auto load = [&](int kk) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + u * 256;
      const int k = e / (128 / PER), i = (e % (128 / PER)) * PER;
      ra[u] = *reinterpret_cast<const V*>(A + (size_t)(k0 + kk + k) * npad + r0 + i);
    }
#pragma unroll
    for (int u = 0; u < NBV; ++u) {
      const int e = tid + u * 256;
      const int j = e / (KC / PER), k = (e % (KC / PER)) * PER;
      rb[u] = *reinterpret_cast<const V*>(A + (size_t)(c0 + j) * npad + k0 + kk + k);
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
  constexpr int NCH = KD / KC;
  constexpr int NV = 128 * RP / PER / 256;   // vectors per thread per pass
  V pre[NPP > 0 ? NPP : 1][NV];
  auto prefetch = [&](int pass, V (&dst)[NV]) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = tid + u * 256;
      const int col = e / (RP / PER), rr = (e % (RP / PER)) * PER;
      dst[u] = ntload(reinterpret_cast<const V*>(A + (size_t)(c0 + col) * npad + r0 + pass * RP + rr));
    }
  };
  for (int ch = 0; ch < NCH; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < NCH) load((ch + 1) * KC);
    else {
#pragma unroll
      for (int pp = 0; pp < NPP; ++pp) prefetch(pp, pre[pp]);
    }
#pragma unroll
    for (int k = 0; k < KC; k += 4) {
      T av[4], bv[4];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) av[bi] = sA[buf][k + lk][wr + bi * 16 + li];
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) bv[bj] = sB[buf][k + lk][wc + (bj * 16 ^ sw(k)) + li];
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
  T* sC = smem;
#pragma unroll
  for (int pass = 0; pass < P; ++pass) {
    V old[NV];
    if (pass >= NPP) prefetch(pass, old);
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
      if ((wr + bi * 16) / RP == pass) {
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
          for (int it = 0; it < 4; ++it)
            sC[(wc + bj * 16 + li) * LDC + wr + bi * 16 - pass * RP + Mma<T>::row(lk, it)] = acc[bi][bj][it];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int e = tid + u * 256;
      const int col = e / (RP / PER), rr = (e % (RP / PER)) * PER;
      V* p = reinterpret_cast<V*>(A + (size_t)(c0 + col) * npad + r0 + pass * RP + rr);
      V o;
      if (pass < NPP) o = pre[pass < NPP ? pass : 0][u];
      else o = old[u];
      const V a = *reinterpret_cast<const V*>(sC + col * LDC + rr);
      T* po = reinterpret_cast<T*>(&o);
      const T* pa = reinterpret_cast<const T*>(&a);
#pragma unroll
      for (int m = 0; m < PER; ++m) po[m] -= pa[m];
      *p = o;
    }
  }
}

template <int KD>
void launch_update_k(int kind, void* LU, int npad, int k0, int mtr, int mtc, int tj0, int nmat, bool alt_kc,
                     hipStream_t s, int lrow) {
  const dim3 gu = xcd_grid(mtr * mtc + lrow, nmat);
  switch (kind) {
    case 0:
      if (alt_kc) k_update<double, 8, 4, 2, 1, KD><<<gu, 256, 0, s>>>(static_cast<double*>(LU), npad, k0, mtr, mtc, tj0, nmat, lrow);
      else k_update<double, 16, 4, 2, 1, KD><<<gu, 256, 0, s>>>(static_cast<double*>(LU), npad, k0, mtr, mtc, tj0, nmat, lrow);
      break;
    case 2:
      k_update_bf16<1, KD><<<gu, 256, 0, s>>>(static_cast<float*>(LU), npad, k0, mtr, mtc, tj0, nmat, lrow);
      break;
    case 3:
      k_update_bf16<3, KD><<<gu, 256, 0, s>>>(static_cast<float*>(LU), npad, k0, mtr, mtc, tj0, nmat, lrow);
      break;
    default:
      if (alt_kc) k_update<float, 32, 1, 2, 1, KD><<<gu, 256, 0, s>>>(static_cast<float*>(LU), npad, k0, mtr, mtc, tj0, nmat, lrow);
      else k_update<float, 16, 4, 4, 1, KD><<<gu, 256, 0, s>>>(static_cast<float*>(LU), npad, k0, mtr, mtc, tj0, nmat, lrow);
      break;
  }
}

}  // namespace

void launch_update(int kind, void* LU, int npad, int k0, int mtr, int mtc, int tj0, int nmat, bool alt_kc,
                   hipStream_t s, int kd, int lrow) {
  switch (kd) {
    case 4 * NB: launch_update_k<4 * NB>(kind, LU, npad, k0, mtr, mtc, tj0, nmat, alt_kc, s, lrow); break;
    case 3 * NB: launch_update_k<3 * NB>(kind, LU, npad, k0, mtr, mtc, tj0, nmat, alt_kc, s, lrow); break;
    case 2 * NB: launch_update_k<2 * NB>(kind, LU, npad, k0, mtr, mtc, tj0, nmat, alt_kc, s, lrow); break;
    default: launch_update_k<NB>(kind, LU, npad, k0, mtr, mtc, tj0, nmat, alt_kc, s, lrow); break;
  }
}

}  // namespace bte

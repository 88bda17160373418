// Internal declarations shared by the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace bte {

// Blocking of the batched LU: outer panel width (trailing-update rank); the
// register-resident sub-panel inside the panel factorization is 8 (FP64) or
// 16 (FP32) columns wide.
constexpr int kNB = 128;
constexpr int kPanelThreads = 512;
constexpr int kMaxSwapRows = 2 * kNB;   // rows touched by one panel's interchanges
constexpr int kMaxRows = 2048;          // largest padded system (n = Nr * Ntheta <= 2048)
constexpr int kMaxPanels = kMaxRows / kNB;
constexpr int kPermStride = 1 + 2 * kMaxSwapRows;  // one panel's row permutation: nR, rows, sources
// per matrix: the eight 16 x 16 diagonal-block inverses of a panel's unit lower
// block L11 (row-major), then the inverse of L11 itself (column-major)
constexpr int kLinvXOff = 8 * 256 + kNB * kNB;   // after L11's inverses: U11^-1 of a statically pivoted panel
constexpr int kLinvElems = kLinvXOff + kNB * kNB;
constexpr int kFactorsFp16 = 4;   // solve precision code: FP32 factors stored in FP16

// Device status word bits.
enum : int { kStSingular = 1, kStNoConv = 2, kStNonFinite = 4 };

struct DevOps {
  int nr = 0, nth = 0, n = 0, npad = 0, nh = 0;
  int nd = 0, nx_total = 0, n_params = 0, n_bins = 1, precision = 0;
  int max_nx = 0;
  int update_kc = 0;           // K chunk of the trailing update (0: default)
  int band_kl = 0, band_ku = 0;  // banded systems: lower / upper bandwidth (0: dense)
  int form_xpb = 0;            // matrices per formation block (0: default)
  int static_piv = 0;          // FP32 factors: static pivoting (no interchanges) instead of partial
  int* mirror = nullptr;       // [matrices] static pivoting: 1 where the factors are of the angularly
                               // mirrored matrix (E < 0, formed with |E|; the solves mirror in and out)
  double dt = 0.0;
  // per discharge (device)
  int* x_off = nullptr;        // [nd+1]
  int* nx_of = nullptr;        // [nd]
  size_t* q_off = nullptr;     // [nd] element offset of Q (per discharge)
  size_t* p_off = nullptr;     // [nd] element offset of the Poisson matrix
  double* n0_of = nullptr;     // [nd]
  double* E0_of = nullptr;     // [nd]
  // per global x (device)
  int* x_disc = nullptr;       // [nx_total]
  double* xhat = nullptr;      // [nx_total]
  double* n0x = nullptr;       // [nx_total]
  // operators (device)
  double* U = nullptr;         // [nr*nr]
  double* Uinv = nullptr;      // [nr*nr]
  double* Cord = nullptr;      // [n*n]
  double* Aord = nullptr;      // [n*n]
  double* CordT = nullptr;     // [n*n] transposed (columns contiguous), for the matrix formation
  double* AordT = nullptr;     // [n*n]
  double* Csb = nullptr;       // [n_params*n*n]
  double* mom = nullptr;       // [3*n]
  double* Qt = nullptr;        // concatenated Q of all discharges, FP64
  float* Qt32 = nullptr;       // FP32 copy (mixed modes)
  double* poisson = nullptr;   // concatenated [nx_d][nx_d]
  // workspaces (device)
  double* Y = nullptr;         // [nx_total*n] mode-major scratch of the X step
  void* lu = nullptr;          // [nx_total][npad][npad] of T (double or float), column-major
  void* xscr = nullptr;        // [nx_total][npad][kNB] of T: interchange staging of extra rows
  int lu_pairs = 2;             // dense factors: 1 panels in pairs (K = 256 trailing updates), 2 statically
                                // pivoted factors in groups of four (K = 512; pairs otherwise), 0 single panels
  void* linv = nullptr;        // [nx_total][kLinvElems] of T: inverses of L11's diagonal blocks, of L11, of U11
  int* piv = nullptr;          // [nx_total][npad]
  int* perm = nullptr;         // [nx_total][kMaxPanels][kPermStride] row permutation of every panel
  double* E = nullptr;         // [nx_total]
  double* field_rhs = nullptr; // [nx_total] right-hand side of the Poisson field solve
  double* B = nullptr;         // [nx_total][npad] right-hand side copy
  double* X = nullptr;         // [nx_total][npad] solution (mixed refinement)
  double* R = nullptr;         // [nx_total][npad] residual / correction
  double* Fs = nullptr;        // [nx_total][n] adjoint: post-V state
  double* mu = nullptr;        // [nx_total][n] adjoint: A^-T X^T lambda
  double* adj_part = nullptr;  // adjoint gradient partial sums, one slot per block:
                               // [n_params][ceil(nx/32)][ceil(n/64)] then [nx_total][ceil(n/64)]
  unsigned long long* rmax = nullptr;  // [nx_total] max|r| (as ordered bits)
  unsigned long long* bmax = nullptr;  // [nx_total] max|b|
  unsigned long long* xmax = nullptr;  // [nx_total] max|x|
  // bounds of the operator norms for the refinement stop: inf-norm (row sums)
  // and 1-norm (column sums) of C_ord and A_ord
  double c_inf = 0.0, a_inf = 0.0, c_one = 0.0, a_one = 0.0;
  int* status = nullptr;       // [4]: status bits, done flag, sweeps, spare
  double* resid = nullptr;     // [1] final max_x |r|/|b|
  double* scratch3 = nullptr;  // [3*nx_total] moments scratch
  // heavies' update of the hybrid model (Poisson field mode only)
  double* dxT = nullptr;       // concatenated [nx_d][nx_d] CGL derivative (physical), column-major, offsets p_off
                               // (the implicit step's forward operator, the ion systems)
  double* dx2 = nullptr;       // concatenated D_x D_x, column-major
  double* ion_M = nullptr;     // concatenated [nx_d][nx_d] ion systems (column-major)
  double* ion_b = nullptr;     // [nx_total] right-hand sides
  double* ion_E = nullptr;     // [nx_total] E^n
  double* ni1 = nullptr;       // [nx_total] n_i^{n+1} of the hybrid step
  double* lam = nullptr;       // [nr] eigenvalues of M^-1 G (speed advection)
  double* mu_th = nullptr;     // [nth] cos theta of the ordinates
};

// Batched restarted GMRES of the V step (kernels_gmres.hip): workspace of the
// Krylov solver and the field-binned preconditioner.
struct GmresOps {
  int m = 20;                  // restart length (<= 63)
  int nbins = 0;               // field bins per discharge
  double S0 = 0.0, width = 1.0;  // bin p covers u in [S0 + p width, S0 + (p+1) width)
  double scale = 0.0;          // u = E (0) or asinh(E / scale) (bins graded towards E = 0)
  double rtol = 1e-12;         // ||b - M x||_2 <= rtol ||b||_2 per point
  int* mat_of = nullptr;       // [nx_total] factor set of the point's bin
  double* V = nullptr;         // [m+1][nx_total][npad] Krylov basis
  double* W = nullptr;         // [nx_total][npad]
  double* Z = nullptr;         // [nx_total][npad]
  double* R = nullptr;         // [nx_total][npad]
  double* H = nullptr;         // [nx_total][m][m+1] Hessenberg columns (rotated)
  double* cs = nullptr;        // [nx_total][m]
  double* sn = nullptr;        // [nx_total][m]
  double* g = nullptr;         // [nx_total][m+1]
  double* bnorm = nullptr;     // [nx_total]
  int* conv = nullptr;         // [nx_total] converged
  int* inact = nullptr;        // [nx_total] converged before the current cycle
  int* kcount = nullptr;       // [nx_total] basis vectors of the current cycle
  int* ktot = nullptr;         // [nx_total] iterations of the current step
  double* rest = nullptr;      // [nx_total] last relative residual estimate
};
void launch_bin_map(const DevOps& d, const GmresOps& q, hipStream_t s);
void launch_gmres_init(const DevOps& d, const GmresOps& q, bool first, hipStream_t s);
void launch_gmres_arnoldi(const DevOps& d, const GmresOps& q, int j, hipStream_t s);
void launch_gmres_combine(const DevOps& d, const GmresOps& q, hipStream_t s);
void launch_gmres_status(const DevOps& d, const GmresOps& q, hipStream_t s);

// ---- Hessenberg form of the V systems (kernels_hess.hip) ------------------------
// Out[x] = M In[x] for points x0 .. x0+nx-1 (M row-major n x n; M, In and Out rows
// of length ld, even, with M zero beyond column n).
void launch_mat_apply(const double* M, const double* In, double* Out, int n, int ld, int x0, int nx, hipStream_t s);
// Column stride of the device layout of H for an order-n solve: column c of
// H_d holds row n-1-j at entry j (rows in reverse), zeros from j = n to the stride.
int hess_col_stride(int n);
// (I - dt E_x H_d) Z[x] = Y[x] for every point (H_d in that layout at Hr + h_off[d]);
// a zero rotation latches kStSingular, a non-finite solution kStNonFinite.
void launch_hess_solve(const DevOps& d, const double* Hr, const size_t* h_off, int n, int ld, const double* Y,
                       double* Z, hipStream_t s);

// ---- heavies' update (kernels_ion.hip) ----------------------------------------
// n_i^{n+1} of eq. fluid_step for every discharge, with E^n already in d.ion_E.
void launch_ion_update(const DevOps& d, const double* F, const double* ni_in, double* ni_out, hipStream_t s);
// The same with the ion systems, right-hand sides and E^n in caller-given
// buffers (M: sum Nx_d^2 at the offsets p_off, b and E: [nx_total]).
void launch_ion_update_ws(const DevOps& d, const double* F, const double* ni_in, double* ni_out, double* M, double* b,
                          const double* E, hipStream_t s);
// Fixed device scratch of the allocation-free ion step: the address of this
// GPU's copy (looked up once per device, with that device current).
constexpr size_t kIonScratchDoubles = size_t(1) << 21;
hipError_t ion_scratch(double** out);

// ---- fully implicit step (kernels_implicit.hip) -------------------------------
// d.Y <- A_x applied mode by mode (lambda_i cos theta_a D_x) to the modes in d.Y.
void launch_x_forward(const DevOps& d, hipStream_t s);
// out = X at the inflow entries of every discharge's walls.
void launch_wall_rows(const DevOps& d, double* out, const double* X, hipStream_t s);
int dot_blocks();
// partial[b][v] (b < dot_blocks()) = partial sums of w . V_v, v < nvec.
void launch_dots(const double* w, const double* V, int nvec, size_t stride, size_t N, double* partial,
                 hipStream_t s);
// y = beta y + sum_v coef[v] V_v (coef on the device).
void launch_comb(double* y, double beta, const double* V, const double* coef, int nvec, size_t stride, size_t N,
                 hipStream_t s);
void launch_axpby(double* y, const double* x, double a, double b, size_t N, hipStream_t s);
// One Gram-Schmidt pass from launch_dots' partials (block order): h[v] = t_v, or
// h[v] += t_v with accumulate, and coef[v] = -t_v, v < nvec.
void launch_gs_reduce(const double* partial, int nvec, int accumulate, double* h, double* coef, hipStream_t s);
// *h = ||w|| from launch_dots(w, w, 1, ...) partials; y /= *h where *h > 0.
void launch_norm_reduce(const double* partial, double* h, hipStream_t s);
void launch_scale_inv(double* y, const double* h, size_t N, hipStream_t s);
// Operator action on padded rows with a given field: mode 2: R = (I - dt (n0 C + E A)) X;
// mode 3: R = B - dt E (X A^T).
void launch_apply_field(const DevOps& d, int mode, const double* B, const double* X, double* R, const double* E,
                        hipStream_t s);

// ---- X step (kernels_x.hip) -------------------------------------------------
void launch_x_to_modes(const DevOps& d, const double* F, hipStream_t s);
// Qt (optional): FP64 inverses in the layout of d.Qt to apply instead (forward)
void launch_advect(const DevOps& d, bool fp32, bool transpose, hipStream_t s, const double* Qt = nullptr);
void launch_modes_to_x(const DevOps& d, double* F, hipStream_t s);
void launch_x_to_modes_T(const DevOps& d, const double* F, hipStream_t s);   // U^T contraction
void launch_modes_to_x_T(const DevOps& d, double* F, hipStream_t s);         // Uinv^T contraction
void launch_field(const DevOps& d, int mode, double t_half, double freq, double a1, double V0,
                  const double* Fh, const double* E_given, const double* ni, double* E, hipStream_t s,
                  double* rhs = nullptr);   // Poisson right-hand side scratch (NULL: d.field_rhs)
void launch_field_dE0(const DevOps& d, int mode, double t_half, double freq, double a1, const double* gE,
                      double* gE0, hipStream_t s);
void launch_moments(const DevOps& d, const double* F, double* out, hipStream_t s);
void launch_moments_vjp(const DevOps& d, const double* F, const double* gbar, double* lam, hipStream_t s);
void launch_maxwellian(const DevOps& d, const double* ne, const double* coeff, double* F, hipStream_t s);

// Event pairs recorded around the LU kernels when timing is enabled:
// pairs [0, n_panels) bracket the trailing updates, [n_panels, 2 n_panels) the
// panel + interchange/TRSM launches of each panel step.
struct LuTimer {
  // 8 * max_panels events, one pair per panel each: [0, 2P) trailing update,
  // [2P, 4P) panel and diagonal-block inverses, [4P, 6P) unused (kept empty),
  // [6P, 8P) L11 inverse and U12
  hipEvent_t* ev = nullptr;
  int max_panels = 0;
  int used = 0;               // panel steps recorded
  int launches = 0;           // trailing-update launches recorded
};

// Dense factors are formed with the panels in pairs (the solve must know).
inline bool lu_paired(const DevOps& d) { return d.lu_pairs != 0 && d.band_kl == 0; }

// ---- V step (kernels_lu.hip) ------------------------------------------------
// Forms I - dt (n0 C + E A) (padded to npad with identity) and factors it in
// place, for the points m0 .. m0+count-1 (count < 0: to the last point).
// Look-ahead of the statically pivoted FP32 factorization: a side stream and
// 2 kMaxPanels events (no timing).  Where a trailing update precedes the next
// panel, its first tile column (that panel's columns) goes first, and the next
// panel's diagonal-block factorization and L21 run on the side stream while the
// rest of the update runs on the main stream.
// Formation overlap (form_overlap; statically pivoted dense factors with the
// panels in pairs): the columns and rows below 256 are formed on the main
// stream, the rest on the side stream between form_ev[0] and form_ev[1], and
// the first K = 256 update waits for it.
struct LuLookAhead {
  hipStream_t side = nullptr;
  hipEvent_t* ev = nullptr;
  int look_ahead = 0;
  int form_overlap = 0;
  hipEvent_t form_ev[2] = {nullptr, nullptr};
};
void launch_lu_factor(const DevOps& d, int precision, hipStream_t s, LuTimer* timer = nullptr, int m0 = 0,
                      int count = -1, const LuLookAhead* la = nullptr);
// A22 -= L21 U12 of the kd = 128 (one panel) or 256 (two panels) columns from
// k0 for nmat matrices (mtr x mtc tiles of 128, column tiles tj0 .. tj0 + mtc - 1
// of the trailing matrix from k0 + kd): kind 0 FP64, 1 FP32, 2 FP32 with bf16
// operands, 3 FP32 with split bf16 operands; alt_kc: K chunk 32 (FP32) / 8
// (FP64) instead of 16.  lrow: that many more tiles in the first tile row, after
// the rectangle's mtc columns (an L-shaped tile set in one launch).
void launch_update(int kind, void* LU, int npad, int k0, int mtr, int mtc, int tj0, int nmat, bool alt_kc,
                   hipStream_t s, int kd = kNB, int lrow = 0);
// X = LU^-1 B (or LU^-T B with transpose), rows of length npad, FP64 right-hand sides.
void launch_lu_solve(const DevOps& d, int precision, bool transpose, const double* Bin, double* Xout,
                     bool accumulate, bool check_done, hipStream_t s);
// As launch_lu_solve for nrows right-hand sides, row r solved with the factors
// of matrix mat_of[r] of f (mat_of NULL: matrix r); rows with skip[r] != 0 are
// left untouched (skip may be NULL).
void launch_lu_solve_mapped(const DevOps& f, int precision, bool transpose, const int* mat_of, const int* skip,
                            int nrows, const double* Bin, double* Xout, bool accumulate, bool check_done,
                            hipStream_t s);
// FP32 -> FP16 copy of n elements (factor storage for preconditioning solves).
void launch_to_half(const float* src, void* dst, size_t n, hipStream_t s);
// Ordinate -> harmonic coefficients (P_S, l-major, rows of npad_h, l < nl) and
// back: F = P_O Xh for nl = nth, F += P_O (Xh - Bh) for nl < nth.
void launch_to_harm(const DevOps& d, int nl, int npad_h, const double* F, const double* TS, double* Bh,
                    hipStream_t s);
void launch_from_harm(const DevOps& d, int nl, int npad_h, const double* Xh, const double* Bh, const double* TO,
                      double* F, hipStream_t s);
// Copy F (rows of n) into padded rows of npad and back.
void launch_pad_rows(const DevOps& d, const double* F, double* Bp, hipStream_t s);
void launch_unpad_rows(const DevOps& d, const double* Bp, double* F, hipStream_t s);
// FP64 residual R = B - (I - dt (n0 C + E A)) X (or with A^T for transpose) + per-x norms.
void launch_residual(const DevOps& d, bool transpose, hipStream_t s);
// Operator M = I - dt (n0 C + E A) on padded rows: mode 1: R = B - M X; mode 2: R = M X.
// Tiles of 32 points that all have skip[x] != 0 are left out (skip may be NULL).
void launch_apply(const DevOps& d, int mode, const double* B, const double* X, double* R, const int* skip,
                  hipStream_t s);
void launch_refine_check(const DevOps& d, bool transpose, double rtol, int sweep, bool final_sweep, hipStream_t s);
void launch_reset_refine(const DevOps& d, hipStream_t s);
// p[0..n) = v (a kernel, so that captured graphs hold no memset nodes).
void launch_fill(double* p, double v, size_t n, hipStream_t s);
// Adjoint gradient contractions (fixed-order two-pass sums; grad_E overwritten,
// grad_scal accumulated).
void launch_adjoint_grads(const DevOps& d, double* grad_scal, double* grad_E, hipStream_t s);

}  // namespace bte

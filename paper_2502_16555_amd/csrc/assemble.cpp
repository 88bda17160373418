// Host-side FP64 assembly of the semi-implicit BTE operators.
//
// Follows the "Hybrid fluid-BTE solver" section of the paper:
//   * speed: cubic B-splines on a regular grid of [0, vmax] (eq. f_expansion);
//     with f(vmax) = 0 the clamped spline that is non-zero at vmax is dropped;
//   * mass matrices M = int v^2 phi_p phi_k, G = int v^3 phi_p phi_k (eq. A_x);
//   * collisions (eq. c_en_mat_1d): per process s and pre-collision energy bin b,
//       C[(p,q),(k,l)] = d_ql ( g_s d_q0 int v^3 s phi_k(v) phi_p(u_s(v)) - int v^3 s phi_p phi_k )
//     with the v^3 weight (volume element times collision frequency n0 v sigma),
//     multiplicity g = 2 for ionization, and the gas-temperature term
//     (eq. c_T0_mat_1d) -(k_B T0/m0) int v^3 s_el phi_p' phi_k' on the l = 0 block;
//   * acceleration (eq. adv_v_ws, re-derived from eq. bte-1d with q_e = +e):
//       A = (e/m_e) [ <Y_q|mu|Y_l> int v^2 phi_p phi_k'  +  <Y_q|(1-mu^2) d_mu|Y_l> int v phi_p phi_k ];
//   * ordinate operators P_O (M^-1 (x) I) X P_S (eq. proj_ops), assembled through the
//     Kronecker structure of every term (speed factor (x) angular factor);
//   * x: Chebyshev-Gauss-Lobatto collocation; Q_ij = (I + dt/2 lam_i cos(th_j) D_x)^-1 with
//     the zero-inflow row (eq. hybrid_cnt_b_bdy), computed once (Alg. bte_spatial_adv).
#include "assemble.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <thread>

namespace bte {
namespace {

constexpr int kGauss = 12;  // points per smooth sub-interval

// ---------------------------------------------------------------------------
// Small dense linear algebra (row-major).
// ---------------------------------------------------------------------------
void cholesky(std::vector<double>& A, int n) {  // in place, lower triangle
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0)) throw std::runtime_error("mass matrix not positive definite");
    d = std::sqrt(d);
    A[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / d;
    }
    for (int k = j + 1; k < n; ++k) A[j * n + k] = 0.0;
  }
}

// Solve L Y = B (L lower, n x n; B n x m), in place in B.
void lower_solve(const std::vector<double>& L, int n, std::vector<double>& B, int m) {
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < m; ++c) {
      double s = B[i * m + c];
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * B[k * m + c];
      B[i * m + c] = s / L[i * n + i];
    }
}

// Solve L^T Y = B in place.
void lower_T_solve(const std::vector<double>& L, int n, std::vector<double>& B, int m) {
  for (int i = n - 1; i >= 0; --i)
    for (int c = 0; c < m; ++c) {
      double s = B[i * m + c];
      for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * B[k * m + c];
      B[i * m + c] = s / L[i * n + i];
    }
}

// Cyclic Jacobi eigen-decomposition of a symmetric matrix: S = V diag(e) V^T.
void jacobi_eigen(std::vector<double> S, int n, std::vector<double>* e, std::vector<double>* V) {
  V->assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) (*V)[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += S[i * n + j] * S[i * n + j];
        if (i != j) off += S[i * n + j] * S[i * n + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = S[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = S[p * n + p], aqq = S[q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double skp = S[k * n + p], skq = S[k * n + q];
          S[k * n + p] = c * skp - s * skq;
          S[k * n + q] = s * skp + c * skq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double spk = S[p * n + k], sqk = S[q * n + k];
          S[p * n + k] = c * spk - s * sqk;
          S[q * n + k] = s * spk + c * sqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = (*V)[k * n + p], vkq = (*V)[k * n + q];
          (*V)[k * n + p] = c * vkp - s * vkq;
          (*V)[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  e->resize(n);
  for (int i = 0; i < n; ++i) (*e)[i] = S[i * n + i];
}

// Inverse by Gauss-Jordan elimination with partial pivoting.
void invert(std::vector<double> A, int n, std::vector<double>* Ainv) {
  std::vector<double>& X = *Ainv;
  X.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) X[i * n + i] = 1.0;
  for (int j = 0; j < n; ++j) {
    int p = j;
    double best = std::fabs(A[j * n + j]);
    for (int i = j + 1; i < n; ++i)
      if (std::fabs(A[i * n + j]) > best) { best = std::fabs(A[i * n + j]); p = i; }
    if (best == 0.0) throw std::runtime_error("singular x-advection system");
    if (p != j)
      for (int k = 0; k < n; ++k) { std::swap(A[j * n + k], A[p * n + k]); std::swap(X[j * n + k], X[p * n + k]); }
    double inv = 1.0 / A[j * n + j];
    for (int k = 0; k < n; ++k) { A[j * n + k] *= inv; X[j * n + k] *= inv; }
    for (int i = 0; i < n; ++i) {
      if (i == j) continue;
      double f = A[i * n + j];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { A[i * n + k] -= f * A[j * n + k]; X[i * n + k] -= f * X[j * n + k]; }
    }
  }
}

// -Dx A^-1 for the Poisson operator, A = D_x^2 with Dirichlet rows at both
// walls, formed and inverted (LU with partial pivoting) in extended precision
// (x87 80-bit long double) throughout and rounded to double once at the end.
// A has a condition number of order nx^4;
// Gauss-Jordan in double left relative errors of 2e-10 (nx = 130) to 8e-9
// (nx = 512) in the field it produces, against 1e-13 to 3e-12 for an LU-based
// inverse in double.
std::vector<double> poisson_operator(const std::vector<double>& Dx, int n) {
  using LD = long double;
  // A = D_x^2 with the Dirichlet rows of both walls
  std::vector<LD> A((size_t)n * n, 0);
  for (int i = 1; i < n - 1; ++i)
    for (int k = 0; k < n; ++k) {
      const LD a = Dx[(size_t)i * n + k];
      for (int c = 0; c < n; ++c) A[(size_t)i * n + c] += a * Dx[(size_t)k * n + c];
    }
  A[0] = 1;
  A[(size_t)(n - 1) * n + n - 1] = 1;
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int j = 0; j < n; ++j) {
    int p = j;
    LD best = std::fabs(A[(size_t)j * n + j]);
    for (int i = j + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + j]) > best) { best = std::fabs(A[(size_t)i * n + j]); p = i; }
    if (best == 0) throw std::runtime_error("singular Poisson system");
    if (p != j) {
      for (int k = 0; k < n; ++k) std::swap(A[(size_t)j * n + k], A[(size_t)p * n + k]);
      std::swap(perm[j], perm[p]);
    }
    const LD d = A[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) {
      const LD f = A[(size_t)i * n + j] / d;
      A[(size_t)i * n + j] = f;
      if (f == 0) continue;
      for (int k = j + 1; k < n; ++k) A[(size_t)i * n + k] -= f * A[(size_t)j * n + k];
    }
  }
  // X = U^-1 L^-1 (P I), all columns at once, row by row
  std::vector<LD> X((size_t)n * n, 0);
  for (int i = 0; i < n; ++i) X[(size_t)i * n + perm[i]] = 1;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < i; ++k) {
      const LD f = A[(size_t)i * n + k];
      if (f == 0) continue;
      for (int c = 0; c < n; ++c) X[(size_t)i * n + c] -= f * X[(size_t)k * n + c];
    }
  for (int i = n - 1; i >= 0; --i) {
    for (int k = i + 1; k < n; ++k) {
      const LD f = A[(size_t)i * n + k];
      if (f == 0) continue;
      for (int c = 0; c < n; ++c) X[(size_t)i * n + c] -= f * X[(size_t)k * n + c];
    }
    const LD d = A[(size_t)i * n + i];
    for (int c = 0; c < n; ++c) X[(size_t)i * n + c] /= d;
  }
  std::vector<double> P((size_t)n * n);
  std::vector<LD> row(n);
  for (int i = 0; i < n; ++i) {
    std::fill(row.begin(), row.end(), LD(0));
    for (int k = 0; k < n; ++k) {
      const LD a = Dx[(size_t)i * n + k];
      if (a == 0) continue;
      for (int c = 0; c < n; ++c) row[c] += a * X[(size_t)k * n + c];
    }
    for (int c = 0; c < n; ++c) P[(size_t)i * n + c] = static_cast<double>(-row[c]);
  }
  return P;
}

std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int n, int k, int m) {
  std::vector<double> C(n * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < k; ++l) {
      double a = A[i * k + l];
      if (a == 0.0) continue;
      for (int j = 0; j < m; ++j) C[i * m + j] += a * B[l * m + j];
    }
  return C;
}

// ---------------------------------------------------------------------------
// Speed basis: clamped cubic B-splines, de Boor's triangular evaluation.
// ---------------------------------------------------------------------------
struct Spline {
  std::vector<double> t;  // knots
  int ntot = 0;           // number of clamped splines on t
  int nkeep = 0;          // the first nkeep are the basis
  double vmax = 0.0;

  // Non-zero degree-3 basis values and derivatives at v: N[0..3] belong to
  // splines j0..j0+3.  Returns false outside [0, vmax].
  bool eval(double v, int* j0, double N[4], double dN[4]) const {
    if (v < 0.0 || v > vmax) return false;
    // interval index s with t[s] <= v < t[s+1] (the last interval is closed)
    int lo = 3, hi = ntot;  // valid intervals: [t[3], t[ntot]]
    int s = lo;
    if (v >= t[hi]) s = hi - 1;
    else {
      int a = lo, b = hi;  // t[a] <= v < t[b]
      while (b - a > 1) { int m = (a + b) / 2; if (t[m] <= v) a = m; else b = m; }
      s = a;
    }
    // degree-2 values (for the derivative) and degree-3 values by the recurrence
    double B[4] = {1.0, 0.0, 0.0, 0.0};  // B[r] = N_{s-d+r, d}
    double B2[3] = {0, 0, 0};
    for (int d = 1; d <= 3; ++d) {
      double nb[4] = {0, 0, 0, 0};
      for (int r = 0; r <= d; ++r) {
        int j = s - d + r;
        double val = 0.0;
        if (r - 1 >= 0) {  // term from N_{j, d-1}: (v - t_j)/(t_{j+d} - t_j)
          double den = t[j + d] - t[j];
          if (den > 0) val += (v - t[j]) / den * B[r - 1];
        }
        if (r <= d - 1) {  // term from N_{j+1, d-1}
          double den = t[j + d + 1] - t[j + 1];
          if (den > 0) val += (t[j + d + 1] - v) / den * B[r];
        }
        nb[r] = val;
      }
      for (int r = 0; r < 4; ++r) B[r] = nb[r];
      if (d == 2) for (int r = 0; r < 3; ++r) B2[r] = B[r];
    }
    // N'_{j,3} = 3 [N_{j,2}/(t_{j+3}-t_j) - N_{j+1,2}/(t_{j+4}-t_{j+1})], B2[r] = N_{s-2+r,2}
    for (int r = 0; r < 4; ++r) {
      int j = s - 3 + r;
      double d = 0.0;
      double a = t[j + 3] - t[j], b = t[j + 4] - t[j + 1];
      double n2j = (r - 1 >= 0) ? B2[r - 1] : 0.0;   // N_{j,2} = B2[j - (s-2)] = B2[r-1]
      double n2j1 = (r <= 2) ? B2[r] : 0.0;          // N_{j+1,2} = B2[r]
      if (a > 0) d += 3.0 * n2j / a;
      if (b > 0) d -= 3.0 * n2j1 / b;
      dN[r] = d;
      N[r] = B[r];
    }
    *j0 = s - 3;
    return true;
  }
};

Spline make_spline(int nr, double vmax, int v_bc) {
  Spline sp;
  int nint = (v_bc == 0) ? nr - 3 : nr - 2;
  if (nint < 1) throw std::runtime_error("too few speed basis functions");
  sp.vmax = vmax;
  sp.t.assign(3, 0.0);
  for (int i = 0; i <= nint; ++i) sp.t.push_back(vmax * static_cast<double>(i) / nint);
  for (int i = 0; i < 3; ++i) sp.t.push_back(vmax);
  sp.t[3 + nint] = vmax;
  sp.ntot = nint + 3;
  sp.nkeep = nr;
  return sp;
}

double speed_of(double eps_eV) { return std::sqrt(2.0 * kECharge * eps_eV / kMElectron); }
double energy_of(double v) { return 0.5 * kMElectron * v * v / kECharge; }

double sigma_at(const Process& p, double v) {
  double e = energy_of(v);
  const auto& E = p.eps_eV;
  const auto& S = p.sigma_m2;
  if (e <= E.front()) return S.front();
  if (e >= E.back()) return S.back();
  size_t k = std::upper_bound(E.begin(), E.end(), e) - E.begin();  // E[k-1] <= e < E[k]
  double f = (e - E[k - 1]) / (E[k] - E[k - 1]);
  return S[k - 1] + f * (S[k] - S[k - 1]);
}

int bin_of(const std::vector<double>& edges_v, double v) {
  int nb = static_cast<int>(edges_v.size()) - 1;
  int b = static_cast<int>(std::upper_bound(edges_v.begin(), edges_v.end(), v) - edges_v.begin()) - 1;
  return std::min(std::max(b, 0), nb - 1);
}

// Sorted unique breakpoints restricted to [lo, hi], plus the composite rule.
struct Rule { std::vector<double> x, w; };

Rule composite(std::vector<double> br, double lo, double hi, const std::vector<double>& gx,
               const std::vector<double>& gw) {
  br.push_back(lo);
  br.push_back(hi);
  std::vector<double> b2;
  for (double v : br) if (v >= lo && v <= hi) b2.push_back(v);
  std::sort(b2.begin(), b2.end());
  b2.erase(std::unique(b2.begin(), b2.end()), b2.end());
  Rule r;
  for (size_t i = 0; i + 1 < b2.size(); ++i) {
    double a = b2[i], b = b2[i + 1];
    if (!(b > a)) continue;
    double h = 0.5 * (b - a), m = 0.5 * (a + b);
    for (size_t q = 0; q < gx.size(); ++q) { r.x.push_back(m + h * gx[q]); r.w.push_back(h * gw[q]); }
  }
  return r;
}

// Legendre P_0..P_{L-1} at mu, and (1-mu^2) dP_l/dmu = l (P_{l-1} - mu P_l).
void legendre_all(int L, double mu, std::vector<double>* P, std::vector<double>* Q) {
  P->assign(L, 0.0);
  Q->assign(L, 0.0);
  (*P)[0] = 1.0;
  if (L > 1) (*P)[1] = mu;
  for (int l = 1; l + 1 < L; ++l) (*P)[l + 1] = ((2 * l + 1) * mu * (*P)[l] - l * (*P)[l - 1]) / (l + 1);
  for (int l = 1; l < L; ++l) (*Q)[l] = l * ((*P)[l - 1] - mu * (*P)[l]);
}

}  // namespace

void gauss_legendre(int n, std::vector<double>* x, std::vector<double>* w) {
  x->assign(n, 0.0);
  w->assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));  // initial guess of the i-th largest root
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < n; ++k) { double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1); p0 = p1; p1 = p2; }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        // one more evaluation for the final derivative
        p0 = 1.0; p1 = z;
        for (int k = 1; k < n; ++k) { double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1); p0 = p1; p1 = p2; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        break;
      }
    }
    (*x)[n - 1 - i] = z;
    (*x)[i] = -z;
    double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    (*w)[i] = wt;
    (*w)[n - 1 - i] = wt;
  }
  if (n % 2 == 1) (*x)[n / 2] = 0.0;
}

void assemble(const AssemblyInput& in, HostOps* out) {
  HostOps& H = *out;
  const int nr = in.nr, nth = in.ntheta, nl = in.nl;
  if (nr < 4 || nth < 2 || nl < 1 || nl > nth || nth % 2 != 0)
    throw std::runtime_error("need nr >= 4, even ntheta >= 2 and 1 <= nl <= ntheta");
  if (in.proc.empty()) throw std::runtime_error("no collision process");
  const int n = nr * nth;
  const int nhm = nr * nl;   // harmonic unknowns
  const int nproc = static_cast<int>(in.proc.size());
  const int nbins = static_cast<int>(in.bin_edges_eV.size()) - 1;
  if (nbins < 1) throw std::runtime_error("need at least one energy bin");
  H.nr = nr; H.nth = nth; H.nl = nl; H.n = n; H.nh = nhm; H.n_bins = nbins; H.n_params = nproc * nbins;
  H.vmax = speed_of(in.eps_max_eV);
  Spline sp = make_spline(nr, H.vmax, in.v_bc);
  H.knots = sp.t;
  std::vector<double> gx, gw;
  gauss_legendre(kGauss, &gx, &gw);

  // --- speed-space matrices ---------------------------------------------------
  std::vector<double> knots_in(sp.t.begin() + 3, sp.t.end() - 3);
  Rule rk = composite(knots_in, 0.0, H.vmax, gx, gw);
  H.M.assign(nr * nr, 0.0);
  H.G.assign(nr * nr, 0.0);
  std::vector<double> D1(nr * nr, 0.0), D0(nr * nr, 0.0);
  std::vector<double> m2(nr, 0.0), m4(nr, 0.0);
  for (size_t q = 0; q < rk.x.size(); ++q) {
    double v = rk.x[q], wq = rk.w[q];
    int j0;
    double N[4], dN[4];
    if (!sp.eval(v, &j0, N, dN)) continue;
    for (int r = 0; r < 4; ++r) {
      int p = j0 + r;
      if (p < 0 || p >= nr) continue;
      m2[p] += wq * v * v * N[r];
      m4[p] += wq * v * v * v * v * N[r];
      for (int c = 0; c < 4; ++c) {
        int k = j0 + c;
        if (k < 0 || k >= nr) continue;
        H.M[p * nr + k] += wq * v * v * N[r] * N[c];
        H.G[p * nr + k] += wq * v * v * v * N[r] * N[c];
        D1[p * nr + k] += wq * v * v * N[r] * dN[c];
        D0[p * nr + k] += wq * v * N[r] * N[c];
      }
    }
  }
  // M^-1 (Cholesky)
  std::vector<double> Lm = H.M;
  cholesky(Lm, nr);
  std::vector<double> Minv(nr * nr, 0.0);
  for (int i = 0; i < nr; ++i) Minv[i * nr + i] = 1.0;
  lower_solve(Lm, nr, Minv, nr);
  lower_T_solve(Lm, nr, Minv, nr);
  // generalized eigenproblem G u = lam M u:  S = L^-1 G L^-T = V diag V^T, U = L^-T V
  {
    std::vector<double> S = H.G;
    lower_solve(Lm, nr, S, nr);                   // L^-1 G
    std::vector<double> St(nr * nr);
    for (int i = 0; i < nr; ++i) for (int j = 0; j < nr; ++j) St[i * nr + j] = S[j * nr + i];
    lower_solve(Lm, nr, St, nr);                  // L^-1 (L^-1 G)^T = L^-1 G L^-T
    for (int i = 0; i < nr; ++i)
      for (int j = i + 1; j < nr; ++j) { double a = 0.5 * (St[i * nr + j] + St[j * nr + i]); St[i * nr + j] = St[j * nr + i] = a; }
    std::vector<double> e, V;
    jacobi_eigen(St, nr, &e, &V);
    std::vector<int> idx(nr);
    for (int i = 0; i < nr; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return e[a] < e[b]; });
    std::vector<double> Vs(nr * nr);
    H.lam.resize(nr);
    for (int c = 0; c < nr; ++c) {
      H.lam[c] = e[idx[c]];
      for (int r = 0; r < nr; ++r) Vs[r * nr + c] = V[r * nr + idx[c]];
    }
    lower_T_solve(Lm, nr, Vs, nr);                // U = L^-T V
    H.U = Vs;
    // U^-1 = U^T M
    std::vector<double> Ut(nr * nr);
    for (int i = 0; i < nr; ++i) for (int j = 0; j < nr; ++j) Ut[i * nr + j] = H.U[j * nr + i];
    H.Uinv = matmul(Ut, H.M, nr, nr, nr);
  }

  // --- angular operators ---------------------------------------------------------
  gauss_legendre(nth, &H.mu, &H.w);
  const double pi = 3.14159265358979323846;
  std::vector<double> TO(nth * nl), TS(nl * nth), acpl(nl * nl, 0.0), bcpl(nl * nl, 0.0);
  {
    std::vector<double> Y(nth * nl), Z(nth * nl);  // Y_l(mu_a), (1-mu^2) dY_l/dmu
    for (int a = 0; a < nth; ++a) {
      std::vector<double> P, Q;
      legendre_all(nl, H.mu[a], &P, &Q);
      for (int l = 0; l < nl; ++l) {
        double c = std::sqrt((2.0 * l + 1.0) / (4.0 * pi));
        Y[a * nl + l] = c * P[l];
        Z[a * nl + l] = c * Q[l];
      }
    }
    for (int a = 0; a < nth; ++a)
      for (int l = 0; l < nl; ++l) {
        TO[a * nl + l] = Y[a * nl + l];
        TS[l * nth + a] = Y[a * nl + l] * 2.0 * pi * H.w[a];
      }
    for (int q = 0; q < nl; ++q)
      for (int l = 0; l < nl; ++l)
        for (int a = 0; a < nth; ++a) {
          acpl[q * nl + l] += TS[q * nth + a] * H.mu[a] * Y[a * nl + l];
          bcpl[q * nl + l] += TS[q * nth + a] * Z[a * nl + l];
        }
  }
  // angular factors of the ordinate-space terms: T_O X T_S (nth x nth)
  auto ang = [&](const std::vector<double>& X) {
    return matmul(matmul(TO, X, nth, nl, nl), TS, nth, nl, nth);
  };
  std::vector<double> Il(nl * nl, 0.0), e00(nl * nl, 0.0);
  for (int l = 0; l < nl; ++l) Il[l * nl + l] = 1.0;
  e00[0] = 1.0;
  const std::vector<double> th_I = ang(Il), th_0 = ang(e00), th_a = ang(acpl), th_b = ang(bcpl);
  // kron accumulate: Out[(k,a),(j,b)] += R[k][j] * T[a][b]
  auto kron_add = [&](std::vector<double>& Out, const std::vector<double>& R, const std::vector<double>& T,
                      double s) {
    for (int k = 0; k < nr; ++k)
      for (int j = 0; j < nr; ++j) {
        double r = s * R[k * nr + j];
        if (r == 0.0) continue;
        for (int a = 0; a < nth; ++a)
          for (int b = 0; b < nth; ++b) Out[(size_t)(k * nth + a) * n + j * nth + b] += r * T[a * nth + b];
      }
  };

  // harmonic-space Kronecker accumulate (l-major): Out[(q,k),(l,j)] += R[k][j] * X[q][l]
  auto kron_h = [&](std::vector<double>& Out, const std::vector<double>& R, const std::vector<double>& X,
                    double s) {
    for (int q = 0; q < nl; ++q)
      for (int l = 0; l < nl; ++l) {
        const double x = s * X[q * nl + l];
        if (x == 0.0) continue;
        for (int k = 0; k < nr; ++k)
          for (int j = 0; j < nr; ++j) Out[(size_t)(q * nr + k) * nhm + l * nr + j] += R[k * nr + j] * x;
      }
  };
  H.TO = TO;
  H.TS = TS;

  // --- acceleration operator -------------------------------------------------------
  H.Aord.assign((size_t)n * n, 0.0);
  H.Ah.assign((size_t)nhm * nhm, 0.0);
  {
    std::vector<double> R1 = matmul(Minv, D1, nr, nr, nr), R0 = matmul(Minv, D0, nr, nr, nr);
    kron_add(H.Aord, R1, th_a, kECharge / kMElectron);
    kron_add(H.Aord, R0, th_b, kECharge / kMElectron);
    // the recurrences of the Legendre polynomials for mu P_l and (1 - mu^2) P_l'
    // couple l to l +- 1 only; the quadrature leaves rounding noise elsewhere,
    // which the harmonic operator drops so that it is exactly banded
    std::vector<double> ab(acpl), bb(bcpl);
    for (int q = 0; q < nl; ++q)
      for (int l = 0; l < nl; ++l)
        if (std::abs(q - l) != 1) ab[q * nl + l] = bb[q * nl + l] = 0.0;
    kron_h(H.Ah, R1, ab, kECharge / kMElectron);
    kron_h(H.Ah, R0, bb, kECharge / kMElectron);
  }

  // --- collision operators per process and bin -------------------------------------
  std::vector<double> edges_v(nbins + 1);
  for (int b = 0; b <= nbins; ++b) edges_v[b] = speed_of(in.bin_edges_eV[b]);
  H.Csb.assign((size_t)H.n_params * n * n, 0.0);
  H.Cord.assign((size_t)n * n, 0.0);
  H.Ch.assign((size_t)nhm * nhm, 0.0);
  std::vector<double> ki(nr, 0.0);
  for (int s = 0; s < nproc; ++s) {
    const Process& P = in.proc[s];
    if (P.eps_eV.size() < 2 || P.eps_eV.size() != P.sigma_m2.size()) throw std::runtime_error("bad cross-section table");
    const double g = (P.kind == 2) ? 2.0 : 1.0;
    std::vector<std::vector<double>> Loss(nbins, std::vector<double>(nr * nr, 0.0)), Gain = Loss, CT = Loss;
    std::vector<std::vector<double>> kis(nbins, std::vector<double>(nr, 0.0));
    // breakpoints in v: knots, table points, bin edges, threshold
    std::vector<double> br(knots_in);
    for (double e : P.eps_eV) br.push_back(speed_of(e));
    for (double v : edges_v) br.push_back(v);
    if (P.kind != 0) br.push_back(speed_of(P.threshold_eV));
    const double c_el = (P.kind == 0) ? std::sqrt(1.0 - 2.0 * P.mass_ratio) : 0.0;
    if (P.kind == 0) for (double k : knots_in) br.push_back(k / c_el);
    Rule rv = composite(br, 0.0, H.vmax, gx, gw);
    const double kT_m0 = kKBoltzmann * in.T0_K * P.mass_ratio / kMElectron;
    for (size_t q = 0; q < rv.x.size(); ++q) {
      double v = rv.x[q];
      double wt = rv.w[q] * v * v * v * sigma_at(P, v);
      if (wt == 0.0) continue;
      int b = bin_of(edges_v, v);
      int j0;
      double N[4], dN[4];
      if (!sp.eval(v, &j0, N, dN)) continue;
      int ju = 0;
      double Nu[4] = {0, 0, 0, 0}, dNu[4];
      bool has_u = (P.kind == 0) && sp.eval(c_el * v, &ju, Nu, dNu);
      for (int c = 0; c < 4; ++c) {
        int k = j0 + c;
        if (k < 0 || k >= nr) continue;
        if (P.kind == 2) kis[b][k] += wt * N[c];
        for (int r = 0; r < 4; ++r) {
          int p = j0 + r;
          if (p >= 0 && p < nr) {
            Loss[b][p * nr + k] += wt * N[r] * N[c];
            if (P.kind == 0 && in.T0_K > 0) CT[b][p * nr + k] -= kT_m0 * wt * dN[r] * dN[c];
          }
          if (has_u) {
            int pu = ju + r;
            if (pu >= 0 && pu < nr) Gain[b][pu * nr + k] += wt * Nu[r] * N[c];
          }
        }
      }
    }
    if (P.kind != 0) {
      // inelastic gain in the post-collision speed u: v^2 = alpha u^2 + vth^2, v^3 dv = v^2 alpha u du
      const double alpha = (P.kind == 1) ? 1.0 : 2.0;
      const double vth = speed_of(P.threshold_eV);
      if (vth < H.vmax) {
        auto u_of_v = [&](double v) { return std::sqrt(std::max(v * v - vth * vth, 0.0) / alpha); };
        const double umax = u_of_v(H.vmax);
        std::vector<double> ub;
        for (double k : knots_in) if (k < umax) ub.push_back(k);
        std::vector<double> vb(knots_in);
        for (double e : P.eps_eV) vb.push_back(speed_of(e));
        for (double v : edges_v) vb.push_back(v);
        for (double v : vb) if (v > vth && v < H.vmax) ub.push_back(u_of_v(v));
        Rule ru = composite(ub, 0.0, umax, gx, gw);
        for (size_t q = 0; q < ru.x.size(); ++q) {
          double u = ru.x[q];
          double v = std::sqrt(alpha * u * u + vth * vth);
          double wt = ru.w[q] * v * v * sigma_at(P, v) * alpha * u;
          if (wt == 0.0) continue;
          int b = bin_of(edges_v, v);
          int jv, ju;
          double Nv[4], dNv[4], Nu[4], dNu[4];
          if (!sp.eval(v, &jv, Nv, dNv) || !sp.eval(u, &ju, Nu, dNu)) continue;
          for (int c = 0; c < 4; ++c) {
            int k = jv + c;
            if (k < 0 || k >= nr) continue;
            for (int r = 0; r < 4; ++r) {
              int p = ju + r;
              if (p >= 0 && p < nr) Gain[b][p * nr + k] += wt * Nu[r] * Nv[c];
            }
          }
        }
      }
    }
    for (int b = 0; b < nbins; ++b) {
      std::vector<double> iso(nr * nr), loss(nr * nr);
      for (int i = 0; i < nr * nr; ++i) { iso[i] = g * Gain[b][i] + CT[b][i]; loss[i] = -Loss[b][i]; }
      std::vector<double> Riso = matmul(Minv, iso, nr, nr, nr), Rloss = matmul(Minv, loss, nr, nr, nr);
      std::vector<double> Cb((size_t)n * n, 0.0);
      kron_add(Cb, Riso, th_0, 1.0);
      kron_add(Cb, Rloss, th_I, 1.0);
      const double sc = in.scal[s * nbins + b];
      double* dst = H.Csb.data() + (size_t)(s * nbins + b) * n * n;
      for (size_t i = 0; i < (size_t)n * n; ++i) { dst[i] = Cb[i]; H.Cord[i] += sc * Cb[i]; }
      kron_h(H.Ch, Riso, e00, sc);
      kron_h(H.Ch, Rloss, Il, sc);
      if (P.kind == 2) for (int k = 0; k < nr; ++k) ki[k] += sc * kis[b][k];
    }
  }

  // --- moment weights [3][n] ----------------------------------------------------
  H.mom.assign(3 * n, 0.0);
  for (int k = 0; k < nr; ++k)
    for (int a = 0; a < nth; ++a) {
      double W = 2.0 * pi * H.w[a];
      H.mom[0 * n + k * nth + a] = m2[k] * W;
      H.mom[1 * n + k * nth + a] = 0.5 * kMElectron / kECharge * m4[k] * W;
      H.mom[2 * n + k * nth + a] = ki[k] * W;
    }

  // --- x operators per discharge ---------------------------------------------------
  H.xops.clear();
  for (int nx : in.nx_per) {
    if (nx < 3) throw std::runtime_error("need nx >= 3");
    XOps X;
    X.nx = nx;
    X.xhat.resize(nx);
    for (int i = 0; i < nx; ++i) X.xhat[i] = -std::cos(pi * i / (nx - 1));
    std::vector<double> bw(nx);
    for (int j = 0; j < nx; ++j) bw[j] = ((j % 2) ? -1.0 : 1.0) * ((j == 0 || j == nx - 1) ? 0.5 : 1.0);
    X.Dx.assign(nx * nx, 0.0);
    for (int i = 0; i < nx; ++i) {
      double diag = 0.0;
      for (int j = 0; j < nx; ++j) {
        if (i == j) continue;
        double d = (bw[j] / bw[i]) / (X.xhat[i] - X.xhat[j]);
        X.Dx[i * nx + j] = d;
        diag -= d;
      }
      X.Dx[i * nx + i] = diag;
    }
    for (double& d : X.Dx) d *= 2.0 / in.L;
    advection_inverses(H, X, 0.5 * in.dt, &X.Qt);
    // Poisson: D2 with Dirichlet rows, E = -Dx D2^-1 rhs
    X.poisson = poisson_operator(X.Dx, nx);
    H.xops.push_back(std::move(X));
  }
}

void advection_inverses(const HostOps& H, const XOps& X, double h, std::vector<double>* Qt) {
  // Q for the ordinates with cos(theta) > 0 (upper half of the ascending GL nodes);
  // the lower half follows from the mirror symmetry Q(-mu) = J Q(mu) J.
  const int nx = X.nx, nr = H.nr, nh = H.nth / 2;
  Qt->assign((size_t)nr * nh * nx * nx, 0.0);
  const int nmode = nr * nh;
  unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  std::vector<std::string> errs(nthreads);
  for (unsigned tid = 0; tid < nthreads; ++tid) {
    pool.emplace_back([&, tid]() {
      try {
        for (int m = tid; m < nmode; m += nthreads) {
          int i = m / nh, hh = m % nh;
          double c = h * H.lam[i] * H.mu[nh + hh];
          std::vector<double> B(nx * nx);
          for (int r = 0; r < nx; ++r)
            for (int cc = 0; cc < nx; ++cc) B[r * nx + cc] = (r == cc ? 1.0 : 0.0) + c * X.Dx[r * nx + cc];
          for (int cc = 0; cc < nx; ++cc) B[cc] = (cc == 0) ? 1.0 : 0.0;  // inflow row at xhat = -1
          std::vector<double> Bi;
          invert(B, nx, &Bi);
          double* Q = Qt->data() + (size_t)m * nx * nx;
          for (int r = 0; r < nx; ++r)
            for (int cc = 0; cc < nx; ++cc) Q[(size_t)cc * nx + r] = (cc == 0) ? 0.0 : Bi[r * nx + cc];
        }
      } catch (const std::exception& e) {
        errs[tid] = e.what();
      }
    });
  }
  for (auto& t : pool) t.join();
  for (auto& e : errs) if (!e.empty()) throw std::runtime_error(e);
}

std::vector<double> maxwellian_coeffs(const HostOps& H, double Te_eV) {
  const int nr = H.nr;
  Spline sp;
  sp.t = H.knots;
  sp.ntot = static_cast<int>(H.knots.size()) - 4;
  sp.nkeep = nr;
  sp.vmax = H.vmax;
  std::vector<double> gx, gw;
  gauss_legendre(2 * kGauss, &gx, &gw);
  std::vector<double> knots_in(sp.t.begin() + 3, sp.t.end() - 3);
  Rule r = composite(knots_in, 0.0, H.vmax, gx, gw);
  const double pi = 3.14159265358979323846;
  const double vth = std::sqrt(2.0 * kECharge * Te_eV / kMElectron);
  std::vector<double> b(nr, 0.0);
  for (size_t q = 0; q < r.x.size(); ++q) {
    double v = r.x[q];
    double fM = std::exp(-(v / vth) * (v / vth)) / (std::pow(pi, 1.5) * vth * vth * vth);
    int j0;
    double N[4], dN[4];
    if (!sp.eval(v, &j0, N, dN)) continue;
    for (int c = 0; c < 4; ++c) {
      int p = j0 + c;
      if (p >= 0 && p < nr) b[p] += r.w[q] * v * v * fM * N[c];
    }
  }
  std::vector<double> Lm = H.M;
  cholesky(Lm, nr);
  lower_solve(Lm, nr, b, 1);
  lower_T_solve(Lm, nr, b, 1);
  return b;
}

}  // namespace bte

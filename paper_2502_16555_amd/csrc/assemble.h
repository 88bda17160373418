// Host-side FP64 assembly of the velocity- and x-space operators of the
// semi-implicit BTE step ("Hybrid fluid-BTE solver" section of the paper).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace bte {

constexpr double kECharge = 1.602176634e-19;     // C
constexpr double kMElectron = 9.1093837015e-31;  // kg
constexpr double kKBoltzmann = 1.380649e-23;     // J/K
constexpr double kEps0 = 8.8541878128e-12;       // F/m

struct Process {
  int kind = 0;                // 0 elastic, 1 excitation, 2 ionization
  double threshold_eV = 0.0;
  double mass_ratio = 0.0;
  std::vector<double> eps_eV, sigma_m2;
};

struct AssemblyInput {
  int nr = 0, ntheta = 0, nl = 0;
  int v_bc = 0;                // 0 natural, 1 f(vmax) = 0
  double eps_max_eV = 0.0, T0_K = 0.0, dt = 0.0, L = 0.0;
  std::vector<Process> proc;
  std::vector<double> bin_edges_eV;   // n_bins + 1
  std::vector<double> scal;           // n_proc * n_bins
  std::vector<int> nx_per;            // per discharge
};

// Spatial operators of one discharge.
struct XOps {
  int nx = 0;
  std::vector<double> xhat;      // [nx]
  std::vector<double> Dx;        // [nx][nx], physical (2/L factor)
  std::vector<double> Qt;        // [nr][ntheta/2][nx][nx]: Qt[i][h][c][r] = Q_{i,a}[r][c], a = ntheta/2 + h
  std::vector<double> poisson;   // [nx][nx]: E = P rhs, rhs = [V_left, -(e/eps0)(ni-ne) interior, 0]
};

struct HostOps {
  int nr = 0, nth = 0, nl = 0, n = 0, nh = 0, n_params = 0, n_bins = 1;   // n = nr nth, nh = nr nl
  double vmax = 0.0;
  std::vector<double> knots;
  std::vector<double> mu, w;          // GL ordinates
  std::vector<double> M, G;           // [nr][nr]
  std::vector<double> lam;            // [nr] eigenvalues of M^-1 G
  std::vector<double> U, Uinv;        // [nr][nr]
  std::vector<double> Cord;           // [n][n] sum_sb scal C^(s,b)_ord (per unit n0)
  std::vector<double> Aord;           // [n][n] per unit field
  std::vector<double> Csb;            // [n_params][n][n]
  // harmonic-space operators, unknowns ordered l-major (index l * nr + k): the
  // collision operator is block diagonal in l and the acceleration operator
  // couples l to l +- 1, so both are banded with half-bandwidth 2 nr - 1
  std::vector<double> Ch, Ah;         // [nh][nh]
  std::vector<double> TO, TS;         // [nth][nl] and [nl][nth] (T_S T_O = I_nl: Gauss-Legendre
                                      // quadrature is exact for Y_q Y_l, q + l <= 2 nl - 2 < 2 nth)
  std::vector<double> mom;            // [3][n] number, energy (eV), ionization weights
  std::vector<XOps> xops;             // per discharge
};

// Throws std::runtime_error on invalid input.
void assemble(const AssemblyInput& in, HostOps* out);

// Inverses of the backward-Euler x systems over a step h, I + h lam_i cos(theta_a) D_x
// with the inflow row replaced by the zero-inflow condition (eq.
// bte_semi_implicit_xspace0 takes h = dt / 2), for the ordinates with
// cos(theta) > 0, in the layout of XOps::Qt.
void advection_inverses(const HostOps& H, const XOps& X, double h, std::vector<double>* Qt);

// Unit-density Maxwellian at Te projected on the speed basis (M c = b).
std::vector<double> maxwellian_coeffs(const HostOps& ops, double Te_eV);

// Gauss-Legendre nodes/weights on [-1, 1] (ascending).
void gauss_legendre(int n, std::vector<double>* x, std::vector<double>* w);

}  // namespace bte

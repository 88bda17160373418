// Hessenberg form of the velocity-space systems (host setup, FP64).
#pragma once

#include <vector>

#include "assemble.h"

namespace bte {

// One discharge's transforms (harmonic basis, n = nr nl unknowns, l-major):
// (B - s A_h)^-1 = Q (I - s H)^-1 W with B = I - dt n0 C_h, K = B^-1 A_h = Q H Q^T.
struct HessForm {
  int n = 0;
  std::vector<double> W;    // [n][n] row-major: Q^T B^-1
  std::vector<double> Q;    // [n][n] row-major, orthogonal
  std::vector<double> Hc;   // [n][n] column-major upper Hessenberg H
};

// Householder reduction of the row-major n x n matrix K to upper Hessenberg form
// in place (entries below the subdiagonal set to zero), K_in = Q K_out Q^T.
void hessenberg_reduce(std::vector<double>& K, int n, std::vector<double>* Q, int nthreads);

// The transforms of one discharge with neutral density n0 and time step dt.
void hessenberg_setup(const HostOps& H, double n0, double dt, int nthreads, HessForm* out);

}  // namespace bte

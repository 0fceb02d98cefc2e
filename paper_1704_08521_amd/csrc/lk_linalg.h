// Small dense host linear algebra used at set-up and by the Krylov drivers.
#pragma once

#include <vector>

namespace lk {

// Eigen-decomposition of the symmetric tridiagonal matrix with diagonal a[0..n-1]
// and off-diagonal b[0..n-2]: T = Q diag(lam) Q^T, lam ascending, Q row-major
// n x n with the eigenvectors as columns.  Returns false if it fails to converge.
bool sym_tridiag_eig(int n, std::vector<double> a, std::vector<double> b, std::vector<double>& lam,
                     std::vector<double>& Q);

// Modes of the 1D Neumann operator A = M^-1 K of one axis (M = diag(d), K the
// couplings 1/dd across interior faces): K s = lam M s.  S (row-major, columns
// s_m, S^T M S = I) and Wf = S^T M (row-major).  lam ascending (last ~ 0).
bool neumann_modes(int n, const double* d, const double* dd, std::vector<double>& lam, std::vector<double>& S,
                   std::vector<double>& Wf);

}  // namespace lk

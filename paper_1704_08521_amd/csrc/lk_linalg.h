// Small dense host linear algebra used at set-up and by the Krylov drivers.
#pragma once

#include <complex>
#include <vector>

namespace lk {

using cplx = std::complex<double>;

// Eigenvalues of a real m x m matrix in upper Hessenberg form (row-major), by
// the shifted QR iteration in complex arithmetic (Wilkinson shifts, deflation of
// negligible subdiagonal entries).  Returns false if it fails to converge.
bool hess_eigvals(int m, const std::vector<double>& H, std::vector<cplx>& lam);

// Unit eigenvector y of H for eigenvalue lam by inverse iteration with a complex
// LU factorization (partial pivoting); the largest-modulus entry is made real
// positive.
bool hess_eigvec(int m, const std::vector<double>& H, cplx lam, std::vector<cplx>& y);

// One shifted QR step on H (m x m, Hessenberg) in real arithmetic: with
// M = H - re I (single real shift) or M = H^2 - 2 re H + (re^2 + im^2) I (complex
// pair), M = Qs R, H <- Qs^T H Qs and Q <- Q Qs (Q is m x m, row-major).  Entries
// below the subdiagonal are reset to zero afterwards.
void shifted_qr_step(int m, std::vector<double>& H, std::vector<double>& Q, double re, double im, bool pair);

// Eigen-decomposition of the symmetric tridiagonal matrix with diagonal a[0..n-1]
// and off-diagonal b[0..n-2]: T = Q diag(lam) Q^T, lam ascending, Q row-major
// n x n with the eigenvectors as columns.  Returns false if it fails to converge.
bool sym_tridiag_eig(int n, std::vector<double> a, std::vector<double> b, std::vector<double>& lam,
                     std::vector<double>& Q);

// Modes of the 1D Neumann operator A = M^-1 K of one axis (M = diag(d), K the
// couplings 1/dd across interior faces): K s = lam M s.  S (row-major, columns
// s_m, S^T M S = I) and Wf = S^T M (row-major).  lam ascending (last ~ 0).
// Even (odd = false) or odd modes of a mirror-symmetric axis in the half basis; see
// lk_linalg.cpp.
bool neumann_half_modes(int n, const double* d, const double* dd, bool odd, std::vector<double>& lam,
                        std::vector<double>& Sh);
bool neumann_modes(int n, const double* d, const double* dd, std::vector<double>& lam, std::vector<double>& S,
                   std::vector<double>& Wf);

}  // namespace lk

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

// Modes of a 1D operator A = M^-1 K with K symmetric tridiagonal (diagonal kd[0..n-1],
// off-diagonal ko[0..n-2]) and M = diag(m), m > 0: K s = lam M s.  lam ascending; S
// (row-major, columns s_k, S^T M S = I) and Wf = S^T M (row-major).
bool tridiag_modes(int n, const double* kd, const double* ko, const double* m, std::vector<double>& lam,
                   std::vector<double>& S, std::vector<double>& Wf);
// Even (odd = false) or odd modes of a mirror-symmetric operator in the half basis; see
// lk_linalg.cpp.
bool tridiag_half_modes(int n, const double* kd, const double* ko, const double* m, bool odd,
                        std::vector<double>& lam, std::vector<double>& Sh);

// The 1D factors of the discrete operators of one axis with cell widths d[0..n-1] and
// centre distances dd[0..n] (half widths at the walls), as K of K s = lam M s:
//  * neumann_operator: the pressure-correction operator D G (n cells, M = diag(d)), no flux
//    through the walls (the last mode is the constant one, lam ~ 0);
//  * dirichlet_cell_operator: the viscous operator of a velocity component along an axis on
//    which it is cell-centred (n cells, M = diag(d)), wall value 0 reached over a half width;
//  * dirichlet_face_operator: the viscous operator of a component along its own axis on the
//    n + 1 faces 0..n (M = dd on interior faces); the wall faces (value 0) are decoupled
//    points with K = -1, M = 1, so their data never mixes into the interior modes.
void neumann_operator(int n, const double* dd, std::vector<double>& kd, std::vector<double>& ko);
void dirichlet_cell_operator(int n, const double* dd, std::vector<double>& kd, std::vector<double>& ko);
void dirichlet_face_operator(int n, const double* d, const double* dd, std::vector<double>& kd,
                             std::vector<double>& ko, std::vector<double>& m);

// Modes of the 1D Neumann operator A = M^-1 K of one axis (M = diag(d), K the
// couplings 1/dd across interior faces): K s = lam M s.  S (row-major, columns
// s_m, S^T M S = I) and Wf = S^T M (row-major).  lam ascending (last ~ 0).
bool neumann_half_modes(int n, const double* d, const double* dd, bool odd, std::vector<double>& lam,
                        std::vector<double>& Sh);
bool neumann_modes(int n, const double* d, const double* dd, std::vector<double>& lam, std::vector<double>& S,
                   std::vector<double>& Wf);

}  // namespace lk

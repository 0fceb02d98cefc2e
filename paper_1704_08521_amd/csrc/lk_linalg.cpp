// Small dense host linear algebra (float64) for set-up and Krylov drivers.
#include "lk_linalg.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace lk {

// Implicit symmetric QR with Wilkinson shifts on the unreduced trailing block;
// each step chases the bulge with plane rotations J = [[c, -s], [s, c]] applied
// as T <- J^T T J on indices (k, k+1) and accumulated into Q <- Q J.
bool sym_tridiag_eig(int n, std::vector<double> a, std::vector<double> b, std::vector<double>& lam,
                     std::vector<double>& Q) {
  Q.assign((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r) Q[(size_t)r * n + r] = 1.0;
  b.resize(std::max(n, 1), 0.0);
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  long budget = 60L * n + 100;
  while (hi > 0) {
    if (std::fabs(b[hi - 1]) <= eps * (std::fabs(a[hi - 1]) + std::fabs(a[hi]))) {
      b[hi - 1] = 0.0;
      --hi;
      continue;
    }
    if (--budget < 0) return false;
    int lo = hi - 1;
    while (lo > 0 && std::fabs(b[lo - 1]) > eps * (std::fabs(a[lo - 1]) + std::fabs(a[lo]))) --lo;
    // Wilkinson shift: eigenvalue of the trailing 2x2 block nearer to a[hi]
    const double d = 0.5 * (a[hi - 1] - a[hi]);
    const double bh = b[hi - 1];
    const double den = d + std::copysign(std::hypot(d, bh), d);
    const double mu = (den != 0.0) ? a[hi] - bh * bh / den : a[hi];
    double x = a[lo] - mu, z = b[lo];
    double bulge = 0.0;
    for (int k = lo; k < hi; ++k) {
      double r = std::hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r != 0.0) {
        c = x / r;
        s = z / r;
      }
      if (k > lo) b[k - 1] = r;  // the bulge at (k-1, k+1) is annihilated
      const double ak = a[k], ak1 = a[k + 1], bk = b[k];
      a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1;
      a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1;
      b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        bulge = s * b[k + 1];
        b[k + 1] = c * b[k + 1];
        x = b[k];
        z = bulge;
      }
      for (int row = 0; row < n; ++row) {
        double* q = &Q[(size_t)row * n];
        const double qk = q[k], qk1 = q[k + 1];
        q[k] = c * qk + s * qk1;
        q[k + 1] = -s * qk + c * qk1;
      }
    }
  }
  // sort ascending
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int p, int q) { return a[p] < a[q]; });
  lam.resize(n);
  std::vector<double> Qs((size_t)n * n);
  for (int m = 0; m < n; ++m) {
    lam[m] = a[idx[m]];
    for (int row = 0; row < n; ++row) Qs[(size_t)row * n + m] = Q[(size_t)row * n + idx[m]];
  }
  Q.swap(Qs);
  return true;
}

bool neumann_modes(int n, const double* d, const double* dd, std::vector<double>& lam, std::vector<double>& S,
                   std::vector<double>& Wf) {
  // K: couplings 1/dd on interior faces; M = diag(d).  T = M^-1/2 K M^-1/2.
  std::vector<double> a(n, 0.0), b(std::max(n - 1, 1), 0.0);
  for (int f = 1; f < n; ++f) {
    const double c = 1.0 / dd[f];
    a[f - 1] -= c;
    a[f] -= c;
    b[f - 1] = c / std::sqrt(d[f - 1] * d[f]);
  }
  for (int i = 0; i < n; ++i) a[i] /= d[i];
  std::vector<double> Q;
  if (!sym_tridiag_eig(n, a, b, lam, Q)) return false;
  S.resize((size_t)n * n);
  Wf.resize((size_t)n * n);
  for (int i = 0; i < n; ++i) {
    const double sq = std::sqrt(d[i]);
    for (int m = 0; m < n; ++m) {
      const double q = Q[(size_t)i * n + m];
      S[(size_t)i * n + m] = q / sq;   // S = M^-1/2 Q, S^T M S = I
      Wf[(size_t)m * n + i] = q * sq;  // S^T M
    }
  }
  return true;
}

}  // namespace lk
